// Binning: (tile, depth) ordering of all (tile, splat) intersections.
//
// Decomposition (an LSD radix sort split at the duplication step):
//   1. depth presort   stable LSD radix sort of the M (camera, splat) pairs by
//                      their 32-bit depth key; ties keep pair order.  Culled
//                      pairs carry key 0xFFFFFFFF and land at the end.
//   2. scan            exclusive scan (int64) of tiles-touched in that order;
//                      the total is the intersection count.
//   3. keygen          one entry (global tile id, pair id) per touched tile,
//                      written in depth order, load-balanced: each block owns
//                      a fixed span of output entries, whatever the splat
//                      sizes (one splat may cover the whole screen).
//   4. tile sort       stable LSD radix sort of the entries by tile id only
//                      (ceil(tile_bits / 8) passes).  Stability keeps the
//                      depth order inside every tile, so the result equals a
//                      sort by (tile, depth, pair id).
//   5. ranges          ranges[t] = first sorted position with tile >= t.
// Versus one sort of 64-bit (tile | depth) keys this moves ~3x fewer bytes:
// the depth digits are sorted over M pairs instead of over the duplicated
// entries.
//
// Radix passes: 8-bit digits, reduce-then-scan with a fixed grid of G blocks
// (each owning a contiguous span, so the order is stable), 256 threads per
// block, 4096-key tiles; wave64 ballot matching ranks keys inside a wave,
// LDS staging turns the scatter into runs of consecutive addresses per digit.
#include <algorithm>

#include "internal.h"

namespace lsplat {

namespace {

constexpr int kKeygenThreads = 256;
constexpr int kKeygenBlocks = 4096;
constexpr int kRangeThreads = 256;

__device__ __forceinline__ int64_t effective_n(const int64_t* n_dev, int64_t n_host, int64_t cap) {
  if (!n_dev) return n_host;
  int64_t n = *n_dev;
  return (n <= cap) ? n : 0;   // on overflow nothing is sorted
}

__device__ __forceinline__ void block_span(int64_t n, int G, int64_t* beg, int64_t* end) {
  int64_t tiles = (n + kSortTile - 1) / kSortTile;
  int64_t per = (tiles + G - 1) / G;
  int64_t b = (int64_t)blockIdx.x * per * kSortTile;
  *beg = b < n ? b : n;
  int64_t e = b + per * kSortTile;
  *end = e < n ? e : n;
}

// exclusive scan of one uint32 per thread over a 256-thread block
__device__ __forceinline__ uint32_t block_excl_scan_256(uint32_t v, uint32_t* s_tmp /*[4]*/,
                                                        uint32_t* total) {
  int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  uint32_t x = v;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    uint32_t y = __shfl_up(x, d, 64);
    if (lane >= d) x += y;
  }
  if (lane == 63) s_tmp[wave] = x;
  __syncthreads();
  uint32_t wbase = 0, tot = 0;
#pragma unroll
  for (int w = 0; w < 4; ++w) {
    uint32_t t = s_tmp[w];
    if (w < wave) wbase += t;
    tot += t;
  }
  __syncthreads();
  if (total) *total = tot;
  return wbase + x - v;
}

__global__ __launch_bounds__(kSortThreads) void radix_upsweep(const uint32_t* __restrict__ keys,
                                                              const int64_t* n_dev, int64_t n_host,
                                                              int64_t cap, int shift, int G,
                                                              uint32_t* __restrict__ hist) {
  __shared__ uint32_t h[4][256];
  int tid = threadIdx.x, wave = tid >> 6;
  for (int i = tid; i < 4 * 256; i += kSortThreads) (&h[0][0])[i] = 0;
  __syncthreads();
  int64_t n = effective_n(n_dev, n_host, cap);
  int64_t beg, end;
  block_span(n, G, &beg, &end);
  for (int64_t i = beg + tid; i < end; i += kSortThreads) {
    uint32_t d = (keys[i] >> shift) & 255u;
    atomicAdd(&h[wave][d], 1u);
  }
  __syncthreads();
  uint32_t s = h[0][tid] + h[1][tid] + h[2][tid] + h[3][tid];
  hist[(int64_t)tid * G + blockIdx.x] = s;
}

// One block per digit: exclusive scan of that digit's G block counts; the
// digit total goes to tot[d].
__global__ __launch_bounds__(256) void radix_scan_rows(uint32_t* __restrict__ hist, int G,
                                                       uint32_t* __restrict__ tot) {
  __shared__ uint32_t s_tmp[4];
  int d = blockIdx.x, tid = threadIdx.x;
  uint32_t* row = hist + (int64_t)d * G;
  constexpr int kPer = kMaxSortBlocks / 256;
  uint32_t v[kPer];
  uint32_t sum = 0;
#pragma unroll
  for (int k = 0; k < kPer; ++k) {
    int i = tid * kPer + k;
    v[k] = i < G ? row[i] : 0u;
    sum += v[k];
  }
  uint32_t total;
  uint32_t base = block_excl_scan_256(sum, s_tmp, &total);
#pragma unroll
  for (int k = 0; k < kPer; ++k) {
    int i = tid * kPer + k;
    if (i < G) row[i] = base;
    base += v[k];
  }
  if (tid == 0) tot[d] = total;
}

template <bool kIdentVals, bool kWriteKeys>
__global__ __launch_bounds__(kSortThreads) void radix_downsweep(
    const uint32_t* __restrict__ keys_in, const uint32_t* __restrict__ vals_in,
    uint32_t* __restrict__ keys_out, uint32_t* __restrict__ vals_out, const int64_t* n_dev,
    int64_t n_host, int64_t cap, int shift, int G, const uint32_t* __restrict__ hist,
    const uint32_t* __restrict__ tot) {
  __shared__ uint32_t s_base[256];
  __shared__ uint32_t s_wcnt[4][256];
  __shared__ uint32_t s_tstart[256];
  __shared__ uint32_t s_tmp[4];
  __shared__ uint32_t s_keys[kSortTile];
  __shared__ uint32_t s_vals[kSortTile];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  int64_t n = effective_n(n_dev, n_host, cap);
  int64_t beg, end;
  block_span(n, G, &beg, &end);
  // running global base of each digit for this block
  {
    uint32_t t = tot[tid];
    uint32_t ex = block_excl_scan_256(t, s_tmp, nullptr);
    s_base[tid] = ex + hist[(int64_t)tid * G + blockIdx.x];
  }
  const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  for (int64_t tb = beg; tb < end; tb += kSortTile) {
    const int cnt = (int)((end - tb) < kSortTile ? (end - tb) : kSortTile);
#pragma unroll
    for (int w = 0; w < 4; ++w) s_wcnt[w][tid] = 0;
    __syncthreads();
    uint32_t k[kSortItems], v[kSortItems], r[kSortItems];
#pragma unroll
    for (int j = 0; j < kSortItems; ++j) {
      const int idx = wave * (64 * kSortItems) + j * 64 + lane;
      const bool valid = idx < cnt;
      uint32_t key = valid ? keys_in[tb + idx] : 0u;
      uint32_t val;
      if (kIdentVals) val = (uint32_t)(tb + idx);
      else val = valid ? vals_in[tb + idx] : 0u;
      const uint32_t d = (key >> shift) & 255u;
      uint64_t m = __builtin_amdgcn_ballot_w64(valid);
#pragma unroll
      for (int b = 0; b < 8; ++b) {
        const bool bit = (d >> b) & 1u;
        const uint64_t bb = __builtin_amdgcn_ballot_w64(bit);
        m &= bit ? bb : ~bb;
      }
      const uint32_t pre = (uint32_t)__popcll(m & lt_mask);
      uint32_t base = 0;
      if (valid) base = s_wcnt[wave][d];
      if (valid && pre == 0) s_wcnt[wave][d] = base + (uint32_t)__popcll(m);
      k[j] = key;
      v[j] = val;
      r[j] = base + pre;
    }
    __syncthreads();
    // per digit: wave prefix and tile-local start
    const uint32_t c0 = s_wcnt[0][tid], c1 = s_wcnt[1][tid], c2 = s_wcnt[2][tid], c3 = s_wcnt[3][tid];
    const uint32_t dtot = c0 + c1 + c2 + c3;
    __syncthreads();
    s_wcnt[0][tid] = 0;
    s_wcnt[1][tid] = c0;
    s_wcnt[2][tid] = c0 + c1;
    s_wcnt[3][tid] = c0 + c1 + c2;
    s_tstart[tid] = block_excl_scan_256(dtot, s_tmp, nullptr);
    __syncthreads();
#pragma unroll
    for (int j = 0; j < kSortItems; ++j) {
      const int idx = wave * (64 * kSortItems) + j * 64 + lane;
      if (idx < cnt) {
        const uint32_t d = (k[j] >> shift) & 255u;
        const uint32_t pos = s_tstart[d] + s_wcnt[wave][d] + r[j];
        s_keys[pos] = k[j];
        s_vals[pos] = v[j];
      }
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < kSortItems; ++j) {
      const int p = tid + j * kSortThreads;
      if (p < cnt) {
        const uint32_t key = s_keys[p];
        const uint32_t d = (key >> shift) & 255u;
        const uint32_t gpos = s_base[d] + (uint32_t)p - s_tstart[d];
        if ((int64_t)gpos < n) {
          if (kWriteKeys) keys_out[gpos] = key;
          vals_out[gpos] = s_vals[p];
        }
      }
    }
    __syncthreads();
    s_base[tid] += dtot;
  }
}

// ---------------------------------------------------------------------------
// Exclusive scan of ntiles[order[p]] over p in [0, M) into int64 isect_off.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void scan_span(int64_t M, int B, int64_t* beg, int64_t* end) {
  const int64_t unit = kScanThreads * 16;
  int64_t units = (M + unit - 1) / unit;
  int64_t per = (units + B - 1) / B;
  int64_t b = (int64_t)blockIdx.x * per * unit;
  *beg = b < M ? b : M;
  int64_t e = b + per * unit;
  *end = e < M ? e : M;
}

__global__ __launch_bounds__(kScanThreads) void scan_reduce(const uint32_t* __restrict__ order,
                                                            const uint32_t* __restrict__ ntiles,
                                                            int64_t M, int B,
                                                            int64_t* __restrict__ part) {
  __shared__ int64_t s[kScanThreads / 64];
  int64_t beg, end;
  scan_span(M, B, &beg, &end);
  int64_t acc = 0;
  for (int64_t p = beg + threadIdx.x; p < end; p += kScanThreads) {
    const uint32_t m = order[p];
    acc += (m < (uint64_t)M) ? ntiles[m] : 0u;
  }
  for (int d = 32; d > 0; d >>= 1) acc += __shfl_xor(acc, d, 64);
  if ((threadIdx.x & 63) == 0) s[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    int64_t t = 0;
    for (int w = 0; w < kScanThreads / 64; ++w) t += s[w];
    part[blockIdx.x] = t;
  }
}

__global__ void scan_parts(int64_t* __restrict__ part, int B, int64_t M,
                           int64_t* __restrict__ isect_off, int64_t* __restrict__ n_isect) {
  if (threadIdx.x != 0) return;
  int64_t run = 0;
  for (int b = 0; b < B; ++b) {
    int64_t v = part[b];
    part[b] = run;
    run += v;
  }
  isect_off[M] = run;
  *n_isect = run;
}

// Also records, for every key-generation span of kKeygenSpan output entries,
// the pair that owns the span's first entry (span_owner[s]); the entry past
// the last span names the last pair with entries.
__global__ __launch_bounds__(kScanThreads) void scan_down(const uint32_t* __restrict__ order,
                                                          const uint32_t* __restrict__ ntiles,
                                                          int64_t M, int B,
                                                          const int64_t* __restrict__ part,
                                                          int64_t* __restrict__ isect_off,
                                                          const int64_t* __restrict__ n_isect,
                                                          uint32_t* __restrict__ span_owner,
                                                          int64_t n_spans) {
  const int64_t n_total = *n_isect;
  __shared__ int64_t s_w[kScanThreads / 64];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  int64_t beg, end;
  scan_span(M, B, &beg, &end);
  int64_t run = part[blockIdx.x];
  constexpr int kPer = 16;
  for (int64_t tb = beg; tb < end; tb += kScanThreads * kPer) {
    int64_t v[kPer];
    int64_t sum = 0;
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
      int64_t p = tb + (int64_t)tid * kPer + k;
      const uint32_t m = p < end ? order[p] : 0xFFFFFFFFu;
      v[k] = (m < (uint64_t)M) ? (int64_t)ntiles[m] : 0;
      sum += v[k];
    }
    int64_t x = sum;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
      int64_t y = __shfl_up(x, d, 64);
      if (lane >= d) x += y;
    }
    if (lane == 63) s_w[wave] = x;
    __syncthreads();
    int64_t wbase = 0, tot = 0;
    for (int w = 0; w < kScanThreads / 64; ++w) {
      if (w < wave) wbase += s_w[w];
      tot += s_w[w];
    }
    __syncthreads();
    int64_t base = run + wbase + x - sum;
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
      int64_t p = tb + (int64_t)tid * kPer + k;
      if (p < end) {
        isect_off[p] = base;
        if (v[k] > 0) {
          for (int64_t sp = (base + kKeygenSpan - 1) / kKeygenSpan;
               sp * kKeygenSpan < base + v[k] && sp < n_spans; ++sp)
            span_owner[sp] = (uint32_t)p;
          if (base + v[k] == n_total) {
            const int64_t term = (n_total + kKeygenSpan - 1) / kKeygenSpan;
            if (term < n_spans) span_owner[term] = (uint32_t)p;
          }
        }
      }
      base += v[k];
    }
    run += tot;
  }
}

// ---------------------------------------------------------------------------
// Key generation.  Block iteration covers output entries [k0, k0 + span).
// ---------------------------------------------------------------------------
__device__ __forceinline__ int64_t upper_bound_i64(const int64_t* a, int64_t n, int64_t x) {
  int64_t lo = 0, hi = n;
  while (lo < hi) {
    int64_t mid = (lo + hi) >> 1;
    if (a[mid] <= x) lo = mid + 1;
    else hi = mid;
  }
  return lo;
}

__device__ __forceinline__ int cam_of_pair(const CamInfo* cams, int C, int64_t m) {
  int lo = 0, hi = C - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (cams[mid].pair_off <= m) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

__global__ __launch_bounds__(kKeygenThreads) void keygen_kernel(
    const uint32_t* __restrict__ order, const int64_t* __restrict__ isect_off,
    const ushort4* __restrict__ rect, const CamInfo* __restrict__ cams, int C, int64_t M,
    const int64_t* __restrict__ n_isect, int64_t cap, const uint32_t* __restrict__ span_owner,
    uint32_t* __restrict__ keys, uint32_t* __restrict__ vals) {
  __shared__ int32_t s_owner[kKeygenSpan];
  __shared__ int64_t s_off[kKeygenSpan];
  __shared__ uint32_t s_m[kKeygenSpan];
  __shared__ uint32_t s_gbase[kKeygenSpan];
  __shared__ uint32_t s_w[kKeygenSpan];
  __shared__ uint32_t s_gx[kKeygenSpan];
  __shared__ int64_t s_plo, s_phi;
  __shared__ int32_t s_wmax[kKeygenThreads / 64];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t n = *n_isect;
  if (n > cap) return;
  for (int64_t k0 = (int64_t)blockIdx.x * kKeygenSpan; k0 < n; k0 += (int64_t)gridDim.x * kKeygenSpan) {
    const int64_t k1 = (k0 + kKeygenSpan < n) ? k0 + kKeygenSpan : n;
    if (tid == 0) {
      const int64_t sp = k0 / kKeygenSpan;
      int64_t lo = span_owner[sp], hi = span_owner[sp + 1];
      if (lo > M - 1) lo = M - 1;
      if (hi > M - 1) hi = M - 1;
      if (hi < lo) hi = lo;
      s_plo = lo;
      s_phi = hi;
    }
    for (int i = tid; i < kKeygenSpan; i += kKeygenThreads) s_owner[i] = 0;
    __syncthreads();
    const int64_t plo = s_plo, phi = s_phi;
    // per-pair data of every pair owning entries of this span
    for (int64_t p = plo + tid; p <= phi && p - plo < kKeygenSpan; p += kKeygenThreads) {
      const int pl = (int)(p - plo);
      const int64_t off = isect_off[p];
      uint32_t m = order[p];
      if (m >= (uint64_t)M) m = 0;   // unreachable for a valid order
      const ushort4 rc = rect[m];
      const int c = cam_of_pair(cams, C, (int64_t)m);
      const CamInfo& ci = cams[c];
      s_off[pl] = off;
      s_m[pl] = m;
      s_gbase[pl] = (uint32_t)(ci.tile_off + (int64_t)rc.y * ci.GX + rc.x);
      s_w[pl] = (uint32_t)(rc.z - rc.x + 1);
      s_gx[pl] = (uint32_t)ci.GX;
      if (p > plo && off > k0 && off < k0 + kKeygenSpan) s_owner[(int)(off - k0)] = pl;
    }
    __syncthreads();
    // inclusive max-scan of s_owner: each entry learns its pair
    constexpr int kPer = kKeygenSpan / kKeygenThreads;
    int32_t loc[kPer];
    int32_t mx = 0;
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
      int32_t o = s_owner[tid * kPer + k];
      mx = o > mx ? o : mx;
      loc[k] = mx;
    }
    int32_t x = mx;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
      int32_t y = __shfl_up(x, d, 64);
      if (lane >= d) x = y > x ? y : x;
    }
    if (lane == 63) s_wmax[wave] = x;
    int32_t ex = __shfl_up(x, 1, 64);
    if (lane == 0) ex = 0;
    __syncthreads();
    int32_t wpre = 0;
    for (int w = 0; w < wave; ++w) wpre = s_wmax[w] > wpre ? s_wmax[w] : wpre;
    ex = ex > wpre ? ex : wpre;
#pragma unroll
    for (int k = 0; k < kPer; ++k) s_owner[tid * kPer + k] = loc[k] > ex ? loc[k] : ex;
    __syncthreads();
    for (int i = tid; i < (int)(k1 - k0); i += kKeygenThreads) {
      const int pl = s_owner[i];
      const uint32_t local = (uint32_t)(k0 + i - s_off[pl]);
      const uint32_t w = s_w[pl];
      // local / w with a float estimate corrected to the exact quotient
      uint32_t ty = (uint32_t)((float)local * __builtin_amdgcn_rcpf((float)w));
      int32_t rem = (int32_t)local - (int32_t)(ty * w);
      while (rem < 0) { --ty; rem += (int32_t)w; }
      while (rem >= (int32_t)w) { ++ty; rem -= (int32_t)w; }
      keys[k0 + i] = s_gbase[pl] + ty * s_gx[pl] + (uint32_t)rem;
      vals[k0 + i] = s_m[pl];
    }
    __syncthreads();
  }
}

// ranges[t] = number of sorted keys < t, for t in [0, T]
__global__ __launch_bounds__(kRangeThreads) void ranges_kernel(const uint32_t* __restrict__ keys,
                                                               const int64_t* __restrict__ n_isect,
                                                               int64_t cap, int64_t T,
                                                               int64_t* __restrict__ ranges) {
  int64_t n = *n_isect;
  if (n > cap) n = 0;
  for (int64_t t = (int64_t)blockIdx.x * kRangeThreads + threadIdx.x; t <= T;
       t += (int64_t)gridDim.x * kRangeThreads) {
    int64_t lo = 0, hi = n;
    while (lo < hi) {
      int64_t mid = (lo + hi) >> 1;
      if ((int64_t)keys[mid] < t) lo = mid + 1;
      else hi = mid;
    }
    ranges[t] = lo;
  }
}

struct SortBufs {
  uint32_t *ka, *va, *kb, *vb;
};

// One LSD pass; returns the launch error.
template <bool kIdent, bool kWriteKeys>
hipError_t radix_pass(const char* const names[3], const uint32_t* kin, const uint32_t* vin,
                      uint32_t* kout, uint32_t* vout, const int64_t* n_dev, int64_t n_host,
                      int64_t cap, int shift, int G, uint32_t* hist, uint32_t* tot, hipStream_t s) {
  {
    ProfScope ps(names[0], s);
    hipLaunchKernelGGL(radix_upsweep, dim3(G), dim3(kSortThreads), 0, s, kin, n_dev, n_host, cap,
                       shift, G, hist);
  }
  {
    ProfScope ps(names[1], s);
    hipLaunchKernelGGL(radix_scan_rows, dim3(256), dim3(256), 0, s, hist, G, tot);
  }
  {
    ProfScope ps(names[2], s);
    hipLaunchKernelGGL((radix_downsweep<kIdent, kWriteKeys>), dim3(G), dim3(kSortThreads), 0, s,
                       kin, vin, kout, vout, n_dev, n_host, cap, shift, G, hist, tot);
  }
  return hipGetLastError();
}

const char* const kPreNames[3] = {"presort_upsweep", "presort_scan", "presort_downsweep"};
const char* const kTileNames[3] = {"tilesort_upsweep", "tilesort_scan", "tilesort_downsweep"};

}  // namespace

hipError_t launch_bin_sort(const Plan& p, const ls_config* cfg, char* ws, hipStream_t s) {
  (void)cfg;
  hipError_t e;
  const int64_t M = p.M;
  uint32_t* hist = (uint32_t*)(ws + p.hist);
  uint32_t* tot = (uint32_t*)(ws + p.digit_tot);
  int64_t* n_isect = (int64_t*)(ws + p.lay.n_isect);
  int64_t* isect_off = (int64_t*)(ws + p.lay.isect_off);
  uint32_t* order = (uint32_t*)(ws + p.lay.order);
  const uint32_t* ntiles = (const uint32_t*)(ws + p.lay.ntiles);
  const uint32_t* dkey = (const uint32_t*)(ws + p.lay.depth_key);

  // 1. depth presort of the M pairs: 4 passes of 8 bits
  if (M > 0) {
    uint32_t* kA = (uint32_t*)(ws + p.pre_keys_a);
    uint32_t* vA = (uint32_t*)(ws + p.pre_vals_a);
    uint32_t* kB = (uint32_t*)(ws + p.pre_keys_b);
    uint32_t* vB = (uint32_t*)(ws + p.pre_vals_b);
    const int G = p.pre_blocks;
    if ((e = radix_pass<true, true>(kPreNames, dkey, nullptr, kB, vB, nullptr, M, M, 0, G, hist, tot, s))) return e;
    if ((e = radix_pass<false, true>(kPreNames, kB, vB, kA, vA, nullptr, M, M, 8, G, hist, tot, s))) return e;
    if ((e = radix_pass<false, true>(kPreNames, kA, vA, kB, vB, nullptr, M, M, 16, G, hist, tot, s))) return e;
    if ((e = radix_pass<false, false>(kPreNames, kB, vB, nullptr, order, nullptr, M, M, 24, G, hist, tot, s)))
      return e;
  }
  // 2. scan of tile counts in depth order
  {
    int64_t* part = (int64_t*)(ws + p.scan_part);
    const int B = p.scan_blocks;
    ProfScope ps("scan", s);
    if (M > 0) {
      hipLaunchKernelGGL(scan_reduce, dim3(B), dim3(kScanThreads), 0, s, order, ntiles, M, B, part);
    }
    hipLaunchKernelGGL(scan_parts, dim3(1), dim3(64), 0, s, part, M > 0 ? B : 0, M, isect_off,
                       n_isect);
    if (M > 0) {
      hipLaunchKernelGGL(scan_down, dim3(B), dim3(kScanThreads), 0, s, order, ntiles, M, B, part,
                         isect_off, n_isect, (uint32_t*)(ws + p.span_owner), p.n_spans);
    }
    if ((e = hipGetLastError())) return e;
  }
  // 3 + 4. key generation and the tile sort
  int passes = (p.tile_bits + 7) / 8;
  uint32_t* kA = (uint32_t*)(ws + p.lay.keys);
  uint32_t* vA = (uint32_t*)(ws + p.lay.vals);
  uint32_t* kB = (uint32_t*)(ws + p.sort_keys_b);
  uint32_t* vB = (uint32_t*)(ws + p.sort_vals_b);
  const CamInfo* cams = (const CamInfo*)(ws + p.lay.cams);
  if (p.cap > 0 && M > 0) {
    uint32_t* k0 = (passes % 2 == 0) ? kA : kB;
    uint32_t* v0 = (passes % 2 == 0) ? vA : vB;
    int64_t spans = (p.cap + kKeygenSpan - 1) / kKeygenSpan;
    int blocks = (int)std::min<int64_t>(spans, kKeygenBlocks);
    {
      ProfScope ps("keygen", s);
      hipLaunchKernelGGL(keygen_kernel, dim3(blocks), dim3(kKeygenThreads), 0, s, order, isect_off,
                         (const ushort4*)(ws + p.lay.rect), cams, p.C, M, n_isect, p.cap,
                         (const uint32_t*)(ws + p.span_owner), k0, v0);
    }
    if ((e = hipGetLastError())) return e;
    const int G = p.sort_blocks;
    uint32_t *kin = k0, *vin = v0;
    for (int pass = 0; pass < passes; ++pass) {
      uint32_t* kout = (kin == kA) ? kB : kA;
      uint32_t* vout = (vin == vA) ? vB : vA;
      if ((e = radix_pass<false, true>(kTileNames, kin, vin, kout, vout, n_isect, 0, p.cap, 8 * pass, G, hist,
                                       tot, s)))
        return e;
      kin = kout;
      vin = vout;
    }
  }
  // 5. ranges
  {
    int64_t blocks = std::min<int64_t>((p.T + 1 + kRangeThreads - 1) / kRangeThreads, 4096);
    ProfScope ps("ranges", s);
    hipLaunchKernelGGL(ranges_kernel, dim3((unsigned)blocks), dim3(kRangeThreads), 0, s, kA, n_isect,
                       p.cap, p.T, (int64_t*)(ws + p.lay.ranges));
    if ((e = hipGetLastError())) return e;
  }
  return hipSuccess;
}

}  // namespace lsplat
