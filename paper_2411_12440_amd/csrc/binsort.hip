// Binning: (tile, depth) ordering of the (tile, splat) intersections.
//
// Decomposition (an LSD radix sort split at the duplication step):
//   1. depth presort   stable LSD radix sort of the M (camera, splat) pairs by
//                      their 32-bit depth key; ties keep pair order.  Culled
//                      pairs carry key 0xFFFFFFFF and land at the end.
//   2. scan            exclusive scan (int64) of tiles-touched in that order;
//                      the total is the intersection count.  The scan also
//                      records which pair owns the first entry of every span
//                      of kKeygenSpan output entries.
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
// Depth chunks.  With K > 1 chunks, steps 3-5 run once per chunk of the
// depth order (pair positions [pos_c, pos_c+1)), from the rasterizer, and a
// chunk only emits entries for tiles that still have a pixel whose
// transmittance has not run out.  Each tile's list is then the concatenation
// of its chunk segments: a prefix of the complete list that holds every entry
// the composite can reach.  A per-camera summed-area table of the alive
// tiles lets each pair count its alive tiles in O(1) (count, scan, write),
// so the chunk's entries keep exactly the (tile, depth, pair id) order and
// pairs whose rectangle holds no alive tile cost four loads.
//
// Radix passes: 8-bit digits, reduce-then-scan with a fixed grid of G blocks
// (each owning a contiguous span, so the order is stable), 256 threads per
// block, 4096-key tiles; wave64 ballot matching ranks keys inside a wave,
// LDS staging turns the scatter into runs of consecutive addresses per digit.
// Counts and bases may live in device memory, so no launch shape depends on
// a value the host has not seen.
#include <algorithm>

#include "internal.h"

namespace lsplat {

namespace {

constexpr int kKeygenThreads = 256;
constexpr int kKeygenBlocks = 4096;
constexpr int kRangeThreads = 256;
constexpr int kScanBlocksMax = kMaxScanBlocks;

__device__ __forceinline__ int64_t dev_or(const int64_t* p, int64_t v) { return p ? *p : v; }

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

// ---------------------------------------------------------------------------
// Radix sort passes over [base, base + n) of the key/value arrays.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kSortThreads) void radix_upsweep(const uint32_t* __restrict__ keys,
                                                              const int64_t* base_dev,
                                                              const int64_t* n_dev, int64_t n_host,
                                                              int shift, int G,
                                                              uint32_t* __restrict__ hist) {
  __shared__ uint32_t h[4][256];
  int tid = threadIdx.x, wave = tid >> 6;
  for (int i = tid; i < 4 * 256; i += kSortThreads) (&h[0][0])[i] = 0;
  __syncthreads();
  keys += dev_or(base_dev, 0);
  const int64_t n = dev_or(n_dev, n_host);
  int64_t beg, end;
  block_span(n, G, &beg, &end);
  // 16 independent loads in flight per thread per iteration
  for (int64_t tb = beg; tb < end; tb += kSortTile) {
    uint32_t k[kSortItems];
#pragma unroll
    for (int j = 0; j < kSortItems; ++j) {
      const int64_t i = tb + j * kSortThreads + tid;
      k[j] = i < end ? keys[i] : 0xFFFFFFFFu;
    }
#pragma unroll
    for (int j = 0; j < kSortItems; ++j)
      if (tb + j * kSortThreads + tid < end) atomicAdd(&h[wave][(k[j] >> shift) & 255u], 1u);
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
    uint32_t* __restrict__ keys_out, uint32_t* __restrict__ vals_out, const int64_t* base_dev,
    const int64_t* n_dev, int64_t n_host, int shift, int G, const uint32_t* __restrict__ hist,
    const uint32_t* __restrict__ tot, const ushort4* __restrict__ grect_src,
    ushort4* __restrict__ grect_dst) {
  __shared__ uint32_t s_base[256];
  __shared__ uint32_t s_wcnt[4][256];
  __shared__ uint32_t s_tstart[256];
  __shared__ uint32_t s_tmp[4];
  __shared__ uint32_t s_keys[kSortTile];
  __shared__ uint32_t s_vals[kSortTile];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t base_off = dev_or(base_dev, 0);
  keys_in += base_off;
  if (!kIdentVals) vals_in += base_off;
  if (kWriteKeys) keys_out += base_off;
  vals_out += base_off;
  const int64_t n = dev_or(n_dev, n_host);
  int64_t beg, end;
  block_span(n, G, &beg, &end);
  // running global base of each digit for this block
  {
    uint32_t t = tot[tid];
    uint32_t ex = block_excl_scan_256(t, s_tmp, nullptr);
    s_base[tid] = ex + hist[(int64_t)tid * G + blockIdx.x];
  }
  // the next tile's keys and values are loaded while this one is ranked
  uint32_t nk[kSortItems], nv[kSortItems];
  auto load_tile = [&](int64_t t0) {
    const int c = (int)((end - t0) < kSortTile ? (end - t0) : kSortTile);
#pragma unroll
    for (int j = 0; j < kSortItems; ++j) {
      const int idx = wave * (64 * kSortItems) + j * 64 + lane;
      const bool valid = idx < c;
      nk[j] = valid ? keys_in[t0 + idx] : 0u;
      if (kIdentVals) nv[j] = (uint32_t)(t0 + idx);
      else nv[j] = valid ? vals_in[t0 + idx] : 0u;
    }
  };
  if (beg < end) load_tile(beg);
  for (int64_t tb = beg; tb < end; tb += kSortTile) {
    const int cnt = (int)((end - tb) < kSortTile ? (end - tb) : kSortTile);
#pragma unroll
    for (int w = 0; w < 4; ++w) s_wcnt[w][tid] = 0;
    __syncthreads();
    uint32_t k[kSortItems], v[kSortItems], r[kSortItems], lead[kSortItems], base[kSortItems];
#pragma unroll
    for (int j = 0; j < kSortItems; ++j) {
      k[j] = nk[j];
      v[j] = nv[j];
    }
    if (tb + kSortTile < end) load_tile(tb + kSortTile);
    // Rank every key among the wave's keys of the same digit: ballot matching
    // finds the lanes that share the digit; the lowest of them (the leader)
    // adds the group's size to the wave's running count of that digit with
    // an LDS atomic that returns the count before the add.  The atomics
    // do not wait for each other (one wave's LDS operations complete in
    // order), and the leaders' results are broadcast afterwards.
#pragma unroll
    for (int j = 0; j < kSortItems; ++j) {
      const int idx = wave * (64 * kSortItems) + j * 64 + lane;
      const bool valid = idx < cnt;
      const uint32_t key = k[j];
      const uint32_t d = (key >> shift) & 255u;
      uint64_t m = __builtin_amdgcn_ballot_w64(valid);
#pragma unroll
      for (int b = 0; b < 8; ++b) {
        const bool bit = (d >> b) & 1u;
        const uint64_t bb = __builtin_amdgcn_ballot_w64(bit);
        m &= bit ? bb : ~bb;
      }
      // lanes below this one with the same digit
      const uint32_t pre = __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                                     __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
      base[j] = 0;
      if (valid && pre == 0) base[j] = atomicAdd(&s_wcnt[wave][d], (uint32_t)__popcll(m));
      lead[j] = m ? (uint32_t)__builtin_ctzll(m) : 0u;
      r[j] = pre;
    }
#pragma unroll
    for (int j = 0; j < kSortItems; ++j) r[j] += (uint32_t)__shfl((int)base[j], (int)lead[j], 64);
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
          const uint32_t val = s_vals[p];
          if (kWriteKeys) keys_out[gpos] = key;
          vals_out[gpos] = val;
          if (grect_dst) grect_dst[gpos] = grect_src[val];   // per-pair data in the new order
        }
      }
    }
    __syncthreads();
    s_base[tid] += dtot;
  }
}

// ---------------------------------------------------------------------------
// Three-kernel exclusive scan (per-block sums, one block scans the sums, each
// block rescans its span) over inputs given by an accessor.
// ---------------------------------------------------------------------------
// tiles in a rectangle (an empty rectangle marks a culled pair)
__device__ __forceinline__ uint32_t rect_tiles(ushort4 r) {
  return (r.z >= r.x && r.w >= r.y) ? (uint32_t)(r.z - r.x + 1) * (uint32_t)(r.w - r.y + 1) : 0u;
}

struct PairCount {          // tiles touched by the pair at depth position p
  const ushort4* drect;
  __device__ int64_t operator()(int64_t p) const { return (int64_t)rect_tiles(drect[p]); }
};

struct SpanCount {
  const uint32_t* cnt;
  __device__ int64_t operator()(int64_t s) const { return (int64_t)cnt[s]; }
};

__device__ __forceinline__ void scan_span(int64_t n, int B, int64_t* beg, int64_t* end) {
  const int64_t unit = kScanThreads * 16;
  int64_t units = (n + unit - 1) / unit;
  int64_t per = (units + B - 1) / B;
  int64_t b = (int64_t)blockIdx.x * per * unit;
  *beg = b < n ? b : n;
  int64_t e = b + per * unit;
  *end = e < n ? e : n;
}

template <class In>
__global__ __launch_bounds__(kScanThreads) void scan_reduce(In in, const int64_t* n_dev,
                                                            int64_t n_host, int B,
                                                            int64_t* __restrict__ part) {
  __shared__ int64_t s[kScanThreads / 64];
  const int64_t n = dev_or(n_dev, n_host);
  int64_t beg, end;
  scan_span(n, B, &beg, &end);
  int64_t acc = 0;
  for (int64_t p = beg + threadIdx.x; p < end; p += kScanThreads) acc += in(p);
  for (int d = 32; d > 0; d >>= 1) acc += __shfl_xor(acc, d, 64);
  if ((threadIdx.x & 63) == 0) s[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    int64_t t = 0;
    for (int w = 0; w < kScanThreads / 64; ++w) t += s[w];
    part[blockIdx.x] = t;
  }
}

// exclusive scan of part[0..B) in place (B <= 1024); part[B] = total
__global__ __launch_bounds__(1024) void scan_parts(int64_t* __restrict__ part, int B) {
  __shared__ int64_t s_w[16];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t v = tid < B ? part[tid] : 0;
  int64_t x = v;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    int64_t y = __shfl_up(x, d, 64);
    if (lane >= d) x += y;
  }
  if (lane == 63) s_w[wave] = x;
  __syncthreads();
  int64_t wbase = 0, tot = 0;
  for (int w = 0; w < 16; ++w) {
    if (w < wave) wbase += s_w[w];
    tot += s_w[w];
  }
  if (tid < B) part[tid] = wbase + x - v;
  if (tid == 0) part[B] = tot;
}

// pair scan output: offsets, and the owner pair of every keygen span
struct PairOffsets {
  int64_t* isect_off;
  uint32_t* span_owner;
  int64_t n_spans;
  const int64_t* total;   // part[B]
  __device__ void operator()(int64_t p, int64_t base, int64_t v) const {
    isect_off[p] = base;
    if (v > 0) {
      for (int64_t sp = (base + kKeygenSpan - 1) / kKeygenSpan;
           sp * kKeygenSpan < base + v && sp < n_spans; ++sp)
        span_owner[sp] = (uint32_t)p;
      const int64_t n_total = *total;
      if (base + v == n_total) {
        const int64_t term = (n_total + kKeygenSpan - 1) / kKeygenSpan;
        if (term < n_spans) span_owner[term] = (uint32_t)p;
      }
    }
  }
};

// chunk mode: each pair's offset inside the chunk, and for every span of
// kChunkSpan output entries the (chunk-local) pair that owns its first entry;
// the pair owning the chunk's last entry is also recorded one span further,
// so span s always finds its pairs between owner[s] and owner[s + 1]
struct ChunkOffsets {
  uint32_t* off;
  uint32_t* owner;
  int64_t n_spans;
  const int64_t* total;
  __device__ void operator()(int64_t q, int64_t base, int64_t v) const {
    off[q] = (uint32_t)base;
    if (v > 0) {
      for (int64_t sp = (base + kChunkSpan - 1) / kChunkSpan; sp * kChunkSpan < base + v && sp < n_spans;
           ++sp)
        owner[sp] = (uint32_t)q;
      const int64_t n_total = *total;
      if (base + v == n_total) {
        const int64_t term = (n_total + kChunkSpan - 1) / kChunkSpan;
        if (term < n_spans) owner[term] = (uint32_t)q;
      }
    }
  }
};

template <class In, class Out>
__global__ __launch_bounds__(kScanThreads) void scan_down(In in, Out out, const int64_t* n_dev,
                                                          int64_t n_host, int B,
                                                          const int64_t* __restrict__ part) {
  __shared__ int64_t s_w[kScanThreads / 64];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t n = dev_or(n_dev, n_host);
  int64_t beg, end;
  scan_span(n, B, &beg, &end);
  int64_t run = part[blockIdx.x];
  constexpr int kPer = 16;
  for (int64_t tb = beg; tb < end; tb += kScanThreads * kPer) {
    int64_t v[kPer];
    int64_t sum = 0;
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
      int64_t p = tb + (int64_t)tid * kPer + k;
      v[k] = p < end ? in(p) : 0;
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
      if (p < end) out(p, base, v[k]);
      base += v[k];
    }
    run += tot;
  }
}

// After the pair scan: total intersections, and (complete-list mode) the
// single chunk's count clamped to the capacity.
// The span table must cover every span of the complete lists (plus the
// terminal entry); otherwise the run is flagged as an overflow and no list is
// built.
__global__ void pairs_finalize(const int64_t* __restrict__ total, int64_t M,
                               int64_t* __restrict__ isect_off, int64_t* __restrict__ n_isect,
                               int64_t* __restrict__ chunk_base, int64_t* __restrict__ chunk_n,
                               int32_t* __restrict__ flags, int64_t cap, int64_t n_spans,
                               int full_lists) {
  if (threadIdx.x != 0) return;
  const int64_t n = *total;
  isect_off[M] = n;
  *n_isect = n;
  chunk_base[0] = 0;
  const bool covered = !full_lists || (n + kKeygenSpan - 1) / kKeygenSpan + 1 < n_spans;
  flags[0] = covered ? 0 : 1;
  if (full_lists) {
    const bool ok = covered && n <= cap;
    chunk_n[0] = ok ? n : 0;
    chunk_base[1] = ok ? n : 0;
    if (!ok) flags[0] = 1;
  }
}

// ---------------------------------------------------------------------------
// Key generation.  One block iteration covers the output entries of one span
// [s * kKeygenSpan, (s + 1) * kKeygenSpan); every entry learns its pair from
// an LDS max-scan of the pairs' start positions and its tile from its offset
// inside the pair's tile rectangle.
// ---------------------------------------------------------------------------
struct SpanTables {
  int32_t owner[kKeygenSpan];
  int64_t off[kKeygenSpan];
  uint32_t m[kKeygenSpan];
  uint32_t gbase[kKeygenSpan];
  uint32_t w[kKeygenSpan];
  uint32_t gx[kKeygenSpan];
  int64_t plo, phi;
  int32_t wmax[kKeygenThreads / 64];
  int32_t wcnt[kKeygenThreads / 64];
};

__device__ __forceinline__ int cam_of_pair(const CamInfo* cams, int C, int64_t m) {
  int lo = 0, hi = C - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (cams[mid].pair_off <= m) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// Fill the tables for span s (entries k0 = s * span ...).  Block-uniform.
__device__ __forceinline__ void span_setup(SpanTables& t, int64_t s,
                                           const uint32_t* __restrict__ order,
                                           const int64_t* __restrict__ isect_off,
                                           const ushort4* __restrict__ rect,
                                           const CamInfo* __restrict__ cams, int C, int64_t M,
                                           const uint32_t* __restrict__ span_owner) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t k0 = s * kKeygenSpan;
  if (tid == 0) {
    int64_t lo = span_owner[s], hi = span_owner[s + 1];
    if (lo > M - 1) lo = M - 1;
    if (hi > M - 1) hi = M - 1;
    if (hi < lo) hi = lo;
    t.plo = lo;
    t.phi = hi;
  }
  for (int i = tid; i < kKeygenSpan; i += kKeygenThreads) t.owner[i] = 0;
  __syncthreads();
  const int64_t plo = t.plo, phi = t.phi;
  for (int64_t p = plo + tid; p <= phi && p - plo < kKeygenSpan; p += kKeygenThreads) {
    const int pl = (int)(p - plo);
    const int64_t off = isect_off[p];
    uint32_t m = order[p];
    if (m >= (uint64_t)M) m = 0;   // unreachable for a valid order
    const ushort4 rc = rect[m];
    const int c = cam_of_pair(cams, C, (int64_t)m);
    const CamInfo& ci = cams[c];
    t.off[pl] = off;
    t.m[pl] = m;
    t.gbase[pl] = (uint32_t)(ci.tile_off + (int64_t)rc.y * ci.GX + rc.x);
    t.w[pl] = (uint32_t)(rc.z - rc.x + 1);
    t.gx[pl] = (uint32_t)ci.GX;
    if (p > plo && off > k0 && off < k0 + kKeygenSpan) t.owner[(int)(off - k0)] = pl;
  }
  __syncthreads();
  // inclusive max-scan of owner: each entry learns its pair
  constexpr int kPer = kKeygenSpan / kKeygenThreads;
  int32_t loc[kPer];
  int32_t mx = 0;
#pragma unroll
  for (int k = 0; k < kPer; ++k) {
    int32_t o = t.owner[tid * kPer + k];
    mx = o > mx ? o : mx;
    loc[k] = mx;
  }
  int32_t x = mx;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    int32_t y = __shfl_up(x, d, 64);
    if (lane >= d) x = y > x ? y : x;
  }
  if (lane == 63) t.wmax[wave] = x;
  int32_t ex = __shfl_up(x, 1, 64);
  if (lane == 0) ex = 0;
  __syncthreads();
  int32_t wpre = 0;
  for (int w = 0; w < wave; ++w) wpre = t.wmax[w] > wpre ? t.wmax[w] : wpre;
  ex = ex > wpre ? ex : wpre;
#pragma unroll
  for (int k = 0; k < kPer; ++k) t.owner[tid * kPer + k] = loc[k] > ex ? loc[k] : ex;
  __syncthreads();
}

// global tile id and pair id of entry k0 + i
__device__ __forceinline__ void span_entry(const SpanTables& t, int64_t k0, int i,
                                           uint32_t* gtile, uint32_t* m) {
  const int pl = t.owner[i];
  const uint32_t local = (uint32_t)(k0 + i - t.off[pl]);
  const uint32_t w = t.w[pl];
  // local / w with a float estimate corrected to the exact quotient
  uint32_t ty = (uint32_t)((float)local * __builtin_amdgcn_rcpf((float)w));
  int32_t rem = (int32_t)local - (int32_t)(ty * w);
  while (rem < 0) { --ty; rem += (int32_t)w; }
  while (rem >= (int32_t)w) { ++ty; rem -= (int32_t)w; }
  *gtile = t.gbase[pl] + ty * t.gx[pl] + (uint32_t)rem;
  *m = t.m[pl];
}

// complete lists: every entry, at its own index
__global__ __launch_bounds__(kKeygenThreads) void keygen_kernel(
    const uint32_t* __restrict__ order, const int64_t* __restrict__ isect_off,
    const ushort4* __restrict__ rect, const CamInfo* __restrict__ cams, int C, int64_t M,
    const int64_t* __restrict__ n_dev, const uint32_t* __restrict__ span_owner,
    uint32_t* __restrict__ keys, uint32_t* __restrict__ vals) {
  __shared__ SpanTables t;
  const int64_t n = *n_dev;
  for (int64_t s = blockIdx.x; s * kKeygenSpan < n; s += gridDim.x) {
    span_setup(t, s, order, isect_off, rect, cams, C, M, span_owner);
    const int64_t k0 = s * kKeygenSpan;
    const int cnt = (int)((n - k0) < kKeygenSpan ? (n - k0) : kKeygenSpan);
    for (int i = threadIdx.x; i < cnt; i += kKeygenThreads) {
      uint32_t g, m;
      span_entry(t, k0, i, &g, &m);
      keys[k0 + i] = g;
      vals[k0 + i] = m;
    }
    __syncthreads();
  }
}

// Per-camera inclusive summed-area table of the alive flags (one block per
// camera): sat[t] counts the alive tiles in the rectangle from the camera's
// first tile to t.
// inclusive prefix sum over a wave (lane i receives x_0 + ... + x_i)
__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t x, int lane) {
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const uint32_t y = __shfl_up(x, d, 64);
    if (lane >= d) x += y;
  }
  return x;
}

// Per-camera inclusive summed-area table of the alive flags, in two passes of
// one wave per line: prefix sums along each tile row, then down each tile
// column.  Grid: (ceil(max lines / 4), cameras), 4 waves per block.
__global__ __launch_bounds__(256) void alive_sat_rows(const CamInfo* __restrict__ cams,
                                                      const uint32_t* __restrict__ alive,
                                                      uint32_t* __restrict__ sat) {
  const CamInfo& ci = cams[blockIdx.y];
  const int lane = threadIdx.x & 63;
  const int r = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (r >= ci.GY) return;
  const uint32_t* A = alive + ci.tile_off + (int64_t)r * ci.GX;
  uint32_t* S = sat + ci.tile_off + (int64_t)r * ci.GX;
  uint32_t carry = 0;
  for (int x0 = 0; x0 < ci.GX; x0 += 64) {
    const int x = x0 + lane;
    const uint32_t v = (x < ci.GX && A[x] != 0u) ? 1u : 0u;
    const uint32_t inc = wave_incl_scan(v, lane) + carry;
    if (x < ci.GX) S[x] = inc;
    carry = __shfl(inc, 63, 64);
  }
}

__global__ __launch_bounds__(256) void alive_sat_cols(const CamInfo* __restrict__ cams,
                                                      uint32_t* __restrict__ sat) {
  const CamInfo& ci = cams[blockIdx.y];
  const int lane = threadIdx.x & 63;
  const int x = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (x >= ci.GX) return;
  uint32_t* S = sat + ci.tile_off + x;
  uint32_t carry = 0;
  for (int y0 = 0; y0 < ci.GY; y0 += 64) {
    const int y = y0 + lane;
    const uint32_t v = y < ci.GY ? S[(int64_t)y * ci.GX] : 0u;
    const uint32_t inc = wave_incl_scan(v, lane) + carry;
    if (y < ci.GY) S[(int64_t)y * ci.GX] = inc;
    carry = __shfl(inc, 63, 64);
  }
}

// The alive flags one bit per tile, in global tile id order (bit t & 31 of
// word t >> 5), one wave per 64 tiles; the grid has one more wave, which
// writes the two zero words past the end.
__global__ __launch_bounds__(256) void alive_bits_kernel(const uint32_t* __restrict__ alive,
                                                         int64_t T, int64_t nwaves,
                                                         uint32_t* __restrict__ abits) {
  const int lane = threadIdx.x & 63;
  const int64_t w = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (w >= nwaves) return;
  const int64_t t = w * 64 + lane;
  const uint64_t b = __builtin_amdgcn_ballot_w64(t < T && alive[t] != 0u);
  if (lane == 0) {
    abits[2 * w] = (uint32_t)b;
    abits[2 * w + 1] = (uint32_t)(b >> 32);
  }
}

// alive bits of the n <= 32 tiles t, t + 1, ... (bit i: tile t + i)
__device__ __forceinline__ uint32_t alive_run(const uint32_t* __restrict__ abits, uint32_t t,
                                              uint32_t n) {
  const uint32_t i = t >> 5;
  const uint64_t v = ((uint64_t)abits[i + 1] << 32) | abits[i];
  const uint32_t x = (uint32_t)(v >> (t & 31u));
  return n >= 32u ? x : x & ((1u << n) - 1u);
}

__device__ __forceinline__ uint32_t sat_query(const uint32_t* S, int GX, int x0, int y0, int x1,
                                              int y1) {
  auto at = [&](int x, int y) -> uint32_t {
    return (x < 0 || y < 0) ? 0u : S[(int64_t)y * GX + x];
  };
  return at(x1, y1) - at(x0 - 1, y1) - at(x1, y0 - 1) + at(x0 - 1, y0 - 1);
}

// Chunk c of the depth order (pair positions [lo, hi)): for each pair the
// number of alive tiles in its rectangle (from the summed-area table), and a
// mask that tells the writer where they are: all ones when every tile is
// alive; for a partly alive rectangle of at most kSmallRect tiles, bit j is
// tile j (row-major) of the rectangle; 0 for a larger partly alive one (the
// second write kernel writes it) or an empty count.
constexpr int kSmallRect = 32;

__global__ __launch_bounds__(256) void chunk_count_kernel(
    const uint32_t* __restrict__ order, const ushort4* __restrict__ drect,
    const CamInfo* __restrict__ cams, int C, int64_t M, int64_t lo, int64_t hi,
    const uint32_t* __restrict__ sat, const uint32_t* __restrict__ abits,
    const int32_t* __restrict__ flags, uint32_t* __restrict__ pcnt,
    uint32_t* __restrict__ pmask) {
  const int64_t p = lo + (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (p >= hi) return;
  uint32_t k = 0, mask = 0;
  const ushort4 r = drect[p];
  const uint32_t area = rect_tiles(r);
  if (flags[0] == 0 && area != 0) {
    uint32_t m = order[p];
    if (m >= (uint64_t)M) m = 0;
    const CamInfo& ci = cams[cam_of_pair(cams, C, (int64_t)m)];
    k = sat_query(sat + ci.tile_off, ci.GX, r.x, r.y, r.z, r.w);
    if (k == area) {
      mask = 0xFFFFFFFFu;                  // every tile alive
    } else if (k != 0 && area <= (uint32_t)kSmallRect) {
      const uint32_t w = (uint32_t)(r.z - r.x + 1);
      uint32_t t = (uint32_t)(ci.tile_off + (int64_t)r.y * ci.GX + r.x);
      for (uint32_t j = 0; j < area; j += w, t += (uint32_t)ci.GX) mask |= alive_run(abits, t, w) << j;
    }
  }
  pcnt[p - lo] = k;
  pmask[p - lo] = mask;
}

// position of the k-th (from 0) set bit of x; requires k < popcount(x)
__device__ __forceinline__ uint32_t select_bit(uint32_t x, uint32_t k) {
  uint32_t pos = 0, c;
  c = (uint32_t)__popc(x & 0xFFFFu);
  if (k >= c) { k -= c; x >>= 16; pos += 16; }
  c = (uint32_t)__popc(x & 0xFFu);
  if (k >= c) { k -= c; x >>= 8; pos += 8; }
  c = (uint32_t)__popc(x & 0xFu);
  if (k >= c) { k -= c; x >>= 4; pos += 4; }
  c = (uint32_t)__popc(x & 0x3u);
  if (k >= c) { k -= c; x >>= 2; pos += 2; }
  c = x & 1u;
  if (k >= c) pos += 1;
  return pos;
}

// q / w for q < 2^24, w >= 1: a float estimate corrected to the exact quotient
__device__ __forceinline__ uint32_t div_small(uint32_t q, uint32_t w, uint32_t* rem) {
  uint32_t d = (uint32_t)((float)q * __builtin_amdgcn_rcpf((float)w));
  int32_t r = (int32_t)q - (int32_t)(d * w);
  while (r < 0) { --d; r += (int32_t)w; }
  while (r >= (int32_t)w) { ++d; r -= (int32_t)w; }
  *rem = (uint32_t)r;
  return d;
}

// Write the chunk's entries at their scanned offsets, pairs in depth order, so
// the chunk's entries keep the relative order of the complete lists.  Each
// block iteration owns a span of kChunkSpan output entries: the span's owning
// pairs are found between two entries of the span-owner table (skipping the
// pairs with no alive tile), their start positions marked in LDS, and an LDS
// max-scan gives every entry its pair; the entry's tile is its rank among the
// pair's alive tiles (the mask), and consecutive threads write consecutive
// entries.  Entries of a large, partly alive rectangle are left to
// chunk_write_big_kernel.
struct ChunkSpan {
  uint32_t slot[kChunkSpan];
  uint32_t off[kChunkSpan], mask[kChunkSpan], m[kChunkSpan], gbase[kChunkSpan], wgx[kChunkSpan];
  int32_t wmax[4];
};

__device__ __forceinline__ void chunk_span_pair(ChunkSpan& t, int sl, int64_t q, int64_t lo,
                                                const uint32_t* __restrict__ order,
                                                const ushort4* __restrict__ drect,
                                                const CamInfo* __restrict__ cams, int C, int64_t M,
                                                const uint32_t* __restrict__ poff,
                                                const uint32_t* __restrict__ pmask) {
  uint32_t m = order[lo + q];
  if (m >= (uint64_t)M) m = 0;
  const ushort4 rc = drect[lo + q];
  const CamInfo& ci = cams[cam_of_pair(cams, C, (int64_t)m)];
  t.off[sl] = poff[q];
  t.mask[sl] = pmask[q];
  t.m[sl] = m;
  t.gbase[sl] = (uint32_t)(ci.tile_off + (int64_t)rc.y * ci.GX + rc.x);
  t.wgx[sl] = (uint32_t)(rc.z - rc.x + 1) | ((uint32_t)ci.GX << 16);
}

__global__ __launch_bounds__(256) void chunk_write_span_kernel(
    const uint32_t* __restrict__ order, const ushort4* __restrict__ drect,
    const CamInfo* __restrict__ cams, int C, int64_t M, int64_t lo, int64_t hi,
    const uint32_t* __restrict__ pcnt, const uint32_t* __restrict__ poff,
    const uint32_t* __restrict__ pmask, const uint32_t* __restrict__ owner, int64_t n_spans,
    const int64_t* __restrict__ chunk_base, const int64_t* __restrict__ chunk_n,
    uint32_t* __restrict__ keys, uint32_t* __restrict__ vals) {
  __shared__ ChunkSpan t;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t n = *chunk_n;
  const int64_t base = *chunk_base;
  const int64_t np = hi - lo;
  for (int64_t s = blockIdx.x; s * kChunkSpan < n && s + 1 < n_spans; s += gridDim.x) {
    const int64_t k0 = s * kChunkSpan;
    const int cnt = (int)((n - k0) < kChunkSpan ? (n - k0) : kChunkSpan);
    int64_t qa = owner[s], qb = owner[s + 1];
    if (qa > np - 1) qa = np - 1;
    if (qb > np - 1) qb = np - 1;
    if (qb < qa) qb = qa;
    for (int i = tid; i < kChunkSpan; i += 256) t.slot[i] = 0;
    if (tid == 0) chunk_span_pair(t, 0, qa, lo, order, drect, cams, C, M, poff, pmask);
    __syncthreads();
    for (int64_t q = qa + 1 + tid; q <= qb; q += 256) {
      if (pcnt[q] == 0) continue;
      const int64_t o = (int64_t)poff[q];
      if (o <= k0 || o >= k0 + kChunkSpan) continue;
      const int sl = (int)(o - k0);
      t.slot[sl] = (uint32_t)sl;
      chunk_span_pair(t, sl, q, lo, order, drect, cams, C, M, poff, pmask);
    }
    __syncthreads();
    // inclusive max-scan of the start marks: entry i's pair is at slot[i]
    constexpr int kPer = kChunkSpan / 256;
    uint32_t loc[kPer];
    uint32_t mx = 0;
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
      const uint32_t o = t.slot[tid * kPer + k];
      mx = o > mx ? o : mx;
      loc[k] = mx;
    }
    uint32_t x = mx;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
      const uint32_t y = __shfl_up(x, d, 64);
      if (lane >= d) x = y > x ? y : x;
    }
    if (lane == 63) t.wmax[wave] = (int32_t)x;
    uint32_t ex = __shfl_up(x, 1, 64);
    if (lane == 0) ex = 0;
    __syncthreads();
    for (int w = 0; w < wave; ++w) ex = (uint32_t)t.wmax[w] > ex ? (uint32_t)t.wmax[w] : ex;
#pragma unroll
    for (int k = 0; k < kPer; ++k) t.slot[tid * kPer + k] = loc[k] > ex ? loc[k] : ex;
    __syncthreads();
    for (int i = tid; i < cnt; i += 256) {
      const uint32_t sl = t.slot[i];
      const uint32_t mask = t.mask[sl];
      if (mask == 0u) continue;            // a large, partly alive rectangle
      const uint32_t local = (uint32_t)(k0 + i - (int64_t)t.off[sl]);
      const uint32_t pos = mask == 0xFFFFFFFFu ? local : select_bit(mask, local);
      const uint32_t wgx = t.wgx[sl];
      uint32_t tx;
      const uint32_t ty = div_small(pos, wgx & 0xFFFFu, &tx);
      keys[base + k0 + i] = t.gbase[sl] + ty * (wgx >> 16) + tx;
      vals[base + k0 + i] = t.m[sl];
    }
    __syncthreads();
  }
}

// The large, partly alive rectangles of the chunk.  A block collects those of
// its 256 pairs, and each wave takes up to 64 of them.  The wave cuts their
// rows into units of up to 32 tiles (one word of the alive bits each),
// numbered rectangle after rectangle, and walks the units 64 at a time: each
// lane finds its unit's rectangle, reads the unit's alive bits and writes one
// entry per set bit.  A wave-wide scan of the bit counts numbers the entries
// of the wave's rectangles one after another (each rectangle's count is its
// number of alive tiles), which places every entry in its rectangle's range
// in row-major tile order.
__global__ __launch_bounds__(256) void chunk_write_big_kernel(
    const uint32_t* __restrict__ order, const ushort4* __restrict__ drect,
    const CamInfo* __restrict__ cams, int C, int64_t M, int64_t lo, int64_t hi,
    const uint32_t* __restrict__ abits, const uint32_t* __restrict__ pcnt,
    const uint32_t* __restrict__ poff, const uint32_t* __restrict__ pmask,
    const int64_t* __restrict__ chunk_base, const int64_t* __restrict__ chunk_n,
    uint32_t* __restrict__ keys, uint32_t* __restrict__ vals) {
  __shared__ uint32_t s_big[256];
  __shared__ int s_nbig;
  __shared__ uint32_t s_ustart[4][65];
  __shared__ uint32_t s_row0[4][64], s_gx[4][64], s_w[4][64], s_nseg[4][64], s_m[4][64];
  __shared__ int64_t s_dst[4][64];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  if (*chunk_n == 0) return;
  if (tid == 0) s_nbig = 0;
  __syncthreads();
  const int64_t p0 = lo + (int64_t)blockIdx.x * 256 + tid;
  if (p0 < hi && pcnt[p0 - lo] > 0 && pmask[p0 - lo] == 0u)
    s_big[atomicAdd(&s_nbig, 1)] = (uint32_t)p0;
  __syncthreads();
  const int nbig = s_nbig;
  const int64_t base = *chunk_base;
  {
    const int b = wave * 64 + lane;
    if (wave * 64 >= nbig) return;
    uint32_t units = 0, k = 0;
    int64_t dst = 0;
    if (b < nbig) {
      const uint32_t q = s_big[b];
      uint32_t m = order[q];
      if (m >= (uint64_t)M) m = 0;
      const ushort4 r = drect[q];
      const CamInfo& ci = cams[cam_of_pair(cams, C, (int64_t)m)];
      const uint32_t w = (uint32_t)(r.z - r.x + 1), h = (uint32_t)(r.w - r.y + 1);
      const uint32_t nseg = (w + 31u) >> 5;
      units = h * nseg;
      k = pcnt[q - lo];
      dst = base + (int64_t)poff[q - lo];
      s_row0[wave][lane] = (uint32_t)(ci.tile_off + (int64_t)r.y * ci.GX + r.x);
      s_gx[wave][lane] = (uint32_t)ci.GX;
      s_w[wave][lane] = w;
      s_nseg[wave][lane] = nseg;
      s_m[wave][lane] = m;
    }
    // exclusive scans over the wave of the units and of the entries
    uint32_t xu = units, xk = k;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
      const uint32_t yu = (uint32_t)__shfl_up((int)xu, d, 64), yk = (uint32_t)__shfl_up((int)xk, d, 64);
      if (lane >= d) {
        xu += yu;
        xk += yk;
      }
    }
    const uint32_t U = (uint32_t)__shfl((int)xu, 63, 64);
    s_ustart[wave][lane] = xu - units;
    if (lane == 63) s_ustart[wave][64] = U;
    s_dst[wave][lane] = dst - (int64_t)(xk - k);   // entry f of the batch: s_dst[j] + f
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    uint32_t run = 0;   // entries of the batch before this step's
    for (uint32_t u0 = 0; u0 < U; u0 += 64u) {
      const uint32_t u = u0 + (uint32_t)lane;
      uint32_t bits = 0, t0 = 0, j = 0;
      if (u < U) {
        // the rectangle holding unit u: the last j with ustart[j] <= u
#pragma unroll
        for (uint32_t hstep = 32; hstep > 0; hstep >>= 1)
          if (s_ustart[wave][j + hstep] <= u) j += hstep;
        uint32_t seg;
        const uint32_t ty = div_small(u - s_ustart[wave][j], s_nseg[wave][j], &seg);
        const uint32_t x = seg << 5;
        t0 = s_row0[wave][j] + ty * s_gx[wave][j] + x;
        bits = alive_run(abits, t0, s_w[wave][j] - x);
      }
      const uint32_t c = (uint32_t)__popc(bits);
      uint32_t xc = c;
#pragma unroll
      for (int d = 1; d < 64; d <<= 1) {
        const uint32_t y = (uint32_t)__shfl_up((int)xc, d, 64);
        if (lane >= d) xc += y;
      }
      if (bits) {
        int64_t at = s_dst[wave][j] + (int64_t)(run + xc - c);
        const uint32_t mm = s_m[wave][j];
        // single entries up to a 16-byte boundary, then four per store
        while (bits && (at & 3)) {
          keys[at] = t0 + (uint32_t)__builtin_ctz(bits);
          vals[at] = mm;
          ++at;
          bits &= bits - 1u;
        }
        while (__popc(bits) >= 4) {
          uint32_t e[4];
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            e[q] = t0 + (uint32_t)__builtin_ctz(bits);
            bits &= bits - 1u;
          }
          *reinterpret_cast<uint4*>(keys + at) = make_uint4(e[0], e[1], e[2], e[3]);
          *reinterpret_cast<uint4*>(vals + at) = make_uint4(mm, mm, mm, mm);
          at += 4;
        }
        while (bits) {
          keys[at] = t0 + (uint32_t)__builtin_ctz(bits);
          vals[at] = mm;
          ++at;
          bits &= bits - 1u;
        }
      }
      run += (uint32_t)__shfl((int)xc, 63, 64);
    }
  }
}

// After the span-count scan of chunk c: the chunk's entry count, its base and
// the capacity check.  A chunk that would overflow is dropped (count 0) and
// the overflow flag raised; later chunks then see no room either.
__global__ void chunk_finalize(const int64_t* __restrict__ total, int64_t* __restrict__ chunk_base,
                               int64_t* __restrict__ chunk_n, int32_t* __restrict__ flags,
                               int64_t cap) {
  if (threadIdx.x != 0) return;
  const int64_t n = *total;
  const int64_t b = chunk_base[0];
  const bool ok = flags[0] == 0 && b + n <= cap;
  chunk_n[0] = ok ? n : 0;
  chunk_base[1] = ok ? b + n : b;
  if (!ok && n > 0) flags[0] = 1;
}

__global__ void chunk_empty(int64_t* __restrict__ chunk_base, int64_t* __restrict__ chunk_n) {
  if (threadIdx.x != 0) return;
  chunk_n[0] = 0;
  chunk_base[1] = chunk_base[0];
}

// ranges[t] = number of sorted keys < t among keys[base, base + n), t in [0, T]
__global__ __launch_bounds__(kRangeThreads) void ranges_kernel(const uint32_t* __restrict__ keys,
                                                               const int64_t* __restrict__ base_dev,
                                                               const int64_t* __restrict__ n_dev,
                                                               int64_t T,
                                                               int64_t* __restrict__ ranges) {
  const int64_t n = *n_dev;
  keys += *base_dev;
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

// One LSD pass; returns the launch error.
template <bool kIdent, bool kWriteKeys>
hipError_t radix_pass(const char* const names[3], const uint32_t* kin, const uint32_t* vin,
                      uint32_t* kout, uint32_t* vout, const int64_t* base_dev,
                      const int64_t* n_dev, int64_t n_host, int shift, int G, uint32_t* hist,
                      uint32_t* tot, hipStream_t s, const ushort4* grect_src = nullptr,
                      ushort4* grect_dst = nullptr) {
  {
    ProfScope ps(names[0], s);
    hipLaunchKernelGGL(radix_upsweep, dim3(G), dim3(kSortThreads), 0, s, kin, base_dev, n_dev,
                       n_host, shift, G, hist);
  }
  {
    ProfScope ps(names[1], s);
    hipLaunchKernelGGL(radix_scan_rows, dim3(256), dim3(256), 0, s, hist, G, tot);
  }
  {
    ProfScope ps(names[2], s);
    hipLaunchKernelGGL((radix_downsweep<kIdent, kWriteKeys>), dim3(G), dim3(kSortThreads), 0, s,
                       kin, vin, kout, vout, base_dev, n_dev, n_host, shift, G, hist, tot,
                       grect_src, grect_dst);
  }
  return hipGetLastError();
}

const char* const kPreNames[3] = {"presort_upsweep", "presort_scan", "presort_downsweep"};
const char* const kTileNames[3] = {"tilesort_upsweep", "tilesort_scan", "tilesort_downsweep"};

int scan_blocks_for(int64_t n) {
  int64_t b = (n + kScanThreads * 16 - 1) / (kScanThreads * 16);
  return (int)std::max<int64_t>(1, std::min<int64_t>(b, kScanBlocksMax));
}

// Sort the entries [base, base + n) of (keys, vals) by tile id, then ranges.
hipError_t tile_sort_and_ranges(const Plan& p, char* ws, const int64_t* base_dev,
                                const int64_t* n_dev, int64_t* ranges_out, hipStream_t s) {
  hipError_t e;
  const int passes = (p.tile_bits + 7) / 8;
  uint32_t* kA = (uint32_t*)(ws + p.lay.keys);
  uint32_t* vA = (uint32_t*)(ws + p.lay.vals);
  uint32_t* kB = (uint32_t*)(ws + p.sort_keys_b);
  uint32_t* vB = (uint32_t*)(ws + p.sort_vals_b);
  uint32_t* hist = (uint32_t*)(ws + p.hist);
  uint32_t* tot = (uint32_t*)(ws + p.digit_tot);
  uint32_t *kin = (passes % 2 == 0) ? kA : kB, *vin = (passes % 2 == 0) ? vA : vB;
  for (int pass = 0; pass < passes; ++pass) {
    uint32_t* kout = (kin == kA) ? kB : kA;
    uint32_t* vout = (vin == vA) ? vB : vA;
    if ((e = radix_pass<false, true>(kTileNames, kin, vin, kout, vout, base_dev, n_dev, 0,
                                     8 * pass, p.sort_blocks, hist, tot, s)))
      return e;
    kin = kout;
    vin = vout;
  }
  int64_t blocks = std::min<int64_t>((p.T + 1 + kRangeThreads - 1) / kRangeThreads, 4096);
  ProfScope ps("ranges", s);
  hipLaunchKernelGGL(ranges_kernel, dim3((unsigned)blocks), dim3(kRangeThreads), 0, s, kA,
                     base_dev, n_dev, p.T, ranges_out);
  return hipGetLastError();
}

// Deterministic backward.  A stable LSD radix sort of the list entries by
// pair id (identity values first, so that a pair's entries keep ascending
// list positions) gives every entry a slot in pair order; the backward pass
// stores the entry's nine per-tile sums at partial[9 slot + f], and one
// thread per pair adds its contiguous slots in order.
__global__ __launch_bounds__(256) void det_slot_kernel(const uint32_t* __restrict__ pos,
                                                       const int64_t* __restrict__ n_dev,
                                                       uint32_t* __restrict__ slot) {
  const int64_t n = *n_dev;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
    slot[pos[i]] = (uint32_t)i;
}

// Pairs with at most kDetShort entries are summed by one thread in slot
// order; longer ones are queued and summed by one wave each: lane l adds the
// segment's slots l, l + 64, ..., then a fixed butterfly combines the lanes.
// Both rules depend only on the pair's own segment, so a pair's sum is the
// same wherever its segment lies (batched or per-view calls).
constexpr int kDetShort = 64;

__global__ void det_count_zero(uint32_t* __restrict__ cnt) {
  if (threadIdx.x == 0) cnt[0] = 0u;
}

__global__ __launch_bounds__(256) void det_reduce_short(
    const uint32_t* __restrict__ keys, const int64_t* __restrict__ n_dev,
    const double* __restrict__ partial, double* __restrict__ grad2d, int64_t M,
    uint32_t* __restrict__ long_start, uint32_t* __restrict__ long_cnt) {
  const int64_t n = *n_dev;
  const int64_t stride = (int64_t)gridDim.x * 256;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += stride) {
    const uint32_t m = keys[i];
    if (i > 0 && keys[i - 1] == m) continue;
    int64_t j = i + 1;
    while (j < n && j - i <= kDetShort && keys[j] == m) ++j;
    if (j - i > kDetShort) {
      long_start[atomicAdd(long_cnt, 1u)] = (uint32_t)i;
      continue;
    }
    double acc[kGrad2d];
#pragma unroll
    for (int f = 0; f < kGrad2d; ++f) acc[f] = 0.0;
    for (int64_t k = i; k < j; ++k) {
#pragma unroll
      for (int f = 0; f < kGrad2d; ++f) acc[f] += partial[k * kGrad2d + f];
    }
#pragma unroll
    for (int f = 0; f < kGrad2d; ++f) grad2d[(int64_t)f * M + m] = acc[f];
  }
}

__global__ __launch_bounds__(256) void det_reduce_long(
    const uint32_t* __restrict__ keys, const int64_t* __restrict__ n_dev,
    const double* __restrict__ partial, double* __restrict__ grad2d, int64_t M,
    const uint32_t* __restrict__ long_start, const uint32_t* __restrict__ long_cnt) {
  const int64_t n = *n_dev;
  const uint32_t nl = *long_cnt;
  const int lane = threadIdx.x & 63;
  const int64_t wave = ((int64_t)blockIdx.x * 256 + threadIdx.x) >> 6;
  const int64_t waves = ((int64_t)gridDim.x * 256) >> 6;
  for (int64_t w = wave; w < nl; w += waves) {
    const int64_t i = long_start[w];
    const uint32_t m = keys[i];
    double acc[kGrad2d];
#pragma unroll
    for (int f = 0; f < kGrad2d; ++f) acc[f] = 0.0;
    for (int64_t base = i;; base += 64) {
      const int64_t k = base + lane;
      const bool mine = k < n && keys[k] == m;
      if (mine) {
#pragma unroll
        for (int f = 0; f < kGrad2d; ++f) acc[f] += partial[k * kGrad2d + f];
      }
      // the segment is contiguous: once a lane falls outside it, it ends
      if (__builtin_amdgcn_ballot_w64(!mine) != 0ull) break;
    }
#pragma unroll
    for (int f = 0; f < kGrad2d; ++f)
      for (int d = 1; d < 64; d <<= 1) acc[f] += __shfl_xor(acc[f], d, 64);
    if (lane == 0) {
#pragma unroll
      for (int f = 0; f < kGrad2d; ++f) grad2d[(int64_t)f * M + m] = acc[f];
    }
  }
}

// The buffer the key generation writes to, so that the sort ends in (keys, vals).
void keygen_targets(const Plan& p, char* ws, uint32_t** k0, uint32_t** v0) {
  const int passes = (p.tile_bits + 7) / 8;
  *k0 = (uint32_t*)(ws + ((passes % 2 == 0) ? p.lay.keys : p.sort_keys_b));
  *v0 = (uint32_t*)(ws + ((passes % 2 == 0) ? p.lay.vals : p.sort_vals_b));
}

}  // namespace

static const char* const kDetNames[3] = {"detsort_upsweep", "detsort_scan", "detsort_downsweep"};

// buffers of the pair-order sort: sorted pair ids end in k[cur], the entry
// positions in v[cur], and the slot of every entry goes to v[cur ^ 1]
static int det_passes(const Plan& p) {
  int bits = 0;
  while (bits < 32 && ((p.M - 1) >> bits) > 0) ++bits;
  return std::max(1, (bits + 7) / 8);
}

const uint32_t* det_sorted_keys(const Plan& p, char* ws) {
  const int cur = (det_passes(p) - 1) & 1;
  return (const uint32_t*)(ws + (cur ? p.det_k1 : p.det_k0));
}

const uint32_t* det_slots(const Plan& p, char* ws) {
  const int cur = (det_passes(p) - 1) & 1;
  return (const uint32_t*)(ws + (cur ? p.det_v0 : p.det_v1));
}

hipError_t launch_det_order(const Plan& p, char* ws, hipStream_t s) {
  hipError_t e;
  const int64_t* n_dev = (const int64_t*)(ws + p.lay.chunk_base) + p.K;
  const int passes = det_passes(p);
  const uint32_t* vals = (const uint32_t*)(ws + p.lay.vals);
  uint32_t* kb[2] = {(uint32_t*)(ws + p.det_k0), (uint32_t*)(ws + p.det_k1)};
  uint32_t* vb[2] = {(uint32_t*)(ws + p.det_v0), (uint32_t*)(ws + p.det_v1)};
  uint32_t* hist = (uint32_t*)(ws + p.hist);
  uint32_t* tot = (uint32_t*)(ws + p.digit_tot);
  if ((e = radix_pass<true, true>(kDetNames, vals, nullptr, kb[0], vb[0], nullptr, n_dev, 0, 0,
                                  p.sort_blocks, hist, tot, s)))
    return e;
  int cur = 0;
  for (int pass = 1; pass < passes; ++pass) {
    if ((e = radix_pass<false, true>(kDetNames, kb[cur], vb[cur], kb[cur ^ 1], vb[cur ^ 1], nullptr,
                                     n_dev, 0, 8 * pass, p.sort_blocks, hist, tot, s)))
      return e;
    cur ^= 1;
  }
  const unsigned blocks = (unsigned)std::max<int64_t>(1, std::min<int64_t>((p.cap + 255) / 256, 4096));
  ProfScope ps("det_slot", s);
  hipLaunchKernelGGL(det_slot_kernel, dim3(blocks), dim3(256), 0, s, vb[cur], n_dev, vb[cur ^ 1]);
  return hipGetLastError();
}

hipError_t launch_det_reduce(const Plan& p, char* ws, hipStream_t s) {
  const int64_t* n_dev = (const int64_t*)(ws + p.lay.chunk_base) + p.K;
  const unsigned blocks = (unsigned)std::max<int64_t>(1, std::min<int64_t>((p.cap + 255) / 256, 4096));
  // the sort buffer the slots do not use holds the queue of long segments
  const int cur = (det_passes(p) - 1) & 1;
  uint32_t* long_start = (uint32_t*)(ws + (cur ? p.det_k0 : p.det_k1));
  uint32_t* long_cnt = (uint32_t*)(ws + p.det_cnt);
  const uint32_t* keys = det_sorted_keys(p, ws);
  const double* partial = (const double*)(ws + p.det_partial);
  double* grad2d = (double*)(ws + p.lay.grad2d);
  ProfScope ps("det_reduce", s);
  hipLaunchKernelGGL(det_count_zero, dim3(1), dim3(64), 0, s, long_cnt);
  hipLaunchKernelGGL(det_reduce_short, dim3(blocks), dim3(256), 0, s, keys, n_dev, partial, grad2d,
                     p.M, long_start, long_cnt);
  hipLaunchKernelGGL(det_reduce_long, dim3(1024), dim3(256), 0, s, keys, n_dev, partial, grad2d, p.M,
                     (const uint32_t*)long_start, (const uint32_t*)long_cnt);
  return hipGetLastError();
}

hipError_t launch_bin_sort(const Plan& p, const ls_config* cfg, char* ws, hipStream_t s) {
  (void)cfg;
  hipError_t e;
  const int64_t M = p.M;
  uint32_t* hist = (uint32_t*)(ws + p.hist);
  uint32_t* tot = (uint32_t*)(ws + p.digit_tot);
  int64_t* n_isect = (int64_t*)(ws + p.lay.n_isect);
  int64_t* isect_off = (int64_t*)(ws + p.lay.isect_off);
  uint32_t* order = (uint32_t*)(ws + p.lay.order);
  const uint32_t* dkey = (const uint32_t*)(ws + p.lay.depth_key);
  int64_t* chunk_base = (int64_t*)(ws + p.lay.chunk_base);
  int64_t* chunk_n = (int64_t*)(ws + p.lay.chunk_n);
  int32_t* flags = (int32_t*)(ws + p.lay.flags);

  // 1. depth presort of the M pairs: 4 passes of 8 bits
  if (M > 0) {
    uint32_t* kA = (uint32_t*)(ws + p.pre_keys_a);
    uint32_t* vA = (uint32_t*)(ws + p.pre_vals_a);
    uint32_t* kB = (uint32_t*)(ws + p.pre_keys_b);
    uint32_t* vB = (uint32_t*)(ws + p.pre_vals_b);
    const int G = p.pre_blocks;
    if ((e = radix_pass<true, true>(kPreNames, dkey, nullptr, kB, vB, nullptr, nullptr, M, 0, G,
                                    hist, tot, s)))
      return e;
    if ((e = radix_pass<false, true>(kPreNames, kB, vB, kA, vA, nullptr, nullptr, M, 8, G, hist,
                                     tot, s)))
      return e;
    if ((e = radix_pass<false, true>(kPreNames, kA, vA, kB, vB, nullptr, nullptr, M, 16, G, hist,
                                     tot, s)))
      return e;
    if ((e = radix_pass<false, false>(kPreNames, kB, vB, nullptr, order, nullptr, nullptr, M, 24,
                                      G, hist, tot, s, (const ushort4*)(ws + p.lay.rect),
                                      (ushort4*)(ws + p.drect))))
      return e;
  }
  // 2. scan of tile counts in depth order (+ span owners)
  {
    int64_t* part = (int64_t*)(ws + p.scan_part);
    const int B = scan_blocks_for(M);
    PairCount in{(const ushort4*)(ws + p.drect)};
    // span owners serve the complete-list key generation only
    PairOffsets out{isect_off, (uint32_t*)(ws + p.span_owner), p.K == 1 ? p.n_spans : 0,
                    part + B};
    ProfScope ps("scan", s);
    hipLaunchKernelGGL(scan_reduce<PairCount>, dim3(B), dim3(kScanThreads), 0, s, in, nullptr, M,
                       B, part);
    hipLaunchKernelGGL(scan_parts, dim3(1), dim3(1024), 0, s, part, B);
    // the per-pair offsets serve the complete lists; chunks need the total only
    if (p.K == 1)
      hipLaunchKernelGGL((scan_down<PairCount, PairOffsets>), dim3(B), dim3(kScanThreads), 0, s,
                         in, out, nullptr, M, B, part);
    hipLaunchKernelGGL(pairs_finalize, dim3(1), dim3(64), 0, s, part + B, M, isect_off, n_isect,
                       chunk_base, chunk_n, flags, p.cap, p.n_spans, p.K == 1 ? 1 : 0);
    if ((e = hipGetLastError())) return e;
  }
  if (p.K > 1) return hipSuccess;   // lists are built chunk by chunk by the rasterizer
  // 3 + 4 + 5. key generation, tile sort and ranges of the complete lists
  if (p.cap > 0 && M > 0) {
    uint32_t *k0, *v0;
    keygen_targets(p, ws, &k0, &v0);
    int64_t spans = (p.cap + kKeygenSpan - 1) / kKeygenSpan;
    int blocks = (int)std::min<int64_t>(spans, kKeygenBlocks);
    {
      ProfScope ps("keygen", s);
      hipLaunchKernelGGL(keygen_kernel, dim3(blocks), dim3(kKeygenThreads), 0, s, order,
                         isect_off, (const ushort4*)(ws + p.lay.rect),
                         (const CamInfo*)(ws + p.lay.cams), p.C, M, chunk_n,
                         (const uint32_t*)(ws + p.span_owner), k0, v0);
    }
    if ((e = hipGetLastError())) return e;
  }
  return tile_sort_and_ranges(p, ws, chunk_base, chunk_n, (int64_t*)(ws + p.lay.ranges), s);
}

hipError_t launch_chunk_bin(const Plan& p, int c, char* ws, hipStream_t s) {
  hipError_t e;
  const int64_t M = p.M;
  int64_t* chunk_base = (int64_t*)(ws + p.lay.chunk_base) + c;
  int64_t* chunk_n = (int64_t*)(ws + p.lay.chunk_n) + c;
  const int64_t lo = p.chunk_pos[c], hi = p.chunk_pos[c + 1];
  if (M > 0 && p.cap > 0 && hi > lo) {
    const CamInfo* cams = (const CamInfo*)(ws + p.lay.cams);
    const uint32_t* order = (const uint32_t*)(ws + p.lay.order);
    const uint32_t* alive = (const uint32_t*)(ws + p.alive);
    uint32_t* sat = (uint32_t*)(ws + p.sat);
    int32_t* flags = (int32_t*)(ws + p.lay.flags);
    uint32_t* pcnt = (uint32_t*)(ws + p.span_cnt);
    uint32_t* poff = (uint32_t*)(ws + p.span_off);
    uint32_t* pmask = (uint32_t*)(ws + p.pmask);
    uint32_t* owner = (uint32_t*)(ws + p.span_owner);
    uint32_t* abits = (uint32_t*)(ws + p.abits);
    const ushort4* drect = (const ushort4*)(ws + p.drect);
    uint32_t *k0, *v0;
    keygen_targets(p, ws, &k0, &v0);
    const int64_t n = hi - lo;
    const unsigned grid = (unsigned)((n + 255) / 256);
    {
      ProfScope ps("chunk_count", s);
      int gxm = 1, gym = 1;
      for (int q = 0; q < p.C; ++q) {
        gxm = std::max(gxm, p.GX[q]);
        gym = std::max(gym, p.GY[q]);
      }
      hipLaunchKernelGGL(alive_sat_rows, dim3((unsigned)((gym + 3) / 4), (unsigned)p.C), dim3(256),
                         0, s, cams, alive, sat);
      hipLaunchKernelGGL(alive_sat_cols, dim3((unsigned)((gxm + 3) / 4), (unsigned)p.C), dim3(256),
                         0, s, cams, sat);
      const int64_t bwaves = (p.T + 63) / 64 + 1;
      hipLaunchKernelGGL(alive_bits_kernel, dim3((unsigned)((bwaves + 3) / 4)), dim3(256), 0, s,
                         alive, p.T, bwaves, abits);
      hipLaunchKernelGGL(chunk_count_kernel, dim3(grid), dim3(256), 0, s, order, drect, cams, p.C,
                         M, lo, hi, sat, abits, flags, pcnt, pmask);
    }
    {
      int64_t* part = (int64_t*)(ws + p.scan_part);
      const int B = scan_blocks_for(n);
      SpanCount in{pcnt};
      ChunkOffsets out{poff, owner, p.n_spans, part + B};
      ProfScope ps("chunk_scan", s);
      hipLaunchKernelGGL(scan_reduce<SpanCount>, dim3(B), dim3(kScanThreads), 0, s, in, nullptr, n,
                         B, part);
      hipLaunchKernelGGL(scan_parts, dim3(1), dim3(1024), 0, s, part, B);
      hipLaunchKernelGGL((scan_down<SpanCount, ChunkOffsets>), dim3(B), dim3(kScanThreads), 0, s,
                         in, out, nullptr, n, B, part);
      hipLaunchKernelGGL(chunk_finalize, dim3(1), dim3(64), 0, s, part + B, chunk_base, chunk_n,
                         flags, p.cap);
    }
    {
      ProfScope ps("chunk_write", s);
      const int64_t spans = (p.cap + kChunkSpan - 1) / kChunkSpan;
      const unsigned sgrid = (unsigned)std::max<int64_t>(1, std::min<int64_t>(spans, 4096));
      hipLaunchKernelGGL(chunk_write_span_kernel, dim3(sgrid), dim3(256), 0, s, order, drect, cams,
                         p.C, M, lo, hi, pcnt, poff, pmask, owner, p.n_spans, chunk_base, chunk_n,
                         k0, v0);
      hipLaunchKernelGGL(chunk_write_big_kernel, dim3(grid), dim3(256), 0, s, order, drect, cams,
                         p.C, M, lo, hi, abits, pcnt, poff, pmask, chunk_base, chunk_n, k0, v0);
    }
    if ((e = hipGetLastError())) return e;
  } else {
    hipLaunchKernelGGL(chunk_empty, dim3(1), dim3(64), 0, s, chunk_base, chunk_n);
    if ((e = hipGetLastError())) return e;
  }
  return tile_sort_and_ranges(p, ws, chunk_base, chunk_n,
                              (int64_t*)(ws + p.lay.ranges) + (int64_t)c * (p.T + 1), s);
}

}  // namespace lsplat
