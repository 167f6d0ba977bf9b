// Per-tile compositing with the linear kernel (forward) and its reverse pass;
// the other kernels of the appendix's family (Gaussian, Laplacian, raised
// cosine, quadratic, each with alignment lambda) are template instances of
// the same kernels.
//
// Forward (Eq. 6 with Eq. 10-12): alpha = min(alpha_max, o * max(0, 1 - D'/lambda)),
// D'^2 = A dx^2 + 2B dx dy + C dy^2.  Blending rules kept from 3DGS (Sec. 3.2):
// skip alpha < alpha_min, stop before a splat that would take T below t_min.
//
// Backward: walk each tile's list back to front from the pixel's last
// contributor, recover T_i = T_{i+1} / (1 - alpha_i), and accumulate the
// per-pair 2D gradients; adaptive gradient scaling (Eq. 13-14) multiplies the
// gradient through L' by omega(D') = exp(-D'^2).
//
// One workgroup per tile, one or two pixels per lane (wave64: a 16x16 tile
// is two waves of 16x8 pixels).  The tile's list is consumed in batches
// staged in LDS (gathered 64-byte records, turned into the coefficients of
// the quadratic form in tile-local coordinates).
// Blocks are remapped so that each XCD (blocks are dealt round-robin over
// the 8 XCDs) works on one contiguous band of tiles and keeps the records of
// neighbouring tiles in its own L2.
//
// Numerics: the quadratic form, D', alpha, the transmittance and colour
// state and every backward term are FP64 (full rate on CDNA, and free of the
// FP32 cancellation of needle-shaped splats).  1 - alpha is formed as
// (1 - o) + o D'/lambda, a sum of two non-negative terms, so transmittance
// keeps full relative precision when alpha is close to 1.
#include <algorithm>

#include "internal.h"

namespace lsplat {

namespace {

struct RasterParams {
  double lam2;        // lambda^2: D' >= lambda <=> outside the support
  double inv_lam;     // 1 / lambda
  double inv_lam2;    // 1 / lambda^2
  double amin, amax, oma_max, tmin;
  double amin_pos;    // a pair is used iff alpha >= amin_pos: alpha > 0 and alpha >= amin
  float bg0, bg1, bg2;
  int ags, ags_arg, ags_scope;
  double ags_scale;   // AGS exponent per unit D'^2: 1 / lambda^2 or 1
  double qmax;        // extent^2: a pair is kept while D'^2 < qmax (the support)
  double ghalf;       // 1 / (2 lambda^2), the Gaussian's exponent per unit D'^2
};

// e^-x for x >= 0 in FP64: x = k ln2/2 + r with |r| <= ln2 / 4 (ln2/2 split
// in a high part whose products with k are exact and a low part), e^-r from
// its Taylor series to degree 8 (truncation below 1e-13), scaled by
// 2^-(k/2) (with 1/sqrt 2 for odd k).
__device__ __forceinline__ double exp_neg(double x) {
  x = fmin(x, 708.0);   // below 1e-307 the weight is as good as 0
  const double k = rint(x * 2.8853900817779268);          // 2 / ln 2
  double r = fma(-k, 3.46573590184561908245e-01, x);      // ln2 / 2, high part
  r = fma(-k, 9.54107464635293850010e-11, r);             // low part
  const double t = -r;
  double p = 1.0 / 40320.0;
  p = fma(p, t, 1.0 / 5040.0);
  p = fma(p, t, 1.0 / 720.0);
  p = fma(p, t, 1.0 / 120.0);
  p = fma(p, t, 1.0 / 24.0);
  p = fma(p, t, 1.0 / 6.0);
  p = fma(p, t, 0.5);
  p = fma(p, t, 1.0);
  p = fma(p, t, 1.0);
  const int ki = (int)k;
  if (ki & 1) p *= 0.70710678118654752440;
  return ldexp(p, -(ki >> 1));
}

// e^-x on [0, kExpTabN / kExpTabStep) from a table of e^-(j / kExpTabStep)
// (built with exp_neg) times e^-r for the remainder 0 <= r < 1 / kExpTabStep,
// the latter from the degree-5 polynomial interpolating e^-r at the six
// Chebyshev nodes of [0, 1/16] (relative error below 5e-14 on the interval).
// Arguments above the range are clamped into it (NaN too, which fmin turns
// into the bound) and the index is clamped at 0 from below, so the table read
// stays in bounds; callers use it only where every argument that matters lies
// inside.
constexpr int kExpTabStep = 16;
constexpr int kExpTabN = 128;
__device__ __forceinline__ double exp_neg_tab(double x, const double* tab) {
  x = fmin(x, (double)kExpTabN / kExpTabStep - 0.01);
  const int j = max((int)(x * (double)kExpTabStep), 0);
  const double r = fma((double)j, -1.0 / kExpTabStep, x);   // exact
  double p = -0.008077218246913261;
  p = fma(p, r, 0.041648755648710845);
  p = fma(p, r, -0.16666608768855815);
  p = fma(p, r, 0.4999999915303285);
  p = fma(p, r, -0.999999999954658);
  p = fma(p, r, 0.9999999999999607);
  return tab[j] * p;
}


// alpha and 1 - alpha of one (pixel, splat) pair, in FP64.  Shared by the
// forward and backward kernels and evaluated without contraction, so both
// kernels take every skip/stop decision identically.
struct PairEval {
  double D, alpha, oma;
  double invD;   // 1 / D, 0 where D = 0 (the forward pass ignores it)
  double f;      // kernel value f(D/lambda) (alpha = o f below the clamp)
  double sx;     // raised cosine: sin(pi D/lambda), for its slope
  double nc;     // 1 below the alpha clamp, 0 at it (alpha does not depend on o or D there)
};

// sqrt(q) for q >= 0 (a negative q, possible only by rounding of the
// expanded quadratic form at a splat's centre, counts as 0), with 1/sqrt(q)
// in *inv: the FP32 reciprocal square root as a start and one FP64 Newton
// step for the reciprocal square root bring the relative error of 1/sqrt(q)
// from about 2^-22 to below 1e-13, and sqrt(q) = q / sqrt(q) keeps it.  Below
// 1e-30 both are 0 (an absolute error under 1e-15, and no slope at the apex).
__device__ __forceinline__ double sqrt_nonneg(double q, double* inv) {
  const double y = (double)__builtin_amdgcn_rsqf((float)q);
  const double r = y * fma(-0.5 * q, y * y, 1.5);
  *inv = q > 1e-30 ? r : 0.0;
  return q * *inv;
}

// Kernels of the family (LS_KERNEL_*), a template parameter of the raster
// kernels.  The ones that fall to 0 (linear, quadratic) form 1 - alpha as
// (1 - o) + o (1 - f), a sum of non-negative terms; the others as 1 - o f.
// The exponential kernels read e^-x from the LDS table `tab`.
template <int KF>
constexpr bool kernel_uses_exp() {
  return KF == LS_KERNEL_GAUSSIAN || KF == LS_KERNEL_LAPLACIAN;
}

// min and max of two doubles that are not NaN, as single instructions: with
// fmin and fmax the compiler canonicalises a bound that is carried in a
// register at every use.
__device__ __forceinline__ double min_nn(double a, double b) {
  double r;
  asm("v_min_f64 %0, %1, %2" : "=v"(r) : "v"(a), "v"(b));
  return r;
}
__device__ __forceinline__ double max_nn(double a, double b) {
  double r;
  asm("v_max_f64 %0, %1, %2" : "=v"(r) : "v"(a), "v"(b));
  return r;
}

template <int KF>
__device__ __forceinline__ PairEval pair_eval(double q, double o, const RasterParams& rp,
                                              const double* tab) {
#pragma clang fp contract(off)
  PairEval e;
  e.sx = 0.0;
  if constexpr (KF == LS_KERNEL_LINEAR) {
    e.D = sqrt_nonneg(q, &e.invD);
    const double t = o * (e.D * rp.inv_lam);
    e.alpha = o - t;
    e.oma = (1.0 - o) + t;
    e.f = 1.0 - e.D * rp.inv_lam;
  } else if constexpr (KF == LS_KERNEL_QUADRATIC) {
    e.D = 0.0;
    e.invD = 0.0;
    const double u = fmax(q, 0.0) * rp.inv_lam2;
    const double t = o * u;
    e.alpha = o - t;
    e.oma = (1.0 - o) + t;
    e.f = 1.0 - u;
  } else if constexpr (KF == LS_KERNEL_GAUSSIAN) {
    e.D = 0.0;
    e.invD = 0.0;
    e.f = exp_neg_tab(fmax(q, 0.0) * rp.ghalf, tab);
    e.alpha = o * e.f;
    e.oma = 1.0 - e.alpha;
  } else if constexpr (KF == LS_KERNEL_LAPLACIAN) {
    e.D = sqrt_nonneg(q, &e.invD);
    e.f = exp_neg_tab(e.D * rp.inv_lam, tab);
    e.alpha = o * e.f;
    e.oma = 1.0 - e.alpha;
  } else {   // raised cosine
    e.D = sqrt_nonneg(q, &e.invD);
    double cs;
    sincospi(fmin(e.D * rp.inv_lam, 1.0), &e.sx, &cs);
    e.f = 0.5 * (1.0 + cs);
    e.alpha = o * e.f;
    e.oma = 1.0 - e.alpha;
  }
  // the clamp: alpha at most alpha_max, 1 - alpha at least 1 - alpha_max
  e.nc = e.alpha > rp.amax ? 0.0 : 1.0;
  e.alpha = min_nn(e.alpha, rp.amax);
  e.oma = max_nn(e.oma, rp.oma_max);
  return e;
}

// Tile of block b of nb.  Blocks are dealt to the 8 XCDs round-robin
// (b mod 8), each with its own L2.  Tiles are taken in strips of 64
// consecutive tiles (a run along a tile row), and XCD x works through strips
// x, x + 8, x + 16, ... in order, so each XCD's blocks share the splats of
// their strip while every view's work is spread over all eight XCDs.  (With
// one contiguous eighth of the tiles per XCD, eight views put one view on
// each XCD, and after the first depth chunk the XCD of the busiest view was
// left running alone.)  Blocks past the last whole group of 8 strips map to
// themselves.
__device__ __forceinline__ int64_t xcd_remap(int64_t b, int64_t nb) {
  constexpr int64_t G = 64;
  const int64_t full = nb / (8 * G) * (8 * G);
  if (b >= full) return b;
  const int64_t x = b & 7, k = b >> 3;
  return ((k / G) * 8 + x) * G + k % G;
}

__device__ __forceinline__ int cam_of_tile(const CamInfo* cams, int C, int64_t t) {
  int lo = 0, hi = C - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (cams[mid].tile_off <= t) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// LDS staging of one batch of a tile's list.  Each entry becomes the
// coefficients of its quadratic form in the tile's local pixel coordinates
// (lx, ly) = (0..TW-1, 0..TH-1):
//   D'^2 = qa lx^2 + qb lx ly + qc ly^2 + qd lx + qe ly + qf,
// five FP64 FMAs per pixel.  Entries whose support ellipse misses the tile's
// pixel-centre rectangle are dropped and the survivors compacted in list
// order, so the per-pixel loop only sees splats that can touch the tile.
// NS staged entries at most; NW waves in the block
// The FP32 colour and opacity are staged for the forward pass (RGBO); the
// backward pass stages them widened in StageExt instead.
template <int NS, int NW, bool RGBO = true>
struct Stage {
  // D'^2 at tile-local pixel (x, y) = qa x^2 + qb xy + qc y^2 + qd x + qe y + qf
  double qa[NS], qb[NS], qc[NS], qd[NS], qe[NS], qf[NS];
  float r[RGBO ? NS : 1], g[RGBO ? NS : 1], b[RGBO ? NS : 1], o[RGBO ? NS : 1];
  int32_t pos[NS];           // position in the tile list
  uint32_t m[NS];            // pair id
  int32_t wcount[NW];
};

// Per-entry constants only the backward kernel reads, staged beside the
// quadratic form so that the entry loop does not recompute them per entry.
template <int NS>
struct StageExt {
  double o[NS], r[NS], g[NS], b[NS];      // opacity and colour, widened
  double nol[NS];                         // -o / (2 lambda)
};

// D'^2 at tile-local pixel (x, y), nested as
// (qf + x (qd + qa x)) + y ((qe + qb x) + qc y): five FMA and no per-pixel
// squares.  The two x-only terms are shared by the pixels of a column, so a
// thread that holds several pixels of one column pays two FMA per pixel.  The
// forward and backward kernels evaluate it in this order, so they take the
// same decisions.
struct QuadX {
  double P, R;   // qf + x (qd + qa x) and qe + qb x
};
__device__ __forceinline__ QuadX quad_x(double qa, double qb, double qd, double qe, double qf,
                                        double x) {
  return QuadX{fma(x, fma(qa, x, qd), qf), fma(qb, x, qe)};
}
__device__ __forceinline__ double quad_y(const QuadX& h, double qc, double y) {
  return fma(y, fma(qc, y, h.R), h.P);
}

// true if min over [0, w] x [0, h] of A dx^2 + 2B dx dy + C dy^2 (dx = x - ox,
// dy = y - oy) may be below lam2; a relative margin keeps every splat that the
// per-pixel evaluation could still find inside its support.
__device__ __forceinline__ bool ellipse_hits_rect(double ox, double oy, double A, double B,
                                                  double C, double lam2, double w, double h) {
  if (ox >= 0.0 && ox <= w && oy >= 0.0 && oy <= h) return true;
  double best = 1e300;
#pragma unroll
  for (int e = 0; e < 2; ++e) {
    const double dx = (e ? w : 0.0) - ox;
    const double y = fmin(h, fmax(0.0, oy - B * dx / C));
    const double dy = y - oy;
    best = fmin(best, A * dx * dx + 2.0 * B * dx * dy + C * dy * dy);
  }
#pragma unroll
  for (int e = 0; e < 2; ++e) {
    const double dy = (e ? h : 0.0) - oy;
    const double x = fmin(w, fmax(0.0, ox - B * dy / A));
    const double dx = x - ox;
    best = fmin(best, A * dx * dx + 2.0 * B * dx * dy + C * dy * dy);
  }
  return best < lam2 * (1.0 + 1e-6);
}

// Stage one batch: thread i (i < NT) brings entry `vidx` of the sorted
// values (if `has`), whose position in the tile's list is `gpos`.  Returns the
// number of surviving entries (block-uniform).
template <int TW, int TH, int NS, int NWB, bool RGBO>
__device__ __forceinline__ int stage_batch(Stage<NS, NWB, RGBO>& st, const uint32_t* __restrict__ vals,
                                           const ProjRec* __restrict__ proj, int64_t M, bool has,
                                           int64_t vidx, int32_t gpos, double x0c, double y0c,
                                           double lam2, StageExt<NS>* ext = nullptr,
                                           double inv_lam = 0.0) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  bool keep = false;
  uint32_t m = 0;
  ProjRec rec;
  double ox = 0.0, oy = 0.0;
  if (has) {
    m = vals[vidx];
    if (m >= (uint64_t)M) m = 0;   // unreachable for a valid list
    rec = proj[m];
    ox = rec.mx - x0c;
    oy = rec.my - y0c;
    keep = ellipse_hits_rect(ox, oy, rec.A, rec.B, rec.C, lam2, (double)(TW - 1), (double)(TH - 1));
  }
  const uint64_t bal = __builtin_amdgcn_ballot_w64(keep);
  if (lane == 0) st.wcount[wave] = (int32_t)__popcll(bal);
  __syncthreads();
  int base = 0, total = 0;
#pragma unroll
  for (int w = 0; w < NWB; ++w) {
    const int c = st.wcount[w];
    base += (w < wave) ? c : 0;
    total += c;
  }
  if (keep) {
    const int k = base + (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(bal >> 32),
                                                        __builtin_amdgcn_mbcnt_lo((uint32_t)bal, 0u));
    const double A = rec.A, B = rec.B, C = rec.C;
    const double u = A * ox + B * oy, v = B * ox + C * oy;
    st.qa[k] = A;
    st.qb[k] = 2.0 * B;
    st.qc[k] = C;
    st.qd[k] = -2.0 * u;
    st.qe[k] = -2.0 * v;
    st.qf[k] = ox * u + oy * v;
    if constexpr (RGBO) {
      st.r[k] = rec.r;
      st.g[k] = rec.g;
      st.b[k] = rec.b;
      st.o[k] = rec.o;
    }
    st.pos[k] = gpos;
    st.m[k] = m;
    if (ext) {
      ext->o[k] = rec.o;
      ext->r[k] = rec.r;
      ext->g[k] = rec.g;
      ext->b[k] = rec.b;
      ext->nol[k] = -0.5 * (double)rec.o * inv_lam;
    }
  }
  __syncthreads();
  return total;
}

// Forward composite of chunk c of K: each tile continues from the state its
// pixels reached in the previous chunks (T and colour in FP64, the stop flag
// and `last`) over its segment of this chunk's sorted list.
// Threads of the raster kernels: a tile of 128 or more pixels gives each lane
// two vertically adjacent pixels, so one read of the staged entry (and in the
// backward pass one wave-wide reduction) serves both.
template <int TW, int TH>
constexpr int raster_ppl() { return TW * TH >= 128 ? 2 : 1; }
template <int TW, int TH>
constexpr int raster_threads() { return TW * TH / raster_ppl<TW, TH>(); }

// The forward pass is bound by the latency of its global reads (tile
// state, staged records): six waves per SIMD instead of the five its
// registers would allow (a few values live across the loop go to scratch).
template <int TW, int TH, int KF>
__global__ __launch_bounds__((raster_threads<TW, TH>())) __attribute__((amdgpu_waves_per_eu(6)))
void raster_fwd_kernel(
    const CamInfo* __restrict__ cams, int C, const int64_t* __restrict__ ranges_all, int64_t T_all,
    int c, int K, const int64_t* __restrict__ chunk_base, const uint32_t* __restrict__ vals,
    const ProjRec* __restrict__ proj, int64_t M, int batch, RasterParams rp,
    double4* __restrict__ state, uint8_t* __restrict__ done_px, uint32_t* __restrict__ alive,
    float* __restrict__ image, float* __restrict__ final_T, int32_t* __restrict__ last,
    uint32_t* __restrict__ tile_contrib, double* __restrict__ t64) {
  constexpr int PPL = raster_ppl<TW, TH>();
  constexpr int NTB = raster_threads<TW, TH>();
  constexpr int NWB = NTB / 64;
  __shared__ Stage<NTB, NWB> st;
  __shared__ uint32_t s_cnt[NWB];
  __shared__ double s_exptab[kernel_uses_exp<KF>() ? kExpTabN : 1];
  const int tid = threadIdx.x;
  const int64_t tile = xcd_remap(blockIdx.x, gridDim.x);
  if (c > 0 && alive[tile] == 0u) return;
  if constexpr (kernel_uses_exp<KF>())   // ready at the first batch's barriers
    for (int i = tid; i < kExpTabN; i += NTB) s_exptab[i] = exp_neg((double)i / kExpTabStep);
  const int64_t* ranges = ranges_all + (int64_t)c * (T_all + 1);
  const int32_t len = (int32_t)(ranges[tile + 1] - ranges[tile]);
  // a live tile with no entries in this chunk keeps its state; in the last
  // chunk it still writes the outputs of the pixels that never stopped
  if (c > 0 && c < K - 1 && len == 0) return;
  const int64_t start = chunk_base[c] + ranges[tile];
  int32_t prefix = 0;
  for (int cc = 0; cc < c; ++cc) {
    const int64_t* r = ranges_all + (int64_t)cc * (T_all + 1);
    prefix += (int32_t)(r[tile + 1] - r[tile]);
  }
  const int ci_idx = cam_of_tile(cams, C, tile);
  const CamInfo& ci = cams[ci_idx];
  const int64_t local = tile - ci.tile_off;
  const int ty = (int)(local / ci.GX), tx = (int)(local % ci.GX);
  const double x0c = (double)(tx * TW) + 0.5, y0c = (double)(ty * TH) + 0.5;
  const int lxi = tid % TW;
  const int px = tx * TW + lxi;
  const double lx = (double)lxi;

  // per pixel of this lane: transmittance and colour (FP64), the stop flag
  // and `last`, continued from the previous chunks
  // A pixel's outputs are written once, in the chunk where it stops (or the
  // last chunk); a pixel that stopped in an earlier chunk is not touched
  // again (`fin`), and only a live pixel's state is carried to the next chunk.
  double ly[PPL], T[PPL], cr[PPL], cg[PPL], cb[PPL];
  int64_t pix[PPL];
  bool inside[PPL], done[PPL], fin[PPL];
  int32_t lastc[PPL];
  uint32_t ncon = 0;
#pragma unroll
  for (int j = 0; j < PPL; ++j) {
    const int lyi = (tid / TW) * PPL + j;
    const int py = ty * TH + lyi;
    ly[j] = (double)lyi;
    inside[j] = (px < ci.W) && (py < ci.H);
    pix[j] = ci.pix_off + (int64_t)py * ci.W + px;
    T[j] = 1.0;
    cr[j] = cg[j] = cb[j] = 0.0;
    lastc[j] = 0;
    done[j] = !inside[j];
    fin[j] = !inside[j];
    if (c > 0 && inside[j]) {
      fin[j] = done[j] = done_px[pix[j]] != 0;
      if (!done[j]) {
        const double4 sv = state[pix[j]];
        T[j] = sv.x;
        cr[j] = sv.y;
        cg[j] = sv.z;
        cb[j] = sv.w;
        lastc[j] = last[pix[j]];
      }
    }
  }
  auto all_done = [&]() {
    bool a = true;
#pragma unroll
    for (int j = 0; j < PPL; ++j) a = a && done[j];
    return a;
  };
  const int bsz = batch < NTB ? batch : NTB;
  for (int32_t p0 = 0; p0 < len; p0 += bsz) {
    if (__syncthreads_count(!all_done()) == 0) break;
    const int nb = (len - p0) < bsz ? (len - p0) : bsz;
    const int cnt = stage_batch<TW, TH, NTB, NWB>(st, vals, proj, M, tid < nb, start + p0 + tid,
                                                  prefix + p0 + tid, x0c, y0c, rp.qmax);
    if (!all_done()) {
      for (int k = 0; k < cnt; ++k) {
        const QuadX hx = quad_x(st.qa[k], st.qb[k], st.qd[k], st.qe[k], st.qf[k], lx);
        const double qc = st.qc[k];
#pragma unroll
        for (int j = 0; j < PPL; ++j) {
          if (done[j]) continue;
          const double q = quad_y(hx, qc, ly[j]);
          if (!(q < rp.qmax)) continue;
          const PairEval e = pair_eval<KF>(q, (double)st.o[k], rp, s_exptab);
          if (!(e.alpha >= rp.amin_pos)) continue;
          const double Tn = T[j] * e.oma;
          if (Tn < rp.tmin) {
            done[j] = true;
            continue;
          }
          const double w = e.alpha * T[j];
          cr[j] = fma((double)st.r[k], w, cr[j]);
          cg[j] = fma((double)st.g[k], w, cg[j]);
          cb[j] = fma((double)st.b[k], w, cb[j]);
          T[j] = Tn;
          lastc[j] = st.pos[k] + 1;
          ++ncon;
        }
        if (all_done()) break;
      }
    }
  }
  const int64_t plane = (int64_t)ci.W * ci.H;
  const bool more = K > 1 && c < K - 1;   // chunks follow this one
  bool live = false;
#pragma unroll
  for (int j = 0; j < PPL; ++j) {
    if (fin[j]) continue;
    if (more && !done[j]) {
      // still compositing: carry the state (done_px is already 0 after the
      // first chunk)
      state[pix[j]] = make_double4(T[j], cr[j], cg[j], cb[j]);
      last[pix[j]] = lastc[j];
      if (c == 0) done_px[pix[j]] = 0;
      live = true;
      continue;
    }
    const int64_t ib = 3 * ci.pix_off + (pix[j] - ci.pix_off);
    image[ib] = (float)(cr[j] + T[j] * (double)rp.bg0);
    image[ib + plane] = (float)(cg[j] + T[j] * (double)rp.bg1);
    image[ib + 2 * plane] = (float)(cb[j] + T[j] * (double)rp.bg2);
    final_T[pix[j]] = (float)T[j];
    t64[pix[j]] = T[j];   // the backward pass starts from the FP64 value
    last[pix[j]] = lastc[j];
    if (more) done_px[pix[j]] = 1;
  }
  // contributing pairs of the tile (a statistic for throughput accounting)
  for (int d = 32; d > 0; d >>= 1) ncon += __shfl_xor(ncon, d, 64);
  if ((tid & 63) == 0) s_cnt[tid >> 6] = ncon;
  __syncthreads();
  if (tid == 0) {
    uint32_t t = 0;
#pragma unroll
    for (int w = 0; w < NWB; ++w) t += s_cnt[w];
    tile_contrib[tile] = (c > 0 ? tile_contrib[tile] : 0u) + t;
  }
  if (K > 1 && c < K - 1) {
    const int any_live = __syncthreads_or(live);
    if (tid == 0) alive[tile] = any_live ? 1u : 0u;
  }
}

// Adaptive gradient scaling in the backward kernel, a template parameter:
// off, or omega applied to the geometric gradient only or to every gradient
// of the pair.
enum { kAgsOff = 0, kAgsGeo = 1, kAgsWhole = 2 };
template <int AG>
constexpr bool ags_whole() { return AG == kAgsWhole; }

// The AGS weight omega = e^-x, x >= 0, in FP32 precision: the hardware base-2
// exponential of -x log2(e) formed in FP32.  The FP32 rounding of x and of
// the product puts the relative error below 5e-7 for x < 8 (the D'^2 reading
// with lambda 2.5 reaches 6.25 at the support's edge) and below 1e-6 for
// x < 16; far out, where omega is below 1e-7, it grows with x, and below
// 2^-126 the weight is 0.  omega only scales a gradient direction, so this
// precision is far inside the gradients' 1e-5 tolerance; every other
// per-pixel term stays FP64.
__device__ __forceinline__ double ags_weight(double x) {
  return (double)__builtin_amdgcn_exp2f((float)x * -1.44269504088896341f);
}

// Wave-wide sums of nine FP64 values per lane, through LDS, for a block of
// one wave.  Every lane stores its nine values; field f of lane 8p + q sits at
// f * 80 + 10 p + q (doubles).  Lane l = 8f + p (f < 8) then adds the eight
// values of field f in part p, and every lane the eight of field 8 in part p;
// lanes 0..7 store the latter and all lanes the former, and lane f (f < 9)
// adds the eight partial sums of field f (stored at 10 f + p).  The padding
// (parts of 10, fields of 80) spreads each 16-byte read of eight lanes over
// distinct banks.  Lanes
// 0..8 return the sums of fields 0..8 (the other lanes a copy of field 8's).
// Within one wave the LDS accesses execute in program order; the fences keep
// the compiler from moving one lane's store across another lane's load.
constexpr int kRedField = 80;
constexpr int kRedDoubles = 9 * kRedField;
__device__ __forceinline__ double wave_sum9_lds(const double (&v)[9], double* red, int lane) {
  const int f = lane >> 3, p = lane & 7;
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  double* w = red + 10 * (lane >> 3) + (lane & 7);
#pragma unroll
  for (int i = 0; i < 9; ++i) w[i * kRedField] = v[i];
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  const double2* a = reinterpret_cast<const double2*>(red + f * kRedField + 10 * p);
  const double2* b = reinterpret_cast<const double2*>(red + 8 * kRedField + 10 * p);
  double x = a[0].x + a[0].y, y = b[0].x + b[0].y;
#pragma unroll
  for (int j = 1; j < 4; ++j) {
    x += a[j].x + a[j].y;
    y += b[j].x + b[j].y;
  }
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  red[10 * f + p] = x;
  if (lane < 8) red[80 + p] = y;
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  const double2* c = reinterpret_cast<const double2*>(red + 10 * (lane < 9 ? lane : 8));
  double z = c[0].x + c[0].y;
#pragma unroll
  for (int j = 1; j < 4; ++j) z += c[j].x + c[j].y;
  return z;
}

// Backward kernel: one wave per tile, TW * TH / 64 pixels per lane.  Lane l
// owns column l % TW; its pixels come in groups of (up to) two vertically
// adjacent ones, one group per horizontal band of the tile (a 16x16 tile:
// rows 2r, 2r + 1 in the upper band and 2r + 8, 2r + 9 in the lower, with
// r = l / 16).  One read of a staged entry and one wave-wide reduction of
// its nine gradient sums serve the whole tile; a band whose pixels all lie
// past the entry, or of which no pixel takes the entry, skips it.
template <int TW, int TH>
constexpr int bwd_ppl() { return TW * TH / 64; }

template <int TW, int TH, int KF, int AG>
__global__ __launch_bounds__(64) void raster_bwd_kernel(
    const CamInfo* __restrict__ cams, int C, const int64_t* __restrict__ ranges_all,
    int64_t T_all, int K, const int64_t* __restrict__ chunk_base,
    const uint32_t* __restrict__ vals, const ProjRec* __restrict__ proj, int64_t M, int batch,
    RasterParams rp, const double* __restrict__ t64, const int32_t* __restrict__ last,
    const float* __restrict__ dL_dimage, const float* __restrict__ dL_dalpha,
    double* __restrict__ grad2d, double* __restrict__ partial,
    const uint32_t* __restrict__ det_slot) {
  constexpr int PPL = bwd_ppl<TW, TH>();
  constexpr int PB = PPL < 2 ? PPL : 2;   // pixels per group (vertical neighbours)
  constexpr int NG = PPL / PB;            // groups: horizontal bands of the tile
  constexpr int NS = 64;                  // staged entries per batch, one per lane
  static_assert(PPL >= 1 && (TW * TH) % 64 == 0 && 64 % TW == 0 && TH % (NG * PB) == 0,
                "tile shape");
  __shared__ Stage<NS, 1, false> st;
  __shared__ StageExt<NS> sx;
  __shared__ __align__(16) double s_red[kRedDoubles];
  __shared__ int64_t s_segbase[kMaxDepthChunks];
  __shared__ int32_t s_segpre[kMaxDepthChunks + 1];
  __shared__ double s_exptab[kExpTabN];
  const int lane = threadIdx.x;
  if (kernel_uses_exp<KF>())
    for (int i = lane; i < kExpTabN; i += 64) s_exptab[i] = exp_neg((double)i / kExpTabStep);
  const int64_t tile = xcd_remap(blockIdx.x, gridDim.x);
  const int c = cam_of_tile(cams, C, tile);
  const CamInfo& ci = cams[c];
  const int64_t local = tile - ci.tile_off;
  const int ty = (int)(local / ci.GX), tx = (int)(local % ci.GX);
  const double x0c = (double)(tx * TW) + 0.5, y0c = (double)(ty * TH) + 0.5;
  // the tile's list: its segments of every chunk, in chunk order
  if (lane == 0) {
    int32_t pre = 0;
    for (int cc = 0; cc < K; ++cc) {
      const int64_t* r = ranges_all + (int64_t)cc * (T_all + 1);
      s_segbase[cc] = chunk_base[cc] + r[tile];
      s_segpre[cc] = pre;
      pre += (int32_t)(r[tile + 1] - r[tile]);
    }
    s_segpre[K] = pre;
  }
  __syncthreads();
  const int64_t len = s_segpre[K];

  // per pixel of this lane: position, upstream gradients, transmittance and
  // the upstream gradient's dot product with the suffix colour behind the
  // current splat
  const int lxi = lane % TW, rg = lane / TW;
  const double lx = (double)lxi;
  // the upstream gradient is kept in FP32 (as given) and widened where used
  double ly[PPL], T[PPL], GS[PPL];
  float G0[PPL], G1[PPL], G2[PPL];
  int32_t mylast[PPL];
  int32_t glast[NG];
#pragma unroll
  for (int g = 0; g < NG; ++g) {
    glast[g] = 0;
#pragma unroll
    for (int i = 0; i < PB; ++i) {
      const int j = g * PB + i;
      const int lyi = g * (TH / NG) + PB * rg + i;
      ly[j] = (double)lyi;
      const int px = tx * TW + lxi, py = ty * TH + lyi;
      T[j] = 1.0;
      G0[j] = G1[j] = G2[j] = 0.f;
      double GA = 0.0;
      mylast[j] = 0;
      if (px < ci.W && py < ci.H) {
        const int64_t pix = ci.pix_off + (int64_t)py * ci.W + px;
        const int64_t plane = (int64_t)ci.W * ci.H;
        const int64_t ib = 3 * ci.pix_off + (int64_t)py * ci.W + px;
        // FP64: with t_min = 0 a pixel's final transmittance can fall below
        // the FP32 range, and every T_i is recovered from it by division
        T[j] = t64[pix];
        const int32_t l = last[pix];
        mylast[j] = l < 0 ? 0 : (l > len ? (int32_t)len : l);
        G0[j] = dL_dimage[ib];
        G1[j] = dL_dimage[ib + plane];
        G2[j] = dL_dimage[ib + 2 * plane];
        if (dL_dalpha) GA = dL_dalpha[pix];
      }
      // G . S for the suffix colour S behind the current splat, which starts
      // as the background term T_final bg; the accumulated opacity
      // 1 - T_final is a fourth channel with splat colour 0 and background -1
      GS[j] = T[j] * ((double)G0[j] * (double)rp.bg0 + (double)G1[j] * (double)rp.bg1 +
                      (double)G2[j] * (double)rp.bg2 - GA);
      glast[g] = mylast[j] > glast[g] ? mylast[j] : glast[g];
    }
    // band-wide maximum of `last`: entries at or beyond it concern no pixel
    // of the band
    for (int d = 32; d > 0; d >>= 1) {
      const int32_t y = __shfl_xor(glast[g], d, 64);
      glast[g] = y > glast[g] ? y : glast[g];
    }
    glast[g] = __builtin_amdgcn_readfirstlane(glast[g]);
  }
  int32_t tile_last = 0;
#pragma unroll
  for (int g = 0; g < NG; ++g) tile_last = glast[g] > tile_last ? glast[g] : tile_last;
  // factor of the wave sum of field `lane` (lanes 0..8): the geometric
  // terms are summed with U = 2u in place of u and without their sign, so
  // the centre terms take -1, the diagonal covariance terms -1/4 and the
  // off-diagonal one -1/2 (powers of two: exact)
  const double fac = lane < 2 ? -1.0 : lane == 3 ? -0.5 : lane < 5 ? -0.25 : 1.0;

  const int bsz = batch < NS ? batch : NS;
  for (int32_t hi = tile_last; hi > 0; hi -= bsz) {
    const int32_t lo = hi - bsz > 0 ? hi - bsz : 0;
    __syncthreads();   // the previous batch's entries are no longer read
    const int32_t q = lo + lane;
    int64_t vidx = 0;
    if (q < hi) {
      int cc = 0;
      while (cc + 1 < K && s_segpre[cc + 1] <= q) ++cc;
      vidx = s_segbase[cc] + (q - s_segpre[cc]);
    }
    const int cnt = stage_batch<TW, TH, NS, 1>(st, vals, proj, M, q < hi, vidx, q, x0c, y0c,
                                              rp.qmax, &sx, rp.inv_lam);
    // the staged positions increase with k: the entries the tile needs are
    // the first kend, those before its last contributor
    const int kend =
        __popcll(__builtin_amdgcn_ballot_w64(lane < cnt && st.pos[lane] < tile_last));
    for (int k = kend - 1; k >= 0; --k) {
      // the entry is the same for every lane: its position in the list is
      // read into a scalar register, so the band tests branch uniformly
      const int32_t pos = __builtin_amdgcn_readfirstlane(st.pos[k]);
      const double qc = st.qc[k];
      const QuadX hx = quad_x(st.qa[k], st.qb[k], st.qd[k], st.qe[k], st.qf[k], lx);
      const double o = sx.o[k];
      const double cr = sx.r[k], cg = sx.g[k], cb = sx.b[k];
      // U = 2 cov^-1 (x - centre), the gradient of D'^2 in x:
      // (2 qa x + qb y + qd, qb x + 2 qc y + qe); its x-only parts are shared
      // by the lane's pixels (the second is quad_x's R)
      const double qb = st.qb[k], qc2 = 2.0 * qc;
      const double Ux0 = fma(2.0 * st.qa[k], lx, st.qd[k]), Uy0 = hx.R;
      const double nol = sx.nol[k];
      double gv[kGrad2d];
#pragma unroll
      for (int f = 0; f < kGrad2d; ++f) gv[f] = 0.0;
      bool used = false;
#pragma unroll
      for (int g = 0; g < NG; ++g) {
        if (pos >= glast[g]) continue;   // every pixel of the band stopped before it
        // Evaluated for every lane of the band and masked, so that the wave
        // runs one path; a band with no contributing pixel skips the entry.
        double qq[PB];
        PairEval e[PB];
        bool contrib[PB];
        bool any = false;
#pragma unroll
        for (int i = 0; i < PB; ++i) {
          const int j = g * PB + i;
          qq[i] = quad_y(hx, qc, ly[j]);
          e[i] = pair_eval<KF>(qq[i], o, rp, s_exptab);
          contrib[i] = pos < mylast[j] && qq[i] < rp.qmax && e[i].alpha >= rp.amin_pos;
          any = any || contrib[i];
        }
        if (__builtin_amdgcn_ballot_w64(any) == 0ull) continue;
        used = true;
#pragma unroll
        for (int i = 0; i < PB; ++i) {
          const int j = g * PB + i;
          // Transmittance, G . suffix colour and dL/dalpha (they carry the
          // error of every step), the per-pair terms and their sums: all
          // FP64.  dL/dalpha = (T G.c - G.S) / (1 - alpha) with T the
          // transmittance behind the splat; G.S then takes the splat's share
          // w G.c.  A masked pair gets inv = 0, which zeroes w, dL/dalpha and
          // with them every term it would add.
          const double inv = contrib[i] ? rcp_d(e[i].oma) : 0.0;
          const double Ti = T[j] * inv;
          const double w = e[i].alpha * Ti;
          const double g0 = G0[j], g1 = G1[j], g2 = G2[j];
          const double GdC = g0 * cr + g1 * cg + g2 * cb;
          const double dLda = fma(T[j], GdC, -GS[j]) * inv;
          GS[j] = fma(w, GdC, GS[j]);
          T[j] = contrib[i] ? Ti : T[j];
          double om = 1.0;
          if constexpr (AG != kAgsOff) {
            const double xa = qq[i] * rp.ags_scale;
            om = ags_weight(xa);
          }
          // q = d^T cov^-1 d with d = pixel - centre and u = cov^-1 d:
          // dq/dcentre = -2 u, dq/dcov = -u u^T.  The covariance (not the
          // conic) is what the projection backward differentiates, so its
          // gradient is summed here; going through the inverse after the sum
          // would amplify the sum's rounding for elongated splats.  The sums
          // take U = 2u; the factors are applied to the wave sums.
          // dL/dq = dL/dalpha o f'(q): linear -omega / (2 lambda D); Gaussian
          // -f / (2 lambda^2); quadratic -1 / lambda^2; Laplacian
          // -f / (2 lambda D); raised cosine -pi sin(pi D/lambda) / (4 lambda D)
          // (invD is 0 at D = 0: no slope at the apex).  No geometric
          // gradient at the alpha clamp (nc = 0).
          double gq;
          if constexpr (KF == LS_KERNEL_LINEAR) gq = (nol * e[i].nc) * dLda * om * e[i].invD;
          else if constexpr (KF == LS_KERNEL_GAUSSIAN)
            gq = -(dLda * e[i].alpha) * (rp.ghalf * e[i].nc);
          else if constexpr (KF == LS_KERNEL_QUADRATIC) gq = -(o * dLda) * (rp.inv_lam2 * e[i].nc);
          else if constexpr (KF == LS_KERNEL_LAPLACIAN)
            gq = -0.5 * (dLda * e[i].alpha) * (rp.inv_lam * e[i].nc) * e[i].invD;
          else
            gq = -0.7853981633974483 * (o * dLda) * (rp.inv_lam * e[i].nc) * e[i].sx * e[i].invD;
          const double Ux = fma(qb, ly[j], Ux0);
          const double Uy = fma(qc2, ly[j], Uy0);
          const double gux = gq * Ux, guy = gq * Uy;
          gv[0] += gux;                    // x -1
          gv[1] += guy;                    // x -1
          gv[2] = fma(gux, Ux, gv[2]);     // x -1/4
          gv[3] = fma(gux, Uy, gv[3]);     // x -1/2
          gv[4] = fma(guy, Uy, gv[4]);     // x -1/4
          // opacity and colour: scaled by omega only under the whole-pair scope
          const double go = ags_whole<AG>() ? dLda * e[i].nc * om : dLda * e[i].nc;
          gv[5] = fma(e[i].f, go, gv[5]);
          const double ws = ags_whole<AG>() ? w * om : w;
          gv[6] = fma(ws, g0, gv[6]);
          gv[7] = fma(ws, g1, gv[7]);
          gv[8] = fma(ws, g2, gv[8]);
        }
      }
      if (!used) continue;
      // wave-wide FP64 sums (all lanes active here): lane f < 9 holds
      // field f times its factor
      static_assert(kGrad2d == 9, "nine fields");
      const double sv = wave_sum9_lds(gv, s_red, lane) * fac;
      if (partial) {
        // deterministic mode: the tile's sums of this entry go to the
        // entry's slot in pair order; the pair sums are formed afterwards
        int cc = 0;
        while (cc + 1 < K && s_segpre[cc + 1] <= pos) ++cc;
        const int64_t ent = s_segbase[cc] + (pos - s_segpre[cc]);
        if (lane < kGrad2d) partial[(int64_t)det_slot[ent] * kGrad2d + lane] = sv;
      } else if (lane < kGrad2d && sv != 0.0) {
        unsafeAtomicAdd(grad2d + (int64_t)lane * M + (int64_t)st.m[k], sv);
      }
    }
  }
}

// zero the deterministic mode's per-entry sums of the n built entries
// (entry-major: the nine sums of entry e at 9 e)
__global__ void det_zero_kernel(double* __restrict__ partial, const int64_t* __restrict__ n_dev) {
  const int64_t n = *n_dev * kGrad2d;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
    partial[i] = 0.0;
}

__global__ void zero_kernel(float* __restrict__ p, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
    p[i] = 0.f;
}

RasterParams make_params(const ls_config* cfg) {
  RasterParams rp;
  rp.lam2 = (double)cfg->lambda * (double)cfg->lambda;
  const double ext = (double)kernel_extent(cfg);
  rp.qmax = ext * ext;
  rp.inv_lam = 1.0 / (double)cfg->lambda;
  rp.inv_lam2 = rp.inv_lam * rp.inv_lam;
  rp.ghalf = 0.5 * rp.inv_lam2;
  rp.amin = cfg->alpha_min;
  rp.amin_pos = rp.amin > 0.0 ? rp.amin : 4.9406564584124654e-324;   // smallest positive double
  rp.amax = cfg->alpha_max;
  rp.oma_max = 1.0 - (double)cfg->alpha_max;
  rp.tmin = cfg->t_min;
  rp.bg0 = cfg->bg[0];
  rp.bg1 = cfg->bg[1];
  rp.bg2 = cfg->bg[2];
  rp.ags = cfg->ags;
  rp.ags_arg = cfg->ags_arg;
  rp.ags_scope = cfg->ags_scope;
  rp.ags_scale = cfg->ags_arg ? rp.inv_lam2 : 1.0;
  return rp;
}

}  // namespace

__global__ void fill_u32(uint32_t* __restrict__ p, int64_t n, uint32_t v) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
    p[i] = v;
}

hipError_t launch_raster_fwd(const Plan& p, const ls_config* cfg, char* ws, float* image,
                             float* final_T, int32_t* last, hipStream_t s) {
  if (p.T == 0) return hipSuccess;
  const CamInfo* cams = (const CamInfo*)(ws + p.lay.cams);
  const int64_t* ranges = (const int64_t*)(ws + p.lay.ranges);
  const int64_t* chunk_base = (const int64_t*)(ws + p.lay.chunk_base);
  const uint32_t* vals = (const uint32_t*)(ws + p.lay.vals);
  const ProjRec* proj = (const ProjRec*)(ws + p.lay.proj);
  double4* state = (double4*)(ws + p.state);
  uint32_t* tile_contrib = (uint32_t*)(ws + p.lay.tile_contrib);
  uint8_t* done = (uint8_t*)(ws + p.done);
  uint32_t* alive = (uint32_t*)(ws + p.alive);
  RasterParams rp = make_params(cfg);
  const int npix = cfg->tile_w * cfg->tile_h;
  const int batch = cfg->batch ? cfg->batch : npix;
  dim3 grid((unsigned)p.T);
  hipError_t e;
  if (p.K > 1) {
    int64_t blocks = std::min<int64_t>((p.T + 255) / 256, 4096);
    hipLaunchKernelGGL(fill_u32, dim3((unsigned)blocks), dim3(256), 0, s, alive, p.T, 1u);
    if ((e = hipGetLastError())) return e;
  }
  for (int c = 0; c < p.K; ++c) {
    if (p.K > 1 && (e = launch_chunk_bin(p, c, ws, s))) return e;
    ProfScope ps("raster_fwd", s);
#define LS_FWD(TW_, TH_, KF_)                                                                      \
  hipLaunchKernelGGL((raster_fwd_kernel<TW_, TH_, KF_>), grid, dim3(raster_threads<TW_, TH_>()), 0, \
                     s, cams, p.C, ranges, p.T, c, p.K, chunk_base, vals, proj, p.M, batch, rp,      \
                     state, done, alive, image, final_T, last, tile_contrib, (double*)(ws + p.t64))
#define LS_FWD_K(TW_, TH_)                                                                         \
  switch (cfg->kernel) {                                                                           \
    case LS_KERNEL_GAUSSIAN: LS_FWD(TW_, TH_, LS_KERNEL_GAUSSIAN); break;                          \
    case LS_KERNEL_LAPLACIAN: LS_FWD(TW_, TH_, LS_KERNEL_LAPLACIAN); break;                        \
    case LS_KERNEL_COSINE: LS_FWD(TW_, TH_, LS_KERNEL_COSINE); break;                              \
    case LS_KERNEL_QUADRATIC: LS_FWD(TW_, TH_, LS_KERNEL_QUADRATIC); break;                        \
    default: LS_FWD(TW_, TH_, LS_KERNEL_LINEAR); break;                                           \
  }
    if (cfg->tile_w == 16 && cfg->tile_h == 16) LS_FWD_K(16, 16)
    else if (cfg->tile_w == 16 && cfg->tile_h == 8) LS_FWD_K(16, 8)
    else if (cfg->tile_w == 8 && cfg->tile_h == 8) LS_FWD_K(8, 8)
    else LS_FWD_K(32, 8)
#undef LS_FWD_K
#undef LS_FWD
    if ((e = hipGetLastError())) return e;
  }
  return hipSuccess;
}

hipError_t launch_raster_bwd(const Plan& p, const ls_config* cfg, const ls_splats* sp, char* ws,
                             const float* final_T, const int32_t* last, const float* dL_dimage,
                             const float* dL_dalpha, const ls_grads* g, hipStream_t s) {
  double* grad2d = (double*)(ws + p.lay.grad2d);
  const int64_t ng = 2 * (int64_t)kGrad2d * p.M;   // as float words
  if (ng > 0) {
    int64_t blocks = std::min<int64_t>((ng + 255) / 256, 8192);
    ProfScope ps("zero_grad2d", s);
    hipLaunchKernelGGL(zero_kernel, dim3((unsigned)blocks), dim3(256), 0, s, (float*)grad2d, ng);
  }
  if (p.T > 0) {
    const CamInfo* cams = (const CamInfo*)(ws + p.lay.cams);
    const int64_t* ranges = (const int64_t*)(ws + p.lay.ranges);
    const int64_t* chunk_base = (const int64_t*)(ws + p.lay.chunk_base);
    const uint32_t* vals = (const uint32_t*)(ws + p.lay.vals);
    const ProjRec* proj = (const ProjRec*)(ws + p.lay.proj);
    RasterParams rp = make_params(cfg);
    const int npix = cfg->tile_w * cfg->tile_h;
    const int batch = cfg->batch ? cfg->batch : npix;
    double* partial = nullptr;
    const uint32_t* det_slot = nullptr;
    if (cfg->deterministic && p.cap > 0) {
      hipError_t e = launch_det_order(p, ws, s);
      if (e != hipSuccess) return e;
      det_slot = det_slots(p, ws);
      // entries the backward pass does not stage (culled, or past every
      // pixel's last contributor) keep zero sums
      partial = (double*)(ws + p.det_partial);
      const unsigned blocks = (unsigned)std::min<int64_t>((kGrad2d * p.cap + 255) / 256, 8192);
      ProfScope ps("det_zero", s);
      hipLaunchKernelGGL(det_zero_kernel, dim3(blocks), dim3(256), 0, s, partial, chunk_base + p.K);
    }
    dim3 grid((unsigned)p.T);
    ProfScope ps("raster_bwd", s);
    // AGS is defined for the linear kernel only (checked by the entry point)
    const int ag = !cfg->ags ? kAgsOff : cfg->ags_scope ? kAgsWhole : kAgsGeo;
#define LS_BWD(TW_, TH_, KF_, AG_)                                                                 \
  hipLaunchKernelGGL((raster_bwd_kernel<TW_, TH_, KF_, AG_>), grid, dim3(64), 0, s,                \
                     cams, p.C, ranges, p.T, p.K, chunk_base, vals, proj, p.M, batch, rp,      \
                     (const double*)(ws + p.t64), last, dL_dimage, dL_dalpha, grad2d, partial, det_slot)
#define LS_BWD_K(TW_, TH_)                                                                         \
  switch (cfg->kernel) {                                                                           \
    case LS_KERNEL_GAUSSIAN: LS_BWD(TW_, TH_, LS_KERNEL_GAUSSIAN, kAgsOff); break;                 \
    case LS_KERNEL_LAPLACIAN: LS_BWD(TW_, TH_, LS_KERNEL_LAPLACIAN, kAgsOff); break;               \
    case LS_KERNEL_COSINE: LS_BWD(TW_, TH_, LS_KERNEL_COSINE, kAgsOff); break;                     \
    case LS_KERNEL_QUADRATIC: LS_BWD(TW_, TH_, LS_KERNEL_QUADRATIC, kAgsOff); break;               \
    default:                                                                                       \
      switch (ag) {                                                                                \
        case kAgsGeo: LS_BWD(TW_, TH_, LS_KERNEL_LINEAR, kAgsGeo); break;                          \
        case kAgsWhole: LS_BWD(TW_, TH_, LS_KERNEL_LINEAR, kAgsWhole); break;                      \
        default: LS_BWD(TW_, TH_, LS_KERNEL_LINEAR, kAgsOff); break;                               \
      }                                                                                            \
      break;                                                                                       \
  }
    if (cfg->tile_w == 16 && cfg->tile_h == 16) LS_BWD_K(16, 16)
    else if (cfg->tile_w == 16 && cfg->tile_h == 8) LS_BWD_K(16, 8)
    else if (cfg->tile_w == 8 && cfg->tile_h == 8) LS_BWD_K(8, 8)
    else LS_BWD_K(32, 8)
#undef LS_BWD_K
#undef LS_BWD
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  if (p.T > 0 && cfg->deterministic && p.cap > 0) {
    hipError_t e = launch_det_reduce(p, ws, s);
    if (e != hipSuccess) return e;
  }
  return launch_project_bwd(p, cfg, sp, ws, g, s);
}

}  // namespace lsplat
