// Per-tile compositing with the linear kernel (forward) and its reverse pass.
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
// One workgroup per tile, one lane per pixel (wave64: a 16x16 tile is four
// waves of 16x4 pixels).  The tile's list is consumed in batches staged in
// LDS (gathered 64-byte records, converted to tile-relative FP64 centres).
// Blocks are remapped so that each XCD (blocks are dealt round-robin over
// the 8 XCDs) works on one contiguous band of tiles and keeps the records of
// neighbouring tiles in its own L2.
//
// Numerics: the quadratic form is evaluated in FP64 (full rate on CDNA, and
// free of the FP32 cancellation of needle-shaped splats); everything after
// D'^2 is FP32.  1 - alpha is formed as (1 - o) + o D'/lambda, a sum of two
// non-negative terms, so transmittance keeps full relative precision when
// alpha is close to 1.
#include <algorithm>

#include "internal.h"

namespace lsplat {

namespace {

struct RasterParams {
  double lam2;        // lambda^2: D' >= lambda <=> outside the support
  double inv_lam;     // 1 / lambda
  double amin, amax, oma_max, tmin;
  float bg0, bg1, bg2;
  float inv_lam_f;
  int ags, ags_arg, ags_scope;
};

// alpha and 1 - alpha of one (pixel, splat) pair, in FP64.  Shared by the
// forward and backward kernels and evaluated without contraction, so both
// kernels take every skip/stop decision identically.
struct PairEval {
  double D, alpha, oma;
  bool clamped;
};

__device__ __forceinline__ double quad_form(double dx, double dy, double A, double B2, double C) {
  return fma(dx, fma(A, dx, B2 * dy), (C * dy) * dy);
}

__device__ __forceinline__ PairEval pair_eval(double q, double o, const RasterParams& rp) {
#pragma clang fp contract(off)
  PairEval e;
  e.D = sqrt(q);
  const double t = o * (e.D * rp.inv_lam);
  e.alpha = o - t;
  e.oma = (1.0 - o) + t;
  e.clamped = e.alpha > rp.amax;
  if (e.clamped) {
    e.alpha = rp.amax;
    e.oma = rp.oma_max;
  }
  return e;
}

__device__ __forceinline__ int64_t xcd_remap(int64_t b, int64_t nb) {
  const int64_t x = b & 7, k = b >> 3;
  const int64_t q = nb >> 3, r = nb & 7;
  return x * q + (x < r ? x : r) + k;
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

template <int NT>
struct Stage {
  double ox[NT], oy[NT];     // centre relative to the tile's first pixel centre
  double A[NT], B2[NT], C[NT];
  float r[NT], g[NT], b[NT], o[NT];
};

template <int NT>
__device__ __forceinline__ void stage_one(Stage<NT>& st, int i, const ProjRec& rec, double x0c,
                                          double y0c) {
  st.ox[i] = rec.mx - x0c;
  st.oy[i] = rec.my - y0c;
  st.A[i] = rec.A;
  st.B2[i] = 2.0 * rec.B;
  st.C[i] = rec.C;
  st.r[i] = rec.r;
  st.g[i] = rec.g;
  st.b[i] = rec.b;
  st.o[i] = rec.o;
}

template <int TW, int TH>
__global__ __launch_bounds__(TW* TH) void raster_fwd_kernel(
    const CamInfo* __restrict__ cams, int C, const int64_t* __restrict__ ranges,
    const uint32_t* __restrict__ vals, const ProjRec* __restrict__ proj, int64_t M, int batch,
    RasterParams rp, float* __restrict__ image, float* __restrict__ final_T,
    int32_t* __restrict__ last) {
  constexpr int NT = TW * TH;
  __shared__ Stage<NT> st;
  const int tid = threadIdx.x;
  const int64_t tile = xcd_remap(blockIdx.x, gridDim.x);
  const int c = cam_of_tile(cams, C, tile);
  const CamInfo& ci = cams[c];
  const int64_t local = tile - ci.tile_off;
  const int ty = (int)(local / ci.GX), tx = (int)(local % ci.GX);
  const int lx = tid % TW, ly = tid / TW;
  const int px = tx * TW + lx, py = ty * TH + ly;
  const bool inside = (px < ci.W) && (py < ci.H);
  const double x0c = (double)(tx * TW) + 0.5, y0c = (double)(ty * TH) + 0.5;
  const double lxd = (double)lx, lyd = (double)ly;
  const int64_t start = ranges[tile], end = ranges[tile + 1];

  double T = 1.0, cr = 0.0, cg = 0.0, cb = 0.0;
  int32_t lastc = 0;
  bool done = !inside;
  for (int64_t b0 = start; b0 < end; b0 += batch) {
    if (__syncthreads_count(!done) == 0) break;
    const int nb = (int)((end - b0) < batch ? (end - b0) : batch);
    if (tid < nb) {
      const uint32_t m = vals[b0 + tid];
      stage_one(st, tid, proj[m < (uint64_t)M ? m : 0], x0c, y0c);
    }
    __syncthreads();
    if (!done) {
      for (int j = 0; j < nb; ++j) {
        const double dx = lxd - st.ox[j];
        const double dy = lyd - st.oy[j];
        const double q = quad_form(dx, dy, st.A[j], st.B2[j], st.C[j]);
        if (!(q < rp.lam2)) continue;
        const PairEval e = pair_eval(q, (double)st.o[j], rp);
        if (!(e.alpha > 0.0) || e.alpha < rp.amin) continue;
        const double Tn = T * e.oma;
        if (Tn < rp.tmin) {
          done = true;
          break;
        }
        const double w = e.alpha * T;
        cr = fma((double)st.r[j], w, cr);
        cg = fma((double)st.g[j], w, cg);
        cb = fma((double)st.b[j], w, cb);
        T = Tn;
        lastc = (int32_t)(b0 - start) + j + 1;
      }
    }
  }
  if (inside) {
    const int64_t pix = ci.pix_off + (int64_t)py * ci.W + px;
    const int64_t plane = (int64_t)ci.W * ci.H;
    const int64_t ib = 3 * ci.pix_off + (int64_t)py * ci.W + px;
    image[ib] = (float)(cr + T * (double)rp.bg0);
    image[ib + plane] = (float)(cg + T * (double)rp.bg1);
    image[ib + 2 * plane] = (float)(cb + T * (double)rp.bg2);
    final_T[pix] = (float)T;
    last[pix] = lastc;
  }
}

template <int TW, int TH>
__global__ __launch_bounds__(TW* TH) void raster_bwd_kernel(
    const CamInfo* __restrict__ cams, int C, const int64_t* __restrict__ ranges,
    const uint32_t* __restrict__ vals, const ProjRec* __restrict__ proj, int64_t M, int batch,
    RasterParams rp, const float* __restrict__ final_T, const int32_t* __restrict__ last,
    const float* __restrict__ dL_dimage, float* __restrict__ grad2d) {
  constexpr int NT = TW * TH;
  constexpr int NW = NT / 64;
  __shared__ Stage<NT> st;
  __shared__ uint32_t s_m[NT];
  __shared__ float s_acc[kGrad2d][NT];
  __shared__ int32_t s_max[NW];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t tile = xcd_remap(blockIdx.x, gridDim.x);
  const int c = cam_of_tile(cams, C, tile);
  const CamInfo& ci = cams[c];
  const int64_t local = tile - ci.tile_off;
  const int ty = (int)(local / ci.GX), tx = (int)(local % ci.GX);
  const int lx = tid % TW, ly = tid / TW;
  const int px = tx * TW + lx, py = ty * TH + ly;
  const bool inside = (px < ci.W) && (py < ci.H);
  const double x0c = (double)(tx * TW) + 0.5, y0c = (double)(ty * TH) + 0.5;
  const double lxd = (double)lx, lyd = (double)ly;
  const int64_t start = ranges[tile];
  const int64_t len = ranges[tile + 1] - start;

  double T = 1.0, G0 = 0.0, G1 = 0.0, G2 = 0.0;
  int32_t mylast = 0;
  if (inside) {
    const int64_t pix = ci.pix_off + (int64_t)py * ci.W + px;
    const int64_t plane = (int64_t)ci.W * ci.H;
    const int64_t ib = 3 * ci.pix_off + (int64_t)py * ci.W + px;
    T = final_T[pix];
    mylast = last[pix];
    mylast = mylast < 0 ? 0 : (mylast > len ? (int32_t)len : mylast);
    G0 = dL_dimage[ib];
    G1 = dL_dimage[ib + plane];
    G2 = dL_dimage[ib + 2 * plane];
  }
  // suffix colour behind the current splat, starting with the background term
  double S0 = T * (double)rp.bg0, S1 = T * (double)rp.bg1, S2 = T * (double)rp.bg2;
  // tile-wide maximum of `last`
  int32_t mx = mylast;
  for (int d = 32; d > 0; d >>= 1) {
    int32_t y = __shfl_xor(mx, d, 64);
    mx = y > mx ? y : mx;
  }
  if (lane == 0) s_max[wave] = mx;
  __syncthreads();
  int32_t maxlast = 0;
#pragma unroll
  for (int w = 0; w < NW; ++w) maxlast = s_max[w] > maxlast ? s_max[w] : maxlast;

  for (int32_t hi = maxlast; hi > 0; hi -= batch) {
    const int32_t lo = hi - batch > 0 ? hi - batch : 0;
    const int nb = hi - lo;
    __syncthreads();
    if (tid < nb) {
      uint32_t m = vals[start + lo + tid];
      if (m >= (uint64_t)M) m = 0;   // unreachable for a valid list
      s_m[tid] = m;
      stage_one(st, tid, proj[m], x0c, y0c);
    }
    for (int i = tid; i < kGrad2d * NT; i += NT) (&s_acc[0][0])[i] = 0.f;
    __syncthreads();
    for (int jj = nb - 1; jj >= 0; --jj) {
      const int32_t j = lo + jj;
      float gv[kGrad2d];
#pragma unroll
      for (int f = 0; f < kGrad2d; ++f) gv[f] = 0.f;
      bool contrib = false;
      if (j < mylast) {
        const double dx = lxd - st.ox[jj];
        const double dy = lyd - st.oy[jj];
        const double A = st.A[jj], B2 = st.B2[jj], Cc = st.C[jj];
        const double q = quad_form(dx, dy, A, B2, Cc);
        if (q < rp.lam2) {
          const double o = (double)st.o[jj];
          const PairEval e = pair_eval(q, o, rp);
          if (e.alpha > 0.0 && e.alpha >= rp.amin) {
            contrib = true;
            const double inv = 1.0 / e.oma;
            const double Ti = T * inv;
            const double w = e.alpha * Ti;
            const double cr = st.r[jj], cg = st.g[jj], cb = st.b[jj];
            double g_r = w * G0, g_g = w * G1, g_b = w * G2;
            const double GdC = G0 * cr + G1 * cg + G2 * cb;
            const double GdS = G0 * S0 + G1 * S1 + G2 * S2;
            const double dLda = Ti * GdC - GdS * inv;
            S0 = fma(cr, w, S0);
            S1 = fma(cg, w, S1);
            S2 = fma(cb, w, S2);
            T = Ti;
            const double Dl = e.D * rp.inv_lam;
            double om = 1.0;
            if (rp.ags) {
              const float arg = (float)(rp.ags_arg ? Dl : e.D);
              om = (double)__expf(-arg * arg);
            }
            double g_o = 0.0;
            if (!e.clamped) {
              g_o = (1.0 - Dl) * dLda;
              const double dLdD = -(o * dLda) * rp.inv_lam * om;
              if (e.D > 0.0) {
                const double gq = 0.5 * dLdD / e.D;
                gv[0] = (float)(-2.0 * gq * (A * dx + 0.5 * B2 * dy));
                gv[1] = (float)(-2.0 * gq * (0.5 * B2 * dx + Cc * dy));
                gv[2] = (float)(gq * dx * dx);
                gv[3] = (float)(2.0 * gq * dx * dy);
                gv[4] = (float)(gq * dy * dy);
              }
            }
            if (rp.ags_scope) {
              g_o *= om;
              g_r *= om;
              g_g *= om;
              g_b *= om;
            }
            gv[5] = (float)g_o;
            gv[6] = (float)g_r;
            gv[7] = (float)g_g;
            gv[8] = (float)g_b;
          }
        }
      }
      // wave-wide sums (all lanes active here), one LDS add per wave
      if (__builtin_amdgcn_ballot_w64(contrib) != 0ull) {
#pragma unroll
        for (int f = 0; f < kGrad2d; ++f) {
          const float s = wave_sum_to_lane63(gv[f]);
          if (lane == 63 && s != 0.f) atomicAdd(&s_acc[f][jj], s);
        }
      }
    }
    __syncthreads();
    if (tid < nb) {
      const int64_t m = (int64_t)s_m[tid];
#pragma unroll
      for (int f = 0; f < kGrad2d; ++f) {
        const float v = s_acc[f][tid];
        if (v != 0.f) unsafeAtomicAdd(grad2d + (int64_t)f * M + m, v);
      }
    }
  }
}

__global__ void zero_kernel(float* __restrict__ p, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
    p[i] = 0.f;
}

RasterParams make_params(const ls_config* cfg) {
  RasterParams rp;
  rp.lam2 = (double)cfg->lambda * (double)cfg->lambda;
  rp.inv_lam = 1.0 / (double)cfg->lambda;
  rp.inv_lam_f = (float)rp.inv_lam;
  rp.amin = cfg->alpha_min;
  rp.amax = cfg->alpha_max;
  rp.oma_max = 1.0 - (double)cfg->alpha_max;
  rp.tmin = cfg->t_min;
  rp.bg0 = cfg->bg[0];
  rp.bg1 = cfg->bg[1];
  rp.bg2 = cfg->bg[2];
  rp.ags = cfg->ags;
  rp.ags_arg = cfg->ags_arg;
  rp.ags_scope = cfg->ags_scope;
  return rp;
}

}  // namespace

hipError_t launch_raster_fwd(const Plan& p, const ls_config* cfg, char* ws, float* image,
                             float* final_T, int32_t* last, hipStream_t s) {
  if (p.T == 0) return hipSuccess;
  const CamInfo* cams = (const CamInfo*)(ws + p.lay.cams);
  const int64_t* ranges = (const int64_t*)(ws + p.lay.ranges);
  const uint32_t* vals = (const uint32_t*)(ws + p.lay.vals);
  const ProjRec* proj = (const ProjRec*)(ws + p.lay.proj);
  RasterParams rp = make_params(cfg);
  const int npix = cfg->tile_w * cfg->tile_h;
  const int batch = cfg->batch ? cfg->batch : npix;
  dim3 grid((unsigned)p.T);
  ProfScope ps("raster_fwd", s);
#define LS_FWD(TW_, TH_)                                                                        \
  hipLaunchKernelGGL((raster_fwd_kernel<TW_, TH_>), grid, dim3(TW_ * TH_), 0, s, cams, p.C, ranges, \
                     vals, proj, p.M, batch, rp, image, final_T, last)
  if (cfg->tile_w == 16 && cfg->tile_h == 16) LS_FWD(16, 16);
  else if (cfg->tile_w == 16 && cfg->tile_h == 8) LS_FWD(16, 8);
  else if (cfg->tile_w == 8 && cfg->tile_h == 8) LS_FWD(8, 8);
  else LS_FWD(32, 8);
#undef LS_FWD
  return hipGetLastError();
}

hipError_t launch_raster_bwd(const Plan& p, const ls_config* cfg, const ls_splats* sp, char* ws,
                             const float* final_T, const int32_t* last, const float* dL_dimage,
                             const ls_grads* g, hipStream_t s) {
  float* grad2d = (float*)(ws + p.lay.grad2d);
  const int64_t ng = (int64_t)kGrad2d * p.M;
  if (ng > 0) {
    int64_t blocks = std::min<int64_t>((ng + 255) / 256, 8192);
    ProfScope ps("zero_grad2d", s);
    hipLaunchKernelGGL(zero_kernel, dim3((unsigned)blocks), dim3(256), 0, s, grad2d, ng);
  }
  if (p.T > 0) {
    const CamInfo* cams = (const CamInfo*)(ws + p.lay.cams);
    const int64_t* ranges = (const int64_t*)(ws + p.lay.ranges);
    const uint32_t* vals = (const uint32_t*)(ws + p.lay.vals);
    const ProjRec* proj = (const ProjRec*)(ws + p.lay.proj);
    RasterParams rp = make_params(cfg);
    const int npix = cfg->tile_w * cfg->tile_h;
    const int batch = cfg->batch ? cfg->batch : npix;
    dim3 grid((unsigned)p.T);
    ProfScope ps("raster_bwd", s);
#define LS_BWD(TW_, TH_)                                                                         \
  hipLaunchKernelGGL((raster_bwd_kernel<TW_, TH_>), grid, dim3(TW_ * TH_), 0, s, cams, p.C, ranges, \
                     vals, proj, p.M, batch, rp, final_T, last, dL_dimage, grad2d)
    if (cfg->tile_w == 16 && cfg->tile_h == 16) LS_BWD(16, 16);
    else if (cfg->tile_w == 16 && cfg->tile_h == 8) LS_BWD(16, 8);
    else if (cfg->tile_w == 8 && cfg->tile_h == 8) LS_BWD(8, 8);
    else LS_BWD(32, 8);
#undef LS_BWD
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return launch_project_bwd(p, cfg, sp, ws, g, s);
}

}  // namespace lsplat
