// Training-step stages around the rasterizer: the Adam update (Kingma and Ba
// 2015) and the densification statistics and decision with the thresholds of
// the paper's densification table (implementation section).  All three are
// streaming kernels bound by HBM: one pass over their arrays, coalesced, with
// the arithmetic in FP64 on FP32 storage.
#include <math.h>

#include <algorithm>

#include "internal.h"

namespace lsplat {

namespace {

constexpr int kTrainThreads = 256;
constexpr int64_t kMaxTrainBlocks = 8192;   // grid-stride beyond this

struct AdamCoef {
  double lr_bc1;     // lr / (1 - beta1^t)
  double inv_bc2;    // 1 / (1 - beta2^t)
  double b1, b2, eps;
};

// bias corrections of step *step_dev (the graph-replayable variant reads the
// step from device memory; every thread forms the same two coefficients)
__device__ __forceinline__ AdamCoef adam_coef_dev(AdamCoef k, double lr, const int64_t* step_dev) {
  const double t = (double)*step_dev;
  k.lr_bc1 = lr / (1.0 - pow(k.b1, t));
  k.inv_bc2 = 1.0 / (1.0 - pow(k.b2, t));
  return k;
}

__device__ __forceinline__ void adam_one(float& p, float g, float& m, float& v, const AdamCoef& k) {
  const double gd = g;
  const double md = k.b1 * (double)m + (1.0 - k.b1) * gd;
  const double vd = k.b2 * (double)v + (1.0 - k.b2) * gd * gd;
  p = (float)((double)p - k.lr_bc1 * md / (sqrt(vd * k.inv_bc2) + k.eps));
  m = (float)md;
  v = (float)vd;
}

// four elements per thread through 16-byte accesses; the host takes this
// path only when every pointer is 16-byte aligned
__global__ __launch_bounds__(kTrainThreads) void adam_vec4_kernel(
    int64_t n4, float4* __restrict__ p, const float4* __restrict__ g, float4* __restrict__ m,
    float4* __restrict__ v, AdamCoef k, double lr, const int64_t* __restrict__ step_dev) {
  if (step_dev) k = adam_coef_dev(k, lr, step_dev);
  const int64_t stride = (int64_t)gridDim.x * kTrainThreads;
  for (int64_t i = (int64_t)blockIdx.x * kTrainThreads + threadIdx.x; i < n4; i += stride) {
    float4 pp = p[i], mm = m[i], vv = v[i];
    const float4 gg = g[i];
    adam_one(pp.x, gg.x, mm.x, vv.x, k);
    adam_one(pp.y, gg.y, mm.y, vv.y, k);
    adam_one(pp.z, gg.z, mm.z, vv.z, k);
    adam_one(pp.w, gg.w, mm.w, vv.w, k);
    p[i] = pp;
    m[i] = mm;
    v[i] = vv;
  }
}

__global__ __launch_bounds__(kTrainThreads) void adam_kernel(
    int64_t lo, int64_t n, float* __restrict__ p, const float* __restrict__ g,
    float* __restrict__ m, float* __restrict__ v, AdamCoef k, double lr,
    const int64_t* __restrict__ step_dev) {
  if (step_dev) k = adam_coef_dev(k, lr, step_dev);
  const int64_t stride = (int64_t)gridDim.x * kTrainThreads;
  for (int64_t i = lo + (int64_t)blockIdx.x * kTrainThreads + threadIdx.x; i < n; i += stride) {
    float pp = p[i], mm = m[i], vv = v[i];
    adam_one(pp, g[i], mm, vv, k);
    p[i] = pp;
    m[i] = mm;
    v[i] = vv;
  }
}

unsigned grid_for(int64_t n) {
  return (unsigned)std::max<int64_t>(1, std::min<int64_t>((n + kTrainThreads - 1) / kTrainThreads,
                                                          kMaxTrainBlocks));
}

// Statistics of one backward pass, one thread per splat over the cameras of
// its scene: per visible pair (support on at least one tile) the NDC-space
// norm of dL/d(projected centre), a view count, and the support ellipse's
// semi-major axis over the larger image side.  The conic is the inverse of
// the dilated 2D covariance, so that axis is ext / sqrt(smallest conic
// eigenvalue), the eigenvalue taken as det / largest to avoid cancellation.
__global__ __launch_bounds__(kTrainThreads) void densify_stats_kernel(
    const CamInfo* __restrict__ cams, int C, int64_t N, int64_t M, double ext,
    const ProjRec* __restrict__ proj, const uint32_t* __restrict__ ntiles,
    const double* __restrict__ grad2d, float* __restrict__ acc_grad,
    int32_t* __restrict__ acc_count, float* __restrict__ acc_ext) {
  const int64_t i = (int64_t)blockIdx.x * kTrainThreads + threadIdx.x;
  if (i >= N) return;
  double gsum = 0.0, emax = 0.0;
  int32_t cnt = 0;
  for (int c = 0; c < C; ++c) {
    const CamInfo& ci = cams[c];
    if (i < ci.splat_lo || i >= ci.splat_hi) continue;
    const int64_t m = ci.pair_off + (i - ci.splat_lo);
    if (ntiles[m] == 0) continue;
    const double gx = grad2d[m] * (0.5 * ci.W), gy = grad2d[M + m] * (0.5 * ci.H);
    gsum += sqrt(gx * gx + gy * gy);
    ++cnt;
    const ProjRec pr = proj[m];
    const double h = 0.5 * (pr.A - pr.C);
    const double big = 0.5 * (pr.A + pr.C) + sqrt(h * h + pr.B * pr.B);
    const double small = (pr.A * pr.C - pr.B * pr.B) / big;
    const double r = ext / sqrt(small);
    emax = fmax(emax, r / (double)max(ci.W, ci.H));
  }
  if (cnt == 0) return;
  acc_grad[i] = (float)((double)acc_grad[i] + gsum);
  acc_count[i] += cnt;
  acc_ext[i] = (float)fmax((double)acc_ext[i], emax);
}

struct SelectArgs {
  double grad, s2g, s3g, s2p, s3p, op, scene_scale;
  int32_t grow2d, prune_big;
};

__global__ void counts_zero_kernel(unsigned long long* __restrict__ c) {
  if (threadIdx.x < 3) c[threadIdx.x] = 0ull;
}

// The decision compares in FP64 on the stored FP32 statistics; action bits
// 1 duplicate, 2 split, 4 prune.  Each thread counts its own decisions over
// the grid-stride loop; the block sums them in LDS and adds once per counter.
__global__ __launch_bounds__(kTrainThreads) void densify_select_kernel(
    int64_t N, SelectArgs a, const float* __restrict__ scales, const float* __restrict__ opac,
    const float* __restrict__ acc_grad, const int32_t* __restrict__ acc_count,
    const float* __restrict__ acc_ext, uint8_t* __restrict__ action,
    unsigned long long* __restrict__ counts) {
  __shared__ unsigned int red[3][kTrainThreads / 64];
  const int64_t stride = (int64_t)gridDim.x * kTrainThreads;
  unsigned int n_dup = 0, n_split = 0, n_prune = 0;
  for (int64_t i = (int64_t)blockIdx.x * kTrainThreads + threadIdx.x; i < N; i += stride) {
    int act = 0;
    const int32_t cnt = acc_count[i];
    const bool high = cnt > 0 && (double)acc_grad[i] / (double)cnt > a.grad;
    const double s = (double)fmaxf(fmaxf(scales[i], scales[N + i]), scales[2 * N + i]);
    const bool small = s <= a.s3g * a.scene_scale;
    const double e = (double)acc_ext[i];
    const bool split = (high && !small) || (a.grow2d && e > a.s2g);
    if (split)
      act |= 2;
    else if (high && small)
      act |= 1;
    if ((double)opac[i] < a.op || (a.prune_big && (s > a.s3p * a.scene_scale || e > a.s2p)))
      act |= 4;
    action[i] = (uint8_t)act;
    n_dup += act & 1;
    n_split += (act >> 1) & 1;
    n_prune += (act >> 2) & 1;
  }
  if (!counts) return;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int d = 32; d > 0; d >>= 1) {
    n_dup += __shfl_xor(n_dup, d, 64);
    n_split += __shfl_xor(n_split, d, 64);
    n_prune += __shfl_xor(n_prune, d, 64);
  }
  if (lane == 0) {
    red[0][wave] = n_dup;
    red[1][wave] = n_split;
    red[2][wave] = n_prune;
  }
  __syncthreads();
  if (threadIdx.x < 3) {
    unsigned long long v = 0;
    for (int w = 0; w < kTrainThreads / 64; ++w) v += red[threadIdx.x][w];
    if (v) atomicAdd(counts + threadIdx.x, v);
  }
}

}  // namespace

hipError_t launch_adam(const ls_adam_params* prm, const int64_t* step_dev, int64_t n, float* p,
                       const float* g, float* m, float* v, hipStream_t s) {
  if (n == 0) return hipSuccess;
  AdamCoef k;
  const double t = (double)(step_dev ? 1 : prm->step);   // replaced in the kernel
  k.lr_bc1 = prm->lr / (1.0 - pow(prm->beta1, t));
  k.inv_bc2 = 1.0 / (1.0 - pow(prm->beta2, t));
  k.b1 = prm->beta1;
  k.b2 = prm->beta2;
  k.eps = prm->eps;
  ProfScope ps("adam", s);
  const bool aligned = ((uintptr_t)p | (uintptr_t)g | (uintptr_t)m | (uintptr_t)v) % 16 == 0;
  int64_t done = 0;
  if (aligned && n >= 4) {
    const int64_t n4 = n / 4;
    hipLaunchKernelGGL(adam_vec4_kernel, dim3(grid_for(n4)), dim3(kTrainThreads), 0, s, n4,
                       (float4*)p, (const float4*)g, (float4*)m, (float4*)v, k, prm->lr, step_dev);
    done = n4 * 4;
  }
  if (done < n)
    hipLaunchKernelGGL(adam_kernel, dim3(grid_for(n - done)), dim3(kTrainThreads), 0, s, done, n, p,
                       g, m, v, k, prm->lr, step_dev);
  return hipGetLastError();
}

hipError_t launch_densify_stats(const Plan& p, const ls_config* cfg, char* ws,
                                const ls_densify_acc* acc, hipStream_t s) {
  if (p.N == 0) return hipSuccess;
  ProfScope ps("densify_stats", s);
  hipLaunchKernelGGL(densify_stats_kernel, dim3((unsigned)((p.N + kTrainThreads - 1) / kTrainThreads)),
                     dim3(kTrainThreads), 0, s, (const CamInfo*)(ws + p.lay.cams), p.C, p.N, p.M,
                     (double)kernel_extent(cfg), (const ProjRec*)(ws + p.lay.proj),
                     (const uint32_t*)(ws + p.lay.ntiles), (const double*)(ws + p.lay.grad2d),
                     acc->grad, acc->count, acc->max_extent);
  return hipGetLastError();
}

hipError_t launch_densify_select(const ls_densify_params* prm, int64_t n, const float* scales,
                                 const float* opacity, const ls_densify_acc* acc, uint8_t* action,
                                 int64_t* counts, hipStream_t s) {
  ProfScope ps("densify_select", s);
  if (counts) hipLaunchKernelGGL(counts_zero_kernel, dim3(1), dim3(64), 0, s,
                                 (unsigned long long*)counts);
  if (n > 0) {
    SelectArgs a;
    a.grad = prm->grad_threshold;
    a.s2g = prm->grow_scale2d;
    a.s3g = prm->grow_scale3d;
    a.s2p = prm->prune_scale2d;
    a.s3p = prm->prune_scale3d;
    a.op = prm->prune_opacity;
    a.scene_scale = prm->scene_scale;
    a.grow2d = prm->grow2d;
    a.prune_big = prm->prune_big;
    const unsigned blocks = (unsigned)std::min<int64_t>((n + kTrainThreads - 1) / kTrainThreads, 2048);
    hipLaunchKernelGGL(densify_select_kernel, dim3(blocks), dim3(kTrainThreads), 0, s, n, a,
                       scales, opacity, acc->grad, acc->count, acc->max_extent, action,
                       (unsigned long long*)counts);
  }
  return hipGetLastError();
}

}  // namespace lsplat
