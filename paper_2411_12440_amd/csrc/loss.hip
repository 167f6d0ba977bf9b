// Training loss of the implementation section (Sec. 4.1, "Loss Functions"):
// per camera L = 0.6 L1 + 0.2 L2 + 0.2 (1 - SSIM) over its 3 x H x W image,
// and dL/dimage.  SSIM (Wang et al. 2004) with an 11 x 11 Gaussian window of
// sigma 1.5 (normalised), zero padding, C1 = 0.01^2, C2 = 0.03^2.
//
// Two passes, each over 48 x 16 pixel tiles of one channel (up to 16 cameras
// per launch, one block per tile and channel), the window applied separably
// (a column pass in registers into LDS, then a row pass), all in FP64 (the
// local variances sxx - mx^2 cancel badly in FP32):
//   1. local moments mx, my, sxx, syy, sxy; the SSIM map S and its partial
//      derivatives dS/dmx, dS/dsxx, dS/dsxy (written per pixel, FP64), and
//      the block's sums of S, |x - y|, (x - y)^2 (one FP64 atomic each);
//   2. the window applied to the three derivative maps, giving
//      dSSIM/dx_p = w*dS/dmx + 2 x_p w*dS/dsxx + y_p w*dS/dsxy, and the
//      gradient of the weighted loss.
// A last kernel turns the sums into the per-camera loss.  The derivative maps
// (72 bytes per pixel) and the sums (24 bytes per camera) live in the
// caller's workspace.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <mutex>

#include "internal.h"

namespace lsplat {

namespace {

// Tiles of 48 x 16 outputs.  The column pass runs first, straight from
// global memory: each of 58 x 4 threads owns one column of the tile plus its
// 5-pixel halo and 4 consecutive output rows, sliding the 11-row window over
// 14 loaded rows in registers, and leaves its column sums in LDS.  The row
// pass then gives each thread 3 consecutive outputs of one row from 13 LDS
// values per sum.  Both passes together read about 220 LDS bytes per output.
constexpr int kLTX = 48, kLTY = 16, kHalo = 5, kWin = 11;
constexpr int kLX = kLTX + 2 * kHalo;            // 58 staged columns
constexpr int kSeg = 4;                           // output rows per column thread
constexpr int kColThreads = kLX * (kLTY / kSeg);  // 232
constexpr int kRowOut = 3;                        // outputs per row thread
constexpr int kLXP = kLX + 1;                     // padded LDS row
static_assert((kLTX / kRowOut) * kLTY == 256, "row pass covers the tile with 256 threads");
constexpr double kC1 = 0.0001, kC2 = 0.0009;
constexpr double kWL1 = 0.6, kWL2 = 0.2, kWSSIM = 0.2;

__device__ __forceinline__ double wave_sum_d(double v) {
  for (int d = 32; d > 0; d >>= 1) v += __shfl_xor(v, d, 64);
  return v;
}

// Cameras of one launch: each block finds its camera from the prefix of tile
// counts (at most kLossCams entries, uniform across the block).
constexpr int kLossCams = 16;
struct LossArgs {
  double g[kWin];                 // the normalised 1D window (host-computed)
  int32_t count;                  // cameras in this launch
  int32_t cam0;                   // global index of the first one
  int32_t W[kLossCams], H[kLossCams], GX[kLossCams];
  int32_t blk[kLossCams + 1];     // first tile block of each camera
  int64_t pix[kLossCams];         // first pixel of each camera
};

struct LossTile {
  int k, W, H, x0, y0;
  int64_t plane, base;            // channel plane, offset of the camera's image
};

__device__ __forceinline__ LossTile loss_tile(const LossArgs& a) {
  const int b = blockIdx.x;
  int k = 0;
  while (k + 1 < a.count && b >= a.blk[k + 1]) ++k;
  LossTile t;
  t.k = k;
  t.W = a.W[k];
  t.H = a.H[k];
  const int lb = b - a.blk[k];
  t.x0 = (lb % a.GX[k]) * kLTX;
  t.y0 = (lb / a.GX[k]) * kLTY;
  t.plane = (int64_t)t.W * t.H;
  t.base = 3 * a.pix[k] + blockIdx.y * t.plane;
  return t;
}

// pass 1: one (camera, 48 x 16 tile, channel) per block of 256 threads
__global__ __launch_bounds__(256) void ssim_moments_kernel(
    LossArgs a, const float* __restrict__ img, const float* __restrict__ tgt,
    double* __restrict__ coef, double* __restrict__ acc) {
  __shared__ double vm[5][kLTY][kLXP];
  __shared__ double red[3][4];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const LossTile t = loss_tile(a);
  const int W = t.W, H = t.H, x0 = t.x0, y0 = t.y0;
  const float* xi = img + t.base;
  const float* yi = tgt + t.base;
  // this thread's row-pass outputs; their own pixel values are fetched first
  // (clamped into the image) so that the load overlaps the column pass
  const int row = tid / (kLTX / kRowOut), c0 = (tid % (kLTX / kRowOut)) * kRowOut;
  const int py = y0 + row;
  float cx[kRowOut], cy[kRowOut];
#pragma unroll
  for (int q = 0; q < kRowOut; ++q) {
    const int64_t o = (int64_t)min(py, H - 1) * W + min(x0 + c0 + q, W - 1);
    cx[q] = xi[o];
    cy[q] = yi[o];
  }
  if (tid < kColThreads) {
    const int col = tid % kLX, seg = tid / kLX;
    const int gx = x0 - kHalo + col;
    const int r0 = seg * kSeg;                    // first output row (tile-relative)
    // every load is issued (clamped into the image) and its bits masked
    // afterwards, so the 28 loads go out back to back without a branch
    // between them
    const bool xin = gx >= 0 && gx < W;
    const int gxc = min(max(gx, 0), W - 1);
    double u[kSeg + kWin - 1], v[kSeg + kWin - 1];
#pragma unroll
    for (int j = 0; j < kSeg + kWin - 1; ++j) {
      const int gy = y0 - kHalo + r0 + j;
      const int64_t o = (int64_t)min(max(gy, 0), H - 1) * W + gxc;
      const int keep = (xin && gy >= 0 && gy < H) ? -1 : 0;
      u[j] = (double)__int_as_float(__float_as_int(xi[o]) & keep);
      v[j] = (double)__int_as_float(__float_as_int(yi[o]) & keep);
    }
#pragma unroll
    for (int j = 0; j < kSeg; ++j) {
      double mx = 0, my = 0, xx = 0, yy = 0, xy = 0;
#pragma unroll
      for (int k = 0; k < kWin; ++k) {
        const double w = a.g[k], p = u[j + k], q = v[j + k];
        mx = fma(w, p, mx);
        my = fma(w, q, my);
        xx = fma(w, p * p, xx);
        yy = fma(w, q * q, yy);
        xy = fma(w, p * q, xy);
      }
      vm[0][r0 + j][col] = mx; vm[1][r0 + j][col] = my; vm[2][r0 + j][col] = xx;
      vm[3][r0 + j][col] = yy; vm[4][r0 + j][col] = xy;
    }
  }
  __syncthreads();
  double ss = 0.0, s1 = 0.0, s2 = 0.0;
  {
    double m[5][kRowOut];
#pragma unroll
    for (int f = 0; f < 5; ++f) {
      double h[kRowOut + kWin - 1];
#pragma unroll
      for (int j = 0; j < kRowOut + kWin - 1; ++j) h[j] = vm[f][row][c0 + j];
#pragma unroll
      for (int q = 0; q < kRowOut; ++q) {
        double acc_f = 0.0;
#pragma unroll
        for (int k = 0; k < kWin; ++k) acc_f = fma(a.g[k], h[q + k], acc_f);
        m[f][q] = acc_f;
      }
    }
    double* cm = coef + 3 * t.base;   // the derivative maps follow the image layout, 3 per channel
#pragma unroll
    for (int q = 0; q < kRowOut; ++q) {
      const int px = x0 + c0 + q;
      if (px < W && py < H) {
        const double mx = m[0][q], my = m[1][q];
        const double a1 = 2.0 * mx * my + kC1;
        const double a2 = 2.0 * (m[4][q] - mx * my) + kC2;
        const double b1 = mx * mx + my * my + kC1;
        const double b2 = (m[2][q] - mx * mx) + (m[3][q] - my * my) + kC2;
        // one division: 1/d with d = b1 b2, and 1/b2 = b1/d
        const double inv_d = 1.0 / (b1 * b2);
        const double S = a1 * a2 * inv_d;
        const int64_t o = (int64_t)py * W + px;
        cm[o] = (2.0 * my * (a2 - a1) - 2.0 * mx * S * (b2 - b1)) * inv_d;
        cm[t.plane + o] = -S * (b1 * inv_d);
        cm[2 * t.plane + o] = 2.0 * a1 * inv_d;
        const double df = (double)cx[q] - (double)cy[q];
        ss += S;
        s1 += fabs(df);
        s2 += df * df;
      }
    }
  }
  ss = wave_sum_d(ss);
  s1 = wave_sum_d(s1);
  s2 = wave_sum_d(s2);
  if (lane == 0) {
    red[0][wave] = ss;
    red[1][wave] = s1;
    red[2][wave] = s2;
  }
  __syncthreads();
  if (tid < 3) {
    // sums enter already divided by the camera's 3 H W values
    const double inv_n = 1.0 / (3.0 * (double)t.plane);
    const double val = (red[tid][0] + red[tid][1]) + (red[tid][2] + red[tid][3]);
    atomicAdd(acc + 3 * (a.cam0 + t.k) + tid, val * inv_n);
  }
}

// pass 2: the window over the three derivative maps (same two-pass
// structure), then the gradient of the weighted loss
__global__ __launch_bounds__(256) void ssim_grad_kernel(
    LossArgs a, const float* __restrict__ img, const float* __restrict__ tgt,
    const double* __restrict__ coef, float* __restrict__ grad) {
  __shared__ double vb[3][kLTY][kLXP];
  const int tid = threadIdx.x;
  const LossTile t = loss_tile(a);
  const int W = t.W, H = t.H, x0 = t.x0, y0 = t.y0;
  const double* cm = coef + 3 * t.base;
  const int row = tid / (kLTX / kRowOut), c0 = (tid % (kLTX / kRowOut)) * kRowOut;
  const int py = y0 + row;
  float cx[kRowOut], cy[kRowOut];
#pragma unroll
  for (int q = 0; q < kRowOut; ++q) {
    const int64_t o = t.base + (int64_t)min(py, H - 1) * W + min(x0 + c0 + q, W - 1);
    cx[q] = img[o];
    cy[q] = tgt[o];
  }
  if (tid < kColThreads) {
    const int col = tid % kLX, seg = tid / kLX;
    const int gx = x0 - kHalo + col;
    const int r0 = seg * kSeg;
    const bool xin = gx >= 0 && gx < W;
    const int gxc = min(max(gx, 0), W - 1);
#pragma unroll
    for (int f = 0; f < 3; ++f) {
      double u[kSeg + kWin - 1];
#pragma unroll
      for (int j = 0; j < kSeg + kWin - 1; ++j) {
        const int gy = y0 - kHalo + r0 + j;
        const double val = cm[f * t.plane + (int64_t)min(max(gy, 0), H - 1) * W + gxc];
        // zero outside the image by masking the bits: the value is always
        // used, so the load cannot be moved into a branch of its own
        const long long keep = (xin && gy >= 0 && gy < H) ? -1ll : 0ll;
        u[j] = __longlong_as_double(__double_as_longlong(val) & keep);
      }
#pragma unroll
      for (int j = 0; j < kSeg; ++j) {
        double acc_f = 0.0;
#pragma unroll
        for (int k = 0; k < kWin; ++k) acc_f = fma(a.g[k], u[j + k], acc_f);
        vb[f][r0 + j][col] = acc_f;
      }
    }
  }
  __syncthreads();
  double bl[3][kRowOut];
#pragma unroll
  for (int f = 0; f < 3; ++f) {
    double h[kRowOut + kWin - 1];
#pragma unroll
    for (int j = 0; j < kRowOut + kWin - 1; ++j) h[j] = vb[f][row][c0 + j];
#pragma unroll
    for (int q = 0; q < kRowOut; ++q) {
      double acc_f = 0.0;
#pragma unroll
      for (int k = 0; k < kWin; ++k) acc_f = fma(a.g[k], h[q + k], acc_f);
      bl[f][q] = acc_f;
    }
  }
  const double inv_n = 1.0 / (3.0 * (double)t.plane);
#pragma unroll
  for (int q = 0; q < kRowOut; ++q) {
    const int px = x0 + c0 + q;
    if (px >= W || py >= H) continue;
    const int64_t o = t.base + (int64_t)py * W + px;
    const double x = (double)cx[q], y = (double)cy[q];
    const double df = x - y;
    const double sg = df > 0.0 ? 1.0 : (df < 0.0 ? -1.0 : 0.0);
    const double dssim = bl[0][q] + 2.0 * x * bl[1][q] + y * bl[2][q];
    grad[o] = (float)((kWL1 * sg + kWL2 * 2.0 * df - kWSSIM * dssim) * inv_n);
  }
}

__global__ void loss_zero_kernel(double* __restrict__ acc, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) acc[i] = 0.0;
}

__global__ void loss_finalize_kernel(const double* __restrict__ acc, int C,
                                     double* __restrict__ loss) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c < C) loss[c] = kWL1 * acc[3 * c + 1] + kWL2 * acc[3 * c + 2] + kWSSIM * (1.0 - acc[3 * c]);
}

size_t align256(size_t x) { return (x + 255) / 256 * 256; }

}  // namespace

// ---------------------------------------------------------------------------
// Static scratch of ls_loss_noalloc: the derivative maps and per-camera sums
// of one call, for callers that cannot allocate.  Every device the library
// runs on holds its own copy until the process ends.  In host code `scratch`
// names a host-side stand-in, never a device address: the address on each
// device comes from hipGetSymbolAddress, taken once per device with that
// device current, and only that address is handed to kernels.
// ---------------------------------------------------------------------------
static __device__ __align__(256) unsigned char scratch[LS_LOSS_NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int kMaxScratchDevices = 64;
std::mutex g_scratch_mu;
char* g_scratch_ptr[kMaxScratchDevices];   // per device ordinal, set on first use
}  // namespace

hipError_t loss_noalloc_scratch(hipStream_t s, char** out) {
  *out = nullptr;
  int cur = -1;
  hipError_t e = hipGetDevice(&cur);
  if (e != hipSuccess) return e;
  int dev = cur;
  if (s != nullptr && (e = hipStreamGetDevice(s, &dev)) != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxScratchDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    // the stream's device must be current while its copy's address is taken
    if (dev != cur && (e = hipSetDevice(dev)) != hipSuccess) return e;
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (dev != cur) {
      const hipError_t r = hipSetDevice(cur);
      if (e == hipSuccess) e = r;
    }
    if (e != hipSuccess) return e;
    g_scratch_ptr[dev] = (char*)p;
  }
  *out = g_scratch_ptr[dev];
  return hipSuccess;
}

size_t loss_workspace_bytes(int64_t P, int C) {
  // FP64 derivative maps (3 per channel and pixel), then the per-camera sums
  return align256((size_t)P * 72) + align256((size_t)C * 24);
}

hipError_t launch_loss(const int32_t* W, const int32_t* H, int C, const float* image,
                       const float* target, float* dL_dimage, double* loss, char* ws,
                       hipStream_t s, bool timed) {
  int64_t P = 0;
  for (int c = 0; c < C; ++c) P += (int64_t)W[c] * H[c];
  double* coef = (double*)ws;
  double* acc = (double*)(ws + align256((size_t)P * 72));
  hipError_t e;
  ProfScope ps(timed ? "loss" : nullptr, s);
  hipLaunchKernelGGL(loss_zero_kernel, dim3((3 * C + 255) / 256), dim3(256), 0, s, acc, 3 * C);
  if ((e = hipGetLastError())) return e;
  double win[kWin], wsum = 0.0;
  for (int k = 0; k < kWin; ++k) {
    win[k] = exp(-(double)((k - kHalo) * (k - kHalo)) / 4.5);   // sigma 1.5
    wsum += win[k];
  }
  int64_t pix = 0;
  for (int first = 0; first < C; first += kLossCams) {
    LossArgs a;
    memset(&a, 0, sizeof(a));
    for (int k = 0; k < kWin; ++k) a.g[k] = win[k] / wsum;
    a.cam0 = first;
    a.count = std::min(kLossCams, C - first);
    a.blk[0] = 0;
    for (int k = 0; k < a.count; ++k) {
      const int c = first + k;
      a.W[k] = W[c];
      a.H[k] = H[c];
      a.GX[k] = (W[c] + kLTX - 1) / kLTX;
      a.blk[k + 1] = a.blk[k] + a.GX[k] * ((H[c] + kLTY - 1) / kLTY);
      a.pix[k] = pix;
      pix += (int64_t)W[c] * H[c];
    }
    const dim3 grid((unsigned)a.blk[a.count], 3);
    hipLaunchKernelGGL(ssim_moments_kernel, grid, dim3(256), 0, s, a, image, target, coef, acc);
    hipLaunchKernelGGL(ssim_grad_kernel, grid, dim3(256), 0, s, a, image, target, coef, dL_dimage);
    if ((e = hipGetLastError())) return e;
  }
  hipLaunchKernelGGL(loss_finalize_kernel, dim3((C + 255) / 256), dim3(256), 0, s, acc, C, loss);
  return hipGetLastError();
}

}  // namespace lsplat
