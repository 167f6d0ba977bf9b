// Projection of splats into every camera of their scene (forward) and the
// chain rule back to splat parameters (backward).
//
// Sec. 3.1 of the paper: Sigma = R S S^T R^T (Eq. 2), Sigma' = J W Sigma W^T J^T
// (Eq. 3), Sigma_2D = top-left 2x2 block (Eq. 4); the linear kernel's support
// is the ellipse D' < lambda of Eq. 11-12.  The 2D covariance is dilated by
// eps2d and the Jacobian's tangent clamped (3DGS framework conventions).
//
// Layout: one thread per splat, looping over the cameras of its scene, so a
// splat's attributes (up to 236 bytes at SH degree 3) are read from HBM once
// for all cameras ("splat-major").  Attribute reads are structure-of-arrays
// and coalesced; per-pair outputs are written at pair index
// pair_off[c] + (splat - splat_lo[c]), coalesced within a camera.
#include <string.h>

#include <algorithm>

#include "internal.h"

namespace lsplat {

namespace {

constexpr int kCamsPerSetup = 32;
constexpr int kProjThreads = 256;

struct CamSetupArgs {
  int32_t first, count;
  int32_t W[kCamsPerSetup], H[kCamsPerSetup], GX[kCamsPerSetup], GY[kCamsPerSetup],
      scene[kCamsPerSetup];
  int64_t pair_off[kCamsPerSetup], tile_off[kCamsPerSetup], pix_off[kCamsPerSetup],
      lo[kCamsPerSetup], hi[kCamsPerSetup];
};

__global__ void cam_setup_kernel(CamSetupArgs a, const float* __restrict__ viewmat,
                                 const float* __restrict__ intrin, CamInfo* __restrict__ out) {
  int i = threadIdx.x;
  if (i >= a.count) return;
  int c = a.first + i;
  const float* v = viewmat + 12 * (int64_t)c;
  const float* in = intrin + 4 * (int64_t)c;
  CamInfo ci;
  for (int k = 0; k < 12; ++k) ci.vm32[k] = v[k];
  for (int k = 0; k < 4; ++k) ci.in32[k] = in[k];
  for (int r = 0; r < 3; ++r) {
    for (int k = 0; k < 3; ++k) ci.R[3 * r + k] = (double)v[4 * r + k];
    ci.t[r] = (double)v[4 * r + 3];
  }
  for (int k = 0; k < 3; ++k)
    ci.campos[k] = -(ci.R[k] * ci.t[0] + ci.R[3 + k] * ci.t[1] + ci.R[6 + k] * ci.t[2]);
  ci.fx = in[0]; ci.fy = in[1]; ci.cx = in[2]; ci.cy = in[3];
  ci.pair_off = a.pair_off[i]; ci.tile_off = a.tile_off[i]; ci.pix_off = a.pix_off[i];
  ci.splat_lo = a.lo[i]; ci.splat_hi = a.hi[i];
  ci.W = a.W[i]; ci.H = a.H[i]; ci.GX = a.GX[i]; ci.GY = a.GY[i]; ci.scene = a.scene[i];
  ci.pad[0] = ci.pad[1] = ci.pad[2] = 0;
  out[c] = ci;
}

// ---------------------------------------------------------------------------
// FP32 binning sequence.  Every operation rounds to FP32 in the written order:
// no contraction into fused multiply-add; division and square root are the
// correctly rounded ones (the library is built with
// -fhip-fp32-correctly-rounded-divide-sqrt and without fast-math).
// ---------------------------------------------------------------------------
struct BinOut {
  ushort4 rect;
  uint32_t ntiles;
  uint32_t dkey;
};

// The splat's 3D covariance in the FP32 sequence (it does not depend on the
// camera, so a splat computes it once for all its cameras).
struct CovF {
  float S[3][3];
};

__device__ __forceinline__ CovF bin_cov_fp32(float s0, float s1, float s2, float qw, float qx,
                                             float qy, float qz) {
#pragma clang fp contract(off)
  float n2 = ((qw * qw + qx * qx) + qy * qy) + qz * qz;
  float r = sqrtf(n2);
  float w = qw / r, x = qx / r, y = qy / r, z = qz / r;
  float R[3][3];
  R[0][0] = 1.0f - 2.0f * (y * y + z * z);
  R[0][1] = 2.0f * (x * y - w * z);
  R[0][2] = 2.0f * (x * z + w * y);
  R[1][0] = 2.0f * (x * y + w * z);
  R[1][1] = 1.0f - 2.0f * (x * x + z * z);
  R[1][2] = 2.0f * (y * z - w * x);
  R[2][0] = 2.0f * (x * z - w * y);
  R[2][1] = 2.0f * (y * z + w * x);
  R[2][2] = 1.0f - 2.0f * (x * x + y * y);
  float s[3] = {s0, s1, s2};
  float M[3][3];
  for (int rr = 0; rr < 3; ++rr)
    for (int cc = 0; cc < 3; ++cc) M[rr][cc] = R[rr][cc] * s[cc];
  CovF cv;
  for (int rr = 0; rr < 3; ++rr)
    for (int cc = 0; cc < 3; ++cc)
      cv.S[rr][cc] = (M[rr][0] * M[cc][0] + M[rr][1] * M[cc][1]) + M[rr][2] * M[cc][2];
  return cv;
}

__device__ __noinline__ BinOut bin_fp32(float mx_, float my_, float mz_, const CovF& cv,
                                         const float* V, const float* in4, float Wf, float Hf,
                                         float lam, float eps, float clip, float near_z,
                                         float far_z, int TW, int TH) {
#pragma clang fp contract(off)
  const float (*Sg)[3] = cv.S;
  float t0 = ((V[0] * mx_ + V[1] * my_) + V[2] * mz_) + V[3];
  float t1 = ((V[4] * mx_ + V[5] * my_) + V[6] * mz_) + V[7];
  float t2 = ((V[8] * mx_ + V[9] * my_) + V[10] * mz_) + V[11];
  float fx = in4[0], fy = in4[1], cx = in4[2], cy = in4[3];
  float u = t0 / t2;
  float v = t1 / t2;
  float mx = fx * u + cx;
  float my = fy * v + cy;
  float limx = (clip * (0.5f * Wf)) / fx;
  float limy = (clip * (0.5f * Hf)) / fy;
  float uc = fminf(limx, fmaxf(-limx, u));
  float vc = fminf(limy, fmaxf(-limy, v));
  float J00 = fx / t2;
  float J02 = -((fx * uc) / t2);
  float J11 = fy / t2;
  float J12 = -((fy * vc) / t2);
  float T0[3], T1[3];
  for (int cc = 0; cc < 3; ++cc) {
    T0[cc] = J00 * V[cc] + J02 * V[8 + cc];
    T1[cc] = J11 * V[4 + cc] + J12 * V[8 + cc];
  }
  float P0[3], P1[3];
  for (int cc = 0; cc < 3; ++cc) {
    P0[cc] = (T0[0] * Sg[0][cc] + T0[1] * Sg[1][cc]) + T0[2] * Sg[2][cc];
    P1[cc] = (T1[0] * Sg[0][cc] + T1[1] * Sg[1][cc]) + T1[2] * Sg[2][cc];
  }
  float a = ((P0[0] * T0[0] + P0[1] * T0[1]) + P0[2] * T0[2]) + eps;
  float c = ((P1[0] * T1[0] + P1[1] * T1[1]) + P1[2] * T1[2]) + eps;
  float rx = lam * sqrtf(a);
  float ry = lam * sqrtf(c);
  float xlo = ceilf((mx - rx) - 0.5f);
  float xhi = floorf((mx + rx) - 0.5f);
  float ylo = ceilf((my - ry) - 0.5f);
  float yhi = floorf((my + ry) - 0.5f);
  xlo = fmaxf(xlo, 0.0f);
  ylo = fmaxf(ylo, 0.0f);
  xhi = fminf(xhi, Wf - 1.0f);
  yhi = fminf(yhi, Hf - 1.0f);
  bool finite = isfinite(t0) && isfinite(t1) && isfinite(t2) && isfinite(mx) && isfinite(my) &&
                isfinite(rx) && isfinite(ry);
  bool keep = finite && (t2 > near_z) && (t2 < far_z) && (xlo <= xhi) && (ylo <= yhi);
  BinOut o;
  if (!keep) {
    o.rect = make_ushort4(1, 1, 0, 0);   // empty rectangle
    o.ntiles = 0;
    o.dkey = 0xFFFFFFFFu;
    return o;
  }
  int ix0 = (int)xlo / TW, iy0 = (int)ylo / TH, ix1 = (int)xhi / TW, iy1 = (int)yhi / TH;
  o.rect = make_ushort4((unsigned short)ix0, (unsigned short)iy0, (unsigned short)ix1,
                        (unsigned short)iy1);
  o.ntiles = (uint32_t)((ix1 - ix0 + 1) * (iy1 - iy0 + 1));
  o.dkey = __float_as_uint(t2);
  return o;
}

// ---------------------------------------------------------------------------
// Real SH basis (degree <= 3, 3DGS sign convention) in FP64, and the
// contraction of its gradient with per-band colour weights.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void sh_eval(int deg, double x, double y, double z, double* Y) {
  const double c0 = 0.28209479177387814;   // 1 / (2 sqrt(pi))
  const double c1 = 0.4886025119029199;    // sqrt(3 / (4 pi))
  const double c2a = 1.0925484305920792, c2b = 0.31539156525252005, c2c = 0.5462742152960396;
  const double c3a = 0.5900435899266435, c3b = 2.890611442640554, c3c = 0.4570457994644658,
               c3d = 0.3731763325901154, c3e = 1.445305721320277;
  Y[0] = c0;
  if (deg < 1) return;
  Y[1] = -c1 * y; Y[2] = c1 * z; Y[3] = -c1 * x;
  if (deg < 2) return;
  double xx = x * x, yy = y * y, zz = z * z;
  Y[4] = c2a * x * y; Y[5] = -c2a * y * z; Y[6] = c2b * (2.0 * zz - xx - yy);
  Y[7] = -c2a * x * z; Y[8] = c2c * (xx - yy);
  if (deg < 3) return;
  Y[9] = -c3a * y * (3.0 * xx - yy);
  Y[10] = c3b * x * y * z;
  Y[11] = -c3c * y * (4.0 * zz - xx - yy);
  Y[12] = c3d * z * (2.0 * zz - 3.0 * xx - 3.0 * yy);
  Y[13] = -c3c * x * (4.0 * zz - xx - yy);
  Y[14] = c3e * z * (xx - yy);
  Y[15] = -c3a * x * (xx - 3.0 * yy);
}

// g = sum_k w_k dY_k/d(x, y, z)
__device__ __forceinline__ void sh_grad_dot(int deg, double x, double y, double z, const double* w,
                                            double* g) {
  const double c1 = 0.4886025119029199;
  const double c2a = 1.0925484305920792, c2b = 0.31539156525252005, c2c = 0.5462742152960396;
  const double c3a = 0.5900435899266435, c3b = 2.890611442640554, c3c = 0.4570457994644658,
               c3d = 0.3731763325901154, c3e = 1.445305721320277;
  double gx = 0, gy = 0, gz = 0;
  if (deg >= 1) {
    gy += -c1 * w[1];
    gz += c1 * w[2];
    gx += -c1 * w[3];
  }
  if (deg >= 2) {
    gx += c2a * y * w[4]; gy += c2a * x * w[4];
    gy += -c2a * z * w[5]; gz += -c2a * y * w[5];
    gx += -2.0 * c2b * x * w[6]; gy += -2.0 * c2b * y * w[6]; gz += 4.0 * c2b * z * w[6];
    gx += -c2a * z * w[7]; gz += -c2a * x * w[7];
    gx += 2.0 * c2c * x * w[8]; gy += -2.0 * c2c * y * w[8];
  }
  if (deg >= 3) {
    double xx = x * x, yy = y * y, zz = z * z;
    gx += -c3a * 6.0 * x * y * w[9]; gy += -c3a * (3.0 * xx - 3.0 * yy) * w[9];
    gx += c3b * y * z * w[10]; gy += c3b * x * z * w[10]; gz += c3b * x * y * w[10];
    gx += c3c * 2.0 * x * y * w[11]; gy += -c3c * (4.0 * zz - xx - 3.0 * yy) * w[11];
    gz += -c3c * 8.0 * y * z * w[11];
    gx += -c3d * 6.0 * x * z * w[12]; gy += -c3d * 6.0 * y * z * w[12];
    gz += c3d * (6.0 * zz - 3.0 * xx - 3.0 * yy) * w[12];
    gx += -c3c * (4.0 * zz - 3.0 * xx - yy) * w[13]; gy += c3c * 2.0 * x * y * w[13];
    gz += -c3c * 8.0 * x * z * w[13];
    gx += c3e * 2.0 * x * z * w[14]; gy += -c3e * 2.0 * y * z * w[14]; gz += c3e * (xx - yy) * w[14];
    gx += -c3a * (3.0 * xx - 3.0 * yy) * w[15]; gy += c3a * 6.0 * x * y * w[15];
  }
  g[0] = gx; g[1] = gy; g[2] = gz;
}

// raw colour 0.5 + sum_k Y_k(d) sh_k (before the clamp); shc holds the
// splat's coefficients as [k][channel].
template <int DEG>
__device__ __forceinline__ void sh_raw(double x, double y, double z, const float* shc,
                                       double raw[3]) {
  constexpr int K = (DEG + 1) * (DEG + 1);
  double Y[16];
  sh_eval(DEG, x, y, z, Y);
  raw[0] = raw[1] = raw[2] = 0.5;
#pragma unroll
  for (int k = 0; k < K; ++k)
#pragma unroll
    for (int ch = 0; ch < 3; ++ch) raw[ch] += Y[k] * (double)shc[3 * k + ch];
}

// gd = sum_k (sum_c graw_c sh_kc) dY_k/dd
template <int DEG>
__device__ __forceinline__ void sh_dir_grad(double x, double y, double z, const float* shc,
                                            const double graw[3], double gd[3]) {
  constexpr int K = (DEG + 1) * (DEG + 1);
  double wk[16];
#pragma unroll
  for (int k = 0; k < K; ++k)
    wk[k] = graw[0] * (double)shc[3 * k] + graw[1] * (double)shc[3 * k + 1] +
            graw[2] * (double)shc[3 * k + 2];
  sh_grad_dot(DEG, x, y, z, wk, gd);
}

// FP64 geometry of one (camera, splat) pair, shared by forward and backward.
struct Geo {
  double q[4], qn;         // normalised quaternion and the input norm
  double R[9];             // rotation, row-major
  double M[9];             // R diag(s)
  double S[6];             // Sigma: xx, xy, xz, yy, yz, zz
  double t[3];             // camera-space centre
  double u, v, uc, vc;     // tangents, clipped tangents
  double T[6];             // J W (2x3, row-major)
  double a, b, c;          // dilated Sigma_2D
  double A, B, C;          // conic
  double mx, my;
};

// The camera-independent part: normalised quaternion, rotation, R diag(s)
// and the 3D covariance.
__device__ __forceinline__ void geo_splat(double s0, double s1, double s2, double qw, double qx,
                                          double qy, double qz, Geo& g) {
  double qn = sqrt(qw * qw + qx * qx + qy * qy + qz * qz);
  g.qn = qn;
  const double iqn = rcp_d(qn);
  double w = qw * iqn, x = qx * iqn, y = qy * iqn, z = qz * iqn;
  g.q[0] = w; g.q[1] = x; g.q[2] = y; g.q[3] = z;
  double* R = g.R;
  R[0] = 1.0 - 2.0 * (y * y + z * z); R[1] = 2.0 * (x * y - w * z); R[2] = 2.0 * (x * z + w * y);
  R[3] = 2.0 * (x * y + w * z); R[4] = 1.0 - 2.0 * (x * x + z * z); R[5] = 2.0 * (y * z - w * x);
  R[6] = 2.0 * (x * z - w * y); R[7] = 2.0 * (y * z + w * x); R[8] = 1.0 - 2.0 * (x * x + y * y);
  double s[3] = {s0, s1, s2};
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c) g.M[3 * r + c] = R[3 * r + c] * s[c];
  const double* M = g.M;
  auto dot3 = [&](int r, int c) {
    return M[3 * r] * M[3 * c] + M[3 * r + 1] * M[3 * c + 1] + M[3 * r + 2] * M[3 * c + 2];
  };
  g.S[0] = dot3(0, 0); g.S[1] = dot3(0, 1); g.S[2] = dot3(0, 2);
  g.S[3] = dot3(1, 1); g.S[4] = dot3(1, 2); g.S[5] = dot3(2, 2);
}

// The camera's part (needs g.S from geo_splat): camera-space centre,
// projection, clipped Jacobian, dilated 2D covariance and its conic.
__device__ __forceinline__ void geo_cam(const CamInfo& ci, double mux, double muy, double muz,
                                        double clip, double eps, Geo& g) {
  const double* Wr = ci.R;
  for (int r = 0; r < 3; ++r)
    g.t[r] = Wr[3 * r] * mux + Wr[3 * r + 1] * muy + Wr[3 * r + 2] * muz + ci.t[r];
  double tx = g.t[0], ty = g.t[1], tz = g.t[2];
  const double iz = rcp_d(tz);
  g.mx = ci.fx * tx * iz + ci.cx;
  g.my = ci.fy * ty * iz + ci.cy;
  double limx = clip * 0.5 * (double)ci.W * rcp_d(ci.fx);
  double limy = clip * 0.5 * (double)ci.H * rcp_d(ci.fy);
  g.u = tx * iz; g.v = ty * iz;
  g.uc = fmin(limx, fmax(-limx, g.u));
  g.vc = fmin(limy, fmax(-limy, g.v));
  double J00 = ci.fx * iz, J02 = -ci.fx * g.uc * iz, J11 = ci.fy * iz, J12 = -ci.fy * g.vc * iz;
  for (int c = 0; c < 3; ++c) {
    g.T[c] = J00 * Wr[c] + J02 * Wr[6 + c];
    g.T[3 + c] = J11 * Wr[3 + c] + J12 * Wr[6 + c];
  }
  const double* T = g.T;
  const double* S = g.S;
  // P = T Sigma (2x3)
  double P0[3] = {T[0] * S[0] + T[1] * S[1] + T[2] * S[2], T[0] * S[1] + T[1] * S[3] + T[2] * S[4],
                  T[0] * S[2] + T[1] * S[4] + T[2] * S[5]};
  double P1[3] = {T[3] * S[0] + T[4] * S[1] + T[5] * S[2], T[3] * S[1] + T[4] * S[3] + T[5] * S[4],
                  T[3] * S[2] + T[4] * S[4] + T[5] * S[5]};
  g.a = P0[0] * T[0] + P0[1] * T[1] + P0[2] * T[2] + eps;
  g.b = P0[0] * T[3] + P0[1] * T[4] + P0[2] * T[5];
  g.c = P1[0] * T[3] + P1[1] * T[4] + P1[2] * T[5] + eps;
  double det = g.a * g.c - g.b * g.b;
  const double idet = rcp_d(det);
  g.A = g.c * idet; g.B = -g.b * idet; g.C = g.a * idet;
}

__device__ __forceinline__ void geo_compute(const CamInfo& ci, double mux, double muy, double muz,
                                            double s0, double s1, double s2, double qw, double qx,
                                            double qy, double qz, double clip, double eps, Geo& g) {
  geo_splat(s0, s1, s2, qw, qx, qy, qz, g);
  geo_cam(ci, mux, muy, muz, clip, eps, g);
}

template <int DEG>
__global__ __launch_bounds__(kProjThreads) void project_kernel(
    const CamInfo* __restrict__ cams, int C, int64_t N, const float* __restrict__ means,
    const float* __restrict__ scales, const float* __restrict__ quats,
    const float* __restrict__ opac, const float* __restrict__ sh, float lam, float eps,
    float clip, float near_z, float far_z, int TW, int TH, ProjRec* __restrict__ proj,
    ushort4* __restrict__ rect, uint32_t* __restrict__ ntiles, uint32_t* __restrict__ dkey) {
  constexpr int K = (DEG + 1) * (DEG + 1);
  int64_t i = (int64_t)blockIdx.x * kProjThreads + threadIdx.x;
  if (i >= N) return;
  float mu[3], s[3], q[4];
  for (int k = 0; k < 3; ++k) {
    mu[k] = means[k * N + i];
    s[k] = scales[k * N + i];
  }
  for (int k = 0; k < 4; ++k) q[k] = quats[k * N + i];
  float o = opac[i];
  float shc[K * 3];
#pragma unroll
  for (int k = 0; k < K * 3; ++k) shc[k] = sh[(int64_t)k * N + i];
  // the 3D covariance, FP32 (binning) and FP64 (geometry), once per splat
  const CovF cv = bin_cov_fp32(s[0], s[1], s[2], q[0], q[1], q[2], q[3]);
  Geo g;
  geo_splat(s[0], s[1], s[2], q[0], q[1], q[2], q[3], g);

  for (int c = 0; c < C; ++c) {
    const CamInfo& ci = cams[c];
    if (i < ci.splat_lo || i >= ci.splat_hi) continue;
    int64_t m = ci.pair_off + (i - ci.splat_lo);
    BinOut bo = bin_fp32(mu[0], mu[1], mu[2], cv, ci.vm32, ci.in32, (float)ci.W, (float)ci.H, lam,
                         eps, clip, near_z, far_z, TW, TH);
    rect[m] = bo.rect;
    ntiles[m] = bo.ntiles;
    dkey[m] = bo.dkey;
    if (bo.ntiles == 0) continue;
    geo_cam(ci, mu[0], mu[1], mu[2], clip, eps, g);
    // colour: SH at the unit direction from the camera centre to the splat
    double vx = mu[0] - ci.campos[0], vy = mu[1] - ci.campos[1], vz = mu[2] - ci.campos[2];
    double inv = rsqrt_d(vx * vx + vy * vy + vz * vz);
    double Y[16];
    sh_eval(DEG, vx * inv, vy * inv, vz * inv, Y);
    double col[3] = {0.5, 0.5, 0.5};
#pragma unroll
    for (int k = 0; k < K; ++k)
#pragma unroll
      for (int ch = 0; ch < 3; ++ch) col[ch] += Y[k] * (double)shc[3 * k + ch];
    ProjRec rec;
    rec.mx = g.mx; rec.my = g.my;
    rec.A = g.A; rec.B = g.B; rec.C = g.C;
    rec.r = (float)fmax(col[0], 0.0);
    rec.g = (float)fmax(col[1], 0.0);
    rec.b = (float)fmax(col[2], 0.0);
    rec.o = o;
    rec.pad0 = 0.f; rec.pad1 = 0.f;
    proj[m] = rec;
  }
}

// ---------------------------------------------------------------------------
// Backward.  grad2d[f][m] holds, per pair, the sums over its pixels of
//   dL/dmean2d (x, y), dL/da, dL/db, dL/dc for the 2D covariance
//   [[a, b], [b, c]] (b one parameter in both off-diagonal slots), dL/do,
//   dL/drgb (3).
// ---------------------------------------------------------------------------
template <int DEG>
__global__ __launch_bounds__(kProjThreads) void project_bwd_kernel(
    const CamInfo* __restrict__ cams, int C, int64_t N, const float* __restrict__ means,
    const float* __restrict__ scales, const float* __restrict__ quats,
    const float* __restrict__ sh, float eps, float clip, const double* __restrict__ grad2d,
    int64_t M, float* __restrict__ g_means, float* __restrict__ g_scales,
    float* __restrict__ g_quats, float* __restrict__ g_opac, float* __restrict__ g_m2norm) {
  int64_t i = (int64_t)blockIdx.x * kProjThreads + threadIdx.x;
  if (i >= N) return;
  double mu[3], s[3], q[4];
  for (int k = 0; k < 3; ++k) {
    mu[k] = means[k * N + i];
    s[k] = scales[k * N + i];
  }
  for (int k = 0; k < 4; ++k) q[k] = quats[k * N + i];
  double gmu[3] = {0, 0, 0}, gs[3] = {0, 0, 0}, gq[4] = {0, 0, 0, 0}, go = 0;

  for (int c = 0; c < C; ++c) {
    const CamInfo& ci = cams[c];
    if (i < ci.splat_lo || i >= ci.splat_hi) continue;
    int64_t m = ci.pair_off + (i - ci.splat_lo);
    double g2[kGrad2d];
    bool any = false;
#pragma unroll
    for (int f = 0; f < kGrad2d; ++f) {
      g2[f] = grad2d[(int64_t)f * M + m];
      any |= (g2[f] != 0.0);
    }
    if (g_m2norm) g_m2norm[m] = (float)sqrt(g2[0] * g2[0] + g2[1] * g2[1]);
    if (!any) continue;
    Geo g;
    geo_compute(ci, mu[0], mu[1], mu[2], s[0], s[1], s[2], q[0], q[1], q[2], q[3], clip, eps, g);
    go += g2[5];
    // the raster pass accumulates dL/dcov2d directly (entries a, b, c of
    // [[a, b], [b, c]], b one parameter in both off-diagonal slots)
    const double G00 = g2[2], G01 = 0.5 * (double)g2[3], G11 = g2[4];
    const double* T = g.T;
    const double* S = g.S;
    double TS0[3] = {T[0] * S[0] + T[1] * S[1] + T[2] * S[2], T[0] * S[1] + T[1] * S[3] + T[2] * S[4],
                     T[0] * S[2] + T[1] * S[4] + T[2] * S[5]};
    double TS1[3] = {T[3] * S[0] + T[4] * S[1] + T[5] * S[2], T[3] * S[1] + T[4] * S[3] + T[5] * S[4],
                     T[3] * S[2] + T[4] * S[4] + T[5] * S[5]};
    // dL/dT = 2 G T Sigma
    double gT[6];
    for (int k = 0; k < 3; ++k) {
      gT[k] = 2.0 * (G00 * TS0[k] + G01 * TS1[k]);
      gT[3 + k] = 2.0 * (G01 * TS0[k] + G11 * TS1[k]);
    }
    // dL/dSigma = T^T G T (symmetric 3x3)
    double GT0[3], GT1[3];   // rows of G T
    for (int k = 0; k < 3; ++k) {
      GT0[k] = G00 * T[k] + G01 * T[3 + k];
      GT1[k] = G01 * T[k] + G11 * T[3 + k];
    }
    double gS[9];
    for (int r = 0; r < 3; ++r)
      for (int k = 0; k < 3; ++k) gS[3 * r + k] = T[r] * GT0[k] + T[3 + r] * GT1[k];
    // T = J W  =>  dL/dJ = dL/dT W^T ; only J00, J02, J11, J12 vary
    const double* Wr = ci.R;
    double gJ00 = gT[0] * Wr[0] + gT[1] * Wr[1] + gT[2] * Wr[2];
    double gJ02 = gT[0] * Wr[6] + gT[1] * Wr[7] + gT[2] * Wr[8];
    double gJ11 = gT[3] * Wr[3] + gT[4] * Wr[4] + gT[5] * Wr[5];
    double gJ12 = gT[3] * Wr[6] + gT[4] * Wr[7] + gT[5] * Wr[8];
    double tx = g.t[0], ty = g.t[1], tz = g.t[2];
    double fx = ci.fx, fy = ci.fy;
    double iz = rcp_d(tz), iz2 = iz * iz, iz3 = iz2 * iz;
    double gt[3] = {0, 0, 0};
    gt[2] += gJ00 * (-fx * iz2) + gJ11 * (-fy * iz2);
    double limx = clip * 0.5 * (double)ci.W / fx;
    double limy = clip * 0.5 * (double)ci.H / fy;
    if (fabs(g.u) < limx) {
      gt[0] += gJ02 * (-fx * iz2);
      gt[2] += gJ02 * (2.0 * fx * tx * iz3);
    } else {
      gt[2] += gJ02 * (fx * g.uc * iz2);
    }
    if (fabs(g.v) < limy) {
      gt[1] += gJ12 * (-fy * iz2);
      gt[2] += gJ12 * (2.0 * fy * ty * iz3);
    } else {
      gt[2] += gJ12 * (fy * g.vc * iz2);
    }
    double gmx = g2[0], gmy = g2[1];
    gt[0] += gmx * fx * iz;
    gt[1] += gmy * fy * iz;
    gt[2] += -(gmx * fx * tx + gmy * fy * ty) * iz2;
    for (int k = 0; k < 3; ++k) gmu[k] += Wr[k] * gt[0] + Wr[3 + k] * gt[1] + Wr[6 + k] * gt[2];
    // Sigma = M M^T, M = R diag(s)
    const double* Mm = g.M;
    double gM[9];
    for (int r = 0; r < 3; ++r)
      for (int k = 0; k < 3; ++k)
        gM[3 * r + k] = 2.0 * (gS[3 * r] * Mm[k] + gS[3 * r + 1] * Mm[3 + k] + gS[3 * r + 2] * Mm[6 + k]);
    const double* R = g.R;
    double gR[9];
    for (int r = 0; r < 3; ++r)
      for (int k = 0; k < 3; ++k) {
        gs[k] += gM[3 * r + k] * R[3 * r + k];
        gR[3 * r + k] = gM[3 * r + k] * s[k];
      }
    double w = g.q[0], x = g.q[1], y = g.q[2], z = g.q[3];
    double gqh[4];
    gqh[0] = 2.0 * (-z * gR[1] + y * gR[2] + z * gR[3] - x * gR[5] - y * gR[6] + x * gR[7]);
    gqh[1] = 2.0 * (y * gR[1] + z * gR[2] + y * gR[3] - 2.0 * x * gR[4] - w * gR[5] + z * gR[6] +
                    w * gR[7] - 2.0 * x * gR[8]);
    gqh[2] = 2.0 * (-2.0 * y * gR[0] + x * gR[1] + w * gR[2] + x * gR[3] + z * gR[5] - w * gR[6] +
                    z * gR[7] - 2.0 * y * gR[8]);
    gqh[3] = 2.0 * (-2.0 * z * gR[0] - w * gR[1] + x * gR[2] + w * gR[3] - 2.0 * z * gR[4] +
                    y * gR[5] + x * gR[6] + y * gR[7]);
    double dq = w * gqh[0] + x * gqh[1] + y * gqh[2] + z * gqh[3];
    for (int k = 0; k < 4; ++k) gq[k] += (gqh[k] - g.q[k] * dq) / g.qn;
  }
  for (int k = 0; k < 3; ++k) {
    g_means[k * N + i] = (float)gmu[k];
    g_scales[k * N + i] = (float)gs[k];
  }
  for (int k = 0; k < 4; ++k) g_quats[k * N + i] = (float)gq[k];
  g_opac[i] = (float)go;
}

// SH coefficient gradients: dL/dsh_kc = sum over cameras of Y_k(d) dL/drgb_c
// where the colour clamp is inactive.  Kept apart from the geometry chain so
// that neither kernel holds both working sets in registers.
template <int DEG>
__global__ __launch_bounds__(kProjThreads) void project_bwd_sh_kernel(
    const CamInfo* __restrict__ cams, int C, int64_t N, const float* __restrict__ means,
    const float* __restrict__ sh, const double* __restrict__ grad2d, int64_t M,
    float* __restrict__ g_sh, float* __restrict__ g_means) {
  constexpr int K = (DEG + 1) * (DEG + 1);
  int64_t i = (int64_t)blockIdx.x * kProjThreads + threadIdx.x;
  if (i >= N) return;
  const double mu0 = means[i], mu1 = means[N + i], mu2 = means[2 * N + i];
  float gsh[K * 3], shc[K * 3];
  double gmv[3] = {0.0, 0.0, 0.0};
#pragma unroll
  for (int k = 0; k < K * 3; ++k) {
    gsh[k] = 0.f;
    shc[k] = sh[(int64_t)k * N + i];
  }
  for (int c = 0; c < C; ++c) {
    const CamInfo& ci = cams[c];
    if (i < ci.splat_lo || i >= ci.splat_hi) continue;
    const int64_t m = ci.pair_off + (i - ci.splat_lo);
    const double gr = grad2d[6 * M + m], gg = grad2d[7 * M + m], gb = grad2d[8 * M + m];
    if (gr == 0.0 && gg == 0.0 && gb == 0.0) continue;
    double vx = mu0 - ci.campos[0], vy = mu1 - ci.campos[1], vz = mu2 - ci.campos[2];
    double inv = rsqrt_d(vx * vx + vy * vy + vz * vz);
    double dx = vx * inv, dy = vy * inv, dz = vz * inv;
    double raw[3];
    sh_raw<DEG>(dx, dy, dz, shc, raw);
    const double graw[3] = {raw[0] > 0.0 ? (double)gr : 0.0, raw[1] > 0.0 ? (double)gg : 0.0,
                            raw[2] > 0.0 ? (double)gb : 0.0};
    double Y[16];
    sh_eval(DEG, dx, dy, dz, Y);
#pragma unroll
    for (int k = 0; k < K; ++k)
#pragma unroll
      for (int ch = 0; ch < 3; ++ch) gsh[3 * k + ch] += (float)(Y[k] * graw[ch]);
    if (DEG > 0) {
      // the view direction moves with the centre: d = v/|v|, v = mu - campos
      double gd[3];
      sh_dir_grad<DEG>(dx, dy, dz, shc, graw, gd);
      const double dd = dx * gd[0] + dy * gd[1] + dz * gd[2];
      gmv[0] += (gd[0] - dx * dd) * inv;
      gmv[1] += (gd[1] - dy * dd) * inv;
      gmv[2] += (gd[2] - dz * dd) * inv;
    }
  }
#pragma unroll
  for (int k = 0; k < K * 3; ++k) g_sh[(int64_t)k * N + i] = gsh[k];
  if (DEG > 0) {
    for (int k = 0; k < 3; ++k) g_means[k * N + i] = (float)((double)g_means[k * N + i] + gmv[k]);
  }
}

}  // namespace

hipError_t launch_cam_setup(const Plan& p, const ls_cameras* cams, char* ws, hipStream_t s) {
  CamInfo* out = (CamInfo*)(ws + p.lay.cams);
  for (int first = 0; first < p.C; first += kCamsPerSetup) {
    CamSetupArgs a;
    memset(&a, 0, sizeof(a));
    a.first = first;
    a.count = std::min(kCamsPerSetup, p.C - first);
    for (int i = 0; i < a.count; ++i) {
      int c = first + i;
      a.W[i] = p.W[c]; a.H[i] = p.H[c]; a.GX[i] = p.GX[c]; a.GY[i] = p.GY[c]; a.scene[i] = p.scene[c];
      a.pair_off[i] = p.pair_off[c]; a.tile_off[i] = p.tile_off[c]; a.pix_off[i] = p.pix_off[c];
      a.lo[i] = p.splat_lo[c]; a.hi[i] = p.splat_hi[c];
    }
    {
      ProfScope ps("cam_setup", s);
      hipLaunchKernelGGL(cam_setup_kernel, dim3(1), dim3(kCamsPerSetup), 0, s, a, cams->viewmat,
                         cams->intrin, out);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_project(const Plan& p, const ls_config* cfg, const ls_splats* sp, char* ws,
                          hipStream_t s) {
  if (p.N == 0) return hipSuccess;
  const CamInfo* cams = (const CamInfo*)(ws + p.lay.cams);
  dim3 grid((unsigned)((p.N + kProjThreads - 1) / kProjThreads));
#define LS_PROJ(D)                                                                               \
  hipLaunchKernelGGL(project_kernel<D>, grid, dim3(kProjThreads), 0, s, cams, p.C, p.N, sp->means, \
                     sp->scales, sp->quats, sp->opacity, sp->sh, kernel_extent(cfg), cfg->eps2d,         \
                     cfg->clip, cfg->near_z, cfg->far_z, cfg->tile_w, cfg->tile_h,              \
                     (ProjRec*)(ws + p.lay.proj), (ushort4*)(ws + p.lay.rect),                  \
                     (uint32_t*)(ws + p.lay.ntiles), (uint32_t*)(ws + p.lay.depth_key))
  ProfScope ps("project", s);
  switch (cfg->sh_degree) {
    case 0: LS_PROJ(0); break;
    case 1: LS_PROJ(1); break;
    case 2: LS_PROJ(2); break;
    default: LS_PROJ(3); break;
  }
#undef LS_PROJ
  return hipGetLastError();
}

hipError_t launch_project_bwd(const Plan& p, const ls_config* cfg, const ls_splats* sp, char* ws,
                              const ls_grads* gr, hipStream_t s) {
  if (p.N == 0) return hipSuccess;
  const CamInfo* cams = (const CamInfo*)(ws + p.lay.cams);
  dim3 grid((unsigned)((p.N + kProjThreads - 1) / kProjThreads));
#define LS_PBWD(D)                                                                                 \
  do {                                                                                             \
    {                                                                                              \
      ProfScope ps("project_bwd", s);                                                              \
      hipLaunchKernelGGL(project_bwd_kernel<D>, grid, dim3(kProjThreads), 0, s, cams, p.C, p.N,   \
                         sp->means, sp->scales, sp->quats, sp->sh, cfg->eps2d, cfg->clip,         \
                         (const double*)(ws + p.lay.grad2d), p.M, gr->means, gr->scales,          \
                         gr->quats, gr->opacity, gr->mean2d_norm);                                \
    }                                                                                              \
    {                                                                                              \
      ProfScope ps("project_bwd_sh", s);                                                           \
      hipLaunchKernelGGL(project_bwd_sh_kernel<D>, grid, dim3(kProjThreads), 0, s, cams, p.C, p.N, \
                         sp->means, sp->sh, (const double*)(ws + p.lay.grad2d), p.M, gr->sh,      \
                         gr->means);                                                              \
    }                                                                                              \
  } while (0)
  switch (cfg->sh_degree) {
    case 0: LS_PBWD(0); break;
    case 1: LS_PBWD(1); break;
    case 2: LS_PBWD(2); break;
    default: LS_PBWD(3); break;
  }
#undef LS_PBWD
  return hipGetLastError();
}

}  // namespace lsplat
