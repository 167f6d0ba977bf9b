// Internal declarations shared by the HIP translation units of liblsplat.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/lsplat.h"

namespace lsplat {

// ---------------------------------------------------------------------------
// Device-side camera record, written into the workspace by the projection
// call.  Double copies of the matrices feed the FP64 geometry, float copies
// feed the FP32 binning sequence.
// ---------------------------------------------------------------------------
struct alignas(16) CamInfo {
  double R[9];          // world->camera rotation, row-major
  double t[3];          // translation
  double campos[3];     // camera centre in world space, -R^T t
  double fx, fy, cx, cy;
  float vm32[12];       // FP32 viewmat as given
  float in32[4];        // FP32 (fx, fy, cx, cy) as given
  int64_t pair_off;     // first pair index of this camera
  int64_t tile_off;     // first global tile id
  int64_t pix_off;      // first pixel index
  int64_t splat_lo;     // first splat of the camera's scene
  int64_t splat_hi;     // one past the last
  int32_t W, H, GX, GY;
  int32_t scene;
  int32_t pad[3];
};

// 64-byte projected record (gathered per tile by the raster kernels).
struct alignas(16) ProjRec {
  double mx, my;        // projected centre (FP64)
  double A, B, C;       // conic: D'^2 = A dx^2 + 2 B dx dy + C dy^2
  float r, g, b;        // colour
  float o;              // opacity
  float pad0, pad1;
};
static_assert(sizeof(ProjRec) == 64, "ProjRec must be 64 bytes");

constexpr int kGrad2d = 9;   // per-pair 2D gradient sums, see raster.hip

// Launch plan derived on the host from the settings and the cameras.
struct Plan {
  int32_t C = 0, S = 0;
  int64_t N = 0;          // splats
  int64_t M = 0;          // (camera, splat) pairs
  int64_t T = 0;          // tiles
  int64_t P = 0;          // pixels
  int64_t cap = 0;        // intersection capacity
  int32_t tile_bits = 0;  // bits of the largest global tile id
  int32_t max_scene = 0;  // largest scene size (splats)
  std::vector<int32_t> W, H, GX, GY, scene;
  std::vector<int64_t> pair_off, tile_off, pix_off, splat_lo, splat_hi;
  ls_layout lay{};
  // scratch sub-allocations (byte offsets from the workspace base)
  size_t sort_keys_b = 0, sort_vals_b = 0, pre_keys_a = 0, pre_keys_b = 0, pre_vals_a = 0, pre_vals_b = 0,
         hist = 0, digit_tot = 0, scan_part = 0, span_owner = 0, span_cnt = 0, span_off = 0,
         alive = 0, state = 0, done = 0, sat = 0, drect = 0, pmask = 0,
         abits = 0;
  // deterministic backward: per-entry sums [9][cap] and the pair-order sort
  size_t det_partial = 0, det_k0 = 0, det_v0 = 0, det_k1 = 0, det_v1 = 0, det_cnt = 0;
  size_t t64 = 0;             // FP64 final transmittance [P], forward -> backward
  int64_t n_spans = 0;        // entries of span_owner: ceil(cap / kKeygenSpan) + 1
  int32_t K = 1;              // depth chunks
  std::vector<int64_t> chunk_pos;   // [K + 1] pair positions in depth order
  int32_t sort_blocks = 0;    // radix sort grid for the intersection sort
  int32_t pre_blocks = 0;     // radix sort grid for the depth presort
  int32_t scan_blocks = 0;
};

// Radix sort geometry: 256 threads, 8 keys per thread per tile; at most 1024
// blocks (four per compute unit, all resident at once).
constexpr int kSortThreads = 256;
constexpr int kSortItems = 8;
constexpr int kSortTile = kSortThreads * kSortItems;
constexpr int kMaxSortBlocks = 1024;
constexpr int kScanThreads = 256;
constexpr int kKeygenSpan = 2048;   // output entries per key-generation block iteration
constexpr int kChunkSpan = 1024;    // output entries per chunk-write block iteration
constexpr int kMaxDepthChunks = 12;

// Support radius of the kernel in aligned distance D'/lambda, and the FP32
// extent lambda * s_f that bounds the binning ellipse and the composite.
__host__ __device__ inline float kernel_support(int kernel) {
  switch (kernel) {
    case LS_KERNEL_GAUSSIAN: return 3.0f;
    case LS_KERNEL_LAPLACIAN: return 5.541263545158426f;   // ln 255
    default: return 1.0f;
  }
}
inline float kernel_extent(const ls_config* cfg) { return cfg->lambda * kernel_support(cfg->kernel); }
constexpr int kMaxScanBlocks = 1024;

// ---------------------------------------------------------------------------
// wave64 sum with DPP (gfx9 row rotations, then row broadcasts).  Every lane
// passes its value; the full sum is returned in all lanes of row 3 (lanes
// 48..63); read it with __builtin_amdgcn_readlane(x, 63).
// ---------------------------------------------------------------------------
template <int CTRL, int ROWMASK = 0xF>
__device__ __forceinline__ float dpp_move(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, ROWMASK, 0xF, false));
}

// Sums of 8 values over the wave at once.  Each step halves the lanes a value
// spans while pairing values up, so that eight wave-wide sums cost 18
// instructions rather than 48:
//   1. v_permlane32_swap pairs (v0,v1) ... (v6,v7): after the add, lanes 0..31
//      hold partial sums of the first value of the pair, lanes 32..63 of the
//      second;
//   2. v_permlane16_swap pairs the four results: each 16-lane row then holds
//      one value (rows: v0 v2 v1 v3 and v4 v6 v5 v7);
//   3. a row rotation by 8 and a select pack the two registers into one, each
//      8-lane group holding one value;
//   4. a half-row mirror and two quad permutations finish each group's sum in
//      its first lane.
// Result: lane 8g (g = 0..7) holds the sum of v[wave_sum8_field(g)]; other
// lanes hold partial sums.  All lanes must be active.
__host__ __device__ __forceinline__ int wave_sum8_field(int g) {   // 3-bit reversal
  return ((g & 1) << 2) | (g & 2) | ((g >> 2) & 1);
}

__device__ __forceinline__ float swap32_add(float a, float b) {
  const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(a), __float_as_uint(b), false, false);
  return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}

__device__ __forceinline__ float swap16_add(float a, float b) {
  const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(a), __float_as_uint(b), false, false);
  return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}

__device__ __forceinline__ float wave_sum8(const float* v, int lane) {
  const float a = swap32_add(v[0], v[1]), b = swap32_add(v[2], v[3]);
  const float c = swap32_add(v[4], v[5]), d = swap32_add(v[6], v[7]);
  float x = swap16_add(a, b), y = swap16_add(c, d);
  x += dpp_move<0x128>(x);        // row_ror:8
  y += dpp_move<0x128>(y);
  float z = (lane & 8) ? y : x;
  z += dpp_move<0x141>(z);        // row_half_mirror
  z += dpp_move<0x4E>(z);         // quad_perm [2,3,0,1]
  z += dpp_move<0xB1>(z);         // quad_perm [1,0,3,2]
  return z;
}

// FP64 versions: the same lane movements applied to both 32-bit halves.
// (A full row mask writes every lane, so no old value is needed; with a
// partial mask the lanes outside it receive 0.)
template <int CTRL, int ROWMASK = 0xF>
__device__ __forceinline__ double dpp_move_d(double v) {
  const long long b = __double_as_longlong(v);
  int lo, hi;
  if constexpr (ROWMASK == 0xF) {
    lo = __builtin_amdgcn_mov_dpp((int)(b & 0xFFFFFFFFll), CTRL, ROWMASK, 0xF, false);
    hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), CTRL, ROWMASK, 0xF, false);
  } else {
    lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xFFFFFFFFll), CTRL, ROWMASK, 0xF, false);
    hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, ROWMASK, 0xF, false);
  }
  return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

__device__ __forceinline__ double swap32_add_d(double a, double b) {
  const long long x = __double_as_longlong(a), y = __double_as_longlong(b);
  const auto lo = __builtin_amdgcn_permlane32_swap((unsigned)x, (unsigned)y, false, false);
  const auto hi = __builtin_amdgcn_permlane32_swap((unsigned)(x >> 32), (unsigned)(y >> 32), false,
                                                   false);
  const double a2 = __longlong_as_double(((long long)hi[0] << 32) | (long long)lo[0]);
  const double b2 = __longlong_as_double(((long long)hi[1] << 32) | (long long)lo[1]);
  return a2 + b2;
}

__device__ __forceinline__ double swap16_add_d(double a, double b) {
  const long long x = __double_as_longlong(a), y = __double_as_longlong(b);
  const auto lo = __builtin_amdgcn_permlane16_swap((unsigned)x, (unsigned)y, false, false);
  const auto hi = __builtin_amdgcn_permlane16_swap((unsigned)(x >> 32), (unsigned)(y >> 32), false,
                                                   false);
  const double a2 = __longlong_as_double(((long long)hi[0] << 32) | (long long)lo[0]);
  const double b2 = __longlong_as_double(((long long)hi[1] << 32) | (long long)lo[1]);
  return a2 + b2;
}

// 1/x in FP64 from the hardware estimate and two Newton steps (for normal,
// nonzero x the result is within an ulp or two of the rounded quotient).
__device__ __forceinline__ double rcp_d(double x) {
  double r = __builtin_amdgcn_rcp(x);
  double e = fma(-x, r, 1.0);
  r = fma(r, e, r);
  e = fma(-x, r, 1.0);
  return fma(r, e, r);
}

// 1/sqrt(x) in FP64 for normal x > 0: the hardware estimate and two Newton
// steps for the reciprocal square root.
__device__ __forceinline__ double rsqrt_d(double x) {
  double y = __builtin_amdgcn_rsq(x);
  y = y * fma(-0.5 * x, y * y, 1.5);
  return y * fma(-0.5 * x, y * y, 1.5);
}

// wave_sum8 in FP64: lane 8g receives the sum of v[wave_sum8_field(g)].
__device__ __forceinline__ double wave_sum8_d(const double* v, int lane) {
  const double a = swap32_add_d(v[0], v[1]), b = swap32_add_d(v[2], v[3]);
  const double c = swap32_add_d(v[4], v[5]), d = swap32_add_d(v[6], v[7]);
  double x = swap16_add_d(a, b), y = swap16_add_d(c, d);
  x += dpp_move_d<0x128>(x);        // row_ror:8
  y += dpp_move_d<0x128>(y);
  double z = (lane & 8) ? y : x;
  z += dpp_move_d<0x141>(z);        // row_half_mirror
  z += dpp_move_d<0x4E>(z);         // quad_perm [2,3,0,1]
  z += dpp_move_d<0xB1>(z);         // quad_perm [1,0,3,2]
  return z;
}

// Sum over the wave in every lane (all lanes active): half-wave and
// half-row exchanges, then within each 16-lane row a rotation by 8, a
// half-row mirror and two quad permutations.
__device__ __forceinline__ double wave_sum_all_d(double x) {
  x = swap32_add_d(x, x);
  x = swap16_add_d(x, x);
  x += dpp_move_d<0x128>(x);        // row_ror:8
  x += dpp_move_d<0x141>(x);        // row_half_mirror
  x += dpp_move_d<0x4E>(x);         // quad_perm [2,3,0,1]
  x += dpp_move_d<0xB1>(x);         // quad_perm [1,0,3,2]
  return x;
}

__device__ __forceinline__ double wave_sum_to_lane63_d(double x) {
  x += dpp_move_d<0x128>(x);
  x += dpp_move_d<0x124>(x);
  x += dpp_move_d<0x122>(x);
  x += dpp_move_d<0x121>(x);
  x += dpp_move_d<0x142, 0xA>(x);
  x += dpp_move_d<0x143, 0xC>(x);
  return x;
}

__device__ __forceinline__ float wave_sum_to_lane63(float x) {
  x += dpp_move<0x128>(x);        // row_ror:8
  x += dpp_move<0x124>(x);        // row_ror:4
  x += dpp_move<0x122>(x);        // row_ror:2
  x += dpp_move<0x121>(x);        // row_ror:1  -> every lane holds its row sum
  x += dpp_move<0x142, 0xA>(x);   // row_bcast:15 -> rows 1, 3 add rows 0, 2
  x += dpp_move<0x143, 0xC>(x);   // row_bcast:31 -> rows 2, 3 add lane 31
  return x;
}

// Kernel timing: while profiling is enabled, a ProfScope brackets the launches
// made during its lifetime with two events on the launch stream.
struct ProfScope {
  ProfScope(const char* name, hipStream_t s);
  ~ProfScope();
  const char* name_;
  hipStream_t s_;
  int slot_;
};

// host launchers (each returns hipSuccess or the launch error)
hipError_t launch_cam_setup(const Plan& p, const ls_cameras* cams, char* ws, hipStream_t s);
hipError_t launch_project(const Plan& p, const ls_config* cfg, const ls_splats* sp, char* ws,
                          hipStream_t s);
hipError_t launch_bin_sort(const Plan& p, const ls_config* cfg, char* ws, hipStream_t s);
hipError_t launch_chunk_bin(const Plan& p, int c, char* ws, hipStream_t s);
hipError_t launch_raster_fwd(const Plan& p, const ls_config* cfg, char* ws, float* image,
                             float* final_T, int32_t* last, hipStream_t s);
hipError_t launch_project_bwd(const Plan& p, const ls_config* cfg, const ls_splats* sp, char* ws,
                              const ls_grads* g, hipStream_t s);
hipError_t launch_adam(const ls_adam_params* prm, const int64_t* step_dev, int64_t n, float* p,
                       const float* g, float* m, float* v, hipStream_t s);
hipError_t launch_densify_stats(const Plan& p, const ls_config* cfg, char* ws,
                                const ls_densify_acc* acc, hipStream_t s);
hipError_t launch_densify_select(const ls_densify_params* prm, int64_t n, const float* scales,
                                 const float* opacity, const ls_densify_acc* acc, uint8_t* action,
                                 int64_t* counts, hipStream_t s);
hipError_t launch_det_order(const Plan& p, char* ws, hipStream_t s);
hipError_t launch_det_reduce(const Plan& p, char* ws, hipStream_t s);
const uint32_t* det_slots(const Plan& p, char* ws);
size_t loss_workspace_bytes(int64_t P, int C);
hipError_t launch_loss(const int32_t* W, const int32_t* H, int C, const float* image,
                       const float* target, float* dL_dimage, double* loss, char* ws,
                       hipStream_t s, bool timed = true);
// device address of the static loss scratch on the stream's device
hipError_t loss_noalloc_scratch(hipStream_t s, char** out);
hipError_t launch_raster_bwd(const Plan& p, const ls_config* cfg, const ls_splats* sp, char* ws,
                             const float* final_T, const int32_t* last, const float* dL_dimage,
                             const float* dL_dalpha, const ls_grads* g, hipStream_t s);

}  // namespace lsplat
