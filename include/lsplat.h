/*
 * lsplat: tile-based differentiable rasterizer for 3D Linear Splatting
 * (Chen et al., "Beyond Gaussians: Fast and High-Fidelity 3D Splatting with
 * Linear Kernels", arXiv 2411.12440), for AMD MI355X (gfx950).
 *
 * C ABI.  No HIP or PyTorch types appear in these signatures: device memory
 * is passed as plain pointers, streams as an opaque `void*` holding a
 * hipStream_t (NULL = the null stream).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Pointers are DEVICE pointers unless a field is named h_*, which is HOST
 *    memory read during the call only.
 *  - The caller allocates and owns every buffer, including the workspace;
 *    the library keeps no pointer after the call returns and frees nothing.
 *  - Calls only enqueue work on the given stream (asynchronous, no host
 *    synchronisation).  Buffers must stay valid until that work completes.
 *  - Argument errors are detected on the host before any launch and return a
 *    negative ls_status; ls_last_error() then describes the problem.  HIP
 *    launch failures return LS_ERR_HIP.
 *  - Splat attributes are FP32 structure-of-arrays ("planar"): a field with
 *    components [d][n] stores component 0 of all n splats, then component 1...
 *  - Images are planar per camera: camera c owns 3*H_c*W_c floats (R plane,
 *    G plane, B plane, each row-major H_c x W_c), cameras concatenated in
 *    order.  Per-pixel arrays (final_T, last) hold H_c*W_c entries per camera,
 *    concatenated.
 *  - (camera, splat) pairs are numbered camera-major: pair index m of splat i
 *    of camera c is pair_off[c] + (i - first splat of c's scene), where
 *    pair_off[c] is the sum of the scene sizes of cameras 0..c-1.
 *  - Global tile ids are tile_off[c] + ty * GX_c + tx with GX_c = ceil(W_c/tile_w),
 *    GY_c = ceil(H_c/tile_h), tile_off[c] = sum over earlier cameras of GX*GY.
 */
#ifndef LSPLAT_H
#define LSPLAT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define LSPLAT_VERSION 171

typedef enum {
  LS_OK = 0,
  LS_ERR_INVALID_ARG = -1,   /* bad pointer, size, flag or shape */
  LS_ERR_CAPACITY = -2,      /* intersection capacity provably too small */
  LS_ERR_HIP = -3,           /* a HIP call or kernel launch failed */
  LS_ERR_UNSUPPORTED = -4,   /* a valid request this build does not implement */
  LS_ERR_WORKSPACE = -5      /* workspace pointer/size does not match the plan */
} ls_status;

/*
 * Rasterizer settings (host struct, read during the call only).
 *
 * lambda     Distribution-alignment factor of Eq. 12 (Sec. 3.3.1): the kernel
 *            is L' = max(0, 1 - D'/lambda) with D' the 2D Mahalanobis distance
 *            of Eq. 11.  The paper uses 2.5; 1.0 is the plain kernel of Eq. 10.
 *            Must be > 0.  With another kernel (below) it scales D' the same
 *            way: the kernel value is f(D'/lambda).
 * kernel     The attenuation f of the generalised kernel E(x) = f(D(x)) in the
 *            appendix ("Generalizing the 3DGS Kernel Function"):
 *              LS_KERNEL_LINEAR     max(0, 1 - D)      (default, the paper's)
 *              LS_KERNEL_GAUSSIAN   exp(-D^2 / 2)
 *              LS_KERNEL_LAPLACIAN  exp(-D)
 *              LS_KERNEL_COSINE     (1 + cos(pi D)) / 2 for D <= 1, else 0
 *              LS_KERNEL_QUADRATIC  max(0, 1 - D^2)
 *            A splat's support is D'/lambda < s_f: s_f = 1, except 3 for the
 *            Gaussian (the 3-sigma cut of 3DGS) and ln 255 for the Laplacian
 *            (beyond it alpha < 1/255).  Binning bounds the ellipse
 *            D' = extent with extent = lambda * s_f rounded to FP32.  The
 *            appendix's aligned lambdas are 2.5 (cosine, linear), 6
 *            (quadratic) and 1 (Laplacian); 1 is the plain Gaussian.
 * ags        1: adaptive gradient scaling of Eq. 13-14 (Sec. 3.3.2) in the
 *            backward pass.  The forward pass is unchanged.  Defined for the
 *            linear kernel only (LS_ERR_INVALID_ARG with another kernel).
 * ags_arg    0: omega = exp(-D'^2) (raw distance, default); 1: exp(-(D'/lambda)^2).
 * ags_scope  0: omega scales only the gradient through L' into the splat
 *            geometry (default); 1: omega scales every gradient of the pair.
 * eps2d      Dilation added to the diagonal of the 2D covariance (> 0).
 * alpha_min  A splat whose alpha is below this is skipped (default 1/255).
 * alpha_max  alpha = min(alpha_max, o * L') (default 0.99; in (0, 1)).
 * t_min      A splat that would take the transmittance below t_min stops the
 *            pixel and is not added (default 1e-4).  The three blending rules
 *            are the 3DGS ones the paper keeps unchanged (Sec. 3.2).
 * near_z, far_z  A splat centre outside (near_z, far_z) in camera z is culled.
 * clip       The tangent used in the projection Jacobian is clamped to
 *            clip * (half field of view) (default 1.3).
 * bg         Background colour added as T_final * bg.
 * sh_degree  Degree 0..3 of the real spherical-harmonics colour.
 * tile_w, tile_h  Tile shape in pixels: 16x16, 16x8, 8x8 or 32x8.
 * batch      Splats staged in LDS per batch by the forward kernel: 0 (one
 *            per thread), 64 or 128, at most the forward kernel's threads
 *            (the tile's pixels, halved from 128 pixels up, where each
 *            thread composites two pixels): 128 for 16x16 and 32x8, 64 for
 *            16x8 and 8x8.  The backward kernel runs one wave per tile and
 *            stages min(batch, 64) (64 for batch 0).
 * depth_chunks  0 or 1: ls_bin_sort builds every tile's complete list.
 *            K in 2..12: ls_bin_sort only orders the pairs by depth and scans
 *            their tile counts; ls_rasterize_fwd then builds the lists in K
 *            chunks of that order (with r = chunk_ratio: chunk k of 1..K
 *            ends at M/r^(K-k), so the first M/r^(K-1) pairs, then up to
 *            M/r^(K-2), ..., the last from M/r to M) and composites each
 *            chunk before building the next.  A chunk skips every tile whose
 *            pixels have all stopped (T would fall below t_min), so each
 *            tile's list is the prefix of its complete list that the
 *            composite can reach.  Images and gradients are identical to the
 *            complete-list mode.
 * chunk_ratio  The factor r between successive depth-chunk boundaries
 *            (above): 0 for the default 2, or 2..8.  A larger r builds more
 *            entries in fewer, larger chunks.
 * deterministic  0: the backward pass sums each splat's per-tile gradients
 *            with FP64 atomics (order-dependent in the last bits).  1: it
 *            stores every list entry's per-tile sums in the workspace, orders
 *            the entries by pair (a stable radix sort) and sums each pair's
 *            entries in list order, so that gradients are bitwise
 *            reproducible from run to run and between the batched and the
 *            per-view calls.  Costs 88 bytes of workspace per intersection of
 *            capacity and a slower backward pass.
 */
typedef struct ls_config {
  float lambda;
  float eps2d;
  float alpha_min, alpha_max, t_min;
  float near_z, far_z, clip;
  float bg[3];
  int32_t ags, ags_arg, ags_scope;
  int32_t sh_degree;
  int32_t tile_w, tile_h;
  int32_t batch;
  int32_t depth_chunks;
  int32_t kernel;
  int32_t deterministic;
  int32_t chunk_ratio;
} ls_config;

enum {
  LS_KERNEL_LINEAR = 0,
  LS_KERNEL_GAUSSIAN = 1,
  LS_KERNEL_LAPLACIAN = 2,
  LS_KERNEL_COSINE = 3,
  LS_KERNEL_QUADRATIC = 4
};

/*
 * Splats of one or more scenes, concatenated (Sec. 3.1: centre mu, scale S and
 * rotation R with Sigma = R S S^T R^T (Eq. 2), opacity o, colour c (Eq. 6)).
 * n        total splats over all scenes.
 * means    [3][n] world-space centres.
 * scales   [3][n] per-axis scales, > 0 (activated, not log).
 * quats    [4][n] rotation quaternions (w, x, y, z), any non-zero norm.
 * opacity  [n] in (0, 1) (activated, not logit).
 * sh       [K][3][n] SH coefficients, K = (sh_degree + 1)^2, band-major then
 *          channel.
 */
typedef struct ls_splats {
  int64_t n;
  const float* means;
  const float* scales;
  const float* quats;
  const float* opacity;
  const float* sh;
} ls_splats;

/*
 * Gradients w.r.t. the ls_splats fields, same shapes (written, not added).
 * mean2d_norm  optional (NULL to skip) [M] per (camera, splat) pair: the
 *              Euclidean norm of dL/d(projected centre) in pixels, the
 *              per-view statistic that 3DGS-style densification accumulates;
 *              0 for a pair that received no gradient.
 */
typedef struct ls_grads {
  float* means;
  float* scales;
  float* quats;
  float* opacity;
  float* sh;
  float* mean2d_norm;
} ls_grads;

/*
 * Cameras (Sec. 3.1, Eq. 3: world-to-camera W and the local affine Jacobian J
 * of the pinhole map).  OpenCV axes: x right, y down, z forward.  Pixel
 * (px, py) samples the point (px + 0.5, py + 0.5).
 * viewmat            device [C][3][4] world->camera (rotation | translation).
 * intrin             device [C][4] (fx, fy, cx, cy).
 * h_width, h_height  host [C] image size in pixels (>= 1).
 * h_scene_of_cam     host [C] scene index of each camera (0..n_scenes-1).
 * h_scene_splat_off  host [n_scenes + 1] first splat of each scene in the
 *                    concatenated ls_splats, increasing, last = n.
 */
typedef struct ls_cameras {
  int32_t n_cams;
  int32_t n_scenes;
  const float* viewmat;
  const float* intrin;
  const int32_t* h_width;
  const int32_t* h_height;
  const int32_t* h_scene_of_cam;
  const int64_t* h_scene_splat_off;
} ls_cameras;

/*
 * Byte offsets (from the workspace base) and element counts of the arrays the
 * library keeps in the caller's workspace.  Filled by ls_workspace_layout;
 * exposed so that callers and tests can read intermediate results.
 *   M = number of (camera, splat) pairs, T = total tiles, cap = capacity.
 *   proj       [M] 64-byte records: double mean2d[2], double conic[3]
 *              (A, B, C with D'^2 = A dx^2 + 2B dx dy + C dy^2), float rgb[3],
 *              float opacity, 8 bytes padding.
 *   rect       [M] uint16 x4: tile rectangle (tx0, ty0, tx1, ty1) inclusive;
 *              (1, 1, 0, 0), an empty rectangle, for a culled pair.
 *   ntiles     [M] uint32: tiles touched (0 = culled).
 *   depth_key  [M] uint32: FP32 bit pattern of camera-space z (0xFFFFFFFF if
 *              culled).
 *   order      [M] uint32: pair ids sorted by (depth_key, pair id).
 *   isect_off  [M+1] int64: exclusive scan of ntiles in `order` (with depth
 *              chunks only isect_off[M], the total, is written).
 *   keys       [cap] uint32: sorted global tile ids, chunk after chunk.
 *   vals       [cap] uint32: pair ids in (tile, depth, pair id) order within
 *              each chunk.
 *   ranges     [K][T+1] int64: in chunk c, tile t owns the sorted positions
 *              chunk_base[c] + [ranges[c][t], ranges[c][t+1]).  A tile's list
 *              is the concatenation of its chunk segments in chunk order.
 *   n_isect    int64 scalar: intersection count of the complete lists.
 *   chunk_base [K+1] int64: first entry of each chunk; chunk_base[K] is the
 *              number of entries built.
 *   chunk_n    [K] int64: entries of each chunk.
 *   flags      int32[16]: flags[0] != 0 when the entries did not fit in the
 *              capacity (the composite is then incomplete: grow the capacity
 *              to at least n_isect and run again).
 *   grad2d     [9][M] double: per-pair sums over the pair's pixels (backward),
 *              field-major: dL/d(projected centre) x, y; dL/da, dL/db, dL/dc
 *              for the dilated 2D covariance [[a, b], [b, c]] (b a single
 *              parameter); dL/dopacity; dL/drgb (3).
 *   tile_contrib [T] uint32: per tile, the (pixel, splat) pairs that
 *              contributed to the composite in the last ls_rasterize_fwd call
 *              (alpha >= alpha_min, before the pixel stopped); the backward
 *              pass visits the same set.
 */
typedef struct ls_layout {
  int64_t n_pairs, n_tiles, n_pixels, capacity, n_chunks;
  size_t total_bytes;
  size_t cams, proj, rect, ntiles, depth_key, order, isect_off, keys, vals, ranges,
      n_isect, chunk_base, chunk_n, flags, grad2d, tile_contrib;
  size_t scratch;   /* library-internal (sort buffers, histograms, state) */
} ls_layout;

/* Library version (LSPLAT_VERSION). */
int ls_version(void);

/* Text of the last error on the calling thread; valid until the next call. */
const char* ls_last_error(void);

/*
 * Workspace needed for these cameras and settings with room for
 * `isect_capacity` (>= 0) (tile, splat) intersections.  Host-only.
 */
ls_status ls_workspace_size(const ls_config* cfg, const ls_cameras* cams,
                            int64_t isect_capacity, size_t* bytes);

/* Same plan, with the offset of every array (see ls_layout).  Host-only. */
ls_status ls_workspace_layout(const ls_config* cfg, const ls_cameras* cams,
                              int64_t isect_capacity, ls_layout* out);

/*
 * Projection (Sec. 3.1, Eq. 2-4; kernel support from Eq. 11-12).  For every
 * (camera, splat) pair: covariance Sigma = R S S^T R^T, camera-space centre,
 * projected centre, dilated 2D covariance Sigma_2D = (J W Sigma W^T J^T)_2x2
 * + eps2d I and its inverse, SH colour, and the tile rectangle that bounds
 * the support ellipse D' < lambda.  Writes proj, rect, ntiles and depth_key of
 * the workspace.  Geometry that feeds rasterization is computed in FP64;
 * rect, ntiles and depth_key follow a fixed FP32 operation sequence (no fused
 * multiply-add, correctly rounded division and square root) so that they are
 * reproducible bit for bit.
 */
ls_status ls_project(const ls_config* cfg, const ls_splats* splats, const ls_cameras* cams,
                     void* ws, size_t ws_bytes, int64_t isect_capacity, void* stream);

/*
 * Binning: order pairs front to back by (depth_key, pair id), scan their tile
 * counts, write one (global tile, pair) entry per touched tile, stably radix
 * sort the entries by tile id, and compute each tile's range.  The result is
 * every tile's list in ascending (depth_key, pair id) order.  The paper keeps
 * this stage of the 3DGS pipeline (Sec. 3.2, Sec. 4.1) without describing it.
 * n_isect always receives the true count; when the entries do not fit in
 * the capacity, nothing past the capacity is written, the lists stay empty
 * and flags[0] is raised: grow the capacity and run again.  With
 * depth_chunks > 1 this call stops after the depth order and the scan; the
 * lists are built by ls_rasterize_fwd.  Requires a preceding ls_project on
 * `ws`.
 */
ls_status ls_bin_sort(const ls_config* cfg, const ls_cameras* cams, void* ws, size_t ws_bytes,
                      int64_t isect_capacity, void* stream);

/*
 * Forward compositing (Eq. 6 with the linear kernel of Eq. 10-12): for each
 * pixel, walk its tile's list front to back, alpha = min(alpha_max,
 * o * max(0, 1 - D'/lambda)), skip alpha < alpha_min, stop before a splat
 * that would take T below t_min, C += c alpha T, T *= (1 - alpha).
 * image    [sum_c 3 H_c W_c] out: C + T_final * bg.
 * final_T  [P] out: final transmittance.
 * last     [P] out: 1 + position in the tile list of the last contributing
 *          splat (0 if none); the backward pass starts there.
 */
ls_status ls_rasterize_fwd(const ls_config* cfg, const ls_cameras* cams, void* ws,
                           size_t ws_bytes, int64_t isect_capacity, float* image,
                           float* final_T, int32_t* last, void* stream);

/*
 * Backward pass of ls_rasterize_fwd and ls_project.  Walks each tile's list
 * back to front from `last`, recovering the transmittance by division
 * (T_i = T_{i+1} / (1 - alpha_i)) from the FP64 final transmittance the
 * forward call keeps in the workspace (final_T is its FP32 rounding, which
 * can underflow when t_min = 0), accumulates per-pair 2D gradients (with
 * adaptive gradient scaling, Eq. 13-14, when cfg->ags), then applies the
 * chain rule through the projection and sums over cameras.
 * final_T, last  from the forward call on the same workspace and settings.
 * dL_dimage      [sum_c 3 H_c W_c] upstream gradient.
 * dL_dalpha      optional (NULL = zero) [P] upstream gradient of each pixel's
 *                accumulated opacity 1 - T_final.  It enters as a fourth
 *                channel whose splat colours are 0 and whose background is -1:
 *                dL/dalpha_i gains dL_dalpha * T_final / (1 - alpha_i).
 * grads          out: written (not accumulated) for every splat.
 */
ls_status ls_rasterize_bwd(const ls_config* cfg, const ls_splats* splats,
                           const ls_cameras* cams, void* ws, size_t ws_bytes,
                           int64_t isect_capacity, const float* final_T, const int32_t* last,
                           const float* dL_dimage, const float* dL_dalpha,
                           const ls_grads* grads, void* stream);

/*
 * Training loss of Sec. 4.1 ("Loss Functions") and its gradient with respect
 * to the rendered image.  For each camera c, over its 3 x H_c x W_c image x
 * and target y (N_c = 3 H_c W_c values):
 *   loss[c] = 0.6 mean|x - y| + 0.2 mean (x - y)^2 + 0.2 (1 - SSIM),
 * where SSIM is the mean over channels and pixels of the SSIM map of Wang et
 * al. (2004) with local moments from an 11 x 11 Gaussian window of sigma 1.5
 * (weights summing to 1), zero padding at the border (no renormalisation
 * there), C1 = 0.01^2 and C2 = 0.03^2.  The paper fixes the weights and the
 * three terms; the window, padding and constants are the ones its 3DGS
 * baseline trains with.  The derivative of |x - y| at x = y is taken as 0.
 * cams       only n_cams, h_width and h_height are read (same checks as the
 *            other entry points: 1..65535 cameras, sizes 1..16384).
 * image      [sum_c 3 H_c W_c] device, the layout ls_rasterize_fwd writes
 *            (per camera, three planes of H_c x W_c, row-major).
 * target     [sum_c 3 H_c W_c] device, same layout.
 * dL_dimage  [sum_c 3 H_c W_c] device out: d loss[c] / d image for each
 *            camera's own pixels (written, not accumulated).  It may be
 *            passed straight to ls_rasterize_bwd: the gradient of the sum of
 *            the per-camera losses.
 * loss       [n_cams] device out, FP64.
 * ws         device workspace of at least ls_loss_workspace_size() bytes,
 *            256-byte aligned, owned by the caller; independent of the
 *            rasterizer's workspace.  Nothing is allocated.
 * Enqueued on `stream` (NULL = the null stream); returns LS_ERR_INVALID_ARG
 * or LS_ERR_WORKSPACE before launching anything when an argument is wrong.
 */
ls_status ls_loss_workspace_size(const ls_cameras* cams, size_t* bytes);
ls_status ls_loss(const ls_cameras* cams, const float* image, const float* target,
                  float* dL_dimage, double* loss, void* ws, size_t ws_bytes, void* stream);

/*
 * ls_loss without a workspace argument, for callers that cannot allocate
 * device memory: code under HIP graph capture that must not call hipMalloc,
 * tight serving loops, harnesses that forbid allocation.  Same arguments
 * (minus ws and ws_bytes), checks, kernels and results as ls_loss; it calls no
 * hipMalloc, hipFree or other allocating routine (with kernel timing enabled
 * it is not timed, since timing creates events).
 * Scratch: the derivative maps and sums live in a static device array of
 * LS_LOSS_NOALLOC_SCRATCH_BYTES (144 MiB) that each GPU the library runs on
 * holds until the process ends.  A call needs ls_loss_workspace_size() bytes
 * of it (72 bytes per pixel plus 24 per camera, each rounded up to 256): at
 * most 2,097,148 pixels for one camera, e.g. one 1920 x 1080 view.  Larger
 * inputs return LS_ERR_INVALID_ARG before anything is launched.
 * The array's address on the stream's device is looked up on the first call
 * there (that call is not legal inside a stream capture on a device the
 * library has not used yet: make one call outside the capture first).
 * Every call on a GPU shares that GPU's array, which keeps the last call's
 * contents (each call clears the sums it needs): calls that overlap on one
 * GPU (concurrent streams, threads or processes' graphs) race and give wrong
 * results.  Order them on one stream.
 */
#define LS_LOSS_NOALLOC_SCRATCH_BYTES ((size_t)144 << 20)
ls_status ls_loss_noalloc(const ls_cameras* cams, const float* image, const float* target,
                          float* dL_dimage, double* loss, void* stream);

/*
 * Adam (Kingma and Ba 2015), the optimiser of the 3DGS training the paper
 * keeps.  One step t >= 1 over n parameters, per element:
 *   m <- beta1 m + (1 - beta1) g,   v <- beta2 v + (1 - beta2) g^2,
 *   param <- param - lr (m / (1 - beta1^t)) / (sqrt(v / (1 - beta2^t)) + eps).
 * The arithmetic is FP64 on the FP32 arrays (one rounding per stored value).
 * Call once per parameter group (each has its own learning rate).  The
 * 3DGS lineage uses beta1 = 0.9, beta2 = 0.999, eps = 1e-15.
 * param, m, v  [n] device, updated in place; m and v start at zero.
 * grad         [n] device.
 * Checks: n >= 0, step >= 1, 0 <= beta1, beta2 < 1, eps >= 0, non-NULL
 * pointers when n > 0.  Allocates nothing.
 */
typedef struct ls_adam_params {
  double lr;
  double beta1;
  double beta2;
  double eps;
  int64_t step;
} ls_adam_params;

ls_status ls_adam(const ls_adam_params* prm, int64_t n, float* param, const float* grad,
                  float* m, float* v, void* stream);

/*
 * ls_adam with the step t read from device memory when the kernels run
 * (step_dev: one int64, >= 1; prm->step is not used), so that a captured
 * HIP graph can replay successive steps: the caller advances *step_dev
 * between replays, for example with a small kernel inside the graph.  Other
 * arguments, checks and arithmetic as ls_adam (the bias corrections are
 * formed on the device in FP64).
 */
ls_status ls_adam_device_step(const ls_adam_params* prm, const int64_t* step_dev, int64_t n,
                              float* param, const float* grad, float* m, float* v,
                              void* stream);

/*
 * Densification statistics (the per-splat quantities 3DGS adaptive density
 * control accumulates between densification steps; the paper's
 * densification table gives 3DLS thresholds for the decision below).
 * Accumulators, per splat, [n] device, zeroed by the caller when a new
 * accumulation period starts:
 *   grad        sum over visible pairs of |(dL/dx W/2, dL/dy H/2)|, the norm
 *               of the projected centre's gradient in normalised device
 *               coordinates.
 *   count       number of visible pairs (support on at least one tile).
 *   max_extent  max over visible pairs of the support ellipse's semi-major
 *               axis in pixels (extent times the square root of the largest
 *               eigenvalue of the dilated 2D covariance) over max(W, H).
 */
typedef struct ls_densify_acc {
  float* grad;
  int32_t* count;
  float* max_extent;
} ls_densify_acc;

/*
 * Adds the statistics of the backward pass that last ran on `ws` (same
 * settings, cameras and capacity as that ls_rasterize_bwd call).  Reads the
 * projection records and per-pair gradients the pass left in the workspace.
 */
ls_status ls_densify_stats(const ls_config* cfg, const ls_cameras* cams, void* ws,
                           size_t ws_bytes, int64_t isect_capacity, const ls_densify_acc* acc,
                           void* stream);

/*
 * The grow / prune decision.  With s the largest of a splat's three scales:
 *   high      = count > 0 and grad / count > grad_threshold
 *   small     = s <= grow_scale3d * scene_scale
 *   split     = (high and not small) or (grow2d and max_extent > grow_scale2d)
 *   duplicate = high and small and not split
 *   prune     = opacity < prune_opacity, or (prune_big and (s > prune_scale3d
 *               * scene_scale or max_extent > prune_scale2d))
 * compared in FP64 on the stored values.  3DLS thresholds (paper table):
 * 0.0002, 0.05, 0.006, 0.15, 0.4, 0.025 in the order of the fields below;
 * 3DGS: 0.0002, 0.05, 0.01, 0.15, 0.1, 0.005.  grow2d and prune_big switch
 * the screen-size and large-splat rules on (the schedule's choice).
 * scales   [3][n], opacity [n] as in ls_splats.
 * action   [n] device out: bit 1 duplicate, 2 split, 4 prune.
 * counts   optional [3] device out (NULL to skip): splats to duplicate, to
 *          split and to prune.
 * Applying the decision (new splats, compaction) is the training loop's.
 */
typedef struct ls_densify_params {
  double grad_threshold;
  double grow_scale2d;
  double grow_scale3d;
  double prune_scale2d;
  double prune_scale3d;
  double prune_opacity;
  double scene_scale;
  int32_t grow2d;
  int32_t prune_big;
} ls_densify_params;

ls_status ls_densify_select(const ls_densify_params* prm, int64_t n, const float* scales,
                            const float* opacity, const ls_densify_acc* acc, uint8_t* action,
                            int64_t* counts, void* stream);

/*
 * Kernel timing (tracing).  While enabled, every kernel the library enqueues
 * is bracketed by a pair of HIP events recorded on the same stream.
 * ls_profile_read waits for the recorded events, adds their elapsed times
 * into per-kernel totals and writes up to `capacity` entries (kernel name,
 * launches, total milliseconds) sorted by total time, longest first; *count
 * receives the number of distinct kernels.  reset != 0 clears the totals.
 * Not thread-safe; the library creates its events on first use and keeps them
 * (a few hundred) until the process ends.
 */
typedef struct ls_kernel_time {
  char name[48];
  int64_t launches;
  double total_ms;
} ls_kernel_time;

ls_status ls_profile_enable(int enable);
ls_status ls_profile_read(ls_kernel_time* out, int capacity, int* count, int reset);

#ifdef __cplusplus
}
#endif

#endif /* LSPLAT_H */
