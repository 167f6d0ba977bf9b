// C-ABI entry points of liblsplat: argument validation, workspace planning and
// the enqueue of each stage.  Kernels live in project.hip, binsort.hip,
// raster.hip, and (training-step stages) loss.hip and train.hip.
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <rocprofiler-sdk-roctx/roctx.h>

#include <algorithm>

#include "internal.h"

namespace lsplat {

static thread_local char g_err[512] = "";

static ls_status fail(ls_status st, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
  return st;
}

static ls_status hip_fail(hipError_t e, const char* where) {
  return fail(LS_ERR_HIP, "%s: %s", where, hipGetErrorString(e));
}

static size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// One roctx range per entry point (visible to rocprofv3 --marker-trace; a
// no-op without a tool attached).
struct Range {
  explicit Range(const char* name) { roctxRangePushA(name); }
  ~Range() { roctxRangePop(); }
};

static bool tile_shape_ok(int w, int h) {
  return (w == 16 && h == 16) || (w == 16 && h == 8) || (w == 8 && h == 8) || (w == 32 && h == 8);
}

static ls_status check_config(const ls_config* c) {
  if (!c) return fail(LS_ERR_INVALID_ARG, "cfg is NULL");
  if (!(c->lambda > 0.f) || !(c->lambda < 1e6f)) return fail(LS_ERR_INVALID_ARG, "lambda must be in (0, 1e6)");
  if (!(c->eps2d > 0.f)) return fail(LS_ERR_INVALID_ARG, "eps2d must be > 0");
  if (!(c->alpha_max > 0.f && c->alpha_max < 1.f)) return fail(LS_ERR_INVALID_ARG, "alpha_max must be in (0, 1)");
  if (!(c->alpha_min >= 0.f && c->alpha_min <= c->alpha_max))
    return fail(LS_ERR_INVALID_ARG, "alpha_min must be in [0, alpha_max]");
  if (!(c->t_min >= 0.f && c->t_min < 1.f)) return fail(LS_ERR_INVALID_ARG, "t_min must be in [0, 1)");
  if (!(c->near_z > 0.f && c->far_z > c->near_z)) return fail(LS_ERR_INVALID_ARG, "need 0 < near_z < far_z");
  if (!(c->clip > 0.f)) return fail(LS_ERR_INVALID_ARG, "clip must be > 0");
  for (int i = 0; i < 3; ++i)
    if (!(c->bg[i] == c->bg[i])) return fail(LS_ERR_INVALID_ARG, "bg must be finite");
  if (c->ags != 0 && c->ags != 1) return fail(LS_ERR_INVALID_ARG, "ags must be 0 or 1");
  if (c->ags_arg != 0 && c->ags_arg != 1) return fail(LS_ERR_INVALID_ARG, "ags_arg must be 0 or 1");
  if (c->ags_scope != 0 && c->ags_scope != 1) return fail(LS_ERR_INVALID_ARG, "ags_scope must be 0 or 1");
  if (c->sh_degree < 0 || c->sh_degree > 3) return fail(LS_ERR_INVALID_ARG, "sh_degree must be 0..3");
  if (c->kernel < LS_KERNEL_LINEAR || c->kernel > LS_KERNEL_QUADRATIC)
    return fail(LS_ERR_INVALID_ARG, "kernel must be 0..4 (LS_KERNEL_*)");
  if (c->deterministic != 0 && c->deterministic != 1)
    return fail(LS_ERR_INVALID_ARG, "deterministic must be 0 or 1");
  if (c->ags && c->kernel != LS_KERNEL_LINEAR)
    return fail(LS_ERR_INVALID_ARG, "ags is defined for the linear kernel only");
  if (!tile_shape_ok(c->tile_w, c->tile_h))
    return fail(LS_ERR_UNSUPPORTED, "tile shape %dx%d not supported (16x16, 16x8, 8x8, 32x8)",
                c->tile_w, c->tile_h);
  if (c->depth_chunks < 0 || c->depth_chunks > kMaxDepthChunks)
    return fail(LS_ERR_INVALID_ARG, "depth_chunks must be 0..%d", kMaxDepthChunks);
  if (c->chunk_ratio != 0 && (c->chunk_ratio < 2 || c->chunk_ratio > 8))
    return fail(LS_ERR_INVALID_ARG, "chunk_ratio must be 0 (2) or 2..8");
  // the forward kernel stages at most one entry per thread (two pixels per
  // thread from 128 pixels up), the backward kernel one per lane of its wave
  const int pix = c->tile_w * c->tile_h;
  const int stage_cap = pix >= 128 ? pix / 2 : pix;
  if (!(c->batch == 0 || c->batch == 64 || c->batch == 128) || c->batch > stage_cap)
    return fail(LS_ERR_INVALID_ARG,
                "batch must be 0, 64 or 128 and at most %d for %dx%d tiles (entries staged per "
                "batch by the forward pass)", stage_cap, c->tile_w, c->tile_h);
  return LS_OK;
}

static ls_status make_plan(const ls_config* cfg, const ls_cameras* cams, int64_t cap, Plan* p) {
  ls_status st = check_config(cfg);
  if (st != LS_OK) return st;
  if (!cams) return fail(LS_ERR_INVALID_ARG, "cams is NULL");
  if (cams->n_cams < 1 || cams->n_cams > 65535) return fail(LS_ERR_INVALID_ARG, "n_cams must be 1..65535");
  if (cams->n_scenes < 1) return fail(LS_ERR_INVALID_ARG, "n_scenes must be >= 1");
  if (!cams->h_width || !cams->h_height || !cams->h_scene_of_cam || !cams->h_scene_splat_off)
    return fail(LS_ERR_INVALID_ARG, "camera host arrays must not be NULL");
  if (cap < 0) return fail(LS_ERR_INVALID_ARG, "isect_capacity must be >= 0");
  if (cap >= (int64_t)0xFFFFFFFFll) return fail(LS_ERR_INVALID_ARG, "isect_capacity must be < 2^32 - 1");
  const int64_t* so = cams->h_scene_splat_off;
  if (so[0] != 0) return fail(LS_ERR_INVALID_ARG, "scene_splat_off[0] must be 0");
  for (int s = 0; s < cams->n_scenes; ++s)
    if (so[s + 1] < so[s]) return fail(LS_ERR_INVALID_ARG, "scene_splat_off must be non-decreasing");
  p->C = cams->n_cams;
  p->S = cams->n_scenes;
  p->N = so[p->S];
  p->cap = cap;
  p->W.resize(p->C); p->H.resize(p->C); p->GX.resize(p->C); p->GY.resize(p->C); p->scene.resize(p->C);
  p->pair_off.assign(p->C + 1, 0); p->tile_off.assign(p->C + 1, 0); p->pix_off.assign(p->C + 1, 0);
  p->splat_lo.resize(p->C); p->splat_hi.resize(p->C);
  p->max_scene = 0;
  for (int c = 0; c < p->C; ++c) {
    int w = cams->h_width[c], h = cams->h_height[c], s = cams->h_scene_of_cam[c];
    if (w < 1 || h < 1 || w > 16384 || h > 16384)
      return fail(LS_ERR_INVALID_ARG, "camera %d: image size %dx%d outside 1..16384", c, w, h);
    if (s < 0 || s >= p->S) return fail(LS_ERR_INVALID_ARG, "camera %d: scene %d out of range", c, s);
    p->W[c] = w; p->H[c] = h; p->scene[c] = s;
    p->GX[c] = (w + cfg->tile_w - 1) / cfg->tile_w;
    p->GY[c] = (h + cfg->tile_h - 1) / cfg->tile_h;
    p->splat_lo[c] = so[s];
    p->splat_hi[c] = so[s + 1];
    p->pair_off[c + 1] = p->pair_off[c] + (so[s + 1] - so[s]);
    p->tile_off[c + 1] = p->tile_off[c] + (int64_t)p->GX[c] * p->GY[c];
    p->pix_off[c + 1] = p->pix_off[c] + (int64_t)w * h;
    p->max_scene = std::max<int64_t>(p->max_scene, so[s + 1] - so[s]);
  }
  p->M = p->pair_off[p->C];
  p->T = p->tile_off[p->C];
  p->P = p->pix_off[p->C];
  if (p->M >= 0xFFFFFFFFll) return fail(LS_ERR_UNSUPPORTED, "more than 2^32-1 (camera, splat) pairs");
  if (p->T >= 0xFFFFFFFFll) return fail(LS_ERR_UNSUPPORTED, "more than 2^32-1 tiles");
  int bits = 0;
  while (bits < 32 && ((p->T - 1) >> bits) > 0) ++bits;
  p->tile_bits = bits;
  // depth chunks: geometric boundaries M/r^(K-1), ..., M/r, M
  p->K = cfg->depth_chunks < 1 ? 1 : cfg->depth_chunks;
  const int64_t ratio = cfg->chunk_ratio == 0 ? 2 : cfg->chunk_ratio;
  p->chunk_pos.assign(p->K + 1, 0);
  for (int c = 1; c <= p->K; ++c) {
    int64_t v = p->M;
    for (int q = c; q < p->K; ++q) v /= ratio;
    p->chunk_pos[c] = v;
  }

  // workspace layout
  size_t off = 0;
  auto take = [&](size_t bytes) { size_t o = off; off = align_up(off + bytes, 256); return o; };
  ls_layout& L = p->lay;
  memset(&L, 0, sizeof(L));
  L.n_pairs = p->M; L.n_tiles = p->T; L.n_pixels = p->P; L.capacity = cap;
  const size_t M = (size_t)p->M, T = (size_t)p->T, CAP = (size_t)cap;
  L.cams = take(sizeof(CamInfo) * p->C);
  L.proj = take(sizeof(ProjRec) * M);
  L.rect = take(8 * M);
  L.ntiles = take(4 * M);
  L.depth_key = take(4 * M);
  L.order = take(4 * M);
  L.isect_off = take(8 * (M + 1));
  L.keys = take(4 * CAP);
  L.vals = take(4 * CAP);
  const size_t K = (size_t)p->K;
  L.n_chunks = p->K;
  L.ranges = take(8 * K * (T + 1));
  L.n_isect = take(8);
  L.chunk_base = take(8 * (K + 1));
  L.chunk_n = take(8 * K);
  L.flags = take(64);
  L.grad2d = take(8 * kGrad2d * M);
  L.tile_contrib = take(4 * T);
  L.scratch = off;
  p->pre_keys_a = take(4 * M);
  p->pre_keys_b = take(4 * M);
  p->pre_vals_a = take(4 * M);
  p->pre_vals_b = take(4 * M);
  p->sort_keys_b = take(4 * CAP);
  p->sort_vals_b = take(4 * CAP);
  auto blocks_for = [](int64_t n) {
    int64_t tiles = (n + kSortTile - 1) / kSortTile;
    return (int32_t)std::max<int64_t>(1, std::min<int64_t>(tiles, kMaxSortBlocks));
  };
  p->sort_blocks = blocks_for(cap);
  p->pre_blocks = blocks_for(p->M);
  int32_t hb = std::max(p->sort_blocks, p->pre_blocks);
  p->hist = take(4 * 256 * (size_t)hb);
  p->digit_tot = take(4 * 256);
  int64_t sb = (p->M + 1 + kScanThreads * 16 - 1) / (kScanThreads * 16);
  p->scan_blocks = (int32_t)std::max<int64_t>(1, std::min<int64_t>(sb, kMaxScanBlocks));
  p->scan_part = take(8 * (size_t)(p->scan_blocks + 1));
  // The span table covers the complete lists; with depth chunks the capacity
  // only holds the entries actually built, so the table is sized for
  // kSpanCover times the capacity (2 bytes per covered intersection).
  // complete lists: owner pair of every key-generation span
  const int64_t span = p->K == 1 ? kKeygenSpan : kChunkSpan;
  p->n_spans = (std::max<int64_t>(cap, 1) + span - 1) / span + 2;
  p->span_owner = take(4 * (size_t)p->n_spans);
  // depth chunks: per-pair alive counts and offsets, tile summed-area table
  p->span_cnt = take(4 * (p->K > 1 ? M : 1));
  p->span_off = take(4 * (p->K > 1 ? M : 1));
  p->pmask = take(4 * (p->K > 1 ? M : 1));
  p->alive = take(4 * T);
  p->sat = take(4 * T);
  // depth chunks: the alive flags one bit per tile (global tile id order,
  // two zero words past the end)
  p->abits = take(4 * (p->K > 1 ? 2 * ((T + 63) / 64) + 2 : 1));
  p->drect = take(8 * M);
  if (p->K > 1) {
    p->state = take(32 * (size_t)p->P);
    p->done = take((size_t)p->P);
  }
  p->t64 = take(8 * (size_t)p->P);
  if (cfg->deterministic) {
    p->det_partial = take(8 * (size_t)kGrad2d * CAP);
    p->det_k0 = take(4 * CAP);
    p->det_v0 = take(4 * CAP);
    p->det_k1 = take(4 * CAP);
    p->det_v1 = take(4 * CAP);
    p->det_cnt = take(8);
  }
  L.total_bytes = off;
  return LS_OK;
}

static ls_status check_ws(const Plan& p, void* ws, size_t ws_bytes) {
  if (!ws) return fail(LS_ERR_WORKSPACE, "workspace is NULL");
  if ((uintptr_t)ws % 256) return fail(LS_ERR_WORKSPACE, "workspace must be 256-byte aligned");
  if (ws_bytes < p.lay.total_bytes)
    return fail(LS_ERR_WORKSPACE, "workspace has %zu bytes, plan needs %zu", ws_bytes,
                p.lay.total_bytes);
  return LS_OK;
}

static ls_status check_splats(const ls_config* cfg, const Plan& p, const ls_splats* sp) {
  if (!sp) return fail(LS_ERR_INVALID_ARG, "splats is NULL");
  if (sp->n != p.N)
    return fail(LS_ERR_INVALID_ARG, "splats.n = %lld but scene offsets end at %lld",
                (long long)sp->n, (long long)p.N);
  if (p.N > 0 && (!sp->means || !sp->scales || !sp->quats || !sp->opacity || !sp->sh))
    return fail(LS_ERR_INVALID_ARG, "splat attribute pointer is NULL");
  (void)cfg;
  return LS_OK;
}

static ls_status check_loss_cams(const ls_cameras* cams, int64_t* P) {
  if (!cams) return fail(LS_ERR_INVALID_ARG, "cams is NULL");
  if (cams->n_cams < 1 || cams->n_cams > 65535) return fail(LS_ERR_INVALID_ARG, "n_cams must be 1..65535");
  if (!cams->h_width || !cams->h_height) return fail(LS_ERR_INVALID_ARG, "camera host arrays must not be NULL");
  int64_t n = 0;
  for (int c = 0; c < cams->n_cams; ++c) {
    const int w = cams->h_width[c], h = cams->h_height[c];
    if (w < 1 || h < 1 || w > 16384 || h > 16384)
      return fail(LS_ERR_INVALID_ARG, "camera %d: image size %dx%d outside 1..16384", c, w, h);
    n += (int64_t)w * h;
  }
  *P = n;
  return LS_OK;
}

}  // namespace lsplat

using namespace lsplat;

extern "C" {

int ls_version(void) { return LSPLAT_VERSION; }

const char* ls_last_error(void) { return g_err; }

ls_status ls_workspace_size(const ls_config* cfg, const ls_cameras* cams, int64_t cap,
                            size_t* bytes) {
  if (!bytes) return fail(LS_ERR_INVALID_ARG, "bytes is NULL");
  Plan p;
  ls_status st = make_plan(cfg, cams, cap, &p);
  if (st != LS_OK) return st;
  *bytes = p.lay.total_bytes;
  return LS_OK;
}

ls_status ls_workspace_layout(const ls_config* cfg, const ls_cameras* cams, int64_t cap,
                              ls_layout* out) {
  if (!out) return fail(LS_ERR_INVALID_ARG, "out is NULL");
  Plan p;
  ls_status st = make_plan(cfg, cams, cap, &p);
  if (st != LS_OK) return st;
  *out = p.lay;
  return LS_OK;
}

ls_status ls_project(const ls_config* cfg, const ls_splats* sp, const ls_cameras* cams, void* ws,
                     size_t ws_bytes, int64_t cap, void* stream) {
  Range range("ls_project");
  Plan p;
  ls_status st = make_plan(cfg, cams, cap, &p);
  if (st != LS_OK) return st;
  if ((st = check_ws(p, ws, ws_bytes)) != LS_OK) return st;
  if ((st = check_splats(cfg, p, sp)) != LS_OK) return st;
  if (!cams->viewmat || !cams->intrin) return fail(LS_ERR_INVALID_ARG, "viewmat/intrin is NULL");
  hipStream_t s = (hipStream_t)stream;
  hipError_t e = launch_cam_setup(p, cams, (char*)ws, s);
  if (e != hipSuccess) return hip_fail(e, "cam_setup");
  e = launch_project(p, cfg, sp, (char*)ws, s);
  if (e != hipSuccess) return hip_fail(e, "project");
  return LS_OK;
}

ls_status ls_bin_sort(const ls_config* cfg, const ls_cameras* cams, void* ws, size_t ws_bytes,
                      int64_t cap, void* stream) {
  Range range("ls_bin_sort");
  Plan p;
  ls_status st = make_plan(cfg, cams, cap, &p);
  if (st != LS_OK) return st;
  if ((st = check_ws(p, ws, ws_bytes)) != LS_OK) return st;
  hipError_t e = launch_bin_sort(p, cfg, (char*)ws, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "bin_sort");
  return LS_OK;
}

ls_status ls_rasterize_fwd(const ls_config* cfg, const ls_cameras* cams, void* ws,
                           size_t ws_bytes, int64_t cap, float* image, float* final_T,
                           int32_t* last, void* stream) {
  Range range("ls_rasterize_fwd");
  Plan p;
  ls_status st = make_plan(cfg, cams, cap, &p);
  if (st != LS_OK) return st;
  if ((st = check_ws(p, ws, ws_bytes)) != LS_OK) return st;
  if (!image || !final_T || !last) return fail(LS_ERR_INVALID_ARG, "image/final_T/last is NULL");
  hipError_t e = launch_raster_fwd(p, cfg, (char*)ws, image, final_T, last, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "rasterize_fwd");
  return LS_OK;
}

ls_status ls_rasterize_bwd(const ls_config* cfg, const ls_splats* sp, const ls_cameras* cams,
                           void* ws, size_t ws_bytes, int64_t cap, const float* final_T,
                           const int32_t* last, const float* dL_dimage, const float* dL_dalpha,
                           const ls_grads* g, void* stream) {
  Range range("ls_rasterize_bwd");
  Plan p;
  ls_status st = make_plan(cfg, cams, cap, &p);
  if (st != LS_OK) return st;
  if ((st = check_ws(p, ws, ws_bytes)) != LS_OK) return st;
  if ((st = check_splats(cfg, p, sp)) != LS_OK) return st;
  if (!final_T || !last || !dL_dimage) return fail(LS_ERR_INVALID_ARG, "final_T/last/dL_dimage is NULL");
  if (!g || (p.N > 0 && (!g->means || !g->scales || !g->quats || !g->opacity || !g->sh)))
    return fail(LS_ERR_INVALID_ARG, "gradient pointer is NULL");
  hipError_t e = launch_raster_bwd(p, cfg, sp, (char*)ws, final_T, last, dL_dimage, dL_dalpha,
                                   g, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "rasterize_bwd");
  return LS_OK;
}

ls_status ls_loss_workspace_size(const ls_cameras* cams, size_t* bytes) {
  if (!bytes) return fail(LS_ERR_INVALID_ARG, "bytes is NULL");
  int64_t P = 0;
  ls_status st = check_loss_cams(cams, &P);
  if (st != LS_OK) return st;
  *bytes = loss_workspace_bytes(P, cams->n_cams);
  return LS_OK;
}

ls_status ls_loss(const ls_cameras* cams, const float* image, const float* target,
                  float* dL_dimage, double* loss, void* ws, size_t ws_bytes, void* stream) {
  Range range("ls_loss");
  int64_t P = 0;
  ls_status st = check_loss_cams(cams, &P);
  if (st != LS_OK) return st;
  if (!image || !target || !dL_dimage || !loss)
    return fail(LS_ERR_INVALID_ARG, "image/target/dL_dimage/loss is NULL");
  if (!ws) return fail(LS_ERR_WORKSPACE, "workspace is NULL");
  if ((uintptr_t)ws % 256) return fail(LS_ERR_WORKSPACE, "workspace must be 256-byte aligned");
  const size_t need = loss_workspace_bytes(P, cams->n_cams);
  if (ws_bytes < need) return fail(LS_ERR_WORKSPACE, "workspace has %zu bytes, loss needs %zu", ws_bytes, need);
  hipError_t e = launch_loss(cams->h_width, cams->h_height, cams->n_cams, image, target, dL_dimage,
                             loss, (char*)ws, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "loss");
  return LS_OK;
}

ls_status ls_loss_noalloc(const ls_cameras* cams, const float* image, const float* target,
                          float* dL_dimage, double* loss, void* stream) {
  int64_t P = 0;
  ls_status st = check_loss_cams(cams, &P);
  if (st != LS_OK) return st;
  if (!image || !target || !dL_dimage || !loss)
    return fail(LS_ERR_INVALID_ARG, "image/target/dL_dimage/loss is NULL");
  const size_t need = loss_workspace_bytes(P, cams->n_cams);
  if (need > LS_LOSS_NOALLOC_SCRATCH_BYTES)
    return fail(LS_ERR_INVALID_ARG,
                "ls_loss_noalloc: %lld pixels over %d cameras need %zu bytes of scratch; the static "
                "scratch holds %zu (about %zu pixels); use ls_loss with a workspace",
                (long long)P, cams->n_cams, need, (size_t)LS_LOSS_NOALLOC_SCRATCH_BYTES,
                (size_t)LS_LOSS_NOALLOC_SCRATCH_BYTES / 72);
  char* ws = nullptr;
  hipError_t e = loss_noalloc_scratch((hipStream_t)stream, &ws);
  if (e != hipSuccess) return hip_fail(e, "loss scratch address");
  e = launch_loss(cams->h_width, cams->h_height, cams->n_cams, image, target, dL_dimage, loss, ws,
                  (hipStream_t)stream, false);
  if (e != hipSuccess) return hip_fail(e, "loss");
  return LS_OK;
}

static ls_status check_adam(const ls_adam_params* prm, bool need_step, int64_t n, float* param,
                            const float* grad, float* m, float* v) {
  if (!prm) return fail(LS_ERR_INVALID_ARG, "prm is NULL");
  if (n < 0) return fail(LS_ERR_INVALID_ARG, "n must be >= 0");
  if (need_step && prm->step < 1) return fail(LS_ERR_INVALID_ARG, "step must be >= 1");
  if (!(prm->beta1 >= 0.0 && prm->beta1 < 1.0) || !(prm->beta2 >= 0.0 && prm->beta2 < 1.0))
    return fail(LS_ERR_INVALID_ARG, "beta1 and beta2 must be in [0, 1)");
  if (!(prm->eps >= 0.0) || !(prm->lr == prm->lr)) return fail(LS_ERR_INVALID_ARG, "eps must be >= 0, lr finite");
  if (n > 0 && (!param || !grad || !m || !v)) return fail(LS_ERR_INVALID_ARG, "param/grad/m/v is NULL");
  return LS_OK;
}

ls_status ls_adam(const ls_adam_params* prm, int64_t n, float* param, const float* grad,
                  float* m, float* v, void* stream) {
  Range range("ls_adam");
  ls_status st = check_adam(prm, true, n, param, grad, m, v);
  if (st != LS_OK) return st;
  hipError_t e = launch_adam(prm, nullptr, n, param, grad, m, v, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "adam");
  return LS_OK;
}

ls_status ls_adam_device_step(const ls_adam_params* prm, const int64_t* step_dev, int64_t n,
                              float* param, const float* grad, float* m, float* v,
                              void* stream) {
  Range range("ls_adam_device_step");
  if (!step_dev) return fail(LS_ERR_INVALID_ARG, "step_dev is NULL");
  ls_status st = check_adam(prm, false, n, param, grad, m, v);
  if (st != LS_OK) return st;
  hipError_t e = launch_adam(prm, step_dev, n, param, grad, m, v, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "adam_device_step");
  return LS_OK;
}

ls_status ls_densify_stats(const ls_config* cfg, const ls_cameras* cams, void* ws,
                           size_t ws_bytes, int64_t cap, const ls_densify_acc* acc,
                           void* stream) {
  Range range("ls_densify_stats");
  Plan p;
  ls_status st = make_plan(cfg, cams, cap, &p);
  if (st != LS_OK) return st;
  if ((st = check_ws(p, ws, ws_bytes)) != LS_OK) return st;
  if (!acc || (p.N > 0 && (!acc->grad || !acc->count || !acc->max_extent)))
    return fail(LS_ERR_INVALID_ARG, "accumulator pointer is NULL");
  hipError_t e = launch_densify_stats(p, cfg, (char*)ws, acc, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "densify_stats");
  return LS_OK;
}

ls_status ls_densify_select(const ls_densify_params* prm, int64_t n, const float* scales,
                            const float* opacity, const ls_densify_acc* acc, uint8_t* action,
                            int64_t* counts, void* stream) {
  Range range("ls_densify_select");
  if (!prm) return fail(LS_ERR_INVALID_ARG, "prm is NULL");
  if (n < 0) return fail(LS_ERR_INVALID_ARG, "n must be >= 0");
  const double th[7] = {prm->grad_threshold, prm->grow_scale2d, prm->grow_scale3d,
                        prm->prune_scale2d, prm->prune_scale3d, prm->prune_opacity,
                        prm->scene_scale};
  for (double t : th)
    if (!(t >= 0.0) || !(t < 1e300)) return fail(LS_ERR_INVALID_ARG, "thresholds must be finite and >= 0");
  if ((prm->grow2d != 0 && prm->grow2d != 1) || (prm->prune_big != 0 && prm->prune_big != 1))
    return fail(LS_ERR_INVALID_ARG, "grow2d and prune_big must be 0 or 1");
  if (n > 0 && (!scales || !opacity || !action || !acc || !acc->grad || !acc->count ||
                !acc->max_extent))
    return fail(LS_ERR_INVALID_ARG, "scales/opacity/action/accumulator pointer is NULL");
  hipError_t e = launch_densify_select(prm, n, scales, opacity, acc, action, counts,
                                       (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "densify_select");
  return LS_OK;
}

}  // extern "C"
