// C ABI of libhgs: argument validation, camera packing, workspace sizing and
// the launch sequence of each entry point.  No entry point allocates device
// memory or synchronises the stream.

#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <mutex>

#include "hgs_internal.h"

namespace {

thread_local char g_err[512] = "";

int fail(int code, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
  return code;
}

int hip_fail(hipError_t e, const char* where) {
  return fail(HGS_EHIP, "%s: %s", where, hipGetErrorString(e));
}

int ilog2(int x) {
  int r = 0;
  while ((1 << r) < x) ++r;
  return r;
}

int check_opts(const hgs_options* o) {
  if (!o) return fail(HGS_EINVAL, "options is null");
  if (o->tile != 8 && o->tile != 16 && o->tile != 32)
    return fail(HGS_EINVAL, "tile must be 8, 16 or 32 (got %d)", o->tile);
  if (o->batch != 128 && o->batch != 256 && o->batch != 512)
    return fail(HGS_EINVAL, "batch must be 128, 256 or 512 (got %d)", o->batch);
  if (!(o->kappa > 0.0f) || !(o->lowpass >= 0.0f) || !(o->alpha_max > 0.0f) ||
      !(o->alpha_max < 1.0f) || !(o->alpha_min >= 0.0f) || !(o->t_min > 0.0f) ||
      !(o->t_min < 1.0f) || !(o->fov_clamp > 0.0f))
    return fail(HGS_EINVAL, "option value out of range");
  return HGS_OK;
}

// Builds the kernel-side camera pack; returns an error code.
int make_pack(const hgs_camera* cams, int32_t n_cams, const hgs_options* o, hgs::CamPack* cp) {
  if (!cams) return fail(HGS_EINVAL, "cameras is null");
  if (n_cams < 1 || n_cams > HGS_MAX_CAMERAS)
    return fail(HGS_EINVAL, "n_cams must be in 1..%d (got %d)", HGS_MAX_CAMERAS, n_cams);
  memset(cp, 0, sizeof(*cp));
  cp->n_cams = n_cams;
  cp->tile = o->tile;
  cp->tile_shift = ilog2(o->tile);
  uint64_t toff = 0, poff = 0;
  for (int c = 0; c < n_cams; ++c) {
    const hgs_camera& s = cams[c];
    if (s.width < 1 || s.height < 1 || s.width > HGS_MAX_IMAGE_SIDE || s.height > HGS_MAX_IMAGE_SIDE)
      return fail(HGS_EINVAL, "camera %d: image size %dx%d out of range", c, s.width, s.height);
    if (!(s.fx > 0.0f) || !(s.fy > 0.0f) || !isfinite(s.fx) || !isfinite(s.fy))
      return fail(HGS_EINVAL, "camera %d: focal lengths must be positive and finite", c);
    // a near plane at or behind the camera would let kernels with camera z
    // in (znear, 0] through, projected mirrored and sorted after every
    // positive depth
    if (!(s.znear > 0.0f) || !isfinite(s.znear))
      return fail(HGS_EINVAL, "camera %d: znear must be positive and finite (got %g)", c, (double)s.znear);
    hgs::CamDev& d = cp->cam[c];
    memcpy(d.R, s.R, sizeof(d.R));
    memcpy(d.t, s.t, sizeof(d.t));
    d.fx = s.fx;
    d.fy = s.fy;
    d.cx = s.cx;
    d.cy = s.cy;
    d.znear = s.znear;
    d.width = s.width;
    d.height = s.height;
    d.tiles_x = (s.width + o->tile - 1) / o->tile;
    d.tiles_y = (s.height + o->tile - 1) / o->tile;
    d.tile_off = (uint32_t)toff;
    d.pix_off = poff;
    toff += (uint64_t)d.tiles_x * d.tiles_y;
    poff += (uint64_t)s.width * s.height;
  }
  if (toff >= (1ull << 31)) return fail(HGS_EINVAL, "too many tiles");
  cp->tiles_total = (uint32_t)toff;
  return HGS_OK;
}

int make_params(const hgs_params* p, hgs::Params* out) {
  if (!p) return fail(HGS_EINVAL, "params is null");
  if (p->n < 0) return fail(HGS_EINVAL, "n must be >= 0");
  if (p->stride < p->n) return fail(HGS_EINVAL, "stride must be >= n");
  if (p->sh_degree < 0 || p->sh_degree > 3) return fail(HGS_EINVAL, "sh_degree must be 0..3");
  if (p->n > 0 && (!p->means || !p->scales || !p->quats || !p->normals || !p->opac1 || !p->opac2 ||
                   !p->sh))
    return fail(HGS_EINVAL, "a parameter pointer is null");
  if (p->n > (int64_t)INT32_MAX / HGS_MAX_CAMERAS) return fail(HGS_EINVAL, "n too large");
  out->means = p->means;
  out->scales = p->scales;
  out->quats = p->quats;
  out->normals = p->normals;
  out->opac1 = p->opac1;
  out->opac2 = p->opac2;
  out->sh = p->sh;
  out->filter3d = p->filter3d;
  out->n = p->n;
  out->stride = p->stride;
  out->sh_degree = p->sh_degree;
  return HGS_OK;
}

}  // namespace

// A mutable plane set with every field present.
int planes_ok(const hgs_param_grads* g, const char* what) {
  if (!g) return fail(HGS_EINVAL, "%s is null", what);
  if (!g->means || !g->scales || !g->quats || !g->normals || !g->opac1 || !g->opac2 || !g->sh)
    return fail(HGS_EINVAL, "%s: a plane pointer is null", what);
  return HGS_OK;
}

hgs::Grads to_grads(const hgs_param_grads& g) {
  return hgs::Grads{g.means, g.scales, g.quats, g.normals, g.opac1, g.opac2, g.sh};
}

int check_sizes(int64_t n, int64_t stride, int32_t sh_degree) {
  if (n < 0) return fail(HGS_EINVAL, "n must be >= 0");
  if (stride < n) return fail(HGS_EINVAL, "stride must be >= n");
  if (sh_degree < 0 || sh_degree > 3) return fail(HGS_EINVAL, "sh_degree must be 0..3");
  return HGS_OK;
}

bool aligned16(const void* p) { return ((uintptr_t)p & 15u) == 0; }

namespace {

// ---------------------------------------------------------------------------
// Device scratch of hgs_preprocess_noalloc: the partial sums of the entry
// count (one uint64 per 256 kernels, or per 4096 records with offsets), for
// callers that cannot allocate.  Each device holds its own copy of the array for the life of the
// process.  In host code `scratch` names a host-side stand-in, not device
// memory: its device address on the current device comes from
// hipGetSymbolAddress, taken once per device and kept in g_scratch.  The
// partials are overwritten by every call (nothing needs clearing), so two
// calls in flight on one device at the same time race on them.
constexpr size_t kNoAllocScratchBytes = 4 * 1024 * 1024;
constexpr int64_t kNoAllocMaxRecords =
    (int64_t)(kNoAllocScratchBytes / sizeof(uint64_t)) * hgs::kPreprocessRecordsPerPartial;
static_assert(kNoAllocMaxRecords == HGS_NOALLOC_MAX_RECORDS, "hgs.h states the no-alloc limit");
static __device__ __align__(256) uint8_t scratch[kNoAllocScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch[kMaxDevices] = {};

// Device address of `scratch` on the current device.
int scratch_address(void** out) {
  int dev = 0;
  hipError_t h = hipGetDevice(&dev);
  if (h != hipSuccess) return hip_fail(h, "hipGetDevice");
  if (dev < 0 || dev >= kMaxDevices) return fail(HGS_EINVAL, "device index %d out of range", dev);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch[dev]) {
    void* p = nullptr;
    h = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (h != hipSuccess) return hip_fail(h, "hipGetSymbolAddress(scratch)");
    if (!p) return fail(HGS_EHIP, "hipGetSymbolAddress(scratch) returned null");
    g_scratch[dev] = p;
  }
  *out = g_scratch[dev];
  return HGS_OK;
}

// hgs_preprocess with the caller's workspace, or (no_alloc) the scratch array.
int preprocess_impl(const hgs_params* params, const hgs_camera* cams, int32_t n_cams, const hgs_options* opts,
                    void* records, uint32_t* tiles_touched, uint64_t* offsets, uint64_t* n_dup, void* workspace,
                    size_t workspace_bytes, bool no_alloc, hipStream_t stream) {
  int e;
  if ((e = check_opts(opts)) != HGS_OK) return e;
  hgs::Params p;
  if ((e = make_params(params, &p)) != HGS_OK) return e;
  hgs::CamPack cp;
  if ((e = make_pack(cams, n_cams, opts, &cp)) != HGS_OK) return e;
  const int64_t n_rec = p.n * n_cams;
  if (!n_dup || (n_rec > 0 && (!records || !tiles_touched)))
    return fail(HGS_EINVAL, "an output pointer is null");
  const size_t need = hgs::preprocess_workspace_bytes(n_rec);
  if (no_alloc) {
    if (need > kNoAllocScratchBytes)
      return fail(HGS_ECAPACITY, "n_cams * n = %lld records exceed the no-alloc limit of %lld",
                  (long long)n_rec, (long long)kNoAllocMaxRecords);
    if ((e = scratch_address(&workspace)) != HGS_OK) return e;
    workspace_bytes = kNoAllocScratchBytes;
  }
  if (!workspace || workspace_bytes < need)
    return fail(HGS_ECAPACITY, "workspace too small: need %zu bytes", need);
  const hgs::Opts o = hgs::to_opts(*opts);
  const hipError_t h = hgs::launch_preprocess(p, cp, o, (hgs::Record*)records, tiles_touched, offsets, n_dup,
                                              workspace, stream);
  if (h != hipSuccess) return hip_fail(h, "preprocess launch");
  return HGS_OK;
}

}  // namespace

extern "C" {

void hgs_default_options(hgs_options* o) {
  if (!o) return;
  o->tile = 16;
  o->batch = 256;
  o->lowpass = 0.3f;
  o->kappa = 3.0f;
  o->alpha_min = 1.0f / 255.0f;
  o->alpha_max = 0.99f;
  o->t_min = 1e-4f;
  o->fov_clamp = 1.3f;
  o->bg[0] = o->bg[1] = o->bg[2] = 0.0f;
  o->flags = 0u;
}

int64_t hgs_tiles_total(const hgs_camera* cams, int32_t n_cams, const hgs_options* opts) {
  if (check_opts(opts) != HGS_OK) return -1;
  hgs::CamPack cp;
  if (make_pack(cams, n_cams, opts, &cp) != HGS_OK) return -1;
  return (int64_t)cp.tiles_total;
}

int64_t hgs_pixels_total(const hgs_camera* cams, int32_t n_cams) {
  if (!cams || n_cams < 1) return -1;
  int64_t t = 0;
  for (int c = 0; c < n_cams; ++c) t += (int64_t)cams[c].width * cams[c].height;
  return t;
}

size_t hgs_workspace_bytes(int32_t which, int64_t n_rec, const hgs_camera* cams, int32_t n_cams,
                           const hgs_options* opts, int64_t capacity) {
  if (n_rec < 0) return 0;
  switch (which) {
    case HGS_WS_PREPROCESS:
      return hgs::preprocess_workspace_bytes(n_rec);
    case HGS_WS_BIN_SORT: {
      if (check_opts(opts) != HGS_OK || capacity < 0) return 0;
      hgs::CamPack cp;
      if (make_pack(cams, n_cams, opts, &cp) != HGS_OK) return 0;
      return hgs::sort_workspace_bytes(n_rec, capacity, cp,
                                       (opts->flags & HGS_FLAG_SORT_FULL_KEYS) != 0);
    }
    case HGS_WS_RENDER:
      if (check_opts(opts) != HGS_OK) return 0;
      return hgs::render_workspace_bytes(opts->tile, capacity);
    default:
      return 0;
  }
}

int hgs_preprocess(const hgs_params* params, const hgs_camera* cams, int32_t n_cams,
                   const hgs_options* opts, void* records, uint32_t* tiles_touched,
                   uint64_t* offsets, uint64_t* n_dup, void* workspace, size_t workspace_bytes,
                   hipStream_t stream) {
  return preprocess_impl(params, cams, n_cams, opts, records, tiles_touched, offsets, n_dup, workspace,
                         workspace_bytes, false, stream);
}

int hgs_preprocess_noalloc(const hgs_params* params, const hgs_camera* cams, int32_t n_cams,
                           const hgs_options* opts, void* records, uint32_t* tiles_touched,
                           uint64_t* offsets, uint64_t* n_dup, hipStream_t stream) {
  return preprocess_impl(params, cams, n_cams, opts, records, tiles_touched, offsets, n_dup, nullptr, 0, true,
                         stream);
}

int hgs_bin_sort(const void* records, const uint32_t* tiles_touched, const uint64_t* offsets,
                 const uint64_t* n_dup, int64_t n_rec, const hgs_camera* cams, int32_t n_cams,
                 const hgs_options* opts, uint64_t* keys, uint32_t* values, int64_t capacity,
                 uint32_t* ranges, uint32_t* tile_order, int32_t* overflow, void* workspace,
                 size_t workspace_bytes, hipStream_t stream) {
  int e;
  if ((e = check_opts(opts)) != HGS_OK) return e;
  hgs::CamPack cp;
  if ((e = make_pack(cams, n_cams, opts, &cp)) != HGS_OK) return e;
  if (n_rec < 0 || n_rec % n_cams != 0) return fail(HGS_EINVAL, "n_rec must be n_cams * n");
  if (capacity < 0 || capacity >= (int64_t)UINT32_MAX) return fail(HGS_EINVAL, "capacity out of range");
  const bool full_keys = (opts->flags & HGS_FLAG_SORT_FULL_KEYS) != 0;
  if (!n_dup || !ranges || !overflow || (n_rec > 0 && (!records || !tiles_touched || (full_keys && !offsets))) ||
      (capacity > 0 && (!values || (full_keys && !keys))))
    return fail(HGS_EINVAL, "a pointer is null");
  const size_t need = hgs::sort_workspace_bytes(n_rec, capacity, cp, full_keys);
  if (!workspace || workspace_bytes < need)
    return fail(HGS_ECAPACITY, "workspace too small: need %zu bytes", need);
  if (((uintptr_t)workspace & 255u) != 0)
    return fail(HGS_EINVAL, "workspace must be 256-byte aligned");
  hipError_t h = hgs::launch_bin_sort((const hgs::Record*)records, tiles_touched, offsets, n_dup,
                                      n_rec, n_rec / n_cams, cp, keys, values, capacity, ranges,
                                      tile_order, overflow, workspace, full_keys, stream);
  if (h != hipSuccess) return hip_fail(h, "bin_sort launch");
  return HGS_OK;
}

int hgs_render_fwd(const void* records, const uint32_t* values, const uint32_t* ranges,
                   const uint32_t* tile_order, const hgs_camera* cams, int32_t n_cams,
                   const hgs_options* opts, float* images,
                   float* T_final, int32_t* last_idx, int32_t* n_contrib, float* depth, void* workspace,
                   size_t workspace_bytes, hipStream_t stream) {
  int e;
  if ((e = check_opts(opts)) != HGS_OK) return e;
  hgs::CamPack cp;
  if ((e = make_pack(cams, n_cams, opts, &cp)) != HGS_OK) return e;
  if (!ranges || !images || !T_final || !last_idx || !n_contrib)
    return fail(HGS_EINVAL, "a pointer is null");
  if (!workspace || workspace_bytes < hgs::render_workspace_bytes())
    return fail(HGS_ECAPACITY, "workspace too small");
  const hgs::Opts o = hgs::to_opts(*opts);
  hipError_t h = hgs::launch_render_fwd((const hgs::Record*)records, values, ranges, tile_order, cp, o,
                                        images, T_final, last_idx, n_contrib, depth, workspace, workspace_bytes,
                                        stream);
  if (h != hipSuccess) return hip_fail(h, "render_fwd launch");
  return HGS_OK;
}

int hgs_depth_normals(const float* depth, const float* T_final, const hgs_camera* cams, int32_t n_cams,
                      float* normals, hipStream_t stream) {
  if (!depth || !T_final || !normals) return fail(HGS_EINVAL, "a pointer is null");
  hgs_options o;
  hgs_default_options(&o);
  hgs::CamPack cp;
  int e;
  if ((e = make_pack(cams, n_cams, &o, &cp)) != HGS_OK) return e;
  const int64_t n_pix = hgs_pixels_total(cams, n_cams);
  hipError_t h = hgs::launch_depth_normals(depth, T_final, cp, (uint64_t)n_pix, normals, stream);
  if (h != hipSuccess) return hip_fail(h, "depth_normals launch");
  return HGS_OK;
}

int hgs_raster_bwd(const void* records, const uint32_t* values, const uint32_t* ranges,
                   const uint32_t* tile_order, const hgs_camera* cams, int32_t n_cams,
                   const hgs_options* opts, const float* T_final, const int32_t* last_idx,
                   const float* dL_dimages, float* record_grads, void* workspace,
                   size_t workspace_bytes, hipStream_t stream) {
  int e;
  if ((e = check_opts(opts)) != HGS_OK) return e;
  hgs::CamPack cp;
  if ((e = make_pack(cams, n_cams, opts, &cp)) != HGS_OK) return e;
  if (!ranges || !T_final || !last_idx || !dL_dimages || !record_grads)
    return fail(HGS_EINVAL, "a pointer is null");
  if (!workspace || workspace_bytes < hgs::render_workspace_bytes())
    return fail(HGS_ECAPACITY, "workspace too small");
  const hgs::Opts o = hgs::to_opts(*opts);
  hipError_t h = hgs::launch_render_bwd((const hgs::Record*)records, values, ranges, tile_order, cp, o,
                                        T_final, last_idx, dL_dimages, record_grads, workspace, workspace_bytes,
                                        stream);
  if (h != hipSuccess) return hip_fail(h, "raster_bwd launch");
  return HGS_OK;
}

int hgs_preprocess_bwd(const hgs_params* params, const hgs_camera* cams, int32_t n_cams,
                       const hgs_options* opts, const void* records, float* record_grads,
                       const hgs_param_grads* grads, hipStream_t stream) {
  int e;
  if ((e = check_opts(opts)) != HGS_OK) return e;
  hgs::Params p;
  if ((e = make_params(params, &p)) != HGS_OK) return e;
  hgs::CamPack cp;
  if ((e = make_pack(cams, n_cams, opts, &cp)) != HGS_OK) return e;
  if (!grads) return fail(HGS_EINVAL, "grads is null");
  if (p.n > 0 && (!records || !record_grads || !grads->means || !grads->scales || !grads->quats ||
                  !grads->normals || !grads->opac1 || !grads->opac2 || !grads->sh))
    return fail(HGS_EINVAL, "a pointer is null");
  const hgs::Opts o = hgs::to_opts(*opts);
  hgs::Grads g{grads->means, grads->scales, grads->quats, grads->normals,
               grads->opac1, grads->opac2,  grads->sh};
  hipError_t h = hgs::launch_preprocess_bwd(p, cp, o, record_grads, g, stream);
  if (h != hipSuccess) return hip_fail(h, "preprocess_bwd launch");
  return HGS_OK;
}

int hgs_render_bwd(const hgs_params* params, const hgs_camera* cams, int32_t n_cams,
                   const hgs_options* opts, const void* records, const uint32_t* values,
                   const uint32_t* ranges, const uint32_t* tile_order, const float* T_final,
                   const int32_t* last_idx,
                   const float* dL_dimages, float* record_grads, const hgs_param_grads* grads,
                   void* workspace, size_t workspace_bytes, hipStream_t stream) {
  int e;
  if ((e = check_opts(opts)) != HGS_OK) return e;
  hgs::Params p;
  if ((e = make_params(params, &p)) != HGS_OK) return e;
  hgs::CamPack cp;
  if ((e = make_pack(cams, n_cams, opts, &cp)) != HGS_OK) return e;
  if (!workspace || workspace_bytes < hgs::render_workspace_bytes())
    return fail(HGS_ECAPACITY, "workspace too small");
  if (p.n > 0 && !record_grads) return fail(HGS_EINVAL, "record_grads is null");
  hipError_t h = hgs::launch_zero_f32(record_grads, p.n * n_cams * HGS_RECORD_GRAD_FLOATS, stream);
  if (h != hipSuccess) return hip_fail(h, "clear launch");
  if ((e = hgs_raster_bwd(records, values, ranges, tile_order, cams, n_cams, opts, T_final, last_idx,
                          dL_dimages, record_grads, workspace, workspace_bytes, stream)) != HGS_OK)
    return e;
  return hgs_preprocess_bwd(params, cams, n_cams, opts, records, record_grads, grads, stream);
}

int hgs_mip_filter3d(const float* means, int64_t n, int64_t stride, const hgs_camera* cams, int32_t n_cams,
                     float s, float margin, float* filter3d, void* workspace, hipStream_t stream) {
  int e;
  hgs_options o;
  hgs_default_options(&o);
  hgs::CamPack cp;
  if ((e = make_pack(cams, n_cams, &o, &cp)) != HGS_OK) return e;
  if (n < 0 || stride < n) return fail(HGS_EINVAL, "need 0 <= n <= stride");
  if (!(s >= 0.0f) || !(margin >= 0.0f)) return fail(HGS_EINVAL, "s and margin must be >= 0");
  if (n == 0) return HGS_OK;
  if (!means || !filter3d || !workspace) return fail(HGS_EINVAL, "a pointer is null");
  const hipError_t h = hgs::launch_mip_filter3d(means, n, stride, cp, (double)s, (double)margin, filter3d,
                                                (uint32_t*)workspace, stream);
  if (h != hipSuccess) return hip_fail(h, "mip_filter3d launch");
  return HGS_OK;
}

int hgs_l1_loss_grad(const float* images, const float* target, int64_t n, float scale, float* dL_dimages,
                     float* loss, hipStream_t stream) {
  if (n < 0) return fail(HGS_EINVAL, "n must be >= 0");
  if (n == 0) return HGS_OK;
  if (!images || !target || !dL_dimages) return fail(HGS_EINVAL, "a pointer is null");
  const hipError_t h = hgs::launch_l1_grad(images, target, n, scale, dL_dimages, loss, stream);
  if (h != hipSuccess) return hip_fail(h, "l1 gradient launch");
  return HGS_OK;
}

int hgs_adam_schedule(int32_t step, float extent, float normal_lr, hgs_adam_config* cfg) {
  if (!cfg) return fail(HGS_EINVAL, "cfg is null");
  if (step < 1) return fail(HGS_EINVAL, "step must be >= 1");
  if (!(extent > 0.0f)) return fail(HGS_EINVAL, "extent must be > 0");
  const double r = step >= 30000 ? 1.0 : (double)step / 30000.0;
  const double lr0 = 1.6e-4 * (double)extent, lr1 = 1.6e-6 * (double)extent;
  const double decay = pow(1.4, -(double)(step / 5000));
  cfg->lr_means = (float)exp((1.0 - r) * log(lr0) + r * log(lr1));
  cfg->lr_scales = 0.005f;
  cfg->lr_quats = 0.001f;
  cfg->lr_normals = (float)((double)normal_lr * decay);
  cfg->lr_opacity = (float)(0.05 * decay);
  cfg->lr_sh_dc = 0.0025f;
  cfg->lr_sh_rest = (float)(0.0025 / 20.0);
  cfg->beta1 = 0.9f;
  cfg->beta2 = 0.999f;
  cfg->eps = 1e-15f;
  cfg->step = step;
  cfg->reserved = 0;
  return HGS_OK;
}

int hgs_adam_step(const hgs_adam_config* cfg, int64_t n, int64_t stride, int32_t sh_degree,
                  const hgs_param_grads* raw, const hgs_param_grads* grads, const hgs_param_grads* m,
                  const hgs_param_grads* v, const hgs_param_grads* act, hipStream_t stream) {
  int e;
  if (!cfg) return fail(HGS_EINVAL, "cfg is null");
  if (cfg->step < 1) return fail(HGS_EINVAL, "step must be >= 1");
  if ((e = check_sizes(n, stride, sh_degree)) != HGS_OK) return e;
  if (n == 0) return HGS_OK;
  if ((e = planes_ok(raw, "raw")) != HGS_OK || (e = planes_ok(grads, "grads")) != HGS_OK ||
      (e = planes_ok(m, "m")) != HGS_OK || (e = planes_ok(v, "v")) != HGS_OK ||
      (e = planes_ok(act, "act")) != HGS_OK)
    return e;
  hgs::AdamPlan plan{};
  const double c1 = 1.0 - pow((double)cfg->beta1, (double)cfg->step);
  const double c2 = 1.0 - pow((double)cfg->beta2, (double)cfg->step);
  const float lrs[8] = {cfg->lr_means, cfg->lr_scales, cfg->lr_quats, cfg->lr_normals,
                        cfg->lr_opacity, cfg->lr_opacity, cfg->lr_sh_dc, cfg->lr_sh_rest};
  for (int k = 0; k < 8; ++k) plan.step_size[k] = (float)((double)lrs[k] / c1);
  plan.beta1 = cfg->beta1;
  plan.beta2 = cfg->beta2;
  plan.inv_sqrt_bc2 = (float)(1.0 / sqrt(c2));
  plan.eps = cfg->eps;
  const float* gp[7] = {grads->means, grads->scales, grads->quats, grads->normals,
                        grads->opac1, grads->opac2, grads->sh};
  bool vec = stride % 4 == 0;
  const hgs_param_grads* sets[5] = {raw, m, v, act, grads};
  for (const hgs_param_grads* g : sets)
    vec = vec && aligned16(g->means) && aligned16(g->scales) && aligned16(g->quats) && aligned16(g->normals) &&
          aligned16(g->opac1) && aligned16(g->opac2) && aligned16(g->sh);
  plan.vec4 = vec ? 1 : 0;
  const hipError_t h = hgs::launch_adam(to_grads(*raw), gp, to_grads(*m), to_grads(*v), to_grads(*act), n, stride,
                                        sh_degree, plan, stream);
  if (h != hipSuccess) return hip_fail(h, "adam launch");
  return HGS_OK;
}

int hgs_activate(int64_t n, int64_t stride, int32_t sh_degree, const hgs_param_grads* raw,
                 const hgs_param_grads* act, hipStream_t stream) {
  int e;
  if ((e = check_sizes(n, stride, sh_degree)) != HGS_OK) return e;
  if (n == 0) return HGS_OK;
  if ((e = planes_ok(raw, "raw")) != HGS_OK || (e = planes_ok(act, "act")) != HGS_OK) return e;
  const hipError_t h = hgs::launch_activate(to_grads(*raw), to_grads(*act), n, stride, sh_degree, stream);
  if (h != hipSuccess) return hip_fail(h, "activate launch");
  return HGS_OK;
}

int hgs_densify_stats(const void* records, const float* record_grads, const hgs_camera* cams, int32_t n_cams,
                      const hgs_options* opts, int64_t n, float* grad_accum, int32_t* grad_count,
                      float* max_radii, hipStream_t stream) {
  int e;
  if ((e = check_opts(opts)) != HGS_OK) return e;
  hgs::CamPack cp;
  if ((e = make_pack(cams, n_cams, opts, &cp)) != HGS_OK) return e;
  if (n < 0) return fail(HGS_EINVAL, "n must be >= 0");
  if (n > (int64_t)INT32_MAX / HGS_MAX_CAMERAS) return fail(HGS_EINVAL, "n too large");
  if (n == 0) return HGS_OK;
  if (!records || !record_grads || !grad_accum || !grad_count || !max_radii)
    return fail(HGS_EINVAL, "a pointer is null");
  const hipError_t h = hgs::launch_densify_stats((const hgs::Record*)records, record_grads, cp, n,
                                                 (double)opts->kappa, grad_accum, grad_count, max_radii, stream);
  if (h != hipSuccess) return hip_fail(h, "densify_stats launch");
  return HGS_OK;
}

void hgs_densify_default(float extent, hgs_densify_config* cfg) {
  if (!cfg) return;
  cfg->extent = extent;
  cfg->grad_threshold = 0.0002f;
  cfg->percent_dense = 0.01f;
  cfg->min_opacity = 0.01f;
  cfg->max_screen_radius = 0.0f;
  cfg->max_world_scale = 0.0f;
}

size_t hgs_densify_workspace_bytes(int64_t n) { return n < 0 ? 0 : hgs::densify_workspace_bytes(n); }

int hgs_densify(const hgs_densify_config* cfg, int64_t n, int64_t stride, int32_t sh_degree,
                const hgs_param_grads* raw, const hgs_param_grads* m, const hgs_param_grads* v,
                const float* grad_accum, const int32_t* grad_count, const float* max_radii, const float* samples,
                int64_t capacity, int64_t stride_out, const hgs_param_grads* raw_out,
                const hgs_param_grads* m_out, const hgs_param_grads* v_out, int64_t* n_out, int32_t* overflow,
                void* workspace, size_t workspace_bytes, hipStream_t stream) {
  int e;
  if (!cfg) return fail(HGS_EINVAL, "cfg is null");
  if ((e = check_sizes(n, stride, sh_degree)) != HGS_OK) return e;
  if (capacity < 0 || stride_out < capacity) return fail(HGS_EINVAL, "need 0 <= capacity <= stride_out");
  if (n > (int64_t)UINT32_MAX) return fail(HGS_EINVAL, "n too large");
  if (!(cfg->extent > 0.0f) || !(cfg->percent_dense > 0.0f) || !(cfg->min_opacity > 0.0f) ||
      !(cfg->min_opacity < 1.0f) || !(cfg->grad_threshold >= 0.0f) || !(cfg->max_screen_radius >= 0.0f) ||
      !(cfg->max_world_scale >= 0.0f))
    return fail(HGS_EINVAL, "densify threshold out of range");
  if (!n_out || !overflow) return fail(HGS_EINVAL, "n_out or overflow is null");
  if ((e = planes_ok(raw, "raw")) != HGS_OK || (e = planes_ok(m, "m")) != HGS_OK ||
      (e = planes_ok(v, "v")) != HGS_OK || (e = planes_ok(raw_out, "raw_out")) != HGS_OK ||
      (e = planes_ok(m_out, "m_out")) != HGS_OK || (e = planes_ok(v_out, "v_out")) != HGS_OK)
    return e;
  if (n > 0 && (!grad_accum || !grad_count || !max_radii || !samples)) return fail(HGS_EINVAL, "a pointer is null");
  if (!workspace || workspace_bytes < hgs::densify_workspace_bytes(n))
    return fail(HGS_ECAPACITY, "workspace too small");
  hgs::DensifyPlan dp{};
  const double ext = (double)cfg->extent, mo = (double)cfg->min_opacity;
  dp.grad_threshold = (double)cfg->grad_threshold;
  dp.log_dense = log((double)cfg->percent_dense * ext);
  dp.logit_min_opacity = log(mo / (1.0 - mo));
  dp.world_on = cfg->max_world_scale > 0.0f ? 1 : 0;
  dp.log_world = dp.world_on ? log((double)cfg->max_world_scale * ext) : 0.0;
  dp.screen_on = cfg->max_screen_radius > 0.0f ? 1 : 0;
  dp.max_screen = (double)cfg->max_screen_radius;
  dp.shrink = (float)log(0.8 * 2.0);
  const hipError_t h = hgs::launch_densify(to_grads(*raw), to_grads(*m), to_grads(*v), n, stride, sh_degree, dp,
                                           grad_accum, grad_count, max_radii, samples, capacity, stride_out,
                                           to_grads(*raw_out), to_grads(*m_out), to_grads(*v_out), n_out,
                                           overflow, workspace, stream);
  if (h != hipSuccess) return hip_fail(h, "densify launch");
  return HGS_OK;
}

int hgs_reset_opacity(float value, int64_t n, const hgs_param_grads* raw, const hgs_param_grads* m,
                      const hgs_param_grads* v, const hgs_param_grads* act, hipStream_t stream) {
  if (!(value > 0.0f) || !(value < 1.0f)) return fail(HGS_EINVAL, "value must be in (0, 1)");
  if (n < 0) return fail(HGS_EINVAL, "n must be >= 0");
  if (n == 0) return HGS_OK;
  if (!raw || !m || !v || !raw->opac1 || !raw->opac2 || !m->opac1 || !m->opac2 || !v->opac1 || !v->opac2)
    return fail(HGS_EINVAL, "an opacity plane pointer is null");
  if (act && (!act->opac1 || !act->opac2)) return fail(HGS_EINVAL, "act opacity plane is null");
  const hgs_param_grads none{};
  const double vv = (double)value;
  const float cap = (float)log(vv / (1.0 - vv));
  const hipError_t h = hgs::launch_reset_opacity(to_grads(*raw), to_grads(*m), to_grads(*v),
                                                 to_grads(act ? *act : none), n, cap, stream);
  if (h != hipSuccess) return hip_fail(h, "reset_opacity launch");
  return HGS_OK;
}

const char* hgs_strerror(int code) {
  switch (code) {
    case HGS_OK: return "ok";
    case HGS_EINVAL: return "invalid argument";
    case HGS_ECAPACITY: return "buffer too small";
    case HGS_EHIP: return "HIP runtime error";
    default: return "unknown error";
  }
}

const char* hgs_last_error(void) { return g_err; }

}  // extern "C"
