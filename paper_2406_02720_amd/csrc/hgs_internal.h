// Internal definitions shared by the HIP translation units of libhgs.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "hgs.h"

namespace hgs {

// Camera as the kernels see it: the public camera plus the derived tile grid
// and the offsets of its tiles and pixels in the global numbering.
struct CamDev {
  float R[9];
  float t[3];
  float fx, fy, cx, cy;
  float znear;
  int32_t width, height;
  int32_t tiles_x, tiles_y;
  uint32_t tile_off;
  uint32_t pad0;
  uint64_t pix_off;
};

// Passed by value as a kernel argument (under the 4 KiB limit), so a launch
// captures the cameras without any host->device copy.
struct CamPack {
  int32_t n_cams;
  int32_t tile;       // tile edge (8, 16 or 32)
  int32_t tile_shift; // log2(tile)
  uint32_t tiles_total;
  CamDev cam[HGS_MAX_CAMERAS];
};

// Projected record, 64 bytes = 4 x 16 bytes so that one record moves with
// four dwordx4 loads and stages in LDS as four 16-byte slots.
//   q0: centre relative to the pixel-rect corner (x0, y0), half-factor vector
//   q1: conic (a, b, c) of the dilated screen covariance, alpha2
//   q2: colour, (alpha1 - alpha2) / 2
//   q3: rect x0 | x1 << 16, rect y0 | y1 << 16, fp32 depth bits, tiles
struct alignas(16) Record {
  float mx, my, kx, ky;
  float qa, qb, qc, alpha2;
  float r, g, b, d_o;
  uint32_t xr, yr, depth, tiles;
};
static_assert(sizeof(Record) == HGS_RECORD_BYTES, "record layout");
// explicit arguments beside the pack and the implicit ones stay under 4 KiB
static_assert(sizeof(CamPack) <= 3584, "camera pack must fit the kernel-argument segment");

struct Opts {
  float lowpass, kappa, alpha_min, alpha_max, t_min, fov_clamp;
  float bg[3];
  uint32_t flags;
  int32_t tile, batch;
};

inline Opts to_opts(const hgs_options& o) {
  Opts r;
  r.lowpass = o.lowpass;
  r.kappa = o.kappa;
  r.alpha_min = o.alpha_min;
  r.alpha_max = o.alpha_max;
  r.t_min = o.t_min;
  r.fov_clamp = o.fov_clamp;
  r.bg[0] = o.bg[0];
  r.bg[1] = o.bg[1];
  r.bg[2] = o.bg[2];
  r.flags = o.flags;
  r.tile = o.tile;
  r.batch = o.batch;
  return r;
}

struct Params {
  const float* means;
  const float* scales;
  const float* quats;
  const float* normals;
  const float* opac1;
  const float* opac2;
  const float* sh;
  const float* filter3d;  // may be null
  int64_t n;
  int64_t stride;
  int32_t sh_degree;
};

struct Grads {
  float* means;
  float* scales;
  float* quats;
  float* normals;
  float* opac1;
  float* opac2;
  float* sh;
};

// Host-prepared constants of one Adam step: per learning-rate group (means,
// scales, quats, normals, opac1, opac2, SH degree 0, SH higher) the step
// size lr / (1 - beta1^t); 1 / sqrt(1 - beta2^t).
struct AdamPlan {
  float step_size[8];
  float beta1, beta2, inv_sqrt_bc2, eps;
  int32_t vec4;   // every plane 16-byte aligned with stride % 4 == 0
};

// Densify thresholds in the raw domain, FP64 (see hgs_densify).
struct DensifyPlan {
  double grad_threshold;     // average NDC gradient threshold
  double log_dense;          // log(percent_dense * extent)
  double logit_min_opacity;  // logit(min_opacity)
  double log_world;          // log(max_world_scale * extent)
  double max_screen;         // screen radius limit, px
  int32_t world_on, screen_on;
  float shrink;              // log(0.8 * 2), float32
};

// Camera of a global tile id (cameras are few: linear scan).
__device__ inline int cam_of_tile(const CamPack& cp, uint32_t tile) {
  int c = 0;
  for (int i = 1; i < cp.n_cams; ++i)
    if (tile >= cp.cam[i].tile_off) c = i;
  return c;
}

// ---------------------------------------------------------------------------
// host-side launch helpers (defined in the .hip files)
// ---------------------------------------------------------------------------
// projection of every (camera, kernel) pair, then the entry total (and, with
// offsets, the exclusive scan of the tiles touched)
hipError_t launch_preprocess(const Params& p, const CamPack& cp, const Opts& o, Record* rec,
                             uint32_t* tiles, uint64_t* offsets, uint64_t* total, void* ws, hipStream_t s);
// records per uint64 partial sum of the entry-count scan, and kernels per
// partial of the projection's own total (the preprocess workspace holds
// whichever is larger)
constexpr int64_t kScanRecordsPerPartial = 1024;
constexpr int64_t kPreprocessRecordsPerPartial = 256;
size_t scan_workspace_bytes(int64_t n);
size_t preprocess_workspace_bytes(int64_t n_rec);
hipError_t launch_scan(const uint32_t* tiles, int64_t n, uint64_t* offsets, uint64_t* total,
                       void* ws, hipStream_t s);
int tile_bits(uint32_t tiles_total);
size_t sort_workspace_bytes(int64_t n_rec, int64_t capacity, const CamPack& cp, bool full_keys);
hipError_t launch_bin_sort(const Record* rec, const uint32_t* tiles, const uint64_t* offsets,
                           const uint64_t* n_dup, int64_t n_rec, int64_t n_per_cam,
                           const CamPack& cp, uint64_t* keys, uint32_t* vals, int64_t capacity,
                           uint32_t* ranges, uint32_t* tile_order, int32_t* overflow, void* ws,
                           bool full_keys, hipStream_t s);
// the fixed head of the render workspace (work counters, mark tag), and the
// whole workspace with strip-mark planes for lists of up to `capacity`
// entries (tile: the tile size)
size_t render_workspace_bytes();
size_t render_workspace_bytes(int tile, int64_t capacity);
// tile_order non-null selects the persistent raster (workspace holds its
// work counters: [0] forward, [1] backward); the forward pass writes the
// strip marks that fit in ws_bytes, the backward pass reads them
hipError_t launch_render_fwd(const Record* rec, const uint32_t* vals, const uint32_t* ranges,
                             const uint32_t* tile_order, const CamPack& cp, const Opts& o,
                             float* img, float* T_final, int32_t* last_idx, int32_t* n_contrib,
                             float* depth, void* ws, size_t ws_bytes, hipStream_t s);
hipError_t launch_depth_normals(const float* depth, const float* T_final, const CamPack& cp, uint64_t n_pix,
                                float* normals, hipStream_t s);
hipError_t launch_zero_f32(float* p, int64_t n, hipStream_t s);
hipError_t launch_render_bwd(const Record* rec, const uint32_t* vals, const uint32_t* ranges,
                             const uint32_t* tile_order, const CamPack& cp, const Opts& o,
                             const float* T_final, const int32_t* last_idx, const float* dL_dimg,
                             float* rec_grads, void* ws, size_t ws_bytes, hipStream_t s);
hipError_t launch_mip_filter3d(const float* means, int64_t n, int64_t stride, const CamPack& cp, double s,
                               double margin, float* out, uint32_t* scratch, hipStream_t st);
int planes_of(int sh_degree);
hipError_t launch_adam(const Grads& raw, const float* const grad[7], const Grads& m, const Grads& v,
                       const Grads& act, int64_t n, int64_t stride, int sh_degree, const AdamPlan& plan,
                       hipStream_t s);
hipError_t launch_activate(const Grads& raw, const Grads& act, int64_t n, int64_t stride, int sh_degree,
                           hipStream_t s);
hipError_t launch_reset_opacity(const Grads& raw, const Grads& m, const Grads& v, const Grads& act, int64_t n,
                                float cap, hipStream_t s);
hipError_t launch_densify_stats(const Record* rec, const float* rgrad, const CamPack& cp, int64_t n, double kappa,
                                float* accum, int32_t* count, float* max_radii, hipStream_t s);
hipError_t launch_l1_grad(const float* img, const float* tgt, int64_t n, float scale, float* dL, float* loss,
                          hipStream_t s);
size_t densify_workspace_bytes(int64_t n);
hipError_t launch_densify(const Grads& raw, const Grads& m, const Grads& v, int64_t n, int64_t stride,
                          int sh_degree, const DensifyPlan& dp, const float* accum, const int32_t* count,
                          const float* max_radii, const float* samples, int64_t capacity, int64_t stride_out,
                          const Grads& raw_out, const Grads& m_out, const Grads& v_out, int64_t* n_out,
                          int32_t* overflow, void* ws, hipStream_t s);
hipError_t launch_preprocess_bwd(const Params& p, const CamPack& cp, const Opts& o, float* rec_grads,
                                 const Grads& g, hipStream_t s);

}  // namespace hgs
