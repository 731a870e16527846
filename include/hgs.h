/*
 * hgs.h -- C ABI of the MI355X tile rasterizer for 3D half-Gaussian splatting.
 *
 * The library renders scenes of half-Gaussian kernels (3D-HGS): every kernel
 * is a 3-D Gaussian (centre, scales, rotation; Eq. 1-2 of the paper) split by
 * a plane through its centre with unit normal n, the half on the +n side
 * carrying opacity alpha1 and the other half alpha2 (Sec. 3.2).  A pixel
 * blends the kernels that cover it front to back with the paired-half
 * opacity of Eq. 10 (Sec. 3.3).  The valid screen region of each kernel is
 * the half-aware box of Sec. 3.4, built from the splitting ellipse of Alg. 1
 * (Supp. B.1).
 *
 * Pipeline (each call only enqueues work on `stream`; nothing blocks):
 *   hgs_preprocess  projection, half factor, valid region, SH colour, depth,
 *                   tiles touched, their total (and exclusive scan)
 *   hgs_bin_sort    one (tile | depth, record) entry per covered tile in
 *                   key order (depth sort of the records, then placement
 *                   by counting), per-tile ranges
 *   hgs_render_fwd  per-pixel front-to-back blending
 *   hgs_render_bwd  per-pixel back-to-front replay, per-record gradients,
 *                   chain rule to every kernel parameter
 * Around it: blended depth (an hgs_render_fwd output) and depth-derived
 * normals (hgs_depth_normals); the training step after the backward pass
 * (hgs_l1_loss_grad, hgs_adam_step with hgs_adam_schedule, hgs_activate,
 * hgs_densify_stats, hgs_densify, hgs_reset_opacity); the Mip-Splatting-HGS
 * filters (hgs_params.filter3d from hgs_mip_filter3d, HGS_FLAG_MIP_2D).
 *
 * Conventions (the paper leaves them open):
 *   - camera axes x right, y down, z forward; pixel (i, j) has its centre at
 *     (i + 1/2, j + 1/2); records are sorted by camera-space z, ties by
 *     record id;
 *   - record id = camera * n + kernel; records of all cameras are stored
 *     camera-major, [n_cams][n] records of HGS_RECORD_BYTES each;
 *   - the low-pass `lowpass` (px^2) is added to the 2x2 screen covariance and
 *     the half factor is taken on that dilated covariance;
 *   - alpha = min(alpha_max, HG); a kernel with alpha < alpha_min is skipped;
 *     blending stops before the kernel that would take the transmittance
 *     below t_min.
 *
 * Memory: every pointer named "device" is device memory owned by the caller.
 * The library never allocates device memory, never synchronises the stream
 * and keeps no state between calls, so calls may be captured in a HIP graph.
 * Host pointers (cameras, options, parameter structs) are read during the
 * call only.
 *
 * Errors: every entry point returns HGS_OK (0) or a positive HGS_E* code,
 * never throws, and leaves a message for hgs_last_error() (thread local).
 */
#ifndef HGS_H
#define HGS_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

#define HGS_OK 0
#define HGS_EINVAL 1     /* an argument is out of range or a pointer is null */
#define HGS_ECAPACITY 2  /* a caller buffer is smaller than the call needs   */
#define HGS_EHIP 3       /* the HIP runtime reported an error                */

#define HGS_MAX_CAMERAS 32       /* cameras per call                           */
#define HGS_MAX_IMAGE_SIDE 16384 /* width and height limit                     */
#define HGS_RECORD_BYTES 64      /* one projected record                       */
#define HGS_RECORD_GRAD_FLOATS 12 /* per-record gradient accumulators          */

/* options.flags */
#define HGS_FLAG_FULL_BOX 1u     /* splat both halves with the full ellipse box,
                                    no half-aware region and no opacity cull  */
#define HGS_FLAG_SORT_FULL_KEYS 2u /* hgs_bin_sort: radix-sort the duplicated
                                    entries over all 32 + tile bits of their
                                    64-bit keys instead of placing them by
                                    counting after a depth sort of the
                                    records (same result)                     */
#define HGS_FLAG_MIP_2D 4u       /* the screen low-pass is Mip-Splatting's 2-D
                                    mip filter (lowpass ~0.1 px^2): both
                                    opacities times sqrt(det S / det(S +
                                    lowpass I)), S the undilated screen
                                    covariance (Mip-Splatting-HGS, Sec. 4)   */

/* Pinhole camera.  R is the world->camera rotation (row-major 3x3), t the
 * translation (x_cam = R x_world + t).  fx, fy, cx, cy in pixels (fx, fy
 * positive and finite).  Kernels with camera z <= znear are culled; znear
 * must be positive and finite (HGS_EINVAL otherwise). */
typedef struct hgs_camera {
  float R[9];
  float t[3];
  float fx, fy, cx, cy;
  int32_t width, height;
  float znear;
  int32_t reserved;
} hgs_camera;

/* Kernel parameters, structure of arrays, device pointers.  Plane p of a
 * field is at ptr + p * stride, kernel i at element i (stride >= n):
 *   means   3 planes  world centre
 *   scales  3 planes  activated axis lengths (> 0)
 *   quats   4 planes  rotation (w, x, y, z), any non-zero length; zero means
 *                     the identity
 *   normals 3 planes  splitting-plane normal, any length; zero means I = 1
 *   opac1   1 plane   opacity of the +normal half, activated, in [0, 1]
 *   opac2   1 plane   opacity of the -normal half
 *   sh      3 (D+1)^2 planes, plane (k * 3 + channel) holds coefficient k of
 *                     the real spherical harmonics of degree <= D (0..3)
 *   filter3d 1 plane (optional, NULL = none): variance f of Mip-Splatting's
 *                     3-D smoothing filter (Mip-Splatting-HGS, Sec. 4):
 *                     the covariance becomes Sigma + f I everywhere (half
 *                     factor and valid region included) and both opacities
 *                     are multiplied by sqrt(det Sigma / det(Sigma + f I));
 *                     see hgs_mip_filter3d.  Not differentiated.
 * A non-finite value in any of the fields above culls the kernel (as does a
 * non-finite colour). */
typedef struct hgs_params {
  const float* means;
  const float* scales;
  const float* quats;
  const float* normals;
  const float* opac1;
  const float* opac2;
  const float* sh;
  int64_t n;
  int64_t stride;
  int32_t sh_degree;
  int32_t reserved;
  const float* filter3d;
} hgs_params;

/* Gradients of the scalar loss with respect to every field of hgs_params,
 * same layout (device pointers, overwritten, not accumulated). */
typedef struct hgs_param_grads {
  float* means;
  float* scales;
  float* quats;
  float* normals;
  float* opac1;
  float* opac2;
  float* sh;
} hgs_param_grads;

/* Rasterizer options; hgs_default_options() fills the defaults given in
 * brackets.  tile: tile edge in pixels, 8, 16 or 32 [16].  batch: how many
 * entry ids of its tile list a raster wavefront fetches per round (batch / 64
 * per lane, one vector load each; the records themselves are read as
 * wave-uniform loads, not staged), 128, 256 or 512 [256].  Outputs do not
 * depend on tile or batch. */
typedef struct hgs_options {
  int32_t tile;
  int32_t batch;
  float lowpass;    /* [0.3]  px^2 added to the screen covariance            */
  float kappa;      /* [3]    sigma extent of the valid region               */
  float alpha_min;  /* [1/255]                                               */
  float alpha_max;  /* [0.99]                                                */
  float t_min;      /* [1e-4]                                                */
  float fov_clamp;  /* [1.3]  clamp of x/z, y/z in the Jacobian, in units of
                               the half field of view                        */
  float bg[3];      /* [0]    background colour                              */
  uint32_t flags;   /* [0]    HGS_FLAG_*                                     */
} hgs_options;

void hgs_default_options(hgs_options* opts);

/* Workspace sizes (bytes) of the calls that take one.  `which` is one of the
 * HGS_WS_* values; n_rec = n_cams * n; capacity = key capacity of
 * hgs_bin_sort.  Returns 0 for invalid arguments.  The hgs_bin_sort
 * workspace must be 256-byte aligned (any hipMalloc result is).
 * HGS_WS_RENDER: 256 bytes, plus room for the strip marks of lists of up to
 * `capacity` entries (one byte per entry and forward wavefront of a tile:
 * 4 at 32-pixel tiles, 1 otherwise); capacity 0 gives the 256 bytes without
 * marks.  Any size from 256 bytes on is valid: marks only make the backward
 * pass faster (see hgs_raster_bwd). */
#define HGS_WS_PREPROCESS 0
#define HGS_WS_BIN_SORT 1
#define HGS_WS_RENDER 2
size_t hgs_workspace_bytes(int32_t which, int64_t n_rec, const hgs_camera* cams, int32_t n_cams,
                           const hgs_options* opts, int64_t capacity);

/* Number of tiles over all cameras (tile ids are global: the tiles of
 * camera c follow those of cameras 0..c-1, row-major inside a camera). */
int64_t hgs_tiles_total(const hgs_camera* cams, int32_t n_cams, const hgs_options* opts);

/* Pixels over all cameras; camera c's per-pixel outputs start at the sum of
 * width * height of cameras 0..c-1. */
int64_t hgs_pixels_total(const hgs_camera* cams, int32_t n_cams);

/* Projection of every (camera, kernel) pair -- Eq. 2, Eq. 3, Eq. 6 (+ the
 * low-pass), the half factor of Eq. 7-8 in camera-space form, Alg. 1 and the
 * half-aware region of Sec. 3.4, SH colour and depth.  Geometry is computed
 * in FP64 and stored in FP32.
 *   records        device, [n_cams * n] records of HGS_RECORD_BYTES (out)
 *   tiles_touched  device, uint32 [n_cams * n], 0 for culled records (out)
 *   offsets        device, uint64 [n_cams * n], exclusive prefix sum of
 *                  tiles_touched (out); may be NULL (then only n_dup is
 *                  computed): hgs_bin_sort needs it only with
 *                  HGS_FLAG_SORT_FULL_KEYS
 *   n_dup          device, uint64 [1], sum of tiles_touched (out)
 *   workspace      device, hgs_workspace_bytes(HGS_WS_PREPROCESS, ...) bytes
 * Errors: HGS_EINVAL for null pointers, n < 0, stride < n, sh_degree not in
 * 0..3, n_cams not in 1..HGS_MAX_CAMERAS, image sides not in
 * 1..HGS_MAX_IMAGE_SIDE, invalid tile or batch; HGS_ECAPACITY if
 * workspace_bytes is too small; HGS_EHIP on a launch failure. */
int hgs_preprocess(const hgs_params* params, const hgs_camera* cams, int32_t n_cams,
                   const hgs_options* opts, void* records, uint32_t* tiles_touched,
                   uint64_t* offsets, uint64_t* n_dup, void* workspace, size_t workspace_bytes,
                   hipStream_t stream);

/* hgs_preprocess for callers that cannot allocate device memory at all (code
 * under HIP graph capture that must not add allocations, tight serving loops,
 * harnesses that forbid hipMalloc): the same computation and outputs, with no
 * workspace argument.  The entry count keeps its partial sums in a device
 * array inside the library (4 MiB per device, held from the first call on
 * that device until the process ends), which limits n_cams * n to
 * HGS_NOALLOC_MAX_RECORDS; larger calls return HGS_ECAPACITY before any work
 * is enqueued.  Uses the array of the current device: `stream` must belong to
 * it.  Every call on a device shares that device's array, so calls that
 * overlap on one device (other streams, other threads) race: serialise them.
 * Calls no hipMalloc, hipFree or allocating library routine.  Errors as
 * hgs_preprocess, plus HGS_EHIP if the array's address cannot be obtained. */
#define HGS_NOALLOC_MAX_RECORDS 134217728ll
int hgs_preprocess_noalloc(const hgs_params* params, const hgs_camera* cams, int32_t n_cams,
                           const hgs_options* opts, void* records, uint32_t* tiles_touched,
                           uint64_t* offsets, uint64_t* n_dup, hipStream_t stream);

/* The tile lists of the tile-based rasterizer (Sec. 3.1, built as in 3D-GS):
 * one (tile, record) entry per tile of every record's tile rectangle, in the
 * order of the key (global tile << 32 | fp32 depth bits), ties by record id,
 * and the [start, end) range of every tile.  By default the records are
 * radix-sorted by (depth, id) and each entry is then written straight to its
 * final position (per-tile counts over blocks of depth-ordered records,
 * their scans, then cursors that hand out each tile's positions in record
 * order); HGS_FLAG_SORT_FULL_KEYS duplicates the 64-bit keys and radix-sorts
 * them over all bits.  Both give the same entries, ranges and order.
 *   records, tiles_touched, offsets, n_dup   from hgs_preprocess (device);
 *                  offsets may be NULL unless HGS_FLAG_SORT_FULL_KEYS is set
 *   n_rec          n_cams * n
 *   keys, values   device, `capacity` entries each (out: sorted entries in
 *                  the first *n_dup positions); keys may be NULL unless
 *                  HGS_FLAG_SORT_FULL_KEYS is set (the raster needs only the
 *                  values and ranges; by default keys, when given, are
 *                  written from the ranges after placement)
 *   ranges         device, uint32 [tiles_total][2] (out); a tile without
 *                  entries gets [0, 0)
 *   tile_order     device, uint32 [tiles_total] (out), may be NULL: the tile
 *                  ids, longest lists first, the order in which the
 *                  persistent raster takes tiles: ascending key
 *                  255 - min(255, 16 m + f), m = floor(log2(n + 1)) and f
 *                  the four bits of n + 1 below its leading one (n = the
 *                  tile's entries), ties by tile id
 *   overflow       device, int32 [1] (out): 0, or 1 when *n_dup > capacity;
 *                  then no entry is written and every range is empty
 *   workspace      device, hgs_workspace_bytes(HGS_WS_BIN_SORT, ...) bytes
 * capacity must be below 2^32.  The device-side *n_dup decides how much work
 * is done; capacity only bounds it (so a graph can be captured once with a
 * generous capacity). */
int hgs_bin_sort(const void* records, const uint32_t* tiles_touched, const uint64_t* offsets,
                 const uint64_t* n_dup, int64_t n_rec, const hgs_camera* cams, int32_t n_cams,
                 const hgs_options* opts, uint64_t* keys, uint32_t* values, int64_t capacity,
                 uint32_t* ranges, uint32_t* tile_order, int32_t* overflow, void* workspace,
                 size_t workspace_bytes, hipStream_t stream);

/* Front-to-back blending of every pixel of every camera (Sec. 3.3, Eq. 10).
 * With tile_order (from hgs_bin_sort) the raster runs as a persistent grid
 * sized to the device whose wavefronts take (tile, pixel block) work items
 * in that order from a counter in the workspace; with NULL, one workgroup
 * per tile.  The outputs are identical either way.
 *   images     device, float [3][H][W] per camera, camera c at 3 * pixel
 *              offset c (out): blended colour + final transmittance * bg
 *   T_final    device, float per pixel (out)
 *   last_idx   device, int32 per pixel (out): index, within the pixel's
 *              tile list (values[start .. end) of its tile), of the last
 *              blended entry; -1 if none
 *   n_contrib  device, int32 per pixel (out): number of blended kernels
 *   depth      device, float per pixel (out), may be NULL: the blended
 *              camera-space depth of the kernel centres, sum of w_i z_i with
 *              the colour weights w_i (no background term; the depth maps of
 *              Sec. 4, divide by 1 - T_final for the expected depth)
 *   workspace  device, at least hgs_workspace_bytes(HGS_WS_RENDER, ...) bytes
 *              (capacity 0); with room for the marks of these lists, the
 *              pass also records, per list position it walks, which pixel
 *              strips blended that entry, for hgs_raster_bwd */
int hgs_render_fwd(const void* records, const uint32_t* values, const uint32_t* ranges,
                   const uint32_t* tile_order, const hgs_camera* cams, int32_t n_cams,
                   const hgs_options* opts, float* images, float* T_final, int32_t* last_idx,
                   int32_t* n_contrib, float* depth, void* workspace, size_t workspace_bytes,
                   hipStream_t stream);

/* Surface normals estimated from the depth map (Sec. 4 shows them; the
 * estimate follows 2D-GS): per pixel the expected depth d = depth / (1 -
 * T_final) is back-projected through the camera, P = d ((u + 1/2 - cx) / fx,
 * (v + 1/2 - cy) / fy, 1), and n = -(P(u+1, v) - P(u-1, v)) x (P(u, v+1) -
 * P(u, v-1)), normalised: camera axes, facing the camera.  Zero on the image
 * border, next to a pixel with 1 - T_final = 0, and where the cross product
 * vanishes.  Computed in FP64.
 *   depth, T_final  device, float per pixel, as from hgs_render_fwd
 *   normals         device, float [3][H][W] per camera, camera c at
 *                   3 * pixel offset c (out)
 * HGS_EINVAL for a null pointer or bad cameras. */
int hgs_depth_normals(const float* depth, const float* T_final, const hgs_camera* cams, int32_t n_cams,
                      float* normals, hipStream_t stream);

/* Gradient of a scalar loss L given dL/d(image) (same layout as `images`).
 * Replays every pixel back to front from last_idx using T_final (no blend
 * history is stored), accumulates the gradients of each record's screen
 * centre (2), conic (3), half-factor vector (2), alpha2, (alpha1-alpha2)/2
 * and colour (3) in `record_grads`, then applies the chain rule through the
 * projection to every kernel parameter, summed over cameras.
 *   record_grads  device, float [n_cams * n][HGS_RECORD_GRAD_FLOATS] scratch
 *                 (any contents on entry; cleared on return)
 *   grads         device pointers, overwritten
 *   workspace     device, the workspace (same pointer and size) given to the
 *                 hgs_render_fwd call that produced T_final and last_idx
 * params, cams and opts must be those given to hgs_preprocess. */
int hgs_render_bwd(const hgs_params* params, const hgs_camera* cams, int32_t n_cams,
                   const hgs_options* opts, const void* records, const uint32_t* values,
                   const uint32_t* ranges, const uint32_t* tile_order, const float* T_final,
                   const int32_t* last_idx,
                   const float* dL_dimages, float* record_grads, const hgs_param_grads* grads,
                   void* workspace, size_t workspace_bytes, hipStream_t stream);

/* The two halves of hgs_render_bwd, for callers that want the per-record
 * gradients themselves (the screen-space centre gradient drives the
 * densification heuristics of 3D-GS training) or schedule the halves
 * separately.
 *
 * hgs_raster_bwd: the per-pixel back-to-front replay only; ADDS each
 * record's 12 gradients to record_grads (device, float
 * [n_cams * n][HGS_RECORD_GRAD_FLOATS]), which the caller must have cleared
 * (hgs_preprocess_bwd leaves it cleared).  n is the kernel count given to
 * hgs_preprocess.  workspace: the one (same pointer and size) given to the
 * hgs_render_fwd call over these lists.  Where that call left strip marks,
 * entries and pixel strips that blended nothing are skipped (they add
 * nothing to any gradient); the forward pass tags the marks with a key of
 * the lists, the plane size and the tiling, and a workspace without the
 * matching tag is replayed in full, with the same gradients.
 *
 * hgs_preprocess_bwd: the chain rule from record_grads to every kernel
 * parameter (summed over cameras, grads overwritten); clears record_grads
 * after reading it.  `records` (those of hgs_preprocess) must be non-null but
 * are not read: a record whose twelve gradients are all zero -- every culled
 * record, since hgs_raster_bwd adds only to records in the tile lists --
 * contributes nothing and is skipped. */
int hgs_raster_bwd(const void* records, const uint32_t* values, const uint32_t* ranges,
                   const uint32_t* tile_order, const hgs_camera* cams, int32_t n_cams,
                   const hgs_options* opts, const float* T_final, const int32_t* last_idx,
                   const float* dL_dimages, float* record_grads, void* workspace,
                   size_t workspace_bytes, hipStream_t stream);
int hgs_preprocess_bwd(const hgs_params* params, const hgs_camera* cams, int32_t n_cams,
                       const hgs_options* opts, const void* records, float* record_grads,
                       const hgs_param_grads* grads, hipStream_t stream);

/* Mip-Splatting's 3-D filter variance per kernel (used by Mip-Splatting-HGS,
 * Sec. 4): the kernel's sampling rate nu is the largest fx / z over the
 * cameras that see its centre (camera z > znear and the projected centre
 * inside the image widened by `margin` times its size on every side); the
 * variance is s / nu^2 (s = 0.2 in Mip-Splatting).  Kernels seen by no
 * camera get the smallest rate among the seen ones (the widest filter), or 0
 * if no kernel is seen.  means: device, 3 planes of `stride`; filter3d:
 * device float[n] (out); workspace: device, 256 bytes.  Errors: HGS_EINVAL
 * for null pointers, bad cameras, n < 0, stride < n, s < 0, margin < 0. */
int hgs_mip_filter3d(const float* means, int64_t n, int64_t stride, const hgs_camera* cams, int32_t n_cams,
                     float s, float margin, float* filter3d, void* workspace, hipStream_t stream);

/* ------------------------------------------------------------------------
 * Training step after the backward pass (Sec. 4, implementation: the normal
 * uses 3D-GS's three unused normal parameters, one opacity per half, the
 * 3D-GS training recipe otherwise, normal learning rate 0.003; Supp.,
 * training settings: opacity and normal learning rates divided by 1.4 every
 * 5000 iterations, pruning opacity threshold 0.01, opacity reset to 0.02).
 *
 * The optimised ("raw") parameters use the hgs_params plane layout with
 * log-scales in place of scales and opacity logits in place of opacities;
 * the rasterizer takes exp(log-scale) and sigmoid(logit).  An
 * hgs_param_grads struct names any set of mutable planes in that layout:
 * raw values, Adam moments, activated copies.  All pointers are device
 * pointers; n kernels, plane p of a field at ptr + p * stride.
 * ------------------------------------------------------------------------ */

/* The photometric L1 term of the 3D-GS loss the paper trains with: the
 * gradient of L = scale * sum |images - target| with respect to the
 * images, dL_dimages[i] = scale * sign(images[i] - target[i]) (0 where
 * equal), over n floats (packed images of any number of cameras); scale =
 * 1/n gives the mean, 1/N one view's share of a mean over N values.  loss
 * may be NULL; otherwise L is ADDED to *loss (device float, float atomics:
 * clear it first).  HGS_EINVAL for n < 0 or a null array. */
int hgs_l1_loss_grad(const float* images, const float* target, int64_t n, float scale, float* dL_dimages,
                     float* loss, hipStream_t stream);

/* Adam step constants.  lr_*: learning rate per group; beta1, beta2, eps;
 * step: the step number t >= 1 (bias corrections 1 - beta^t). */
typedef struct hgs_adam_config {
  float lr_means, lr_scales, lr_quats, lr_normals, lr_opacity, lr_sh_dc, lr_sh_rest;
  float beta1;   /* [0.9]   */
  float beta2;   /* [0.999] */
  float eps;     /* [1e-15] */
  int32_t step;
  int32_t reserved;
} hgs_adam_config;

/* The half-Gaussian schedule at iteration `step` (1-based) for a scene of
 * radius `extent`: means 1.6e-4 * extent decaying log-linearly to
 * 1.6e-6 * extent at 30000; log-scales 0.005; quaternions 0.001; SH degree
 * 0 0.0025, higher 0.0025 / 20; opacities 0.05 and normals `normal_lr`
 * (0.003; 0.3 was used for one dataset), both times 1.4^-floor(step/5000).
 * Host only.  HGS_EINVAL for step < 1, extent <= 0 or a null cfg. */
int hgs_adam_schedule(int32_t step, float extent, float normal_lr, hgs_adam_config* cfg);

/* One Adam step on every raw plane.  grads: loss gradient with respect to
 * the ACTIVATED parameters (as hgs_render_bwd writes it); the chain rule
 * through exp and sigmoid is applied here.  raw, m, v are updated in place;
 * act receives the activated values (a plane of act may alias the raw plane
 * where the activation is the identity, which then skips its write).
 * Errors: HGS_EINVAL for null pointers, n < 0, stride < n, bad sh_degree,
 * step < 1; HGS_EHIP on a launch failure. */
int hgs_adam_step(const hgs_adam_config* cfg, int64_t n, int64_t stride, int32_t sh_degree,
                  const hgs_param_grads* raw, const hgs_param_grads* grads, const hgs_param_grads* m,
                  const hgs_param_grads* v, const hgs_param_grads* act, hipStream_t stream);

/* act = activation(raw) for the log-scale and opacity planes and a copy of
 * the others (planes of act that alias raw are skipped). */
int hgs_activate(int64_t n, int64_t stride, int32_t sh_degree, const hgs_param_grads* raw,
                 const hgs_param_grads* act, hipStream_t stream);

/* Densification statistics of 3D-GS, accumulated over the cameras of one
 * step: for every record with tiles > 0 (visible), grad_accum[i] += the
 * norm of the loss gradient with respect to the record's screen centre in
 * normalised device coordinates (the pixel-space gradient in record_grads
 * times W/2 and H/2), grad_count[i] += 1, and max_radii[i] = max(max_radii[i],
 * ceil(kappa * sqrt(lambda_max))) of the dilated screen covariance (from the
 * record's conic, FP64).  Call after hgs_raster_bwd and before
 * hgs_preprocess_bwd (which clears record_grads).  records, record_grads:
 * as given to hgs_raster_bwd, n kernels per camera.  grad_accum float[n],
 * grad_count int32[n], max_radii float[n]: device, accumulated (the caller
 * clears them). */
int hgs_densify_stats(const void* records, const float* record_grads, const hgs_camera* cams, int32_t n_cams,
                      const hgs_options* opts, int64_t n, float* grad_accum, int32_t* grad_count,
                      float* max_radii, hipStream_t stream);

/* Densify / prune thresholds ([] = hgs_densify_default values). */
typedef struct hgs_densify_config {
  float extent;             /* scene radius (> 0)                            */
  float grad_threshold;     /* [0.0002] average NDC centre gradient          */
  float percent_dense;      /* [0.01]   clone below, split above, x extent    */
  float min_opacity;        /* [0.01]   prune when BOTH halves are below      */
  float max_screen_radius;  /* [0] px, 0 = off (3D-GS: 20 after the first
                                opacity reset)                               */
  float max_world_scale;    /* [0] x extent, 0 = off (3D-GS: 0.1 together
                                with the screen rule)                        */
} hgs_densify_config;

/* Fills cfg with the bracketed defaults above and the given extent (host
 * only; a null cfg is ignored). */
void hgs_densify_default(float extent, hgs_densify_config* cfg);
/* Device workspace bytes hgs_densify needs for n input kernels (flags,
 * their scans and the scan partials); 0 for n < 0.  Host only. */
size_t hgs_densify_workspace_bytes(int64_t n);

/* Clone, split and prune (3D-GS densification with the half-Gaussian
 * opacity threshold).  A kernel whose average gradient
 * grad_accum / grad_count reaches grad_threshold (grad_count > 0) is cloned
 * when its largest scale is <= percent_dense * extent, else split into two
 * children centred at mean + R(q) (scale * z) with z = samples[c][0..2][i]
 * (standard normal draws, float [2][3][n], the caller's), log-scales reduced
 * by log(0.8 * 2), everything else copied; the parent of a split is
 * removed.  Pruned: both opacities below min_opacity, or (when enabled)
 * max_radii > max_screen_radius or largest scale > max_world_scale * extent
 * (new kernels have radius 0).  Thresholds are compared on the raw values
 * (log / logit of the threshold, FP64).  Output order: surviving kernels,
 * clones, first children, second children, each in kernel order; raw_out,
 * m_out, v_out (planes of stride stride_out >= capacity, distinct from the
 * inputs) get the raw values and moments (zero for new kernels).  *n_out
 * (device int64) receives the new count; if it exceeds capacity nothing is
 * written and *overflow (device int32) is 1.  workspace:
 * hgs_densify_workspace_bytes(n) bytes.  The densification statistics are
 * not carried over (the caller clears them for the new kernels). */
int hgs_densify(const hgs_densify_config* cfg, int64_t n, int64_t stride, int32_t sh_degree,
                const hgs_param_grads* raw, const hgs_param_grads* m, const hgs_param_grads* v,
                const float* grad_accum, const int32_t* grad_count, const float* max_radii, const float* samples,
                int64_t capacity, int64_t stride_out, const hgs_param_grads* raw_out,
                const hgs_param_grads* m_out, const hgs_param_grads* v_out, int64_t* n_out, int32_t* overflow,
                void* workspace, size_t workspace_bytes, hipStream_t stream);

/* Opacity reset (Supp., training settings): each half's opacity becomes
 * min(opacity, value) (value 0.02 in the paper), its Adam moments are
 * cleared, and act's opacity planes (if not NULL and not aliasing raw) are
 * refreshed.  Only the opac1/opac2 fields of raw, m, v, act are used. */
int hgs_reset_opacity(float value, int64_t n, const hgs_param_grads* raw, const hgs_param_grads* m,
                      const hgs_param_grads* v, const hgs_param_grads* act, hipStream_t stream);

const char* hgs_strerror(int code);
const char* hgs_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* HGS_H */
