// Host-side checks of libhgs built with AddressSanitizer and
// UndefinedBehaviorSanitizer on its host code (tests/test_host_sanitizers.py
// builds and runs this program; no GPU is needed).  Every call here stays on
// the host: sizes, option and camera validation, argument errors of every
// entry point (which are reported before any device work), the learning-rate
// schedule and the densification defaults.  Exit status 0 when every check
// holds; a sanitizer report aborts the program.
#include <cmath>
#include <cstdio>
#include <cstring>

#include "hgs.h"

static int failures = 0;

#define CHECK(cond)                                                                 \
  do {                                                                              \
    if (!(cond)) {                                                                  \
      std::fprintf(stderr, "%s:%d: check failed: %s (last error: %s)\n", __FILE__, \
                   __LINE__, #cond, hgs_last_error());                              \
      ++failures;                                                                   \
    }                                                                               \
  } while (0)

static bool last_error_has(const char* word) { return std::strstr(hgs_last_error(), word) != nullptr; }

static hgs_camera camera(int w, int h) {
  hgs_camera c;
  std::memset(&c, 0, sizeof c);
  c.R[0] = c.R[4] = c.R[8] = 1.0f;
  c.t[2] = 4.0f;
  c.fx = c.fy = 0.8f * (float)w;
  c.cx = 0.5f * (float)w;
  c.cy = 0.5f * (float)h;
  c.width = w;
  c.height = h;
  c.znear = 0.01f;
  return c;
}

int main() {
  hgs_options o;
  hgs_default_options(&o);
  CHECK(o.tile == 16 && o.batch == 256 && o.flags == 0u);
  CHECK(o.alpha_min == 1.0f / 255.0f && o.t_min == 1e-4f && o.alpha_max == 0.99f);

  // sizes
  hgs_camera hd = camera(1920, 1080);
  CHECK(hgs_tiles_total(&hd, 1, &o) == 120 * 68);
  CHECK(hgs_pixels_total(&hd, 1) == 1920 * 1080);
  hgs_options o8 = o, o32 = o, bad_tile = o, bad_batch = o;
  o8.tile = 8;
  o32.tile = 32;
  bad_tile.tile = 12;
  bad_batch.batch = 100;
  CHECK(hgs_tiles_total(&hd, 1, &o8) == 240 * 135);
  CHECK(hgs_tiles_total(&hd, 1, &o32) == 60 * 34);
  CHECK(hgs_tiles_total(&hd, 1, &bad_tile) == -1);
  CHECK(hgs_tiles_total(&hd, 1, &bad_batch) == -1);
  CHECK(hgs_workspace_bytes(HGS_WS_BIN_SORT, 100, &hd, 1, &o, 1000) > 12 * 1000);
  CHECK(hgs_workspace_bytes(HGS_WS_BIN_SORT, 100, &hd, 1, &bad_tile, 1000) == 0);
  CHECK(hgs_workspace_bytes(HGS_WS_PREPROCESS, 1 << 20, &hd, 1, &o, 0) > 0);
  CHECK(hgs_workspace_bytes(HGS_WS_RENDER, 1 << 20, &hd, 1, &o, 0) > 0);
  CHECK(hgs_workspace_bytes(7, 100, &hd, 1, &o, 1000) == 0);

  // many cameras of uneven sizes: the tile and pixel sums
  hgs_camera many[HGS_MAX_CAMERAS + 1];
  long long tiles = 0, pixels = 0;
  for (int c = 0; c <= HGS_MAX_CAMERAS; ++c) {
    many[c] = camera(17 + 29 * c, 9 + 13 * c);
    if (c < HGS_MAX_CAMERAS) {
      tiles += (long long)((many[c].width + 15) / 16) * ((many[c].height + 15) / 16);
      pixels += (long long)many[c].width * many[c].height;
    }
  }
  CHECK(hgs_tiles_total(many, HGS_MAX_CAMERAS, &o) == tiles);
  CHECK(hgs_pixels_total(many, HGS_MAX_CAMERAS) == pixels);
  CHECK(hgs_tiles_total(many, HGS_MAX_CAMERAS + 1, &o) == -1);
  CHECK(hgs_tiles_total(many, 0, &o) == -1);

  // camera validation
  hgs_camera wide = camera(70000, 10);
  CHECK(hgs_tiles_total(&wide, 1, &o) == -1);
  const float bad_near[] = {0.0f, -0.5f, NAN, INFINITY};
  for (float zn : bad_near) {
    hgs_camera c = camera(64, 64);
    c.znear = zn;
    CHECK(hgs_tiles_total(&c, 1, &o) == -1);
    CHECK(hgs_workspace_bytes(HGS_WS_BIN_SORT, 10, &c, 1, &o, 100) == 0);
  }
  hgs_camera bad_f = camera(64, 64);
  bad_f.fx = -1.0f;
  CHECK(hgs_tiles_total(&bad_f, 1, &o) == -1);

  // argument errors are reported before any device work
  hgs_params p;
  std::memset(&p, 0, sizeof p);
  CHECK(hgs_preprocess(nullptr, &hd, 1, &o, nullptr, nullptr, nullptr, nullptr, nullptr, 0, nullptr) ==
        HGS_EINVAL);
  CHECK(last_error_has("params"));
  p.n = p.stride = 10;
  p.sh_degree = 4;
  CHECK(hgs_preprocess(&p, &hd, 1, &o, nullptr, nullptr, nullptr, nullptr, nullptr, 0, nullptr) == HGS_EINVAL);
  CHECK(last_error_has("sh_degree"));
  p.sh_degree = 0;
  CHECK(hgs_preprocess(&p, &hd, 0, &o, nullptr, nullptr, nullptr, nullptr, nullptr, 0, nullptr) == HGS_EINVAL);
  p.n = p.stride = 0;  // no kernels: the null planes are not an error
  for (float zn : bad_near) {
    hgs_camera c = camera(64, 64);
    c.znear = zn;
    CHECK(hgs_preprocess(&p, &c, 1, &o, nullptr, nullptr, nullptr, nullptr, nullptr, 0, nullptr) == HGS_EINVAL);
    CHECK(last_error_has("znear"));
  }
  p.n = 10;
  p.stride = 5;  // stride < n
  CHECK(hgs_preprocess(&p, &hd, 1, &o, nullptr, nullptr, nullptr, nullptr, nullptr, 0, nullptr) == HGS_EINVAL);

  // the no-alloc preprocess: more records than its array serves
  {
    hgs_camera three[3] = {camera(64, 64), camera(64, 64), camera(64, 64)};
    hgs_params q;
    std::memset(&q, 0, sizeof q);
    const float* fake = reinterpret_cast<const float*>(1ull << 40);
    q.means = q.scales = q.quats = q.normals = q.opac1 = q.opac2 = q.sh = fake;
    q.n = q.stride = HGS_NOALLOC_MAX_RECORDS / 3 + 1;
    void* out = reinterpret_cast<void*>(1ull << 40);
    CHECK(hgs_preprocess_noalloc(&q, three, 3, &o, out, static_cast<uint32_t*>(out), nullptr,
                                 static_cast<uint64_t*>(out), nullptr) == HGS_ECAPACITY);
    CHECK(last_error_has("no-alloc limit"));
    CHECK(hgs_preprocess_noalloc(&q, three, 3, &o, nullptr, nullptr, nullptr, static_cast<uint64_t*>(out),
                                 nullptr) == HGS_EINVAL);
  }

  // every other entry point with null buffers
  CHECK(hgs_bin_sort(nullptr, nullptr, nullptr, nullptr, 10, &hd, 1, &o, nullptr, nullptr, 100, nullptr, nullptr,
                     nullptr, nullptr, 0, nullptr) == HGS_EINVAL);
  CHECK(hgs_render_fwd(nullptr, nullptr, nullptr, nullptr, &hd, 1, &o, nullptr, nullptr, nullptr, nullptr,
                       nullptr, nullptr, 0, nullptr) == HGS_EINVAL);
  CHECK(hgs_depth_normals(nullptr, nullptr, &hd, 1, nullptr, nullptr) == HGS_EINVAL);
  CHECK(hgs_render_bwd(nullptr, &hd, 1, &o, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr,
                       nullptr, nullptr, 0, nullptr) == HGS_EINVAL);
  CHECK(hgs_raster_bwd(nullptr, nullptr, nullptr, nullptr, &hd, 1, &o, nullptr, nullptr, nullptr, nullptr, nullptr,
                       0, nullptr) == HGS_EINVAL);
  CHECK(hgs_preprocess_bwd(nullptr, &hd, 1, &o, nullptr, nullptr, nullptr, nullptr) == HGS_EINVAL);
  CHECK(hgs_mip_filter3d(nullptr, 10, 10, &hd, 1, 0.2f, 1.0f, nullptr, nullptr, nullptr) == HGS_EINVAL);
  CHECK(hgs_l1_loss_grad(nullptr, nullptr, 10, 1.0f, nullptr, nullptr, nullptr) == HGS_EINVAL);
  CHECK(hgs_adam_step(nullptr, 10, 10, 0, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr) == HGS_EINVAL);
  CHECK(hgs_activate(10, 10, 0, nullptr, nullptr, nullptr) == HGS_EINVAL);
  CHECK(hgs_densify_stats(nullptr, nullptr, &hd, 1, &o, 10, nullptr, nullptr, nullptr, nullptr) == HGS_EINVAL);
  CHECK(hgs_densify(nullptr, 10, 10, 0, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, 20, 20,
                    nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, 0, nullptr) == HGS_EINVAL);
  CHECK(hgs_reset_opacity(0.01f, 10, nullptr, nullptr, nullptr, nullptr, nullptr) == HGS_EINVAL);

  // the learning-rate schedule and the densification defaults
  hgs_adam_config a;
  CHECK(hgs_adam_schedule(1, 2.0f, 0.003f, &a) == HGS_OK);
  CHECK(a.step == 1 && a.beta1 == 0.9f && a.beta2 == 0.999f && a.eps == 1e-15f);
  CHECK(a.lr_means > 0.0f && a.lr_opacity > 0.0f && a.lr_sh_rest < a.lr_sh_dc);
  hgs_adam_config late;
  CHECK(hgs_adam_schedule(30000, 2.0f, 0.003f, &late) == HGS_OK);
  CHECK(late.lr_means < a.lr_means && late.lr_scales == a.lr_scales);
  CHECK(hgs_adam_schedule(0, 1.0f, 0.003f, &a) == HGS_EINVAL);
  CHECK(hgs_adam_schedule(1, 0.0f, 0.003f, &a) == HGS_EINVAL);
  CHECK(hgs_adam_schedule(1, 1.0f, 0.003f, nullptr) == HGS_EINVAL);
  hgs_densify_config d;
  hgs_densify_default(2.0f, &d);
  CHECK(d.extent == 2.0f && d.grad_threshold == 0.0002f && d.percent_dense == 0.01f && d.min_opacity == 0.01f);
  CHECK(hgs_densify_workspace_bytes(1000) > 3 * 4 * 1000 + 3 * 8 * 1000);
  CHECK(hgs_densify_workspace_bytes(-1) == 0);

  // error strings
  CHECK(std::strcmp(hgs_strerror(HGS_ECAPACITY), "buffer too small") == 0);
  CHECK(hgs_strerror(HGS_OK) != nullptr && hgs_strerror(12345) != nullptr);

  if (failures) {
    std::fprintf(stderr, "%d host check(s) failed\n", failures);
    return 1;
  }
  std::printf("host checks passed\n");
  return 0;
}
