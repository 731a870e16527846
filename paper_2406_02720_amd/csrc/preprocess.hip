// Preprocess: per-(camera, kernel) projection to a 64-byte record, the
// exclusive scan of tiles touched, and the chain-rule backward of the
// projection.
//
// One thread owns one kernel and loops over the cameras, so the 63 floats of
// parameters are read from HBM once per kernel (coalesced structure-of-arrays
// planes) whatever the number of views.  Geometry runs in FP64 (full rate on
// CDNA4) so that integer decisions -- pixel rects, tiles, fp32 depth keys --
// agree with an FP64 evaluation of the same formulas.

#include "hgs_internal.h"
#include "geometry.h"

namespace hgs {

namespace {

constexpr int kPreBlock = 256;
static_assert(kPreBlock == kPreprocessRecordsPerPartial, "preprocess workspace: one partial per kPreBlock kernels");

__device__ __forceinline__ bool finite(double x) { return isfinite(x); }

// Element `off4` / 4 of plane `plane` of a parameter field: the plane's
// start is wave-uniform (scalar registers) and the element's byte offset a
// 32-bit vector value (n <= INT32_MAX / HGS_MAX_CAMERAS keeps it below
// 2^31), so each load is one instruction with no 64-bit address arithmetic
// per lane.
typedef __attribute__((address_space(1))) char gchar_t;
typedef __attribute__((address_space(1))) float gfloat_t;
__device__ __forceinline__ gfloat_t* plane_ptr(const float* field, int64_t plane, int64_t stride, uint32_t off4) {
  gchar_t* base = (gchar_t*)(field + plane * stride);
  asm("" : "+s"(base));   // the plane start as an opaque scalar: not folded into per-lane address math
  return (gfloat_t*)(base + off4);
}
__device__ __forceinline__ float plane_at(const float* field, int64_t plane, int64_t stride, uint32_t off4) {
  return *plane_ptr(field, plane, stride, off4);
}

// Extents (E-x, E+x, E-y, E+y) of the union of the splatted halves (Sec. 3.4):
// per direction, a half reaches the full-ellipse tangent extent when the
// tangent point lies on its side of the plane (sign of g on that axis),
// otherwise the projected splitting ellipse bounds it.
struct Box {
  double emx, epx, emy, epy;
  bool any;
};

__device__ __forceinline__ Box half_box(const KernelGeo& k, const ViewGeo& vg, const Sym3& Ss,
                                        double a1, double a2, const Opts& o) {
  Box b;
  const double kap = o.kappa;
  const double ex = kap * sqrt(vg.A);
  const double ey = kap * sqrt(vg.C);
  if (o.flags & HGS_FLAG_FULL_BOX) {
    b.emx = b.epx = ex;
    b.emy = b.epy = ey;
    b.any = true;
    return b;
  }
  double cx = ex, cy = ey;
  if (!k.nzero) {
    const double sxx = sym_form(Ss, vg.M, vg.M);
    const double syy = sym_form(Ss, vg.M + 3, vg.M + 3);
    cx = fmin(kap * sqrt(sxx + (double)o.lowpass), ex);
    cy = fmin(kap * sqrt(syy + (double)o.lowpass), ey);
  }
  const bool s1 = a1 >= (double)o.alpha_min;
  const bool s2 = a2 >= (double)o.alpha_min;
  const double gx = vg.g[0], gy = vg.g[1];
  const double ninf = -INFINITY;
  // half +1 (alpha1 side)
  const double m1x = s1 ? (gx <= 0.0 ? ex : cx) : ninf;
  const double p1x = s1 ? (gx >= 0.0 ? ex : cx) : ninf;
  const double m1y = s1 ? (gy <= 0.0 ? ey : cy) : ninf;
  const double p1y = s1 ? (gy >= 0.0 ? ey : cy) : ninf;
  // half -1 (alpha2 side)
  const double m2x = s2 ? (-gx <= 0.0 ? ex : cx) : ninf;
  const double p2x = s2 ? (-gx >= 0.0 ? ex : cx) : ninf;
  const double m2y = s2 ? (-gy <= 0.0 ? ey : cy) : ninf;
  const double p2y = s2 ? (-gy >= 0.0 ? ey : cy) : ninf;
  b.emx = fmax(m1x, m2x);
  b.epx = fmax(p1x, p2x);
  b.emy = fmax(m1y, m2y);
  b.epy = fmax(p1y, p2y);
  b.any = s1 || s2;
  return b;
}

__device__ __forceinline__ int clamp_ceil(double x, int lo) {
  x = fmin(fmax(x, -1e9), 1e9);
  const int v = (int)ceil(x);
  return v < lo ? lo : v;
}
__device__ __forceinline__ int clamp_floor(double x, int hi) {
  x = fmin(fmax(x, -1e9), 1e9);
  const int v = (int)floor(x);
  return v > hi ? hi : v;
}

// The records of kernel i for every camera; returns the sum of their tiles.
// ONE: a single camera.  Its SH coefficients are then loaded before the
// kernel geometry, so that their loads are in flight while the FP64 geometry
// runs (with several cameras they are read per camera, from cache, after it:
// held across the camera loop they would double the register footprint).
template <int D, bool ONE>
__device__ __forceinline__ uint64_t preprocess_one(const Params& p, const CamPack& cp, const Opts& o,
                                                   Record* __restrict__ rec, uint32_t* __restrict__ tiles_out,
                                                   int64_t i) {
  constexpr int K = (D + 1) * (D + 1);
  uint64_t tiles_sum = 0;
  const int64_t S = p.stride;
  const uint32_t off4 = (uint32_t)i * 4u;
  float shv[ONE ? 3 * K : 1];
  if (ONE) {
#pragma unroll
    for (int j = 0; j < 3 * K; ++j) shv[j] = plane_at(p.sh, j, S, off4);
  }
  float mu[3], s[3], q[4], nrm[3];
  for (int c = 0; c < 3; ++c) {
    mu[c] = plane_at(p.means, c, S, off4);
    s[c] = plane_at(p.scales, c, S, off4);
    nrm[c] = plane_at(p.normals, c, S, off4);
  }
  for (int c = 0; c < 4; ++c) q[c] = plane_at(p.quats, c, S, off4);
  const float a1 = plane_at(p.opac1, 0, S, off4);
  const float a2 = plane_at(p.opac2, 0, S, off4);
  // any non-finite parameter culls the kernel
  bool params_ok = finite((double)a1) && finite((double)a2);
  for (int c = 0; c < 3; ++c)
    params_ok = params_ok && finite((double)mu[c]) && finite((double)s[c]) && finite((double)nrm[c]);
  for (int c = 0; c < 4; ++c) params_ok = params_ok && finite((double)q[c]);

  const double f3 = p.filter3d ? (double)plane_at(p.filter3d, 0, S, off4) : 0.0;
  params_ok = params_ok && finite(f3) && f3 >= 0.0;
  KernelGeo kg;
  kernel_geo(mu, s, q, nrm, kg, params_ok ? f3 : 0.0);
  Sym3 Ss = kg.Sw;
  if (!(o.flags & HGS_FLAG_FULL_BOX) && !kg.nzero) Ss = splitting_cov(kg);
  const int tsh = cp.tile_shift;

  const int n_cams = ONE ? 1 : cp.n_cams;
  for (int c = 0; c < n_cams; ++c) {
    const CamDev& cam = cp.cam[c];
    Record r;
    uint32_t tiles = 0;
    r.mx = r.my = r.kx = r.ky = 0.0f;
    r.qa = r.qb = r.qc = r.alpha2 = 0.0f;
    r.r = r.g = r.b = r.d_o = 0.0f;
    r.xr = r.yr = r.depth = 0u;
    // SH colour first (its basis values die before the geometry starts)
    double col0 = 0.0, col1 = 0.0, col2 = 0.0;
    if (params_ok) {
      double oc[3];
      camera_centre(cam, oc);
      double dx = kg.mu[0] - oc[0], dy = kg.mu[1] - oc[1], dz = kg.mu[2] - oc[2];
      const double il = 1.0 / sqrt(dx * dx + dy * dy + dz * dz);
      dx *= il; dy *= il; dz *= il;
      double Y[K];
      sh_eval<D>(dx, dy, dz, Y);
#pragma unroll
      for (int kk = 0; kk < K; ++kk) {
        if (ONE) {
          col0 += Y[kk] * (double)shv[kk * 3 + 0];
          col1 += Y[kk] * (double)shv[kk * 3 + 1];
          col2 += Y[kk] * (double)shv[kk * 3 + 2];
        } else {
          // plain indexing: the compiler reloads these per camera (48 more
          // live registers would not fit), but from addresses it computes
          // once; through an opaque plane base the loop took 2.5 times as
          // long
          col0 += Y[kk] * (double)p.sh[(kk * 3 + 0) * S + i];
          col1 += Y[kk] * (double)p.sh[(kk * 3 + 1) * S + i];
          col2 += Y[kk] * (double)p.sh[(kk * 3 + 2) * S + i];
        }
      }
      col0 = fmax(col0 + 0.5, 0.0);
      col1 = fmax(col1 + 0.5, 0.0);
      col2 = fmax(col2 + 0.5, 0.0);
    }
    ViewGeo vg;
    view_geo(kg, cam, (double)o.lowpass, (double)o.fov_clamp, vg);
    bool ok = params_ok && finite(vg.t[2]) && vg.t[2] > (double)cam.znear;
    ok = ok && finite(vg.det) && vg.det > 0.0 && finite(vg.qa) && finite(vg.qb) &&
         finite(vg.qc) && finite(vg.mx) && finite(vg.my) && finite(vg.k[0]) && finite(vg.k[1]);
    ok = ok && finite(col0) && finite(col1) && finite(col2);
    // opacity compensation of the Mip-Splatting filters (3-D, and 2-D mip)
    double comp = kg.comp3;
    if (o.flags & HGS_FLAG_MIP_2D) comp *= sqrt(fmax(vg.det0, 0.0) / vg.det);
    const double a1e = (double)a1 * comp, a2e = (double)a2 * comp;
    Box bx;
    if (ok) {
      bx = half_box(kg, vg, Ss, a1e, a2e, o);
      ok = bx.any;
    }
    if (ok) {
      const double lo_x = vg.mx - bx.emx - 0.5, hi_x = vg.mx + bx.epx - 0.5;
      const double lo_y = vg.my - bx.emy - 0.5, hi_y = vg.my + bx.epy - 0.5;
      ok = finite(lo_x) && finite(hi_x) && finite(lo_y) && finite(hi_y);
      if (ok) {
        const int x0 = clamp_ceil(lo_x, 0), x1 = clamp_floor(hi_x, cam.width - 1);
        const int y0 = clamp_ceil(lo_y, 0), y1 = clamp_floor(hi_y, cam.height - 1);
        ok = x0 <= x1 && y0 <= y1;
        if (ok) {
          const int tx0 = x0 >> tsh, tx1 = x1 >> tsh, ty0 = y0 >> tsh, ty1 = y1 >> tsh;
          tiles = (uint32_t)((tx1 - tx0 + 1) * (ty1 - ty0 + 1));
          r.mx = (float)(vg.mx - (double)x0);
          r.my = (float)(vg.my - (double)y0);
          r.kx = (float)vg.k[0];
          r.ky = (float)vg.k[1];
          r.qa = (float)vg.qa;
          r.qb = (float)vg.qb;
          r.qc = (float)vg.qc;
          r.alpha2 = (float)a2e;
          r.r = (float)col0;
          r.g = (float)col1;
          r.b = (float)col2;
          r.d_o = (float)((a1e - a2e) / 2.0);
          r.xr = (uint32_t)x0 | ((uint32_t)x1 << 16);
          r.yr = (uint32_t)y0 | ((uint32_t)y1 << 16);
          r.depth = __float_as_uint((float)vg.t[2]);
        }
      }
    }
    r.tiles = tiles;
    const int64_t ri = (int64_t)c * p.n + i;
    rec[ri] = r;
    tiles_out[ri] = tiles;
    tiles_sum += tiles;
  }
  return tiles_sum;
}

// One thread per kernel.  With block_tiles, each workgroup also stores the
// sum of its records' tiles (the entry total is then the sum of these
// partials: no second pass over tiles_out).
template <int D, bool ONE>
__global__ __launch_bounds__(kPreBlock) void preprocess_kernel(Params p, CamPack cp, Opts o,
                                                               Record* __restrict__ rec,
                                                               uint32_t* __restrict__ tiles_out,
                                                               uint64_t* __restrict__ block_tiles) {
  const int64_t i = (int64_t)blockIdx.x * kPreBlock + threadIdx.x;
  uint64_t mine = 0;
  if (i < p.n) mine = preprocess_one<D, ONE>(p, cp, o, rec, tiles_out, i);
  if (!block_tiles) return;
  __shared__ uint64_t s_w[kPreBlock / 64];
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) mine += __shfl_xor(mine, off, 64);
  if ((threadIdx.x & 63) == 0) s_w[threadIdx.x >> 6] = mine;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint64_t t = 0;
#pragma unroll
    for (int w = 0; w < kPreBlock / 64; ++w) t += s_w[w];
    block_tiles[blockIdx.x] = t;
  }
}

// ---------------------------------------------------------------------------
// exclusive scan of tiles touched (uint32 -> uint64), reduce-then-scan
// ---------------------------------------------------------------------------
constexpr int kScanBlock = 256;
constexpr int kScanItems = 4;    // 1024-item tiles: a million items make ~1000 workgroups
constexpr int kScanTile = kScanBlock * kScanItems;
static_assert(kScanTile == kScanRecordsPerPartial, "scan workspace: one partial per kScanTile records");

__device__ __forceinline__ uint64_t wave_incl_scan(uint64_t x) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const uint64_t y = __shfl_up(x, off, 64);
    if (lane >= off) x += y;
  }
  return x;
}

// Exclusive block scan over kScanBlock threads; returns the block total too.
__device__ __forceinline__ uint64_t block_excl_scan(uint64_t x, uint64_t* total, uint64_t* lds) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const uint64_t inc = wave_incl_scan(x);
  if (lane == 63) lds[wave] = inc;
  __syncthreads();
  uint64_t pre = 0, tot = 0;
#pragma unroll
  for (int w = 0; w < kScanBlock / 64; ++w) {
    const uint64_t v = lds[w];
    if (w < wave) pre += v;
    tot += v;
  }
  __syncthreads();
  *total = tot;
  return pre + inc - x;
}

__global__ __launch_bounds__(kScanBlock) void scan_reduce_kernel(const uint32_t* __restrict__ in,
                                                                 int64_t n,
                                                                 uint64_t* __restrict__ partial) {
  __shared__ uint64_t lds[kScanBlock / 64];
  const int64_t base = (int64_t)blockIdx.x * kScanTile;
  uint64_t acc = 0;
#pragma unroll
  for (int j = 0; j < kScanItems; ++j) {
    const int64_t idx = base + j * kScanBlock + threadIdx.x;
    if (idx < n) acc += in[idx];
  }
  uint64_t tot;
  block_excl_scan(acc, &tot, lds);
  if (threadIdx.x == 0) partial[blockIdx.x] = tot;
}

__global__ __launch_bounds__(kScanBlock) void scan_partials_kernel(uint64_t* __restrict__ partial,
                                                                   int64_t m,
                                                                   uint64_t* __restrict__ total) {
  __shared__ uint64_t lds[kScanBlock / 64];
  uint64_t run = 0;
  for (int64_t base = 0; base < m; base += kScanBlock) {
    const int64_t idx = base + threadIdx.x;
    const uint64_t x = idx < m ? partial[idx] : 0;
    uint64_t tot;
    const uint64_t ex = block_excl_scan(x, &tot, lds);
    if (idx < m) partial[idx] = run + ex;
    run += tot;
  }
  if (threadIdx.x == 0) *total = run;
}

// The entry total from the projection's per-workgroup partials: one
// workgroup, every load issued at once (a scan is not needed here).
constexpr int kSumThreads = 1024;
__global__ __launch_bounds__(kSumThreads) void sum_partials_kernel(const uint64_t* __restrict__ partial, int64_t m,
                                                                   uint64_t* __restrict__ total) {
  __shared__ uint64_t s_w[kSumThreads / 64];
  uint64_t x = 0;
  for (int64_t i = threadIdx.x; i < m; i += kSumThreads) x += partial[i];
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) x += __shfl_xor(x, off, 64);
  if ((threadIdx.x & 63) == 0) s_w[threadIdx.x >> 6] = x;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint64_t t = 0;
#pragma unroll
    for (int w = 0; w < kSumThreads / 64; ++w) t += s_w[w];
    *total = t;
  }
}

// Small inputs: the whole scan in one workgroup (one launch instead of
// three).
constexpr int64_t kScanSmall = 8192;

__global__ __launch_bounds__(kScanBlock) void scan_small_kernel(const uint32_t* __restrict__ in, int64_t n,
                                                                uint64_t* __restrict__ out,
                                                                uint64_t* __restrict__ total) {
  __shared__ uint64_t lds[kScanBlock / 64];
  uint64_t run = 0;
  for (int64_t base = 0; base < n; base += kScanBlock) {
    const int64_t idx = base + threadIdx.x;
    const uint64_t x = idx < n ? (uint64_t)in[idx] : 0ull;
    uint64_t tot;
    const uint64_t ex = block_excl_scan(x, &tot, lds);
    if (idx < n) out[idx] = run + ex;
    run += tot;
  }
  if (threadIdx.x == 0) *total = run;
}

__global__ __launch_bounds__(kScanBlock) void scan_apply_kernel(const uint32_t* __restrict__ in,
                                                                int64_t n,
                                                                const uint64_t* __restrict__ partial,
                                                                uint64_t* __restrict__ out) {
  __shared__ uint64_t lds[kScanBlock / 64];
  const int64_t base = (int64_t)blockIdx.x * kScanTile;
  uint64_t run = partial[blockIdx.x];
#pragma unroll
  for (int j = 0; j < kScanItems; ++j) {
    const int64_t idx = base + j * kScanBlock + threadIdx.x;
    const uint64_t x = idx < n ? in[idx] : 0;
    uint64_t tot;
    const uint64_t ex = block_excl_scan(x, &tot, lds);
    if (idx < n) out[idx] = run + ex;
    run += tot;
  }
}

// ---------------------------------------------------------------------------
// backward of the projection (chain rule to every kernel parameter)
// ---------------------------------------------------------------------------
// symmetric part of u v^T, added to S
__device__ __forceinline__ void add_sym_outer(Sym3& S, const double* u, const double* v, double w) {
  S.xx += w * u[0] * v[0];
  S.yy += w * u[1] * v[1];
  S.zz += w * u[2] * v[2];
  S.xy += w * 0.5 * (u[0] * v[1] + u[1] * v[0]);
  S.xz += w * 0.5 * (u[0] * v[2] + u[2] * v[0]);
  S.yz += w * 0.5 * (u[1] * v[2] + u[2] * v[1]);
}

template <int D, bool ONE>
__global__ __launch_bounds__(kPreBlock) void preprocess_bwd_kernel(
    Params p, CamPack cp, Opts o, float* __restrict__ rgrad, Grads G) {
  constexpr int K = (D + 1) * (D + 1);
  const int64_t i = (int64_t)blockIdx.x * kPreBlock + threadIdx.x;
  if (i >= p.n) return;
  const int64_t S = p.stride;
  // a single camera: no loops (their registers are then scheduled as one
  // straight-line body)
  const int n_cams = ONE ? 1 : cp.n_cams;
  double g_mu[3] = {0.0, 0.0, 0.0};
  // every input the geometry below reads is requested here, before the SH
  // gradients are stored: the vector memory counter orders loads and
  // stores, so a load issued after those 48 stores would wait for them
  // (0.126 -> 0.089 ms on one 1080p view of 1M kernels).  With one camera
  // that includes the record's twelve gradients.
  float4 rg1[3] = {};
  if (ONE) {
    const float4* g4 = reinterpret_cast<const float4*>(rgrad + i * HGS_RECORD_GRAD_FLOATS);
    rg1[0] = g4[0];
    rg1[1] = g4[1];
    rg1[2] = g4[2];
  }
  float mu[3], s[3], q[4], nrm[3];
  for (int c = 0; c < 3; ++c) {
    mu[c] = p.means[c * S + i];
    s[c] = p.scales[c * S + i];
    nrm[c] = p.normals[c * S + i];
  }
  for (int c = 0; c < 4; ++c) q[c] = p.quats[c * S + i];
  const float a1f = p.opac1[i], a2f = p.opac2[i];
  const float f3f = p.filter3d ? p.filter3d[i] : 0.0f;

  // ---- colour = max(0, sum_k f_k Y_k(d) + 0.5), d = (mu - o) / |mu - o|,
  // over all cameras first: the SH coefficients, basis values and their
  // gradients are dead before the geometry below starts
  {
    const double mu0 = (double)p.means[i], mu1 = (double)p.means[S + i], mu2 = (double)p.means[2 * S + i];
    float g_sh[3 * K];
#pragma unroll
    for (int j = 0; j < 3 * K; ++j) g_sh[j] = 0.0f;
    for (int c = 0; c < n_cams; ++c) {
      const int64_t ri = (int64_t)c * p.n + i;
      const float4 r2 = ONE ? rg1[2] : reinterpret_cast<const float4*>(rgrad + ri * HGS_RECORD_GRAD_FLOATS)[2];
      // no colour gradient (a culled record has none: the raster adds only
      // to records in the tile lists, into a cleared buffer)
      if (r2.y == 0.0f && r2.z == 0.0f && r2.w == 0.0f) continue;
      const double gcol[3] = {r2.y, r2.z, r2.w};
      double oc[3];
      camera_centre(cp.cam[c], oc);
      const double dv0 = mu0 - oc[0], dv1 = mu1 - oc[1], dv2 = mu2 - oc[2];
      const double dl = sqrt(dv0 * dv0 + dv1 * dv1 + dv2 * dv2);
      const double il = 1.0 / dl;
      const double d0 = dv0 * il, d1 = dv1 * il, d2 = dv2 * il;
      double Y[K];
      sh_eval<D>(d0, d1, d2, Y);
      double raw[3] = {0.0, 0.0, 0.0};
#pragma unroll
      for (int kk = 0; kk < K; ++kk)
#pragma unroll
        for (int ch = 0; ch < 3; ++ch) raw[ch] += Y[kk] * (double)p.sh[(kk * 3 + ch) * S + i];
      double gc[3];
#pragma unroll
      for (int ch = 0; ch < 3; ++ch) gc[ch] = (raw[ch] + 0.5 > 0.0) ? gcol[ch] : 0.0;
      double wk[K];
#pragma unroll
      for (int kk = 0; kk < K; ++kk) {
        double acc = 0.0;
#pragma unroll
        for (int ch = 0; ch < 3; ++ch) {
          g_sh[kk * 3 + ch] += (float)(gc[ch] * Y[kk]);
          acc += gc[ch] * (double)p.sh[(kk * 3 + ch) * S + i];
        }
        wk[kk] = acc;
      }
      double gd0, gd1, gd2;
      sh_grad<D>(d0, d1, d2, wk, &gd0, &gd1, &gd2);
      const double dot = gd0 * d0 + gd1 * d1 + gd2 * d2;
      g_mu[0] += (gd0 - d0 * dot) * il;
      g_mu[1] += (gd1 - d1 * dot) * il;
      g_mu[2] += (gd2 - d2 * dot) * il;
    }
#pragma unroll
    for (int j = 0; j < 3 * K; ++j) G.sh[j * S + i] = g_sh[j];
  }

  const double f3 = (double)f3f;
  KernelGeo kg;
  kernel_geo(mu, s, q, nrm, kg, (isfinite(f3) && f3 >= 0.0) ? f3 : 0.0);
  const double a1 = (double)a1f, a2 = (double)a2f;
  double g_c3 = 0.0;   // dL / d comp3

  Sym3 g_Sw = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  double g_nh[3] = {0.0, 0.0, 0.0};
  double g_a1 = 0.0, g_a2 = 0.0;

  for (int c = 0; c < n_cams; ++c) {
    const int64_t ri = (int64_t)c * p.n + i;
    float* gr = rgrad + ri * HGS_RECORD_GRAD_FLOATS;
    float4* gr4 = reinterpret_cast<float4*>(gr);
    const float4 r0 = ONE ? rg1[0] : gr4[0], r1 = ONE ? rg1[1] : gr4[1], r2 = ONE ? rg1[2] : gr4[2];
    // all twelve zero (every culled record, and visible ones no pixel
    // blended): no contribution and nothing to clear.  The records
    // themselves are not read.
    const uint32_t nz = (__float_as_uint(r0.x) | __float_as_uint(r0.y) | __float_as_uint(r0.z) |
                         __float_as_uint(r0.w) | __float_as_uint(r1.x) | __float_as_uint(r1.y) |
                         __float_as_uint(r1.z) | __float_as_uint(r1.w) | __float_as_uint(r2.x) |
                         __float_as_uint(r2.y) | __float_as_uint(r2.z) | __float_as_uint(r2.w)) &
                        0x7fffffffu;
    if (nz == 0u) continue;
    const float gdo_f = r2.x;
    gr4[0] = gr4[1] = gr4[2] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);  // leave the buffer cleared
    const double gmx = r0.x, gmy = r0.y;
    const double gqa = r0.z, gqb = r0.w, gqc = r1.x;
    const double gkx = r1.y, gky = r1.z;
    const double galpha2 = r1.w, gdo = gdo_f;

    const CamDev& cam = cp.cam[c];
    ViewGeo vg;
    view_geo(kg, cam, (double)o.lowpass, (double)o.fov_clamp, vg);

    // alpha2 = comp a2 and (alpha1 - alpha2) / 2 = comp (a1 - a2) / 2, with
    // comp = comp3 c2 (Mip-Splatting compensations; 1 without filters)
    const bool mip2 = (o.flags & HGS_FLAG_MIP_2D) != 0;
    const double c2 = mip2 ? (vg.det0 > 0.0 ? sqrt(vg.det0 / vg.det) : 0.0) : 1.0;
    const double comp = kg.comp3 * c2;
    g_a2 += comp * (galpha2 - 0.5 * gdo);
    g_a1 += comp * 0.5 * gdo;
    const double gcomp = galpha2 * a2 + 0.5 * gdo * (a1 - a2);
    g_c3 += gcomp * c2;
    const double g_c2 = gcomp * kg.comp3;

    // ---- k = w r, r = (2 s2)^-1/2, w = Q g, s2 = v - g.w (or 1e-12 v)
    double gg0 = 0.0, gg1 = 0.0, gv = 0.0;
    double gQa = gqa, gQb = gqb, gQc = gqc;
    if (!kg.nzero && vg.s2 > 0.0) {
      double gw0 = gkx * vg.r, gw1 = gky * vg.r;
      const double grr = gkx * vg.w[0] + gky * vg.w[1];
      const double gs2 = -grr * vg.r * vg.r * vg.r;
      if (!vg.s2clamp) {
        gv += gs2;
        gg0 -= gs2 * vg.w[0];
        gg1 -= gs2 * vg.w[1];
        gw0 -= gs2 * vg.g[0];
        gw1 -= gs2 * vg.g[1];
      } else {
        gv += 1e-12 * gs2;
      }
      gQa += gw0 * vg.g[0];
      gQb += gw0 * vg.g[1] + gw1 * vg.g[0];
      gQc += gw1 * vg.g[1];
      gg0 += vg.qa * gw0 + vg.qb * gw1;
      gg1 += vg.qb * gw0 + vg.qc * gw1;
    }
    // ---- conic = inverse of (A, B; B, C)
    const double A = vg.A, B = vg.B, C = vg.C;
    const double id2 = 1.0 / (vg.det * vg.det);
    double gA = (-C * C * gQa + B * C * gQb - B * B * gQc) * id2;
    double gB = (2.0 * B * C * gQa - (A * C + B * B) * gQb + 2.0 * A * B * gQc) * id2;
    double gC = (-B * B * gQa + A * B * gQb - A * A * gQc) * id2;
    // c2 = sqrt(det0 / det): d c2 = c2 / 2 (d det0 / det0 - d det / det),
    // det0 = (A - l)(C - l) - B^2, det = A C - B^2
    if (mip2 && vg.det0 > 0.0) {
      const double h = 0.5 * g_c2 * c2;
      const double A0 = A - (double)o.lowpass, C0 = C - (double)o.lowpass;
      gA += h * (C0 / vg.det0 - C / vg.det);
      gC += h * (A0 / vg.det0 - A / vg.det);
      gB += h * (2.0 * B / vg.det - 2.0 * B / vg.det0);
    }
    // G_S = [[gA, gB/2], [gB/2, gC]].  Shat = M Sw M^T: dM += 2 G_S M Sw,
    // dSw += M^T G_S M.  g = M Sn: dM += gg Sn^T, dSn = M^T gg.
    const double* M = vg.M;
    const double GS00 = gA, GS01 = 0.5 * gB, GS11 = gC;
    double MS0[3], MS1[3];  // rows of M Sw
    sym_mul_vec(kg.Sw, M, MS0);
    sym_mul_vec(kg.Sw, M + 3, MS1);
    double gM[6];
#pragma unroll
    for (int cc = 0; cc < 3; ++cc) {
      gM[cc] = 2.0 * (GS00 * MS0[cc] + GS01 * MS1[cc]) + gg0 * kg.Sn[cc];
      gM[3 + cc] = 2.0 * (GS01 * MS0[cc] + GS11 * MS1[cc]) + gg1 * kg.Sn[cc];
    }
    // M^T G_S M (symmetric)
    add_sym_outer(g_Sw, M, M, GS00);
    add_sym_outer(g_Sw, M + 3, M + 3, GS11);
    add_sym_outer(g_Sw, M, M + 3, 2.0 * GS01);
    double gSn[3];
#pragma unroll
    for (int r = 0; r < 3; ++r) {
      gSn[r] = M[r] * gg0 + M[3 + r] * gg1 + gv * kg.nh[r];
      g_nh[r] += gv * kg.Sn[r];
    }
    // Sn = Sw n: dSw += sym(dSn n^T), dn += Sw dSn
    add_sym_outer(g_Sw, gSn, kg.nh, 1.0);
    double SgSn[3];
    sym_mul_vec(kg.Sw, gSn, SgSn);
    g_nh[0] += SgSn[0];
    g_nh[1] += SgSn[1];
    g_nh[2] += SgSn[2];

    // ---- M = J R_c: dJ = dM R_c^T
    const float* Rc = cam.R;
    double gJ00 = 0.0, gJ02 = 0.0, gJ11 = 0.0, gJ12 = 0.0;
#pragma unroll
    for (int cc = 0; cc < 3; ++cc) {
      gJ00 += gM[cc] * (double)Rc[0 * 3 + cc];
      gJ02 += gM[cc] * (double)Rc[2 * 3 + cc];
      gJ11 += gM[3 + cc] * (double)Rc[1 * 3 + cc];
      gJ12 += gM[3 + cc] * (double)Rc[2 * 3 + cc];
    }
    const double tx = vg.t[0], ty = vg.t[1], tz = vg.t[2];
    const double fx = cam.fx, fy = cam.fy;
    const double tz2 = tz * tz, tz3 = tz2 * tz;
    double gt0 = 0.0, gt1 = 0.0, gt2 = 0.0;
    gt2 += -fx / tz2 * gJ00 - fy / tz2 * gJ11;
    if (!vg.clx) {
      gt0 += -fx / tz2 * gJ02;
      gt2 += 2.0 * fx * tx / tz3 * gJ02;
    } else {
      gt2 += fx * vg.xc / tz2 * gJ02;
    }
    if (!vg.cly) {
      gt1 += -fy / tz2 * gJ12;
      gt2 += 2.0 * fy * ty / tz3 * gJ12;
    } else {
      gt2 += fy * vg.yc / tz2 * gJ12;
    }
    // screen centre
    gt0 += gmx * fx / tz;
    gt1 += gmy * fy / tz;
    gt2 += -gmx * fx * tx / tz2 - gmy * fy * ty / tz2;
    // t = R_c mu + t_c
#pragma unroll
    for (int a = 0; a < 3; ++a)
      g_mu[a] += (double)Rc[0 * 3 + a] * gt0 + (double)Rc[1 * 3 + a] * gt1 + (double)Rc[2 * 3 + a] * gt2;
  }

  // ---- Sigma_w = Rq diag(s^2) Rq^T:  dRq = 2 Gs Rq D,  ds_c = 2 s_c (Rq^T Gs Rq)_cc
  double qh[4], qn, Rq[9];
  quat_rot(q, qh, qn, Rq);
  const double sc[3] = {(double)s[0], (double)s[1], (double)s[2]};
  double g_s[3];
  double GR[9];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const double col[3] = {Rq[0 * 3 + c], Rq[1 * 3 + c], Rq[2 * 3 + c]};
    double Gc[3];
    sym_mul_vec(g_Sw, col, Gc);
    g_s[c] = 2.0 * sc[c] * (col[0] * Gc[0] + col[1] * Gc[1] + col[2] * Gc[2]);
    const double dsq = sc[c] * sc[c];
    // comp3 = prod s / sqrt(s^2 + f): d ln comp3 / d s = f / (s (s^2 + f))
    if (kg.f > 0.0) g_s[c] += g_c3 * kg.comp3 * kg.f / (sc[c] * (dsq + kg.f));
    GR[0 * 3 + c] = 2.0 * Gc[0] * dsq;
    GR[1 * 3 + c] = 2.0 * Gc[1] * dsq;
    GR[2 * 3 + c] = 2.0 * Gc[2] * dsq;
  }
  const double qw = qh[0], qx = qh[1], qy = qh[2], qz = qh[3];
  const double* g = GR;
  double gq[4];
  gq[0] = 2.0 * (-qz * g[1] + qy * g[2] + qz * g[3] - qx * g[5] - qy * g[6] + qx * g[7]);
  gq[1] = 2.0 * (qy * g[1] + qz * g[2] + qy * g[3] - 2.0 * qx * g[4] - qw * g[5] + qz * g[6] +
                 qw * g[7] - 2.0 * qx * g[8]);
  gq[2] = 2.0 * (-2.0 * qy * g[0] + qx * g[1] + qw * g[2] + qx * g[3] + qz * g[5] - qw * g[6] +
                 qz * g[7] - 2.0 * qy * g[8]);
  gq[3] = 2.0 * (-2.0 * qz * g[0] - qw * g[1] + qx * g[2] + qw * g[3] - 2.0 * qz * g[4] +
                 qy * g[5] + qx * g[6] + qy * g[7]);
  double gq_raw[4] = {0.0, 0.0, 0.0, 0.0};
  if (qn > 0.0) {
    const double dot = gq[0] * qw + gq[1] * qx + gq[2] * qy + gq[3] * qz;
#pragma unroll
    for (int a = 0; a < 4; ++a) gq_raw[a] = (gq[a] - qh[a] * dot) / qn;
  }
  double gn_raw[3] = {0.0, 0.0, 0.0};
  if (!kg.nzero) {
    const double dot = g_nh[0] * kg.nh[0] + g_nh[1] * kg.nh[1] + g_nh[2] * kg.nh[2];
#pragma unroll
    for (int a = 0; a < 3; ++a) gn_raw[a] = (g_nh[a] - kg.nh[a] * dot) / kg.nn;
  }
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    G.means[c * S + i] = (float)g_mu[c];
    G.scales[c * S + i] = (float)g_s[c];
    G.normals[c * S + i] = (float)gn_raw[c];
  }
#pragma unroll
  for (int c = 0; c < 4; ++c) G.quats[c * S + i] = (float)gq_raw[c];
  G.opac1[i] = (float)g_a1;
  G.opac2[i] = (float)g_a2;
}

template <int D>
void launch_projection(unsigned grid, const Params& p, const CamPack& cp, const Opts& o, Record* rec,
                       uint32_t* tiles, uint64_t* partial, hipStream_t s) {
  auto kern = cp.n_cams == 1 ? preprocess_kernel<D, true> : preprocess_kernel<D, false>;
  hipLaunchKernelGGL(kern, dim3(grid), dim3(kPreBlock), 0, s, p, cp, o, rec, tiles, partial);
}

template <int D>
void launch_projection_bwd(unsigned grid, const Params& p, const CamPack& cp, const Opts& o, float* rec_grads,
                           const Grads& g, hipStream_t s) {
  auto kern = cp.n_cams == 1 ? preprocess_bwd_kernel<D, true> : preprocess_bwd_kernel<D, false>;
  hipLaunchKernelGGL(kern, dim3(grid), dim3(kPreBlock), 0, s, p, cp, o, rec_grads, g);
}

}  // namespace

hipError_t launch_preprocess(const Params& p, const CamPack& cp, const Opts& o, Record* rec,
                             uint32_t* tiles, uint64_t* offsets, uint64_t* total, void* ws, hipStream_t s) {
  const int64_t n_rec = p.n * cp.n_cams;
  const unsigned grid = (unsigned)((p.n + kPreBlock - 1) / kPreBlock);
  // the total alone: summed from per-workgroup partials written by the
  // projection itself; with offsets, the scan over the records
  uint64_t* partial = offsets ? nullptr : (uint64_t*)ws;
  if (p.n > 0) {
    switch (p.sh_degree) {
      case 0: launch_projection<0>(grid, p, cp, o, rec, tiles, partial, s); break;
      case 1: launch_projection<1>(grid, p, cp, o, rec, tiles, partial, s); break;
      case 2: launch_projection<2>(grid, p, cp, o, rec, tiles, partial, s); break;
      default: launch_projection<3>(grid, p, cp, o, rec, tiles, partial, s); break;
    }
  }
  if (offsets) return launch_scan(tiles, n_rec, offsets, total, ws, s);
  hipLaunchKernelGGL(sum_partials_kernel, dim3(1), dim3(kSumThreads), 0, s, partial, p.n > 0 ? (int64_t)grid : 0,
                     total);
  return hipGetLastError();
}

size_t preprocess_workspace_bytes(int64_t n_rec) {
  // the scan (with offsets), or one partial per kPreBlock kernels (at most
  // one per kPreBlock records)
  const size_t a = scan_workspace_bytes(n_rec);
  const int64_t blocks = (n_rec + kPreBlock - 1) / kPreBlock;
  const size_t b = (size_t)(blocks > 0 ? blocks : 1) * sizeof(uint64_t);
  return a > b ? a : b;
}

size_t scan_workspace_bytes(int64_t n) {
  const int64_t blocks = (n + kScanTile - 1) / kScanTile;
  return (size_t)(blocks > 0 ? blocks : 1) * sizeof(uint64_t);
}

hipError_t launch_scan(const uint32_t* tiles, int64_t n, uint64_t* offsets, uint64_t* total,
                       void* ws, hipStream_t s) {
  if (n <= kScanSmall && offsets) {
    hipLaunchKernelGGL(scan_small_kernel, dim3(1), dim3(kScanBlock), 0, s, tiles, n, offsets, total);
    return hipGetLastError();
  }
  const int64_t blocks = (n + kScanTile - 1) / kScanTile;
  uint64_t* partial = (uint64_t*)ws;
  if (blocks > 0)
    hipLaunchKernelGGL(scan_reduce_kernel, dim3((unsigned)blocks), dim3(kScanBlock), 0, s, tiles,
                       n, partial);
  hipLaunchKernelGGL(scan_partials_kernel, dim3(1), dim3(kScanBlock), 0, s, partial, blocks, total);
  if (blocks > 0 && offsets)   // no offsets wanted: the total alone
    hipLaunchKernelGGL(scan_apply_kernel, dim3((unsigned)blocks), dim3(kScanBlock), 0, s, tiles, n,
                       partial, offsets);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Mip-Splatting 3-D filter variance per kernel: the largest sampling rate
// fx / z over the cameras that see the centre (in front of the near plane,
// projected inside the image widened by `margin`), variance s / nu^2.
// Kernels no camera sees take the smallest rate of the seen ones (FP64,
// uncontracted, so that the visibility decisions are reproducible).
__global__ void mip_init_kernel(uint32_t* nu_min) {
  if (threadIdx.x == 0) nu_min[0] = 0x7f800000u;   // +inf
}

__global__ __launch_bounds__(kPreBlock) void mip_nu_kernel(const float* __restrict__ means, int64_t n,
                                                           int64_t stride, CamPack cp, double s, double margin,
                                                           float* __restrict__ out, uint32_t* __restrict__ nu_min) {
#pragma clang fp contract(off)
  const int64_t i = (int64_t)blockIdx.x * kPreBlock + threadIdx.x;
  if (i >= n) return;
  const double m0 = means[i], m1 = means[stride + i], m2 = means[2 * stride + i];
  double nu = 0.0;
  for (int c = 0; c < cp.n_cams; ++c) {
    const CamDev& cam = cp.cam[c];
    const float* R = cam.R;
    const double tx = (double)R[0] * m0 + (double)R[1] * m1 + (double)R[2] * m2 + (double)cam.t[0];
    const double ty = (double)R[3] * m0 + (double)R[4] * m1 + (double)R[5] * m2 + (double)cam.t[1];
    const double tz = (double)R[6] * m0 + (double)R[7] * m1 + (double)R[8] * m2 + (double)cam.t[2];
    if (!(tz > (double)cam.znear)) continue;
    const double fx = cam.fx, fy = cam.fy;
    const double x = fx * tx / tz + (double)cam.cx, y = fy * ty / tz + (double)cam.cy;
    const double W = cam.width, H = cam.height;
    if (x >= -margin * W && x <= (1.0 + margin) * W && y >= -margin * H && y <= (1.0 + margin) * H)
      nu = fmax(nu, fx / tz);
  }
  if (nu > 0.0) {
    out[i] = (float)(s / (nu * nu));
    atomicMin(nu_min, __float_as_uint((float)nu));
  } else {
    out[i] = -1.0f;
  }
}

__global__ __launch_bounds__(kPreBlock) void mip_fill_kernel(int64_t n, double s, const uint32_t* __restrict__ nu_min,
                                                             float* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * kPreBlock + threadIdx.x;
  if (i >= n || !(out[i] < 0.0f)) return;
  const uint32_t b = *nu_min;
  const double nu = b == 0x7f800000u ? 0.0 : (double)__uint_as_float(b);
  out[i] = nu > 0.0 ? (float)(s / (nu * nu)) : 0.0f;
}

hipError_t launch_mip_filter3d(const float* means, int64_t n, int64_t stride, const CamPack& cp, double s,
                               double margin, float* out, uint32_t* scratch, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  const unsigned grid = (unsigned)((n + kPreBlock - 1) / kPreBlock);
  hipLaunchKernelGGL(mip_init_kernel, dim3(1), dim3(64), 0, st, scratch);
  hipLaunchKernelGGL(mip_nu_kernel, dim3(grid), dim3(kPreBlock), 0, st, means, n, stride, cp, s, margin, out,
                     scratch);
  hipLaunchKernelGGL(mip_fill_kernel, dim3(grid), dim3(kPreBlock), 0, st, n, s, (const uint32_t*)scratch, out);
  return hipGetLastError();
}

hipError_t launch_preprocess_bwd(const Params& p, const CamPack& cp, const Opts& o, float* rec_grads,
                                 const Grads& g, hipStream_t s) {
  if (p.n == 0) return hipSuccess;
  const unsigned grid = (unsigned)((p.n + kPreBlock - 1) / kPreBlock);
  switch (p.sh_degree) {
    case 0: launch_projection_bwd<0>(grid, p, cp, o, rec_grads, g, s); break;
    case 1: launch_projection_bwd<1>(grid, p, cp, o, rec_grads, g, s); break;
    case 2: launch_projection_bwd<2>(grid, p, cp, o, rec_grads, g, s); break;
    default: launch_projection_bwd<3>(grid, p, cp, o, rec_grads, g, s); break;
  }
  return hipGetLastError();
}

}  // namespace hgs
