// Tile rasterizer: per-pixel front-to-back blending with the paired-half
// opacity of Eq. 10, and its back-to-front replay for gradients.
//
// Work decomposition (CDNA, wave64): a wavefront owns a 16x16 block of
// pixels (8x8 for 8-pixel tiles) and each lane owns 4 pixels of it (1 for
// 8-pixel tiles) -- pixel rows ly, ly+4, ly+8, ly+12 of column lx.  A 32-pixel
// tile is four such wavefronts walking the same list.  Every lane of a
// wavefront needs the same record at the same time, so the list is walked
// with wave-uniform indices: a round fetches `batch` entry ids with one
// vector load per lane, then each id is broadcast with v_readlane and its
// 64-byte record is loaded as uniform (scalar) data, one entry ahead of its
// use.  No LDS staging and no workgroup barriers: each wavefront stops as
// soon as all of its pixels are done.
//
// Backward: each lane replays its pixels back to front from the last blended
// entry, dividing the transmittance back out, and sums its pixels'
// gradients for the entry; the 12 sums are then reduced across the 64 lanes
// with DPP row operations and one lane issues the float atomics, so there is
// one reduction and one set of atomics per (entry, 256 pixels).

#include "hgs_internal.h"

// Every fused multiply-add below is written out: with contraction left to the
// compiler, instantiations with different pixels-per-lane fused differently
// and images depended on the tile size in the last bit.
#pragma clang fp contract(off)

namespace hgs {

namespace {

constexpr float kTwoOverSqrtPi = 1.12837916709551257390f;

// erfc(x) from the Chebyshev-fitted form of Numerical Recipes (Press et al.,
// 2nd ed., Sec. 6.2, "erfcc"): erfc(z) = t exp(-z^2 + P(t)), t = 1/(1 + z/2)
// for z = |x|, fractional error below 1.2e-7 everywhere; erfc(-z) = 2 -
// erfc(z).  Branch-free (one v_rcp, one exp2, ten fma), so the lanes
// of a wavefront never diverge on the argument's range.  Result in [0, 2].
__device__ __forceinline__ float erfc_fast(float x) {
  const float z = fabsf(x);
  const float t = __builtin_amdgcn_rcpf(fmaf(0.5f, z, 1.0f));
  float p = 0.17087277f;
  p = fmaf(p, t, -0.82215223f);
  p = fmaf(p, t, 1.48851587f);
  p = fmaf(p, t, -1.13520398f);
  p = fmaf(p, t, 0.27886807f);
  p = fmaf(p, t, -0.18628806f);
  p = fmaf(p, t, 0.09678418f);
  p = fmaf(p, t, 0.37409196f);
  p = fmaf(p, t, 1.00002368f);
  p = fmaf(p, t, -1.26551223f);
  const float e = t * __expf(fmaf(-z, z, p));
  return x >= 0.0f ? e : 2.0f - e;
}

struct Pair {
  bool live;   // in rect and power <= 0
  float dx, dy, G, I, HG, a;
};

// One pixel against one record.  Pure function of its inputs, so the forward
// and backward passes take identical decisions.  `amax_half` is
// max(alpha2, alpha2 + 2 d_o) rounded as below: since I lies in [0, 2] and
// every rounding is monotone, HG <= G * amax_half, so a pair whose bound is
// already below alpha_min is skipped without the half factor -- the same
// decision the full evaluation takes.
__device__ __forceinline__ void eval_pair(const Record& r, float amax_half, int px, int py,
                                          float alpha_min, float alpha_max, Pair& P) {
  const int x0 = (int)(r.xr & 0xffffu), x1 = (int)(r.xr >> 16);
  const int y0 = (int)(r.yr & 0xffffu), y1 = (int)(r.yr >> 16);
  P.live = px >= x0 && px <= x1 && py >= y0 && py <= y1;
  if (!P.live) return;
  P.dx = ((float)(px - x0) + 0.5f) - r.mx;
  P.dy = ((float)(py - y0) + 0.5f) - r.my;
  const float quad = fmaf(r.qa * P.dx, P.dx, (r.qc * P.dy) * P.dy);
  const float power = fmaf(-0.5f, quad, -((r.qb * P.dx) * P.dy));
  P.live = !(power > 0.0f);
  if (!P.live) return;
  P.G = __expf(power);
  if (P.G * amax_half < alpha_min) {  // cannot reach alpha_min
    P.a = 0.0f;
    P.HG = 0.0f;
    P.I = 1.0f;
    return;
  }
  if (r.d_o != 0.0f) {
    P.I = erfc_fast(-fmaf(r.kx, P.dx, r.ky * P.dy));
    P.HG = fmaf(r.d_o, P.I, r.alpha2) * P.G;
  } else {
    P.I = 1.0f;
    P.HG = r.alpha2 * P.G;
  }
  P.a = fminf(alpha_max, P.HG);
}

__device__ __forceinline__ float half_bound(const Record& r) {
  return fmaxf(r.alpha2, fmaf(r.d_o, 2.0f, r.alpha2));
}

template <int T>
struct Geometry {
  static constexpr int SUB = (T == 8) ? 8 : 16;       // pixels per wavefront side
  static constexpr int PPL = SUB * SUB / 64;          // pixels per lane
  static constexpr int WAVES = (T / SUB) * (T / SUB); // wavefronts per tile
  static constexpr int ROWSTEP = 64 / SUB;            // rows between a lane's pixels
};

__device__ __forceinline__ Record load_record(const Record* __restrict__ rec, uint32_t id) {
  return rec[id];
}

// Sum over the 64 lanes; the total lands in lane 63.
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ float dpp(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, ROW_MASK, 0xf, true));
}
__device__ __forceinline__ float wave_sum_last(float v) {
  v += dpp<0xb1, 0xf>(v);   // quad_perm [1,0,3,2]
  v += dpp<0x4e, 0xf>(v);   // quad_perm [2,3,0,1]
  v += dpp<0x124, 0xf>(v);  // row_ror:4
  v += dpp<0x128, 0xf>(v);  // row_ror:8   (every lane holds its row's sum)
  v += dpp<0x142, 0xa>(v);  // row_bcast:15 into rows 1 and 3
  v += dpp<0x143, 0xc>(v);  // row_bcast:31 into rows 2 and 3
  return v;
}

__device__ __forceinline__ int wave_max(int v) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) {
    const int o = __shfl_xor(v, m, 64);
    v = o > v ? o : v;
  }
  return v;
}

// One wavefront's block of pixels (sub-block `wave` of `tile`), front to back.
template <int T, int IPL>
__device__ __forceinline__ void fwd_block(
    const Record* __restrict__ rec, const uint32_t* __restrict__ vals,
    const uint32_t* __restrict__ ranges, const CamPack& cp, const Opts& o, float* __restrict__ img,
    float* __restrict__ T_final, int32_t* __restrict__ last_idx, int32_t* __restrict__ n_contrib,
    uint32_t tile, int wave, int lane) {
  using Gm = Geometry<T>;
  constexpr int PPL = Gm::PPL;
  if (tile >= cp.tiles_total) return;  // never index past the tile arrays
  const int c = cam_of_tile(cp, tile);
  const CamDev& cam = cp.cam[c];
  const uint32_t lt = tile - cam.tile_off;
  const int ty = (int)(lt / (uint32_t)cam.tiles_x);
  const int tx = (int)(lt - (uint32_t)ty * (uint32_t)cam.tiles_x);
  const int ox = tx * T + (wave % (T / Gm::SUB)) * Gm::SUB;
  const int oy = ty * T + (wave / (T / Gm::SUB)) * Gm::SUB;
  const int px = ox + lane % Gm::SUB;
  int py[PPL];
  bool inside[PPL];
  float Tr[PPL], C0[PPL], C1[PPL], C2[PPL];
  int32_t cnt[PPL], last[PPL];
  bool done[PPL];
#pragma unroll
  for (int j = 0; j < PPL; ++j) {
    py[j] = oy + lane / Gm::SUB + j * Gm::ROWSTEP;
    inside[j] = px < cam.width && py[j] < cam.height;
    Tr[j] = 1.0f;
    C0[j] = C1[j] = C2[j] = 0.0f;
    cnt[j] = 0;
    last[j] = -1;
    done[j] = !inside[j];
  }
  // the tile's list; positions below are indices into it (fit int32: a
  // list holds at most one entry per record)
  const uint32_t* __restrict__ lst = vals + ranges[2 * tile];
  const int64_t len = (int64_t)ranges[2 * tile + 1] - (int64_t)ranges[2 * tile];
  const float amin = o.alpha_min, amax = o.alpha_max, tmin = o.t_min;

  for (int64_t base = 0; base < len; base += 64 * IPL) {
    bool any = false;
#pragma unroll
    for (int j = 0; j < PPL; ++j) any |= !done[j];
    if (__ballot(any) == 0ull) break;
    uint32_t ids[IPL];
#pragma unroll
    for (int k = 0; k < IPL; ++k) {
      const int64_t p = base + k * 64 + lane;
      ids[k] = p < len ? lst[p] : 0u;
    }
    const int64_t nb = (len - base) < (int64_t)(64 * IPL) ? (len - base) : (int64_t)(64 * IPL);
#pragma unroll
    for (int k = 0; k < IPL; ++k) {
      const int lim = (int)nb - k * 64;
      if (lim <= 0) break;
      const int cntk = lim < 64 ? lim : 64;
      for (int l = 0; l < cntk; ++l) {
        const uint32_t id = (uint32_t)__builtin_amdgcn_readlane((int)ids[k], l);
        const Record r = load_record(rec, id);
        const float hb = half_bound(r);
        const int32_t pos = (int32_t)(base + k * 64 + l);
#pragma unroll
        for (int j = 0; j < PPL; ++j) {
          if (done[j]) continue;
          Pair P;
          eval_pair(r, hb, px, py[j], amin, amax, P);
          if (!P.live || P.a < amin) continue;
          const float Tn = Tr[j] * (1.0f - P.a);
          if (Tn < tmin) {
            done[j] = true;
            continue;
          }
          const float w = P.a * Tr[j];
          C0[j] = fmaf(r.r, w, C0[j]);
          C1[j] = fmaf(r.g, w, C1[j]);
          C2[j] = fmaf(r.b, w, C2[j]);
          Tr[j] = Tn;
          ++cnt[j];
          last[j] = pos;
        }
      }
    }
  }
  const uint64_t plane = (uint64_t)cam.width * cam.height;
  float* im = img + 3 * cam.pix_off;
#pragma unroll
  for (int j = 0; j < PPL; ++j) {
    if (!inside[j]) continue;
    const uint64_t pix = (uint64_t)py[j] * cam.width + px;
    im[pix] = fmaf(Tr[j], o.bg[0], C0[j]);
    im[plane + pix] = fmaf(Tr[j], o.bg[1], C1[j]);
    im[2 * plane + pix] = fmaf(Tr[j], o.bg[2], C2[j]);
    T_final[cam.pix_off + pix] = Tr[j];
    last_idx[cam.pix_off + pix] = last[j];
    n_contrib[cam.pix_off + pix] = cnt[j];
  }
}

// Next work item of a persistent wavefront: (tile of rank w in `order`, sub-block).
__device__ __forceinline__ uint32_t next_work(uint32_t* counter, int lane) {
  uint32_t w = 0;
  if (lane == 0) w = atomicAdd(counter, 1u);
  return (uint32_t)__builtin_amdgcn_readfirstlane((int)w);
}

template <int T, int IPL>
__global__ __launch_bounds__(64 * Geometry<T>::WAVES) void render_fwd_kernel(
    const Record* __restrict__ rec, const uint32_t* __restrict__ vals,
    const uint32_t* __restrict__ ranges, CamPack cp, Opts o, float* __restrict__ img,
    float* __restrict__ T_final, int32_t* __restrict__ last_idx, int32_t* __restrict__ n_contrib) {
  fwd_block<T, IPL>(rec, vals, ranges, cp, o, img, T_final, last_idx, n_contrib, blockIdx.x,
                    threadIdx.x >> 6, threadIdx.x & 63);
}

// Persistent form: one wavefront per workgroup, a grid sized to the chip;
// every wavefront takes work items (tile rank, sub-block) from a counter,
// tiles in `order` (longest list first) so that long tiles do not start last.
template <int T, int IPL>
__global__ __launch_bounds__(64) void render_fwd_persistent_kernel(
    const Record* __restrict__ rec, const uint32_t* __restrict__ vals,
    const uint32_t* __restrict__ ranges, const uint32_t* __restrict__ order, CamPack cp, Opts o,
    float* __restrict__ img, float* __restrict__ T_final, int32_t* __restrict__ last_idx,
    int32_t* __restrict__ n_contrib, uint32_t* __restrict__ counter) {
  constexpr uint32_t WAVES = Geometry<T>::WAVES;
  const uint32_t n_work = cp.tiles_total * WAVES;
  const int lane = threadIdx.x & 63;
  for (uint32_t w = next_work(counter, lane); w < n_work; w = next_work(counter, lane))
    fwd_block<T, IPL>(rec, vals, ranges, cp, o, img, T_final, last_idx, n_contrib, order[w / WAVES],
                      (int)(w % WAVES), lane);
}

// One wavefront's block of pixels, back to front.
template <int T, int IPL>
__device__ __forceinline__ void bwd_block(
    const Record* __restrict__ rec, const uint32_t* __restrict__ vals,
    const uint32_t* __restrict__ ranges, const CamPack& cp, const Opts& o,
    const float* __restrict__ T_final, const int32_t* __restrict__ last_idx,
    const float* __restrict__ dL_dimg, float* __restrict__ rgrad, uint32_t tile, int wave, int lane) {
  using Gm = Geometry<T>;
  constexpr int PPL = Gm::PPL;
  if (tile >= cp.tiles_total) return;  // never index past the tile arrays
  const int c = cam_of_tile(cp, tile);
  const CamDev& cam = cp.cam[c];
  const uint32_t lt = tile - cam.tile_off;
  const int ty = (int)(lt / (uint32_t)cam.tiles_x);
  const int tx = (int)(lt - (uint32_t)ty * (uint32_t)cam.tiles_x);
  const int ox = tx * T + (wave % (T / Gm::SUB)) * Gm::SUB;
  const int oy = ty * T + (wave / (T / Gm::SUB)) * Gm::SUB;
  const int px = ox + lane % Gm::SUB;
  const uint64_t plane = (uint64_t)cam.width * cam.height;
  const float* g = dL_dimg + 3 * cam.pix_off;

  int py[PPL];
  int32_t last[PPL];
  float Tf[PPL], Tr[PPL], dL0[PPL], dL1[PPL], dL2[PPL];
  float acc0[PPL], acc1[PPL], acc2[PPL], la[PPL], lc0[PPL], lc1[PPL], lc2[PPL], bgdot[PPL];
  int top = -1;
#pragma unroll
  for (int j = 0; j < PPL; ++j) {
    py[j] = oy + lane / Gm::SUB + j * Gm::ROWSTEP;
    const bool inside = px < cam.width && py[j] < cam.height;
    last[j] = -1;
    Tf[j] = 1.0f;
    dL0[j] = dL1[j] = dL2[j] = 0.0f;
    if (inside) {
      const uint64_t pix = (uint64_t)py[j] * cam.width + px;
      Tf[j] = T_final[cam.pix_off + pix];
      last[j] = last_idx[cam.pix_off + pix];
      dL0[j] = g[pix];
      dL1[j] = g[plane + pix];
      dL2[j] = g[2 * plane + pix];
    }
    Tr[j] = Tf[j];
    acc0[j] = acc1[j] = acc2[j] = 0.0f;
    la[j] = lc0[j] = lc1[j] = lc2[j] = 0.0f;
    bgdot[j] = o.bg[0] * dL0[j] + o.bg[1] * dL1[j] + o.bg[2] * dL2[j];
    top = last[j] > top ? last[j] : top;
  }
  top = wave_max(top);
  if (top < 0) return;
  const uint32_t* __restrict__ lst = vals + ranges[2 * tile];
  const float amin = o.alpha_min, amax = o.alpha_max;

  // list indices top, top-1, ..., 0 in rounds of 64 * IPL
  for (int32_t hi = top; hi >= 0; hi -= 64 * IPL) {
    uint32_t ids[IPL];
#pragma unroll
    for (int k = 0; k < IPL; ++k) {
      const int32_t p = hi - (k * 64 + lane);
      ids[k] = p >= 0 ? lst[p] : 0u;
    }
    const int32_t nb = (hi + 1) < 64 * IPL ? (hi + 1) : 64 * IPL;
#pragma unroll
    for (int k = 0; k < IPL; ++k) {
      const int lim = nb - k * 64;
      if (lim <= 0) break;
      const int cntk = lim < 64 ? lim : 64;
      for (int l = 0; l < cntk; ++l) {
        const uint32_t id = (uint32_t)__builtin_amdgcn_readlane((int)ids[k], l);
        const Record r = load_record(rec, id);
        const float hb = half_bound(r);
        const int32_t pos = hi - (k * 64 + l);
        float gs[HGS_RECORD_GRAD_FLOATS];
#pragma unroll
        for (int q = 0; q < HGS_RECORD_GRAD_FLOATS; ++q) gs[q] = 0.0f;
        bool any = false;
#pragma unroll
        for (int j = 0; j < PPL; ++j) {
          if (pos > last[j]) continue;
          Pair P;
          eval_pair(r, hb, px, py[j], amin, amax, P);
          if (!P.live || P.a < amin) continue;
          any = true;
          const float a = P.a;
          const float Tb = Tr[j] / (1.0f - a);
          const float wcol = a * Tb;
          gs[9] += wcol * dL0[j];
          gs[10] += wcol * dL1[j];
          gs[11] += wcol * dL2[j];
          acc0[j] = la[j] * lc0[j] + (1.0f - la[j]) * acc0[j];
          acc1[j] = la[j] * lc1[j] + (1.0f - la[j]) * acc1[j];
          acc2[j] = la[j] * lc2[j] + (1.0f - la[j]) * acc2[j];
          la[j] = a;
          lc0[j] = r.r;
          lc1[j] = r.g;
          lc2[j] = r.b;
          float dLda = ((r.r - acc0[j]) * dL0[j] + (r.g - acc1[j]) * dL1[j] + (r.b - acc2[j]) * dL2[j]) * Tb;
          dLda += -Tf[j] / (1.0f - a) * bgdot[j];
          Tr[j] = Tb;
          const float dHG = (P.HG > amax) ? 0.0f : dLda;
          const float dG = dHG * (r.alpha2 + r.d_o * P.I);
          gs[7] += dHG * P.G;
          gs[8] += dHG * P.I * P.G;
          float du = 0.0f;
          if (r.d_o != 0.0f) {
            const float u = r.kx * P.dx + r.ky * P.dy;
            du = dHG * r.d_o * P.G * kTwoOverSqrtPi * __expf(-u * u);
          }
          gs[5] += du * P.dx;
          gs[6] += du * P.dy;
          const float GG = dG * P.G;
          gs[0] += GG * (r.qa * P.dx + r.qb * P.dy) - du * r.kx;
          gs[1] += GG * (r.qb * P.dx + r.qc * P.dy) - du * r.ky;
          gs[2] += -0.5f * GG * P.dx * P.dx;
          gs[3] += -GG * P.dx * P.dy;
          gs[4] += -0.5f * GG * P.dy * P.dy;
        }
        if (__ballot(any) == 0ull) continue;
#pragma unroll
        for (int q = 0; q < HGS_RECORD_GRAD_FLOATS; ++q) gs[q] = wave_sum_last(gs[q]);
        if (lane == 63) {
          float* dst = rgrad + (uint64_t)id * HGS_RECORD_GRAD_FLOATS;
#pragma unroll
          for (int q = 0; q < HGS_RECORD_GRAD_FLOATS; ++q)
            if (gs[q] != 0.0f) atomicAdd(dst + q, gs[q]);
        }
      }
    }
  }
}

template <int T, int IPL>
__global__ __launch_bounds__(64 * Geometry<T>::WAVES) void render_bwd_kernel(
    const Record* __restrict__ rec, const uint32_t* __restrict__ vals,
    const uint32_t* __restrict__ ranges, CamPack cp, Opts o, const float* __restrict__ T_final,
    const int32_t* __restrict__ last_idx, const float* __restrict__ dL_dimg,
    float* __restrict__ rgrad) {
  bwd_block<T, IPL>(rec, vals, ranges, cp, o, T_final, last_idx, dL_dimg, rgrad, blockIdx.x,
                    threadIdx.x >> 6, threadIdx.x & 63);
}

template <int T, int IPL>
__global__ __launch_bounds__(64) void render_bwd_persistent_kernel(
    const Record* __restrict__ rec, const uint32_t* __restrict__ vals,
    const uint32_t* __restrict__ ranges, const uint32_t* __restrict__ order, CamPack cp, Opts o,
    const float* __restrict__ T_final, const int32_t* __restrict__ last_idx,
    const float* __restrict__ dL_dimg, float* __restrict__ rgrad, uint32_t* __restrict__ counter) {
  constexpr uint32_t WAVES = Geometry<T>::WAVES;
  const uint32_t n_work = cp.tiles_total * WAVES;
  const int lane = threadIdx.x & 63;
  for (uint32_t w = next_work(counter, lane); w < n_work; w = next_work(counter, lane))
    bwd_block<T, IPL>(rec, vals, ranges, cp, o, T_final, last_idx, dL_dimg, rgrad, order[w / WAVES],
                      (int)(w % WAVES), lane);
}

__global__ void clear_counter_kernel(uint32_t* __restrict__ p) { *p = 0u; }

__global__ void zero_f32_kernel(float* __restrict__ p, int64_t n) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = t; i < n; i += stride) p[i] = 0.0f;
}

// Workgroups of the persistent grid: as many one-wavefront workgroups as
// the chip keeps resident, never more than there are work items.
template <typename F>
unsigned persistent_grid(F kernel, uint32_t n_work) {
  int dev = 0, cus = 0, per_cu = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    cus = 256;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, 64, 0) != hipSuccess || per_cu < 1)
    per_cu = 8;
  const uint64_t g = (uint64_t)cus * (uint64_t)per_cu;
  return (unsigned)(g < n_work ? g : (n_work > 0 ? n_work : 1));
}

template <int T, int B>
hipError_t fwd_launch(const Record* rec, const uint32_t* vals, const uint32_t* ranges,
                      const uint32_t* order, const CamPack& cp, const Opts& o, float* img, float* Tf,
                      int32_t* li, int32_t* nc, void* ws, hipStream_t s) {
  if (order) {
    uint32_t* counter = static_cast<uint32_t*>(ws);
    hipLaunchKernelGGL(clear_counter_kernel, dim3(1), dim3(1), 0, s, counter);
    const uint32_t n_work = cp.tiles_total * Geometry<T>::WAVES;
    hipLaunchKernelGGL((render_fwd_persistent_kernel<T, B / 64>),
                       dim3(persistent_grid(render_fwd_persistent_kernel<T, B / 64>, n_work)), dim3(64), 0,
                       s, rec, vals, ranges, order, cp, o, img, Tf, li, nc, counter);
  } else {
    hipLaunchKernelGGL((render_fwd_kernel<T, B / 64>), dim3(cp.tiles_total), dim3(64 * Geometry<T>::WAVES),
                       0, s, rec, vals, ranges, cp, o, img, Tf, li, nc);
  }
  return hipGetLastError();
}

template <int T, int B>
hipError_t bwd_launch(const Record* rec, const uint32_t* vals, const uint32_t* ranges,
                      const uint32_t* order, const CamPack& cp, const Opts& o, const float* Tf,
                      const int32_t* li, const float* dL, float* rg, void* ws, hipStream_t s) {
  if (order) {
    uint32_t* counter = static_cast<uint32_t*>(ws) + 1;
    hipLaunchKernelGGL(clear_counter_kernel, dim3(1), dim3(1), 0, s, counter);
    const uint32_t n_work = cp.tiles_total * Geometry<T>::WAVES;
    hipLaunchKernelGGL((render_bwd_persistent_kernel<T, B / 64>),
                       dim3(persistent_grid(render_bwd_persistent_kernel<T, B / 64>, n_work)), dim3(64), 0,
                       s, rec, vals, ranges, order, cp, o, Tf, li, dL, rg, counter);
  } else {
    hipLaunchKernelGGL((render_bwd_kernel<T, B / 64>), dim3(cp.tiles_total), dim3(64 * Geometry<T>::WAVES),
                       0, s, rec, vals, ranges, cp, o, Tf, li, dL, rg);
  }
  return hipGetLastError();
}

#define HGS_DISPATCH(T_, B_, CALL) \
  if (o.tile == T_ && o.batch == B_) return CALL<T_, B_>

}  // namespace

size_t render_workspace_bytes() { return 256; }

hipError_t launch_render_fwd(const Record* rec, const uint32_t* vals, const uint32_t* ranges,
                             const uint32_t* tile_order, const CamPack& cp, const Opts& o,
                             float* img, float* T_final, int32_t* last_idx, int32_t* n_contrib,
                             void* ws, hipStream_t s) {
  if (cp.tiles_total == 0) return hipSuccess;
#define ARGS (rec, vals, ranges, tile_order, cp, o, img, T_final, last_idx, n_contrib, ws, s)
  HGS_DISPATCH(8, 128, fwd_launch) ARGS;
  HGS_DISPATCH(8, 256, fwd_launch) ARGS;
  HGS_DISPATCH(8, 512, fwd_launch) ARGS;
  HGS_DISPATCH(16, 128, fwd_launch) ARGS;
  HGS_DISPATCH(16, 256, fwd_launch) ARGS;
  HGS_DISPATCH(16, 512, fwd_launch) ARGS;
  HGS_DISPATCH(32, 128, fwd_launch) ARGS;
  HGS_DISPATCH(32, 256, fwd_launch) ARGS;
  HGS_DISPATCH(32, 512, fwd_launch) ARGS;
#undef ARGS
  return hipErrorInvalidValue;
}

hipError_t launch_zero_f32(float* p, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  int64_t g = (n + 255) / 256;
  g = g < 1 ? 1 : (g > 8192 ? 8192 : g);
  hipLaunchKernelGGL(zero_f32_kernel, dim3((unsigned)g), dim3(256), 0, s, p, n);
  return hipGetLastError();
}

hipError_t launch_render_bwd(const Record* rec, const uint32_t* vals, const uint32_t* ranges,
                             const uint32_t* tile_order, const CamPack& cp, const Opts& o,
                             const float* T_final, const int32_t* last_idx, const float* dL_dimg,
                             float* rec_grads, void* ws, hipStream_t s) {
  if (cp.tiles_total == 0) return hipSuccess;
#define ARGS (rec, vals, ranges, tile_order, cp, o, T_final, last_idx, dL_dimg, rec_grads, ws, s)
  HGS_DISPATCH(8, 128, bwd_launch) ARGS;
  HGS_DISPATCH(8, 256, bwd_launch) ARGS;
  HGS_DISPATCH(8, 512, bwd_launch) ARGS;
  HGS_DISPATCH(16, 128, bwd_launch) ARGS;
  HGS_DISPATCH(16, 256, bwd_launch) ARGS;
  HGS_DISPATCH(16, 512, bwd_launch) ARGS;
  HGS_DISPATCH(32, 128, bwd_launch) ARGS;
  HGS_DISPATCH(32, 256, bwd_launch) ARGS;
  HGS_DISPATCH(32, 512, bwd_launch) ARGS;
#undef ARGS
  return hipErrorInvalidValue;
}

}  // namespace hgs
