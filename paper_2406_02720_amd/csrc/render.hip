// Tile rasterizer: per-pixel front-to-back blending with the paired-half
// opacity of Eq. 10, and its back-to-front replay for gradients.
//
// One workgroup owns one tile (T x T pixels, one thread per pixel: 1, 4 or 16
// wavefronts).  The tile's sorted list is consumed in batches of BATCH
// records that the workgroup stages in LDS (64 bytes each, four 16-byte
// slots), so every record is read from HBM once per tile and then broadcast
// to all pixels from LDS.  Blending stops per pixel before the kernel that
// would take the transmittance below t_min, and the tile stops when all its
// pixels have.  For each pixel the forward pass keeps only the final
// transmittance, the position of the last blended entry and the count; the
// backward pass recomputes each pair from the records and walks the list
// backwards, dividing the transmittance back out.

#include "hgs_internal.h"

namespace hgs {

namespace {

struct Pair {
  bool live;   // in rect and power <= 0
  float dx, dy, G, I, HG, a;
};

__device__ __forceinline__ bool in_rect(uint32_t xr, uint32_t yr, int px, int py) {
  const int x0 = (int)(xr & 0xffffu), x1 = (int)(xr >> 16);
  const int y0 = (int)(yr & 0xffffu), y1 = (int)(yr >> 16);
  return px >= x0 && px <= x1 && py >= y0 && py <= y1;
}

__device__ __forceinline__ void eval_pair(const float4& q0, const float4& q1, const float4& q3,
                                          float d_o, int px, int py, float alpha_max, Pair& P) {
  const uint32_t xr = __float_as_uint(q3.x), yr = __float_as_uint(q3.y);
  P.live = in_rect(xr, yr, px, py);
  if (!P.live) return;
  P.dx = (float)(px - (int)(xr & 0xffffu)) + 0.5f - q0.x;
  P.dy = (float)(py - (int)(yr & 0xffffu)) + 0.5f - q0.y;
  const float power = -0.5f * (q1.x * P.dx * P.dx + q1.z * P.dy * P.dy) - q1.y * P.dx * P.dy;
  P.live = !(power > 0.0f);
  if (!P.live) return;
  P.G = __expf(power);
  if (d_o != 0.0f) {
    P.I = erfcf(-(q0.z * P.dx + q0.w * P.dy));
    P.HG = (q1.w + d_o * P.I) * P.G;
  } else {
    P.I = 1.0f;
    P.HG = q1.w * P.G;
  }
  P.a = fminf(alpha_max, P.HG);
}

template <int T, int BATCH>
__global__ __launch_bounds__(T* T) void render_fwd_kernel(
    const Record* __restrict__ rec, const uint32_t* __restrict__ vals,
    const uint32_t* __restrict__ ranges, CamPack cp, Opts o, float* __restrict__ img,
    float* __restrict__ T_final, int32_t* __restrict__ last_idx, int32_t* __restrict__ n_contrib) {
  constexpr int NT = T * T;
  __shared__ float4 s_q[4][BATCH];
  const uint32_t tile = blockIdx.x;
  const int c = cam_of_tile(cp, tile);
  const CamDev& cam = cp.cam[c];
  const uint32_t lt = tile - cam.tile_off;
  const int ty = (int)(lt / (uint32_t)cam.tiles_x);
  const int tx = (int)(lt - (uint32_t)ty * (uint32_t)cam.tiles_x);
  const int px = tx * T + (int)(threadIdx.x % T);
  const int py = ty * T + (int)(threadIdx.x / T);
  const bool inside = px < cam.width && py < cam.height;
  const uint32_t start = ranges[2 * tile], end = ranges[2 * tile + 1];

  float Tr = 1.0f, C0 = 0.0f, C1 = 0.0f, C2 = 0.0f;
  int32_t count = 0, last = -1;
  bool done = !inside;
  const float amin = o.alpha_min, amax = o.alpha_max, tmin = o.t_min;

  for (uint32_t b = start; b < end; b += BATCH) {
    if (__syncthreads_count(done) == NT) break;
    const uint32_t nb = (end - b) < (uint32_t)BATCH ? (end - b) : (uint32_t)BATCH;
    for (uint32_t j = threadIdx.x; j < nb; j += NT) {
      const float4* rp = reinterpret_cast<const float4*>(rec + vals[b + j]);
      s_q[0][j] = rp[0];
      s_q[1][j] = rp[1];
      s_q[2][j] = rp[2];
      s_q[3][j] = rp[3];
    }
    __syncthreads();
    if (!done) {
      for (uint32_t j = 0; j < nb; ++j) {
        const float4 q2 = s_q[2][j];
        Pair P;
        eval_pair(s_q[0][j], s_q[1][j], s_q[3][j], q2.w, px, py, amax, P);
        if (!P.live || P.a < amin) continue;
        const float Tn = Tr * (1.0f - P.a);
        if (Tn < tmin) {
          done = true;
          break;
        }
        const float w = P.a * Tr;
        C0 += q2.x * w;
        C1 += q2.y * w;
        C2 += q2.z * w;
        Tr = Tn;
        ++count;
        last = (int32_t)(b + j);
      }
    }
  }
  if (inside) {
    const uint64_t plane = (uint64_t)cam.width * cam.height;
    const uint64_t pix = (uint64_t)py * cam.width + px;
    float* im = img + 3 * cam.pix_off;
    im[pix] = C0 + Tr * o.bg[0];
    im[plane + pix] = C1 + Tr * o.bg[1];
    im[2 * plane + pix] = C2 + Tr * o.bg[2];
    T_final[cam.pix_off + pix] = Tr;
    last_idx[cam.pix_off + pix] = last;
    n_contrib[cam.pix_off + pix] = count;
  }
}

__device__ __forceinline__ float wave_sum(float x) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) x += __shfl_xor(x, m, 64);
  return x;
}

template <int T, int BATCH>
__global__ __launch_bounds__(T* T) void render_bwd_kernel(
    const Record* __restrict__ rec, const uint32_t* __restrict__ vals,
    const uint32_t* __restrict__ ranges, CamPack cp, Opts o, const float* __restrict__ T_final,
    const int32_t* __restrict__ last_idx, const float* __restrict__ dL_dimg,
    float* __restrict__ rgrad) {
  constexpr int NT = T * T;
  __shared__ float4 s_q[4][BATCH];
  __shared__ uint32_t s_id[BATCH];
  __shared__ int32_t s_max;
  const uint32_t tile = blockIdx.x;
  const int c = cam_of_tile(cp, tile);
  const CamDev& cam = cp.cam[c];
  const uint32_t lt = tile - cam.tile_off;
  const int ty = (int)(lt / (uint32_t)cam.tiles_x);
  const int tx = (int)(lt - (uint32_t)ty * (uint32_t)cam.tiles_x);
  const int px = tx * T + (int)(threadIdx.x % T);
  const int py = ty * T + (int)(threadIdx.x / T);
  const bool inside = px < cam.width && py < cam.height;
  const uint32_t start = ranges[2 * tile];

  float Tf = 1.0f, dL0 = 0.0f, dL1 = 0.0f, dL2 = 0.0f;
  int32_t last = -1;
  if (inside) {
    const uint64_t plane = (uint64_t)cam.width * cam.height;
    const uint64_t pix = (uint64_t)py * cam.width + px;
    Tf = T_final[cam.pix_off + pix];
    last = last_idx[cam.pix_off + pix];
    const float* g = dL_dimg + 3 * cam.pix_off;
    dL0 = g[pix];
    dL1 = g[plane + pix];
    dL2 = g[2 * plane + pix];
  }
  if (threadIdx.x == 0) s_max = -1;
  __syncthreads();
  if (last >= 0) atomicMax(&s_max, last);
  __syncthreads();
  const int32_t top = s_max;
  if (top < 0) return;

  const float amin = o.alpha_min, amax = o.alpha_max;
  const float bgdot = o.bg[0] * dL0 + o.bg[1] * dL1 + o.bg[2] * dL2;
  float Tr = Tf;
  float acc0 = 0.0f, acc1 = 0.0f, acc2 = 0.0f;
  float la = 0.0f, lc0 = 0.0f, lc1 = 0.0f, lc2 = 0.0f;
  const float kTwoOverSqrtPi = 1.12837916709551257390f;

  for (int64_t bend = (int64_t)top + 1; bend > (int64_t)start; bend -= BATCH) {
    const int64_t bbeg = bend - BATCH > (int64_t)start ? bend - BATCH : (int64_t)start;
    const uint32_t nb = (uint32_t)(bend - bbeg);
    __syncthreads();
    for (uint32_t j = threadIdx.x; j < nb; j += NT) {
      const uint32_t id = vals[bbeg + j];
      const float4* rp = reinterpret_cast<const float4*>(rec + id);
      s_id[j] = id;
      s_q[0][j] = rp[0];
      s_q[1][j] = rp[1];
      s_q[2][j] = rp[2];
      s_q[3][j] = rp[3];
    }
    __syncthreads();
    for (int j = (int)nb - 1; j >= 0; --j) {
      const int64_t pos = bbeg + j;
      const float4 q0 = s_q[0][j], q1 = s_q[1][j], q2 = s_q[2][j];
      Pair P;
      bool contrib = false;
      if (pos <= last) {
        eval_pair(q0, q1, s_q[3][j], q2.w, px, py, amax, P);
        contrib = P.live && P.a >= amin;
      }
      if (__ballot(contrib) == 0ull) continue;
      float g[HGS_RECORD_GRAD_FLOATS];
#pragma unroll
      for (int k = 0; k < HGS_RECORD_GRAD_FLOATS; ++k) g[k] = 0.0f;
      if (contrib) {
        const float a = P.a;
        const float Tb = Tr / (1.0f - a);
        const float wcol = a * Tb;
        g[9] = wcol * dL0;
        g[10] = wcol * dL1;
        g[11] = wcol * dL2;
        acc0 = la * lc0 + (1.0f - la) * acc0;
        acc1 = la * lc1 + (1.0f - la) * acc1;
        acc2 = la * lc2 + (1.0f - la) * acc2;
        la = a;
        lc0 = q2.x;
        lc1 = q2.y;
        lc2 = q2.z;
        float dLda = ((q2.x - acc0) * dL0 + (q2.y - acc1) * dL1 + (q2.z - acc2) * dL2) * Tb;
        dLda += -Tf / (1.0f - a) * bgdot;
        Tr = Tb;
        const float dHG = (P.HG > amax) ? 0.0f : dLda;
        const float d_o = q2.w;
        const float dG = dHG * (q1.w + d_o * P.I);
        g[7] = dHG * P.G;
        g[8] = dHG * P.I * P.G;
        float du = 0.0f;
        if (d_o != 0.0f) {
          const float u = q0.z * P.dx + q0.w * P.dy;
          du = dHG * d_o * P.G * kTwoOverSqrtPi * __expf(-u * u);
        }
        g[5] = du * P.dx;
        g[6] = du * P.dy;
        const float GG = dG * P.G;
        g[0] = GG * (q1.x * P.dx + q1.y * P.dy) - du * q0.z;
        g[1] = GG * (q1.y * P.dx + q1.z * P.dy) - du * q0.w;
        g[2] = -0.5f * GG * P.dx * P.dx;
        g[3] = -GG * P.dx * P.dy;
        g[4] = -0.5f * GG * P.dy * P.dy;
      }
#pragma unroll
      for (int k = 0; k < HGS_RECORD_GRAD_FLOATS; ++k) g[k] = wave_sum(g[k]);
      if ((threadIdx.x & 63) == 0) {
        float* dst = rgrad + (uint64_t)s_id[j] * HGS_RECORD_GRAD_FLOATS;
#pragma unroll
        for (int k = 0; k < HGS_RECORD_GRAD_FLOATS; ++k)
          if (g[k] != 0.0f) atomicAdd(dst + k, g[k]);
      }
    }
  }
}

__global__ void zero_f32_kernel(float* __restrict__ p, int64_t n) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = t; i < n; i += stride) p[i] = 0.0f;
}

template <int T, int B>
hipError_t fwd_launch(const Record* rec, const uint32_t* vals, const uint32_t* ranges,
                      const CamPack& cp, const Opts& o, float* img, float* Tf, int32_t* li,
                      int32_t* nc, hipStream_t s) {
  hipLaunchKernelGGL((render_fwd_kernel<T, B>), dim3(cp.tiles_total), dim3(T * T), 0, s, rec, vals,
                     ranges, cp, o, img, Tf, li, nc);
  return hipGetLastError();
}

template <int T, int B>
hipError_t bwd_launch(const Record* rec, const uint32_t* vals, const uint32_t* ranges,
                      const CamPack& cp, const Opts& o, const float* Tf, const int32_t* li,
                      const float* dL, float* rg, hipStream_t s) {
  hipLaunchKernelGGL((render_bwd_kernel<T, B>), dim3(cp.tiles_total), dim3(T * T), 0, s, rec, vals,
                     ranges, cp, o, Tf, li, dL, rg);
  return hipGetLastError();
}

#define HGS_DISPATCH(T_, B_, CALL)        \
  if (o.tile == T_ && o.batch == B_) return CALL<T_, B_>

}  // namespace

size_t render_workspace_bytes() { return 256; }

hipError_t launch_render_fwd(const Record* rec, const uint32_t* vals, const uint32_t* ranges,
                             const CamPack& cp, const Opts& o, float* img, float* T_final,
                             int32_t* last_idx, int32_t* n_contrib, void* ws, hipStream_t s) {
  (void)ws;
  if (cp.tiles_total == 0) return hipSuccess;
#define ARGS (rec, vals, ranges, cp, o, img, T_final, last_idx, n_contrib, s)
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

hipError_t launch_render_bwd(const Record* rec, const uint32_t* vals, const uint32_t* ranges,
                             const CamPack& cp, const Opts& o, const float* T_final,
                             const int32_t* last_idx, const float* dL_dimg, float* rec_grads,
                             int64_t n_rec, void* ws, hipStream_t s) {
  (void)ws;
  {
    const int64_t n = n_rec * HGS_RECORD_GRAD_FLOATS;
    int64_t g = (n + 255) / 256;
    g = g < 1 ? 1 : (g > 8192 ? 8192 : g);
    hipLaunchKernelGGL(zero_f32_kernel, dim3((unsigned)g), dim3(256), 0, s, rec_grads, n);
  }
  if (cp.tiles_total == 0) return hipGetLastError();
#define ARGS (rec, vals, ranges, cp, o, T_final, last_idx, dL_dimg, rec_grads, s)
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
