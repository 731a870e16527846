// The optimisation step after the rasterizer's backward pass (Sec. 4,
// implementation; Supp., training settings): Adam on the raw parameters
// with the activation chain rule fused in, the densification statistics
// gathered from the per-record gradients, clone / split / prune with the
// half-Gaussian thresholds, and the opacity reset.  Everything here is
// elementwise or a scan: HBM-bound, one pass over each plane.

#include <math.h>

#include "hgs_internal.h"

namespace hgs {
namespace {

constexpr int kBlock = 256;

// What a plane of the hgs_params layout is: its field, activation and
// learning-rate group.
enum Act : int { kIdentity = 0, kExp = 1, kSigmoid = 2 };

struct PlaneSets {
  // raw (in/out), gradient (activated space), first and second moment,
  // activated output
  float* raw[7];
  const float* grad[7];
  float* m[7];
  float* v[7];
  float* act[7];
};

__device__ __forceinline__ void plane_of(int p, int* field, int* sub) {
  // means 3, scales 3, quats 4, normals 3, opac1 1, opac2 1, sh rest
  if (p < 3) { *field = 0; *sub = p; }
  else if (p < 6) { *field = 1; *sub = p - 3; }
  else if (p < 10) { *field = 2; *sub = p - 6; }
  else if (p < 13) { *field = 3; *sub = p - 10; }
  else if (p == 13) { *field = 4; *sub = 0; }
  else if (p == 14) { *field = 5; *sub = 0; }
  else { *field = 6; *sub = p - 15; }
}

__device__ __forceinline__ float activate(float x, int act) {
  if (act == kExp) return expf(x);
  if (act == kSigmoid) return 1.0f / (1.0f + expf(-x));
  return x;
}

// One Adam step on plane blockIdx.y, four kernels per thread.  The
// gradient arrives with respect to the activated value and is carried to
// the raw one (exp: times exp(x); sigmoid: times s (1 - s)).  The update is
// raw -= (lr / (1 - b1^t)) m / (sqrt(v) / sqrt(1 - b2^t) + eps).
__global__ __launch_bounds__(kBlock) void adam_kernel(PlaneSets ps, int64_t n, int64_t stride, AdamPlan plan) {
  const int p = blockIdx.y;
  int field, sub;
  plane_of(p, &field, &sub);
  const int act = field == 1 ? kExp : (field == 4 || field == 5) ? kSigmoid : kIdentity;
  const float step = plan.step_size[field == 6 ? (sub < 3 ? 6 : 7) : field];
  const int64_t off = (int64_t)sub * stride;
  float* raw = ps.raw[field] + off;
  const float* grad = ps.grad[field] + off;
  float* m = ps.m[field] + off;
  float* v = ps.v[field] + off;
  float* out = ps.act[field] == ps.raw[field] ? nullptr : ps.act[field] + off;
  const float b1 = plan.beta1, b2 = plan.beta2, c1 = 1.0f - plan.beta1, c2 = 1.0f - plan.beta2;
  const float inv_sc2 = plan.inv_sqrt_bc2, eps = plan.eps;
  const int64_t i0 = ((int64_t)blockIdx.x * kBlock + threadIdx.x) * 4;
  if (i0 >= n) return;
  const int cnt = n - i0 >= 4 ? 4 : (int)(n - i0);
  float x[4], g[4], mm[4], vv[4];
  if (cnt == 4 && plan.vec4) {
    const float4 a = *(const float4*)(raw + i0), b = *(const float4*)(grad + i0);
    const float4 c = *(const float4*)(m + i0), d = *(const float4*)(v + i0);
    x[0] = a.x; x[1] = a.y; x[2] = a.z; x[3] = a.w;
    g[0] = b.x; g[1] = b.y; g[2] = b.z; g[3] = b.w;
    mm[0] = c.x; mm[1] = c.y; mm[2] = c.z; mm[3] = c.w;
    vv[0] = d.x; vv[1] = d.y; vv[2] = d.z; vv[3] = d.w;
  } else {
    for (int j = 0; j < 4; ++j) {
      const bool ok = j < cnt;
      x[j] = ok ? raw[i0 + j] : 0.0f;
      g[j] = ok ? grad[i0 + j] : 0.0f;
      mm[j] = ok ? m[i0 + j] : 0.0f;
      vv[j] = ok ? v[i0 + j] : 0.0f;
    }
  }
  float y[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    float gr = g[j];
    if (act == kExp) gr *= expf(x[j]);
    else if (act == kSigmoid) {
      const float s = 1.0f / (1.0f + expf(-x[j]));
      gr *= s * (1.0f - s);
    }
    mm[j] = b1 * mm[j] + c1 * gr;
    vv[j] = b2 * vv[j] + c2 * (gr * gr);
    x[j] -= step * (mm[j] / (sqrtf(vv[j]) * inv_sc2 + eps));
    y[j] = activate(x[j], act);
  }
  if (cnt == 4 && plan.vec4) {
    *(float4*)(raw + i0) = make_float4(x[0], x[1], x[2], x[3]);
    *(float4*)(m + i0) = make_float4(mm[0], mm[1], mm[2], mm[3]);
    *(float4*)(v + i0) = make_float4(vv[0], vv[1], vv[2], vv[3]);
    if (out) *(float4*)(out + i0) = make_float4(y[0], y[1], y[2], y[3]);
  } else {
    for (int j = 0; j < cnt; ++j) {
      raw[i0 + j] = x[j];
      m[i0 + j] = mm[j];
      v[i0 + j] = vv[j];
      if (out) out[i0 + j] = y[j];
    }
  }
}

// Activated planes from raw ones (planes whose output aliases the input
// are identities and are skipped).
__global__ __launch_bounds__(kBlock) void activate_kernel(PlaneSets ps, int64_t n, int64_t stride) {
  const int p = blockIdx.y;
  int field, sub;
  plane_of(p, &field, &sub);
  if (ps.act[field] == ps.raw[field]) return;
  const int act = field == 1 ? kExp : (field == 4 || field == 5) ? kSigmoid : kIdentity;
  const int64_t off = (int64_t)sub * stride;
  const float* raw = ps.raw[field] + off;
  float* out = ps.act[field] + off;
  const int64_t s = (int64_t)gridDim.x * kBlock;
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += s) out[i] = activate(raw[i], act);
}

// Opacity reset: each half's logit capped at logit(value); its moments
// cleared; the activated opacity refreshed when an output is given.
__global__ __launch_bounds__(kBlock) void reset_opacity_kernel(PlaneSets ps, int64_t n, float cap) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
#pragma unroll
  for (int f = 4; f <= 5; ++f) {
    const float x = fminf(ps.raw[f][i], cap);
    ps.raw[f][i] = x;
    ps.m[f][i] = 0.0f;
    ps.v[f][i] = 0.0f;
    if (ps.act[f] && ps.act[f] != ps.raw[f]) ps.act[f][i] = 1.0f / (1.0f + expf(-x));
  }
}

// Densification statistics, one thread per kernel over the cameras: for
// every camera whose record of the kernel is visible (tiles > 0), the norm
// of the centre gradient in normalised device coordinates (the pixel
// gradient times W/2 and H/2) is added and the view counted; the largest
// screen radius ceil(kappa sqrt(lambda_max)) of the dilated screen
// covariance (from the record's conic, in FP64, uncontracted) is kept.
__global__ __launch_bounds__(kBlock) void densify_stats_kernel(const Record* __restrict__ rec,
                                                               const float* __restrict__ rgrad, CamPack cp,
                                                               int64_t n, double kappa, float* __restrict__ accum,
                                                               int32_t* __restrict__ count,
                                                               float* __restrict__ max_radii) {
#pragma clang fp contract(off)
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  float acc = accum[i];
  int32_t cnt = count[i];
  float rad = max_radii[i];
  for (int c = 0; c < cp.n_cams; ++c) {
    const int64_t ri = (int64_t)c * n + i;
    const uint4 q3 = *(const uint4*)&rec[ri].xr;
    if (q3.w == 0u) continue;
    const float4 q1 = *(const float4*)&rec[ri].qa;
    const float2 gm = *(const float2*)&rgrad[ri * HGS_RECORD_GRAD_FLOATS];
    const float gx = gm.x * (0.5f * (float)cp.cam[c].width);
    const float gy = gm.y * (0.5f * (float)cp.cam[c].height);
    acc += sqrtf(gx * gx + gy * gy);
    cnt += 1;
    const double a = q1.x, b = q1.y, cc = q1.z;
    const double mid = 0.5 * (a + cc);
    const double d = 0.25 * ((a - cc) * (a - cc)) + b * b;
    const double lam_min = mid - sqrt(d > 0.0 ? d : 0.0);
    const double r = ceil(kappa * sqrt(1.0 / lam_min));
    rad = (float)r > rad ? (float)r : rad;
  }
  accum[i] = acc;
  count[i] = cnt;
  max_radii[i] = rad;
}

// Densify decisions per kernel: bit 0 keep (neither split nor pruned),
// bit 1 clone kept, bit 2 split children kept.  Thresholds arrive in the
// raw domain (log of a scale, logit of an opacity), in FP64.
__global__ __launch_bounds__(kBlock) void densify_flags_kernel(PlaneSets ps, int64_t n, int64_t stride,
                                                               DensifyPlan dp, const float* __restrict__ accum,
                                                               const int32_t* __restrict__ count,
                                                               const float* __restrict__ max_radii,
                                                               uint32_t* __restrict__ f_keep,
                                                               uint32_t* __restrict__ f_clone,
                                                               uint32_t* __restrict__ f_child) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  const float* ls = ps.raw[1];
  const float s0 = ls[i], s1 = ls[stride + i], s2 = ls[2 * stride + i];
  const float smax = fmaxf(fmaxf(s0, s1), s2);
  const double omax = fmax((double)ps.raw[4][i], (double)ps.raw[5][i]);
  const int32_t cnt = count[i];
  const bool big = cnt > 0 && (double)accum[i] >= dp.grad_threshold * (double)cnt;
  const bool small = (double)smax <= dp.log_dense;
  const bool clone = big && small, split = big && !small;
  const bool transparent = omax < dp.logit_min_opacity;
  const bool wide = dp.world_on && (double)smax > dp.log_world;
  const bool pruned = transparent || wide || (dp.screen_on && (double)max_radii[i] > dp.max_screen);
  const float cmax = fmaxf(fmaxf(s0 - dp.shrink, s1 - dp.shrink), s2 - dp.shrink);
  const bool child_pruned = transparent || (dp.world_on && (double)cmax > dp.log_world);
  f_keep[i] = (!split && !pruned) ? 1u : 0u;
  f_clone[i] = (clone && !transparent && !wide) ? 1u : 0u;
  f_child[i] = (split && !child_pruned) ? 1u : 0u;
}

// quaternion (w, x, y, z), any length (zero: identity) -> rotation matrix
__device__ inline void rotation(float w, float x, float y, float z, float R[9]) {
  const float l2 = w * w + x * x + y * y + z * z;
  if (!(l2 > 0.0f)) {
    w = 1.0f; x = y = z = 0.0f;
  } else {
    const float il = 1.0f / sqrtf(l2);
    w *= il; x *= il; y *= il; z *= il;
  }
  R[0] = 1.0f - 2.0f * (y * y + z * z); R[1] = 2.0f * (x * y - w * z); R[2] = 2.0f * (x * z + w * y);
  R[3] = 2.0f * (x * y + w * z); R[4] = 1.0f - 2.0f * (x * x + z * z); R[5] = 2.0f * (y * z - w * x);
  R[6] = 2.0f * (x * z - w * y); R[7] = 2.0f * (y * z + w * x); R[8] = 1.0f - 2.0f * (x * x + y * y);
}

// Writes the kept kernels, the clones and the children at their scanned
// positions: [kept | clones | first children | second children].  A thread
// owns one kernel and a group of kWriteGroup planes (grid y is the group):
// the flags and destinations are read once per group, the group's loads are
// all issued before its stores, and every plane is read and written in
// coalesced runs.  New kernels get zero moments; a child's centre is
// mean + R (scale * z), its log-scales the parent's minus log(0.8 * 2).
constexpr int kWriteGroup = 8;

__global__ __launch_bounds__(kBlock) void densify_write_kernel(
    PlaneSets in, PlaneSets out, int64_t n, int64_t stride, int64_t stride_out, int planes, float shrink,
    const float* __restrict__ samples, const uint32_t* __restrict__ f_keep, const uint32_t* __restrict__ f_clone,
    const uint32_t* __restrict__ f_child, const uint64_t* __restrict__ o_keep, const uint64_t* __restrict__ o_clone,
    const uint64_t* __restrict__ o_child, const uint64_t* __restrict__ totals, int64_t capacity,
    int64_t* __restrict__ n_out, int32_t* __restrict__ overflow) {
  const uint64_t nk = totals[0], nc = totals[1], nh = totals[2];
  const uint64_t total = nk + nc + 2 * nh;
  const int p0 = (int)blockIdx.y * kWriteGroup;
  const int np = planes - p0 < kWriteGroup ? planes - p0 : kWriteGroup;
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (blockIdx.y == 0 && i == 0) {
    *n_out = (int64_t)total;
    *overflow = total > (uint64_t)capacity ? 1 : 0;
  }
  if (i >= n || total > (uint64_t)capacity) return;
  const bool keep = f_keep[i] != 0u, clone = f_clone[i] != 0u, child = f_child[i] != 0u;
  if (!keep && !clone && !child) return;
  const int64_t dk = keep ? (int64_t)o_keep[i] : 0;
  const int64_t dc = clone ? (int64_t)(nk + o_clone[i]) : 0;
  const int64_t d0 = child ? (int64_t)(nk + nc + o_child[i]) : 0;
  const int64_t d1 = d0 + (int64_t)nh;

  float x[kWriteGroup], mm[kWriteGroup], vv[kWriteGroup];
#pragma unroll
  for (int k = 0; k < kWriteGroup; ++k) {
    x[k] = mm[k] = vv[k] = 0.0f;
    if (k < np) {
      int field, sub;
      plane_of(p0 + k, &field, &sub);
      const int64_t io = (int64_t)sub * stride + i;
      x[k] = in.raw[field][io];
      if (keep) {
        mm[k] = in.m[field][io];
        vv[k] = in.v[field][io];
      }
    }
  }
  // the children's centre offsets R (scale * z); the means are planes 0..2,
  // so only group 0 needs them
  float dmu[2][3] = {{0.0f, 0.0f, 0.0f}, {0.0f, 0.0f, 0.0f}};
  if (child && p0 == 0) {
    float R[9];
    rotation(in.raw[2][i], in.raw[2][stride + i], in.raw[2][2 * stride + i], in.raw[2][3 * stride + i], R);
    float sz[3];
    for (int c = 0; c < 2; ++c) {
      for (int a = 0; a < 3; ++a)
        sz[a] = samples[((int64_t)c * 3 + a) * n + i] * expf(in.raw[1][(int64_t)a * stride + i]);
      for (int a = 0; a < 3; ++a) dmu[c][a] = R[3 * a] * sz[0] + R[3 * a + 1] * sz[1] + R[3 * a + 2] * sz[2];
    }
  }
#pragma unroll
  for (int k = 0; k < kWriteGroup; ++k) {
    if (k >= np) break;
    int field, sub;
    plane_of(p0 + k, &field, &sub);
    const int64_t po = (int64_t)sub * stride_out;
    if (keep) {
      out.raw[field][po + dk] = x[k];
      out.m[field][po + dk] = mm[k];
      out.v[field][po + dk] = vv[k];
    }
    if (clone) {
      out.raw[field][po + dc] = x[k];
      out.m[field][po + dc] = 0.0f;
      out.v[field][po + dc] = 0.0f;
    }
    if (child) {
      float y0 = x[k], y1 = x[k];
      if (field == 1) {
        y0 = y1 = x[k] - shrink;
      } else if (field == 0) {          // then p0 == 0 and sub == k
        y0 = x[k] + dmu[0][k < 3 ? k : 0];
        y1 = x[k] + dmu[1][k < 3 ? k : 0];
      }
      out.raw[field][po + d0] = y0;
      out.m[field][po + d0] = 0.0f;
      out.v[field][po + d0] = 0.0f;
      out.raw[field][po + d1] = y1;
      out.m[field][po + d1] = 0.0f;
      out.v[field][po + d1] = 0.0f;
    }
  }
}

// Gradient of scale * sum |img - target| with respect to the images:
// scale * sign(img - target), and optionally the loss itself (block sums,
// one float atomic per block).
__global__ __launch_bounds__(kBlock) void l1_grad_kernel(const float* __restrict__ img,
                                                         const float* __restrict__ tgt, int64_t n, float inv_n,
                                                         float* __restrict__ dL, float* __restrict__ loss) {
  __shared__ float s_sum[kBlock / 64];
  float acc = 0.0f;
  const int64_t stride = (int64_t)gridDim.x * kBlock;
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += stride) {
    const float d = img[i] - tgt[i];
    dL[i] = d > 0.0f ? inv_n : (d < 0.0f ? -inv_n : 0.0f);
    acc += fabsf(d);
  }
  if (!loss) return;
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) acc += __shfl_xor(acc, off, 64);
  if ((threadIdx.x & 63) == 0) s_sum[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    float t = 0.0f;
    for (int w = 0; w < kBlock / 64; ++w) t += s_sum[w];
    atomicAdd(loss, t * inv_n);
  }
}

PlaneSets make_sets(const Grads& raw, const float* const* grad, const Grads& m, const Grads& v, const Grads& act) {
  PlaneSets ps{};
  float* const r[7] = {raw.means, raw.scales, raw.quats, raw.normals, raw.opac1, raw.opac2, raw.sh};
  float* const mm[7] = {m.means, m.scales, m.quats, m.normals, m.opac1, m.opac2, m.sh};
  float* const vv[7] = {v.means, v.scales, v.quats, v.normals, v.opac1, v.opac2, v.sh};
  float* const aa[7] = {act.means, act.scales, act.quats, act.normals, act.opac1, act.opac2, act.sh};
  for (int f = 0; f < 7; ++f) {
    ps.raw[f] = r[f];
    ps.grad[f] = grad ? grad[f] : nullptr;
    ps.m[f] = mm[f];
    ps.v[f] = vv[f];
    ps.act[f] = aa[f];
  }
  return ps;
}

unsigned blocks_for(int64_t n, int64_t per) { return (unsigned)((n + per - 1) / per > 0 ? (n + per - 1) / per : 1); }

}  // namespace

int planes_of(int sh_degree) { return 15 + 3 * (sh_degree + 1) * (sh_degree + 1); }

hipError_t launch_adam(const Grads& raw, const float* const grad[7], const Grads& m, const Grads& v,
                       const Grads& act, int64_t n, int64_t stride, int sh_degree, const AdamPlan& plan,
                       hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const PlaneSets ps = make_sets(raw, grad, m, v, act);
  hipLaunchKernelGGL(adam_kernel, dim3(blocks_for(n, 4 * kBlock), planes_of(sh_degree)), dim3(kBlock), 0, s, ps,
                     n, stride, plan);
  return hipGetLastError();
}

hipError_t launch_activate(const Grads& raw, const Grads& act, int64_t n, int64_t stride, int sh_degree,
                           hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const PlaneSets ps = make_sets(raw, nullptr, raw, raw, act);
  const unsigned bx = blocks_for(n, kBlock) < 1024u ? blocks_for(n, kBlock) : 1024u;
  hipLaunchKernelGGL(activate_kernel, dim3(bx, planes_of(sh_degree)), dim3(kBlock), 0, s, ps, n, stride);
  return hipGetLastError();
}

hipError_t launch_reset_opacity(const Grads& raw, const Grads& m, const Grads& v, const Grads& act, int64_t n,
                                float cap, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const PlaneSets ps = make_sets(raw, nullptr, m, v, act);
  hipLaunchKernelGGL(reset_opacity_kernel, dim3(blocks_for(n, kBlock)), dim3(kBlock), 0, s, ps, n, cap);
  return hipGetLastError();
}

hipError_t launch_densify_stats(const Record* rec, const float* rgrad, const CamPack& cp, int64_t n, double kappa,
                                float* accum, int32_t* count, float* max_radii, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(densify_stats_kernel, dim3(blocks_for(n, kBlock)), dim3(kBlock), 0, s, rec, rgrad, cp, n,
                     kappa, accum, count, max_radii);
  return hipGetLastError();
}

hipError_t launch_l1_grad(const float* img, const float* tgt, int64_t n, float scale, float* dL, float* loss,
                          hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const unsigned grid = blocks_for(n, 4 * kBlock) < 4096u ? blocks_for(n, 4 * kBlock) : 4096u;
  hipLaunchKernelGGL(l1_grad_kernel, dim3(grid), dim3(kBlock), 0, s, img, tgt, n, scale, dL, loss);
  return hipGetLastError();
}

size_t densify_workspace_bytes(int64_t n) {
  const size_t a = ((size_t)(n > 0 ? n : 1) * sizeof(uint32_t) + 255) & ~(size_t)255;
  const size_t b = ((size_t)(n > 0 ? n : 1) * sizeof(uint64_t) + 255) & ~(size_t)255;
  return 3 * a + 3 * b + 256 + ((scan_workspace_bytes(n) + 255) & ~(size_t)255);
}

hipError_t launch_densify(const Grads& raw, const Grads& m, const Grads& v, int64_t n, int64_t stride,
                          int sh_degree, const DensifyPlan& dp, const float* accum, const int32_t* count,
                          const float* max_radii, const float* samples, int64_t capacity, int64_t stride_out,
                          const Grads& raw_out, const Grads& m_out, const Grads& v_out, int64_t* n_out,
                          int32_t* overflow, void* ws, hipStream_t s) {
  const int64_t nn = n > 0 ? n : 1;
  const size_t a = ((size_t)nn * sizeof(uint32_t) + 255) & ~(size_t)255;
  const size_t b = ((size_t)nn * sizeof(uint64_t) + 255) & ~(size_t)255;
  char* p = (char*)ws;
  uint32_t* f[3];
  uint64_t* o[3];
  for (int k = 0; k < 3; ++k) { f[k] = (uint32_t*)p; p += a; }
  for (int k = 0; k < 3; ++k) { o[k] = (uint64_t*)p; p += b; }
  uint64_t* totals = (uint64_t*)p;
  p += 256;
  void* scan_ws = p;
  const PlaneSets in = make_sets(raw, nullptr, m, v, raw);
  const PlaneSets out = make_sets(raw_out, nullptr, m_out, v_out, raw_out);
  if (n > 0)
    hipLaunchKernelGGL(densify_flags_kernel, dim3(blocks_for(n, kBlock)), dim3(kBlock), 0, s, in, n, stride, dp,
                       accum, count, max_radii, f[0], f[1], f[2]);
  for (int k = 0; k < 3; ++k) {
    const hipError_t e = launch_scan(f[k], n, o[k], totals + k, scan_ws, s);
    if (e != hipSuccess) return e;
  }
  const int planes = planes_of(sh_degree);
  hipLaunchKernelGGL(densify_write_kernel, dim3(blocks_for(n, kBlock), (planes + kWriteGroup - 1) / kWriteGroup),
                     dim3(kBlock), 0, s, in, out, n, stride, stride_out, planes, dp.shrink, samples, f[0], f[1], f[2],
                     o[0], o[1], o[2], totals, capacity, n_out, overflow);
  return hipGetLastError();
}

}  // namespace hgs
