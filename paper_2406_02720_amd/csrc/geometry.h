// FP64 per-(kernel, camera) geometry of a half-Gaussian, used by the forward
// projection and recomputed by its backward.
//
// Forward (per kernel i and camera c):
//   t       = R_c mu + t_c                         camera space
//   Sigma_w = R(q) diag(s^2) R(q)^T                Eq. 2
//   J       = d(screen)/d(camera) with x/z, y/z clamped to fov_clamp times
//             the half field of view               Eq. 3 (two screen rows)
//   M       = J R_c                                world -> screen, 2x3
//   Shat    = M Sigma_w M^T + lowpass I            Eq. 6 (+ dilation)
//   Q       = Shat^-1 = (a, b, c)                  conic
//   g       = M Sigma_w n,  v = n^T Sigma_w n      covariance of the screen
//                                                  offset with the plane
//                                                  value, plane variance
//   k       = Q g / sqrt(2 (v - g^T Q g))          half factor
//             I(delta) = erfc(-k . delta)          Eq. 7-8 (camera-space,
//                                                  sign-safe form)
// The conditional variance is clamped to >= 1e-12 v.  All array indices are
// compile-time constants so that everything stays in registers.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>

#include "hgs_internal.h"

namespace hgs {

// Symmetric 3x3.
struct Sym3 {
  double xx, xy, xz, yy, yz, zz;
};

__device__ __forceinline__ void sym_mul_vec(const Sym3& S, const double* v, double* out) {
  out[0] = S.xx * v[0] + S.xy * v[1] + S.xz * v[2];
  out[1] = S.xy * v[0] + S.yy * v[1] + S.yz * v[2];
  out[2] = S.xz * v[0] + S.yz * v[1] + S.zz * v[2];
}

// u^T S w
__device__ __forceinline__ double sym_form(const Sym3& S, const double* u, const double* w) {
  double Sw[3];
  sym_mul_vec(S, w, Sw);
  return u[0] * Sw[0] + u[1] * Sw[1] + u[2] * Sw[2];
}

// Real spherical harmonics up to degree D with the Condon-Shortley phase,
// ordered l = 0..D, m = -l..l; the normalisations are the textbook ones.
namespace shc {
constexpr double c0 = 0.28209479177387814347;   // 1/(2 sqrt(pi))
constexpr double c1 = 0.48860251190291992159;   // sqrt(3/(4 pi))
constexpr double a2 = 1.09254843059207907054;   // sqrt(15/pi)/2
constexpr double b2 = 0.31539156525252000603;   // sqrt(5/pi)/4
constexpr double c2 = 0.54627421529603953527;   // sqrt(15/pi)/4
constexpr double k33 = 0.59004358992664351035;  // sqrt(35/(2 pi))/4
constexpr double k32 = 2.89061144264055405538;  // sqrt(105/pi)/2
constexpr double k31 = 0.45704579946446573616;  // sqrt(21/(2 pi))/4
constexpr double k30 = 0.37317633259011539141;  // sqrt(7/pi)/4
constexpr double k22 = 1.44530572132027702769;  // sqrt(105/pi)/4
}  // namespace shc

template <int D, typename F>
__device__ __forceinline__ void sh_eval(F x, F y, F z, F* Y) {
  using namespace shc;
  Y[0] = (F)c0;
  if constexpr (D >= 1) {
    Y[1] = (F)(-c1) * y;
    Y[2] = (F)c1 * z;
    Y[3] = (F)(-c1) * x;
  }
  if constexpr (D >= 2) {
    const F xx = x * x, yy = y * y, zz = z * z;
    Y[4] = (F)a2 * x * y;
    Y[5] = (F)(-a2) * y * z;
    Y[6] = (F)b2 * ((F)2 * zz - xx - yy);
    Y[7] = (F)(-a2) * x * z;
    Y[8] = (F)c2 * (xx - yy);
  }
  if constexpr (D >= 3) {
    const F xx = x * x, yy = y * y, zz = z * z;
    Y[9] = (F)(-k33) * y * ((F)3 * xx - yy);
    Y[10] = (F)k32 * x * y * z;
    Y[11] = (F)(-k31) * y * ((F)4 * zz - xx - yy);
    Y[12] = (F)k30 * z * ((F)2 * zz - (F)3 * xx - (F)3 * yy);
    Y[13] = (F)(-k31) * x * ((F)4 * zz - xx - yy);
    Y[14] = (F)k22 * z * (xx - yy);
    Y[15] = (F)(-k33) * x * (xx - (F)3 * yy);
  }
}

// Gradient of sum_k wk * Y_k(x, y, z) with respect to (x, y, z), the three
// components taken as independent variables.
template <int D, typename F>
__device__ __forceinline__ void sh_grad(F x, F y, F z, const F* wk, F* gx, F* gy, F* gz) {
  using namespace shc;
  F X = 0, Yv = 0, Z = 0;
  if constexpr (D >= 1) {
    Yv += (F)(-c1) * wk[1];
    Z += (F)c1 * wk[2];
    X += (F)(-c1) * wk[3];
  }
  if constexpr (D >= 2) {
    X += (F)a2 * y * wk[4];
    Yv += (F)a2 * x * wk[4];
    Yv += (F)(-a2) * z * wk[5];
    Z += (F)(-a2) * y * wk[5];
    X += (F)(-2.0 * b2) * x * wk[6];
    Yv += (F)(-2.0 * b2) * y * wk[6];
    Z += (F)(4.0 * b2) * z * wk[6];
    X += (F)(-a2) * z * wk[7];
    Z += (F)(-a2) * x * wk[7];
    X += (F)(2.0 * c2) * x * wk[8];
    Yv += (F)(-2.0 * c2) * y * wk[8];
  }
  if constexpr (D >= 3) {
    const F xx = x * x, yy = y * y, zz = z * z;
    X += (F)(-6.0 * k33) * x * y * wk[9];
    Yv += (F)(-k33) * ((F)3 * xx - (F)3 * yy) * wk[9];
    X += (F)k32 * y * z * wk[10];
    Yv += (F)k32 * x * z * wk[10];
    Z += (F)k32 * x * y * wk[10];
    X += (F)(2.0 * k31) * x * y * wk[11];
    Yv += (F)(-k31) * ((F)4 * zz - xx - (F)3 * yy) * wk[11];
    Z += (F)(-8.0 * k31) * y * z * wk[11];
    X += (F)(-6.0 * k30) * x * z * wk[12];
    Yv += (F)(-6.0 * k30) * y * z * wk[12];
    Z += (F)k30 * ((F)6 * zz - (F)3 * xx - (F)3 * yy) * wk[12];
    X += (F)(-k31) * ((F)4 * zz - (F)3 * xx - yy) * wk[13];
    Yv += (F)(2.0 * k31) * x * y * wk[13];
    Z += (F)(-8.0 * k31) * x * z * wk[13];
    X += (F)(2.0 * k22) * x * z * wk[14];
    Yv += (F)(-2.0 * k22) * y * z * wk[14];
    Z += (F)k22 * (xx - yy) * wk[14];
    X += (F)(-k33) * ((F)3 * xx - (F)3 * yy) * wk[15];
    Yv += (F)(6.0 * k33) * x * y * wk[15];
  }
  *gx = X;
  *gy = Yv;
  *gz = Z;
}

// Normalised quaternion (identity for q == 0) and its rotation matrix.
__device__ __forceinline__ void quat_rot(const float* q, double* qh, double& qn, double* R) {
  double qw = q[0], qx = q[1], qy = q[2], qz = q[3];
  qn = sqrt(qw * qw + qx * qx + qy * qy + qz * qz);
  if (qn == 0.0) {
    qw = 1.0; qx = qy = qz = 0.0;
  } else {
    const double iq = 1.0 / qn;
    qw *= iq; qx *= iq; qy *= iq; qz *= iq;
  }
  qh[0] = qw; qh[1] = qx; qh[2] = qy; qh[3] = qz;
  R[0] = 1.0 - 2.0 * (qy * qy + qz * qz);
  R[1] = 2.0 * (qx * qy - qw * qz);
  R[2] = 2.0 * (qx * qz + qw * qy);
  R[3] = 2.0 * (qx * qy + qw * qz);
  R[4] = 1.0 - 2.0 * (qx * qx + qz * qz);
  R[5] = 2.0 * (qy * qz - qw * qx);
  R[6] = 2.0 * (qx * qz - qw * qy);
  R[7] = 2.0 * (qy * qz + qw * qx);
  R[8] = 1.0 - 2.0 * (qx * qx + qy * qy);
}

// Camera-independent part of a kernel.
struct KernelGeo {
  double mu[3];
  Sym3 Sw;        // world covariance
  double nn;      // |n|
  double nh[3];   // unit normal (0 if n == 0)
  double Sn[3];   // Sigma_w n
  double v;       // n^T Sigma_w n
  bool nzero;
  double f;       // 3-D filter variance (0: none)
  double comp3;   // sqrt(det Sigma / det(Sigma + f I))
};

// With a 3-D filter variance f > 0 (Mip-Splatting) the covariance is
// Sigma + f I; comp3 = prod_i s_i / sqrt(s_i^2 + f) is the opacity factor
// sqrt(det Sigma / det(Sigma + f I)) (the eigenvalues of Sigma are s_i^2).
__device__ __forceinline__ void kernel_geo(const float* mu, const float* s, const float* q,
                                           const float* n, KernelGeo& k, double f = 0.0) {
  for (int i = 0; i < 3; ++i) k.mu[i] = (double)mu[i];
  double qh[4], qn, R[9];
  quat_rot(q, qh, qn, R);
  const double d0 = (double)s[0] * s[0], d1 = (double)s[1] * s[1], d2 = (double)s[2] * s[2];
  k.Sw.xx = R[0] * d0 * R[0] + R[1] * d1 * R[1] + R[2] * d2 * R[2];
  k.Sw.xy = R[0] * d0 * R[3] + R[1] * d1 * R[4] + R[2] * d2 * R[5];
  k.Sw.xz = R[0] * d0 * R[6] + R[1] * d1 * R[7] + R[2] * d2 * R[8];
  k.Sw.yy = R[3] * d0 * R[3] + R[4] * d1 * R[4] + R[5] * d2 * R[5];
  k.Sw.yz = R[3] * d0 * R[6] + R[4] * d1 * R[7] + R[5] * d2 * R[8];
  k.Sw.zz = R[6] * d0 * R[6] + R[7] * d1 * R[7] + R[8] * d2 * R[8];
  k.f = f;
  k.comp3 = 1.0;
  if (f > 0.0) {
    k.Sw.xx += f;
    k.Sw.yy += f;
    k.Sw.zz += f;
    k.comp3 = sqrt(d0 / (d0 + f)) * sqrt(d1 / (d1 + f)) * sqrt(d2 / (d2 + f));
  }
  const double nx = n[0], ny = n[1], nz = n[2];
  k.nn = sqrt(nx * nx + ny * ny + nz * nz);
  k.nzero = !(k.nn > 0.0);
  const double inv = k.nzero ? 0.0 : 1.0 / k.nn;
  k.nh[0] = nx * inv; k.nh[1] = ny * inv; k.nh[2] = nz * inv;
  sym_mul_vec(k.Sw, k.nh, k.Sn);
  k.v = k.nh[0] * k.Sn[0] + k.nh[1] * k.Sn[1] + k.nh[2] * k.Sn[2];
}

// Alg. 1 (Supp. B.1): covariance of the flattened ellipsoid standing for the
// splitting plane.  In the plane it is the Gaussian's planar cross-section,
// the covariance conditioned on a zero plane value,
// S0 = Sigma - (Sigma n)(Sigma n)^T / (n^T Sigma n) -- in Alg. 1's basis
// (v1, v2, n) the Schur complement with a zero row and column for n; along n
// it gets the variance min(a', c') / 100, where a' and c' are S0's variances
// along v1 and v2.  Sigma n and n^T Sigma n are the kernel's Sn and v.
__device__ __forceinline__ Sym3 splitting_cov(const KernelGeo& k) {
  const double iv = 1.0 / k.v;
  const double* Sn = k.Sn;
  Sym3 S;
  S.xx = k.Sw.xx - Sn[0] * Sn[0] * iv;
  S.xy = k.Sw.xy - Sn[0] * Sn[1] * iv;
  S.xz = k.Sw.xz - Sn[0] * Sn[2] * iv;
  S.yy = k.Sw.yy - Sn[1] * Sn[1] * iv;
  S.yz = k.Sw.yz - Sn[1] * Sn[2] * iv;
  S.zz = k.Sw.zz - Sn[2] * Sn[2] * iv;
  // Alg. 1's plane axes: v1 = (ny, -nx, 0) / |.|, v2 = n x v1 / |.|, and
  // (e1, e2) for a normal along z
  const double nx = k.nh[0], ny = k.nh[1], nz = k.nh[2];
  double v1[3], v2[3];
  if (nx == 0.0 && ny == 0.0) {
    v1[0] = 1.0; v1[1] = 0.0; v1[2] = 0.0;
    v2[0] = 0.0; v2[1] = 1.0; v2[2] = 0.0;
  } else {
    const double i1 = 1.0 / sqrt(ny * ny + nx * nx);
    v1[0] = ny * i1; v1[1] = -nx * i1; v1[2] = 0.0;
    const double c0 = ny * v1[2] - nz * v1[1];
    const double c1 = nz * v1[0] - nx * v1[2];
    const double c2 = nx * v1[1] - ny * v1[0];
    const double i2 = 1.0 / sqrt(c0 * c0 + c1 * c1 + c2 * c2);
    v2[0] = c0 * i2; v2[1] = c1 * i2; v2[2] = c2 * i2;
  }
  const double t = fmin(sym_form(S, v1, v1), sym_form(S, v2, v2)) / 100.0;
  S.xx += t * nx * nx;
  S.xy += t * nx * ny;
  S.xz += t * nx * nz;
  S.yy += t * ny * ny;
  S.yz += t * ny * nz;
  S.zz += t * nz * nz;
  return S;
}

// Per-camera part.
struct ViewGeo {
  double t[3];
  double xc, yc;       // clamped x/z, y/z
  bool clx, cly;       // clamp active
  double M[6];         // 2x3 row-major
  double A, B, C;      // dilated screen covariance
  double det;
  double det0;         // determinant of the undilated screen covariance
  double qa, qb, qc;   // conic
  double mx, my;       // screen centre
  double g[2], w[2];
  double s2;
  bool s2clamp;
  double r;            // 1 / sqrt(2 s2)
  double k[2];
};

__device__ __forceinline__ void view_geo(const KernelGeo& k, const CamDev& cam, double lowpass,
                                         double fov_clamp, ViewGeo& vg) {
  const float* R = cam.R;
  for (int r = 0; r < 3; ++r)
    vg.t[r] = (double)R[r * 3 + 0] * k.mu[0] + (double)R[r * 3 + 1] * k.mu[1] +
              (double)R[r * 3 + 2] * k.mu[2] + (double)cam.t[r];
  const double tx = vg.t[0], ty = vg.t[1], tz = vg.t[2];
  const double fx = cam.fx, fy = cam.fy;
  const double lx = fov_clamp * (double)cam.width / (2.0 * fx);
  const double ly = fov_clamp * (double)cam.height / (2.0 * fy);
  const double iz = 1.0 / tz;
  const double rx = tx * iz, ry = ty * iz;
  vg.xc = fmin(fmax(rx, -lx), lx);
  vg.yc = fmin(fmax(ry, -ly), ly);
  vg.clx = !(rx >= -lx && rx <= lx);
  vg.cly = !(ry >= -ly && ry <= ly);
  const double J00 = fx * iz, J02 = -fx * vg.xc * iz;
  const double J11 = fy * iz, J12 = -fy * vg.yc * iz;
  for (int c = 0; c < 3; ++c) {
    vg.M[c] = J00 * (double)R[0 * 3 + c] + J02 * (double)R[2 * 3 + c];
    vg.M[3 + c] = J11 * (double)R[1 * 3 + c] + J12 * (double)R[2 * 3 + c];
  }
  double S0[3], S1[3];  // Sigma_w M^T columns
  sym_mul_vec(k.Sw, vg.M, S0);
  sym_mul_vec(k.Sw, vg.M + 3, S1);
  const double A0 = vg.M[0] * S0[0] + vg.M[1] * S0[1] + vg.M[2] * S0[2];
  const double C0 = vg.M[3] * S1[0] + vg.M[4] * S1[1] + vg.M[5] * S1[2];
  vg.B = vg.M[3] * S0[0] + vg.M[4] * S0[1] + vg.M[5] * S0[2];
  vg.A = A0 + lowpass;
  vg.C = C0 + lowpass;
  vg.det = vg.A * vg.C - vg.B * vg.B;
  vg.det0 = A0 * C0 - vg.B * vg.B;
  const double idet = 1.0 / vg.det;
  vg.qa = vg.C * idet;
  vg.qb = -vg.B * idet;
  vg.qc = vg.A * idet;
  vg.mx = fx * rx + (double)cam.cx;
  vg.my = fy * ry + (double)cam.cy;
  vg.g[0] = vg.M[0] * k.Sn[0] + vg.M[1] * k.Sn[1] + vg.M[2] * k.Sn[2];
  vg.g[1] = vg.M[3] * k.Sn[0] + vg.M[4] * k.Sn[1] + vg.M[5] * k.Sn[2];
  vg.w[0] = vg.qa * vg.g[0] + vg.qb * vg.g[1];
  vg.w[1] = vg.qb * vg.g[0] + vg.qc * vg.g[1];
  const double cond = k.v - (vg.g[0] * vg.w[0] + vg.g[1] * vg.w[1]);
  const double floor_ = 1e-12 * k.v;
  vg.s2clamp = !(cond > floor_);
  vg.s2 = vg.s2clamp ? floor_ : cond;
  if (k.nzero || !(vg.s2 > 0.0)) {
    vg.r = 0.0;
    vg.k[0] = vg.k[1] = 0.0;
  } else {
    vg.r = 1.0 / sqrt(2.0 * vg.s2);
    vg.k[0] = vg.w[0] * vg.r;
    vg.k[1] = vg.w[1] * vg.r;
  }
}

// Camera centre o = -R^T t in world space.
__device__ __forceinline__ void camera_centre(const CamDev& cam, double* oc) {
  const float* R = cam.R;
  for (int a = 0; a < 3; ++a)
    oc[a] = -((double)R[0 * 3 + a] * cam.t[0] + (double)R[1 * 3 + a] * cam.t[1] +
              (double)R[2 * 3 + a] * cam.t[2]);
}

}  // namespace hgs
