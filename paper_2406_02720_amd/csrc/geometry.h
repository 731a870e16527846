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
// The conditional variance is clamped to >= 1e-12 v.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>

#include "hgs_internal.h"

namespace hgs {

// Real spherical harmonics up to degree 3 with the Condon-Shortley phase,
// ordered l = 0..3, m = -l..l; the normalisations are the textbook ones.
struct SHConst {
  static constexpr double PI = 3.14159265358979323846;
};
__device__ __forceinline__ void sh_eval(int deg, double x, double y, double z, double* Y) {
  const double c0 = 0.28209479177387814347;   // 1/(2 sqrt(pi))
  const double c1 = 0.48860251190291992159;   // sqrt(3/(4 pi))
  const double a2 = 1.09254843059207907054;   // sqrt(15/pi)/2
  const double b2 = 0.31539156525252000603;   // sqrt(5/pi)/4
  const double c2 = 0.54627421529603953527;   // sqrt(15/pi)/4
  const double k33 = 0.59004358992664351035;  // sqrt(35/(2 pi))/4
  const double k32 = 2.89061144264055405538;  // sqrt(105/pi)/2
  const double k31 = 0.45704579946446573616;  // sqrt(21/(2 pi))/4
  const double k30 = 0.37317633259011539141;  // sqrt(7/pi)/4
  const double k22 = 1.44530572132027702769;  // sqrt(105/pi)/4
  Y[0] = c0;
  if (deg < 1) return;
  Y[1] = -c1 * y;
  Y[2] = c1 * z;
  Y[3] = -c1 * x;
  if (deg < 2) return;
  const double xx = x * x, yy = y * y, zz = z * z;
  Y[4] = a2 * x * y;
  Y[5] = -a2 * y * z;
  Y[6] = b2 * (2.0 * zz - xx - yy);
  Y[7] = -a2 * x * z;
  Y[8] = c2 * (xx - yy);
  if (deg < 3) return;
  Y[9] = -k33 * y * (3.0 * xx - yy);
  Y[10] = k32 * x * y * z;
  Y[11] = -k31 * y * (4.0 * zz - xx - yy);
  Y[12] = k30 * z * (2.0 * zz - 3.0 * xx - 3.0 * yy);
  Y[13] = -k31 * x * (4.0 * zz - xx - yy);
  Y[14] = k22 * z * (xx - yy);
  Y[15] = -k33 * x * (xx - 3.0 * yy);
}

// Gradient of sum_k wk * Y_k(x, y, z) with respect to (x, y, z), treating
// the three components as independent variables.
__device__ __forceinline__ void sh_grad(int deg, double x, double y, double z, const double* wk,
                                        double* gx, double* gy, double* gz) {
  const double c1 = 0.48860251190291992159;
  const double a2 = 1.09254843059207907054;
  const double b2 = 0.31539156525252000603;
  const double c2 = 0.54627421529603953527;
  const double k33 = 0.59004358992664351035;
  const double k32 = 2.89061144264055405538;
  const double k31 = 0.45704579946446573616;
  const double k30 = 0.37317633259011539141;
  const double k22 = 1.44530572132027702769;
  double X = 0.0, Yv = 0.0, Z = 0.0;
  if (deg >= 1) {
    Yv += -c1 * wk[1];
    Z += c1 * wk[2];
    X += -c1 * wk[3];
  }
  if (deg >= 2) {
    X += a2 * y * wk[4];
    Yv += a2 * x * wk[4];
    Yv += -a2 * z * wk[5];
    Z += -a2 * y * wk[5];
    X += -2.0 * b2 * x * wk[6];
    Yv += -2.0 * b2 * y * wk[6];
    Z += 4.0 * b2 * z * wk[6];
    X += -a2 * z * wk[7];
    Z += -a2 * x * wk[7];
    X += 2.0 * c2 * x * wk[8];
    Yv += -2.0 * c2 * y * wk[8];
  }
  if (deg >= 3) {
    const double xx = x * x, yy = y * y, zz = z * z;
    X += -6.0 * k33 * x * y * wk[9];
    Yv += -k33 * (3.0 * xx - 3.0 * yy) * wk[9];
    X += k32 * y * z * wk[10];
    Yv += k32 * x * z * wk[10];
    Z += k32 * x * y * wk[10];
    X += 2.0 * k31 * x * y * wk[11];
    Yv += -k31 * (4.0 * zz - xx - 3.0 * yy) * wk[11];
    Z += -8.0 * k31 * y * z * wk[11];
    X += -6.0 * k30 * x * z * wk[12];
    Yv += -6.0 * k30 * y * z * wk[12];
    Z += k30 * (6.0 * zz - 3.0 * xx - 3.0 * yy) * wk[12];
    X += -k31 * (4.0 * zz - 3.0 * xx - yy) * wk[13];
    Yv += 2.0 * k31 * x * y * wk[13];
    Z += -8.0 * k31 * x * z * wk[13];
    X += 2.0 * k22 * x * z * wk[14];
    Yv += -2.0 * k22 * y * z * wk[14];
    Z += k22 * (xx - yy) * wk[14];
    X += -k33 * (3.0 * xx - 3.0 * yy) * wk[15];
    Yv += 6.0 * k33 * x * y * wk[15];
  }
  *gx = X;
  *gy = Yv;
  *gz = Z;
}

// Camera-independent part of a kernel.
struct KernelGeo {
  double mu[3];
  double s[3];
  double qn;        // |q|
  double qh[4];     // normalised quaternion (identity if q == 0)
  double Rq[9];     // rotation, row-major
  double Sw[9];     // world covariance, row-major (symmetric)
  double nn;        // |n|
  double nh[3];     // unit normal (0 if n == 0)
  double Sn[3];     // Sigma_w n
  double v;         // n^T Sigma_w n
  bool nzero;
};

__device__ __forceinline__ void kernel_geo(const float* mu, const float* s, const float* q,
                                           const float* n, KernelGeo& k) {
  for (int i = 0; i < 3; ++i) {
    k.mu[i] = (double)mu[i];
    k.s[i] = (double)s[i];
  }
  double qw = q[0], qx = q[1], qy = q[2], qz = q[3];
  k.qn = sqrt(qw * qw + qx * qx + qy * qy + qz * qz);
  if (k.qn == 0.0) {
    qw = 1.0; qx = qy = qz = 0.0;
  } else {
    qw /= k.qn; qx /= k.qn; qy /= k.qn; qz /= k.qn;
  }
  k.qh[0] = qw; k.qh[1] = qx; k.qh[2] = qy; k.qh[3] = qz;
  double* R = k.Rq;
  R[0] = 1.0 - 2.0 * (qy * qy + qz * qz);
  R[1] = 2.0 * (qx * qy - qw * qz);
  R[2] = 2.0 * (qx * qz + qw * qy);
  R[3] = 2.0 * (qx * qy + qw * qz);
  R[4] = 1.0 - 2.0 * (qx * qx + qz * qz);
  R[5] = 2.0 * (qy * qz - qw * qx);
  R[6] = 2.0 * (qx * qz - qw * qy);
  R[7] = 2.0 * (qy * qz + qw * qx);
  R[8] = 1.0 - 2.0 * (qx * qx + qy * qy);
  const double d0 = k.s[0] * k.s[0], d1 = k.s[1] * k.s[1], d2 = k.s[2] * k.s[2];
  for (int r = 0; r < 3; ++r)
    for (int c = r; c < 3; ++c) {
      const double val = R[r * 3 + 0] * d0 * R[c * 3 + 0] + R[r * 3 + 1] * d1 * R[c * 3 + 1] +
                         R[r * 3 + 2] * d2 * R[c * 3 + 2];
      k.Sw[r * 3 + c] = val;
      k.Sw[c * 3 + r] = val;
    }
  const double nx = n[0], ny = n[1], nz = n[2];
  k.nn = sqrt(nx * nx + ny * ny + nz * nz);
  k.nzero = !(k.nn > 0.0);
  const double inv = k.nzero ? 0.0 : 1.0 / k.nn;
  k.nh[0] = nx * inv; k.nh[1] = ny * inv; k.nh[2] = nz * inv;
  for (int r = 0; r < 3; ++r)
    k.Sn[r] = k.Sw[r * 3 + 0] * k.nh[0] + k.Sw[r * 3 + 1] * k.nh[1] + k.Sw[r * 3 + 2] * k.nh[2];
  k.v = k.nh[0] * k.Sn[0] + k.nh[1] * k.Sn[1] + k.nh[2] * k.Sn[2];
}

// Alg. 1 (Supp. B.1): covariance of the flattened ellipsoid standing for the
// splitting plane.  Plane basis (v1, v2, n); the in-plane block is the Schur
// complement of the covariance in that basis; the normal variance is
// min(a', c') / 100.  Output row-major symmetric 3x3.
__device__ __forceinline__ void splitting_cov(const KernelGeo& k, double* S) {
  const double nx = k.nh[0], ny = k.nh[1], nz = k.nh[2];
  double v1[3], v2[3];
  if (nx == 0.0 && ny == 0.0) {
    v1[0] = 1.0; v1[1] = 0.0; v1[2] = 0.0;
    v2[0] = 0.0; v2[1] = 1.0; v2[2] = 0.0;
  } else {
    const double l1 = sqrt(ny * ny + nx * nx);
    v1[0] = ny / l1; v1[1] = -nx / l1; v1[2] = 0.0;
    double c0 = ny * v1[2] - nz * v1[1];
    double c1 = nz * v1[0] - nx * v1[2];
    double c2 = nx * v1[1] - ny * v1[0];
    const double l2 = sqrt(c0 * c0 + c1 * c1 + c2 * c2);
    v2[0] = c0 / l2; v2[1] = c1 / l2; v2[2] = c2 / l2;
  }
  const double B[9] = {v1[0], v2[0], nx, v1[1], v2[1], ny, v1[2], v2[2], nz};  // columns v1 v2 n
  double SB[9];  // Sw * B
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c)
      SB[r * 3 + c] = k.Sw[r * 3 + 0] * B[0 * 3 + c] + k.Sw[r * 3 + 1] * B[1 * 3 + c] +
                      k.Sw[r * 3 + 2] * B[2 * 3 + c];
  double C[9];  // B^T Sw B
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c)
      C[r * 3 + c] = B[0 * 3 + r] * SB[0 * 3 + c] + B[1 * 3 + r] * SB[1 * 3 + c] +
                     B[2 * 3 + r] * SB[2 * 3 + c];
  const double ap = C[0] - C[2] * C[2] / C[8];
  const double bp = C[1] - C[2] * C[5] / C[8];
  const double cp = C[4] - C[5] * C[5] / C[8];
  const double dp = fmin(ap, cp) / 100.0;
  const double Sd[9] = {ap, bp, 0.0, bp, cp, 0.0, 0.0, 0.0, dp};
  double T[9];  // B * Sd
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c)
      T[r * 3 + c] = B[r * 3 + 0] * Sd[0 * 3 + c] + B[r * 3 + 1] * Sd[1 * 3 + c] +
                     B[r * 3 + 2] * Sd[2 * 3 + c];
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c)
      S[r * 3 + c] = T[r * 3 + 0] * B[c * 3 + 0] + T[r * 3 + 1] * B[c * 3 + 1] +
                     T[r * 3 + 2] * B[c * 3 + 2];
}

// Per-camera part.
struct ViewGeo {
  double t[3];
  double xc, yc;       // clamped x/z, y/z
  bool clx, cly;       // clamp active
  double M[6];         // 2x3 row-major
  double A, B, C;      // dilated screen covariance
  double det;
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
  const double rx = tx / tz, ry = ty / tz;
  vg.xc = fmin(fmax(rx, -lx), lx);
  vg.yc = fmin(fmax(ry, -ly), ly);
  vg.clx = !(rx >= -lx && rx <= lx);
  vg.cly = !(ry >= -ly && ry <= ly);
  const double J00 = fx / tz, J02 = -fx * vg.xc / tz;
  const double J11 = fy / tz, J12 = -fy * vg.yc / tz;
  for (int c = 0; c < 3; ++c) {
    vg.M[c] = J00 * (double)R[0 * 3 + c] + J02 * (double)R[2 * 3 + c];
    vg.M[3 + c] = J11 * (double)R[1 * 3 + c] + J12 * (double)R[2 * 3 + c];
  }
  double MS[6];  // M * Sw
  for (int r = 0; r < 2; ++r)
    for (int c = 0; c < 3; ++c)
      MS[r * 3 + c] = vg.M[r * 3 + 0] * k.Sw[0 * 3 + c] + vg.M[r * 3 + 1] * k.Sw[1 * 3 + c] +
                      vg.M[r * 3 + 2] * k.Sw[2 * 3 + c];
  vg.A = MS[0] * vg.M[0] + MS[1] * vg.M[1] + MS[2] * vg.M[2] + lowpass;
  vg.B = MS[0] * vg.M[3] + MS[1] * vg.M[4] + MS[2] * vg.M[5];
  vg.C = MS[3] * vg.M[3] + MS[4] * vg.M[4] + MS[5] * vg.M[5] + lowpass;
  vg.det = vg.A * vg.C - vg.B * vg.B;
  vg.qa = vg.C / vg.det;
  vg.qb = -vg.B / vg.det;
  vg.qc = vg.A / vg.det;
  vg.mx = fx * tx / tz + (double)cam.cx;
  vg.my = fy * ty / tz + (double)cam.cy;
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

}  // namespace hgs
