// Per-(Gaussian, view) projection of the omnidirectional rasterizer and its adjoint, gfx950.
//
// One thread per Gaussian; the thread loops over the views, so the Gaussian's parameters
// (236 bytes at SH degree 3) are read from HBM once per step however many views there are.
// All geometry is evaluated in FP64: the radial depth is a sort key and the footprint rectangle
// decides binning, and both must be bit-identical to an FP64 evaluation of the same formulas.
// On gfx950 FP64 FMA issues at the same rate as non-packed FP32 and this kernel is bound by
// HBM traffic, so double precision costs almost nothing here.
#include <math.h>

#include "common.h"

namespace odgs {
namespace {

constexpr double kPi = 3.14159265358979323846;

struct Params {
  int32_t tile;
  double near_r, far_r, dilation, pole_eps;
};

struct Cam {
  double R[9];
  double t[3];
  double c[3];  // camera centre -R^T t
};

__device__ inline void load_cam(const float* __restrict__ cams, int v, Cam& c) {
#pragma unroll
  for (int k = 0; k < 9; ++k) c.R[k] = (double)cams[v * 12 + k];
#pragma unroll
  for (int k = 0; k < 3; ++k) c.t[k] = (double)cams[v * 12 + 9 + k];
#pragma unroll
  for (int k = 0; k < 3; ++k) c.c[k] = -((c.R[k] * c.t[0] + c.R[3 + k] * c.t[1]) + c.R[6 + k] * c.t[2]);
}

// Real spherical harmonics, degree <= 3, orthonormal, (l, m = -l..l) order; constants are
// 1/(2 sqrt(pi)), sqrt(3/(4 pi)), sqrt(15/pi)/2, sqrt(5/pi)/4, sqrt(15/pi)/4, sqrt(35/(2 pi))/4,
// sqrt(105/pi)/2, sqrt(21/(2 pi))/4, sqrt(7/pi)/4, sqrt(105/pi)/4.
constexpr double kY0 = 0.28209479177387814;
constexpr double kY1 = 0.4886025119029199;
constexpr double kY2a = 1.0925484305920792;
constexpr double kY2b = 0.31539156525252005;
constexpr double kY2c = 0.5462742152960396;
constexpr double kY3a = 0.5900435899266435;
constexpr double kY3b = 2.890611442640554;
constexpr double kY3c = 0.4570457994644658;
constexpr double kY3d = 0.3731763325901154;
constexpr double kY3e = 1.445305721320277;

template <int K>
__device__ inline void sh_basis(double x, double y, double z, double* Y) {
  Y[0] = kY0;
  if constexpr (K > 1) {
    Y[1] = kY1 * y;
    Y[2] = kY1 * z;
    Y[3] = kY1 * x;
  }
  if constexpr (K > 4) {
    const double xx = x * x, yy = y * y, zz = z * z;
    Y[4] = kY2a * (x * y);
    Y[5] = kY2a * (y * z);
    Y[6] = kY2b * (2.0 * zz - xx - yy);
    Y[7] = kY2a * (x * z);
    Y[8] = kY2c * (xx - yy);
    if constexpr (K > 9) {
      Y[9] = kY3a * (y * (3.0 * xx - yy));
      Y[10] = kY3b * (x * y * z);
      Y[11] = kY3c * (y * (4.0 * zz - xx - yy));
      Y[12] = kY3d * (z * (2.0 * zz - 3.0 * xx - 3.0 * yy));
      Y[13] = kY3c * (x * (4.0 * zz - xx - yy));
      Y[14] = kY3e * (z * (xx - yy));
      Y[15] = kY3a * (x * (xx - 3.0 * yy));
    }
  }
}

// sum_k w_k grad Y_k at (x, y, z): the gradient of each basis polynomial (before projection onto
// the sphere) weighted and summed on the fly, without materialising the K x 3 table.
template <int K>
__device__ inline void sh_grad_dot(double x, double y, double z, const double* w, double g[3]) {
  g[0] = g[1] = g[2] = 0.0;
  if constexpr (K > 1) {
    g[0] += kY1 * w[3];
    g[1] += kY1 * w[1];
    g[2] += kY1 * w[2];
  }
  if constexpr (K > 4) {
    g[0] += kY2a * (y * w[4] + z * w[7]) + x * (2.0 * kY2c * w[8] - 2.0 * kY2b * w[6]);
    g[1] += kY2a * (x * w[4] + z * w[5]) - y * (2.0 * kY2b * w[6] + 2.0 * kY2c * w[8]);
    g[2] += kY2a * (y * w[5] + x * w[7]) + 4.0 * kY2b * z * w[6];
    if constexpr (K > 9) {
      const double xx = x * x, yy = y * y, zz = z * z;
      g[0] += 6.0 * kY3a * x * y * w[9] + kY3b * y * z * w[10] - 2.0 * kY3c * x * y * w[11] -
              6.0 * kY3d * x * z * w[12] + kY3c * (4.0 * zz - 3.0 * xx - yy) * w[13] + 2.0 * kY3e * x * z * w[14] +
              3.0 * kY3a * (xx - yy) * w[15];
      g[1] += 3.0 * kY3a * (xx - yy) * w[9] + kY3b * x * z * w[10] + kY3c * (4.0 * zz - xx - 3.0 * yy) * w[11] -
              6.0 * kY3d * y * z * w[12] - 2.0 * kY3c * x * y * w[13] - 2.0 * kY3e * y * z * w[14] -
              6.0 * kY3a * x * y * w[15];
      g[2] += kY3b * x * y * w[10] + 8.0 * kY3c * y * z * w[11] + kY3d * (6.0 * zz - 3.0 * xx - 3.0 * yy) * w[12] +
              8.0 * kY3c * x * z * w[13] + kY3e * (xx - yy) * w[14];
    }
  }
}

// View-independent part: rotation of the normalised quaternion and Sigma = (R S)(R S)^T.
struct Cov3 {
  double qn, w, x, y, z;  // |q| and the normalised quaternion
  double Rq[9];
  double M[9];            // Rq * diag(s)
  double S[9];            // Sigma
};

__device__ inline void cov3(const double s[3], const double q[4], Cov3& c) {
  c.qn = sqrt(((q[0] * q[0] + q[1] * q[1]) + q[2] * q[2]) + q[3] * q[3]);
  c.w = q[0] / c.qn;
  c.x = q[1] / c.qn;
  c.y = q[2] / c.qn;
  c.z = q[3] / c.qn;
  const double w = c.w, x = c.x, y = c.y, z = c.z;
  c.Rq[0] = 1.0 - 2.0 * (y * y + z * z);
  c.Rq[1] = 2.0 * (x * y - w * z);
  c.Rq[2] = 2.0 * (x * z + w * y);
  c.Rq[3] = 2.0 * (x * y + w * z);
  c.Rq[4] = 1.0 - 2.0 * (x * x + z * z);
  c.Rq[5] = 2.0 * (y * z - w * x);
  c.Rq[6] = 2.0 * (x * z - w * y);
  c.Rq[7] = 2.0 * (y * z + w * x);
  c.Rq[8] = 1.0 - 2.0 * (x * x + y * y);
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int k = 0; k < 3; ++k) c.M[3 * r + k] = c.Rq[3 * r + k] * s[k];
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int k = 0; k < 3; ++k)
      c.S[3 * r + k] = (c.M[3 * r] * c.M[3 * k] + c.M[3 * r + 1] * c.M[3 * k + 1]) + c.M[3 * r + 2] * c.M[3 * k + 2];
}

// View-dependent geometry shared by the forward and the adjoint.
struct Geo {
  double mu[3], r2, r, p, rho;  // camera-space mean, |mu|^2, |mu|, mu_x^2 + mu_z^2, sqrt of it
  double depth;                 // sort depth: |mu| (ERP), mu_z (pinhole)
  double u, v;
  double J[6];                  // J_omni = d(u, v) / d mu (closed form of Appendix B)
  double A[6];                  // J_omni * R
  double c2[3];                 // Sigma_2D + dilation: uu, uv, vv
  double det;
};

// Pinhole intrinsics of a view (fx == 0: equirectangular view).
struct Pin {
  double fx, fy, cx, cy;
};

// Returns false when the item is culled (shell and pole tests for ERP views; depth range and
// the 1.3x field-of-view guard band for pinhole views).
__device__ inline bool geometry(const double m[3], const Cam& cam, const Cov3& cv, int W, int H, const Params& P,
                                const Pin& pin, Geo& g) {
#pragma unroll
  for (int r = 0; r < 3; ++r)
    g.mu[r] = ((cam.R[3 * r] * m[0] + cam.R[3 * r + 1] * m[1]) + cam.R[3 * r + 2] * m[2]) + cam.t[r];
  g.r2 = (g.mu[0] * g.mu[0] + g.mu[1] * g.mu[1]) + g.mu[2] * g.mu[2];
  g.r = sqrt(g.r2);
  g.p = g.mu[0] * g.mu[0] + g.mu[2] * g.mu[2];
  g.rho = sqrt(g.p);
  const double Wd = (double)W, Hd = (double)H;
  if (pin.fx > 0.0) {
    // Perspective camera (Sec. 3.1): pi(mu) = K (mu_x / mu_z, mu_y / mu_z), J of Eq. jacob_pers.
    const double x = g.mu[0], y = g.mu[1], z = g.mu[2];
    g.depth = z;
    if (!(z > P.near_r && z < P.far_r)) return false;
    if (!(fabs(x / z) <= 1.3 * (Wd / (2.0 * pin.fx)) && fabs(y / z) <= 1.3 * (Hd / (2.0 * pin.fy)))) return false;
    g.u = pin.fx * (x / z) + pin.cx;
    g.v = pin.fy * (y / z) + pin.cy;
    g.J[0] = pin.fx / z;
    g.J[1] = 0.0;
    g.J[2] = -pin.fx * x / (z * z);
    g.J[3] = 0.0;
    g.J[4] = pin.fy / z;
    g.J[5] = -pin.fy * y / (z * z);
  } else {
  g.depth = g.r;
  if (!(g.r > P.near_r && g.r < P.far_r)) return false;
  if (!(g.rho > P.pole_eps * g.r)) return false;
  const double phi = atan2(g.mu[0], g.mu[2]);
  const double theta = atan2(-g.mu[1], g.rho);
  g.u = (Wd / (2.0 * kPi)) * phi + Wd / 2.0;
  g.v = (-Hd / kPi) * theta + Hd / 2.0;
  // J_omni = S_o Q_o J_o T_mu written with cos(theta) = rho/r, sin(theta) = -mu_y/r,
  // sin(phi) = mu_x/rho, cos(phi) = mu_z/rho.
  const double a1 = Wd / (2.0 * kPi), a2 = Hd / kPi;
  const double x = g.mu[0], y = g.mu[1], z = g.mu[2];
  const double r2rho = g.r2 * g.rho;
  g.J[0] = a1 * z / g.p;
  g.J[1] = 0.0;
  g.J[2] = -a1 * x / g.p;
  g.J[3] = -a2 * x * y / r2rho;
  g.J[4] = a2 * g.rho / g.r2;
  g.J[5] = -a2 * y * z / r2rho;
  }
#pragma unroll
  for (int r = 0; r < 2; ++r)
#pragma unroll
    for (int k = 0; k < 3; ++k)
      g.A[3 * r + k] = (g.J[3 * r] * cam.R[k] + g.J[3 * r + 1] * cam.R[3 + k]) + g.J[3 * r + 2] * cam.R[6 + k];
  double AS[6];
#pragma unroll
  for (int r = 0; r < 2; ++r)
#pragma unroll
    for (int k = 0; k < 3; ++k)
      AS[3 * r + k] = (g.A[3 * r] * cv.S[k] + g.A[3 * r + 1] * cv.S[3 + k]) + g.A[3 * r + 2] * cv.S[6 + k];
  g.c2[0] = ((AS[0] * g.A[0] + AS[1] * g.A[1]) + AS[2] * g.A[2]) + P.dilation;
  g.c2[1] = (AS[0] * g.A[3] + AS[1] * g.A[4]) + AS[2] * g.A[5];
  g.c2[2] = ((AS[3] * g.A[3] + AS[4] * g.A[4]) + AS[5] * g.A[5]) + P.dilation;
  g.det = g.c2[0] * g.c2[2] - g.c2[1] * g.c2[1];
  return true;
}

// float(x) rounded towards +infinity, so a padded extent never shrinks when stored as float.
__device__ inline float round_up_f32(double x) {
  float f = (float)x;
  if ((double)f < x) f = nextafterf(f, INFINITY);
  return f;
}

__device__ inline void view_dir(const double m[3], const Cam& cam, double d[3], double& dist) {
  const double w0 = m[0] - cam.c[0], w1 = m[1] - cam.c[1], w2 = m[2] - cam.c[2];
  dist = sqrt((w0 * w0 + w1 * w1) + w2 * w2);
  d[0] = w0 / dist;
  d[1] = w1 / dist;
  d[2] = w2 / dist;
}

__device__ inline double sym3(const double* C, const double* x, const double* y) {
  return x[0] * (C[0] * y[0] + C[1] * y[1] + C[2] * y[2]) + x[1] * (C[1] * y[0] + C[3] * y[1] + C[4] * y[2]) +
         x[2] * (C[2] * y[0] + C[4] * y[1] + C[5] * y[2]);
}

// Normalised camera-space covariance of the spherical footprint, Sigma~ = W Sigma W^T / |mu|^2
// + dilation (pi / H)^2 I, as (xx, xy, xz, yy, yz, zz); also returns W Sigma W^T.
__device__ inline void sph_cov(const Geo& g, const Cam& cam, const Cov3& cv, int H, const Params& P, double C[6],
                               double Sc[6]) {
  double RS[9];
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int k = 0; k < 3; ++k)
      RS[3 * r + k] = (cam.R[3 * r] * cv.S[k] + cam.R[3 * r + 1] * cv.S[3 + k]) + cam.R[3 * r + 2] * cv.S[6 + k];
  const int idx[6][2] = {{0, 0}, {0, 1}, {0, 2}, {1, 1}, {1, 2}, {2, 2}};
  const double dang = P.dilation * (kPi / (double)H) * (kPi / (double)H);
  const double ir2 = 1.0 / g.r2;
#pragma unroll
  for (int e = 0; e < 6; ++e) {
    const int r = idx[e][0], k = idx[e][1];
    Sc[e] = (RS[3 * r] * cam.R[3 * k] + RS[3 * r + 1] * cam.R[3 * k + 1]) + RS[3 * r + 2] * cam.R[3 * k + 2];
    C[e] = Sc[e] * ir2 + (r == k ? dang : 0.0);
  }
}

// Latitude / longitude range of the bounding box of the item's gnomonic ellipse (see sph_item):
// the box is a spherical quadrilateral of great-circle arcs, so the longitude range is that of
// its corners (longitude is monotonic along a great circle that misses the poles) and the
// latitude extremes are at the corners or at an edge's highest or lowest point when that lies
// on the edge; a pole whose gnomonic image is inside the box takes every longitude.
struct LatLonBox {
  double sin_lo, sin_hi, dphi_lo, dphi_hi;
  bool north, south;
};

__device__ inline void gnomonic_box(const double m[3], const double e1[3], const double e2[3], double p0x, double p0y,
                                    double hx, double hy, double phic, LatLonBox& bx) {
  bx.north = bx.south = false;
  // north pole (0, -1, 0), south pole (0, 1, 0)
  if (-m[1] > 0.0) {
    const double px = -e1[1] / -m[1], py = -e2[1] / -m[1];
    bx.north = fabs(px - p0x) <= hx && fabs(py - p0y) <= hy;
  }
  if (m[1] > 0.0) {
    const double px = e1[1] / m[1], py = e2[1] / m[1];
    bx.south = fabs(px - p0x) <= hx && fabs(py - p0y) <= hy;
  }
  double D[4][3];
  const double sx[4] = {-1.0, 1.0, 1.0, -1.0}, sy[4] = {-1.0, -1.0, 1.0, 1.0};
  bx.sin_lo = 2.0;
  bx.sin_hi = -2.0;
  bx.dphi_lo = 10.0;
  bx.dphi_hi = -10.0;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const double px = p0x + sx[k] * hx, py = p0y + sy[k] * hy;
    double nrm2 = 0.0;
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      D[k][j] = m[j] + px * e1[j] + py * e2[j];
      nrm2 += D[k][j] * D[k][j];
    }
    const double nrm = sqrt(nrm2);
#pragma unroll
    for (int j = 0; j < 3; ++j) D[k][j] /= nrm;
    bx.sin_lo = fmin(bx.sin_lo, -D[k][1]);
    bx.sin_hi = fmax(bx.sin_hi, -D[k][1]);
    double dp = atan2(D[k][0], D[k][2]) - phic;
    if (dp > kPi) dp -= 2.0 * kPi;
    if (dp < -kPi) dp += 2.0 * kPi;
    bx.dphi_lo = fmin(bx.dphi_lo, dp);
    bx.dphi_hi = fmax(bx.dphi_hi, dp);
  }
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const double* A = D[k];
    const double* Bv = D[(k + 1) & 3];
    const double n[3] = {A[1] * Bv[2] - A[2] * Bv[1], A[2] * Bv[0] - A[0] * Bv[2], A[0] * Bv[1] - A[1] * Bv[0]};
    const double nn = n[0] * n[0] + n[1] * n[1] + n[2] * n[2];
    if (!(nn > 0.0)) continue;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const double sg = h == 0 ? -1.0 : 1.0;  // towards the north pole, then the south pole
      // the pole direction projected onto the edge's great-circle plane
      double v[3] = {-(sg * n[1]) * n[0] / nn, sg - (sg * n[1]) * n[1] / nn, -(sg * n[1]) * n[2] / nn};
      const double vn = sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
      if (!(vn > 0.0)) continue;
#pragma unroll
      for (int j = 0; j < 3; ++j) v[j] /= vn;
      const double t1 = (A[1] * v[2] - A[2] * v[1]) * n[0] + (A[2] * v[0] - A[0] * v[2]) * n[1] +
                        (A[0] * v[1] - A[1] * v[0]) * n[2];
      const double t2 = (v[1] * Bv[2] - v[2] * Bv[1]) * n[0] + (v[2] * Bv[0] - v[0] * Bv[2]) * n[1] +
                        (v[0] * Bv[1] - v[1] * Bv[0]) * n[2];
      if (t1 >= 0.0 && t2 >= 0.0) {
        bx.sin_lo = fmin(bx.sin_lo, -v[1]);
        bx.sin_hi = fmax(bx.sin_hi, -v[1]);
      }
    }
  }
  if (bx.north) bx.sin_hi = 1.0;
  if (bx.south) bx.sin_lo = -1.0;
}

// Spherical footprint of one kept ERP item: the float record (tangent frame e1 east, e2 = mu^ x e1;
// P, c, s33 the tangent, tangent-radial and radial blocks of Sigma~; (l0, l1; 0, l2) the factor
// of P^-1 / 2; u1 = l0 e1 + l1 e2, u2 = l2 e2, w = mu^ - (P^-1 c)_1 e1 - (P^-1 c)_2 e2,
// k2 = 2 (s33 - c^T P^-1 c)), the cone (mu^, half-angle beta) and its tile rectangle: latitudes
// theta_c +- beta, longitudes +- asin(sin beta / cos theta_c) unless the cone reaches a pole,
// everything when the ball of radius k sqrt(lambda_max) holds the camera.  Returns false when
// culled (Sigma~ not positive definite, empty rectangle).
__device__ inline bool sph_item(const Geo& g, const Cam& cam, const Cov3& cv, const double s[3], int W, int H,
                                const Params& P, double p_min, float o, const float rgb[3], SphRec& out, SphCull& cn,
                                Rect& rr) {
  double C[6], Sc[6];
  sph_cov(g, cam, cv, H, P, C, Sc);
  const double c00 = C[3] * C[5] - C[4] * C[4], c01 = C[2] * C[4] - C[1] * C[5], c02 = C[1] * C[4] - C[2] * C[3];
  const double det3 = (C[0] * c00 + C[1] * c01) + C[2] * c02;
  if (!(det3 > 0.0)) return false;
  const double m[3] = {g.mu[0] / g.r, g.mu[1] / g.r, g.mu[2] / g.r};
  const double rh = sqrt(m[0] * m[0] + m[2] * m[2]);
  const double e1[3] = {m[2] / rh, 0.0, -m[0] / rh};
  const double e2[3] = {m[1] * e1[2] - m[2] * e1[1], m[2] * e1[0] - m[0] * e1[2], m[0] * e1[1] - m[1] * e1[0]};
  const double P11 = sym3(C, e1, e1), P12 = sym3(C, e1, e2), P22 = sym3(C, e2, e2);
  const double c1 = sym3(C, e1, m), c2 = sym3(C, e2, m), s33 = sym3(C, m, m);
  const double det = P11 * P22 - P12 * P12;
  const double l0 = sqrt(P22 / (2.0 * det)), l1 = -P12 / (2.0 * det * l0), l2 = 1.0 / sqrt(2.0 * P22);
  const double a1 = -(P22 * c1 - P12 * c2) / det, a2 = -(P11 * c2 - P12 * c1) / det;
  double u1[3], u2[3], w[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    u1[k] = l0 * e1[k] + l1 * e2[k];
    u2[k] = l2 * e2[k];
    w[k] = m[k] + a1 * e1[k] + a2 * e2[k];
  }
  const double k2 = 2.0 * (s33 + (a1 * c1 + a2 * c2));
  out.s0 = make_float4((float)u1[0], (float)u1[1], (float)u1[2], (float)u2[0]);
  out.s1 = make_float4((float)u2[1], (float)u2[2], (float)w[0], (float)w[1]);
  out.s2 = make_float4((float)w[2], (float)k2, o, (float)p_min);
  out.s3 = make_float4(rgb[0], rgb[1], rgb[2], 0.0f);
  bool ell = false;
  double ep0x = 0.0, ep0y = 0.0, ehx = 0.0, ehy = 0.0;  // the ellipse's centre and bounding-box half widths
  // Gnomonic ellipse of the rays that can reach alpha >= 1/255: with g = (d . e1, d . e2),
  // s = d . mu^, p = g / s, m <= k^2 reads (1 - k^2 kappa) p^T P^-1 p <= k^2 (1 + a . p)^2
  // (a = -P^-1 c, kappa = s33 - c^T P^-1 c), an ellipse when k^2 s33 < 1 (the ellipsoid stays in
  // front of the camera along mu^): M = (1 - k^2 kappa) P^-1 - k^2 a a^T, p0 = k^2 M^-1 a,
  // rho^2 = k^2 + k^4 a^T M^-1 a.
  {
    const double kk = -2.0 * p_min;
    const double kap = s33 + (a1 * c1 + a2 * c2);
    const double f = 1.0 - kk * kap;
    const double M11 = f * (P22 / det) - kk * a1 * a1, M12 = f * (-P12 / det) - kk * a1 * a2;
    const double M22 = f * (P11 / det) - kk * a2 * a2;
    const double detM = M11 * M22 - M12 * M12;
    float p0x = 0.0f, p0y = 0.0f, rho = -1.0f, sl = 0.0f;
    ell = kk * s33 < 0.999 && detM > 0.0 && M11 > 0.0;
    if (ell) {
      const double q0 = (M22 * a1 - M12 * a2) / detM, q1 = (M11 * a2 - M12 * a1) / detM;  // M^-1 a
      const double rho2 = kk + kk * kk * (a1 * q0 + a2 * q1);
      ep0x = kk * q0;
      ep0y = kk * q1;
      ehx = sqrt(rho2 * M22 / detM) * (1.0 + 1e-3);
      ehy = sqrt(rho2 * M11 / detM) * (1.0 + 1e-3);
      p0x = (float)ep0x;
      p0y = (float)ep0y;
      rho = round_up_f32(sqrt(rho2) * (1.0 + 1e-3));
      sl = round_up_f32(sqrt(0.5 * (M11 + M22 + sqrt((M11 - M22) * (M11 - M22) + 4.0 * M12 * M12))));
    }
    cn.c1 = make_float4((float)e1[0], (float)e1[2], (float)e2[0], (float)e2[1]);
    cn.c2 = make_float4((float)e2[2], p0x, p0y, (float)M11);
    cn.c3 = make_float4((float)M12, (float)M22, rho, sl);
  }
  // cone of the rays that can reach alpha >= 1/255
  const double smax2 = fmax(fmax(s[0] * s[0], s[1] * s[1]), s[2] * s[2]);
  const double lam = smax2 / (g.r * g.r) + P.dilation * (kPi / (double)H) * (kPi / (double)H);
  const double sb = sqrt(-2.0 * p_min * lam) * (1.0 + 1e-3);
  const int B = P.tile;
  const int ntx = W / B, nty = H / B;
  if (!(sb < 1.0)) {
    cn.c0 = make_float4((float)m[0], (float)m[1], (float)m[2], (float)kPi);
    rr = Rect{0, (uint16_t)ntx, 0, (uint16_t)nty};
    return true;
  }
  const double beta = asin(sb);
  cn.c0 = make_float4((float)m[0], (float)m[1], (float)m[2], round_up_f32(beta));
  const double thc = atan2(-g.mu[1], g.rho);
  const double Hd = (double)H, Wd = (double)W;
  if (ell) {
    // tile rectangle from the ellipse's bounding box (tighter than the cone for anisotropic
    // footprints)
    LatLonBox bx;
    gnomonic_box(m, e1, e2, ep0x, ep0y, ehx, ehy, atan2(g.mu[0], g.mu[2]), bx);
    const double vlo = Hd / 2.0 - (Hd / kPi) * asin(fmin(1.0, bx.sin_hi)) - 1e-2;
    const double vhi = Hd / 2.0 - (Hd / kPi) * asin(fmax(-1.0, bx.sin_lo)) + 1e-2;
    const double rlo = fmax(0.0, floor(vlo / B)), rhi = fmin((double)(nty - 1), floor(vhi / B));
    const int nrows = (int)(rhi - rlo + 1.0);
    if (nrows <= 0) return false;
    int col0 = 0, ncols = ntx;
    const double clo = floor((g.u + (Wd / (2.0 * kPi)) * bx.dphi_lo - 1e-2) / B);
    const double chi = floor((g.u + (Wd / (2.0 * kPi)) * bx.dphi_hi + 1e-2) / B);
    if (!bx.north && !bx.south && chi - clo + 1.0 < (double)ntx) {
      long long c0 = (long long)clo % ntx;
      if (c0 < 0) c0 += ntx;
      col0 = (int)c0;
      ncols = (int)(chi - clo + 1.0);
    }
    rr = Rect{(uint16_t)col0, (uint16_t)ncols, (uint16_t)rlo, (uint16_t)nrows};
    return true;
  }
  const double vlo = Hd / 2.0 - (Hd / kPi) * (thc + beta) - 1e-2, vhi = Hd / 2.0 - (Hd / kPi) * (thc - beta) + 1e-2;
  const double rlo = fmax(0.0, floor(vlo / B)), rhi = fmin((double)(nty - 1), floor(vhi / B));
  const int nrows = (int)(rhi - rlo + 1.0);
  if (nrows <= 0) return false;
  int col0 = 0, ncols = ntx;
  if (fabs(thc) + beta < kPi / 2.0) {
    const double eu = (Wd / (2.0 * kPi)) * asin(sin(beta) / cos(thc)) + 1e-2;
    const double clo = floor((g.u - eu) / B), chi = floor((g.u + eu) / B);
    if (chi - clo + 1.0 < (double)ntx) {
      long long c0 = (long long)clo % ntx;
      if (c0 < 0) c0 += ntx;
      col0 = (int)c0;
      ncols = (int)(chi - clo + 1.0);
    }
  }
  rr = Rect{(uint16_t)col0, (uint16_t)ncols, (uint16_t)rlo, (uint16_t)nrows};
  return true;
}

// Ray table of the spherical footprint: per view, (sin phi, cos phi) of the W pixel-centre
// azimuths, then (sin theta, cos theta) of the H pixel-centre elevations (Eq. equirec_proj
// inverted), each angle formed by this exact sequence of double operations.
__global__ void dir_table_kernel(ViewTable vt, double2* __restrict__ tab) {
#pragma clang fp contract(off)
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= vt.dir_base[vt.n_views]) return;
  int v = 0;
  while (i >= vt.dir_base[v + 1]) ++v;
  const int j = i - vt.dir_base[v];
  const double W = (double)vt.W[v], H = (double)vt.H[v];
  double a;
  if (j < vt.W[v]) a = (((double)j + 0.5) - 0.5 * W) * ((2.0 * kPi) / W);
  else a = (0.5 * H - ((double)(j - vt.W[v]) + 0.5)) * (kPi / H);
  tab[i] = make_double2(sin(a), cos(a));
}

// SPH: spherical-footprint records (srec, cone) instead of the affine rectangle (a separate
// instantiation, so the affine kernel carries none of it).
template <int K, bool SPH>
__global__ __launch_bounds__(256) void preprocess_kernel(int64_t n, const float* __restrict__ means,
                                                         const float* __restrict__ scales, const float* __restrict__ quats,
                                                         const float* __restrict__ opac, const float* __restrict__ sh,
                                                         const float* __restrict__ cams, ViewTable vt, Params P,
                                                         Rec* __restrict__ rec, Rect* __restrict__ rect,
                                                         uint32_t* __restrict__ count, uint32_t* __restrict__ dkey,
                                                         float* __restrict__ depth_out, odgs_status* __restrict__ status,
                                                         SphRec* __restrict__ srec, SphCull* __restrict__ cone,
                                                         double* __restrict__ g2d, int g2d_stride, int vgroups,
                                                         uint32_t* __restrict__ part) {
  // One thread per Gaussian and group of views (the views split into `vgroups` runs of equal
  // length but the last).  Workgroups go to the eight XCDs in turn, so the workgroups b, b + 8,
  // b + 16, ... share an XCD: those of one 256-Gaussian chunk (one per view group) are placed
  // there, consecutively, and all groups but the first read the parameters from that XCD's L2.
  const int nv = vt.n_views;
  const int xcd = (int)(blockIdx.x & 7u), kb = (int)(blockIdx.x >> 3);
  const int per = (nv + vgroups - 1) / vgroups;
  const int v0 = (kb % vgroups) * per, v1 = min(nv, v0 + per);
  const int64_t i0 = ((int64_t)(kb / vgroups) * 8 + xcd) * blockDim.x;  // first Gaussian of the chunk
  const int64_t i = i0 + threadIdx.x;
  const bool live = i < n;
  const int64_t ii = live ? i : 0;
  double m[3], s[3], q[4];
#pragma unroll
  for (int k = 0; k < 3; ++k) m[k] = (double)means[k * n + ii];
#pragma unroll
  for (int k = 0; k < 3; ++k) s[k] = (double)scales[k * n + ii];
#pragma unroll
  for (int k = 0; k < 4; ++k) q[k] = (double)quats[k * n + ii];
  const float o = opac[ii];
  float coef[K * 3];
#pragma unroll
  for (int k = 0; k < K * 3; ++k) coef[k] = sh[(int64_t)k * n + ii];
  // a NaN or infinite parameter, or a zero quaternion: every item of the Gaussian is culled
  bool fin = isfinite(o) && (q[0] != 0.0 || q[1] != 0.0 || q[2] != 0.0 || q[3] != 0.0);
#pragma unroll
  for (int k = 0; k < 3; ++k) fin = fin && isfinite(m[k]) && isfinite(s[k]);
#pragma unroll
  for (int k = 0; k < 4; ++k) fin = fin && isfinite(q[k]);
#pragma unroll
  for (int k = 0; k < K * 3; ++k) fin = fin && isfinite(coef[k]);
  Cov3 cv;
  cov3(s, q, cv);
  const double p_min = -log(255.0 * (double)o);
  unsigned long long visible = 0, culled = 0;
  // (one view per thread in the spherical instantiation: a loop of one trip that the compiler sees)
  for (int v = v0; v < (SPH ? min(v1, v0 + 1) : v1); ++v) {
    Cam cam;
    load_cam(cams, v, cam);
    const int W = vt.W[v], H = vt.H[v];
    Geo g;
    const Pin pin{(double)vt.pin[v][0], (double)vt.pin[v][1], (double)vt.pin[v][2], (double)vt.pin[v][3]};
    bool kept = live && fin && geometry(m, cam, cv, W, H, P, pin, g);
    float depth = (float)g.depth;
    Rec out;
    Rect rr{0, 0, 0, 0};
    uint32_t cnt = 0;
    if (kept) {
      // Cholesky factor (l0, l1; 0, l2) of Sigma^-1 / 2, so that the compositor evaluates the
      // exponent -d^T Sigma^-1 d / 2 as -((l0 du + l1 dv)^2 + (l2 dv)^2) without cancellation.
      const double l0 = sqrt(g.c2[2] / (2.0 * g.det));
      const double l1 = -g.c2[1] / (2.0 * g.det * l0);
      const double l2 = 1.0 / sqrt(2.0 * g.c2[2]);
      double d[3], dist;
      view_dir(m, cam, d, dist);
      double Y[K];
      sh_basis<K>(d[0], d[1], d[2], Y);
      float rgb[3];
      bool finite = isfinite(g.u) && isfinite(g.v);
#pragma unroll
      for (int ch = 0; ch < 3; ++ch) {
        double acc = 0.0;
#pragma unroll
        for (int k = 0; k < K; ++k) acc = acc + (double)coef[k * 3 + ch] * Y[k];
        acc = acc + 0.5;
        finite = finite && isfinite(acc);
        rgb[ch] = acc > 0.0 ? (float)acc : 0.0f;
      }
      if constexpr (SPH) {
        // spherical footprint (ERP views only)
        SphRec sr;
        SphCull cn;
        kept = (p_min < 0.0) && finite && sph_item(g, cam, cv, s, W, H, P, p_min, o, rgb, sr, cn, rr);
        if (kept) {
          cnt = (uint32_t)rr.ncols * (uint32_t)rr.nrows;
          const int64_t item = (int64_t)v * n + i;
          srec[item] = sr;
          cone[item] = cn;
          out.r0 = make_float4((float)g.u, (float)g.v, (float)l0, (float)l1);
          out.r1 = make_float4((float)l2, o, (float)p_min, 0.0f);
          out.r2 = make_float4(rgb[0], rgb[1], rgb[2], 0.0f);
        } else {
          rr = Rect{0, 0, 0, 0};
        }
      } else if ((kept = (p_min < 0.0) && (g.det > 0.0) && finite)) {
        // Footprint: alpha >= 1/255 inside d^T Sigma^-1 d <= k2 = -2 p_min; half extents
        // sqrt(k2 Sigma_uu), sqrt(k2 Sigma_vv), padded by 0.1% + 0.01 px.
        const double k2 = -2.0 * p_min;
        const double eu = sqrt(k2 * g.c2[0]) * (1.0 + 1e-3) + 1e-2;
        const double ev = sqrt(k2 * g.c2[2]) * (1.0 + 1e-3) + 1e-2;
        const int B = P.tile;
        const int ntx = W / B, nty = H / B;
        const double clo = floor((g.u - eu) / B), chi = floor((g.u + eu) / B);
        int col0, ncols;
        if (pin.fx > 0.0) {
          // no seam: columns clamp at the image edges like the rows
          const double c0 = fmax(0.0, clo), c1 = fmin((double)(ntx - 1), chi);
          col0 = (int)fmax(0.0, fmin(c0, (double)ntx));
          ncols = (int)(c1 - c0 + 1.0);
        } else if (!(chi - clo + 1.0 < (double)ntx)) {
          col0 = 0;
          ncols = ntx;
        } else {
          long long c0 = (long long)clo % ntx;
          if (c0 < 0) c0 += ntx;
          col0 = (int)c0;
          ncols = (int)(chi - clo + 1.0);
        }
        const double rlo = fmax(0.0, floor((g.v - ev) / B));
        const double rhi = fmin((double)(nty - 1), floor((g.v + ev) / B));
        const int row0 = (int)rlo;
        const int nrows = (int)(rhi - rlo + 1.0);
        kept = nrows > 0 && ncols > 0;
        if (kept) {
          rr = Rect{(uint16_t)col0, (uint16_t)ncols, (uint16_t)row0, (uint16_t)nrows};
          cnt = (uint32_t)ncols * (uint32_t)nrows;
          out.r0 = make_float4((float)g.u, (float)g.v, (float)l0, (float)l1);
          out.r1 = make_float4((float)l2, o, (float)p_min, round_up_f32(eu));
          out.r2 = make_float4(rgb[0], rgb[1], rgb[2], round_up_f32(ev));
        }
      }
    }
    if (live) {
      const int64_t item = (int64_t)v * n + i;
      if (!kept) {
        out.r0 = make_float4(0.f, 0.f, 0.f, 0.f);
        out.r1 = make_float4(0.f, 0.f, 0.f, 0.f);
        out.r2 = make_float4(0.f, 0.f, 0.f, 0.f);
      }
      rec[item] = out;
      depth_out[item] = depth;
      rect[item] = rr;
      count[item] = cnt;
      dkey[item] = kept ? __float_as_uint(depth) : 0xffffffffu;
    }
    visible += kept ? 1 : 0;
    culled += (live && !kept) ? 1 : 0;
  }
  // The reverse compositor adds into the per-item 2D-gradient records: clear this block's records
  // here (contiguous, coalesced), where the HBM traffic overlaps the FP64 arithmetic above instead
  // of taking a pass of its own.
  if (i0 < n) {
    const int64_t words = (n - i0 < (int64_t)blockDim.x ? n - i0 : (int64_t)blockDim.x) * g2d_stride;
    for (int v = v0; v < v1; ++v) {
      double* base = g2d + ((int64_t)v * n + i0) * g2d_stride;
      for (int64_t w = threadIdx.x; w < words; w += blockDim.x) base[w] = 0.0;
    }
  }
  // the workgroup's kept and culled items into part[workgroup] (summed by count_fold_kernel: one
  // atomic per wavefront on a single status word would serialise thousands of them), or, in a
  // launch of few workgroups (part null), by one atomic per workgroup; non-finite Gaussians,
  // counted in the group of their first view, by one atomic per wavefront that has any
  __shared__ uint32_t wsum[256 / kWave];
  uint32_t tw = (uint32_t)visible | ((uint32_t)culled << 16);
  unsigned long long tnf = (live && !fin && v0 == 0) ? 1 : 0;
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    tw += __shfl_xor(tw, off);
    tnf += __shfl_xor(tnf, off);
  }
  if ((threadIdx.x & (kWave - 1)) == 0) {
    wsum[threadIdx.x >> 6] = tw;
    if (tnf) atomicAdd((unsigned long long*)&status->n_nonfinite, tnf);
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    const uint32_t s = wsum[0] + wsum[1] + wsum[2] + wsum[3];
    if (part) {
      part[blockIdx.x] = s;
    } else {
      if (s & 0xFFFFu) atomicAdd((unsigned long long*)&status->n_visible, (unsigned long long)(s & 0xFFFFu));
      if (s >> 16) atomicAdd((unsigned long long*)&status->n_culled, (unsigned long long)(s >> 16));
    }
  }
}

// Sum of the preprocess workgroups' (kept | culled << 16) counts into the status record.
__global__ __launch_bounds__(1024) void count_fold_kernel(const uint32_t* __restrict__ part, int nparts,
                                                          odgs_status* __restrict__ status) {
  __shared__ unsigned long long s_vis[1024 / kWave], s_cul[1024 / kWave];
  unsigned long long vis = 0, cul = 0;
  for (int k = threadIdx.x; k < nparts; k += 1024) {
    const uint32_t x = part[k];
    vis += x & 0xFFFFu;
    cul += x >> 16;
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    vis += __shfl_xor(vis, off);
    cul += __shfl_xor(cul, off);
  }
  if ((threadIdx.x & (kWave - 1)) == 0) {
    s_vis[threadIdx.x >> 6] = vis;
    s_cul[threadIdx.x >> 6] = cul;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long tv = 0, tc = 0;
    for (int w = 0; w < 1024 / kWave; ++w) {
      tv += s_vis[w];
      tc += s_cul[w];
    }
    status->n_visible += (int64_t)tv;
    status->n_culled += (int64_t)tc;
  }
}

// ---------------------------------------------------------------------------------------------
// Adjoint.  Inputs per item: 2D gradients g2d[items][9] = (u, v, S_uu, S_uv, S_vv, opacity, r, g,
// b) with Sigma_2D = [[S_uu, S_uv], [S_uv, S_vv]] (S_uv the shared off-diagonal, dilation
// included).  Sums over views; writes (overwrites) the parameter gradients.
// ---------------------------------------------------------------------------------------------
// Densification statistics (Sec. 3.3) gathered while the 2D gradients are consumed.
struct DensAcc {
  float* grad_sum;
  float* tau_sum;
  int32_t* count;
  double tau_min, tau_max;
};

// Adjoint of one view's colour = max(0, sum_k sh_k Y_k(dir) + 0.5), dir = (m - c) / |m - c|:
// adds dL/dsh to gsh (float accumulators) and the direction path to gm.
template <int K>
__device__ inline void colour_adjoint(const double m[3], const Cam& cam, const float* coef, const double gcol[3],
                                      float* gsh, double gm[3]) {
  double d[3], dist;
  view_dir(m, cam, d, dist);
  double Y[K];
  sh_basis<K>(d[0], d[1], d[2], Y);
  double w[K];
#pragma unroll
  for (int k = 0; k < K; ++k) w[k] = 0.0;
#pragma unroll
  for (int ch = 0; ch < 3; ++ch) {
    double acc = 0.0;
#pragma unroll
    for (int k = 0; k < K; ++k) acc = acc + (double)coef[k * 3 + ch] * Y[k];
    acc = acc + 0.5;
    if (!(acc > 0.0)) continue;
    const double gc = gcol[ch];
#pragma unroll
    for (int k = 0; k < K; ++k) {
      gsh[k * 3 + ch] += (float)(gc * Y[k]);
      w[k] += gc * (double)coef[k * 3 + ch];
    }
  }
  double gdir[3];
  sh_grad_dot<K>(d[0], d[1], d[2], w, gdir);
  const double dd = gdir[0] * d[0] + gdir[1] * d[1] + gdir[2] * d[2];
#pragma unroll
  for (int k = 0; k < 3; ++k) gm[k] += (gdir[k] - d[k] * dd) / dist;
}

// Colour part of the adjoint, one thread per Gaussian, run before the geometry part: dL/dsh
// (written) and the direction path of dL/dmean (written; the geometry part adds to it).  The
// per-item colour gradients sit at offset `off` of records of `stride` values.
template <int K>
__global__ __launch_bounds__(256) void colour_bwd_kernel(int64_t n, const float* __restrict__ means,
                                                         const float* __restrict__ sh, const float* __restrict__ cams,
                                                         ViewTable vt, const uint32_t* __restrict__ count,
                                                         const double* __restrict__ g2d, int stride, int off,
                                                         float* __restrict__ d_means, float* __restrict__ d_sh) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double m[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) m[k] = (double)means[k * n + i];
  float coef[K * 3];
#pragma unroll
  for (int k = 0; k < K * 3; ++k) coef[k] = sh[(int64_t)k * n + i];
  float gsh[K * 3];
#pragma unroll
  for (int k = 0; k < K * 3; ++k) gsh[k] = 0.0f;
  double gm[3] = {0.0, 0.0, 0.0};
  for (int v = 0; v < vt.n_views; ++v) {
    const int64_t item = (int64_t)v * n + i;
    if (count[item] == 0) continue;
    const double gcol[3] = {g2d[item * stride + off], g2d[item * stride + off + 1], g2d[item * stride + off + 2]};
    if (gcol[0] == 0.0 && gcol[1] == 0.0 && gcol[2] == 0.0) continue;
    Cam cam;
    load_cam(cams, v, cam);
    colour_adjoint<K>(m, cam, coef, gcol, gsh, gm);
  }
#pragma unroll
  for (int k = 0; k < 3; ++k) d_means[k * n + i] = (float)gm[k];
#pragma unroll
  for (int k = 0; k < K * 3; ++k) d_sh[(int64_t)k * n + i] = gsh[k];
}

// Last step of both geometry adjoints: dL/dSigma -> scales and (normalised) quaternion, then the
// writes; the mean gradient is added to the colour part already in d_means.
__device__ inline void write_param_grads(int64_t n, int64_t i, const double s[3], const Cov3& cv, const double gm[3],
                                         const double gS[9], double go, float* __restrict__ d_means,
                                         float* __restrict__ d_scales, float* __restrict__ d_quats,
                                         float* __restrict__ d_opac) {
  // Sigma = M M^T, M = Rq diag(s): dM = 2 dSigma M (dSigma symmetric).
  double dM[9];
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int k = 0; k < 3; ++k)
      dM[3 * r + k] = 2.0 * (gS[3 * r] * cv.M[k] + gS[3 * r + 1] * cv.M[3 + k] + gS[3 * r + 2] * cv.M[6 + k]);
  double gs[3], dR[9];
#pragma unroll
  for (int k = 0; k < 3; ++k) gs[k] = dM[k] * cv.Rq[k] + dM[3 + k] * cv.Rq[3 + k] + dM[6 + k] * cv.Rq[6 + k];
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int k = 0; k < 3; ++k) dR[3 * r + k] = dM[3 * r + k] * s[k];
  // Rq of the unit quaternion (w, x, y, z)
  const double w = cv.w, x = cv.x, y = cv.y, z = cv.z;
  double gw = 2.0 * (-z * dR[1] + y * dR[2] + z * dR[3] - x * dR[5] - y * dR[6] + x * dR[7]);
  double gx = 2.0 * (y * dR[1] + z * dR[2] + y * dR[3] - 2.0 * x * dR[4] - w * dR[5] + z * dR[6] + w * dR[7] -
                     2.0 * x * dR[8]);
  double gy = 2.0 * (-2.0 * y * dR[0] + x * dR[1] + w * dR[2] + x * dR[3] + z * dR[5] - w * dR[6] + z * dR[7] -
                     2.0 * y * dR[8]);
  double gz = 2.0 * (-2.0 * z * dR[0] - w * dR[1] + x * dR[2] + w * dR[3] - 2.0 * z * dR[4] + y * dR[5] + x * dR[6] +
                     y * dR[7]);
  // normalisation q_hat = q / |q|
  const double dot = gw * w + gx * x + gy * y + gz * z;
  const double iq = 1.0 / cv.qn;
  d_quats[i] = (float)((gw - w * dot) * iq);
  d_quats[n + i] = (float)((gx - x * dot) * iq);
  d_quats[2 * n + i] = (float)((gy - y * dot) * iq);
  d_quats[3 * n + i] = (float)((gz - z * dot) * iq);
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    d_means[k * n + i] = (float)((double)d_means[k * n + i] + gm[k]);
    d_scales[k * n + i] = (float)gs[k];
  }
  d_opac[i] = (float)go;
}

template <int K, bool STATS>
__global__ __launch_bounds__(256) void preprocess_bwd_kernel(
    int64_t n, const float* __restrict__ means, const float* __restrict__ scales, const float* __restrict__ quats,
    const float* __restrict__ opac, const float* __restrict__ sh, const float* __restrict__ cams, ViewTable vt, Params P,
    const uint32_t* __restrict__ count, double* __restrict__ g2d, int64_t items, float* __restrict__ d_means,
    float* __restrict__ d_scales, float* __restrict__ d_quats, float* __restrict__ d_opac, float* __restrict__ d_sh,
    DensAcc dacc) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double m[3], s[3], q[4];
#pragma unroll
  for (int k = 0; k < 3; ++k) m[k] = (double)means[k * n + i];
#pragma unroll
  for (int k = 0; k < 3; ++k) s[k] = (double)scales[k * n + i];
#pragma unroll
  for (int k = 0; k < 4; ++k) q[k] = (double)quats[k * n + i];
  Cov3 cv;
  cov3(s, q, cv);

  double gm[3] = {0.0, 0.0, 0.0};
  double gS[9] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};  // dL/dSigma (symmetric)
  double go = 0.0;
  double st_grad = 0.0, st_tau = 0.0;
  int st_count = 0;

  for (int v = 0; v < vt.n_views; ++v) {
    const int64_t item = (int64_t)v * n + i;
    if (count[item] == 0) continue;
    double g[9];
    bool any = false;
#pragma unroll
    for (int k = 0; k < 9; ++k) {
      g[k] = g2d[item * 9 + k];
      any = any || g[k] != 0.0;
    }
    if (STATS) {
      // visible in this view: |dL/d(u, v)| in normalised image units, and the threshold at the
      // elevation theta of the mean seen from this camera (cos theta = rho / r)
      Cam c;
      load_cam(cams, v, c);
      double mu[3];
#pragma unroll
      for (int r = 0; r < 3; ++r) mu[r] = ((c.R[3 * r] * m[0] + c.R[3 * r + 1] * m[1]) + c.R[3 * r + 2] * m[2]) + c.t[r];
      const double rr = sqrt((mu[0] * mu[0] + mu[1] * mu[1]) + mu[2] * mu[2]);
      const double ct = sqrt(mu[0] * mu[0] + mu[2] * mu[2]) / rr;
      st_tau += dacc.tau_min + (1.0 - ct) * (dacc.tau_max - dacc.tau_min);
      const double gu = g[0] * (0.5 * (double)vt.W[v]), gv = g[1] * (0.5 * (double)vt.H[v]);
      st_grad += sqrt(gu * gu + gv * gv);
      ++st_count;
    }
    if (!any) continue;
    Cam cam;
    load_cam(cams, v, cam);
    Geo G;
    const Pin pin{(double)vt.pin[v][0], (double)vt.pin[v][1], (double)vt.pin[v][2], (double)vt.pin[v][3]};
    geometry(m, cam, cv, vt.W[v], vt.H[v], P, pin, G);
    // dL/dSigma_2D as a symmetric matrix (the shared off-diagonal derivative split in halves)
    const double G00 = g[2], G01 = 0.5 * g[3], G11 = g[4];
    // Sigma2D = A Sigma A^T: dA = 2 G2 A Sigma, dSigma += A^T G2 A (G2 symmetric 2x2).
    double GA[6];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      GA[k] = G00 * G.A[k] + G01 * G.A[3 + k];
      GA[3 + k] = G01 * G.A[k] + G11 * G.A[3 + k];
    }
    double dA[6];
#pragma unroll
    for (int r = 0; r < 2; ++r)
#pragma unroll
      for (int k = 0; k < 3; ++k)
        dA[3 * r + k] = 2.0 * (GA[3 * r] * cv.S[k] + GA[3 * r + 1] * cv.S[3 + k] + GA[3 * r + 2] * cv.S[6 + k]);
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int b = 0; b < 3; ++b) gS[3 * a + b] += G.A[a] * GA[b] + G.A[3 + a] * GA[3 + b];
    // A = J R  =>  dJ = dA R^T
    double dJ[6];
#pragma unroll
    for (int r = 0; r < 2; ++r)
#pragma unroll
      for (int k = 0; k < 3; ++k)
        dJ[3 * r + k] = dA[3 * r] * cam.R[3 * k] + dA[3 * r + 1] * cam.R[3 * k + 1] + dA[3 * r + 2] * cam.R[3 * k + 2];
    // d(u, v)/d mu = J (mean path) plus the derivative of J itself.
    const double x = G.mu[0], y = G.mu[1], z = G.mu[2];
    const double p = G.p, rho = G.rho, r2 = G.r2, r4 = r2 * r2, p2 = p * p, rho3 = p * rho;
    const double a1 = (double)vt.W[v] / (2.0 * kPi), a2 = (double)vt.H[v] / kPi;
    double dmu[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) dmu[k] = G.J[k] * g[0] + G.J[3 + k] * g[1];
    if (pin.fx > 0.0) {
      // Eq. jacob_pers: J00 = fx / z, J02 = -fx x / z^2, J11 = fy / z, J12 = -fy y / z^2
      const double iz2 = 1.0 / (z * z), iz3 = iz2 / z;
      dmu[0] += dJ[2] * (-pin.fx * iz2);
      dmu[1] += dJ[5] * (-pin.fy * iz2);
      dmu[2] += dJ[0] * (-pin.fx * iz2) + dJ[2] * (2.0 * pin.fx * x * iz3) + dJ[4] * (-pin.fy * iz2) +
                dJ[5] * (2.0 * pin.fy * y * iz3);
    } else {
    const double xz2 = x * x - z * z;
    const double q2 = 2.0 * p + r2;
    const double r2m2y = r2 - 2.0 * y * y;
    const double r2m2p = r2 - 2.0 * p;
    // J00 = a1 z / p, J02 = -a1 x / p
    dmu[0] += dJ[0] * (-2.0 * a1 * x * z / p2) + dJ[2] * (a1 * xz2 / p2);
    dmu[2] += dJ[0] * (a1 * xz2 / p2) + dJ[2] * (2.0 * a1 * x * z / p2);
    // J10 = -a2 x y / (r^2 rho)
    dmu[0] += dJ[3] * (-a2 * y * (r2 * z * z - 2.0 * x * x * p) / (r4 * rho3));
    dmu[1] += dJ[3] * (-a2 * x * r2m2y / (r4 * rho));
    dmu[2] += dJ[3] * (a2 * x * y * z * q2 / (r4 * rho3));
    // J11 = a2 rho / r^2
    dmu[0] += dJ[4] * (a2 * x * r2m2p / (rho * r4));
    dmu[1] += dJ[4] * (-2.0 * a2 * rho * y / r4);
    dmu[2] += dJ[4] * (a2 * z * r2m2p / (rho * r4));
    // J12 = -a2 y z / (r^2 rho)
    dmu[0] += dJ[5] * (a2 * x * y * z * q2 / (r4 * rho3));
    dmu[1] += dJ[5] * (-a2 * z * r2m2y / (r4 * rho));
    dmu[2] += dJ[5] * (-a2 * y * (r2 * x * x - 2.0 * z * z * p) / (r4 * rho3));
    }
    // mu = R m + t  =>  dm = R^T dmu
#pragma unroll
    for (int k = 0; k < 3; ++k) gm[k] += cam.R[k] * dmu[0] + cam.R[3 + k] * dmu[1] + cam.R[6 + k] * dmu[2];
    go += g[5];  // the colour entries g[6..8] went to colour_bwd_kernel
  }

  write_param_grads(n, i, s, cv, gm, gS, go, d_means, d_scales, d_quats, d_opac);
  if (STATS && st_count > 0) {
    dacc.grad_sum[i] = (float)((double)dacc.grad_sum[i] + st_grad);
    dacc.tau_sum[i] = (float)((double)dacc.tau_sum[i] + st_tau);
    dacc.count[i] += st_count;
  }
}

// Adjoint of the spherical footprint.  Inputs per item g2d[items][13]: the gradient w.r.t. the
// unit direction mu^ (3) and the normalised covariance Sigma~ (xx, xy, xz, yy, yz, zz, the
// off-diagonals as one shared variable), opacity, r, g, b.  With Sigma~ = W Sigma W^T / r^2 +
// delta I, mu^ = mu / r and r = |mu|:  dL/d(W Sigma W^T) = dL/dSigma~ / r^2,
// dL/dr = -2 <dL/dSigma~, W Sigma W^T> / r^3,  dL/dmu = (I - mu^ mu^^T) dL/dmu^ / r + mu^ dL/dr;
// colour as in the affine adjoint.  Sums over views, overwrites the parameter gradients.
template <int K>
__global__ __launch_bounds__(256) void preprocess_sph_bwd_kernel(
    int64_t n, const float* __restrict__ means, const float* __restrict__ scales, const float* __restrict__ quats,
    const float* __restrict__ opac, const float* __restrict__ sh, const float* __restrict__ cams, ViewTable vt, Params P,
    const uint32_t* __restrict__ count, double* __restrict__ g2d, float* __restrict__ d_means,
    float* __restrict__ d_scales, float* __restrict__ d_quats, float* __restrict__ d_opac, float* __restrict__ d_sh) {
  constexpr int NV = 13;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double m[3], s[3], q[4];
#pragma unroll
  for (int k = 0; k < 3; ++k) m[k] = (double)means[k * n + i];
#pragma unroll
  for (int k = 0; k < 3; ++k) s[k] = (double)scales[k * n + i];
#pragma unroll
  for (int k = 0; k < 4; ++k) q[k] = (double)quats[k * n + i];
  Cov3 cv;
  cov3(s, q, cv);
  double gm[3] = {0.0, 0.0, 0.0};
  double gS[9] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};  // dL/dSigma (symmetric)
  double go = 0.0;
  for (int v = 0; v < vt.n_views; ++v) {
    const int64_t item = (int64_t)v * n + i;
    if (count[item] == 0) continue;
    double g[NV];
    bool any = false;
#pragma unroll
    for (int k = 0; k < NV; ++k) {
      g[k] = g2d[item * NV + k];
      any = any || g[k] != 0.0;
    }
    if (!any) continue;
    Cam cam;
    load_cam(cams, v, cam);
    Geo G;
    const Pin pin{0.0, 0.0, 0.0, 0.0};
    geometry(m, cam, cv, vt.W[v], vt.H[v], P, pin, G);
    double C[6], Sc[6];
    sph_cov(G, cam, cv, vt.H[v], P, C, Sc);
    const double r = G.r, ir2 = 1.0 / G.r2;
    const double mh[3] = {G.mu[0] / r, G.mu[1] / r, G.mu[2] / r};
    // full symmetric dL/dSigma~ from the shared-off-diagonal values
    const double gC[9] = {g[3], 0.5 * g[4], 0.5 * g[5], 0.5 * g[4], g[6], 0.5 * g[7], 0.5 * g[5], 0.5 * g[7], g[8]};
    const double Sfull[9] = {Sc[0], Sc[1], Sc[2], Sc[1], Sc[3], Sc[4], Sc[2], Sc[4], Sc[5]};
    double inner = 0.0;
#pragma unroll
    for (int e = 0; e < 9; ++e) inner += gC[e] * Sfull[e];
    const double gr = -2.0 * inner * ir2 / r;
    // W Sigma W^T:  dL/dSigma += W^T (dL/dSigma~ / r^2) W
    double RtG[9];
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int b = 0; b < 3; ++b)
        RtG[3 * a + b] = (cam.R[a] * gC[b] + cam.R[3 + a] * gC[3 + b] + cam.R[6 + a] * gC[6 + b]) * ir2;
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int b = 0; b < 3; ++b)
        gS[3 * a + b] += RtG[3 * a] * cam.R[b] + RtG[3 * a + 1] * cam.R[3 + b] + RtG[3 * a + 2] * cam.R[6 + b];
    // mu^ = mu / r, r = |mu|
    const double dot = g[0] * mh[0] + g[1] * mh[1] + g[2] * mh[2];
    double dmu[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) dmu[a] = (g[a] - mh[a] * dot) / r + mh[a] * gr;
#pragma unroll
    for (int k = 0; k < 3; ++k) gm[k] += cam.R[k] * dmu[0] + cam.R[3 + k] * dmu[1] + cam.R[6 + k] * dmu[2];
    go += g[9];  // the colour entries g[10..12] went to colour_bwd_kernel
  }
  write_param_grads(n, i, s, cv, gm, gS, go, d_means, d_scales, d_quats, d_opac);
}

Params make_params(const odgs_plan* p) {
  Params P;
  P.tile = p->s.tile;
  P.near_r = p->s.near_r;
  P.far_r = p->s.far_r;
  P.dilation = p->s.dilation;
  P.pole_eps = p->s.pole_eps;
  return P;
}

}  // namespace

constexpr unsigned kFoldMinBlocks = 512;

hipError_t launch_preprocess(const odgs_plan* p, const float* means, const float* scales, const float* quats,
                             const float* opac, const float* sh, const float* cams, void* ws, hipStream_t st) {
  if (p->n == 0) return hipSuccess;
  const ViewTable vt = make_view_table(p);
  const Params P = make_params(p);
  // a workgroup per (256-Gaussian chunk, view group), chunks padded to a multiple of the eight
  // XCDs; their item counts go to the radix histograms' region, unused until binning.  The
  // spherical footprint's per-item work is heavy enough to take a thread per item (at 500k
  // Gaussians and 8 views of 2048x1024: binning 1.39 -> 1.20 ms); the affine one does all views
  // in one thread, which computes the per-Gaussian part (covariance, opacity threshold) once
  // (two or four groups: 3.31 and 3.37 ms per step, against 3.30 ms).
  const int vgroups = plan_spherical(p) ? p->n_views : 1;
  const unsigned grid = (unsigned)preprocess_blocks(p->n, vgroups);
  // (up to kFoldMinBlocks workgroups add their counts with one atomic each, without the fold launch)
  uint32_t* part = grid > kFoldMinBlocks ? ws_ptr<uint32_t>(ws, p->off_hist) : nullptr;
  Rec* rec = ws_ptr<Rec>(ws, p->off_rec);
  Rect* rect = ws_ptr<Rect>(ws, p->off_rect);
  uint32_t* count = ws_ptr<uint32_t>(ws, p->off_count);
  uint32_t* dkey = ws_ptr<uint32_t>(ws, p->off_dkey[0]);
  float* depth = ws_ptr<float>(ws, p->off_depth);
  odgs_status* status = ws_ptr<odgs_status>(ws, p->off_status);
  double* g2d = ws_ptr<double>(ws, p->off_g2d);
  SphRec* srec = nullptr;
  SphCull* cone = nullptr;
  if (plan_spherical(p)) {
    srec = ws_ptr<SphRec>(ws, p->off_srec);
    cone = ws_ptr<SphCull>(ws, p->off_cone);
    const int entries = vt.dir_base[vt.n_views];
    hipLaunchKernelGGL(dir_table_kernel, dim3((unsigned)((entries + 255) / 256)), dim3(256), 0, st, vt,
                       ws_ptr<double2>(ws, p->off_dirs));
  }
#define ODGS_PRE(KK)                                                                                              \
  if (srec)                                                                                                       \
    hipLaunchKernelGGL((preprocess_kernel<KK, true>), dim3(grid), dim3(256), 0, st, p->n, means, scales, quats,     \
                       opac, sh, cams, vt, P, rec, rect, count, dkey, depth, status, srec, cone, g2d, p->g2d_stride,    \
                       vgroups, part);                                                                                  \
  else                                                                                                            \
    hipLaunchKernelGGL((preprocess_kernel<KK, false>), dim3(grid), dim3(256), 0, st, p->n, means, scales, quats,    \
                       opac, sh, cams, vt, P, rec, rect, count, dkey, depth, status, srec, cone, g2d, p->g2d_stride,    \
                       vgroups, part)
  switch (p->sh_degree) {
    case 0: ODGS_PRE(1); break;
    case 1: ODGS_PRE(4); break;
    case 2: ODGS_PRE(9); break;
    default: ODGS_PRE(16); break;
  }
#undef ODGS_PRE
  if (part) hipLaunchKernelGGL(count_fold_kernel, dim3(1), dim3(1024), 0, st, part, (int)grid, status);
  return hipGetLastError();
}

hipError_t launch_preprocess_bwd(const odgs_plan* p, const float* means, const float* scales, const float* quats,
                                 const float* opac, const float* sh, const float* cams, void* ws, float* d_means,
                                 float* d_scales, float* d_quats, float* d_opac, float* d_sh,
                                 const odgs_densify_acc* acc, hipStream_t st) {
  if (p->n == 0) return hipSuccess;
  DensAcc da{nullptr, nullptr, nullptr, 0.0, 0.0};
  if (acc) da = DensAcc{acc->grad_sum, acc->tau_sum, acc->count, (double)acc->tau_min, (double)acc->tau_max};
  const ViewTable vt = make_view_table(p);
  const Params P = make_params(p);
  const unsigned grid = (unsigned)((p->n + 255) / 256);
  const uint32_t* count = ws_ptr<uint32_t>(ws, p->off_count);
  double* g2d = ws_ptr<double>(ws, p->off_g2d);
  // colour part first (writes d_sh and the colour path of d_means), then the geometry part,
  // which adds to d_means
  const int stride = p->g2d_stride, off = p->g2d_stride - 3;
#define ODGS_COLB(KK)                                                                                              \
  hipLaunchKernelGGL(colour_bwd_kernel<KK>, dim3(grid), dim3(256), 0, st, p->n, means, sh, cams, vt, count, g2d,   \
                     stride, off, d_means, d_sh)
  switch (p->sh_degree) {
    case 0: ODGS_COLB(1); break;
    case 1: ODGS_COLB(4); break;
    case 2: ODGS_COLB(9); break;
    default: ODGS_COLB(16); break;
  }
#undef ODGS_COLB
#define ODGS_PREB(KK)                                                                                        \
  if (plan_spherical(p))                                                                                     \
    hipLaunchKernelGGL((preprocess_sph_bwd_kernel<KK>), dim3(grid), dim3(256), 0, st, p->n, means, scales,     \
                       quats, opac, sh, cams, vt, P, count, g2d, d_means, d_scales, d_quats, d_opac, d_sh);    \
  else if (acc)                                                                                              \
    hipLaunchKernelGGL((preprocess_bwd_kernel<KK, true>), dim3(grid), dim3(256), 0, st, p->n, means, scales,   \
                       quats, opac, sh, cams, vt, P, count, g2d, p->items, d_means, d_scales, d_quats, d_opac, \
                       d_sh, da);                                                                            \
  else                                                                                                       \
    hipLaunchKernelGGL((preprocess_bwd_kernel<KK, false>), dim3(grid), dim3(256), 0, st, p->n, means, scales,  \
                       quats, opac, sh, cams, vt, P, count, g2d, p->items, d_means, d_scales, d_quats, d_opac, \
                       d_sh, da)
  switch (p->sh_degree) {
    case 0: ODGS_PREB(1); break;
    case 1: ODGS_PREB(4); break;
    case 2: ODGS_PREB(9); break;
    default: ODGS_PREB(16); break;
  }
#undef ODGS_PREB
  return hipGetLastError();
}

}  // namespace odgs
