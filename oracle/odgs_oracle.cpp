/*
 * CPU reference ("oracle") for the ODGS omnidirectional Gaussian rasterizer
 * (Lee et al., "ODGS: 3D Scene Reconstruction from Omnidirectional Images with 3D Gaussian
 * Splattings", NeurIPS 2024, arXiv 2410.20686).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the package smoke check and the benchmark's
 * CPU-baseline leg load this library; the product path never calls it and shares no code with
 * it.  It is deliberately plain and slow:
 *
 *   - every geometric quantity is evaluated in double precision, following the paper's steps
 *     in the paper's order (Sec. 3.2: Eq. equirec_proj, Eq. omni_rotation, Eq. omni_J,
 *     Eq. omni_QS, Eq. omni_Jacobian);
 *   - every pixel is composited by brute force against every kept Gaussian of its view, in
 *     (radial depth, index) order (Sec. 3.1, Eq. gaussian2d and Eq. alphablending); tiles are
 *     not used for rendering except in the separate "band" mode, which must agree bit for bit;
 *   - the gradient is the exact derivative of the same definitions: a reverse recursion over
 *     each pixel's contributor list, then forward-mode dual numbers pushed through the very
 *     same per-Gaussian projection template (Appendix C gives a partial hand derivation; it is
 *     not transcribed here, the derivative is taken from the forward definition instead).
 *
 * Readings of points the paper leaves open (pixel centres, radial depth, seam wrap, pole and
 * shell culling, 3DGS compositing constants, footprint rectangle, SH colour model) are fixed
 * in the comments next to the code that implements them.
 *
 * Precision modes of the compositor: mode 64 keeps the per-Gaussian record in double and
 * composites in double (used for finite differences); mode 32 rounds the record to float and
 * takes every compositing decision (footprint test, opacity clamp, early termination) in float
 * with the same fused multiply-add form as the GPU kernel, so that both sides decide in the
 * kernel's precision.  Gradients are always accumulated in double.
 */
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>

#ifdef _OPENMP
#include <omp.h>
#endif

namespace {

// ----------------------------------------------------------------------------------------------
// Dual numbers: value + 11 partial derivatives (mean 3, scale 3, quaternion 4, opacity 1).
// ----------------------------------------------------------------------------------------------
constexpr int ND = 11;

struct Dual {
  double v;
  double d[ND];
  Dual() : v(0.0) { std::memset(d, 0, sizeof(d)); }
  Dual(double x) : v(x) { std::memset(d, 0, sizeof(d)); }  // NOLINT: implicit on purpose
};

inline Dual operator+(const Dual& a, const Dual& b) {
  Dual r(a.v + b.v);
  for (int k = 0; k < ND; ++k) r.d[k] = a.d[k] + b.d[k];
  return r;
}
inline Dual operator-(const Dual& a, const Dual& b) {
  Dual r(a.v - b.v);
  for (int k = 0; k < ND; ++k) r.d[k] = a.d[k] - b.d[k];
  return r;
}
inline Dual operator-(const Dual& a) {
  Dual r(-a.v);
  for (int k = 0; k < ND; ++k) r.d[k] = -a.d[k];
  return r;
}
inline Dual operator*(const Dual& a, const Dual& b) {
  Dual r(a.v * b.v);
  for (int k = 0; k < ND; ++k) r.d[k] = a.d[k] * b.v + a.v * b.d[k];
  return r;
}
inline Dual operator/(const Dual& a, const Dual& b) {
  Dual r(a.v / b.v);
  for (int k = 0; k < ND; ++k) r.d[k] = (a.d[k] * b.v - a.v * b.d[k]) / (b.v * b.v);
  return r;
}
inline Dual operator+(const Dual& a, double b) { return a + Dual(b); }
inline Dual operator+(double a, const Dual& b) { return Dual(a) + b; }
inline Dual operator-(const Dual& a, double b) { return a - Dual(b); }
inline Dual operator-(double a, const Dual& b) { return Dual(a) - b; }
inline Dual operator*(const Dual& a, double b) { return a * Dual(b); }
inline Dual operator*(double a, const Dual& b) { return Dual(a) * b; }
inline Dual operator/(const Dual& a, double b) { return a / Dual(b); }
inline Dual operator/(double a, const Dual& b) { return Dual(a) / b; }

inline Dual chain(const Dual& a, double fv, double dfda) {
  Dual r(fv);
  for (int k = 0; k < ND; ++k) r.d[k] = dfda * a.d[k];
  return r;
}
inline Dual sqrt(const Dual& a) { double s = std::sqrt(a.v); return chain(a, s, 0.5 / s); }
inline Dual cos(const Dual& a) { return chain(a, std::cos(a.v), -std::sin(a.v)); }
inline Dual sin(const Dual& a) { return chain(a, std::sin(a.v), std::cos(a.v)); }
inline Dual atan2(const Dual& y, const Dual& x) {
  Dual r(std::atan2(y.v, x.v));
  double den = x.v * x.v + y.v * y.v;
  for (int k = 0; k < ND; ++k) r.d[k] = (x.v * y.d[k] - y.v * x.d[k]) / den;
  return r;
}

inline double val(double x) { return x; }
inline double val(const Dual& x) { return x.v; }
using std::atan2;
using std::cos;
using std::sin;
using std::sqrt;

// ----------------------------------------------------------------------------------------------
// Inputs
// ----------------------------------------------------------------------------------------------
struct Camera {
  double R[9];  // world -> camera rotation, row-major (the paper's W, Sec. 3.1)
  double t[3];
  int W, H;
  bool pinhole = false;  // perspective camera of Sec. 3.1 (else equirectangular, Sec. 3.2)
  double fx = 0, fy = 0, cx = 0, cy = 0;  // its intrinsics K
};

struct Settings {
  bool spherical = false;  // exact per-ray footprint in equirectangular views (see project())
  int tile;          // tile edge in pixels (binning only)
  double near_r;     // spherical-shell culling radii (Sec. 3.2: shell instead of frustum)
  double far_r;
  double dilation;   // added to the diagonal of the 2D covariance (3DGS low-pass)
  double pole_eps;   // cull when the horizontal radius is below pole_eps * r
  double bg[3];      // background colour behind the final transmittance
};

struct Scene {
  const double *means, *scales, *quats, *opac, *sh;  // SoA, see the Python wrapper
  int64_t n;
  int K;  // number of SH basis functions, (degree+1)^2
};

// Settings array: [tile, near, far, dilation, pole_eps, bg0, bg1, bg2, P] followed by P records
// (view, fx, fy, cx, cy) marking pinhole views, then the footprint model (0 affine, 1 spherical).
void read_pinholes(const double* s, std::vector<Camera>& cams) {
  const int P = (int)s[8];
  for (int k = 0; k < P; ++k) {
    const double* r = s + 9 + 5 * k;
    Camera& c = cams[(int)r[0]];
    c.pinhole = true;
    c.fx = r[1];
    c.fy = r[2];
    c.cx = r[3];
    c.cy = r[4];
  }
}

Settings read_settings(const double* s) {
  Settings st;
  st.tile = (int)s[0];
  st.near_r = s[1];
  st.far_r = s[2];
  st.dilation = s[3];
  st.pole_eps = s[4];
  st.bg[0] = s[5];
  st.bg[1] = s[6];
  st.bg[2] = s[7];
  st.spherical = s[9 + 5 * (int)s[8]] != 0.0;
  return st;
}

std::vector<Camera> read_cameras(const double* cams, const int32_t* wh, int V) {
  std::vector<Camera> out(V);
  for (int v = 0; v < V; ++v) {
    for (int k = 0; k < 9; ++k) out[v].R[k] = cams[v * 12 + k];
    for (int k = 0; k < 3; ++k) out[v].t[k] = cams[v * 12 + 9 + k];
    out[v].W = wh[2 * v];
    out[v].H = wh[2 * v + 1];
  }
  return out;
}

// ----------------------------------------------------------------------------------------------
// Real spherical harmonics up to degree 3 (orthonormal on the unit sphere, no Condon-Shortley
// phase), in (l, m = -l..l) order.  The paper only speaks of a per-Gaussian colour c_j
// (Eq. alphablending); the view-dependent SH colour is the 3DGS colour model it inherits.
// ----------------------------------------------------------------------------------------------
template <typename S>
void sh_basis(const S d[3], int K, S* Y) {
  const double pi = M_PI;
  const S& x = d[0];
  const S& y = d[1];
  const S& z = d[2];
  Y[0] = S(0.5 * std::sqrt(1.0 / pi));
  if (K <= 1) return;
  const double c1 = std::sqrt(3.0 / (4.0 * pi));
  Y[1] = c1 * y;
  Y[2] = c1 * z;
  Y[3] = c1 * x;
  if (K <= 4) return;
  const double c2a = 0.5 * std::sqrt(15.0 / pi);
  const double c2b = 0.25 * std::sqrt(5.0 / pi);
  const double c2c = 0.25 * std::sqrt(15.0 / pi);
  Y[4] = c2a * (x * y);
  Y[5] = c2a * (y * z);
  Y[6] = c2b * (2.0 * (z * z) - x * x - y * y);
  Y[7] = c2a * (x * z);
  Y[8] = c2c * (x * x - y * y);
  if (K <= 9) return;
  const double c3a = 0.25 * std::sqrt(35.0 / (2.0 * pi));
  const double c3b = 0.5 * std::sqrt(105.0 / pi);
  const double c3c = 0.25 * std::sqrt(21.0 / (2.0 * pi));
  const double c3d = 0.25 * std::sqrt(7.0 / pi);
  const double c3e = 0.25 * std::sqrt(105.0 / pi);
  Y[9] = c3a * (y * (3.0 * (x * x) - y * y));
  Y[10] = c3b * (x * y * z);
  Y[11] = c3c * (y * (4.0 * (z * z) - x * x - y * y));
  Y[12] = c3d * (z * (2.0 * (z * z) - 3.0 * (x * x) - 3.0 * (y * y)));
  Y[13] = c3c * (x * (4.0 * (z * z) - x * x - y * y));
  Y[14] = c3e * (z * (x * x - y * y));
  Y[15] = c3a * (x * (x * x - 3.0 * (y * y)));
}

// ----------------------------------------------------------------------------------------------
// Per-(Gaussian, view) projection.  Differentiable outputs go to Proj<S>; discrete outcomes and
// double-valued intermediates go to Info.
// ----------------------------------------------------------------------------------------------
enum Cull { KEPT = 0, CULL_SHELL = 1, CULL_POLE = 2, CULL_OPACITY = 3, CULL_DET = 4, CULL_EMPTY = 5,
            CULL_NONFINITE = 6, CULL_FRUSTUM = 7 };

template <typename S>
struct Proj {
  S u, v;         // ERP pixel position of the mean
  S conic[3];     // inverse 2D covariance (a, b, c) of [[a, b], [b, c]]
  S cov2[3];      // 2D covariance (uu, uv, vv), dilation included
  S opacity;
  S rgb[3];
  // spherical footprint (equirectangular views with Settings::spherical):
  S mu_hat[3];    // unit direction of the camera-space mean
  S C[6];         // normalised covariance Sigma~ (xx xy xz yy yz zz)
  S A[6];         // its inverse
};

struct Info {
  int cull;
  float depth;         // radial distance, rounded to float (the sort key)
  double mu[3], r, rho;
  double J[6];         // J_omni, row-major 2x3
  double cov3[6];      // xx xy xz yy yz zz
  double cov2[3];      // uu uv vv, dilation included
  double p_min;        // log-opacity threshold: alpha >= 1/255  <=>  power >= p_min
  double rgb_raw[3];   // colour before the clamp at zero
  int rgb_clamped[3];
  int col0, ncols, row0, nrows;  // tile rectangle (columns wrap around the seam)
  bool spherical;      // evaluated with the spherical footprint
  double scov[6];      // normalised camera-space covariance Sigma~ (xx xy xz yy yz zz)
  double beta;         // half-angle of the cone of rays that can reach alpha >= 1/255
};

// Angular extent of the rays that can reach alpha >= 1/255 under the spherical footprint,
// through the tangent plane of mu^ (frame e1 east, e2 = mu^ x e1) in gnomonic coordinates
// p = (d . e1, d . e2) / (d . mu^).  There m <= k^2 reads (1 - k^2 kappa) p^T P^-1 p <=
// k^2 (1 + a . p)^2 with P, c, s33 the tangent, tangent-radial and radial blocks of Sigma~,
// a = -P^-1 c and kappa = s33 - c^T P^-1 c: the ellipse (p - p0)^T M (p - p0) <= rho^2,
// M = (1 - k^2 kappa) P^-1 - k^2 a a^T, p0 = k^2 M^-1 a, rho^2 = k^2 + k^4 a^T M^-1 a, whenever
// k^2 s33 < 1.  Its bounding box (half-widths rho sqrt((M^-1)_ii), padded by 1e-3) is a
// spherical quadrilateral whose edges are great-circle arcs: along such an arc the longitude is
// monotonic, so the longitude range is that of the four corners; the latitude extremes are at
// the corners or at an arc's highest (lowest) point when that lies on the arc; a pole inside the
// box takes every longitude.  Returns false when the ellipse form does not apply.
struct SphBox {
  double sin_lo, sin_hi;    // range of sin(latitude) = -d_y
  double dphi_lo, dphi_hi;  // longitude range relative to the mean's azimuth
  bool north, south;        // a pole inside the box
};

bool sph_box(const double m[3], const double C[6], double p_min, double phic, SphBox& bx) {
  auto sym = [&](const double* x, const double* y) {
    return x[0] * (C[0] * y[0] + C[1] * y[1] + C[2] * y[2]) + x[1] * (C[1] * y[0] + C[3] * y[1] + C[4] * y[2]) +
           x[2] * (C[2] * y[0] + C[4] * y[1] + C[5] * y[2]);
  };
  const double rh = std::sqrt(m[0] * m[0] + m[2] * m[2]);
  const double e1[3] = {m[2] / rh, 0.0, -m[0] / rh};
  const double e2[3] = {m[1] * e1[2] - m[2] * e1[1], m[2] * e1[0] - m[0] * e1[2], m[0] * e1[1] - m[1] * e1[0]};
  const double P11 = sym(e1, e1), P12 = sym(e1, e2), P22 = sym(e2, e2);
  const double c1 = sym(e1, m), c2 = sym(e2, m), s33 = sym(m, m);
  const double det = P11 * P22 - P12 * P12;
  const double a1 = -(P22 * c1 - P12 * c2) / det, a2 = -(P11 * c2 - P12 * c1) / det;
  const double kk = -2.0 * p_min;
  const double f = 1.0 - kk * (s33 + (a1 * c1 + a2 * c2));
  const double M11 = f * (P22 / det) - kk * a1 * a1, M12 = f * (-P12 / det) - kk * a1 * a2;
  const double M22 = f * (P11 / det) - kk * a2 * a2;
  const double detM = M11 * M22 - M12 * M12;
  if (!(kk * s33 < 0.999 && detM > 0.0 && M11 > 0.0)) return false;
  const double q0 = (M22 * a1 - M12 * a2) / detM, q1 = (M11 * a2 - M12 * a1) / detM;
  const double p0[2] = {kk * q0, kk * q1};
  const double rho2 = kk + kk * kk * (a1 * q0 + a2 * q1);
  const double hx = std::sqrt(rho2 * M22 / detM) * (1.0 + 1e-3), hy = std::sqrt(rho2 * M11 / detM) * (1.0 + 1e-3);
  // poles: gnomonic image inside the box
  bx.north = bx.south = false;
  for (int sgn = -1; sgn <= 1; sgn += 2) {  // north = (0, -1, 0), south = (0, 1, 0)
    const double sdot = sgn * m[1];
    if (!(sdot > 0.0)) continue;
    const double px = sgn * e1[1] / sdot, py = sgn * e2[1] / sdot;
    if (std::fabs(px - p0[0]) <= hx && std::fabs(py - p0[1]) <= hy) (sgn < 0 ? bx.north : bx.south) = true;
  }
  double D[4][3];
  const double sx[4] = {-1.0, 1.0, 1.0, -1.0}, sy[4] = {-1.0, -1.0, 1.0, 1.0};
  bx.sin_lo = 2.0;
  bx.sin_hi = -2.0;
  bx.dphi_lo = 10.0;
  bx.dphi_hi = -10.0;
  for (int k = 0; k < 4; ++k) {
    const double px = p0[0] + sx[k] * hx, py = p0[1] + sy[k] * hy;
    double nrm2 = 0.0;
    for (int j = 0; j < 3; ++j) {
      D[k][j] = m[j] + px * e1[j] + py * e2[j];
      nrm2 += D[k][j] * D[k][j];
    }
    const double nrm = std::sqrt(nrm2);
    for (int j = 0; j < 3; ++j) D[k][j] /= nrm;
    bx.sin_lo = std::min(bx.sin_lo, -D[k][1]);
    bx.sin_hi = std::max(bx.sin_hi, -D[k][1]);
    double dp = std::atan2(D[k][0], D[k][2]) - phic;
    if (dp > M_PI) dp -= 2.0 * M_PI;
    if (dp < -M_PI) dp += 2.0 * M_PI;
    bx.dphi_lo = std::min(bx.dphi_lo, dp);
    bx.dphi_hi = std::max(bx.dphi_hi, dp);
  }
  // highest / lowest point of each edge's great circle, when it lies on the edge
  for (int k = 0; k < 4; ++k) {
    const double* A = D[k];
    const double* Bv = D[(k + 1) % 4];
    const double n[3] = {A[1] * Bv[2] - A[2] * Bv[1], A[2] * Bv[0] - A[0] * Bv[2], A[0] * Bv[1] - A[1] * Bv[0]};
    const double nn = n[0] * n[0] + n[1] * n[1] + n[2] * n[2];
    if (!(nn > 0.0)) continue;
    for (int sgn = -1; sgn <= 1; sgn += 2) {  // towards north (0, -1, 0), then south (0, 1, 0)
      // projection of the pole direction onto the circle's plane
      double v[3] = {-(sgn * n[1]) * n[0] / nn, sgn - (sgn * n[1]) * n[1] / nn, -(sgn * n[1]) * n[2] / nn};
      const double vn = std::sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
      if (!(vn > 0.0)) continue;
      for (int j = 0; j < 3; ++j) v[j] /= vn;
      const double t1 = (A[1] * v[2] - A[2] * v[1]) * n[0] + (A[2] * v[0] - A[0] * v[2]) * n[1] +
                        (A[0] * v[1] - A[1] * v[0]) * n[2];
      const double t2 = (v[1] * Bv[2] - v[2] * Bv[1]) * n[0] + (v[2] * Bv[0] - v[0] * Bv[2]) * n[1] +
                        (v[0] * Bv[1] - v[1] * Bv[0]) * n[2];
      if (t1 >= 0.0 && t2 >= 0.0) {
        bx.sin_lo = std::min(bx.sin_lo, -v[1]);
        bx.sin_hi = std::max(bx.sin_hi, -v[1]);
      }
    }
  }
  if (bx.north) bx.sin_hi = 1.0;
  if (bx.south) bx.sin_lo = -1.0;
  return true;
}

template <typename S>
void project(const S m[3], const S s[3], const S q[4], const S& o, const double* shg, int64_t sh_stride,
             int K, const Camera& cam, const Settings& st, Proj<S>& out, Info& info) {
  info.cull = KEPT;
  info.spherical = false;
  info.beta = 0.0;
  const double pi = M_PI;
  const double Wd = cam.W, Hd = cam.H;

  // Camera-space mean: mu = W m + t (Sec. 3.1, W = world-to-camera transform).  The products
  // are summed in a fixed order without fused multiply-add: the radial depth computed from mu
  // is a sort key, and the GPU reproduces exactly this sequence.
  S mu[3];
  for (int r = 0; r < 3; ++r)
    mu[r] = ((cam.R[3 * r + 0] * m[0] + cam.R[3 * r + 1] * m[1]) + cam.R[3 * r + 2] * m[2]) + cam.t[r];
  const S r2 = (mu[0] * mu[0] + mu[1] * mu[1]) + mu[2] * mu[2];
  const S rr = sqrt(r2);
  const S rho = sqrt(mu[0] * mu[0] + mu[2] * mu[2]);
  for (int k = 0; k < 3; ++k) info.mu[k] = val(mu[k]);
  info.r = val(rr);
  info.rho = val(rho);
  info.depth = (float)val(cam.pinhole ? mu[2] : rr);

  S phi = S(0.0), theta = S(0.0);
  if (cam.pinhole) {
    // Perspective camera (Sec. 3.1): depth range on the camera's z, and a guard band of 1.3
    // times the field of view around the image for the projected mean.
    const double z = val(mu[2]);
    if (!(z > st.near_r && z < st.far_r)) { info.cull = CULL_SHELL; return; }
    if (!(std::fabs(val(mu[0]) / z) <= 1.3 * (Wd / (2.0 * cam.fx)) &&
          std::fabs(val(mu[1]) / z) <= 1.3 * (Hd / (2.0 * cam.fy)))) {
      info.cull = CULL_FRUSTUM;
      return;
    }
    // pi(mu) = K_{1:2} (mu_x / mu_z, mu_y / mu_z, 1)
    out.u = cam.fx * (mu[0] / mu[2]) + cam.cx;
    out.v = cam.fy * (mu[1] / mu[2]) + cam.cy;
  } else {
    // Culling in a spherical shell (Sec. 3.2, last paragraph) instead of a view frustum.
    if (!(val(rr) > st.near_r && val(rr) < st.far_r)) { info.cull = CULL_SHELL; return; }
    // At the poles the azimuth is undefined and sec(theta) diverges (Eq. omni_QS); such
    // Gaussians are dropped.
    if (!(val(rho) > st.pole_eps * val(rr))) { info.cull = CULL_POLE; return; }
    // Spherical coordinates (Sec. 3.2): azimuth from +z, elevation from the z-x plane, with y
    // pointing down.  atan2 gives the stated ranges [-pi, pi] and [-pi/2, pi/2].
    phi = atan2(mu[0], mu[2]);
    theta = atan2(-mu[1], rho);
    // Eq. equirec_proj.
    out.u = (Wd / (2.0 * pi)) * phi + Wd / 2.0;
    out.v = (-Hd / pi) * theta + Hd / 2.0;
  }

  // 3D covariance Sigma = R S S^T R^T (Sec. 3.1) from the normalised quaternion (w, x, y, z).
  const S qn = sqrt(((q[0] * q[0] + q[1] * q[1]) + q[2] * q[2]) + q[3] * q[3]);
  const S w = q[0] / qn, x = q[1] / qn, y = q[2] / qn, z = q[3] / qn;
  S Rq[9];
  Rq[0] = 1.0 - 2.0 * (y * y + z * z);
  Rq[1] = 2.0 * (x * y - w * z);
  Rq[2] = 2.0 * (x * z + w * y);
  Rq[3] = 2.0 * (x * y + w * z);
  Rq[4] = 1.0 - 2.0 * (x * x + z * z);
  Rq[5] = 2.0 * (y * z - w * x);
  Rq[6] = 2.0 * (x * z - w * y);
  Rq[7] = 2.0 * (y * z + w * x);
  Rq[8] = 1.0 - 2.0 * (x * x + y * y);
  S M[9];
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c) M[3 * r + c] = Rq[3 * r + c] * s[c];
  S Sig[9];
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c) Sig[3 * r + c] = (M[3 * r + 0] * M[3 * c + 0] + M[3 * r + 1] * M[3 * c + 1]) +
                                                 M[3 * r + 2] * M[3 * c + 2];
  info.cov3[0] = val(Sig[0]); info.cov3[1] = val(Sig[1]); info.cov3[2] = val(Sig[2]);
  info.cov3[3] = val(Sig[4]); info.cov3[4] = val(Sig[5]); info.cov3[5] = val(Sig[8]);

  // Spherical footprint (the paper's stated limitation of the local affine approximation, Sec. 5,
  // addressed exactly): instead of a 2D Gaussian on the image, each pixel ray t d (t > 0) is
  // given the largest value the 3D Gaussian takes along it, exp(-m/2) with
  //   m(d) = min_t (t d - mu)^T Sigma_cam^-1 (t d - mu).
  // m is unchanged when mu and Sigma_cam are scaled by 1/r and 1/r^2, so the quadratic form is
  // kept at unit distance: mu^ = mu / r, Sigma~ = Sigma_cam / r^2 + delta I.  The 3DGS low-pass
  // term becomes an isotropic angular variance delta = dilation (pi / H)^2 (dilation in squared
  // pixels at the vertical pixel pitch).
  info.spherical = st.spherical && !cam.pinhole;
  S detA = S(1.0);
  if (info.spherical) {
    S RS[9], Sc[9];  // W Sigma, then W Sigma W^T
    for (int r = 0; r < 3; ++r)
      for (int c = 0; c < 3; ++c)
        RS[3 * r + c] = (cam.R[3 * r + 0] * Sig[0 * 3 + c] + cam.R[3 * r + 1] * Sig[1 * 3 + c]) + cam.R[3 * r + 2] * Sig[2 * 3 + c];
    for (int r = 0; r < 3; ++r)
      for (int c = 0; c < 3; ++c)
        Sc[3 * r + c] = (RS[3 * r + 0] * cam.R[3 * c + 0] + RS[3 * r + 1] * cam.R[3 * c + 1]) + RS[3 * r + 2] * cam.R[3 * c + 2];
    const double dang = st.dilation * (pi / Hd) * (pi / Hd);
    const S ir2 = 1.0 / r2;
    const S C[6] = {Sc[0] * ir2 + dang, Sc[1] * ir2, Sc[2] * ir2, Sc[4] * ir2 + dang, Sc[5] * ir2, Sc[8] * ir2 + dang};
    for (int k = 0; k < 6; ++k) {
      info.scov[k] = val(C[k]);
      out.C[k] = C[k];
    }
    // inverse by cofactors: [[a, b, c], [b, d, e], [c, e, f]]
    const S &a = C[0], &b = C[1], &c = C[2], &d = C[3], &e = C[4], &f = C[5];
    const S c00 = d * f - e * e, c01 = c * e - b * f, c02 = b * e - c * d;
    const S c11 = a * f - c * c, c12 = b * c - a * e, c22 = a * d - b * b;
    const S det3 = (a * c00 + b * c01) + c * c02;
    out.A[0] = c00 / det3; out.A[1] = c01 / det3; out.A[2] = c02 / det3;
    out.A[3] = c11 / det3; out.A[4] = c12 / det3; out.A[5] = c22 / det3;
    detA = det3;
    for (int k = 0; k < 3; ++k) out.mu_hat[k] = mu[k] / rr;
  }

  S J[6];
  if (cam.pinhole) {
    // Eq. jacob_pers.
    J[0] = cam.fx / mu[2];
    J[1] = S(0.0);
    J[2] = -cam.fx * mu[0] / (mu[2] * mu[2]);
    J[3] = S(0.0);
    J[4] = cam.fy / mu[2];
    J[5] = -cam.fy * mu[1] / (mu[2] * mu[2]);
  } else {
  // Tangent-plane projection.  Eq. omni_rotation: T_mu = T_theta * T_phi turns the camera's z
  // axis towards mu.  Eq. omni_J: unit-focal perspective Jacobian at mu_o = (0, 0, |mu|).
  // Eq. omni_QS: horizontal ERP stretch sec(theta), then pixel scale (W/2pi, H/pi).
  // Eq. omni_Jacobian: J_omni = S_o Q_o J_o T_mu.
  const S ct = cos(theta), st_ = sin(theta), cp = cos(phi), sp = sin(phi);
  S Tth[9] = {S(1.0), S(0.0), S(0.0), S(0.0), ct, st_, S(0.0), -st_, ct};
  S Tph[9] = {cp, S(0.0), -sp, S(0.0), S(1.0), S(0.0), sp, S(0.0), cp};
  S Tmu[9];
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c)
      Tmu[3 * r + c] = (Tth[3 * r + 0] * Tph[0 * 3 + c] + Tth[3 * r + 1] * Tph[1 * 3 + c]) + Tth[3 * r + 2] * Tph[2 * 3 + c];
  S Jo[6] = {1.0 / rr, S(0.0), S(0.0), S(0.0), 1.0 / rr, S(0.0)};
  S Qo[4] = {1.0 / ct, S(0.0), S(0.0), S(1.0)};
  S So[4] = {S(Wd / (2.0 * pi)), S(0.0), S(0.0), S(Hd / pi)};
  S SQ[4];
  for (int r = 0; r < 2; ++r)
    for (int c = 0; c < 2; ++c) SQ[2 * r + c] = So[2 * r + 0] * Qo[0 * 2 + c] + So[2 * r + 1] * Qo[1 * 2 + c];
  S SQJ[6];
  for (int r = 0; r < 2; ++r)
    for (int c = 0; c < 3; ++c) SQJ[3 * r + c] = SQ[2 * r + 0] * Jo[0 * 3 + c] + SQ[2 * r + 1] * Jo[1 * 3 + c];
  for (int r = 0; r < 2; ++r)
    for (int c = 0; c < 3; ++c)
      J[3 * r + c] = (SQJ[3 * r + 0] * Tmu[0 * 3 + c] + SQJ[3 * r + 1] * Tmu[1 * 3 + c]) + SQJ[3 * r + 2] * Tmu[2 * 3 + c];
  }
  for (int k = 0; k < 6; ++k) info.J[k] = val(J[k]);

  // Sigma_2D,o = J_omni W Sigma W^T J_omni^T (below Eq. omni_Jacobian).
  S A[6];  // J_omni * W
  for (int r = 0; r < 2; ++r)
    for (int c = 0; c < 3; ++c)
      A[3 * r + c] = (J[3 * r + 0] * cam.R[0 * 3 + c] + J[3 * r + 1] * cam.R[1 * 3 + c]) + J[3 * r + 2] * cam.R[2 * 3 + c];
  S AS[6];  // A * Sigma
  for (int r = 0; r < 2; ++r)
    for (int c = 0; c < 3; ++c)
      AS[3 * r + c] = (A[3 * r + 0] * Sig[0 * 3 + c] + A[3 * r + 1] * Sig[1 * 3 + c]) + A[3 * r + 2] * Sig[2 * 3 + c];
  S c2[3];
  c2[0] = (AS[0] * A[0] + AS[1] * A[1]) + AS[2] * A[2];
  c2[1] = (AS[0] * A[3] + AS[1] * A[4]) + AS[2] * A[5];
  c2[2] = (AS[3] * A[3] + AS[4] * A[4]) + AS[5] * A[5];
  // 3DGS low-pass filter: a constant added to the 2D covariance's diagonal.
  c2[0] = c2[0] + st.dilation;
  c2[2] = c2[2] + st.dilation;
  for (int k = 0; k < 3; ++k) {
    info.cov2[k] = val(c2[k]);
    out.cov2[k] = c2[k];
  }
  const S det = c2[0] * c2[2] - c2[1] * c2[1];
  // Inverse covariance for Eq. gaussian2d.
  out.conic[0] = c2[2] / det;
  out.conic[1] = -c2[1] / det;
  out.conic[2] = c2[0] / det;
  out.opacity = o;

  // View-dependent colour: real SH of the world-space direction from the camera centre
  // c = -R^T t to the mean, plus 0.5, clamped at zero.
  double cc[3];
  for (int k = 0; k < 3; ++k) cc[k] = -((cam.R[0 * 3 + k] * cam.t[0] + cam.R[1 * 3 + k] * cam.t[1]) + cam.R[2 * 3 + k] * cam.t[2]);
  S dv[3] = {m[0] - cc[0], m[1] - cc[1], m[2] - cc[2]};
  const S dn = sqrt((dv[0] * dv[0] + dv[1] * dv[1]) + dv[2] * dv[2]);
  S dir[3] = {dv[0] / dn, dv[1] / dn, dv[2] / dn};
  S Y[16];
  sh_basis(dir, K, Y);
  bool finite = std::isfinite(val(out.u)) && std::isfinite(val(out.v));
  for (int ch = 0; ch < 3; ++ch) {
    S acc = S(0.0);
    for (int k = 0; k < K; ++k) acc = acc + shg[(int64_t)(k * 3 + ch) * sh_stride] * Y[k];
    acc = acc + 0.5;
    info.rgb_raw[ch] = val(acc);
    info.rgb_clamped[ch] = !(val(acc) > 0.0);
    out.rgb[ch] = info.rgb_clamped[ch] ? S(0.0) : acc;
    finite = finite && std::isfinite(val(acc));
  }

  // alpha = o * G >= 1/255 (the 3DGS cut-off) is tested as power >= p_min with
  // p_min = -ln(255 o); Gaussians with o <= 1/255 never contribute.
  info.p_min = -std::log(255.0 * val(o));
  if (!(info.p_min < 0.0)) { info.cull = CULL_OPACITY; return; }
  if (!(val(info.spherical ? detA : det) > 0.0)) { info.cull = CULL_DET; return; }
  if (!finite) { info.cull = CULL_NONFINITE; return; }

  const int B = st.tile;
  const int ntx = cam.W / B, nty = cam.H / B;
  if (info.spherical) {
    // Rays with m <= k^2 and a positive minimiser meet the ellipsoid m <= k^2 around mu^, which
    // lies inside the ball of radius k sqrt(lambda_max(Sigma~)); the rays through that ball form
    // a cone of half-angle beta = asin(k sqrt(lambda_max)) about mu^ (all directions when the
    // ball holds the camera).  lambda_max(Sigma~) = max_i s_i^2 / r^2 + delta exactly.  The
    // cone's latitude range is theta_c +- beta; its longitude half-width asin(sin beta / cos
    // theta_c) unless it reaches a pole (then every column).  Padding as for the ellipse.
    double smax2 = 0.0;
    for (int k = 0; k < 3; ++k) smax2 = std::max(smax2, val(s[k]) * val(s[k]));
    const double lam = smax2 / (info.r * info.r) + st.dilation * (pi / Hd) * (pi / Hd);
    const double sb = std::sqrt(-2.0 * info.p_min * lam) * (1.0 + 1e-3);
    const double thc = val(theta);
    if (!(sb < 1.0)) {
      info.beta = pi;
      info.col0 = 0; info.ncols = ntx; info.row0 = 0; info.nrows = nty;
      return;
    }
    const double beta = std::asin(sb);
    info.beta = beta;
    const double mh[3] = {info.mu[0] / info.r, info.mu[1] / info.r, info.mu[2] / info.r};
    SphBox bx;
    if (sph_box(mh, info.scov, info.p_min, val(phi), bx)) {
      // the box of the gnomonic ellipse (tighter than the cone for anisotropic footprints)
      const double vlo = Hd / 2.0 - (Hd / pi) * std::asin(std::min(1.0, bx.sin_hi)) - 1e-2;
      const double vhi = Hd / 2.0 - (Hd / pi) * std::asin(std::max(-1.0, bx.sin_lo)) + 1e-2;
      const double rlo = std::max(0.0, std::floor(vlo / B)), rhi = std::min((double)(nty - 1), std::floor(vhi / B));
      info.row0 = (int)rlo;
      info.nrows = (int)(rhi - rlo + 1.0);
      if (info.nrows <= 0) { info.cull = CULL_EMPTY; return; }
      const double uu = val(out.u);
      const double clo = std::floor((uu + (Wd / (2.0 * pi)) * bx.dphi_lo - 1e-2) / B);
      const double chi = std::floor((uu + (Wd / (2.0 * pi)) * bx.dphi_hi + 1e-2) / B);
      if (bx.north || bx.south || !(chi - clo + 1.0 < (double)ntx)) {
        info.col0 = 0;
        info.ncols = ntx;
      } else {
        long long c0 = (long long)clo % ntx;
        if (c0 < 0) c0 += ntx;
        info.col0 = (int)c0;
        info.ncols = (int)(chi - clo + 1.0);
      }
      return;
    }
    const double vlo = Hd / 2.0 - (Hd / pi) * (thc + beta) - 1e-2, vhi = Hd / 2.0 - (Hd / pi) * (thc - beta) + 1e-2;
    const double rlo = std::max(0.0, std::floor(vlo / B)), rhi = std::min((double)(nty - 1), std::floor(vhi / B));
    info.row0 = (int)rlo;
    info.nrows = (int)(rhi - rlo + 1.0);
    if (info.nrows <= 0) { info.cull = CULL_EMPTY; return; }
    if (!(std::fabs(thc) + beta < pi / 2.0)) {
      info.col0 = 0;
      info.ncols = ntx;
      return;
    }
    const double eu = (Wd / (2.0 * pi)) * std::asin(std::sin(beta) / std::cos(thc)) + 1e-2;
    const double uu = val(out.u);
    const double clo = std::floor((uu - eu) / B), chi = std::floor((uu + eu) / B);
    if (!(chi - clo + 1.0 < (double)ntx)) {
      info.col0 = 0;
      info.ncols = ntx;
    } else {
      long long c0 = (long long)clo % ntx;
      if (c0 < 0) c0 += ntx;
      info.col0 = (int)c0;
      info.ncols = (int)(chi - clo + 1.0);
    }
    return;
  }

  // Footprint rectangle: the ellipse d^T Sigma^-1 d <= k^2 with k^2 = -2 p_min bounds every
  // pixel where alpha >= 1/255; its half-extents are sqrt(k^2 Sigma_uu), sqrt(k^2 Sigma_vv),
  // padded by 0.1% + 0.01 px against float rounding in the compositor.
  const double k2 = -2.0 * info.p_min;
  const double eu = std::sqrt(k2 * info.cov2[0]) * (1.0 + 1e-3) + 1e-2;
  const double ev = std::sqrt(k2 * info.cov2[2]) * (1.0 + 1e-3) + 1e-2;
  const double uu = val(out.u), vv = val(out.v);
  const double clo = std::floor((uu - eu) / B), chi = std::floor((uu + eu) / B);
  if (cam.pinhole) {
    // no seam: columns clamp at the image edges like the rows
    const double c0 = std::max(0.0, clo), c1 = std::min((double)(ntx - 1), chi);
    info.col0 = (int)std::max(0.0, std::min(c0, (double)ntx));
    info.ncols = (int)(c1 - c0 + 1.0);
    if (info.ncols <= 0) { info.cull = CULL_EMPTY; return; }
  } else if (!(chi - clo + 1.0 < (double)ntx)) {
    info.col0 = 0;
    info.ncols = ntx;
  } else {
    long long c0 = (long long)clo % ntx;
    if (c0 < 0) c0 += ntx;
    info.col0 = (int)c0;
    info.ncols = (int)(chi - clo + 1.0);
  }
  const double rlo = std::max(0.0, std::floor((vv - ev) / B));
  const double rhi = std::min((double)(nty - 1), std::floor((vv + ev) / B));
  info.row0 = (int)rlo;
  info.nrows = (int)(rhi - rlo + 1.0);
  if (info.nrows <= 0) { info.cull = CULL_EMPTY; return; }
}

// Evaluate the projection of item (gaussian i, view) in double.
void project_item(const Scene& sc, int64_t i, const Camera& cam, const Settings& st, Proj<double>& p, Info& info) {
  const int64_t n = sc.n;
  double m[3] = {sc.means[i], sc.means[n + i], sc.means[2 * n + i]};
  double s[3] = {sc.scales[i], sc.scales[n + i], sc.scales[2 * n + i]};
  double q[4] = {sc.quats[i], sc.quats[n + i], sc.quats[2 * n + i], sc.quats[3 * n + i]};
  double o = sc.opac[i];
  project<double>(m, s, q, o, sc.sh + i, n, sc.K, cam, st, p, info);
}

uint32_t float_bits(float f) {
  uint32_t b;
  std::memcpy(&b, &f, 4);
  return b;
}

// ----------------------------------------------------------------------------------------------
// Records used by the compositor, in the compositing precision R.
// ----------------------------------------------------------------------------------------------
// The exponent of Eq. gaussian2d, power = -1/2 d^T Sigma^-1 d, is evaluated as a sum of two
// squares, power = -((l0 du + l1 dv)^2 + (l2 dv)^2), where (l0, l1; 0, l2) is the Cholesky factor
// of Sigma^-1 / 2.  Written this way the float evaluation has no cancellation even for very
// elongated footprints (the expanded quadratic form loses ~1e-3 relative accuracy there).  The
// factor is computed from Sigma_2D in double without cancellation:
//   l0 = sqrt(S_vv / (2 det)),  l1 = -S_uv / (2 det l0),  l2 = 1 / sqrt(2 S_vv).
template <typename R>
struct Rec {
  R u, v, l0, l1, l2, o, pmin, rgb[3];
  R depth;  // the sort depth (float), for the expected-depth output
};

template <typename R>
Rec<R> make_rec(const Proj<double>& p, const Info& info) {
  Rec<R> r;
  r.u = (R)p.u;
  r.v = (R)p.v;
  const double suu = info.cov2[0], suv = info.cov2[1], svv = info.cov2[2];
  const double det = suu * svv - suv * suv;
  const double l0 = std::sqrt(svv / (2.0 * det));
  r.l0 = (R)l0;
  r.l1 = (R)(-suv / (2.0 * det * l0));
  r.l2 = (R)(1.0 / std::sqrt(2.0 * svv));
  r.o = (R)p.opacity;
  r.pmin = (R)info.p_min;
  for (int k = 0; k < 3; ++k) r.rgb[k] = (R)p.rgb[k];
  r.depth = (R)info.depth;
  return r;
}

inline float exp_r(float x) { return (float)std::exp((double)x); }
inline double exp_r(double x) { return std::exp(x); }

struct Contrib {
  int32_t idx;
  int clamped;
  double du, dv;
  double power;  // the exponent as the compositing pass evaluated it (its own precision)
};

struct PixResult {
  double rgb[3];
  double T;
  double depth;  // sum over contributors of alpha T depth (the alpha-weighted depth)
  int32_t n_contrib;
  double margin;   // min over tested steps of |T'/T_stop - 1| (termination decision margin)
  uint64_t sig;    // hash of the decision sequence (contributors, clamps, termination)
};

inline uint64_t mix(uint64_t h, uint64_t x) {
  h ^= x + 0x9e3779b97f4a7c15ULL + (h << 6) + (h >> 2);
  return h;
}

// Front-to-back alpha compositing of one pixel (Eq. gaussian2d, Eq. alphablending) over the
// candidate list `order` (ascending radial depth, ties by Gaussian index).
//   - pixel (x, y) samples the point (x + 0.5, y + 0.5);
//   - the horizontal offset is wrapped into [-W/2, W/2) so a Gaussian straddling the +-pi seam
//     is evaluated at its nearest image;
//   - 3DGS constants: alpha <= 0.99, skip alpha < 1/255 (as power < p_min), stop before the
//     Gaussian that would take the transmittance below 1e-4.
template <typename R>
PixResult composite(const int32_t* order, int64_t count, const Rec<R>* recs, int x, int y, int W, bool wrap,
                    const double* bg, std::vector<Contrib>* contrib) {
  const R px = (R)x + (R)0.5, py = (R)y + (R)0.5;
  const R Wf = (R)W, half = wrap ? (R)W * (R)0.5 : (R)INFINITY;
  const R t_stop = (R)1e-4;
  R T = (R)1.0;
  R C[3] = {(R)0, (R)0, (R)0};
  R D = (R)0;
  PixResult res;
  res.n_contrib = 0;
  res.margin = 1e30;
  res.sig = 0;
  for (int64_t k = 0; k < count; ++k) {
    const int32_t idx = order[k];
    const Rec<R>& g = recs[idx];
    R du = px - g.u;
    if (du >= half) du = du - Wf;
    else if (du < -half) du = du + Wf;
    const R dv = py - g.v;
    const R t1 = std::fma(g.l0, du, g.l1 * dv);
    const R t2 = g.l2 * dv;
    const R power = -std::fma(t1, t1, t2 * t2);
    if (power > (R)0 || power < g.pmin) continue;
    R alpha = g.o * exp_r(power);
    int clamped = 0;
    if (alpha > (R)0.99) { alpha = (R)0.99; clamped = 1; }
    const R Tn = T * ((R)1 - alpha);
    res.margin = std::min(res.margin, std::fabs((double)Tn / 1e-4 - 1.0));
    if (Tn < t_stop) { res.sig = mix(res.sig, 0xffffffffULL); break; }
    const R w = alpha * T;
    for (int c = 0; c < 3; ++c) C[c] = C[c] + w * g.rgb[c];
    D = D + w * g.depth;
    T = Tn;
    res.n_contrib++;
    res.sig = mix(res.sig, ((uint64_t)(uint32_t)idx << 1) | (uint64_t)clamped);
    if (contrib) contrib->push_back(Contrib{idx, clamped, (double)du, (double)dv, (double)power});
  }
  for (int c = 0; c < 3; ++c) res.rgb[c] = (double)C[c] + (double)T * bg[c];
  res.T = (double)T;
  res.depth = (double)D;
  return res;
}

// ----------------------------------------------------------------------------------------------
// Spherical footprint: per-pixel rays and the two record forms.
// ----------------------------------------------------------------------------------------------
// Unit direction of the ray through the centre (x + 0.5, y + 0.5) of an equirectangular pixel:
// Eq. equirec_proj inverted, then the spherical coordinates of Sec. 3.2 (azimuth from +z,
// elevation from the z-x plane, y down).  The angles are formed with this exact sequence of
// double operations (no contraction).
void pixel_dir(int x, int y, int W, int H, double d[3]) {
  const double phi = (((double)x + 0.5) - 0.5 * (double)W) * ((2.0 * M_PI) / (double)W);
  const double th = (0.5 * (double)H - ((double)y + 0.5)) * (M_PI / (double)H);
  const double cth = std::cos(th);
  d[0] = cth * std::sin(phi);
  d[1] = -std::sin(th);
  d[2] = cth * std::cos(phi);
}

// Mode 64: the definition itself.  For the line t d, with a = d^T A d, b = d^T A mu^ and
// c = mu^T A mu^, the minimum over t of the quadratic is c - b^2 / a at t = b / a; rays whose
// minimiser is not in front of the camera (b <= 0) get nothing.
struct SphRec64 {
  double mu[3], A[6], o, pmin, rgb[3], depth;
};

inline double sym3(const double* A, const double* x, const double* y) {
  return x[0] * (A[0] * y[0] + A[1] * y[1] + A[2] * y[2]) + x[1] * (A[1] * y[0] + A[3] * y[1] + A[4] * y[2]) +
         x[2] * (A[2] * y[0] + A[4] * y[1] + A[5] * y[2]);
}

inline bool sph_power(const SphRec64& g, const double d[3], double& power) {
  const double a = sym3(g.A, d, d), b = sym3(g.A, d, g.mu), c = sym3(g.A, g.mu, g.mu);
  if (!(b > 0.0)) return false;
  power = -0.5 * (c - b * b / a);
  return !(power < g.pmin);
}

// Mode 32: the float form both sides decide in.  In the tangent frame of mu^ (e1 east, e2 =
// mu^ x e1) let P, c and s33 be the blocks of Sigma~ (tangent 2x2, tangent-radial, radial).  The
// same minimum is m = 2 qh / (h^2 + k2 qh) with
//   qh = (u1 . d)^2 + (u2 . d)^2,  u1 = l0 e1 + l1 e2,  u2 = l2 e2   ((l0, l1; 0, l2): the
//        factor of P^-1 / 2 used for the affine exponent),
//   h  = w . d,  w = mu^ - (P^-1 c)_1 e1 - (P^-1 c)_2 e2,   k2 = 2 (s33 - c^T P^-1 c),
// a sum of squares with no cancellation at the scale of the footprint.  Accepted iff h > 0 and
// p_min D + qh <= 0 (D = h^2 + k2 qh, one fused multiply-add); the exponent is -qh / D.
struct SphRec32 {
  float u1[3], u2[3], w[3], k2, o, pmin, rgb[3], depth;
};

struct SphForm {
  double u1[3], u2[3], w[3], k2;
};

SphForm sph_form(const Proj<double>& p, const Info& info) {
  const double* m = p.mu_hat;
  const double rh = std::sqrt(m[0] * m[0] + m[2] * m[2]);
  const double e1[3] = {m[2] / rh, 0.0, -m[0] / rh};
  const double e2[3] = {m[1] * e1[2] - m[2] * e1[1], m[2] * e1[0] - m[0] * e1[2], m[0] * e1[1] - m[1] * e1[0]};
  const double* C = info.scov;
  const double P11 = sym3(C, e1, e1), P12 = sym3(C, e1, e2), P22 = sym3(C, e2, e2);
  const double c1 = sym3(C, e1, m), c2 = sym3(C, e2, m), s33 = sym3(C, m, m);
  const double det = P11 * P22 - P12 * P12;
  const double l0 = std::sqrt(P22 / (2.0 * det)), l1 = -P12 / (2.0 * det * l0), l2 = 1.0 / std::sqrt(2.0 * P22);
  const double a1 = -(P22 * c1 - P12 * c2) / det, a2 = -(P11 * c2 - P12 * c1) / det;  // -P^-1 c
  SphForm f;
  for (int k = 0; k < 3; ++k) {
    f.u1[k] = l0 * e1[k] + l1 * e2[k];
    f.u2[k] = l2 * e2[k];
    f.w[k] = m[k] + a1 * e1[k] + a2 * e2[k];
  }
  f.k2 = 2.0 * (s33 + (a1 * c1 + a2 * c2));
  return f;
}

// The form evaluated in double (m, not the exponent; no acceptance test).
double sph_form_m(const SphForm& f, const double d[3]) {
  const double t1 = f.u1[0] * d[0] + f.u1[1] * d[1] + f.u1[2] * d[2];
  const double t2 = f.u2[0] * d[0] + f.u2[1] * d[1] + f.u2[2] * d[2];
  const double h = f.w[0] * d[0] + f.w[1] * d[1] + f.w[2] * d[2];
  const double qh = t1 * t1 + t2 * t2;
  return 2.0 * qh / (h * h + f.k2 * qh);
}

SphRec32 make_sph_rec32(const Proj<double>& p, const Info& info) {
  const SphForm f = sph_form(p, info);
  SphRec32 r;
  for (int k = 0; k < 3; ++k) {
    r.u1[k] = (float)f.u1[k];
    r.u2[k] = (float)f.u2[k];
    r.w[k] = (float)f.w[k];
  }
  r.k2 = (float)f.k2;
  r.o = (float)p.opacity;
  r.pmin = (float)info.p_min;
  for (int k = 0; k < 3; ++k) r.rgb[k] = (float)p.rgb[k];
  r.depth = info.depth;
  return r;
}

SphRec64 make_sph_rec64(const Proj<double>& p, const Info& info) {
  SphRec64 r;
  for (int k = 0; k < 3; ++k) r.mu[k] = p.mu_hat[k];
  for (int k = 0; k < 6; ++k) r.A[k] = p.A[k];
  r.o = p.opacity;
  r.pmin = info.p_min;
  for (int k = 0; k < 3; ++k) r.rgb[k] = p.rgb[k];
  r.depth = info.depth;
  return r;
}

inline bool sph_power(const SphRec32& g, const float d[3], float& power) {
  const float t1 = std::fma(g.u1[2], d[2], std::fma(g.u1[1], d[1], g.u1[0] * d[0]));
  const float t2 = std::fma(g.u2[2], d[2], std::fma(g.u2[1], d[1], g.u2[0] * d[0]));
  const float h = std::fma(g.w[2], d[2], std::fma(g.w[1], d[1], g.w[0] * d[0]));
  const float qh = std::fma(t1, t1, t2 * t2);
  const float D = std::fma(g.k2, qh, h * h);
  if (!(h > 0.0f) || std::fma(g.pmin, D, qh) > 0.0f) return false;
  power = -(qh / D);
  return true;
}

// Front-to-back compositing of one pixel with the spherical footprint (the same 3DGS constants
// and termination as composite()).
template <typename R, typename SR>
PixResult composite_sph(const int32_t* order, int64_t count, const SR* recs, const R d[3], const double* bg,
                        std::vector<Contrib>* contrib) {
  const R t_stop = (R)1e-4;
  R T = (R)1.0;
  R C[3] = {(R)0, (R)0, (R)0};
  R Dp = (R)0;
  PixResult res;
  res.n_contrib = 0;
  res.margin = 1e30;
  res.sig = 0;
  for (int64_t k = 0; k < count; ++k) {
    const int32_t idx = order[k];
    const SR& g = recs[idx];
    R power;
    if (!sph_power(g, d, power)) continue;
    R alpha = g.o * exp_r(power);
    int clamped = 0;
    if (alpha > (R)0.99) { alpha = (R)0.99; clamped = 1; }
    const R Tn = T * ((R)1 - alpha);
    res.margin = std::min(res.margin, std::fabs((double)Tn / 1e-4 - 1.0));
    if (Tn < t_stop) { res.sig = mix(res.sig, 0xffffffffULL); break; }
    const R w = alpha * T;
    for (int c = 0; c < 3; ++c) C[c] = C[c] + w * g.rgb[c];
    Dp = Dp + w * (R)g.depth;
    T = Tn;
    res.n_contrib++;
    res.sig = mix(res.sig, ((uint64_t)(uint32_t)idx << 1) | (uint64_t)clamped);
    if (contrib) contrib->push_back(Contrib{idx, clamped, 0.0, 0.0, (double)power});
  }
  for (int c = 0; c < 3; ++c) res.rgb[c] = (double)C[c] + (double)T * bg[c];
  res.T = (double)T;
  res.depth = (double)Dp;
  return res;
}

// ----------------------------------------------------------------------------------------------
// Whole-scene preparation shared by the entry points.
// ----------------------------------------------------------------------------------------------
struct Prepared {
  std::vector<Camera> cams;
  Settings st;
  int64_t n;
  int V;
  std::vector<Proj<double>> proj;  // [V*N]
  std::vector<Info> info;          // [V*N]
  std::vector<std::vector<int32_t>> order;  // per view: kept Gaussians by (depth, index)
};

void prepare(const Scene& sc, const double* cams, const int32_t* wh, int V, const double* settings, Prepared& P) {
  P.cams = read_cameras(cams, wh, V);
  read_pinholes(settings, P.cams);
  P.st = read_settings(settings);
  P.n = sc.n;
  P.V = V;
  P.proj.resize((size_t)V * sc.n);
  P.info.resize((size_t)V * sc.n);
  P.order.assign(V, {});
  for (int v = 0; v < V; ++v) {
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < sc.n; ++i)
      project_item(sc, i, P.cams[v], P.st, P.proj[(size_t)v * sc.n + i], P.info[(size_t)v * sc.n + i]);
    std::vector<int32_t>& ord = P.order[v];
    for (int64_t i = 0; i < sc.n; ++i)
      if (P.info[(size_t)v * sc.n + i].cull == KEPT) ord.push_back((int32_t)i);
    const Info* inf = &P.info[(size_t)v * sc.n];
    // Sort by depth (Eq. alphablending is accumulated in depth order); equal depths keep the
    // Gaussian index order.
    std::stable_sort(ord.begin(), ord.end(), [inf](int32_t a, int32_t b) { return inf[a].depth < inf[b].depth; });
  }
}

Scene make_scene(const double* means, const double* scales, const double* quats, const double* opac,
                 const double* sh, int64_t n, int deg) {
  Scene sc;
  sc.means = means;
  sc.scales = scales;
  sc.quats = quats;
  sc.opac = opac;
  sc.sh = sh;
  sc.n = n;
  sc.K = (deg + 1) * (deg + 1);
  return sc;
}

// Key list of one view, in emission order: Gaussians ascending, tiles ascending.
// key = (global tile id << 32) | float bits of the radial depth; value = Gaussian index.
void view_pairs(const Prepared& P, int v, int64_t tile_base, std::vector<uint64_t>& keys, std::vector<uint32_t>& vals) {
  const Camera& cam = P.cams[v];
  const int B = P.st.tile, ntx = cam.W / B;
  for (int64_t i = 0; i < P.n; ++i) {
    const Info& inf = P.info[(size_t)v * P.n + i];
    if (inf.cull != KEPT) continue;
    std::vector<int> cols;
    for (int c = 0; c < inf.ncols; ++c) cols.push_back((inf.col0 + c) % ntx);
    std::sort(cols.begin(), cols.end());
    for (int r = 0; r < inf.nrows; ++r)
      for (int c : cols) {
        uint64_t tile = (uint64_t)(tile_base + (int64_t)(inf.row0 + r) * ntx + c);
        keys.push_back((tile << 32) | float_bits(inf.depth));
        vals.push_back((uint32_t)i);
      }
  }
}

void sorted_pairs(const Prepared& P, std::vector<uint64_t>& keys, std::vector<uint32_t>& vals) {
  int64_t base = 0;
  for (int v = 0; v < P.V; ++v) {
    view_pairs(P, v, base, keys, vals);
    base += (int64_t)(P.cams[v].W / P.st.tile) * (P.cams[v].H / P.st.tile);
  }
  std::vector<int64_t> perm(keys.size());
  for (size_t k = 0; k < perm.size(); ++k) perm[k] = (int64_t)k;
  std::stable_sort(perm.begin(), perm.end(), [&](int64_t a, int64_t b) {
    if (keys[a] != keys[b]) return keys[a] < keys[b];
    return vals[a] < vals[b];
  });
  std::vector<uint64_t> k2(keys.size());
  std::vector<uint32_t> v2(vals.size());
  for (size_t k = 0; k < perm.size(); ++k) {
    k2[k] = keys[perm[k]];
    v2[k] = vals[perm[k]];
  }
  keys.swap(k2);
  vals.swap(v2);
}

int64_t pix_offset(const Prepared& P, int v) {
  int64_t off = 0;
  for (int u = 0; u < v; ++u) off += (int64_t)P.cams[u].W * P.cams[u].H;
  return off;
}

// Candidate list of a pixel: brute force = every kept Gaussian of the view.  Band mode = the
// entries of the pixel's tile in the sorted key list (must give identical images).
struct Candidates {
  std::vector<std::vector<int32_t>> band;  // per global tile
  std::vector<int64_t> tile_base;
};

void build_band(const Prepared& P, Candidates& cand) {
  std::vector<uint64_t> keys;
  std::vector<uint32_t> vals;
  sorted_pairs(P, keys, vals);
  int64_t total = 0;
  cand.tile_base.assign(P.V, 0);
  for (int v = 0; v < P.V; ++v) {
    cand.tile_base[v] = total;
    total += (int64_t)(P.cams[v].W / P.st.tile) * (P.cams[v].H / P.st.tile);
  }
  cand.band.assign((size_t)total, {});
  for (size_t k = 0; k < keys.size(); ++k) cand.band[keys[k] >> 32].push_back((int32_t)vals[k]);
}

template <typename R>
std::vector<Rec<R>> make_recs(const Prepared& P, int v) {
  std::vector<Rec<R>> recs((size_t)P.n);
  for (int64_t i = 0; i < P.n; ++i) {
    const size_t it = (size_t)v * P.n + i;
    if (P.info[it].cull == KEPT) recs[i] = make_rec<R>(P.proj[it], P.info[it]);
  }
  return recs;
}

template <typename R>
PixResult render_pixel(const Prepared& P, const std::vector<Rec<R>>& recs, const Candidates* cand, int v, int x, int y,
                       std::vector<Contrib>* contrib) {
  const Camera& cam = P.cams[v];
  if (cand) {
    const int B = P.st.tile;
    const int64_t tile = cand->tile_base[v] + (int64_t)(y / B) * (cam.W / B) + x / B;
    const std::vector<int32_t>& lst = cand->band[tile];
    return composite<R>(lst.data(), (int64_t)lst.size(), recs.data(), x, y, cam.W, !cam.pinhole, P.st.bg, contrib);
  }
  const std::vector<int32_t>& ord = P.order[v];
  return composite<R>(ord.data(), (int64_t)ord.size(), recs.data(), x, y, cam.W, !cam.pinhole, P.st.bg, contrib);
}

inline bool sph_view(const Prepared& P, int v) { return P.st.spherical && !P.cams[v].pinhole; }

template <typename SR>
std::vector<SR> make_sph_recs(const Prepared& P, int v, SR (*make)(const Proj<double>&, const Info&)) {
  std::vector<SR> recs((size_t)P.n);
  for (int64_t i = 0; i < P.n; ++i) {
    const size_t it = (size_t)v * P.n + i;
    if (P.info[it].cull == KEPT) recs[i] = make(P.proj[it], P.info[it]);
  }
  return recs;
}

template <typename R, typename SR>
PixResult render_pixel_sph(const Prepared& P, const std::vector<SR>& recs, const Candidates* cand, int v, int x, int y,
                           std::vector<Contrib>* contrib) {
  const Camera& cam = P.cams[v];
  double dd[3];
  pixel_dir(x, y, cam.W, cam.H, dd);
  const R d[3] = {(R)dd[0], (R)dd[1], (R)dd[2]};
  if (cand) {
    const int B = P.st.tile;
    const int64_t tile = cand->tile_base[v] + (int64_t)(y / B) * (cam.W / B) + x / B;
    const std::vector<int32_t>& lst = cand->band[tile];
    return composite_sph<R, SR>(lst.data(), (int64_t)lst.size(), recs.data(), d, P.st.bg, contrib);
  }
  const std::vector<int32_t>& ord = P.order[v];
  return composite_sph<R, SR>(ord.data(), (int64_t)ord.size(), recs.data(), d, P.st.bg, contrib);
}

// Reverse recursion over one pixel's contributors (Eq. alphablending differentiated):
//   C_c = sum_j rgb_jc a_j T_j + T_final bg_c,  T_j = prod_{k<j} (1 - a_k)
//   dC_c/d rgb_jc = a_j T_j
//   dC_c/d a_j   = rgb_jc T_j - (sum_{k>j} rgb_kc a_k T_k + T_final bg_c) / (1 - a_j)
// then through a = min(0.99, o G), G = exp(power),
//   power = -1/2 (a du^2 + 2 b du dv + c dv^2),  du = x + 0.5 - u (wrapped), dv = y + 0.5 - v,
// with d power / d(a, b, c) = -(du^2/2, du dv, dv^2/2) and d power / d(u, v) = Sigma^-1 d.
// g2d layout per item: [u, v, conic a, conic b, conic c, opacity, r, g, b].
void pixel_backward(const std::vector<Contrib>& cl, const std::vector<Rec<double>>& rec64, const double* gpix,
                    const double* bg, double* g2d_view, int stride, bool decided_power) {
  const size_t n = cl.size();
  std::vector<double> alpha(n), T(n + 1), G(n);
  T[0] = 1.0;
  for (size_t j = 0; j < n; ++j) {
    const Rec<double>& g = rec64[cl[j].idx];
    const double du = cl[j].du, dv = cl[j].dv;
    const double t1 = g.l0 * du + g.l1 * dv, t2 = g.l2 * dv;
    const double power = decided_power ? cl[j].power : -(t1 * t1 + t2 * t2);
    G[j] = std::exp(power);
    alpha[j] = cl[j].clamped ? 0.99 : g.o * G[j];
    T[j + 1] = T[j] * (1.0 - alpha[j]);
  }
  double S[3];
  for (int c = 0; c < 3; ++c) S[c] = T[n] * bg[c];
  for (size_t jj = n; jj-- > 0;) {
    const Rec<double>& g = rec64[cl[jj].idx];
    double* out = g2d_view + (size_t)cl[jj].idx * stride;
    double dL_da = 0.0;
    for (int c = 0; c < 3; ++c) {
      const double grgb = gpix[c] * alpha[jj] * T[jj];
#pragma omp atomic
      out[6 + c] += grgb;
      dL_da += gpix[c] * (g.rgb[c] * T[jj] - S[c] / (1.0 - alpha[jj]));
      S[c] += g.rgb[c] * alpha[jj] * T[jj];
    }
    if (cl[jj].clamped) continue;
    const double du = cl[jj].du, dv = cl[jj].dv;
    const double t1 = g.l0 * du + g.l1 * dv, t2 = g.l2 * dv;
    const double dL_dpow = dL_da * alpha[jj];
    // d power / d u = (Sigma^-1 d)_u = 2 l0 t1,  d power / d v = 2 (l1 t1 + l2 t2)
    const double gu = dL_dpow * (2.0 * g.l0 * t1);
    const double gv = dL_dpow * (2.0 * (g.l1 * t1 + g.l2 * t2));
    const double ga = dL_dpow * (-0.5 * du * du);
    const double gb = dL_dpow * (-du * dv);
    const double gc = dL_dpow * (-0.5 * dv * dv);
    const double go = dL_da * G[jj];
#pragma omp atomic
    out[0] += gu;
#pragma omp atomic
    out[1] += gv;
#pragma omp atomic
    out[2] += ga;
#pragma omp atomic
    out[3] += gb;
#pragma omp atomic
    out[4] += gc;
#pragma omp atomic
    out[5] += go;
  }
}

// Reverse recursion for the spherical footprint (same alpha / T recursion as pixel_backward).
// Per contributor the exponent is power = -m / 2 with m the minimum over t of the quadratic along
// the ray; by the envelope theorem its derivatives are those of the quadratic at the fixed
// minimiser t* = b / a: with v = t* d - mu^, dm/dA = v v^T and dm/dmu^ = -2 A v.
//   g_def [stride]: mu^ (3), A (6, off-diagonals as one shared variable), opacity, r, g, b.
//   g_ker [13] (optional): the kernel's layout, mu^ (3), Sigma~ (6, shared), opacity, rgb, from
//     dm/dSigma~ = -A (dm/dA) A = -z z^T with z = A v.
void pixel_backward_sph(const std::vector<Contrib>& cl, const std::vector<SphRec64>& rec, const double d[3], bool decided_power,
                        const double* gpix, const double* bg, double* g_def, int stride, double* g_ker) {
  const size_t n = cl.size();
  std::vector<double> alpha(n), T(n + 1), G(n), pw(n);
  T[0] = 1.0;
  for (size_t j = 0; j < n; ++j) {
    const SphRec64& g = rec[cl[j].idx];
    double p = 0.0;
    sph_power(g, d, p);
    if (decided_power) p = cl[j].power;
    pw[j] = p;
    G[j] = std::exp(p);
    alpha[j] = cl[j].clamped ? 0.99 : g.o * G[j];
    T[j + 1] = T[j] * (1.0 - alpha[j]);
  }
  double S[3];
  for (int c = 0; c < 3; ++c) S[c] = T[n] * bg[c];
  for (size_t jj = n; jj-- > 0;) {
    const SphRec64& g = rec[cl[jj].idx];
    double out[13] = {0};
    double ker[13] = {0};
    double dL_da = 0.0;
    for (int c = 0; c < 3; ++c) {
      out[10 + c] = gpix[c] * alpha[jj] * T[jj];
      dL_da += gpix[c] * (g.rgb[c] * T[jj] - S[c] / (1.0 - alpha[jj]));
      S[c] += g.rgb[c] * alpha[jj] * T[jj];
    }
    if (!cl[jj].clamped) {
      const double dL_dpow = dL_da * alpha[jj];
      const double a = sym3(g.A, d, d), b = sym3(g.A, d, g.mu);
      const double t = b / a;
      const double v[3] = {t * d[0] - g.mu[0], t * d[1] - g.mu[1], t * d[2] - g.mu[2]};
      const double Av[3] = {g.A[0] * v[0] + g.A[1] * v[1] + g.A[2] * v[2], g.A[1] * v[0] + g.A[3] * v[1] + g.A[4] * v[2],
                            g.A[2] * v[0] + g.A[4] * v[1] + g.A[5] * v[2]};
      // dL/dm = -dL_dpow / 2
      for (int k = 0; k < 3; ++k) out[k] = dL_dpow * Av[k];
      out[3] = -0.5 * dL_dpow * v[0] * v[0];
      out[4] = -dL_dpow * v[0] * v[1];
      out[5] = -dL_dpow * v[0] * v[2];
      out[6] = -0.5 * dL_dpow * v[1] * v[1];
      out[7] = -dL_dpow * v[1] * v[2];
      out[8] = -0.5 * dL_dpow * v[2] * v[2];
      out[9] = dL_da * G[jj];
      // power = -m / 2:  dpower/dmu^ = A v = z,  dpower/dSigma~ = z z^T / 2
      for (int k = 0; k < 3; ++k) ker[k] = out[k];
      ker[3] = 0.5 * dL_dpow * Av[0] * Av[0];
      ker[4] = dL_dpow * Av[0] * Av[1];
      ker[5] = dL_dpow * Av[0] * Av[2];
      ker[6] = 0.5 * dL_dpow * Av[1] * Av[1];
      ker[7] = dL_dpow * Av[1] * Av[2];
      ker[8] = 0.5 * dL_dpow * Av[2] * Av[2];
      ker[9] = out[9];
    }
    for (int c = 0; c < 3; ++c) ker[10 + c] = out[10 + c];
    double* o1 = g_def + (size_t)cl[jj].idx * stride;
    for (int k = 0; k < 13; ++k) {
      if (out[k] == 0.0) continue;
#pragma omp atomic
      o1[k] += out[k];
    }
    if (g_ker) {
      double* o2 = g_ker + (size_t)cl[jj].idx * 13;
      for (int k = 0; k < 13; ++k) {
        if (ker[k] == 0.0) continue;
#pragma omp atomic
        o2[k] += ker[k];
      }
    }
  }
}

// Adjoint of the per-(Gaussian, view) projection, summed over views.  acc [V][N][stride] holds
// per-item gradients of the compositor's inputs.  Affine items: (u, v, three 2D-shape entries,
// opacity, r, g, b), the shape entries with respect to the inverse covariance (a, b, c) or, with
// `sigma`, the covariance (uu, uv, vv; the off-diagonal as one shared variable).  Spherical
// items: (mu^, A, opacity, rgb) as pixel_backward_sph's g_def or, with `sigma`, its kernel
// layout (mu^, Sigma~, opacity, rgb).
void project_adjoint(const Scene& sc, const Prepared& P, const std::vector<double>& acc, int stride, bool sigma,
                     double* d_means, double* d_scales, double* d_quats, double* d_opac, double* d_sh) {
  // Per-Gaussian chain rule: push the 2D gradients through the projection with dual numbers
  // (directions: mean xyz, scale xyz, quaternion wxyz, opacity), and the colour gradient
  // through the SH basis; sum over views.
  const int K = sc.K;
  const int64_t n = sc.n;
  const int V = (int)P.cams.size();
#pragma omp parallel for schedule(dynamic, 64)
  for (int64_t i = 0; i < n; ++i) {
    double gm[3] = {0, 0, 0}, gs[3] = {0, 0, 0}, gq[4] = {0, 0, 0, 0}, go = 0.0;
    std::vector<double> gsh((size_t)K * 3, 0.0);
    for (int v = 0; v < V; ++v) {
      const size_t it = (size_t)v * n + i;
      const double* g = acc.data() + it * stride;
      const bool sph = P.info[it].spherical;
      const int nv = sph ? 13 : 9;
      bool any = false;
      for (int k = 0; k < nv; ++k) any = any || g[k] != 0.0;
      if (!any || P.info[it].cull != KEPT) continue;
      Dual m[3], s[3], q[4], o;
      for (int k = 0; k < 3; ++k) { m[k] = Dual(sc.means[k * n + i]); m[k].d[k] = 1.0; }
      for (int k = 0; k < 3; ++k) { s[k] = Dual(sc.scales[k * n + i]); s[k].d[3 + k] = 1.0; }
      for (int k = 0; k < 4; ++k) { q[k] = Dual(sc.quats[k * n + i]); q[k].d[6 + k] = 1.0; }
      o = Dual(sc.opac[i]);
      o.d[10] = 1.0;
      Proj<Dual> p;
      Info inf;
      project<Dual>(m, s, q, o, sc.sh + i, n, K, P.cams[v], P.st, p, inf);
      const Dual* outs[14];
      if (!sph) {
        const Dual* o9[9] = {&p.u, &p.v, sigma ? &p.cov2[0] : &p.conic[0], sigma ? &p.cov2[1] : &p.conic[1],
                             sigma ? &p.cov2[2] : &p.conic[2], &p.opacity, &p.rgb[0], &p.rgb[1], &p.rgb[2]};
        std::copy(o9, o9 + 9, outs);
      } else {
        for (int k = 0; k < 3; ++k) outs[k] = &p.mu_hat[k];
        for (int k = 0; k < 6; ++k) outs[3 + k] = sigma ? &p.C[k] : &p.A[k];
      }
      if (sph) {
        outs[nv - 4] = &p.opacity;
        for (int k = 0; k < 3; ++k) outs[nv - 3 + k] = &p.rgb[k];
      }
      double gd[ND] = {0};
      for (int k = 0; k < nv; ++k)
        for (int d = 0; d < ND; ++d) gd[d] += g[k] * outs[k]->d[d];
      for (int k = 0; k < 3; ++k) gm[k] += gd[k];
      for (int k = 0; k < 3; ++k) gs[k] += gd[3 + k];
      for (int k = 0; k < 4; ++k) gq[k] += gd[6 + k];
      go += gd[10];
      // colour = sum_k sh_k Y_k(dir) + 0.5 (clamped): d colour / d sh_k = Y_k where unclamped
      double cc[3];
      const Camera& cam = P.cams[v];
      for (int k = 0; k < 3; ++k)
        cc[k] = -((cam.R[0 * 3 + k] * cam.t[0] + cam.R[1 * 3 + k] * cam.t[1]) + cam.R[2 * 3 + k] * cam.t[2]);
      double dv[3] = {sc.means[i] - cc[0], sc.means[n + i] - cc[1], sc.means[2 * n + i] - cc[2]};
      const double dn = std::sqrt((dv[0] * dv[0] + dv[1] * dv[1]) + dv[2] * dv[2]);
      double dir[3] = {dv[0] / dn, dv[1] / dn, dv[2] / dn};
      double Y[16];
      sh_basis<double>(dir, K, Y);
      for (int ch = 0; ch < 3; ++ch) {
        if (inf.rgb_clamped[ch]) continue;
        for (int k = 0; k < K; ++k) gsh[(size_t)k * 3 + ch] += g[nv - 3 + ch] * Y[k];
      }
    }
    for (int k = 0; k < 3; ++k) d_means[k * n + i] = gm[k];
    for (int k = 0; k < 3; ++k) d_scales[k * n + i] = gs[k];
    for (int k = 0; k < 4; ++k) d_quats[k * n + i] = gq[k];
    d_opac[i] = go;
    for (int k = 0; k < K * 3; ++k) d_sh[(int64_t)k * n + i] = gsh[k];
  }
}

}  // namespace

// ==============================================================================================
// C entry points (called through ctypes by the tests; see oracle/oracle.py for array layouts)
// ==============================================================================================
extern "C" {

int oracle_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

// Real SH basis values Y[n][K] for unit directions dirs[n][3].
void oracle_sh_basis(const double* dirs, int64_t n, int K, double* Y) {
  for (int64_t i = 0; i < n; ++i) {
    double d[3] = {dirs[3 * i], dirs[3 * i + 1], dirs[3 * i + 2]};
    double y[16];
    sh_basis<double>(d, K, y);
    for (int k = 0; k < K; ++k) Y[i * K + k] = y[k];
  }
}

// Spherical footprint at single (view, x, y, gaussian) queries q [nq][4], for the pins: out [nq][6]
// = (m by the definition c - b^2/a, b = d^T A mu^, m by the tangent-frame form in double, the
// float exponent (0 where rejected), float acceptance, kept).  Every listed view must be
// equirectangular and the settings must select the spherical footprint.
int oracle_sph_eval(const double* means, const double* scales, const double* quats, const double* opac,
                    const double* sh, int64_t n, int deg, const double* cams, const int32_t* wh, int V,
                    const double* settings, const int32_t* q, int64_t nq, double* out) {
  Scene sc = make_scene(means, scales, quats, opac, sh, n, deg);
  Prepared P;
  prepare(sc, cams, wh, V, settings, P);
  for (int64_t k = 0; k < nq; ++k) {
    const int v = q[4 * k], x = q[4 * k + 1], y = q[4 * k + 2], i = q[4 * k + 3];
    double* o = out + 6 * k;
    std::fill(o, o + 6, 0.0);
    const size_t it = (size_t)v * n + i;
    if (!sph_view(P, v) || P.info[it].cull != KEPT) continue;
    o[5] = 1.0;
    double d[3];
    pixel_dir(x, y, P.cams[v].W, P.cams[v].H, d);
    const SphRec64 r = make_sph_rec64(P.proj[it], P.info[it]);
    const double a = sym3(r.A, d, d), b = sym3(r.A, d, r.mu), c = sym3(r.A, r.mu, r.mu);
    o[0] = c - b * b / a;
    o[1] = b;
    o[2] = sph_form_m(sph_form(P.proj[it], P.info[it]), d);
    const SphRec32 r32 = make_sph_rec32(P.proj[it], P.info[it]);
    const float d32[3] = {(float)d[0], (float)d[1], (float)d[2]};
    float pw = 0.0f;
    const bool ok = sph_power(r32, d32, pw);
    o[3] = ok ? pw : 0.0;
    o[4] = ok;
  }
  return 0;
}

// Per-(view, Gaussian) projection rows of ORACLE_NF doubles, layout [V][N][41]:
//  0 kept  1 cull  2 depth  3 depth bits  4 u  5 v  6..8 conic a,b,c  9 opacity  10 p_min
//  11..13 rgb  14..17 col0 ncols row0 nrows  18..20 cov2 uu uv vv  21..26 J_omni  27..32 cov3
//  33..35 mu  36 r  37..39 rgb before clamp  40 cone half-angle (spherical footprint)
int oracle_project(const double* means, const double* scales, const double* quats, const double* opac,
                   const double* sh, int64_t n, int deg, const double* cams, const int32_t* wh, int V,
                   const double* settings, double* out) {
  Scene sc = make_scene(means, scales, quats, opac, sh, n, deg);
  Prepared P;
  prepare(sc, cams, wh, V, settings, P);
  for (int v = 0; v < V; ++v)
    for (int64_t i = 0; i < n; ++i) {
      const size_t it = (size_t)v * n + i;
      const Proj<double>& p = P.proj[it];
      const Info& f = P.info[it];
      double* o = out + it * 41;
      std::fill(o, o + 41, 0.0);
      o[0] = f.cull == KEPT;
      o[1] = f.cull;
      o[2] = f.depth;
      o[3] = float_bits(f.depth);
      o[33] = f.mu[0]; o[34] = f.mu[1]; o[35] = f.mu[2]; o[36] = f.r;
      if (f.cull == CULL_SHELL || f.cull == CULL_POLE || f.cull == CULL_FRUSTUM) continue;
      o[4] = p.u; o[5] = p.v;
      for (int k = 0; k < 3; ++k) o[6 + k] = p.conic[k];
      o[9] = p.opacity;
      o[10] = f.p_min;
      for (int k = 0; k < 3; ++k) o[11 + k] = p.rgb[k];
      o[14] = f.col0; o[15] = f.ncols; o[16] = f.row0; o[17] = f.nrows;
      for (int k = 0; k < 3; ++k) o[18 + k] = f.cov2[k];
      for (int k = 0; k < 6; ++k) o[21 + k] = f.J[k];
      for (int k = 0; k < 6; ++k) o[27 + k] = f.cov3[k];
      for (int k = 0; k < 3; ++k) o[37 + k] = f.rgb_raw[k];
      o[40] = f.beta;
    }
  return 0;
}

// Sorted key list over all views.  Returns the pair count P; fills keys/vals if P <= cap.
int64_t oracle_keys(const double* means, const double* scales, const double* quats, const double* opac,
                    const double* sh, int64_t n, int deg, const double* cams, const int32_t* wh, int V,
                    const double* settings, uint64_t* keys, uint32_t* vals, int64_t cap) {
  Scene sc = make_scene(means, scales, quats, opac, sh, n, deg);
  Prepared P;
  prepare(sc, cams, wh, V, settings, P);
  std::vector<uint64_t> k;
  std::vector<uint32_t> v;
  sorted_pairs(P, k, v);
  const int64_t total = (int64_t)k.size();
  if (total <= cap) {
    std::memcpy(keys, k.data(), k.size() * sizeof(uint64_t));
    std::memcpy(vals, v.data(), v.size() * sizeof(uint32_t));
  }
  return total;
}

// Render.  mode 32 or 64 (compositing precision), band 0 = brute force, 1 = tile lists.
// pix == NULL: every pixel of every view; rgb [V][3][H][W], T/ncontrib/margin/sig [V][H][W].
// pix != NULL: npix rows of (view, x, y); rgb [npix][3], the rest [npix].
int oracle_render(const double* means, const double* scales, const double* quats, const double* opac,
                  const double* sh, int64_t n, int deg, const double* cams, const int32_t* wh, int V,
                  const double* settings, int mode, int band, const int32_t* pix, int64_t npix, double* rgb,
                  double* T, int32_t* ncontrib, double* margin, uint64_t* sig, double* depth) {
  Scene sc = make_scene(means, scales, quats, opac, sh, n, deg);
  Prepared P;
  prepare(sc, cams, wh, V, settings, P);
  Candidates cand;
  if (band) build_band(P, cand);
  const Candidates* cp = band ? &cand : nullptr;
  std::vector<std::vector<Rec<float>>> r32(V);
  std::vector<std::vector<Rec<double>>> r64(V);
  std::vector<std::vector<SphRec32>> s32(V);
  std::vector<std::vector<SphRec64>> s64(V);
  for (int v = 0; v < V; ++v) {
    if (sph_view(P, v)) {
      if (mode == 32) s32[v] = make_sph_recs<SphRec32>(P, v, make_sph_rec32);
      else s64[v] = make_sph_recs<SphRec64>(P, v, make_sph_rec64);
    } else if (mode == 32) {
      r32[v] = make_recs<float>(P, v);
    } else {
      r64[v] = make_recs<double>(P, v);
    }
  }
  auto one = [&](int v, int x, int y) {
    if (sph_view(P, v))
      return mode == 32 ? render_pixel_sph<float, SphRec32>(P, s32[v], cp, v, x, y, nullptr)
                        : render_pixel_sph<double, SphRec64>(P, s64[v], cp, v, x, y, nullptr);
    return mode == 32 ? render_pixel<float>(P, r32[v], cp, v, x, y, nullptr)
                      : render_pixel<double>(P, r64[v], cp, v, x, y, nullptr);
  };
  if (pix == nullptr) {
    for (int v = 0; v < V; ++v) {
      const int W = P.cams[v].W, H = P.cams[v].H;
      const int64_t off = pix_offset(P, v);
#pragma omp parallel for schedule(dynamic, 4)
      for (int y = 0; y < H; ++y)
        for (int x = 0; x < W; ++x) {
          PixResult r = one(v, x, y);
          const int64_t p = off + (int64_t)y * W + x;
          for (int c = 0; c < 3; ++c) rgb[3 * off + (int64_t)c * W * H + (int64_t)y * W + x] = r.rgb[c];
          T[p] = r.T;
          ncontrib[p] = r.n_contrib;
          margin[p] = r.margin;
          sig[p] = r.sig;
          if (depth) depth[p] = r.depth;
        }
    }
  } else {
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t k = 0; k < npix; ++k) {
      PixResult r = one(pix[3 * k], pix[3 * k + 1], pix[3 * k + 2]);
      for (int c = 0; c < 3; ++c) rgb[3 * k + c] = r.rgb[c];
      T[k] = r.T;
      ncontrib[k] = r.n_contrib;
      margin[k] = r.margin;
      sig[k] = r.sig;
      if (depth) depth[k] = r.depth;
    }
  }
  return 0;
}

// Gradient of L = sum_pixels dL/dC . C (double).  Contributor lists come from the mode-32 or
// mode-64 forward; all gradient arithmetic is double.  dL: with pix == NULL the full
// [V][3][H][W] image gradient, else [npix][3] for the listed pixels only (others are zero).
// Outputs (overwritten): d_means [3][N], d_scales [3][N], d_quats [4][N], d_opac [N],
// d_sh [K*3][N]; g2d (optional, NULL to skip) [V][N][G] per-item gradients of the compositor's
// inputs, G = 9 (affine) or 13 (spherical footprint: mu^, A, opacity, rgb); g2d_kernel
// (optional, spherical footprint only) [V][N][13] the same in the kernel's variables (mu^,
// Sigma~, opacity, rgb).
// mode 33: the mode-32 contributor lists, and each contributor's alpha from the exponent exactly as
// that float pass evaluated it (everything else double): the same derivative taken at the float
// exponents, whose distance from mode 32's gradient measures how far float evaluation of the
// exponent alone moves each gradient element.
int oracle_backward(const double* means, const double* scales, const double* quats, const double* opac,
                    const double* sh, int64_t n, int deg, const double* cams, const int32_t* wh, int V,
                    const double* settings, int mode, const int32_t* pix, int64_t npix, const double* dL,
                    double* d_means, double* d_scales, double* d_quats, double* d_opac, double* d_sh, double* g2d,
                    double* g2d_kernel, int band) {
  const bool decided = mode == 33;
  if (decided) mode = 32;
  Scene sc = make_scene(means, scales, quats, opac, sh, n, deg);
  Prepared P;
  prepare(sc, cams, wh, V, settings, P);
  // band = 1: each pixel's candidates are its tile's key list instead of every kept Gaussian
  // (identical contributor lists by construction, far less work)
  Candidates cand;
  if (band) build_band(P, cand);
  const Candidates* cp = band ? &cand : nullptr;
  const int stride = P.st.spherical ? 13 : 9;
  std::vector<double> acc((size_t)V * n * stride, 0.0);
  std::vector<double> acck(P.st.spherical && g2d_kernel ? (size_t)V * n * 13 : 0, 0.0);
  for (int v = 0; v < V; ++v) {
    if (sph_view(P, v)) {
      std::vector<SphRec32> s32;
      std::vector<SphRec64> s64 = make_sph_recs<SphRec64>(P, v, make_sph_rec64);
      if (mode == 32) s32 = make_sph_recs<SphRec32>(P, v, make_sph_rec32);
      double* gv = acc.data() + (size_t)v * n * stride;
      double* gk = acck.empty() ? nullptr : acck.data() + (size_t)v * n * 13;
      const int W = P.cams[v].W, H = P.cams[v].H;
      auto run = [&](int x, int y, const double* gpix) {
        if (gpix[0] == 0.0 && gpix[1] == 0.0 && gpix[2] == 0.0) return;
        std::vector<Contrib> cl;
        if (mode == 32) render_pixel_sph<float, SphRec32>(P, s32, cp, v, x, y, &cl);
        else render_pixel_sph<double, SphRec64>(P, s64, cp, v, x, y, &cl);
        double d[3];
        pixel_dir(x, y, W, H, d);
        pixel_backward_sph(cl, s64, d, decided, gpix, P.st.bg, gv, stride, gk);
      };
      if (pix == nullptr) {
        const int64_t off = pix_offset(P, v);
#pragma omp parallel for schedule(dynamic, 4)
        for (int y = 0; y < H; ++y)
          for (int x = 0; x < W; ++x) {
            double g[3];
            for (int c = 0; c < 3; ++c) g[c] = dL[3 * off + (int64_t)c * W * H + (int64_t)y * W + x];
            run(x, y, g);
          }
      } else {
#pragma omp parallel for schedule(dynamic, 1)
        for (int64_t k = 0; k < npix; ++k)
          if (pix[3 * k] == v) run(pix[3 * k + 1], pix[3 * k + 2], dL + 3 * k);
      }
      continue;
    }
    std::vector<Rec<float>> r32;
    std::vector<Rec<double>> r64 = make_recs<double>(P, v);
    std::vector<Rec<double>> rvals;  // values used in the gradient arithmetic
    if (mode == 32) {
      r32 = make_recs<float>(P, v);
      rvals.resize(r32.size());
      for (size_t i = 0; i < r32.size(); ++i) {
        rvals[i].u = r32[i].u; rvals[i].v = r32[i].v; rvals[i].l0 = r32[i].l0; rvals[i].l1 = r32[i].l1;
        rvals[i].l2 = r32[i].l2; rvals[i].o = r32[i].o; rvals[i].pmin = r32[i].pmin;
        for (int c = 0; c < 3; ++c) rvals[i].rgb[c] = r32[i].rgb[c];
      }
    } else {
      rvals = r64;
    }
    double* gv = acc.data() + (size_t)v * n * stride;
    const int W = P.cams[v].W, H = P.cams[v].H;
    auto run = [&](int x, int y, const double* gpix) {
      if (gpix[0] == 0.0 && gpix[1] == 0.0 && gpix[2] == 0.0) return;
      std::vector<Contrib> cl;
      if (mode == 32) render_pixel<float>(P, r32, cp, v, x, y, &cl);
      else render_pixel<double>(P, r64, cp, v, x, y, &cl);
      pixel_backward(cl, rvals, gpix, P.st.bg, gv, stride, decided);
    };
    if (pix == nullptr) {
      const int64_t off = pix_offset(P, v);
#pragma omp parallel for schedule(dynamic, 4)
      for (int y = 0; y < H; ++y)
        for (int x = 0; x < W; ++x) {
          double g[3];
          for (int c = 0; c < 3; ++c) g[c] = dL[3 * off + (int64_t)c * W * H + (int64_t)y * W + x];
          run(x, y, g);
        }
    } else {
#pragma omp parallel for schedule(dynamic, 1)
      for (int64_t k = 0; k < npix; ++k)
        if (pix[3 * k] == v) run(pix[3 * k + 1], pix[3 * k + 2], dL + 3 * k);
    }
  }
  if (g2d) std::memcpy(g2d, acc.data(), acc.size() * sizeof(double));
  if (g2d_kernel && !acck.empty()) std::memcpy(g2d_kernel, acck.data(), acck.size() * sizeof(double));

  project_adjoint(sc, P, acc, stride, false, d_means, d_scales, d_quats, d_opac, d_sh);
  return 0;
}

// Adjoint of the projection alone, for per-item gradients in the layout the GPU's reverse
// compositor produces: g2d [V][N][9] = (u, v, Sigma_uu, Sigma_uv (shared), Sigma_vv, opacity,
// r, g, b), or with the spherical footprint [V][N][13] = (mu^ (3), Sigma~ (6, shared
// off-diagonals), opacity, r, g, b).  Outputs as oracle_backward (overwritten).
int oracle_project_adjoint(const double* means, const double* scales, const double* quats, const double* opac,
                           const double* sh, int64_t n, int deg, const double* cams, const int32_t* wh, int V,
                           const double* settings, const double* g2d, double* d_means, double* d_scales,
                           double* d_quats, double* d_opac, double* d_sh) {
  Scene sc = make_scene(means, scales, quats, opac, sh, n, deg);
  Prepared P;
  prepare(sc, cams, wh, V, settings, P);
  const int stride = P.st.spherical ? 13 : 9;
  std::vector<double> acc(g2d, g2d + (size_t)V * n * stride);
  project_adjoint(sc, P, acc, stride, true, d_means, d_scales, d_quats, d_opac, d_sh);
  return 0;
}

}  // extern "C"
