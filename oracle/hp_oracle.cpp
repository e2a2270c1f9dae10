// hp_oracle.cpp -- plain FP64 CPU reference of the HEALPix Gaussian rasterizer.
//
// TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
// call this file; only the test-suite, the smoke check and the CPU-baseline
// leg of the benchmark use it.  It shares no code, header or table with the
// HIP implementation.
//
// Everything is computed in double precision from the float32 inputs, by
// brute force, in the order the paper states the method:
//   * HEALPix geometry from the definitions of Gorski et al. (2005), the grid
//     the paper adopts in Sec. 3.1 (Npix = 12 Nside^2, NESTED (x, y, f)).
//   * Forward projection Pi (Eq. lonlat_projection), 3D covariance
//     R diag(s^2) R^T and radian covariance J W Sigma W^T J^T (Alg. 1,
//     preprocessing), latitude scaling S_phi = diag(cos phi, 1)
//     (Eq. arc_scaling), conic = Sigma_arc^-1, r_s = 3 sqrt(lambda_max).
//   * Spherical offset: haversine great-circle distance decomposed with the
//     bearing angle (Sec. 3.4), blending weight o exp(-d^T Sigma^-1 d / 2),
//     and front-to-back compositing over radially sorted Gaussians
//     (Eq. unified_rendering, Alg. 1 rendering loop).
//   * HEALPix-SSIM (Sec. 4.1): normalised 11x11 Gaussian-window statistics on
//     face-local (x, y) with neighbours taken across face edges; missing
//     quadrants at three-face vertices carry weight zero.
//   * Gradients: the exact derivative of the forward above.  Per-pixel
//     reverse compositing, then forward-mode dual numbers through the offset
//     and the preprocessing (no hand-derived chain rule to get wrong).
//
// Readings of the paper where it is silent are documented with each
// function; the constants arrive as arguments.
//
// Parity pins for this file live in tests/test_oracle_*.py.

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>

#ifdef _OPENMP
#include <omp.h>
#endif

typedef int64_t i64;

// ---------------------------------------------------------------------------
// Dual numbers (forward-mode derivatives) -- one tangent direction.
// ---------------------------------------------------------------------------
struct Dual {
  double v, d;
  Dual(double a = 0.0, double b = 0.0) : v(a), d(b) {}
};
static inline Dual operator+(Dual a, Dual b) { return Dual(a.v + b.v, a.d + b.d); }
static inline Dual operator-(Dual a, Dual b) { return Dual(a.v - b.v, a.d - b.d); }
static inline Dual operator-(Dual a) { return Dual(-a.v, -a.d); }
static inline Dual operator*(Dual a, Dual b) { return Dual(a.v * b.v, a.d * b.v + a.v * b.d); }
static inline Dual operator/(Dual a, Dual b) { return Dual(a.v / b.v, (a.d * b.v - a.v * b.d) / (b.v * b.v)); }
static inline Dual operator+(Dual a, double b) { return Dual(a.v + b, a.d); }
static inline Dual operator+(double b, Dual a) { return Dual(a.v + b, a.d); }
static inline Dual operator-(Dual a, double b) { return Dual(a.v - b, a.d); }
static inline Dual operator-(double b, Dual a) { return Dual(b - a.v, -a.d); }
static inline Dual operator*(Dual a, double b) { return Dual(a.v * b, a.d * b); }
static inline Dual operator*(double b, Dual a) { return Dual(a.v * b, a.d * b); }
static inline Dual operator/(Dual a, double b) { return Dual(a.v / b, a.d / b); }
static inline bool operator<(Dual a, Dual b) { return a.v < b.v; }
static inline double val(double a) { return a; }
static inline double val(Dual a) { return a.v; }
static inline Dual sqrt(Dual a) { double s = std::sqrt(a.v); return Dual(s, s > 0 ? a.d / (2 * s) : 0.0); }
static inline Dual sin(Dual a) { return Dual(std::sin(a.v), std::cos(a.v) * a.d); }
static inline Dual cos(Dual a) { return Dual(std::cos(a.v), -std::sin(a.v) * a.d); }
static inline Dual exp(Dual a) { double e = std::exp(a.v); return Dual(e, e * a.d); }
static inline Dual asin(Dual a) { return Dual(std::asin(a.v), a.d / std::sqrt(std::max(1e-300, 1 - a.v * a.v))); }
static inline Dual atan2(Dual y, Dual x) {
  double r2 = x.v * x.v + y.v * y.v;
  return Dual(std::atan2(y.v, x.v), r2 > 0 ? (x.v * y.d - y.v * x.d) / r2 : 0.0);
}
using std::sqrt; using std::sin; using std::cos; using std::exp; using std::asin; using std::atan2;

// ---------------------------------------------------------------------------
// HEALPix geometry (Gorski et al. 2005).  NESTED index p = f*Nside^2 +
// interleave(x, y) with the bits of x at even and y at odd positions.
// Face f sits in row f/4 (north, equatorial, south); rings are numbered
// jr = 1 .. 4 Nside - 1 from the north pole.
// ---------------------------------------------------------------------------
static const int kJRLL[12] = {2, 2, 2, 2, 3, 3, 3, 3, 4, 4, 4, 4};
static const int kJPLL[12] = {1, 3, 5, 7, 0, 2, 4, 6, 1, 3, 5, 7};

struct XYF { i64 x, y; int f; };

static XYF nest2xyf(int order, i64 p) {
  XYF r; r.f = (int)(p >> (2 * order)); r.x = 0; r.y = 0;
  i64 q = p & ((((i64)1) << (2 * order)) - 1);
  for (int b = 0; b < order; ++b) {
    r.x |= ((q >> (2 * b)) & 1) << b;
    r.y |= ((q >> (2 * b + 1)) & 1) << b;
  }
  return r;
}

static i64 xyf2nest(int order, i64 x, i64 y, int f) {
  i64 q = 0;
  for (int b = 0; b < order; ++b) {
    q |= ((x >> b) & 1) << (2 * b);
    q |= ((y >> b) & 1) << (2 * b + 1);
  }
  return ((i64)f << (2 * order)) + q;
}

struct RingPos { i64 jr, jp, nr; int kshift; };

// Ring number jr (1-based from the north), position jp (1-based) within the
// ring, ring length/4 = nr and the half-pixel shift of equatorial rings.
static RingPos xyf2ringpos(int order, XYF a) {
  i64 N = (i64)1 << order;
  RingPos r;
  r.jr = kJRLL[a.f] * N - a.x - a.y - 1;
  if (r.jr < N) { r.nr = r.jr; r.kshift = 0; }
  else if (r.jr > 3 * N) { r.nr = 4 * N - r.jr; r.kshift = 0; }
  else { r.nr = N; r.kshift = (int)((r.jr - N) & 1); }
  r.jp = (kJPLL[a.f] * r.nr + a.x - a.y + 1 + r.kshift) / 2;
  if (r.jp > 4 * r.nr) r.jp -= 4 * r.nr;
  if (r.jp < 1) r.jp += 4 * r.nr;
  return r;
}

// z = cos(colatitude), HEALPix longitude phi in [0, 2 pi), sin(colatitude).
static void ringpos_zphi(int order, const RingPos& r, double* z, double* phi, double* sth) {
  i64 N = (i64)1 << order;
  double Nd = (double)N;
  if (r.jr < N || r.jr > 3 * N) {
    double nr = (double)r.nr;
    double tmp = nr * nr / (3.0 * Nd * Nd);       // 1 - |z|, exact
    *z = (r.jr < N) ? 1.0 - tmp : -(1.0 - tmp);
    *sth = std::sqrt(tmp * (2.0 - tmp));
    *phi = ((double)r.jp - 0.5) * (M_PI / 2.0) / nr;
  } else {
    *z = (double)(2 * N - r.jr) * 2.0 / (3.0 * Nd);
    *sth = std::sqrt((1.0 - *z) * (1.0 + *z));
    *phi = ((double)r.jp - 0.5 * (1 + r.kshift)) * (M_PI / 2.0) / Nd;
  }
}

// Index in RING ordering.
static i64 ringpos2ring(int order, const RingPos& r) {
  i64 N = (i64)1 << order;
  i64 before;
  if (r.jr < N) before = 2 * r.jr * (r.jr - 1);
  else if (r.jr <= 3 * N) before = 2 * N * (N - 1) + (r.jr - N) * 4 * N;
  else { i64 s = 4 * N - r.jr; before = 12 * N * N - 2 * s * (s + 1); }
  return before + r.jp - 1;
}

// Camera-frame unit vector of a pixel centre.  The grid is fixed in the
// camera frame: HEALPix (x_h, y_h, z_h) = (t_z, t_x, t_y) / r, so the pole is
// camera +y and the HEALPix longitude equals omega = atan2(t_x, t_z).
static void pix_vec(int order, i64 p, double v[3]) {
  XYF a = nest2xyf(order, p);
  RingPos r = xyf2ringpos(order, a);
  double z, phi, sth;
  ringpos_zphi(order, r, &z, &phi, &sth);
  v[0] = sth * std::sin(phi);
  v[1] = z;
  v[2] = sth * std::cos(phi);
}

// Face-extended chart: pixel at face-local (x, y) of face f where x or y may
// leave [0, N) by less than N.  Crossing one edge moves to the neighbouring
// face with its local axes rotated to line up; the diagonal quadrant exists
// only at the four-face vertices (the poles and the equatorial corners).
// Returns -1 in the missing quadrant of a three-face vertex.
static i64 chart_pixel(int order, int f, i64 x, i64 y) {
  i64 N = (i64)1 << order;
  bool xlo = x < 0, xhi = x >= N, ylo = y < 0, yhi = y >= N;
  if (!(xlo || xhi || ylo || yhi)) return xyf2nest(order, x, y, f);
  int row = f / 4, c = f % 4;
  int g = -1; i64 X = 0, Y = 0;
  if ((xlo || xhi) && (ylo || yhi)) {
    if (row == 0) {
      if (xhi && yhi) { g = (c + 2) % 4; X = 2 * N - 1 - x; Y = 2 * N - 1 - y; }
      else if (xlo && ylo) { g = 8 + c; X = x + N; Y = y + N; }
    } else if (row == 1) {
      if (xhi && ylo) { g = 4 + (c + 1) % 4; X = x - N; Y = y + N; }
      else if (xlo && yhi) { g = 4 + (c + 3) % 4; X = x + N; Y = y - N; }
    } else {
      if (xlo && ylo) { g = 8 + (c + 2) % 4; X = -x - 1; Y = -y - 1; }
      else if (xhi && yhi) { g = c; X = x - N; Y = y - N; }
    }
    if (g < 0) return -1;
  } else if (xlo || xhi) {
    if (row == 0) {
      if (xhi) { g = (c + 1) % 4; X = y; Y = 2 * N - 1 - x; }
      else { g = 4 + c; X = x + N; Y = y; }
    } else if (row == 1) {
      if (xhi) { g = c; X = x - N; Y = y; }
      else { g = 8 + (c + 3) % 4; X = x + N; Y = y; }
    } else {
      if (xhi) { g = 4 + (c + 1) % 4; X = x - N; Y = y; }
      else { g = 8 + (c + 3) % 4; X = y; Y = -x - 1; }
    }
  } else {
    if (row == 0) {
      if (yhi) { g = (c + 3) % 4; X = 2 * N - 1 - y; Y = x; }
      else { g = 4 + (c + 1) % 4; X = x; Y = y + N; }
    } else if (row == 1) {
      if (yhi) { g = (c + 3) % 4; X = x; Y = y - N; }
      else { g = 8 + c; X = x; Y = y + N; }
    } else {
      if (yhi) { g = 4 + c; X = x; Y = y - N; }
      else { g = 8 + (c + 1) % 4; X = -y - 1; Y = x; }
    }
  }
  if (X < 0 || X >= N || Y < 0 || Y >= N) return -1;  // more than one face away
  return xyf2nest(order, X, Y, g);
}

// ---------------------------------------------------------------------------
// Camera visibility mask M_C (Sec. 3.1; supp. "Compatibility with Any FoV").
// ---------------------------------------------------------------------------
enum { CAM_FULL = 0, CAM_FISHEYE = 1, CAM_PINHOLE = 2 };

static bool mask_dir(int cam, double fx, double fy, const double t[3]) {
  if (cam == CAM_FULL) return true;
  if (cam == CAM_FISHEYE) {
    // anisotropic equidistant model: incident angle psi = r_m * w_eff(gamma),
    // valid while r_m <= pi/2, w = FoV / 180 deg.
    double psi = std::acos(std::max(-1.0, std::min(1.0, t[2])));
    double gam = std::atan2(t[1], t[0]);
    double wx = fx / M_PI, wy = fy / M_PI;
    double weff = std::sqrt(wx * std::cos(gam) * wx * std::cos(gam) + wy * std::sin(gam) * wy * std::sin(gam));
    return psi <= 0.5 * M_PI * weff;
  }
  // pinhole: in front of the camera and inside both half-FoVs
  if (!(t[2] > 0)) return false;
  return std::fabs(t[0]) <= std::tan(0.5 * fx) * t[2] && std::fabs(t[1]) <= std::tan(0.5 * fy) * t[2];
}

// ---------------------------------------------------------------------------
// Real spherical harmonics, degree <= 3, from associated Legendre functions
// (no Condon-Shortley phase), orthonormal on the unit sphere.
// Index k = l*l + l + m.  Direction v = (x, y, z), polar axis z.
// ---------------------------------------------------------------------------
template <class T>
static void sh_basis(int deg, T x, T y, T z, T* Y) {
  // P_l^m(cos theta) with sin theta factors written as powers of
  // s = sqrt(x^2 + y^2); cos(m az) s^m = Re((x + i y)^m), sin(m az) s^m = Im(...)
  T cm[4], sm[4];
  cm[0] = T(1.0); sm[0] = T(0.0);
  for (int m = 1; m <= 3; ++m) { cm[m] = cm[m - 1] * x - sm[m - 1] * y; sm[m] = sm[m - 1] * x + cm[m - 1] * y; }
  // Legendre part without the s^m factor: Q_l^m(z) = P_l^m(z) / s^m
  auto Q = [&](int l, int m) -> T {
    if (l == 0) return T(1.0);
    if (l == 1) return m == 0 ? z : T(1.0);
    if (l == 2) { if (m == 0) return 0.5 * (3.0 * z * z - 1.0); if (m == 1) return 3.0 * z; return T(3.0); }
    if (m == 0) return 0.5 * (5.0 * z * z * z - 3.0 * z);
    if (m == 1) return 1.5 * (5.0 * z * z - 1.0);
    if (m == 2) return 15.0 * z;
    return T(15.0);
  };
  auto fact = [](int n) { double f = 1; for (int i = 2; i <= n; ++i) f *= i; return f; };
  for (int l = 0; l <= deg; ++l) {
    for (int m = -l; m <= l; ++m) {
      int am = m < 0 ? -m : m;
      double Nlm = std::sqrt((2 * l + 1) / (4 * M_PI) * fact(l - am) / fact(l + am));
      T q = Q(l, am);
      T out;
      if (m == 0) out = Nlm * q;
      else if (m > 0) out = (std::sqrt(2.0) * Nlm) * q * cm[am];
      else out = (std::sqrt(2.0) * Nlm) * q * sm[am];
      Y[l * l + l + m] = out;
    }
  }
}

// ---------------------------------------------------------------------------
// Inputs
// ---------------------------------------------------------------------------
extern "C" {

typedef struct {
  i64 P; int sh_degree;
  const float *mean, *scale, *rot, *opacity, *sh;  // [3][P] [3][P] [4][P] [P] [K][3][P]
} or_scene;

typedef struct {
  double W[9], b[3], center[3];
  int cam_type; double fov_x, fov_y; int order;
} or_view;

typedef struct {
  double eps_T, alpha_max, q_cut, r_min, rs_sigma, bin_guard, sh_offset;
  int tile_log2;   // log2 of the tile side B (16 -> 4); clipped to order
} or_params;

}  // extern "C"

// ---------------------------------------------------------------------------
// Preprocessing of one Gaussian (Alg. 1 preprocessing; Eqs. lonlat_projection
// and arc_scaling).  Templated so the same code yields values (double) and
// directional derivatives (Dual).
// ---------------------------------------------------------------------------
template <class T>
struct ProjT {
  bool valid;
  T omega, phi, rho;      // direction (radians) and radial depth
  T A, B, C;              // conic: q = A dx^2 + 2 B dx dy + C dy^2
  T sa, sb, sc;           // Sigma_arc entries (omega-omega, omega-phi, phi-phi)
  T rs;                   // bounding radius
  T rgb[3];
  bool clamped[3];
};

template <class T>
static ProjT<T> preprocess_one(const T mu[3], const T s[3], const T qr[4], const double* shc /*[K][3]*/,
                               int deg, const or_view& V, const or_params& prm) {
  ProjT<T> o; o.valid = false;
  // quaternion (w, x, y, z), normalised
  T qn = sqrt(qr[0] * qr[0] + qr[1] * qr[1] + qr[2] * qr[2] + qr[3] * qr[3]);
  T w = qr[0] / qn, x = qr[1] / qn, y = qr[2] / qn, z = qr[3] / qn;
  T R[3][3] = {
      {1.0 - 2.0 * (y * y + z * z), 2.0 * (x * y - w * z), 2.0 * (x * z + w * y)},
      {2.0 * (x * y + w * z), 1.0 - 2.0 * (x * x + z * z), 2.0 * (y * z - w * x)},
      {2.0 * (x * z - w * y), 2.0 * (y * z + w * x), 1.0 - 2.0 * (x * x + y * y)}};
  T S3[3][3];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      T acc = T(0.0);
      for (int k = 0; k < 3; ++k) acc = acc + R[i][k] * s[k] * s[k] * R[j][k];
      S3[i][j] = acc;
    }
  // camera-space centre t = W mu + b
  T t[3];
  for (int i = 0; i < 3; ++i) t[i] = V.W[3 * i] * mu[0] + V.W[3 * i + 1] * mu[1] + V.W[3 * i + 2] * mu[2] + V.b[i];
  T r = sqrt(t[0] * t[0] + t[1] * t[1] + t[2] * t[2]);
  o.rho = r;
  if (!(val(r) >= prm.r_min)) return o;
  T rho2 = t[0] * t[0] + t[2] * t[2];
  T rhx = sqrt(rho2);
  if (val(rhx) < 1e-12 * val(r)) return o;  // exactly at a pole: direction frame undefined
  o.omega = atan2(t[0], t[2]);
  o.phi = atan2(t[1], rhx);
  // Jacobian of Pi = (atan2(tx, tz), atan2(ty, sqrt(tx^2 + tz^2)))
  T r2 = r * r;
  T J[2][3] = {{t[2] / rho2, T(0.0), -t[0] / rho2},
               {-(t[0] * t[1]) / (rhx * r2), rhx / r2, -(t[2] * t[1]) / (rhx * r2)}};
  // T = J W (2x3)
  T M[2][3];
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 3; ++j) M[i][j] = J[i][0] * V.W[j] + J[i][1] * V.W[3 + j] + J[i][2] * V.W[6 + j];
  T Sr[2][2];
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j) {
      T acc = T(0.0);
      for (int k = 0; k < 3; ++k)
        for (int l = 0; l < 3; ++l) acc = acc + M[i][k] * S3[k][l] * M[j][l];
      Sr[i][j] = acc;
    }
  // latitude scaling S_phi = diag(cos phi, 1)
  T cp = cos(o.phi);
  o.sa = cp * Sr[0][0] * cp;
  o.sb = cp * Sr[0][1];
  o.sc = Sr[1][1];
  T det = o.sa * o.sc - o.sb * o.sb;
  if (!(val(det) > 0)) return o;
  o.A = o.sc / det; o.B = -o.sb / det; o.C = o.sa / det;
  T hm = 0.5 * (o.sa + o.sc);
  T hd = 0.5 * (o.sa - o.sc);
  T lmax = hm + sqrt(hd * hd + o.sb * o.sb);
  o.rs = prm.rs_sigma * sqrt(lmax);
  if (val(o.rs) > M_PI) o.rs = T(M_PI);
  // view-dependent colour: real SH at the world-space viewing direction
  T v[3] = {mu[0] - V.center[0], mu[1] - V.center[1], mu[2] - V.center[2]};
  T vn = sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
  T Y[16];
  sh_basis<T>(deg, v[0] / vn, v[1] / vn, v[2] / vn, Y);
  int K = (deg + 1) * (deg + 1);
  for (int ch = 0; ch < 3; ++ch) {
    T acc = T(prm.sh_offset);
    for (int k = 0; k < K; ++k) acc = acc + shc[k * 3 + ch] * Y[k];
    o.clamped[ch] = val(acc) < 0;
    o.rgb[ch] = o.clamped[ch] ? T(0.0) : acc;
  }
  o.valid = true;
  return o;
}

// ---------------------------------------------------------------------------
// Spherical offset (Sec. 3.4): haversine great-circle distance from the
// Gaussian centre (omega_i, phi_i) to the pixel centre (omega_p, phi_p),
// decomposed along the bearing beta measured at the Gaussian towards the
// pixel: d = d_gc (sin beta, cos beta) in (east = +omega, north = +phi).
// ---------------------------------------------------------------------------
template <class T>
static void sph_offset(T om_i, T ph_i, double om_p, double ph_p, T* dx, T* dy, T* dgc) {
  T dom = om_p - om_i;
  T dph = ph_p - ph_i;
  T s1 = sin(0.5 * dph), s2 = sin(0.5 * dom);
  T h = s1 * s1 + cos(ph_i) * std::cos(ph_p) * s2 * s2;
  if (val(h) > 1.0) h = T(1.0);
  T d = 2.0 * asin(sqrt(h));
  T beta = atan2(sin(dom) * std::cos(ph_p), cos(ph_i) * std::sin(ph_p) - sin(ph_i) * std::cos(ph_p) * cos(dom));
  *dx = d * sin(beta);
  *dy = d * cos(beta);
  *dgc = d;
}

static void scene_gauss(const or_scene& S, i64 i, double mu[3], double s[3], double q[4], std::vector<double>& shc) {
  for (int k = 0; k < 3; ++k) { mu[k] = S.mean[k * S.P + i]; s[k] = S.scale[k * S.P + i]; }
  for (int k = 0; k < 4; ++k) q[k] = S.rot[k * S.P + i];
  int K = (S.sh_degree + 1) * (S.sh_degree + 1);
  shc.resize(K * 3);
  for (int k = 0; k < K; ++k)
    for (int ch = 0; ch < 3; ++ch) shc[k * 3 + ch] = S.sh[(k * 3 + ch) * S.P + i];
}

// Pixel centre in (omega, phi) and as a camera-frame unit vector.
static void pix_angles(int order, i64 p, double* om, double* ph, double v[3]) {
  pix_vec(order, p, v);
  *om = std::atan2(v[0], v[2]);
  *ph = std::atan2(v[1], std::sqrt(v[0] * v[0] + v[2] * v[2]));
}

static inline double angle_between(const double a[3], const double b[3]) {
  double c[3] = {a[1] * b[2] - a[2] * b[1], a[2] * b[0] - a[0] * b[2], a[0] * b[1] - a[1] * b[0]};
  return std::atan2(std::sqrt(c[0] * c[0] + c[1] * c[1] + c[2] * c[2]), a[0] * b[0] + a[1] * b[1] + a[2] * b[2]);
}

static inline int tile_order(int order, const or_params& prm) {
  int b = std::min(prm.tile_log2, order);
  return order - b;
}

// ---------------------------------------------------------------------------
// C interface
// ---------------------------------------------------------------------------
extern "C" {

int or_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

void or_set_threads(int n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
#else
  (void)n;
#endif
}

// --- geometry -------------------------------------------------------------
void or_nest2xyf(int order, i64 n, const i64* p, i64* x, i64* y, int* f) {
  for (i64 k = 0; k < n; ++k) { XYF a = nest2xyf(order, p[k]); x[k] = a.x; y[k] = a.y; f[k] = a.f; }
}
void or_xyf2nest(int order, i64 n, const i64* x, const i64* y, const int* f, i64* p) {
  for (i64 k = 0; k < n; ++k) p[k] = xyf2nest(order, x[k], y[k], f[k]);
}
void or_nest2ring(int order, i64 n, const i64* p, i64* ring) {
  for (i64 k = 0; k < n; ++k) ring[k] = ringpos2ring(order, xyf2ringpos(order, nest2xyf(order, p[k])));
}
// ring number (1-based), position (1-based), z, phi per nested pixel
void or_pix_ringinfo(int order, i64 n, const i64* p, i64* jr, i64* jp, double* z, double* phi) {
  for (i64 k = 0; k < n; ++k) {
    RingPos r = xyf2ringpos(order, nest2xyf(order, p[k]));
    double sth;
    jr[k] = r.jr; jp[k] = r.jp;
    ringpos_zphi(order, r, &z[k], &phi[k], &sth);
  }
}
// camera-frame unit vectors [n][3]
void or_pix_vec(int order, i64 n, const i64* p, double* v) {
#pragma omp parallel for schedule(static)
  for (i64 k = 0; k < n; ++k) pix_vec(order, p[k], v + 3 * k);
}
i64 or_chart_pixel(int order, int f, i64 x, i64 y) { return chart_pixel(order, f, x, y); }

// --- mask -----------------------------------------------------------------
// Writes the active nested pixels in increasing order; returns their count.
i64 or_mask(const or_view* V, i64* active) {
  int order = V->order;
  i64 npix = 12 * ((i64)1 << (2 * order));
  std::vector<unsigned char> m(npix);
#pragma omp parallel for schedule(static)
  for (i64 p = 0; p < npix; ++p) {
    double t[3];
    pix_vec(order, p, t);
    m[p] = mask_dir(V->cam_type, V->fov_x, V->fov_y, t) ? 1 : 0;
  }
  i64 n = 0;
  for (i64 p = 0; p < npix; ++p)
    if (m[p]) { if (active) active[n] = p; ++n; }
  return n;
}

// --- spherical harmonics --------------------------------------------------
void or_sh_basis(int deg, i64 n, const double* v /*[n][3]*/, double* Y /*[n][16]*/) {
  for (i64 k = 0; k < n; ++k) sh_basis<double>(deg, v[3 * k], v[3 * k + 1], v[3 * k + 2], Y + 16 * k);
}

// --- preprocessing ----------------------------------------------------------
// out arrays, each [P]: valid, omega, phi, rho, A, B, C, sa, sb, sc, rs; rgb [3][P]
void or_preprocess(const or_scene* S, const or_view* V, const or_params* prm, int* valid, double* omega,
                   double* phi, double* rho, double* conic /*[3][P]*/, double* sarc /*[3][P]*/, double* rs,
                   double* rgb /*[3][P]*/) {
  i64 P = S->P;
#pragma omp parallel for schedule(static)
  for (i64 i = 0; i < P; ++i) {
    double mu[3], s[3], q[4];
    std::vector<double> shc;
    scene_gauss(*S, i, mu, s, q, shc);
    ProjT<double> o = preprocess_one<double>(mu, s, q, shc.data(), S->sh_degree, *V, *prm);
    valid[i] = o.valid ? 1 : 0;
    rho[i] = o.rho;
    if (!o.valid) {
      omega[i] = phi[i] = rs[i] = 0;
      for (int k = 0; k < 3; ++k) conic[k * P + i] = sarc[k * P + i] = rgb[k * P + i] = 0;
      continue;
    }
    omega[i] = o.omega; phi[i] = o.phi; rs[i] = o.rs;
    conic[i] = o.A; conic[P + i] = o.B; conic[2 * P + i] = o.C;
    sarc[i] = o.sa; sarc[P + i] = o.sb; sarc[2 * P + i] = o.sc;
    for (int k = 0; k < 3; ++k) rgb[k * P + i] = o.rgb[k];
  }
}

// --- tiles ----------------------------------------------------------------
// Tile caps: for each tile of order kt, centre = normalised sum of the
// camera-frame directions of its B x B pixel centres, radius = largest angle
// from that centre to any of those pixel centres.
void or_tile_caps(int order, int tile_log2, double* centre /*[ntile][3]*/, double* radius /*[ntile]*/) {
  int b = std::min(tile_log2, order);
  int kt = order - b;
  i64 ntile = 12 * ((i64)1 << (2 * kt));
  i64 per = (i64)1 << (2 * b);
#pragma omp parallel for schedule(static)
  for (i64 t = 0; t < ntile; ++t) {
    double c[3] = {0, 0, 0};
    std::vector<double> vs(3 * per);
    for (i64 j = 0; j < per; ++j) {
      pix_vec(order, t * per + j, &vs[3 * j]);
      for (int k = 0; k < 3; ++k) c[k] += vs[3 * j + k];
    }
    double n = std::sqrt(c[0] * c[0] + c[1] * c[1] + c[2] * c[2]);
    for (int k = 0; k < 3; ++k) c[k] /= n;
    double R = 0;
    for (i64 j = 0; j < per; ++j) R = std::max(R, angle_between(c, &vs[3 * j]));
    for (int k = 0; k < 3; ++k) centre[3 * t + k] = c[k];
    radius[t] = R;
  }
}

// Tile sets (the binning definition): tile t belongs to T_i iff t holds at
// least one active pixel and the angular distance from t's cap centre to the
// Gaussian centre is at most r_s,i + R_t + guard.  Brute force over every
// (Gaussian, active tile).  For the Gaussians listed in gids, writes
// (gid, tile, margin) triples where margin = (r_s + R_t + guard) - distance;
// also pairs whose |margin| <= report_band with a negative margin are written
// (flag 0) so the caller can see near misses.  Returns the number written or,
// with out == NULL, the number that would be written.
i64 or_tile_sets(int order, const or_params* prm, const double* tc, const double* tr, const unsigned char* tile_active,
                 i64 n_g, const i64* gids, const int* valid, const double* omega, const double* phi, const double* rs,
                 double report_band, i64 cap, i64* out_gid, i64* out_tile, double* out_margin, int* out_in) {
  int kt = tile_order(order, *prm);
  i64 ntile = 12 * ((i64)1 << (2 * kt));
  std::vector<std::vector<i64>> tl(n_g);
  std::vector<std::vector<double>> ml(n_g);
  std::vector<std::vector<int>> il(n_g);
#pragma omp parallel for schedule(dynamic, 64)
  for (i64 k = 0; k < n_g; ++k) {
    i64 i = gids[k];
    if (!valid[i]) continue;
    double u[3] = {std::cos(phi[i]) * std::sin(omega[i]), std::sin(phi[i]), std::cos(phi[i]) * std::cos(omega[i])};
    for (i64 t = 0; t < ntile; ++t) {
      if (!tile_active[t]) continue;
      double d = angle_between(u, tc + 3 * t);
      double m = rs[i] + tr[t] + prm->bin_guard - d;
      if (m >= 0 || m >= -report_band) { tl[k].push_back(t); ml[k].push_back(m); il[k].push_back(m >= 0); }
    }
  }
  i64 n = 0;
  for (i64 k = 0; k < n_g; ++k)
    for (size_t j = 0; j < tl[k].size(); ++j) {
      if (out_gid && n < cap) {
        out_gid[n] = gids[k]; out_tile[n] = tl[k][j]; out_margin[n] = ml[k][j]; out_in[n] = il[k][j];
      }
      ++n;
    }
  return n;
}

// --- compositing --------------------------------------------------------
// Brute-force render of the listed pixels (Eq. unified_rendering; Alg. 1
// rendering loop).  For pixel p the candidates are all valid Gaussians with
// q_i(p) <= q_cut, ordered by (rho, index); composite front to back with
// alpha = min(alpha_max, o exp(-q/2)) and stop once T < eps_T (after
// compositing the Gaussian that crossed it).
//
// Outputs per pixel: rgb [3][n], T [n], n_used [n] (Gaussians composited),
// frag [n]: an allowance (colour units) covering the decisions whose FP32
// outcome may legitimately differ (fragility bookkeeping): q within the band
// q_band(qtol = {abs, rel, dir}) of q_cut, and T within ttol (relative) of
// eps_T at the stopping point.
// A conservative pre-filter (angular distance <= r_s (1 + 1e-9) + 1e-12)
// skips Gaussians that cannot reach q <= q_cut, since q <= 9 implies d_gc <= r_s.
struct Cand { double rho; i64 i; double q, dx, dy, qband; };


// band of q around q_cut inside which the FP32 decision may differ: qtol_abs,
// plus qtol_rel times the magnitudes of the terms of q (|A| dx^2 + 2 |B| |dx dy|
// + |C| dy^2, which covers cancellation in an ill-conditioned conic), plus
// the change of q that an offset error of qtol_dir radians causes on the
// q = q_cut ellipse, |dq| <= 2 |conic d| |delta d| <= 2 sqrt(q_cut lmax) |delta d|
static double q_band(const double* conic, i64 P, i64 i, double q_cut, double dx, double dy, double qtol_abs,
                     double qtol_rel, double qtol_dir) {
  const double A = conic[i], B = conic[P + i], Cc = conic[2 * P + i];
  const double lmax = 0.5 * (A + Cc) + std::sqrt(0.25 * (A - Cc) * (A - Cc) + B * B);
  const double terms = std::fabs(A) * dx * dx + 2 * std::fabs(B * dx * dy) + std::fabs(Cc) * dy * dy;
  return qtol_abs + qtol_rel * terms + 2.0 * std::sqrt(q_cut * std::max(lmax, 0.0)) * qtol_dir;
}

static void pixel_candidates(const or_scene& S, const or_params& prm, const int* valid, const double* omega,
                             const double* phi, const double* rho, const double* conic, const double* rs,
                             double om_p, double ph_p, const double pv[3], const double qtol[3],
                             std::vector<Cand>& out) {
  i64 P = S.P;
  out.clear();
  for (i64 i = 0; i < P; ++i) {
    if (!valid[i]) continue;
    double u[3] = {std::cos(phi[i]) * std::sin(omega[i]), std::sin(phi[i]), std::cos(phi[i]) * std::cos(omega[i])};
    double ang = angle_between(u, pv);
    if (ang > rs[i] * (1 + 1e-9) + 1e-12) continue;
    double dx, dy, dgc;
    sph_offset<double>(omega[i], phi[i], om_p, ph_p, &dx, &dy, &dgc);
    double q = conic[i] * dx * dx + 2 * conic[P + i] * dx * dy + conic[2 * P + i] * dy * dy;
    if (q <= prm.q_cut * (1 + 1e-3))
      out.push_back(Cand{rho[i], i, q, dx, dy, q_band(conic, P, i, prm.q_cut, dx, dy, qtol[0], qtol[1], qtol[2])});
  }
  std::sort(out.begin(), out.end(), [](const Cand& a, const Cand& b) { return a.rho < b.rho || (a.rho == b.rho && a.i < b.i); });
}

// Front-to-back compositing of one pixel's candidates (already ordered by
// (rho, index)); see or_render for the outputs.
static void composite(const std::vector<Cand>& c, const or_params& prm, const double* opac, const double* rho,
                      const double* rgbg, i64 P, double ttol_rel, double C[3], double* Tout,
                      i64* n_used, double* frag, double* Dout) {
  double Tr = 1.0, fr = 0, D = 0;
  C[0] = C[1] = C[2] = 0;
  i64 used = 0;
  for (const Cand& e : c) {
    double cmax = std::max(std::fabs(rgbg[e.i]), std::max(std::fabs(rgbg[P + e.i]), std::fabs(rgbg[2 * P + e.i])));
    if (std::fabs(e.q - prm.q_cut) <= e.qband) fr += Tr * std::min(prm.alpha_max, opac[e.i] * std::exp(-0.5 * prm.q_cut)) * cmax;
    if (e.q > prm.q_cut) continue;
    double a = std::min(prm.alpha_max, opac[e.i] * std::exp(-0.5 * e.q));
    for (int ch = 0; ch < 3; ++ch) C[ch] += Tr * a * rgbg[ch * P + e.i];
    D += Tr * a / rho[e.i];  // inverse radial depth composited like a colour (Sec. 3.2)
    double Tn = Tr * (1 - a);
    ++used;
    if (std::fabs(Tn - prm.eps_T) <= ttol_rel * prm.eps_T) fr += std::max(Tr, prm.eps_T) * 1.0 * cmax;
    Tr = Tn;
    if (Tr < prm.eps_T) break;
  }
  *Tout = Tr; *n_used = used; *frag = fr; *Dout = D;
}

void or_render(const or_scene* S, const or_view* V, const or_params* prm, const int* valid, const double* omega,
               const double* phi, const double* rho, const double* conic, const double* rs, const double* rgbg,
               i64 n, const i64* pix, const double* qtol, double ttol_rel, double* rgb, double* T,
               i64* n_used, double* frag, double* invd) {
  i64 P = S->P;
  std::vector<double> opac(P);
  for (i64 i = 0; i < P; ++i) opac[i] = S->opacity[i];
#pragma omp parallel for schedule(dynamic, 16)
  for (i64 k = 0; k < n; ++k) {
    double om_p, ph_p, pv[3];
    pix_angles(V->order, pix[k], &om_p, &ph_p, pv);
    std::vector<Cand> c;
    pixel_candidates(*S, *prm, valid, omega, phi, rho, conic, rs, om_p, ph_p, pv, qtol, c);
    double C[3], D;
    composite(c, *prm, opac.data(), rho, rgbg, P, ttol_rel, C, &T[k], &n_used[k], &frag[k], &D);
    for (int ch = 0; ch < 3; ++ch) rgb[ch * n + k] = C[ch];
    if (invd) invd[k] = D;
  }
}

// The same render where pixel p sees only the Gaussians of its tile's list
// (list/ranges as in or_n_contrib): the entries with q <= q_cut, ordered by
// (rho, index).  With the approximate tile sets of the paper's queries a list
// can miss Gaussians that reach the pixel, and then the image differs from
// the exact one (the aliasing the paper reports for coarse queries).
void or_render_lists(const or_scene* S, const or_view* V, const or_params* prm, const double* omega,
                     const double* phi, const double* rho, const double* conic, const double* rgbg, const i64* list,
                     const i64* ranges, i64 n, const i64* pix, const double* qtol, double ttol_rel,
                     double* rgb, double* T, i64* n_used, double* frag) {
  i64 P = S->P;
  int kt = tile_order(V->order, *prm);
  int sh = 2 * (V->order - kt);
  std::vector<double> opac(P);
  for (i64 i = 0; i < P; ++i) opac[i] = S->opacity[i];
#pragma omp parallel for schedule(dynamic, 16)
  for (i64 k = 0; k < n; ++k) {
    double om_p, ph_p, pv[3];
    pix_angles(V->order, pix[k], &om_p, &ph_p, pv);
    i64 t = pix[k] >> sh;
    std::vector<Cand> c;
    for (i64 j = ranges[2 * t]; j < ranges[2 * t + 1]; ++j) {
      i64 i = list[j];
      double dx, dy, dgc;
      sph_offset<double>(omega[i], phi[i], om_p, ph_p, &dx, &dy, &dgc);
      double q = conic[i] * dx * dx + 2 * conic[P + i] * dx * dy + conic[2 * P + i] * dy * dy;
      if (q <= prm->q_cut * (1 + 1e-3))
        c.push_back(Cand{rho[i], i, q, dx, dy, q_band(conic, P, i, prm->q_cut, dx, dy, qtol[0], qtol[1], qtol[2])});
    }
    std::sort(c.begin(), c.end(), [](const Cand& a, const Cand& b) { return a.rho < b.rho || (a.rho == b.rho && a.i < b.i); });
    double C[3], D;
    composite(c, *prm, opac.data(), rho, rgbg, P, ttol_rel, C, &T[k], &n_used[k], &frag[k], &D);
    for (int ch = 0; ch < 3; ++ch) rgb[ch * n + k] = C[ch];
  }
}

// n_contrib as the tiled renderer defines it: entries of the pixel's tile
// list consumed, counting entries skipped because q > q_cut, up to and
// including the entry after which T < eps_T.  list/ranges: the oracle's own
// sorted tile lists (tile t owns list[ranges[2t] .. ranges[2t+1])).
void or_n_contrib(const or_scene* S, const or_view* V, const or_params* prm, const double* omega, const double* phi,
                  const double* conic, const i64* list, const i64* ranges, i64 n, const i64* pix, i64* ncon) {
  i64 P = S->P;
  int kt = tile_order(V->order, *prm);
  int sh = 2 * (V->order - kt);
#pragma omp parallel for schedule(dynamic, 16)
  for (i64 k = 0; k < n; ++k) {
    double om_p, ph_p, pv[3];
    pix_angles(V->order, pix[k], &om_p, &ph_p, pv);
    i64 t = pix[k] >> sh;
    double Tr = 1.0;
    i64 cnt = 0;
    for (i64 j = ranges[2 * t]; j < ranges[2 * t + 1]; ++j) {
      i64 i = list[j];
      ++cnt;
      double dx, dy, dgc;
      sph_offset<double>(omega[i], phi[i], om_p, ph_p, &dx, &dy, &dgc);
      double q = conic[i] * dx * dx + 2 * conic[P + i] * dx * dy + conic[2 * P + i] * dy * dy;
      if (q > prm->q_cut) continue;
      double a = std::min(prm->alpha_max, (double)S->opacity[i] * std::exp(-0.5 * q));
      Tr *= (1 - a);
      if (Tr < prm->eps_T) break;
    }
    ncon[k] = cnt;
  }
}

// --- backward -------------------------------------------------------------
// Gradients of L with respect to every Gaussian parameter, given dL/dC
// ([3][n]) and dL/dT ([n], may be NULL) at the listed pixels.  Accumulates
// into g_mean [3][P], g_scale [3][P], g_rot [4][P], g_opac [P], g_sh [K][3][P].
// Per pixel: reverse compositing gives dL/d alpha_k and dL/dc_k; alpha depends
// on (o, conic, omega, phi); the offset's derivative in (omega, phi) and all
// derivatives of the preprocessing come from dual numbers.
void or_render_bwd(const or_scene* S, const or_view* V, const or_params* prm, const int* valid, const double* omega,
                   const double* phi, const double* rho, const double* conic, const double* rs, const double* rgbg,
                   i64 n, const i64* pix, const double* dLdC, const double* dLdT, double* g_mean, double* g_scale,
                   double* g_rot, double* g_opac, double* g_sh, const double* dLdD, double* g_ang) {
  i64 P = S->P;
  int K = (S->sh_degree + 1) * (S->sh_degree + 1);
  // per-Gaussian gradients of the projected quantities
  // [0] omega [1] phi [2] A [3] B [4] C [5] opacity [6..8] rgb [9] 1/rho
  const int NG = 10;
  std::vector<double> gy((size_t)P * NG, 0.0);
  int nth = or_num_threads();
  std::vector<std::vector<double>> gyt(nth);
#pragma omp parallel
  {
    int tid = 0;
#ifdef _OPENMP
    tid = omp_get_thread_num();
#endif
    std::vector<double>& acc = gyt[tid];
    acc.assign((size_t)P * NG, 0.0);
#pragma omp for schedule(dynamic, 16)
    for (i64 k = 0; k < n; ++k) {
      double om_p, ph_p, pv[3];
      pix_angles(V->order, pix[k], &om_p, &ph_p, pv);
      std::vector<Cand> c;
      const double no_band[3] = {0.0, 0.0, 0.0};
      pixel_candidates(*S, *prm, valid, omega, phi, rho, conic, rs, om_p, ph_p, pv, no_band, c);
      // forward sequence
      std::vector<i64> ids; std::vector<double> al, Ts, qs; std::vector<bool> clampa;
      double Tr = 1.0;
      for (const Cand& e : c) {
        if (e.q > prm->q_cut) continue;
        double a0 = (double)S->opacity[e.i] * std::exp(-0.5 * e.q);
        bool cl = a0 > prm->alpha_max;
        double a = cl ? prm->alpha_max : a0;
        ids.push_back(e.i); al.push_back(a); Ts.push_back(Tr); qs.push_back(e.q); clampa.push_back(cl);
        Tr *= (1 - a);
        if (Tr < prm->eps_T) break;
      }
      double Tfin = Tr;
      double gT = dLdT ? dLdT[k] : 0.0;
      double gC[3] = {dLdC[k], dLdC[n + k], dLdC[2 * n + k]};
      double gD = dLdD ? dLdD[k] : 0.0;
      double behind[3] = {0, 0, 0};  // colour accumulated behind entry j
      double behindD = 0;            // inverse depth accumulated behind entry j
      for (i64 j = (i64)ids.size() - 1; j >= 0; --j) {
        i64 i = ids[j];
        double a = al[j], Tj = Ts[j];
        double ci[3] = {rgbg[i], rgbg[P + i], rgbg[2 * P + i]};
        double dLda = 0;
        for (int ch = 0; ch < 3; ++ch) {
          acc[(size_t)i * NG + 6 + ch] += gC[ch] * a * Tj;
          dLda += gC[ch] * (Tj * ci[ch] - behind[ch] / (1 - a));
        }
        dLda += gT * (-Tfin / (1 - a));
        for (int ch = 0; ch < 3; ++ch) behind[ch] += Tj * a * ci[ch];
        if (gD != 0.0) {
          double ir = 1.0 / rho[i];
          acc[(size_t)i * NG + 9] += gD * a * Tj;
          dLda += gD * (Tj * ir - behindD / (1 - a));
          behindD += Tj * a * ir;
        }
        if (clampa[j]) continue;
        double o = S->opacity[i];
        double G = std::exp(-0.5 * qs[j]);
        acc[(size_t)i * NG + 5] += dLda * G;
        double dLdq = dLda * (-0.5 * o * G);
        // q = A dx^2 + 2 B dx dy + C dy^2 ; d = offset(omega_i, phi_i)
        double A = conic[i], B = conic[P + i], Cc = conic[2 * P + i];
        double dx, dy, dg;
        sph_offset<double>(omega[i], phi[i], om_p, ph_p, &dx, &dy, &dg);
        acc[(size_t)i * NG + 2] += dLdq * dx * dx;
        acc[(size_t)i * NG + 3] += dLdq * 2 * dx * dy;
        acc[(size_t)i * NG + 4] += dLdq * dy * dy;
        for (int dir = 0; dir < 2; ++dir) {
          Dual om(omega[i], dir == 0 ? 1.0 : 0.0), ph(phi[i], dir == 1 ? 1.0 : 0.0);
          Dual ddx, ddy, ddg;
          sph_offset<Dual>(om, ph, om_p, ph_p, &ddx, &ddy, &ddg);
          double dq = 2 * (A * dx + B * dy) * ddx.d + 2 * (B * dx + Cc * dy) * ddy.d;
          acc[(size_t)i * NG + dir] += dLdq * dq;
        }
      }
    }
  }
  for (int t = 0; t < nth; ++t)
    if (!gyt[t].empty())
      for (size_t j = 0; j < gy.size(); ++j) gy[j] += gyt[t][j];
  // chain through the preprocessing
#pragma omp parallel for schedule(dynamic, 64)
  for (i64 i = 0; i < P; ++i) {
    const double* g = &gy[(size_t)i * NG];
    if (g_ang) { g_ang[i] += g[0]; g_ang[P + i] += g[1]; }
    bool any = false;
    for (int j = 0; j < NG; ++j) any = any || g[j] != 0.0;
    if (!any || !valid[i]) continue;
    double mu[3], s[3], q[4];
    std::vector<double> shc;
    scene_gauss(*S, i, mu, s, q, shc);
    g_opac[i] += g[5];
    // SH coefficients: colour is linear in them (zero where clamped)
    {
      ProjT<double> o = preprocess_one<double>(mu, s, q, shc.data(), S->sh_degree, *V, *prm);
      double v[3] = {mu[0] - V->center[0], mu[1] - V->center[1], mu[2] - V->center[2]};
      double vn = std::sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
      double Y[16];
      sh_basis<double>(S->sh_degree, v[0] / vn, v[1] / vn, v[2] / vn, Y);
      for (int ch = 0; ch < 3; ++ch) {
        if (o.clamped[ch]) continue;
        for (int kk = 0; kk < K; ++kk) g_sh[((size_t)kk * 3 + ch) * P + i] += g[6 + ch] * Y[kk];
      }
    }
    // geometry: 10 tangent directions (mean 3, scale 3, rot 4)
    for (int dir = 0; dir < 10; ++dir) {
      Dual dm[3], ds[3], dq[4];
      for (int k = 0; k < 3; ++k) { dm[k] = Dual(mu[k], dir == k ? 1.0 : 0.0); ds[k] = Dual(s[k], dir == 3 + k ? 1.0 : 0.0); }
      for (int k = 0; k < 4; ++k) dq[k] = Dual(q[k], dir == 6 + k ? 1.0 : 0.0);
      ProjT<Dual> o = preprocess_one<Dual>(dm, ds, dq, shc.data(), S->sh_degree, *V, *prm);
      double d = g[0] * o.omega.d + g[1] * o.phi.d + g[2] * o.A.d + g[3] * o.B.d + g[4] * o.C.d;
      for (int ch = 0; ch < 3; ++ch) d += g[6 + ch] * o.rgb[ch].d;
      d += g[9] * (-o.rho.d / (o.rho.v * o.rho.v));  // d(1/rho) = -d rho / rho^2
      if (dir < 3) g_mean[dir * P + i] += d;
      else if (dir < 6) g_scale[(dir - 3) * P + i] += d;
      else g_rot[(dir - 6) * P + i] += d;
    }
  }
}

// --- HEALPix-SSIM and the training loss (Sec. 4.1; supp. HSSIM metric) ---
// Zone-specific windows (Sec. 4.1: isotropic in the equatorial zone where the
// pixels are roughly square, anisotropic in the polar zones where they are
// compressed along the rings).  Reading: a pixel of the equatorial belt
// (ring jr in [N, 3N], |z| <= 2/3) keeps the isotropic window of face-local
// offsets, exp(-(a^2 + b^2) / (2 sigma^2)); a pixel of a polar cap (jr < N or
// jr > 3N) weighs each chart neighbour q by its great-circle distance d,
// exp(-d^2 / (2 sigma^2 Omega)) with Omega = 4 pi / Npix the pixel area, which
// is the same Gaussian of width sigma pitches measured on the sphere instead
// of in chart steps.  In (a, b) it is anisotropic and not separable.
static bool polar_pixel(int order, i64 p) {
  const i64 N = (i64)1 << order;
  const RingPos r = xyf2ringpos(order, nest2xyf(order, p));
  return r.jr < N || r.jr > 3 * N;
}

static double great_circle(const double u[3], const double v[3]) {
  const double c[3] = {u[1] * v[2] - u[2] * v[1], u[2] * v[0] - u[0] * v[2], u[0] * v[1] - u[1] * v[0]};
  return std::atan2(std::sqrt(c[0] * c[0] + c[1] * c[1] + c[2] * c[2]), u[0] * v[0] + u[1] * v[1] + u[2] * v[2]);
}

// Raw window weights of nested pixel p over its 11 x 11 chart neighbourhood
// (index (a + 5) * 11 + (b + 5) for offsets (a, b)); nbq receives the
// neighbour's nested id or -1 in the missing quadrant (weight 0 there).
static void hssim_window(int order, i64 p, double sigma, int zones, i64* nbq, double* w) {
  const int R = 5, Wd = 11;
  const XYF a = nest2xyf(order, p);
  const bool polar = zones && polar_pixel(order, p);
  double up[3];
  if (polar) pix_vec(order, p, up);
  const double omega = 4.0 * M_PI / (double)(12 * ((i64)1 << (2 * order)));
  for (int da = -R; da <= R; ++da)
    for (int db = -R; db <= R; ++db) {
      const int j = (da + R) * Wd + (db + R);
      const i64 q = chart_pixel(order, a.f, a.x + da, a.y + db);
      nbq[j] = q;
      if (q < 0) { w[j] = 0.0; continue; }
      if (polar) {
        double uq[3];
        pix_vec(order, q, uq);
        const double d = great_circle(up, uq);
        w[j] = std::exp(-d * d / (2.0 * sigma * sigma * omega));
      } else {
        w[j] = std::exp(-(double)(da * da + db * db) / (2.0 * sigma * sigma));
      }
    }
}

// The raw window of one pixel (for the pins of the zone reading).
void or_hssim_window(int order, i64 p, double sigma, int zones, i64* nbq, double* w) {
  hssim_window(order, p, sigma, zones, nbq, w);
}

// img, ref: [3][n] over the active pixels; active: sorted nested ids.  Window
// 11x11 (offsets -5..5) on the face-extended chart with the raw weights of
// hssim_window (zones = 0: the isotropic chart window everywhere);
// neighbours that are missing or inactive get weight 0 and the rest are
// renormalised.  Returns mean SSIM over pixels and channels; ssim_map [3][n]
// optional.  With grad != NULL also writes d(mean SSIM)/d img  ([3][n]).
double or_hssim(int order, i64 n, const i64* active, const double* img, const double* ref, double sigma, double C1,
                double C2, int zones, double* ssim_map, double* grad) {
  i64 npix = 12 * ((i64)1 << (2 * order));
  std::vector<i64> idx(npix, -1);
  for (i64 k = 0; k < n; ++k) idx[active[k]] = k;
  const int Wd = 11;
  // neighbour lists (active slots) of every pixel
  std::vector<i64> nb((size_t)n * Wd * Wd);
#pragma omp parallel for schedule(static)
  for (i64 k = 0; k < n; ++k) {
    i64 q[Wd * Wd];
    double w[Wd * Wd];
    hssim_window(order, active[k], sigma, 0, q, w);
    for (int j = 0; j < Wd * Wd; ++j) nb[(size_t)k * Wd * Wd + j] = q[j] >= 0 ? idx[q[j]] : -1;
  }
  double total = 0;
  // per pixel/channel partials of SSIM w.r.t. the three x-dependent sums
  std::vector<double> G1(grad ? 3 * n : 0), G2(grad ? 3 * n : 0), G12(grad ? 3 * n : 0);
#pragma omp parallel for schedule(static) reduction(+ : total)
  for (i64 k = 0; k < n; ++k) {
    const i64* nbk = &nb[(size_t)k * Wd * Wd];
    i64 qk[Wd * Wd];
    double wr[Wd * Wd];
    hssim_window(order, active[k], sigma, zones, qk, wr);
    double Z = 0;
    for (int j = 0; j < Wd * Wd; ++j) if (nbk[j] >= 0) Z += wr[j];
    for (int ch = 0; ch < 3; ++ch) {
      double sx = 0, sy = 0, sxx = 0, syy = 0, sxy = 0;
      for (int j = 0; j < Wd * Wd; ++j) {
        i64 q = nbk[j];
        if (q < 0) continue;
        double w = wr[j] / Z, x = img[ch * n + q], y = ref[ch * n + q];
        sx += w * x; sy += w * y; sxx += w * x * x; syy += w * y * y; sxy += w * x * y;
      }
      double vx = sxx - sx * sx, vy = syy - sy * sy, cxy = sxy - sx * sy;
      double Anum = 2 * sx * sy + C1, Bnum = 2 * cxy + C2;
      double Aden = sx * sx + sy * sy + C1, Bden = vx + vy + C2;
      double s = Anum * Bnum / (Aden * Bden);
      if (ssim_map) ssim_map[ch * n + k] = s;
      total += s;
      if (grad) {
        // s as a function of (sx, sxx, sxy) with y-sums fixed
        double dA_dsx = 2 * sy, dB_dsx = -2 * sy;         // via cxy = sxy - sx sy
        double dAd_dsx = 2 * sx, dBd_dsx = -2 * sx;       // via vx = sxx - sx^2
        double ds_dsx = (dA_dsx * Bnum + Anum * dB_dsx) / (Aden * Bden) - s * (dAd_dsx / Aden + dBd_dsx / Bden);
        double ds_dsxx = -s / Bden;
        double ds_dsxy = Anum * 2 / (Aden * Bden);
        G1[ch * n + k] = ds_dsx / Z;
        G2[ch * n + k] = ds_dsxx / Z;
        G12[ch * n + k] = ds_dsxy / Z;
      }
    }
  }
  double mean = total / (3.0 * (double)n);
  if (grad) {
    // d mean / d x_p = (1/3n) sum_{q : p in W(q)} wraw(q,p)/Z_q (G1_q + 2 x_p G2_q + y_p G12_q)
    std::fill(grad, grad + 3 * n, 0.0);
    for (i64 k = 0; k < n; ++k) {
      const i64* nbk = &nb[(size_t)k * Wd * Wd];
      i64 qk[Wd * Wd];
      double wr[Wd * Wd];
      hssim_window(order, active[k], sigma, zones, qk, wr);
      for (int j = 0; j < Wd * Wd; ++j) {
        i64 p = nbk[j];
        if (p < 0) continue;
        for (int ch = 0; ch < 3; ++ch) {
          double x = img[ch * n + p], y = ref[ch * n + p];
          grad[ch * n + p] += wr[j] * (G1[ch * n + k] + 2 * x * G2[ch * n + k] + y * G12[ch * n + k]) / (3.0 * (double)n);
        }
      }
    }
  }
  return mean;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Image synthesis between the HEALPix grid and camera images (Eq.
// camera_synthesis, Interp_H; supp. "Preprocessing of Omnidirectional
// Images" for the camera mappings; supp. Eq. supp_image_to_healpix for the
// reverse direction).
//
// Readings where the paper is silent or at odds with itself:
//  * One camera frame for all models, y up: the pinhole and fisheye formulas
//    measure image v downwards, the panorama formula looks up at v = 0, so
//    v is flipped in the first two (the optical axis is +z, +x is right).
//  * Pixel (i, j) of a W x H image has its centre at (u, v) = (i + 1/2, j + 1/2).
//  * Interp_H is bilinear over the ring structure: the two rings enclosing
//    the colatitude, in each ring the two pixels enclosing the longitude,
//    linear in longitude within a ring and linear in colatitude between the
//    rings.  Above the first ring (below the last) the pole is taken as the
//    mean of that ring's four pixels.  Neighbours outside the active set get
//    weight zero and the remaining weights are renormalised; a camera pixel
//    with no active neighbour (or outside the camera's valid domain) is 0.
//  * Image to sphere: bilinear in the image at the projected position of
//    the pixel centre, clamped to the border (wrapping in longitude for the
//    panorama).
// ---------------------------------------------------------------------------
static void cam_focal(int cam, int W, int H, double fovx, double fovy, double* fx, double* fy) {
  if (cam == CAM_PINHOLE) {
    *fx = W / (2.0 * std::tan(0.5 * fovx));
    *fy = H / (2.0 * std::tan(0.5 * fovy));
  } else {  // fisheye: valid ellipse tangent to the image border
    *fx = W / M_PI;
    *fy = H / M_PI;
  }
}

// Ray through image position (u, v), camera frame; false outside the domain.
static bool cam_ray(int cam, int W, int H, double fovx, double fovy, double u, double v, double d[3]) {
  if (cam == CAM_FULL) {  // equirectangular panorama
    double om = 2.0 * M_PI * u / W - M_PI, ph = 0.5 * M_PI - M_PI * v / H;
    d[0] = std::cos(ph) * std::sin(om);
    d[1] = std::sin(ph);
    d[2] = std::cos(ph) * std::cos(om);
    return true;
  }
  double fx, fy;
  cam_focal(cam, W, H, fovx, fovy, &fx, &fy);
  double mx = (u - 0.5 * W) / fx, my = -(v - 0.5 * H) / fy;
  if (cam == CAM_PINHOLE) {
    double n = std::sqrt(mx * mx + my * my + 1.0);
    d[0] = mx / n; d[1] = my / n; d[2] = 1.0 / n;
    return true;
  }
  // anisotropic equidistant fisheye: psi = r_m w_eff(gamma), w = FoV / pi
  double rm = std::sqrt(mx * mx + my * my);
  double gam = std::atan2(my, mx);
  double wx = fovx / M_PI, wy = fovy / M_PI;
  double weff = std::sqrt(wx * std::cos(gam) * wx * std::cos(gam) + wy * std::sin(gam) * wy * std::sin(gam));
  double psi = rm * weff;
  d[0] = std::sin(psi) * std::cos(gam);
  d[1] = std::sin(psi) * std::sin(gam);
  d[2] = std::cos(psi);
  return rm <= 0.5 * M_PI;
}

// Image position of direction d (inverse of cam_ray); false outside the domain.
static bool cam_project(int cam, int W, int H, double fovx, double fovy, const double d[3], double* u, double* v) {
  if (cam == CAM_FULL) {
    double om = std::atan2(d[0], d[2]);
    double ph = std::asin(std::max(-1.0, std::min(1.0, d[1])));
    *u = (om + M_PI) * W / (2.0 * M_PI);
    *v = (0.5 * M_PI - ph) * H / M_PI;
    return true;
  }
  double fx, fy;
  cam_focal(cam, W, H, fovx, fovy, &fx, &fy);
  if (cam == CAM_PINHOLE) {
    if (!(d[2] > 0)) return false;
    double mx = d[0] / d[2], my = d[1] / d[2];
    *u = 0.5 * W + fx * mx;
    *v = 0.5 * H - fy * my;
    return *u >= 0 && *u <= W && *v >= 0 && *v <= H;
  }
  double psi = std::acos(std::max(-1.0, std::min(1.0, d[2])));
  double gam = std::atan2(d[1], d[0]);
  double wx = fovx / M_PI, wy = fovy / M_PI;
  double weff = std::sqrt(wx * std::cos(gam) * wx * std::cos(gam) + wy * std::sin(gam) * wy * std::sin(gam));
  double rm = psi / weff;
  *u = 0.5 * W + fx * rm * std::cos(gam);
  *v = 0.5 * H - fy * rm * std::sin(gam);
  return rm <= 0.5 * M_PI;
}

// z of ring i (1 .. 4N-1) and its colatitude, from the ring definitions.
static double ring_z(i64 N, i64 i) {
  if (i < N) return 1.0 - (double)(i * i) / (3.0 * (double)(N * N));
  if (i > 3 * N) return -(1.0 - (double)((4 * N - i) * (4 * N - i)) / (3.0 * (double)(N * N)));
  return (double)(2 * N - i) * 2.0 / (3.0 * (double)N);
}
static double ring_theta(i64 N, i64 i) {
  // polar caps: 1 - |z| = 2 sin^2(theta/2), so theta = 2 asin(i / (N sqrt 6)) without cancellation
  if (i < N) return 2.0 * std::asin((double)i / ((double)N * std::sqrt(6.0)));
  if (i > 3 * N) return M_PI - 2.0 * std::asin((double)(4 * N - i) / ((double)N * std::sqrt(6.0)));
  return std::acos(ring_z(N, i));
}
// pixels in ring i, RING index of its first pixel, longitude offset (in pixels) of pixel 0's centre
static void ring_info(i64 N, i64 i, i64* n, i64* first, double* off) {
  if (i < N) { *n = 4 * i; *first = 2 * i * (i - 1); *off = 0.5; }
  else if (i > 3 * N) { i64 s = 4 * N - i; *n = 4 * s; *first = 12 * N * N - 2 * s * (s + 1); *off = 0.5; }
  else { *n = 4 * N; *first = 2 * N * (N - 1) + (i - N) * 4 * N; *off = ((i - N) & 1) ? 0.0 : 0.5; }
}

// The four RING-scheme pixels and weights of Interp_H at camera-frame direction d.
static void interp_ring(int order, const double d[3], i64 pix[4], double w[4]) {
  i64 N = (i64)1 << order;
  // HEALPix frame (x_h, y_h, z_h) = (d_z, d_x, d_y)
  double xh = d[2], yh = d[0], zh = d[1];
  double theta = std::atan2(std::sqrt(xh * xh + yh * yh), zh);
  double phi = std::atan2(yh, xh);
  if (phi < 0) phi += 2.0 * M_PI;
  // ring above: the last ring whose colatitude is <= theta (0 = north pole)
  i64 lo = 0, hi = 4 * N;  // ring_theta(lo) <= theta < ring_theta(hi), pole rings at 0 and 4N
  while (hi - lo > 1) {
    i64 mid = (lo + hi) / 2;
    if (ring_theta(N, mid) <= theta) lo = mid; else hi = mid;
  }
  i64 i1 = lo, i2 = lo + 1;
  auto pair = [&](i64 i, i64* a, i64* b, double* wb) {
    i64 n, first; double off;
    ring_info(N, i, &n, &first, &off);
    double t = phi / (2.0 * M_PI / (double)n) - off;
    double j1 = std::floor(t);
    *wb = t - j1;
    i64 ja = ((i64)j1 % n + n) % n, jb = (ja + 1) % n;
    *a = first + ja; *b = first + jb;
  };
  if (i1 >= 1 && i2 <= 4 * N - 1) {
    double t1 = ring_theta(N, i1), t2 = ring_theta(N, i2);
    double wt = (theta - t1) / (t2 - t1);
    double f1, f2;
    pair(i1, &pix[0], &pix[1], &f1);
    pair(i2, &pix[2], &pix[3], &f2);
    w[0] = (1 - wt) * (1 - f1); w[1] = (1 - wt) * f1;
    w[2] = wt * (1 - f2); w[3] = wt * f2;
    return;
  }
  // polar cap: between the pole (mean of the four pixels of the nearest
  // ring) and that ring
  i64 ir = (i1 == 0) ? 1 : 4 * N - 1;
  double tr = ring_theta(N, ir);
  double wr = (i1 == 0) ? theta / tr : (M_PI - theta) / (M_PI - tr);  // weight of the ring pair
  i64 n, first; double off;
  ring_info(N, ir, &n, &first, &off);
  i64 a, b; double f;
  pair(ir, &a, &b, &f);
  for (int k = 0; k < 4; ++k) { pix[k] = first + k; w[k] = 0.25 * (1 - wr); }
  w[a - first] += wr * (1 - f);
  w[b - first] += wr * f;
}

// slot of nested pixel q in the sorted active list, or -1
static i64 active_slot(i64 n_active, const i64* active, i64 q) {
  const i64* it = std::lower_bound(active, active + n_active, q);
  return (it != active + n_active && *it == q) ? (i64)(it - active) : -1;
}

extern "C" {

void or_cam_rays(int cam, int W, int H, double fovx, double fovy, i64 n, const double* uv, double* d, int* valid) {
  for (i64 k = 0; k < n; ++k) valid[k] = cam_ray(cam, W, H, fovx, fovy, uv[2 * k], uv[2 * k + 1], d + 3 * k) ? 1 : 0;
}

void or_cam_project(int cam, int W, int H, double fovx, double fovy, i64 n, const double* d, double* uv, int* valid) {
  for (i64 k = 0; k < n; ++k)
    valid[k] = cam_project(cam, W, H, fovx, fovy, d + 3 * k, &uv[2 * k], &uv[2 * k + 1]) ? 1 : 0;
}

// Interp_H weights: NESTED pixels [n][4] and weights [n][4] at directions [n][3];
// ring2nest = the NESTED index of every RING index (length 12 N^2).
void or_interp_weights(int order, const i64* ring2nest, i64 n, const double* d, i64* pix, double* w) {
  for (i64 k = 0; k < n; ++k) {
    i64 r[4];
    interp_ring(order, d + 3 * k, r, w + 4 * k);
    for (int m = 0; m < 4; ++m) pix[4 * k + m] = ring2nest[r[m]];
  }
}

// HEALPix image on the active pixels [3][n_active] -> camera image [3][H][W]
// and its valid flags [H][W] (Eq. camera_synthesis).
void or_sphere_to_image(int order, const i64* ring2nest, i64 n_active, const i64* active, const double* img, int cam,
                        int W, int H, double fovx, double fovy, double* out, int* valid) {
  const i64 HW = (i64)W * H;
#pragma omp parallel for schedule(static)
  for (i64 k = 0; k < HW; ++k) {
    const int i = (int)(k % W), j = (int)(k / W);
    double d[3];
    double acc[3] = {0, 0, 0}, ws = 0;
    if (cam_ray(cam, W, H, fovx, fovy, i + 0.5, j + 0.5, d)) {
      i64 r[4]; double w[4];
      interp_ring(order, d, r, w);
      for (int m = 0; m < 4; ++m) {
        i64 s = active_slot(n_active, active, ring2nest[r[m]]);
        if (s < 0) continue;
        for (int c = 0; c < 3; ++c) acc[c] += w[m] * img[c * n_active + s];
        ws += w[m];
      }
    }
    valid[k] = ws > 0 ? 1 : 0;
    for (int c = 0; c < 3; ++c) out[c * HW + k] = ws > 0 ? acc[c] / ws : 0.0;
  }
}

// Camera image [3][H][W] -> samples at the active HEALPix pixels [3][n_active]
// (supp. Eq. supp_image_to_healpix) and their valid flags.
void or_image_to_sphere(int order, i64 n_active, const i64* active, const double* img, int cam, int W, int H,
                        double fovx, double fovy, double* out, int* valid) {
  const i64 HW = (i64)W * H;
#pragma omp parallel for schedule(static)
  for (i64 k = 0; k < n_active; ++k) {
    double t[3], u = 0.5 * W, v = 0.5 * H;
    pix_vec(order, active[k], t);
    bool ok = cam_project(cam, W, H, fovx, fovy, t, &u, &v);
    valid[k] = ok ? 1 : 0;
    // bilinear over pixel centres at half-integers
    double x = u - 0.5, y = v - 0.5;
    double x0 = std::floor(x), y0 = std::floor(y);
    double fx = x - x0, fy = y - y0;
    i64 xs[2] = {(i64)x0, (i64)x0 + 1}, ys[2] = {(i64)y0, (i64)y0 + 1};
    for (int a = 0; a < 2; ++a) {
      if (cam == CAM_FULL) xs[a] = ((xs[a] % W) + W) % W;
      else xs[a] = std::max<i64>(0, std::min<i64>(W - 1, xs[a]));
      ys[a] = std::max<i64>(0, std::min<i64>(H - 1, ys[a]));
    }
    double wgt[4] = {(1 - fx) * (1 - fy), fx * (1 - fy), (1 - fx) * fy, fx * fy};
    for (int c = 0; c < 3; ++c) {
      double s = wgt[0] * img[c * HW + ys[0] * W + xs[0]] + wgt[1] * img[c * HW + ys[0] * W + xs[1]] +
                 wgt[2] * img[c * HW + ys[1] * W + xs[0]] + wgt[3] * img[c * HW + ys[1] * W + xs[1]];
      out[c * n_active + k] = ok ? s : 0.0;
    }
  }
}

}  // extern "C"

// ---------------------------------------------------------------------------
// The paper's tile queries (Sec. 3.3 and the supplementary description of
// stage 2; Alg. 2 NESTED quadtree traversal, Alg. 3 RING sequential scan).
// Both search at the query order kq = kt + log2 f (f = 2^fl, the "x f" search
// depth of the ablation) and report tiles, the ancestors at the tile order kt
// of what they find.  They approximate the tile overlap by tests on centres,
// so a tile set can miss tiles the disc reaches.
// Readings where the listings leave room:
//  * ZtoRingRange keeps the rings whose centre z lies in [z_min, z_max].
//  * RingInfo's omega_0 is the longitude of the centre of the ring's first
//    pixel in RING order, and Ring2Nest(i_r, j) the nested index of the j-th
//    pixel of ring i_r.
//  * The pole threshold epsilon is 1e-12.
//  * Classify: zone 0 when d > r_s + R, 3 when d <= r_s - R, 2 when d <= r_s,
//    else 1, with R = PixRad(o) the largest angle from a node centre at order
//    o to the centre of one of its descendants at the query order (zero at
//    o = kq).  The traversal then prunes exactly the subtrees that hold no
//    query-order centre within r_s, and leaves report centre hits.
//  * A result is restricted to active tiles (a tile without an active pixel
//    is never rendered).
// ---------------------------------------------------------------------------
static double haversine(double om1, double ph1, double om2, double ph2) {
  double a = std::sin(0.5 * (ph2 - ph1)), b = std::sin(0.5 * (om2 - om1));
  double h = a * a + std::cos(ph1) * std::cos(ph2) * b * b;
  return 2.0 * std::asin(std::sqrt(std::min(1.0, std::max(0.0, h))));
}

// PixRad(o) for o = 0 .. kq by enumerating every query-order centre.
static const std::vector<double>& pixrad_table(int kq) {
  static std::vector<std::vector<double>> cache(32);
  std::vector<double>& R = cache[kq];
  if (!R.empty()) return R;
  const i64 nq = 12ll << (2 * kq);
  std::vector<double> vq(3 * nq);
#pragma omp parallel for schedule(static)
  for (i64 p = 0; p < nq; ++p) pix_vec(kq, p, &vq[3 * p]);
  R.assign(kq + 1, 0.0);
  for (int o = 0; o < kq; ++o) {
    const i64 no = 12ll << (2 * o);
    std::vector<double> vo(3 * no);
    for (i64 a = 0; a < no; ++a) pix_vec(o, a, &vo[3 * a]);
    double m = 0;
#pragma omp parallel for schedule(static) reduction(max : m)
    for (i64 p = 0; p < nq; ++p) m = std::max(m, angle_between(&vo[3 * (p >> (2 * (kq - o)))], &vq[3 * p]));
    R[o] = m;
  }
  return R;
}

// Alg. 2: depth-first search from the 12 base pixels with an explicit stack.
static void query_nested(int kt, int kq, const std::vector<double>& R, double om, double ph, double rs,
                         std::vector<i64>& T) {
  std::vector<std::pair<i64, int>> stack;
  for (i64 p = 11; p >= 0; --p) stack.push_back({p, 0});
  while (!stack.empty()) {
    const i64 p = stack.back().first;
    const int o = stack.back().second;
    stack.pop_back();
    double omn, phn, v[3];
    pix_angles(o, p, &omn, &phn, v);
    const double d = haversine(om, ph, omn, phn);
    const int zone = d > rs + R[o] ? 0 : (d <= rs - R[o] ? 3 : (d <= rs ? 2 : 1));
    if (zone == 0) continue;
    if (zone >= 2 && o >= kt) T.push_back(p >> (2 * (o - kt)));
    else if (o < kq) for (int c = 3; c >= 0; --c) stack.push_back({4 * p + c, o + 1});
    else T.push_back(p >> (2 * (o - kt)));
  }
}

// Alg. 3: the rings of the disc's z range, and on each the pixels whose
// centres fall in the longitude window of Eq. ring_phi_range (its end pixels
// included by the floor / ceil).
static void query_ring(int kt, int kq, const i64* r2n, double om, double ph, double rs, std::vector<i64>& T) {
  const i64 N = (i64)1 << kq;
  const double zc = std::sin(ph);
  const double phmin = std::max(-0.5 * M_PI, ph - rs), phmax = std::min(0.5 * M_PI, ph + rs);
  const double zmin = std::sin(phmin), zmax = std::sin(phmax);
  const double crs = std::cos(rs);
  const int sh = 2 * (kq - kt);
  for (i64 ir = 1; ir <= 4 * N - 1; ++ir) {
    const double zr = ring_z(N, ir);
    if (zr < zmin || zr > zmax) continue;
    i64 nr, first;
    double off;
    ring_info(N, ir, &nr, &first, &off);
    const double om0 = off * 2.0 * M_PI / (double)nr;
    const double delta = std::sqrt(std::max(0.0, 1 - zc * zc)) * std::sqrt(std::max(0.0, 1 - zr * zr));
    if (delta < 1e-12) {
      if (zc * zr >= crs)
        for (i64 j = 0; j < nr; ++j) T.push_back(r2n[first + j] >> sh);
      continue;
    }
    const double cw = (crs - zc * zr) / delta;
    if (cw <= -1) {
      for (i64 j = 0; j < nr; ++j) T.push_back(r2n[first + j] >> sh);
    } else if (cw < 1) {
      const double dw = std::acos(std::min(1.0, std::max(-1.0, cw)));
      const i64 lo = (i64)std::floor((om - dw - om0) * (double)nr / (2.0 * M_PI));
      const i64 hi = (i64)std::ceil((om + dw - om0) * (double)nr / (2.0 * M_PI));
      for (i64 ip = lo; ip <= hi; ++ip) T.push_back(r2n[first + (((ip % nr) + nr) % nr)] >> sh);
    }
  }
}

extern "C" {

// Tile sets of the paper's queries: mode 1 = RING scan (Alg. 3), 2 = NESTED
// traversal (Alg. 2), at query order kt + fl.  Gaussian i (valid ones among
// gids) is queried with radius max(0, rs_i (1 + drs_rel) + drs_abs); the
// widened and narrowed radii bracket a float32 evaluation of the same query
// (the result only grows with the radius).  ring2nest: the RING -> NESTED
// table at the query order (RING mode).  Pairs come Gaussian by Gaussian,
// tiles ascending; returns their number (written only while below cap).
i64 or_query_tiles(int mode, int kt, int fl, const i64* ring2nest, const unsigned char* tile_active, i64 n_g,
                   const i64* gids, const int* valid, const double* omega, const double* phi, const double* rs,
                   double drs_rel, double drs_abs, i64 cap, i64* out_gid, i64* out_tile) {
  const int kq = kt + fl;
  static const std::vector<double> none;
  const std::vector<double>& R = mode == 2 ? pixrad_table(kq) : none;
  std::vector<std::vector<i64>> res(n_g);
#pragma omp parallel for schedule(dynamic, 16)
  for (i64 k = 0; k < n_g; ++k) {
    const i64 i = gids[k];
    if (!valid[i]) continue;
    const double r = std::max(0.0, rs[i] * (1 + drs_rel) + drs_abs);
    std::vector<i64> T;
    if (mode == 1) query_ring(kt, kq, ring2nest, omega[i], phi[i], r, T);
    else query_nested(kt, kq, R, omega[i], phi[i], r, T);
    std::sort(T.begin(), T.end());
    T.erase(std::unique(T.begin(), T.end()), T.end());
    for (i64 t : T)
      if (tile_active[t]) res[k].push_back(t);
  }
  i64 n = 0;
  for (i64 k = 0; k < n_g; ++k)
    for (i64 t : res[k]) {
      if (out_gid && n < cap) { out_gid[n] = gids[k]; out_tile[n] = t; }
      ++n;
    }
  return n;
}

// PixRad(o), o = 0 .. kq (as used by the NESTED query).
void or_pixrad(int kq, double* out) {
  const std::vector<double>& R = pixrad_table(kq);
  for (int o = 0; o <= kq; ++o) out[o] = R[o];
}

}  // extern "C"
