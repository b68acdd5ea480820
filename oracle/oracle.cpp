// FP64 reference tracer -- TEST INFRASTRUCTURE ONLY.
//
// This file is the oracle against which the HIP library is checked.  Only the
// test suite, the smoke check and the CPU-baseline leg of the benchmark may
// load it; the library never does.  It shares no code, header or table with
// the library: it reads the same scene descriptors and photon bundles (built
// by the `scenes` input module) and computes, photon by photon, what the
// paper states (§2.1): a photon (position + momentum direction) is carried
// through a scene of volumes with no fixed surface order; at each step the
// nearest surface among *all* faces of *all* volumes is found by brute force,
// and the volume's role (lens, mirror, focal surface, obscuration) decides
// what happens (reflection, refraction, detection, absorption).
//
// The paper prints no formulas; the physics is textbook and the readings are:
//   * mirrors reflect specularly on the front, absorb on the back; a mirror
//     of reflectivity R absorbs iff a 32-bit draw u >= floor(R 2^32);
//   * lenses: unpolarised Fresnel reflectance R = (Rs + Rp)/2, reflect iff
//     (u >> 8) 2^-24 < R, else vector Snell refraction, total internal
//     reflection when no refracted ray exists;
//   * focal surfaces detect on the front (FOCUSED), absorb on the back;
//   * obscurations absorb.
// Random draws: Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11), key =
// seed, counter = (photon id lo, hi, event >> 2, tag 1), word = event & 3.
//
// Shapes (§2.2): plane, sphere cap (sag form), even asphere (the ray-sag
// equation is a degree-16 polynomial in t; all real roots in the aperture
// are isolated by Lipschitz-bounded subdivision), finite cylinder, box, and
// the hexagonal cone whose wall profile is a cubic Bezier curve (the ray-wall
// equation is a cubic in the curve parameter; roots isolated between the
// critical points).  Every root is enumerated; nothing is culled except by
// conservative bounding spheres, which cannot change the result.
#include <cmath>
#include <cstdint>
#include <cstring>
#include <algorithm>
#include <limits>
#include <thread>
#include <vector>

namespace {

enum { ROLE_MIRROR = 1, ROLE_LENS = 2, ROLE_FOCAL = 3, ROLE_OBSCURATION = 4 };
enum { SH_PLANE = 1, SH_SPHERE = 2, SH_ASPHERE = 3, SH_CYLINDER = 4, SH_BOX = 5, SH_HEXCONE = 6 };
enum { OL_NONE = 0, OL_DISC = 1, OL_ANNULUS = 2, OL_RECT = 3, OL_HEX = 4, OL_SECTOR = 5 };
enum { F_FOCUSED = 1, F_ABSORBED = 2, F_EXITED = 3, F_SUSPENDED = 4, F_FAILED = 5 };
enum { ACT_REFLECT = 0, ACT_REFRACT = 1, ACT_STOP = 2 };

constexpr int NI = 5;    // ints per volume
constexpr int ND = 55;   // doubles per volume
constexpr double PI = 3.14159265358979323846;

struct Vol {
  int role, shape, outline, sparam, tparam;
  double Q[9], c[3], p[16], o[4], refl, n_in;
  double Q0[9], c0[3], piv[3], e1[3], e2[3];
  // derived, oracle-side: bounding sphere (world)
  double bc[3], br;
};

// ------------------------------------------------------------------ Philox
void philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4]) {
  uint32_t c[4] = {ctr_in[0], ctr_in[1], ctr_in[2], ctr_in[3]};
  uint32_t k0 = key_in[0], k1 = key_in[1];
  for (int r = 0; r < 10; ++r) {
    if (r > 0) { k0 += 0x9E3779B9u; k1 += 0xBB67AE85u; }
    uint64_t p0 = (uint64_t)0xD2511F53u * c[0];
    uint64_t p1 = (uint64_t)0xCD9E8D57u * c[2];
    uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    uint32_t n0 = hi1 ^ c[1] ^ k0, n1 = lo1, n2 = hi0 ^ c[3] ^ k1, n3 = lo0;
    c[0] = n0; c[1] = n1; c[2] = n2; c[3] = n3;
  }
  for (int i = 0; i < 4; ++i) out[i] = c[i];
}

// Word event & 3 of the block with counter (id lo, id hi, event >> 2, tag):
// tag 1 for the draw of an interaction (mirror absorption, Fresnel
// reflection), tag 2 for bulk absorption in a lens.
uint32_t draw(uint64_t seed, uint64_t id, int event, uint32_t tag = 1u) {
  uint32_t ctr[4] = {(uint32_t)id, (uint32_t)(id >> 32), (uint32_t)(event >> 2), tag};
  uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
  uint32_t out[4];
  philox4x32_10(ctr, key, out);
  return out[event & 3];
}

// ------------------------------------------------------------------ small algebra
template <class T> struct V3 { T x, y, z; };
template <class T> V3<T> mk(T a, T b, T c) { return V3<T>{a, b, c}; }
template <class T> V3<T> operator+(V3<T> a, V3<T> b) { return {a.x + b.x, a.y + b.y, a.z + b.z}; }
template <class T> V3<T> operator-(V3<T> a, V3<T> b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
template <class T, class S> V3<T> operator*(S s, V3<T> a) { return {a.x * s, a.y * s, a.z * s}; }
template <class T> T dot(V3<T> a, V3<T> b) { return a.x * b.x + a.y * b.y + a.z * b.z; }

// dual numbers (forward mode) with a fixed number of tangent components
constexpr int NDUAL = 8;
struct Dual {
  double v; double d[NDUAL];
  Dual() : v(0) { for (int i = 0; i < NDUAL; ++i) d[i] = 0; }
  Dual(double x) : v(x) { for (int i = 0; i < NDUAL; ++i) d[i] = 0; }
};
inline Dual operator+(const Dual& a, const Dual& b) { Dual r(a.v + b.v); for (int i = 0; i < NDUAL; ++i) r.d[i] = a.d[i] + b.d[i]; return r; }
inline Dual operator-(const Dual& a, const Dual& b) { Dual r(a.v - b.v); for (int i = 0; i < NDUAL; ++i) r.d[i] = a.d[i] - b.d[i]; return r; }
inline Dual operator-(const Dual& a) { Dual r(-a.v); for (int i = 0; i < NDUAL; ++i) r.d[i] = -a.d[i]; return r; }
inline Dual operator*(const Dual& a, const Dual& b) { Dual r(a.v * b.v); for (int i = 0; i < NDUAL; ++i) r.d[i] = a.d[i] * b.v + a.v * b.d[i]; return r; }
inline Dual operator/(const Dual& a, const Dual& b) { Dual r(a.v / b.v); for (int i = 0; i < NDUAL; ++i) r.d[i] = (a.d[i] * b.v - a.v * b.d[i]) / (b.v * b.v); return r; }
inline Dual operator+(const Dual& a, double b) { Dual r = a; r.v += b; return r; }
inline Dual operator+(double b, const Dual& a) { return a + b; }
inline Dual operator-(const Dual& a, double b) { Dual r = a; r.v -= b; return r; }
inline Dual operator-(double b, const Dual& a) { return Dual(b) - a; }
inline Dual operator*(const Dual& a, double b) { Dual r(a.v * b); for (int i = 0; i < NDUAL; ++i) r.d[i] = a.d[i] * b; return r; }
inline Dual operator*(double b, const Dual& a) { return a * b; }
inline Dual operator/(const Dual& a, double b) { return a * (1.0 / b); }
inline Dual operator/(double a, const Dual& b) { return Dual(a) / b; }
inline Dual sqrt(const Dual& a) { double s = std::sqrt(a.v); Dual r(s); for (int i = 0; i < NDUAL; ++i) r.d[i] = a.d[i] / (2.0 * s); return r; }
inline Dual sin(const Dual& a) { Dual r(std::sin(a.v)); double c = std::cos(a.v); for (int i = 0; i < NDUAL; ++i) r.d[i] = a.d[i] * c; return r; }
inline Dual cos(const Dual& a) { Dual r(std::cos(a.v)); double s = -std::sin(a.v); for (int i = 0; i < NDUAL; ++i) r.d[i] = a.d[i] * s; return r; }
inline double val(double x) { return x; }
inline double val(const Dual& x) { return x.v; }
using std::sqrt; using std::sin; using std::cos;

// ------------------------------------------------------------------ geometry of a volume
// Effective geometry with type T: frame and shape parameters.
template <class T> struct Geo {
  T Q[9], c[3], p[16];
};

template <class T> void rodrigues(const double e[3], T ang, T R[9]) {
  T ca = cos(ang), sa = sin(ang);
  T one_m = T(1.0) - ca;
  double K[9] = {0, -e[2], e[1], e[2], 0, -e[0], -e[1], e[0], 0};
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j)
      R[3 * i + j] = (i == j ? ca : T(0.0)) + sa * K[3 * i + j] + one_m * (e[i] * e[j]);
}

// Geometry from the descriptor (params == nullptr) or recomputed from the
// differentiable parameters.
template <class T> Geo<T> geometry(const Vol& v, const T* P) {
  Geo<T> g;
  for (int i = 0; i < 16; ++i) g.p[i] = T(v.p[i]);
  for (int i = 0; i < 9; ++i) g.Q[i] = T(v.Q[i]);
  for (int i = 0; i < 3; ++i) g.c[i] = T(v.c[i]);
  if (!P) return g;
  if (v.sparam >= 0) {
    if (v.shape == SH_SPHERE) g.p[0] = T(1.0) / P[v.sparam];
    else if (v.shape == SH_ASPHERE) for (int i = 0; i < 8; ++i) g.p[1 + i] = P[v.sparam + i];
    else if (v.shape == SH_HEXCONE) { g.p[2] = P[v.sparam]; g.p[3] = P[v.sparam + 1];
                                      g.p[4] = P[v.sparam + 2]; g.p[5] = P[v.sparam + 3]; }
  }
  if (v.tparam >= 0) {
    T Ra[9], Rb[9], R[9];
    rodrigues(v.e1, P[v.tparam], Ra);
    rodrigues(v.e2, P[v.tparam + 1], Rb);
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) {
        T s(0.0);
        for (int k = 0; k < 3; ++k) s = s + Rb[3 * i + k] * Ra[3 * k + j];
        R[3 * i + j] = s;
      }
    // Q = Q0 R^T ; c = pivot - R (pivot - c0)
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) {
        T s(0.0);
        for (int k = 0; k < 3; ++k) s = s + v.Q0[3 * i + k] * R[3 * j + k];
        g.Q[3 * i + j] = s;
      }
    for (int i = 0; i < 3; ++i) {
      T s(0.0);
      for (int k = 0; k < 3; ++k) s = s + R[3 * i + k] * (v.piv[k] - v.c0[k]);
      g.c[i] = v.piv[i] - s;
    }
  }
  return g;
}

template <class T> V3<T> to_local_p(const Geo<T>& g, V3<T> x) {
  V3<T> r = mk(x.x - g.c[0], x.y - g.c[1], x.z - g.c[2]);
  return mk(g.Q[0] * r.x + g.Q[1] * r.y + g.Q[2] * r.z,
            g.Q[3] * r.x + g.Q[4] * r.y + g.Q[5] * r.z,
            g.Q[6] * r.x + g.Q[7] * r.y + g.Q[8] * r.z);
}
template <class T> V3<T> to_local_d(const Geo<T>& g, V3<T> d) {
  return mk(g.Q[0] * d.x + g.Q[1] * d.y + g.Q[2] * d.z,
            g.Q[3] * d.x + g.Q[4] * d.y + g.Q[5] * d.z,
            g.Q[6] * d.x + g.Q[7] * d.y + g.Q[8] * d.z);
}
template <class T> V3<T> to_world_n(const Geo<T>& g, V3<T> n) {
  V3<T> w = mk(g.Q[0] * n.x + g.Q[3] * n.y + g.Q[6] * n.z,
               g.Q[1] * n.x + g.Q[4] * n.y + g.Q[7] * n.z,
               g.Q[2] * n.x + g.Q[5] * n.y + g.Q[8] * n.z);
  T s = sqrt(dot(w, w));
  return mk(w.x / s, w.y / s, w.z / s);
}

// ---- implicit function g(x_l) of a single-unknown face, its gradient (front normal direction)
template <class T> T sag_S(const T* p, T u) {      // asphere: sum b_i u^i (Horner)
  T s = p[8];
  for (int i = 7; i >= 1; --i) s = s * u + p[i];
  return s * u;
}
template <class T> T sag_dS(const T* p, T u) {     // dS/du
  T s = 8.0 * p[8];
  for (int i = 7; i >= 1; --i) s = s * u + double(i) * p[i];
  return s;
}

template <class T> T face_g(int shape, int face, const T* p, V3<T> x) {
  switch (shape) {
    case SH_PLANE: return x.z;
    case SH_SPHERE: return x.z - 0.5 * p[0] * dot(x, x);
    case SH_ASPHERE: { T u = (x.x * x.x + x.y * x.y) / (p[0] * p[0]); return x.z - sag_S(p, u); }
    case SH_CYLINDER: return (x.x * x.x + x.y * x.y - p[0] * p[0]) / (2.0 * p[0]);
    case SH_BOX: {
      int ax = face >> 1; double s = (face & 1) ? -1.0 : 1.0;
      T xv = ax == 0 ? x.x : ax == 1 ? x.y : x.z;
      return s * xv - p[ax];
    }
  }
  return T(0.0);
}
template <class T> V3<T> face_grad(int shape, int face, const T* p, V3<T> x) {
  switch (shape) {
    case SH_PLANE: return mk(T(0.0), T(0.0), T(1.0));
    case SH_SPHERE: return mk(-p[0] * x.x, -p[0] * x.y, T(1.0) - p[0] * x.z);
    case SH_ASPHERE: {
      T rn2 = p[0] * p[0];
      T u = (x.x * x.x + x.y * x.y) / rn2;
      T k = sag_dS(p, u) * 2.0 / rn2;
      return mk(-k * x.x, -k * x.y, T(1.0));
    }
    case SH_CYLINDER: return mk(x.x / p[0], x.y / p[0], T(0.0));
    case SH_BOX: {
      int ax = face >> 1; double s = (face & 1) ? -1.0 : 1.0;
      return mk(T(ax == 0 ? s : 0.0), T(ax == 1 ? s : 0.0), T(ax == 2 ? s : 0.0));
    }
  }
  return mk(T(0.0), T(0.0), T(1.0));
}

// ---- Bezier cone wall
template <class T> void bez(const T* p, T s, T& rho, T& z, T& drho, T& dz) {
  // p: rho0 z0 rho1 z1 rho2 z2 rho3 z3
  T a = T(1.0) - s;
  T b0 = a * a * a, b1 = 3.0 * a * a * s, b2 = 3.0 * a * s * s, b3 = s * s * s;
  rho = b0 * p[0] + b1 * p[2] + b2 * p[4] + b3 * p[6];
  z = b0 * p[1] + b1 * p[3] + b2 * p[5] + b3 * p[7];
  T d0 = 3.0 * a * a, d1 = 6.0 * a * s, d2 = 3.0 * s * s;
  drho = d0 * (p[2] - p[0]) + d1 * (p[4] - p[2]) + d2 * (p[6] - p[4]);
  dz = d0 * (p[3] - p[1]) + d1 * (p[5] - p[3]) + d2 * (p[7] - p[5]);
}
inline void wall_axes(int k, double& nx, double& ny) {
  nx = std::cos(k * PI / 3.0); ny = std::sin(k * PI / 3.0);
}

// ------------------------------------------------------------------ outlines
bool inside_outline(const Vol& v, double x, double y) {
  const double* o = v.o;
  switch (v.outline) {
    case OL_NONE: return true;
    case OL_DISC: return std::hypot(x, y) <= o[0];
    case OL_ANNULUS: { double r = std::hypot(x, y); return r >= o[0] && r <= o[1]; }
    case OL_RECT: return std::fabs(x) <= o[0] && std::fabs(y) <= o[1];
    case OL_HEX: {
      for (int k = 0; k < 3; ++k) {
        double a = k * PI / 3.0;
        if (std::fabs(x * std::cos(a) + y * std::sin(a)) > o[0]) return false;
      }
      return true;
    }
    case OL_SECTOR: {
      double r = std::hypot(x, y);
      if (r < o[0] || r > o[1]) return false;
      double ph = std::atan2(y, x) - o[2];
      ph = std::fmod(ph, 2.0 * PI);
      if (ph < 0) ph += 2.0 * PI;
      return ph <= o[3] - o[2];
    }
  }
  return false;
}
double outline_radius(const Vol& v) {
  const double* o = v.o;
  switch (v.outline) {
    case OL_DISC: return o[0];
    case OL_ANNULUS: case OL_SECTOR: return o[1];
    case OL_RECT: return std::hypot(o[0], o[1]);
    case OL_HEX: return o[0] * 2.0 / std::sqrt(3.0);
  }
  return 1e30;
}

// ------------------------------------------------------------------ root enumeration (double)
// A root of a face: t, face, curve parameter, whether it lies inside the
// face bounds, and its distance to the nearest face boundary (diagnostic).
struct Hit { double t; int face; double s; bool ok; double bd; };

void push_root(std::vector<Hit>& out, double t, int face, double s, bool ok, double bd) {
  out.push_back({t, face, s, ok, bd});
}

// unsigned distance from (x, y) to the boundary of the outline (diagnostic only)
double outline_bdist(const Vol& v, double x, double y) {
  const double* o = v.o;
  double r = std::hypot(x, y);
  switch (v.outline) {
    case OL_DISC: return std::fabs(r - o[0]);
    case OL_ANNULUS: return std::min(std::fabs(r - o[0]), std::fabs(r - o[1]));
    case OL_RECT: {
      double ex = std::fabs(x) - o[0], ey = std::fabs(y) - o[1];
      if (ex <= 0 && ey <= 0) return std::min(-ex, -ey);
      return std::hypot(std::max(ex, 0.0), std::max(ey, 0.0));
    }
    case OL_HEX: {
      double m = -1e300;
      for (int k = 0; k < 3; ++k) {
        double a = k * PI / 3.0;
        m = std::max(m, std::fabs(x * std::cos(a) + y * std::sin(a)) - o[0]);
      }
      return std::fabs(m);
    }
    case OL_SECTOR: {
      double d = std::min(std::fabs(r - o[0]), std::fabs(r - o[1]));
      for (int e = 2; e <= 3; ++e) d = std::min(d, std::fabs(x * std::sin(o[e]) - y * std::cos(o[e])));
      return d;
    }
  }
  return 1e300;
}

void quad_roots(double a, double b, double c, double r[2], int& n) {
  n = 0;
  if (a == 0.0) {
    if (b != 0.0) { r[0] = -c / b; n = 1; }
    return;
  }
  double disc = b * b - 4.0 * a * c;
  if (disc < 0.0) return;
  double sq = std::sqrt(disc);
  double q = -0.5 * (b + (b >= 0 ? sq : -sq));
  if (q == 0.0) { r[0] = 0.0; n = 1; return; }
  r[0] = q / a; r[1] = c / q; n = 2;
}

// all roots of g(t) = z0 + t dz - S(u(t)) on [ta, tb] by Lipschitz subdivision
void asphere_roots(const double* p, double ox, double oy, double oz, double dx, double dy, double dz,
                   double ta, double tb, double wmin, std::vector<double>& roots) {
  double rn2 = p[0] * p[0];
  double A = (dx * dx + dy * dy) / rn2, B = 2.0 * (ox * dx + oy * dy) / rn2, C = (ox * ox + oy * oy) / rn2;
  auto u_of = [&](double t) { return (A * t + B) * t + C; };
  auto g_of = [&](double t) { return oz + t * dz - sag_S(p, u_of(t)); };
  struct Iv { double a, b; };
  std::vector<Iv> stack{{ta, tb}};
  while (!stack.empty()) {
    Iv iv = stack.back(); stack.pop_back();
    double a = iv.a, b = iv.b, m = 0.5 * (a + b);
    double ua = u_of(a), ub = u_of(b);
    double umax = std::max(ua, ub);
    double lp = 0.0, upow = 1.0;
    for (int i = 1; i <= 8; ++i) { lp += i * std::fabs(p[i]) * upow; upow *= std::max(umax, 0.0); }
    double lu = std::max(std::fabs(2.0 * A * a + B), std::fabs(2.0 * A * b + B));
    double L = std::fabs(dz) + lp * lu;
    double gm = g_of(m);
    if (std::fabs(gm) > L * 0.5 * (b - a) * (1.0 + 1e-12) + 1e-300) continue;
    if (b - a > wmin) { stack.push_back({m, b}); stack.push_back({a, m}); continue; }
    double ga = g_of(a), gb = g_of(b);
    if (ga == 0.0) { roots.push_back(a); continue; }
    if (ga * gb > 0.0) continue;                 // no sign change: tangency, not a crossing
    for (int it = 0; it < 200 && b - a > 1e-15 * std::max(1.0, std::fabs(a)); ++it) {
      double mm = 0.5 * (a + b), gmm = g_of(mm);
      if ((gmm <= 0.0) == (ga <= 0.0)) { a = mm; ga = gmm; } else { b = mm; }
    }
    roots.push_back(0.5 * (a + b));
  }
}

// real roots of a cubic in power basis on [0, 1]
void cubic_roots01(const double c[4], std::vector<double>& roots) {
  auto F = [&](double s) { return ((c[3] * s + c[2]) * s + c[1]) * s + c[0]; };
  std::vector<double> br{0.0};
  double cr[2]; int nc = 0;
  quad_roots(3.0 * c[3], 2.0 * c[2], c[1], cr, nc);
  std::sort(cr, cr + nc);
  for (int i = 0; i < nc; ++i) if (cr[i] > 0.0 && cr[i] < 1.0) br.push_back(cr[i]);
  br.push_back(1.0);
  for (size_t i = 0; i + 1 < br.size(); ++i) {
    double a = br[i], b = br[i + 1], fa = F(a), fb = F(b);
    if (fa == 0.0) { if (roots.empty() || roots.back() != a) roots.push_back(a); continue; }
    if (i + 2 == br.size() && fb == 0.0) { roots.push_back(b); continue; }
    if (fa * fb > 0.0) continue;
    for (int it = 0; it < 200 && b - a > 1e-16; ++it) {
      double m = 0.5 * (a + b), fm = F(m);
      if ((fm <= 0.0) == (fa <= 0.0)) { a = m; fa = fm; } else b = m;
    }
    roots.push_back(0.5 * (a + b));
  }
}

// Every crossing of the ray with every face of v, with its face bounds checked.
void volume_hits(const Vol& v, V3<double> ow, V3<double> dw, double l_ref, std::vector<Hit>& out) {
  Geo<double> g = geometry<double>(v, nullptr);
  V3<double> o = to_local_p(g, ow), d = to_local_d(g, dw);
  const double* p = g.p;
  switch (v.shape) {
    case SH_PLANE: {
      if (d.z == 0.0) return;
      double t = -o.z / d.z;
      V3<double> x = o + t * d;
      push_root(out, t, 0, 0.0, inside_outline(v, x.x, x.y), outline_bdist(v, x.x, x.y));
      return;
    }
    case SH_SPHERE: {
      double cv = p[0];
      double a = -0.5 * cv * dot(d, d), b = d.z - cv * dot(o, d), c = o.z - 0.5 * cv * dot(o, o);
      double r[2]; int n;
      quad_roots(a, b, c, r, n);
      for (int i = 0; i < n; ++i) {
        V3<double> x = o + r[i] * d;
        if (1.0 - cv * x.z < 0.0) continue;            // far hemisphere: not the cap
        push_root(out, r[i], 0, 0.0, inside_outline(v, x.x, x.y), outline_bdist(v, x.x, x.y));
      }
      return;
    }
    case SH_ASPHERE: {
      double rb = outline_radius(v);
      double ub = rb * rb / (p[0] * p[0]);
      double zb = 0.0, up = 1.0;
      for (int i = 1; i <= 8; ++i) { up *= ub; zb += std::fabs(p[i]) * up; }
      double A = d.x * d.x + d.y * d.y, B = 2.0 * (o.x * d.x + o.y * d.y), C = o.x * o.x + o.y * o.y;
      std::vector<double> roots;
      double ta = -1e300, tb = 1e300;
      if (d.z != 0.0) {
        double t1 = (-zb - o.z) / d.z, t2 = (zb - o.z) / d.z;
        ta = std::min(t1, t2); tb = std::max(t1, t2);
      } else if (std::fabs(o.z) > zb) return;
      if (A > 0.0) {
        double r[2]; int n;
        quad_roots(A, B, C - rb * rb, r, n);
        if (n < 2) return;
        ta = std::max(ta, std::min(r[0], r[1])); tb = std::min(tb, std::max(r[0], r[1]));
      } else {
        if (C > rb * rb || d.z == 0.0) return;
        double tt = (sag_S(p, C / (p[0] * p[0])) - o.z) / d.z;
        roots.push_back(tt);
        ta = 1.0; tb = 0.0;
      }
      if (ta < tb) asphere_roots(p, o.x, o.y, o.z, d.x, d.y, d.z, ta, tb, 1e-9 * l_ref, roots);
      for (double t : roots) {
        V3<double> x = o + t * d;
        push_root(out, t, 0, 0.0, inside_outline(v, x.x, x.y), outline_bdist(v, x.x, x.y));
      }
      return;
    }
    case SH_CYLINDER: {
      double a = d.x * d.x + d.y * d.y, b = 2.0 * (o.x * d.x + o.y * d.y), c = o.x * o.x + o.y * o.y - p[0] * p[0];
      if (a == 0.0) return;
      double r[2]; int n;
      quad_roots(a, b, c, r, n);
      for (int i = 0; i < n; ++i) {
        double z = o.z + r[i] * d.z;
        push_root(out, r[i], 0, 0.0, z >= 0.0 && z <= p[1], std::min(std::fabs(z), std::fabs(p[1] - z)));
      }
      return;
    }
    case SH_BOX: {
      for (int f = 0; f < 6; ++f) {
        int ax = f >> 1; double s = (f & 1) ? -1.0 : 1.0;
        double oa = ax == 0 ? o.x : ax == 1 ? o.y : o.z, da = ax == 0 ? d.x : ax == 1 ? d.y : d.z;
        if (da == 0.0) continue;
        double t = (s * p[ax] - oa) / da;
        V3<double> x = o + t * d;
        double xs[3] = {x.x, x.y, x.z};
        bool ok = true;
        double bd = 1e300;
        for (int k = 0; k < 3; ++k)
          if (k != ax) {
            if (std::fabs(xs[k]) > p[k]) ok = false;
            bd = std::min(bd, std::fabs(p[k] - std::fabs(xs[k])));
          }
        push_root(out, t, f, 0.0, ok, bd);
      }
      return;
    }
    case SH_HEXCONE: {
      for (int f = 0; f < 6; ++f) {
        double nx, ny; wall_axes(f, nx, ny);
        double u0 = o.x * nx + o.y * ny, du = d.x * nx + d.y * ny;
        double w[4];
        for (int k = 0; k < 4; ++k) w[k] = (p[2 * k] - u0) * d.z - (p[2 * k + 1] - o.z) * du;
        if (w[0] == 0.0 && w[1] == 0.0 && w[2] == 0.0 && w[3] == 0.0) continue;
        double cc[4] = {w[0], 3.0 * (w[1] - w[0]), 3.0 * (w[0] - 2.0 * w[1] + w[2]),
                        w[3] - 3.0 * w[2] + 3.0 * w[1] - w[0]};
        std::vector<double> ss;
        cubic_roots01(cc, ss);
        for (double s : ss) {
          double rho, z, drho, dz;
          bez(p, s, rho, z, drho, dz);
          double t = std::fabs(d.z) >= std::fabs(du) ? (z - o.z) / d.z : (rho - u0) / du;
          V3<double> x = o + t * d;
          double vt = -x.x * ny + x.y * nx;
          double arc = std::hypot(drho, dz);
          double bd = std::min(std::fabs(rho / std::sqrt(3.0) - std::fabs(vt)), std::min(s, 1.0 - s) * arc);
          push_root(out, t, f, s, std::fabs(vt) <= rho / std::sqrt(3.0), bd);
        }
      }
      return;
    }
  }
}

// front normal (world) of face `face` of v at local hit point (double or dual)
template <class T> V3<T> front_normal(const Vol& v, const Geo<T>& g, int face, V3<T> xl, T s) {
  if (v.shape == SH_HEXCONE) {
    T rho, z, dr, dz;
    bez(g.p, s, rho, z, dr, dz);
    double nx, ny; wall_axes(face, nx, ny);
    V3<T> nl = mk(-dz * nx, -dz * ny, dr);
    return to_world_n(g, nl);
  }
  return to_world_n(g, face_grad(v.shape, face, g.p, xl));
}

void bounding_sphere(Vol& v) {
  double lc[3] = {0, 0, 0}, r = 0;
  const double* p = v.p;
  switch (v.shape) {
    case SH_PLANE: r = outline_radius(v); break;
    case SH_SPHERE: {
      double rb = outline_radius(v), cv = std::fabs(p[0]);
      double zr = (cv * rb >= 1.0) ? 1.0 / cv : (cv * rb * rb) / (1.0 + std::sqrt(1.0 - cv * cv * rb * rb));
      r = std::sqrt(rb * rb + zr * zr);
      break;
    }
    case SH_ASPHERE: {
      double rb = outline_radius(v), ub = rb * rb / (p[0] * p[0]), zb = 0.0, up = 1.0;
      for (int i = 1; i <= 8; ++i) { up *= ub; zb += std::fabs(p[i]) * up; }
      r = std::sqrt(rb * rb + zb * zb);
      break;
    }
    case SH_CYLINDER: lc[2] = 0.5 * p[1]; r = std::sqrt(p[0] * p[0] + 0.25 * p[1] * p[1]); break;
    case SH_BOX: r = std::sqrt(p[0] * p[0] + p[1] * p[1] + p[2] * p[2]); break;
    case SH_HEXCONE: {
      double rmax = std::max(std::max(std::fabs(p[0]), std::fabs(p[2])), std::max(std::fabs(p[4]), std::fabs(p[6])));
      double zmin = std::min(std::min(p[1], p[3]), std::min(p[5], p[7]));
      double zmax = std::max(std::max(p[1], p[3]), std::max(p[5], p[7]));
      lc[2] = 0.5 * (zmin + zmax);
      r = std::sqrt(rmax * rmax * 4.0 / 3.0 + 0.25 * (zmax - zmin) * (zmax - zmin));
      break;
    }
  }
  // world centre: c + Q^{-1} lc ; Q is orthonormal up to rounding, pad the radius
  for (int i = 0; i < 3; ++i) v.bc[i] = v.c[i] + v.Q[0 + i] * lc[0] + v.Q[3 + i] * lc[1] + v.Q[6 + i] * lc[2];
  v.br = r * (1.0 + 1e-6) + 1e-9 * (1.0 + std::fabs(v.bc[0]) + std::fabs(v.bc[1]) + std::fabs(v.bc[2]));
}

bool sphere_may_hit(const Vol& v, V3<double> o, V3<double> d, double tlo) {
  V3<double> oc = mk(v.bc[0] - o.x, v.bc[1] - o.y, v.bc[2] - o.z);
  double dd = dot(d, d);
  double tc = dot(oc, d) / dd;
  V3<double> perp = oc - tc * d;
  double r2 = v.br * v.br;
  if (dot(perp, perp) > r2 * 1.000001) return false;
  double half = std::sqrt(std::max(0.0, r2 - dot(perp, perp)) / dd) * 1.000001 + 1e-12;
  return tc + half > tlo;
}

std::vector<Vol> unpack(int nv, const int32_t* vi, const double* vd) {
  std::vector<Vol> vs(nv);
  for (int k = 0; k < nv; ++k) {
    Vol& v = vs[k];
    const int32_t* I = vi + NI * k; const double* D = vd + ND * k;
    v.role = I[0]; v.shape = I[1]; v.outline = I[2]; v.sparam = I[3]; v.tparam = I[4];
    int q = 0;
    for (int i = 0; i < 9; ++i) v.Q[i] = D[q++];
    for (int i = 0; i < 3; ++i) v.c[i] = D[q++];
    for (int i = 0; i < 16; ++i) v.p[i] = D[q++];
    for (int i = 0; i < 4; ++i) v.o[i] = D[q++];
    v.refl = D[q++]; v.n_in = D[q++];
    for (int i = 0; i < 9; ++i) v.Q0[i] = D[q++];
    for (int i = 0; i < 3; ++i) v.c0[i] = D[q++];
    for (int i = 0; i < 3; ++i) v.piv[i] = D[q++];
    for (int i = 0; i < 3; ++i) v.e1[i] = D[q++];
    for (int i = 0; i < 3; ++i) v.e2[i] = D[q++];
    bounding_sphere(v);
  }
  return vs;
}

// ------------------------------------------------------------------ interactions
// Unpolarised Fresnel reflectance for cos_i (incidence) from n1 into n2; 1 on TIR.
double fresnel(double cos_i, double n1, double n2, double& cos_t) {
  double eta = n1 / n2;
  double s2 = eta * eta * (1.0 - cos_i * cos_i);
  if (s2 >= 1.0) { cos_t = 0.0; return 1.0; }
  cos_t = std::sqrt(1.0 - s2);
  double rs = (n1 * cos_i - n2 * cos_t) / (n1 * cos_i + n2 * cos_t);
  double rp = (n2 * cos_i - n1 * cos_t) / (n2 * cos_i + n1 * cos_t);
  return 0.5 * (rs * rs + rp * rp);
}

// Refractive index of a lens volume's medium for a photon of wavelength lam
// (metres; 0 = the photon carries none).  A lens whose descriptor gives a
// Cauchy law (p[13] = A, p[14] = B != 0) has n = A + B / lam^2 for photons
// with a wavelength; otherwise its fixed index n_inside.
double lens_index(const Vol& v, double lam) {
  if (lam > 0.0 && v.p[14] != 0.0) return v.p[13] + v.p[14] / (lam * lam);
  return v.n_in;
}

constexpr uint64_t HASH0 = 0xcbf29ce484222325ull, HASHP = 0x100000001b3ull;

struct Rec {
  uint8_t fate, nev; int32_t last_vol;
  double pos[3], dir[3], opl; uint64_t hash;
};

struct Scn {
  std::vector<Vol> v;
  int max_events; uint64_t seed; double l_ref;
};

// Per-event diagnostics (NDIAG doubles), used only to classify photons whose
// path is ill-conditioned: [0] gap to the next candidate surface (or the hit
// distance when the face just left is met again), [1] distance of the hit to
// its face boundary, [2] smallest boundary distance of a root rejected by the
// bounds nearer than the hit, [3] |d . n|, [4] distance of the random draw
// from its reflect / absorb threshold.
constexpr int NDIAG = 5;

Rec trace_one(const Scn& S, V3<double> o, V3<double> d, double lam, uint64_t id, int culled,
              int32_t* lv, int32_t* lf, int32_t* la, double* lt, double* ls, double* ldiag) {
  Rec r{};
  r.hash = HASH0; r.last_vol = -1;
  double ncur = 1.0;
  int prev_v = -1, prev_f = -1, prev_side = 0;
  const double eps_self = 1e-9 * S.l_ref, eps_tie = 1e-12 * S.l_ref;
  std::vector<Hit> hits;
  // a photon is a position and a unit direction (§2.1); any other input
  // (non-finite, or |d| off 1 by more than rounding) is refused, not traced
  if (!(std::isfinite(o.x) && std::isfinite(o.y) && std::isfinite(o.z) && std::isfinite(d.x) &&
        std::isfinite(d.y) && std::isfinite(d.z)) || !(std::fabs(dot(d, d) - 1.0) <= 1e-5)) {
    r.fate = F_FAILED;
  }
  int k = 0;
  while (!r.fate) {
    if (k == S.max_events) { r.fate = F_SUSPENDED; break; }
    const double INF = std::numeric_limits<double>::infinity();
    double bt = INF, bs = 0.0, bbd = INF;
    int bv = -1, bf = -1;
    std::vector<std::pair<double, double>> rejected;   // (t, boundary distance)
    std::vector<std::pair<double, long>> valid;        // (t, vol * 8 + face)
    for (int vi = 0; vi < (int)S.v.size(); ++vi) {
      const Vol& v = S.v[vi];
      if (culled && !sphere_may_hit(v, o, d, 0.0)) continue;
      hits.clear();
      volume_hits(v, o, d, S.l_ref, hits);
      for (const Hit& h : hits) {
        bool self = vi == prev_v && h.face == prev_f;
        double tlo = self ? eps_self : 0.0;
        if (!(h.t > tlo)) continue;
        if (self) {
          // the face just left is met again only from the side the photon is on
          Geo<double> gs = geometry<double>(v, nullptr);
          V3<double> ns = front_normal(v, gs, h.face, to_local_p(gs, o + h.t * d), h.s);
          if ((dot(d, ns) < 0.0) != (prev_side == 0)) continue;
        }
        if (!h.ok) { if (ldiag) rejected.push_back({h.t, h.bd}); continue; }
        if (ldiag) valid.push_back({h.t, (long)vi * 8 + h.face});
        bool better = h.t < bt - eps_tie ||
                      (std::fabs(h.t - bt) <= eps_tie && (vi < bv || (vi == bv && h.face < bf)));
        if (better) { bt = h.t; bv = vi; bf = h.face; bs = h.s; bbd = h.bd; }
      }
    }
    if (ldiag) {
      double* dg = ldiag + NDIAG * k;
      double gap = INF, miss = INF;
      // exact ties (coincident surfaces) are settled by volume id on any
      // tracer and are not ill-conditioned
      for (auto& c : valid)
        if (c.second != (long)bv * 8 + bf && std::fabs(c.first - bt) > eps_tie)
          gap = std::min(gap, std::fabs(c.first - bt));
      if (bv >= 0 && bv == prev_v && bf == prev_f) gap = std::min(gap, bt);
      double tcut = (bv >= 0 ? bt : INF) + 1e-5 * S.l_ref;
      for (auto& c : rejected)
        if (c.first <= tcut) miss = std::min(miss, c.second);
      dg[0] = gap; dg[1] = bbd; dg[2] = miss; dg[3] = INF; dg[4] = INF;
    }
    if (bv < 0) { r.fate = F_EXITED; break; }
    const Vol& v = S.v[bv];
    V3<double> X = o + bt * d;
    r.opl += ncur * bt;
    Geo<double> g = geometry<double>(v, nullptr);
    V3<double> n = front_normal(v, g, bf, to_local_p(g, X), bs);
    double dn = dot(d, n);
    int back = dn < 0.0 ? 0 : 1;
    if (ldiag) ldiag[NDIAG * k + 3] = std::fabs(dn);
    uint32_t code = ((uint32_t)bv << 4) | ((uint32_t)bf << 1) | (uint32_t)back;
    r.hash = (r.hash ^ code) * HASHP;
    r.last_vol = bv;
    int act = ACT_STOP;
    o = X;
    if (v.role == ROLE_FOCAL) {
      r.fate = back ? F_ABSORBED : F_FOCUSED;
    } else if (v.role == ROLE_OBSCURATION) {
      r.fate = F_ABSORBED;
    } else if (v.role == ROLE_MIRROR) {
      if (back) r.fate = F_ABSORBED;
      else {
        double R = std::min(std::max(v.refl, 0.0), 1.0);
        uint64_t thr = (uint64_t)std::floor(R * 4294967296.0);
        uint32_t u = draw(S.seed, id, k);
        if (ldiag && R < 1.0) ldiag[NDIAG * k + 4] = std::fabs((double)u / 4294967296.0 - R);
        if ((uint64_t)u >= thr) r.fate = F_ABSORBED;
        else { d = d - (2.0 * dn) * n; act = ACT_REFLECT; }
      }
    } else if (v.role == ROLE_LENS) {
      const double nl = lens_index(v, lam);
      double n1 = back ? nl : 1.0, n2 = back ? 1.0 : nl;
      V3<double> no = back ? (-1.0) * n : n;          // oriented against d
      double cos_i = -dot(d, no), cos_t;
      double R = fresnel(cos_i, n1, n2, cos_t);
      uint32_t u = draw(S.seed, id, k);
      if (ldiag) ldiag[NDIAG * k + 4] = std::fabs((double)(u >> 8) * (1.0 / 16777216.0) - R);
      // bulk absorption (p[15] = absorption length L of the lens medium, 0 =
      // none): the segment of length bt just crossed inside the glass is
      // survived with probability exp(-bt / L)
      bool absorbed = false;
      if (back && v.p[15] > 0.0) {
        double surv = std::exp(-bt / v.p[15]);
        double w = (double)draw(S.seed, id, k, 2u) * (1.0 / 4294967296.0);
        if (ldiag) ldiag[NDIAG * k + 4] = std::min(ldiag[NDIAG * k + 4], std::fabs(w - surv));
        absorbed = w >= surv;
      }
      if (absorbed) r.fate = F_ABSORBED;
      else if ((double)(u >> 8) * (1.0 / 16777216.0) < R) { d = d - (2.0 * dot(d, no)) * no; act = ACT_REFLECT; }
      else {
        double eta = n1 / n2;
        d = eta * d + (eta * cos_i - cos_t) * no;
        ncur = n2; act = ACT_REFRACT;
      }
    } else {
      r.fate = F_FAILED;
    }
    if (lv) { lv[k] = bv; lf[k] = bf; la[k] = act; lt[k] = bt; ls[k] = bs; }
    prev_v = bv; prev_f = bf;
    prev_side = back ^ (act == ACT_REFRACT ? 1 : 0);
    ++k;
    if (!(std::isfinite(d.x) && std::isfinite(d.y) && std::isfinite(d.z))) r.fate = F_FAILED;
  }
  r.nev = (uint8_t)k;
  r.pos[0] = o.x; r.pos[1] = o.y; r.pos[2] = o.z;
  r.dir[0] = d.x; r.dir[1] = d.y; r.dir[2] = d.z;
  return r;
}

template <class F> void parallel_for(int64_t n, int nthreads, F f) {
  if (nthreads <= 1 || n < 64) { f(0, n); return; }
  std::vector<std::thread> th;
  int64_t chunk = (n + nthreads - 1) / nthreads;
  for (int t = 0; t < nthreads; ++t) {
    int64_t a = t * chunk, b = std::min(n, a + chunk);
    if (a >= b) break;
    th.emplace_back([=] { f(a, b); });
  }
  for (auto& t : th) t.join();
}

// ------------------------------------------------------------------ forced sequences
// Re-evaluate a photon along a recorded face sequence with parameters P
// (type T), no search.  Each root is continued from the recorded one by
// Newton in double, then a last Newton step is taken in T so derivatives
// follow the implicit-function theorem.
template <class T>
int forced_one(const std::vector<Vol>& vs, const T* P, V3<T> o, V3<T> d, double lam, int nev,
               const int32_t* lv, const int32_t* lf, const int32_t* la, const double* lt,
               const double* ls, V3<T>& pos, V3<T>& dir) {
  for (int e = 0; e < nev; ++e) {
    const Vol& v = vs[lv[e]];
    int face = lf[e];
    Geo<T> g = geometry<T>(v, P);
    V3<T> ol = to_local_p(g, o), dl = to_local_d(g, d);
    T t, s(0.0);
    if (v.shape == SH_HEXCONE) {
      double nx, ny; wall_axes(face, nx, ny);
      double sv = ls[e], tv = lt[e];
      double pd[16]; for (int i = 0; i < 16; ++i) pd[i] = val(g.p[i]);
      double u0 = val(ol.x) * nx + val(ol.y) * ny, du = val(dl.x) * nx + val(dl.y) * ny;
      double z0 = val(ol.z), dz = val(dl.z);
      // unknowns (s, t): F1 = rho(s) - (u0 + t du), F2 = z(s) - (z0 + t dz)
      // J = [[rho', -du], [z', -dz]], det = du z' - rho' dz; Newton step solves J [a b] = -F
      for (int it = 0; it < 60; ++it) {
        double rho, z, dr, dzs;
        bez(pd, sv, rho, z, dr, dzs);
        double F1 = rho - (u0 + tv * du), F2 = z - (z0 + tv * dz);
        double det = du * dzs - dr * dz;
        if (det == 0.0) return -1;
        double a = (F1 * dz - du * F2) / det;
        double b = (F1 * dzs - dr * F2) / det;
        sv += a; tv += b;
        if (std::fabs(a) < 1e-15 && std::fabs(b) < 1e-15 * std::max(1.0, std::fabs(tv))) break;
      }
      // last step in T
      T S_(sv), Tt(tv);
      T rho, z, dr, dzs;
      bez(g.p, S_, rho, z, dr, dzs);
      T u0T = ol.x * nx + ol.y * ny, duT = dl.x * nx + dl.y * ny;
      T F1 = rho - (u0T + Tt * duT), F2 = z - (ol.z + Tt * dl.z);
      T det = duT * dzs - dr * dl.z;
      s = S_ + (F1 * dl.z - duT * F2) / det;
      t = Tt + (F1 * dzs - dr * F2) / det;
    } else {
      double tv = lt[e];
      double pd[16]; for (int i = 0; i < 16; ++i) pd[i] = val(g.p[i]);
      V3<double> old = mk(val(ol.x), val(ol.y), val(ol.z)), dld = mk(val(dl.x), val(dl.y), val(dl.z));
      for (int it = 0; it < 60; ++it) {
        V3<double> x = old + tv * dld;
        double gv = face_g<double>(v.shape, face, pd, x);
        double gd = dot(face_grad<double>(v.shape, face, pd, x), dld);
        if (gd == 0.0) return -1;
        double step = gv / gd;
        tv -= step;
        if (std::fabs(step) < 1e-15 * std::max(1.0, std::fabs(tv))) break;
      }
      T Tt(tv);
      V3<T> x = ol + Tt * dl;
      T gv = face_g<T>(v.shape, face, g.p, x);
      T gd = dot(face_grad<T>(v.shape, face, g.p, x), dl);
      t = Tt - gv / gd;
    }
    V3<T> X = o + t * d;
    V3<T> n = front_normal(v, g, face, to_local_p(g, X), s);
    o = X;
    if (la[e] == ACT_STOP) break;
    T dn = dot(d, n);
    if (la[e] == ACT_REFLECT) {
      d = d - (2.0 * dn) * n;
    } else {
      bool back = val(dn) >= 0.0;
      const double nl = lens_index(v, lam);
      double n1 = back ? nl : 1.0, n2 = back ? 1.0 : nl;
      V3<T> no = back ? (-1.0) * n : n;
      T cos_i = T(0.0) - dot(d, no);
      double eta = n1 / n2;
      T s2 = eta * eta * (T(1.0) - cos_i * cos_i);
      if (val(s2) >= 1.0) return -2;
      T cos_t = sqrt(T(1.0) - s2);
      d = eta * d + (eta * cos_i - cos_t) * no;
    }
  }
  pos = o; dir = d;
  return 0;
}

}  // namespace

extern "C" {

int oracle_abi_version() { return 1; }

void oracle_philox4x32_10(const uint32_t* ctr, const uint32_t* key, uint32_t* out) {
  philox4x32_10(ctr, key, out);
}

uint32_t oracle_draw(uint64_t seed, uint64_t id, int event) { return draw(seed, id, event); }

double oracle_fresnel(double cos_i, double n1, double n2) { double ct; return fresnel(cos_i, n1, n2, ct); }

// Brute-force trace.  Rays and outputs are SoA float64; lam (wavelengths, m)
// and the log arrays (n * max_events) may be NULL.
int oracle_trace(int nv, const int32_t* vi, const double* vd, int max_events, uint64_t seed,
                 double l_ref, int64_t n, const double* ox, const double* oy, const double* oz,
                 const double* dx, const double* dy, const double* dz, const double* lam, uint64_t id_base,
                 uint8_t* fate, uint8_t* nev, int32_t* last_vol, double* pos, double* dir,
                 double* opl, uint64_t* hash, int32_t* log_vol, int32_t* log_face,
                 int32_t* log_act, double* log_t, double* log_s, double* log_diag, int nthreads,
                 int culled) {
  if (nv < 0 || n < 0 || max_events < 1 || max_events > 255) return -1;
  Scn S;
  S.v = unpack(nv, vi, vd);
  S.max_events = max_events; S.seed = seed; S.l_ref = l_ref;
  parallel_for(n, nthreads, [&](int64_t a, int64_t b) {
    for (int64_t i = a; i < b; ++i) {
      int64_t lo = i * (int64_t)max_events;
      Rec r = trace_one(S, mk(ox[i], oy[i], oz[i]), mk(dx[i], dy[i], dz[i]), lam ? lam[i] : 0.0,
                        id_base + (uint64_t)i,
                        culled, log_vol ? log_vol + lo : nullptr, log_face ? log_face + lo : nullptr,
                        log_act ? log_act + lo : nullptr, log_t ? log_t + lo : nullptr,
                        log_s ? log_s + lo : nullptr, log_diag ? log_diag + lo * NDIAG : nullptr);
      fate[i] = r.fate; nev[i] = r.nev; last_vol[i] = r.last_vol;
      for (int k = 0; k < 3; ++k) { pos[3 * i + k] = r.pos[k]; dir[3 * i + k] = r.dir[k]; }
      opl[i] = r.opl; hash[i] = r.hash;
    }
  });
  return 0;
}

// Outline membership and boundary distance of volume 0 at local points
// (x[i], y[i]): the bounds test and the diagnostic distance used by the
// trace, exposed so that tests can pin them against closed forms.
int oracle_outline(const int32_t* vi, const double* vd, int64_t n, const double* x, const double* y,
                   uint8_t* inside, double* bdist) {
  if (n < 0) return -1;
  std::vector<Vol> vs = unpack(1, vi, vd);
  for (int64_t i = 0; i < n; ++i) {
    inside[i] = inside_outline(vs[0], x[i], y[i]) ? 1 : 0;
    bdist[i] = outline_bdist(vs[0], x[i], y[i]);
  }
  return 0;
}

// Forced-sequence evaluation in double with parameters P (FD driver).
int oracle_forced(int nv, const int32_t* vi, const double* vd, const double* P, int64_t n,
                  const double* ox, const double* oy, const double* oz, const double* dx,
                  const double* dy, const double* dz, const double* lam, int max_events, const uint8_t* nev,
                  const int32_t* log_vol, const int32_t* log_face, const int32_t* log_act,
                  const double* log_t, const double* log_s, double* pos, double* dir,
                  int32_t* status, int nthreads) {
  std::vector<Vol> vs = unpack(nv, vi, vd);
  parallel_for(n, nthreads, [&](int64_t a, int64_t b) {
    for (int64_t i = a; i < b; ++i) {
      int64_t lo = i * (int64_t)max_events;
      const double nan = std::numeric_limits<double>::quiet_NaN();
      V3<double> p = mk(nan, nan, nan), q = p;
      status[i] = forced_one<double>(vs, P, mk(ox[i], oy[i], oz[i]), mk(dx[i], dy[i], dz[i]), lam ? lam[i] : 0.0,
                                     nev[i],
                                     log_vol + lo, log_face + lo, log_act + lo, log_t + lo,
                                     log_s + lo, p, q);
      pos[3 * i] = p.x; pos[3 * i + 1] = p.y; pos[3 * i + 2] = p.z;
      dir[3 * i] = q.x; dir[3 * i + 1] = q.y; dir[3 * i + 2] = q.z;
    }
  });
  return 0;
}

// Forward-mode derivatives of the final position and direction with respect
// to parameters [p0, p0 + cnt), cnt <= 8: dpos/ddir are (n, 3, cnt).
int oracle_forced_jac(int nv, const int32_t* vi, const double* vd, const double* P, int np,
                      int p0, int cnt, int64_t n, const double* ox, const double* oy,
                      const double* oz, const double* dx, const double* dy, const double* dz,
                      const double* lam, int max_events, const uint8_t* nev, const int32_t* log_vol,
                      const int32_t* log_face, const int32_t* log_act, const double* log_t,
                      const double* log_s, double* dpos, double* ddir, int32_t* status,
                      int nthreads) {
  if (cnt < 1 || cnt > NDUAL || p0 < 0 || p0 + cnt > np) return -1;
  std::vector<Vol> vs = unpack(nv, vi, vd);
  std::vector<Dual> PD(np);
  for (int i = 0; i < np; ++i) PD[i] = Dual(P[i]);
  for (int j = 0; j < cnt; ++j) PD[p0 + j].d[j] = 1.0;
  parallel_for(n, nthreads, [&](int64_t a, int64_t b) {
    for (int64_t i = a; i < b; ++i) {
      int64_t lo = i * (int64_t)max_events;
      V3<Dual> p, q;
      status[i] = forced_one<Dual>(vs, PD.data(), mk(Dual(ox[i]), Dual(oy[i]), Dual(oz[i])),
                                   mk(Dual(dx[i]), Dual(dy[i]), Dual(dz[i])), lam ? lam[i] : 0.0, nev[i],
                                   log_vol + lo,
                                   log_face + lo, log_act + lo, log_t + lo, log_s + lo, p, q);
      const Dual* pc[3] = {&p.x, &p.y, &p.z};
      const Dual* qc[3] = {&q.x, &q.y, &q.z};
      for (int k = 0; k < 3; ++k)
        for (int j = 0; j < cnt; ++j) {
          dpos[(i * 3 + k) * cnt + j] = pc[k]->d[j];
          ddir[(i * 3 + k) * cnt + j] = qc[k]->d[j];
        }
    }
  });
  return 0;
}

}  // extern "C"
