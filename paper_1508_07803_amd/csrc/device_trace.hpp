// Device-side photon transport for gfx950: Philox draws, per-shape exact
// intersections, the non-sequential nearest-surface search and the
// interaction physics.  All arithmetic is in the scene precision T (float or
// double); group sums are accumulated in double by the kernels.
//
// Physics follows the paper's roles (§2.1): mirrors reflect (absorbing with
// probability 1 - R, and on their back), lenses refract by Snell's law with
// unpolarised Fresnel reflection, focal surfaces detect (front) or absorb
// (back), obscurations absorb.  Shapes follow §2.2.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

#include "scene_layout.hpp"

namespace robast {

template <typename T> struct V3 { T x, y, z; };
template <typename T> __device__ __forceinline__ V3<T> mk3(T a, T b, T c) { return V3<T>{a, b, c}; }
template <typename T> __device__ __forceinline__ V3<T> add(V3<T> a, V3<T> b) { return {a.x + b.x, a.y + b.y, a.z + b.z}; }
template <typename T> __device__ __forceinline__ V3<T> sub(V3<T> a, V3<T> b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
template <typename T> __device__ __forceinline__ V3<T> scl(T s, V3<T> a) { return {s * a.x, s * a.y, s * a.z}; }
template <typename T> __device__ __forceinline__ V3<T> fma3(T s, V3<T> a, V3<T> b) {
  return {s * a.x + b.x, s * a.y + b.y, s * a.z + b.z};
}
template <typename T> __device__ __forceinline__ T dot(V3<T> a, V3<T> b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
template <typename T> __device__ __forceinline__ V3<T> cross(V3<T> a, V3<T> b) {
  return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}

__device__ __forceinline__ float dsqrt(float x) { return __builtin_sqrtf(x); }
__device__ __forceinline__ double dsqrt(double x) { return __builtin_sqrt(x); }
__device__ __forceinline__ float dabs(float x) { return __builtin_fabsf(x); }
__device__ __forceinline__ double dabs(double x) { return __builtin_fabs(x); }
__device__ __forceinline__ float dmin(float a, float b) { return __builtin_fminf(a, b); }
__device__ __forceinline__ double dmin(double a, double b) { return __builtin_fmin(a, b); }
__device__ __forceinline__ float dmax(float a, float b) { return __builtin_fmaxf(a, b); }
__device__ __forceinline__ double dmax(double a, double b) { return __builtin_fmax(a, b); }
__device__ __forceinline__ float dfloor(float a) { return __builtin_floorf(a); }
__device__ __forceinline__ double dfloor(double a) { return __builtin_floor(a); }
__device__ __forceinline__ float dcopysign(float a, float b) { return __builtin_copysignf(a, b); }
__device__ __forceinline__ double dcopysign(double a, double b) { return __builtin_copysign(a, b); }
template <typename T> __device__ __forceinline__ T tinf() { return T(__builtin_huge_valf()); }
// Reciprocal for the search arithmetic: the hardware reciprocal (1 ulp) in
// FP32, exact division in FP64.  Roots found with it differ from correctly
// rounded division by a few ulp, far inside the tracer's tolerances.
__device__ __forceinline__ float frcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double frcp(double x) { return 1.0 / x; }
template <typename T> __device__ __forceinline__ T fdiv(T a, T b) { return a * frcp(b); }
// 1/sqrt(x) in double from the hardware estimate and two Newton steps
__device__ __forceinline__ double rsqrt_d(double x) {
  double y = __builtin_amdgcn_rsq(x);
  y = y * (1.5 - 0.5 * x * y * y);
  y = y * (1.5 - 0.5 * x * y * y);
  return y;
}
// exp(-x) in double for x >= 0, inline and light on registers: x = n ln2 - r
// with ln 2 split into a head exact in 32 bits and a tail (Cody and Waite's
// reduction), |r| <= ln2 / 2, e^r by its Taylor series to degree 13 (the
// remainder is below 1e-17), times 2^n assembled in the exponent field.
__device__ __forceinline__ double exp_neg(double x) {
  if (!(x < 700.0)) return 0.0;
  const double n = __builtin_rint(x * 1.4426950408889634);   // x / ln 2
  const double r = (n * 0.6931471803691238 - x) + n * 1.9082149292705877e-10;
  double e = 1.0 / 6227020800.0;                                // 1/13!, then Horner
  e = e * r + 1.0 / 479001600.0;
  e = e * r + 1.0 / 39916800.0;
  e = e * r + 1.0 / 3628800.0;
  e = e * r + 1.0 / 362880.0;
  e = e * r + 1.0 / 40320.0;
  e = e * r + 1.0 / 5040.0;
  e = e * r + 1.0 / 720.0;
  e = e * r + 1.0 / 120.0;
  e = e * r + 1.0 / 24.0;
  e = e * r + 1.0 / 6.0;
  e = e * r + 0.5;
  e = e * r + 1.0;
  e = e * r + 1.0;
  return e * __builtin_bit_cast(double, (uint64_t)(1023 - (int64_t)n) << 52);
}

template <typename T> __device__ __forceinline__ bool finite3(V3<T> a) {
  return __builtin_isfinite(a.x) && __builtin_isfinite(a.y) && __builtin_isfinite(a.z);
}

// ------------------------------------------------------------------ Philox4x32-10
// Salmon, Moraes, Dror, Shaw (SC'11): 10 rounds of two 32x32->64 multiplies
// with Weyl-sequence key bumps.  Counter (id lo, id hi, event>>2, tag): tag 1
// for the draw of an interaction, tag 2 for bulk absorption in a lens.
__device__ __forceinline__ uint32_t philox_word(uint64_t seed, uint64_t id, int event, uint32_t tag = 1u) {
  uint32_t c0 = (uint32_t)id, c1 = (uint32_t)(id >> 32), c2 = (uint32_t)(event >> 2), c3 = tag;
  uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r > 0) { k0 += 0x9E3779B9u; k1 += 0xBB67AE85u; }
    // each 32x32 -> 64 product formed whole (one v_mad_u64_u32 rather than
    // a separate high and low multiply)
    const uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0, p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
    uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    uint32_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
    c0 = n0; c1 = lo1; c2 = n2; c3 = lo0;
  }
  int w = event & 3;
  return w == 0 ? c0 : w == 1 ? c1 : w == 2 ? c2 : c3;
}

// Bulk absorption over a segment of length seg in a medium of absorption
// length absl: absorbed iff the photon's tag-2 draw w / 2^32 >= exp(-seg/absl).
// Kept out of line: only photons leaving absorbing glass call it, and its
// registers then stay out of the allocation of the tracing loop.
__device__ __noinline__ bool bulk_absorbed(uint64_t seed, uint64_t id, int k, double seg, double absl) {
  return (double)philox_word(seed, id, k, 2u) * (1.0 / 4294967296.0) >= exp_neg(seg / absl);
}

// ------------------------------------------------------------------ frames and outlines
template <typename T> __device__ __forceinline__ V3<T> loc_p(const DVol<T>& v, V3<T> x) {
  T rx = x.x - v.c[0], ry = x.y - v.c[1], rz = x.z - v.c[2];
  return {v.Q[0] * rx + v.Q[1] * ry + v.Q[2] * rz, v.Q[3] * rx + v.Q[4] * ry + v.Q[5] * rz,
          v.Q[6] * rx + v.Q[7] * ry + v.Q[8] * rz};
}
template <typename T> __device__ __forceinline__ V3<T> loc_d(const DVol<T>& v, V3<T> d) {
  return {v.Q[0] * d.x + v.Q[1] * d.y + v.Q[2] * d.z, v.Q[3] * d.x + v.Q[4] * d.y + v.Q[5] * d.z,
          v.Q[6] * d.x + v.Q[7] * d.y + v.Q[8] * d.z};
}
// Local coordinates of a world point kept in double: the offset from the
// volume origin is formed in double and only then rounded to T, so the local
// point carries the precision of the local scale, not of the world scale.
template <typename T> __device__ __forceinline__ V3<T> loc_pd(const DVol<T>& v, V3<double> x) {
  T rx = (T)(x.x - (double)v.c[0]), ry = (T)(x.y - (double)v.c[1]), rz = (T)(x.z - (double)v.c[2]);
  return {v.Q[0] * rx + v.Q[1] * ry + v.Q[2] * rz, v.Q[3] * rx + v.Q[4] * ry + v.Q[5] * rz,
          v.Q[6] * rx + v.Q[7] * ry + v.Q[8] * rz};
}
// The same in double throughout (frame promoted from the record).
template <typename T> __device__ __forceinline__ V3<double> loc_dd(const DVol<T>& v, V3<double> x) {
  double rx = x.x - (double)v.c[0], ry = x.y - (double)v.c[1], rz = x.z - (double)v.c[2];
  return {(double)v.Q[0] * rx + (double)v.Q[1] * ry + (double)v.Q[2] * rz,
          (double)v.Q[3] * rx + (double)v.Q[4] * ry + (double)v.Q[5] * rz,
          (double)v.Q[6] * rx + (double)v.Q[7] * ry + (double)v.Q[8] * rz};
}
template <typename T> __device__ __forceinline__ V3<double> loc_dir_d(const DVol<T>& v, V3<double> d) {
  return {(double)v.Q[0] * d.x + (double)v.Q[1] * d.y + (double)v.Q[2] * d.z,
          (double)v.Q[3] * d.x + (double)v.Q[4] * d.y + (double)v.Q[5] * d.z,
          (double)v.Q[6] * d.x + (double)v.Q[7] * d.y + (double)v.Q[8] * d.z};
}
template <typename T> __device__ __forceinline__ V3<double> adv(V3<double> o, T t, V3<T> d) {
  return {o.x + (double)t * (double)d.x, o.y + (double)t * (double)d.y, o.z + (double)t * (double)d.z};
}
template <typename T> __device__ __forceinline__ V3<T> to_t(V3<double> a) { return {(T)a.x, (T)a.y, (T)a.z}; }

// Q^T n, normalised (world normal of a local gradient)
template <typename T> __device__ __forceinline__ V3<T> world_n(const DVol<T>& v, V3<T> n) {
  V3<T> w = {v.Q[0] * n.x + v.Q[3] * n.y + v.Q[6] * n.z, v.Q[1] * n.x + v.Q[4] * n.y + v.Q[7] * n.z,
             v.Q[2] * n.x + v.Q[5] * n.y + v.Q[8] * n.z};
  T s = T(1) / dsqrt(dot(w, w));
  return scl(s, w);
}

template <typename T> __device__ __forceinline__ bool inside_outline(const DVol<T>& v, T x, T y) {
  const T* o = v.o;
  switch (v.outline) {
    case OL_NONE: return true;
    case OL_DISC: return x * x + y * y <= o[0];
    case OL_ANNULUS: { T r2 = x * x + y * y; return r2 >= o[0] && r2 <= o[1]; }
    case OL_RECT: return dabs(x) <= o[0] && dabs(y) <= o[1];
    case OL_HEX: {
      const T h = T(0.8660254037844386);
      return dabs(x) <= o[0] && dabs(T(0.5) * x + h * y) <= o[0] && dabs(T(-0.5) * x + h * y) <= o[0];
    }
    case OL_SECTOR: {
      T r2 = x * x + y * y;
      if (r2 < o[0] || r2 > o[1]) return false;
      T c0 = o[2] * y - o[3] * x;   // cross(e0, p) >= 0
      T c1 = x * o[5] - y * o[4];   // cross(p, e1) >= 0
      if (o[6] > T(0)) return !(c0 < T(0) && c1 < T(0));  // sector wider than pi
      return c0 >= T(0) && c1 >= T(0);
    }
  }
  return false;
}

// Conservative test of a straight segment (xa, ya)-(xb, yb) of the local xy
// plane against the outline: false only if no point of the segment can pass
// inside_outline.  Each test is against a convex set (a half-plane, a slab,
// the inside of a circle), for which both endpoints outside means the whole
// segment outside; r^2 along a segment is convex, so both endpoints inside
// the hole means the whole segment is.  Padded by 1e-5 of the outline size
// against rounding of the hit point.
template <typename T>
__device__ __forceinline__ bool segment_may_meet_outline(const DVol<T>& v, T xa, T ya, T xb, T yb) {
  const T* o = v.o;
  switch (v.outline) {
    case OL_ANNULUS: {
      const T hole = o[0] * T(1 - 2e-5);
      return !(xa * xa + ya * ya < hole && xb * xb + yb * yb < hole);
    }
    case OL_SECTOR: {
      const T hole = o[0] * T(1 - 2e-5);
      if (xa * xa + ya * ya < hole && xb * xb + yb * yb < hole) return false;
      if (o[6] > T(0)) return true;
      const T pad = T(1e-5) * v.rout;
      if (o[2] * ya - o[3] * xa < -pad && o[2] * yb - o[3] * xb < -pad) return false;
      if (xa * o[5] - ya * o[4] < -pad && xb * o[5] - yb * o[4] < -pad) return false;
      return true;
    }
    case OL_HEX: {
      const T h = T(0.8660254037844386), lim = o[0] * T(1 + 1e-5);
      const T pa[3] = {xa, T(0.5) * xa + h * ya, T(-0.5) * xa + h * ya};
      const T pb[3] = {xb, T(0.5) * xb + h * yb, T(-0.5) * xb + h * yb};
#pragma unroll
      for (int k = 0; k < 3; ++k)
        if ((pa[k] > lim && pb[k] > lim) || (pa[k] < -lim && pb[k] < -lim)) return false;
      return true;
    }
    default: return true;
  }
}

// ------------------------------------------------------------------ candidate bookkeeping
// Nearest candidate so far: tp, the ray parameter formed in double from the
// box-entry shift and the local root, orders the candidates and places the
// hit point; t is its rounding to T, which the searches in precision T use
// to skip farther candidates (it includes the tie margin).  Candidates
// within `tie` of each other are tied and go to the lower volume, then the
// lower face.
template <typename T> struct Best {
  T t;
  double s;   // cone wall parameter of the hit (its normal depends on it)
  double tp, tie;
  int vol, face;
};

template <typename T> __device__ __forceinline__ void offer(Best<T>& b, T t, int vol, int face, double s, double tp) {
  const double dt = tp - b.tp;
  bool better = dt < -b.tie || (!(dt > b.tie) && (vol < b.vol || (vol == b.vol && face < b.face)));
  // the bound for skipping farther candidates keeps those still tied
  if (better) { b.t = t + (T)b.tie; b.vol = vol; b.face = face; b.s = s; b.tp = tp; }
}

__device__ __forceinline__ void wall_dir(int k, float& nx, float& ny);
__device__ __forceinline__ void wall_dir(int k, double& nx, double& ny);
template <typename C, typename P> __device__ __forceinline__ void sag_eval(const P* p, C u, C& S, C& dS);
template <typename C, typename P> __device__ __forceinline__ void bez_eval(const P* p, C s, C& rho, C& z, C& drho, C& dz);

// Gradient of the face's implicit function at local point x, computed in C
// from the record's parameters: it points to the front side (un-normalised).
// local_grad_of<SH> is the one of shape SH (known where a shape's own root
// solver calls it, which keeps the other shapes' code out of that solver);
// local_grad dispatches on the record's shape.
template <int SH, typename C, typename T>
__device__ __forceinline__ V3<C> local_grad_of(const DVol<T>& v, int face, V3<C> x, C s) {
  if constexpr (SH == PLANE) {
    return {C(0), C(0), C(1)};
  } else if constexpr (SH == SPHERE) {
    C c = (C)v.p[0];
    return {-c * x.x, -c * x.y, C(1) - c * x.z};
  } else if constexpr (SH == ASPHERE) {
    C ir = (C)v.p[9];
    C u = (x.x * x.x + x.y * x.y) * ir;
    C S, dS;
    sag_eval(v.p, u, S, dS);
    C k = dS * C(2) * ir;
    return {-k * x.x, -k * x.y, C(1)};
  } else if constexpr (SH == CYLINDER) {
    return {x.x, x.y, C(0)};
  } else if constexpr (SH == BOX) {
    int ax = face >> 1;
    C sg = (face & 1) ? C(-1) : C(1);
    return {ax == 0 ? sg : C(0), ax == 1 ? sg : C(0), ax == 2 ? sg : C(0)};
  } else {
    C rho, z, dr, dz;
    bez_eval(v.p, s, rho, z, dr, dz);
    C nx, ny;
    wall_dir(face, nx, ny);
    return {-dz * nx, -dz * ny, dr};
  }
}

template <typename C, typename T, int SH = kShapesAll>
__device__ __forceinline__ V3<C> local_grad(const DVol<T>& v, int face, V3<C> x, C s) {
  switch (v.shape) {
    case PLANE: return local_grad_of<PLANE, C>(v, face, x, s);
    case SPHERE: return local_grad_of<SPHERE, C>(v, face, x, s);
    case ASPHERE: return local_grad_of<ASPHERE, C>(v, face, x, s);
    case CYLINDER: return local_grad_of<CYLINDER, C>(v, face, x, s);
    case BOX:
      if constexpr ((SH >> BOX) & 1) return local_grad_of<BOX, C>(v, face, x, s);
      else return {C(0), C(0), C(1)};
    default:
      if constexpr ((SH >> HEXCONE) & 1) return local_grad_of<HEXCONE, C>(v, face, x, s);
      else return {C(0), C(0), C(1)};
  }
}

// The face just left may be met again only beyond eps and only from the side
// the photon is on (side 0: front, 1: back); a root that fails this is the
// departure point itself, displaced by rounding.
struct SelfRule {
  int face;   // face of this volume the photon just left, or -1
  int side;   // side of that face the photon is on
};
template <int SH, typename C, typename T>
__device__ __forceinline__ bool self_ok(const DVol<T>& v, const SelfRule& sr, int face, C tt, C eps, V3<C> x, V3<C> d,
                                        C s) {
  if (face != sr.face) return tt > C(0);
  if (!(tt > eps)) return false;
  C sd = dot(d, local_grad_of<SH, C>(v, face, x, s));
  return (sd < C(0)) == (sr.side == 0);
}

// ------------------------------------------------------------------ narrow phase
// Each function receives the local ray (o, d) already advanced by t0 and offers
// roots t' + t0 in (0, b.t] that pass the self rule.

template <typename T> __device__ __forceinline__ void quad2(T a, T b, T c, T& r0, T& r1, int& n) {
  n = 0;
  if (a == T(0)) {
    if (b != T(0)) { r0 = -fdiv(c, b); n = 1; }
    return;
  }
  T disc = b * b - T(4) * a * c;
  if (disc < T(0)) return;
  T q = T(-0.5) * (b + dcopysign(dsqrt(disc), b));
  if (q == T(0)) { r0 = T(0); n = 1; return; }
  r0 = fdiv(q, a); r1 = fdiv(c, q); n = 2;
}

template <typename T> __device__ __forceinline__ void nf_plane(const DVol<T>& v, int vid, V3<T> o, V3<T> d,
                                                               T t0, T eps, SelfRule sr, Best<T>& b) {
  if (d.z == T(0)) return;
  T t = -fdiv(o.z, d.z);
  T tt = t + t0;
  if (tt > b.t) return;
  V3<T> x = fma3(t, d, o);
  if (!self_ok<PLANE>(v, sr, 0, tt, eps, x, d, T(0))) return;
  if (inside_outline(v, x.x, x.y)) offer(b, tt, vid, 0, T(0), (double)t0 + (double)t);
}

template <typename T> __device__ __forceinline__ void nf_sphere(const DVol<T>& v, int vid, V3<T> o, V3<T> d,
                                                                T t0, T eps, SelfRule sr, Best<T>& b) {
  T cv = v.p[0];
  T a = T(-0.5) * cv * dot(d, d), bb = d.z - cv * dot(o, d), c = o.z - T(0.5) * cv * dot(o, o);
  T r[2]; int n;
  quad2(a, bb, c, r[0], r[1], n);
  for (int i = 0; i < n; ++i) {
    T tt = r[i] + t0;
    if (tt > b.t) continue;
    V3<T> x = fma3(r[i], d, o);
    if (T(1) - cv * x.z < T(0)) continue;
    if (!self_ok<SPHERE>(v, sr, 0, tt, eps, x, d, T(0))) continue;
    if (inside_outline(v, x.x, x.y)) offer(b, tt, vid, 0, T(0), (double)t0 + (double)r[i]);
  }
}

template <typename C, typename P> __device__ __forceinline__ void sag_eval(const P* p, C u, C& S, C& dS) {
  // S = sum_{i=1..8} b_i u^i, dS = dS/du ; p[1..8] = b_i
  C s = (C)p[8], ds = C(8) * (C)p[8];
#pragma unroll
  for (int i = 7; i >= 1; --i) { s = s * u + (C)p[i]; ds = ds * u + C(i) * (C)p[i]; }
  S = s * u; dS = ds;
}

// g(t) = z(t) - S(u(t)), u = (x^2 + y^2)/rn^2
template <typename T> __device__ __forceinline__ void asph_g(const DVol<T>& v, V3<T> o, V3<T> d, T t, T& g, T& gp) {
  T x = o.x + t * d.x, y = o.y + t * d.y, z = o.z + t * d.z;
  T u = (x * x + y * y) * v.p[9];
  T S, dS;
  sag_eval(v.p, u, S, dS);
  g = z - S;
  gp = d.z - dS * T(2) * v.p[9] * (x * d.x + y * d.y);
}

template <typename T> __device__ __forceinline__ void nf_asphere(const DVol<T>& v, int vid, V3<T> o, V3<T> d,
                                                                 T t0, T eps, SelfRule sr, Best<T>& b) {
  // bracket: local z-slab of the surface and the cylinder r <= rout
  T tlo = sr.face == 0 ? eps : T(0);
  T ta = tlo - t0, tb = b.t - t0;
  if (d.z != T(0)) {
    T iz = frcp(d.z);
    T t1 = (v.lo[2] - o.z) * iz, t2 = (v.hi[2] - o.z) * iz;
    ta = dmax(ta, dmin(t1, t2)); tb = dmin(tb, dmax(t1, t2));
  } else if (o.z < v.lo[2] || o.z > v.hi[2]) {
    return;
  }
  T A = d.x * d.x + d.y * d.y, B = T(2) * (o.x * d.x + o.y * d.y), C = o.x * o.x + o.y * o.y - v.rout * v.rout;
  if (A > T(0)) {
    T r0, r1; int n;
    quad2(A, B, C, r0, r1, n);
    if (n < 2) return;
    ta = dmax(ta, dmin(r0, r1)); tb = dmin(tb, dmax(r0, r1));
  } else if (C > T(0)) {
    return;
  }
  if (!(ta <= tb)) return;
  // the hit lies on [ta, tb]; skip the solve if that piece of the ray misses
  // the outline (a neighbouring segment of a segmented mirror)
  if (!segment_may_meet_outline(v, o.x + ta * d.x, o.y + ta * d.y, o.x + tb * d.x, o.y + tb * d.y)) return;
  T ga, gpa, gb, gpb;
  asph_g(v, o, d, ta, ga, gpa);
  asph_g(v, o, d, tb, gb, gpb);
  if ((ga > T(0)) == (gb > T(0))) {
    // no sign change; with |d_z| > slope |d_xy| g is monotone, so no root
    if (dabs(d.z) > v.slope * dsqrt(A)) return;
    // grazing ray: first sign change on a uniform subdivision
    const int K = 16;
    T h = (tb - ta) / T(K), tp = ta, gprev = ga;
    bool found = false;
    for (int k = 1; k <= K; ++k) {
      T tk = k == K ? tb : ta + h * T(k);
      T gk, gpk;
      asph_g(v, o, d, tk, gk, gpk);
      if ((gk > T(0)) != (gprev > T(0))) { ta = tp; tb = tk; ga = gprev; gb = gk; found = true; break; }
      tp = tk; gprev = gk;
    }
    if (!found) return;
  }
  // safeguarded Newton on [ta, tb]
  T a = ta, bnd = tb, ga_ = ga;
  T t = (gb - ga) != T(0) ? ta - ga * fdiv(tb - ta, gb - ga) : T(0.5) * (ta + tb);
  const T tol = sizeof(T) == 4 ? T(2e-7) : T(1e-15);
  for (int it = 0; it < 24; ++it) {
    T g, gp;
    asph_g(v, o, d, t, g, gp);
    if (g == T(0)) break;
    if ((g > T(0)) == (ga_ > T(0))) { a = t; ga_ = g; } else { bnd = t; }
    T tn = gp != T(0) ? t - fdiv(g, gp) : T(0.5) * (a + bnd);
    // t is now an end of the bracket: at Newton's fixed point tn == t, which
    // must count as inside (a zero step ends the loop), not send it bisecting
    if (!(tn >= dmin(a, bnd) && tn <= dmax(a, bnd))) tn = T(0.5) * (a + bnd);
    T dt = tn - t;
    t = tn;
    if (dabs(dt) <= tol * (dabs(t) + dabs(t0) + T(1e-30))) break;
  }
  T tt = t + t0;
  if (tt > b.t) return;
  V3<T> x = fma3(t, d, o);
  if (!self_ok<ASPHERE>(v, sr, 0, tt, eps, x, d, T(0))) return;
  if (inside_outline(v, x.x, x.y)) offer(b, tt, vid, 0, T(0), (double)t0 + (double)t);
}

// Cylinders (masts, trusses) are solved in double for every scene
// precision: a ray running nearly along a long strut meets it at glancing
// incidence, where the hit point along the axis carries the rounding of the
// local coordinates (metres from the strut's base) divided by |d . n|.
template <typename C, typename T> __device__ __forceinline__ void nf_cylinder(const DVol<T>& v, int vid, V3<C> o,
                                                                              V3<C> d, C t0, C eps, SelfRule sr,
                                                                              Best<T>& b) {
  C A = d.x * d.x + d.y * d.y;
  if (A == C(0)) return;
  const C rho = (C)v.p[0];
  C B = C(2) * (o.x * d.x + o.y * d.y), Cq = o.x * o.x + o.y * o.y - rho * rho;
  C r[2]; int n;
  quad2(A, B, Cq, r[0], r[1], n);
  const C tbest = (C)(b.tp + b.tie);
  for (int i = 0; i < n; ++i) {
    C tt = r[i] + t0;
    if (tt > tbest) continue;
    V3<C> x = fma3(r[i], d, o);
    if (!self_ok<CYLINDER>(v, sr, 0, tt, eps, x, d, C(0))) continue;
    if (x.z >= C(0) && x.z <= (C)v.p[1]) offer(b, (T)tt, vid, 0, T(0), (double)tt);
  }
}

template <typename T> __device__ __forceinline__ void nf_box(const DVol<T>& v, int vid, V3<T> o, V3<T> d,
                                                             T t0, T eps, SelfRule sr, Best<T>& b) {
  const T oa[3] = {o.x, o.y, o.z}, da[3] = {d.x, d.y, d.z};
  for (int f = 0; f < 6; ++f) {
    int ax = f >> 1;
    T sgn = (f & 1) ? T(-1) : T(1);
    if (da[ax] == T(0)) continue;
    T t = fdiv(sgn * v.p[ax] - oa[ax], da[ax]);
    T tt = t + t0;
    if (tt > b.t) continue;
    if (!self_ok<BOX>(v, sr, f, tt, eps, fma3(t, d, o), d, T(0))) continue;
    bool ok = true;
#pragma unroll
    for (int k = 0; k < 3; ++k)
      if (k != ax && dabs(oa[k] + t * da[k]) > v.p[k]) ok = false;
    if (ok) offer(b, tt, vid, f, T(0), (double)t0 + (double)t);
  }
}

template <typename C, typename P> __device__ __forceinline__ void bez_eval(const P* pp, C s, C& rho, C& z, C& drho, C& dz) {
  C p[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) p[i] = (C)pp[i];
  C a = C(1) - s;
  C b0 = a * a * a, b1 = C(3) * a * a * s, b2 = C(3) * a * s * s, b3 = s * s * s;
  rho = b0 * p[0] + b1 * p[2] + b2 * p[4] + b3 * p[6];
  z = b0 * p[1] + b1 * p[3] + b2 * p[5] + b3 * p[7];
  C d0 = C(3) * a * a, d1 = C(6) * a * s, d2 = C(3) * s * s;
  drho = d0 * (p[2] - p[0]) + d1 * (p[4] - p[2]) + d2 * (p[6] - p[4]);
  dz = d0 * (p[3] - p[1]) + d1 * (p[5] - p[3]) + d2 * (p[7] - p[5]);
}

__device__ __forceinline__ void wall_dir(int k, float& nx, float& ny) {
  const float cs[6] = {1.f, 0.5f, -0.5f, -1.f, -0.5f, 0.5f};
  const float sn[6] = {0.f, 0.8660254037844386f, 0.8660254037844386f, 0.f, -0.8660254037844386f, -0.8660254037844386f};
  nx = cs[k]; ny = sn[k];
}
__device__ __forceinline__ void wall_dir(int k, double& nx, double& ny) {
  const double cs[6] = {1.0, 0.5, -0.5, -1.0, -0.5, 0.5};
  const double sn[6] = {0.0, 0.8660254037844386, 0.8660254037844386, 0.0, -0.8660254037844386, -0.8660254037844386};
  nx = cs[k]; ny = sn[k];
}

// root of the cubic (power basis) on the monotone piece [a, b] with a sign change
// Cubic in Bernstein form, F(s) = sum_k w_k B_k(s), and its derivative.  The
// Bernstein form keeps the value accurate near s = 0 and s = 1 (the exit and
// entrance rims), where the power-basis coefficients cancel.
template <typename T> __device__ __forceinline__ void bern3(const T* w, T s, T& f, T& fp) {
  T a = T(1) - s;
  T b0 = a * a, b1 = T(2) * a * s, b2 = s * s;
  f = a * (b0 * w[0] + T(3) * a * s * w[1]) + s * (T(3) * a * s * w[2] + b2 * w[3]);
  fp = T(3) * (b0 * (w[1] - w[0]) + b1 * (w[2] - w[1]) + b2 * (w[3] - w[2]));
}

// root of F on the monotone piece [a, b] with a sign change, safeguarded Newton
template <typename T> __device__ __forceinline__ T cubic_root_piece(const T* w, T a, T b, T fa) {
  T s = T(0.5) * (a + b);
  for (int it = 0; it < 40; ++it) {
    T f, fp;
    bern3(w, s, f, fp);
    if (f == T(0)) break;
    if ((f > T(0)) == (fa > T(0))) { a = s; fa = f; } else { b = s; }
    T sn = fp != T(0) ? s - fdiv(f, fp) : T(0.5) * (a + b);
    if (!(sn >= a && sn <= b)) sn = T(0.5) * (a + b);   // s is an end: a fixed point stays put
    T ds = sn - s;
    s = sn;
    // s lies in [0, 1]: a double step below 1e-14 leaves an error far under
    // the tie margin of the search (a tolerance at the rounding unit would
    // never be met by an iteration that alternates between neighbours)
    if (dabs(ds) <= (sizeof(T) == 4 ? T(1e-7) : T(1e-14))) break;
  }
  return s;
}

// One wall of a hex cone against the local ray: the wall's cubic in Bernstein
// form (zero where the ray meets the wall's surface of revolution cut by the
// wall plane) and its monotone pieces, split at the critical points in
// (0, 1).  False when the cubic vanishes identically.
template <typename C> struct ConeWall {
  C nx, ny, u0, du;
  C w[4];
  C br[4];
  int nb;
};

template <typename C, typename P>
__device__ __forceinline__ bool cone_wall(const P* p, int f, V3<C> o, V3<C> d, ConeWall<C>& W) {
  wall_dir(f, W.nx, W.ny);
  W.u0 = o.x * W.nx + o.y * W.ny;
  W.du = d.x * W.nx + d.y * W.ny;
#pragma unroll
  for (int k = 0; k < 4; ++k) W.w[k] = ((C)p[2 * k] - W.u0) * d.z - ((C)p[2 * k + 1] - o.z) * W.du;
  if (W.w[0] == C(0) && W.w[1] == C(0) && W.w[2] == C(0) && W.w[3] == C(0)) return false;
  // power-basis coefficients, used only to find the critical points
  const C c1 = C(3) * (W.w[1] - W.w[0]), c2 = C(3) * (W.w[0] - C(2) * W.w[1] + W.w[2]);
  const C c3 = W.w[3] - C(3) * W.w[2] + C(3) * W.w[1] - W.w[0];
  W.nb = 0;
  W.br[W.nb++] = C(0);
  C q0, q1;
  int nq;
  quad2(C(3) * c3, C(2) * c2, c1, q0, q1, nq);
  if (nq == 2 && q0 > q1) { C tq = q0; q0 = q1; q1 = tq; }
  if (nq >= 1 && q0 > C(0) && q0 < C(1)) W.br[W.nb++] = q0;
  if (nq == 2 && q1 > C(0) && q1 < C(1)) W.br[W.nb++] = q1;
  W.br[W.nb++] = C(1);
  return true;
}

// The wall point at parameter s: offered if it lies ahead within the current
// best, passes the self rule and lies within the wall's hexagon sector.
template <typename C, typename T>
__device__ __forceinline__ void cone_hit(const DVol<T>& v, int vid, const ConeWall<C>& W, int f, C s, V3<C> o,
                                         V3<C> d, C t0, C eps, C tbest, SelfRule sr, Best<T>& b) {
  const C inv_sqrt3 = C(0.5773502691896258);
  C rho, z, dr, dzs;
  bez_eval(v.p, s, rho, z, dr, dzs);
  C t = dabs(d.z) >= dabs(W.du) ? fdiv(z - o.z, d.z) : fdiv(rho - W.u0, W.du);
  C tt = t + t0;
  if (tt > tbest) return;
  V3<C> xh = fma3(t, d, o);
  if (!self_ok<HEXCONE>(v, sr, f, tt, eps, xh, d, s)) return;
  C vt = -xh.x * W.ny + xh.y * W.nx;
  if (dabs(vt) <= rho * inv_sqrt3) offer(b, (T)tt, vid, f, (double)s, (double)tt);
}

// The walls are solved in double for every scene precision: neighbouring
// cones of an array share their entrance rims, where one cone's wall and the
// next one's meet tangentially, so near a rim the two candidate roots differ
// by the square of the depth below it -- below what single precision can
// order at the cones' size.  Local coordinates come from the photon position
// in double; the record's parameters are promoted as they are read.
template <typename C, typename T> __device__ __forceinline__ void nf_hexcone(const DVol<T>& v, int vid, V3<C> o, V3<C> d,
                                                                             C t0, C eps, SelfRule sr, Best<T>& b) {
  const T* p = v.p;
  const C tbest = (C)(b.tp + b.tie);
  {
    // the walls lie inside the hexagonal prism |x . n_k| <= rho_max,
    // z in [lo, hi]: skip the cone unless the ray crosses it before the best
    C rm = (C)dmax(dmax(p[0], p[2]), dmax(p[4], p[6]));
    C ta = -t0, tb = tbest - t0;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      C nx, ny;
      wall_dir(k, nx, ny);
      C u0 = o.x * nx + o.y * ny, du = d.x * nx + d.y * ny;
      if (du != C(0)) {
        C iu = frcp(du);
        C t1 = (-rm - u0) * iu, t2 = (rm - u0) * iu;
        ta = dmax(ta, dmin(t1, t2)); tb = dmin(tb, dmax(t1, t2));
      } else if (dabs(u0) > rm) {
        return;
      }
    }
    if (d.z != C(0)) {
      C iz = frcp(d.z);
      C t1 = ((C)v.lo[2] - o.z) * iz, t2 = ((C)v.hi[2] - o.z) * iz;
      ta = dmax(ta, dmin(t1, t2)); tb = dmin(tb, dmax(t1, t2));
    } else if (o.z < (C)v.lo[2] || o.z > (C)v.hi[2]) {
      return;
    }
    if (!(ta <= tb)) return;
  }
  // Every wall's monotone pieces first: a root at a piece's end is taken at
  // once, a piece with a sign change inside is listed (bit 3 f + i) and all
  // listed pieces are solved afterwards in one loop, so that the lanes of a
  // wave run their Newton iterations side by side rather than one wall and
  // one piece at a time.
  uint32_t todo = 0;
  for (int f = 0; f < 6; ++f) {
    ConeWall<C> W;
    if (!cone_wall(p, f, o, d, W)) continue;
    C fa = W.w[0];
    for (int i = 0; i + 1 < W.nb; ++i) {
      C fb, fpb;
      bern3(W.w, W.br[i + 1], fb, fpb);
      if (fa == C(0)) cone_hit(v, vid, W, f, W.br[i], o, d, t0, eps, tbest, sr, b);
      else if (fb == C(0) && i + 2 == W.nb) cone_hit(v, vid, W, f, W.br[i + 1], o, d, t0, eps, tbest, sr, b);
      else if ((fa > C(0)) != (fb > C(0))) todo |= 1u << (3 * f + i);
      fa = fb;
    }
  }
  while (todo) {
    const int j = __builtin_ctz(todo);
    todo &= todo - 1u;
    const int f = j / 3, i = j - 3 * f;
    ConeWall<C> W;
    cone_wall(p, f, o, d, W);
    C fa, fpa;
    bern3(W.w, W.br[i], fa, fpa);
    const C s = cubic_root_piece(W.w, W.br[i], W.br[i + 1], fa);
    cone_hit(v, vid, W, f, s, o, d, t0, eps, tbest, sr, b);
  }
}

// world AABB slab test: entry parameter, or -1 if the box is missed in (0, tmax]
template <typename T> __device__ __forceinline__ bool aabb(const DVol<T>& v, V3<T> o, V3<T> inv, T tmax, T& tin) {
  T t1 = (v.bmin[0] - o.x) * inv.x, t2 = (v.bmax[0] - o.x) * inv.x;
  T lo = dmin(t1, t2), hi = dmax(t1, t2);
  t1 = (v.bmin[1] - o.y) * inv.y; t2 = (v.bmax[1] - o.y) * inv.y;
  lo = dmax(lo, dmin(t1, t2)); hi = dmin(hi, dmax(t1, t2));
  t1 = (v.bmin[2] - o.z) * inv.z; t2 = (v.bmax[2] - o.z) * inv.z;
  lo = dmax(lo, dmin(t1, t2)); hi = dmin(hi, dmax(t1, t2));
  tin = dmax(lo, T(0));
  return hi >= tin && tin <= tmax;
}

// Exact test of one volume; offers its nearest valid face root to b.
// The photon position O is kept in double (world scale); of and inv are its
// rounding and the inverse direction in T for the box tests.
template <typename T, int SH = kShapesAll>
__device__ __forceinline__ void narrow(const DVol<T>& v, int vid, V3<double> O, V3<double> D, V3<T> d,
                                                             T tin, int prev_vol, int prev_face, int prev_side,
                                                             T eps, Best<T>& b) {
  // advance to the box entry to keep the local quadratic well conditioned;
  // planes are not advanced, so coincident planes with the same z-row give
  // bit-identical t and the tie goes to the lower volume id
  T t0 = v.shape == PLANE ? T(0) : tin;
  V3<T> ol = loc_pd(v, adv(O, t0, d)), dl = loc_d(v, d);
  SelfRule sr{vid == prev_vol ? prev_face : -1, prev_side};
  switch (v.shape) {
    case PLANE: nf_plane(v, vid, ol, dl, t0, eps, sr, b); break;
    case SPHERE: nf_sphere(v, vid, ol, dl, t0, eps, sr, b); break;
    case ASPHERE: nf_asphere(v, vid, ol, dl, t0, eps, sr, b); break;
    case CYLINDER: {
      // the origin in double carries the precision; the direction rounded to
      // T is enough here (kernels without cones then keep no double direction)
      const V3<double> Dc = ((SH >> HEXCONE) & 1) ? D : V3<double>{(double)d.x, (double)d.y, (double)d.z};
      const V3<double> Ot = {O.x + (double)t0 * Dc.x, O.y + (double)t0 * Dc.y, O.z + (double)t0 * Dc.z};
      nf_cylinder<double>(v, vid, loc_dd(v, Ot), loc_dir_d(v, Dc), (double)t0, (double)eps, sr, b);
      break;
    }
    case BOX:
      if constexpr ((SH >> BOX) & 1) nf_box(v, vid, ol, dl, t0, eps, sr, b);
      break;
    case HEXCONE:
      if constexpr ((SH >> HEXCONE) & 1) {
        // the photon's direction in double too: near a shared rim the two
        // walls' order depends on where the ray passes to well below the
        // rounding of the direction to T over a cone's length
        const V3<double> Ot = {O.x + (double)t0 * D.x, O.y + (double)t0 * D.y, O.z + (double)t0 * D.z};
        nf_hexcone<double>(v, vid, loc_dd(v, Ot), loc_dir_d(v, D), (double)t0, (double)eps, sr, b);
      }
      break;
  }
}

template <typename T, int SH = kShapesAll> __device__ __forceinline__ void test_volume(const DVol<T>& v, int vid, V3<double> O,
                                                                  V3<double> D, V3<T> of, V3<T> d, V3<T> inv,
                                                                  int prev_vol, int prev_face, int prev_side, T eps,
                                                                  Best<T>& b) {
  T tin;
  if (!aabb(v, of, inv, b.t, tin)) return;
  narrow<T, SH>(v, vid, O, D, d, tin, prev_vol, prev_face, prev_side, eps, b);
}

template <typename T> __device__ __forceinline__ V3<T> inv_dir(V3<T> d) {
  return {frcp(d.x), frcp(d.y), frcp(d.z)};
}

// Non-sequential search: nearest face over the always-list and the grid
// cells crossed by the ray's XY projection.
// Recently tested volumes: a volume listed in several grid cells crossed by
// one ray is tested once per search.
struct Mailbox {
  int m0, m1, m2, m3;
  __device__ __forceinline__ bool seen(int v) const { return v == m0 || v == m1 || v == m2 || v == m3; }
  __device__ __forceinline__ void put(int v) { m3 = m2; m2 = m1; m1 = m0; m0 = v; }
};

// Candidates of one search, gathered before any exact test so that every
// lane of a wave runs the exact tests in one loop at one code site, nearest
// box entry first.  The arrays are only indexed through unrolled selects, so
// they stay in VGPRs.
template <typename T> struct Cands {
  static constexpr int K = 6;
  int vid[K];
  T tin[K];
  int n;
};

template <typename T, int SH = kShapesAll>
__device__ __forceinline__ void run_cands(const SceneView<T>& S, Cands<T>& c, V3<double> O, V3<double> D, V3<T> d,
                                          int prev_vol,
                                          int prev_face, int prev_side, Best<T>& b) {
#pragma unroll 1
  for (int it = 0; it < c.n; ++it) {
    int vid = -1, sel = 0;
    T tin = tinf<T>();
#pragma unroll
    for (int j = 0; j < Cands<T>::K; ++j)
      if (j < c.n && c.tin[j] < tin) { tin = c.tin[j]; vid = c.vid[j]; sel = j; }
#pragma unroll
    for (int j = 0; j < Cands<T>::K; ++j)
      if (j == sel) c.tin[j] = tinf<T>();
    if (vid < 0 || tin > b.t) break;
    narrow<T, SH>(S.vol[vid], vid, O, D, d, tin, prev_vol, prev_face, prev_side, S.eps_self, b);
  }
  c.n = 0;
}

// Conservative cull of a hex cone before its exact test: its walls lie
// inside the hexagonal prism |x . n_k| <= rho_max over its local z range.
// Narrows tin (the box entry) to the ray's entry into that prism, padded by
// 1e-4 of the cone's size so that rounding to T cannot cull a wall hit;
// false when the ray misses the prism before tmax.  Run for every gathered
// cone, it keeps neighbouring cones (whose boxes overlap the one the photon
// is in) out of the candidate list, so that the lanes of a wave run few
// exact cone tests.
template <typename T>
__device__ __forceinline__ bool cone_prism(const DVol<T>& v, V3<double> O, V3<T> d, T tmax, T& tin) {
  const T* p = v.p;
  const T rm = dmax(dmax(p[0], p[2]), dmax(p[4], p[6]));
  const T pad = T(1e-4) * (rm + v.hi[2] - v.lo[2]);
  const V3<T> ol = loc_pd(v, O), dl = loc_d(v, d);
  T ta = tin, tb = tmax;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    T nx, ny;
    wall_dir(k, nx, ny);
    const T u0 = ol.x * nx + ol.y * ny, du = dl.x * nx + dl.y * ny;
    if (du != T(0)) {
      const T iu = frcp(du);
      const T t1 = (-rm - pad - u0) * iu, t2 = (rm + pad - u0) * iu;
      ta = dmax(ta, dmin(t1, t2));
      tb = dmin(tb, dmax(t1, t2));
    } else if (dabs(u0) > rm + pad) {
      return false;
    }
  }
  if (dl.z != T(0)) {
    const T iz = frcp(dl.z);
    const T t1 = (v.lo[2] - pad - ol.z) * iz, t2 = (v.hi[2] + pad - ol.z) * iz;
    ta = dmax(ta, dmin(t1, t2));
    tb = dmin(tb, dmax(t1, t2));
  } else if (ol.z < v.lo[2] - pad || ol.z > v.hi[2] + pad) {
    return false;
  }
  if (!(ta <= tb)) return false;
  tin = ta;
  return true;
}

template <typename T, int SH = kShapesAll>
__device__ __forceinline__ void gather(const SceneView<T>& S, Cands<T>& c, int vid, V3<T> o, V3<T> inv, V3<double> O,
                                       V3<double> D, V3<T> d, int prev_vol, int prev_face, int prev_side, Best<T>& b) {
  T tin;
  if (!aabb(S.vol[vid], o, inv, b.t, tin)) return;
  if constexpr (((SH >> HEXCONE) & 1) != 0) {
    if (S.vol[vid].shape == HEXCONE && !cone_prism(S.vol[vid], O, d, b.t, tin)) return;
  }
  if (c.n == Cands<T>::K) run_cands<T, SH>(S, c, O, D, d, prev_vol, prev_face, prev_side, b);
#pragma unroll
  for (int j = 0; j < Cands<T>::K; ++j)
    if (j == c.n) { c.vid[j] = vid; c.tin[j] = tin; }
  ++c.n;
}

// Non-sequential search: nearest face over the volume just left, the
// always-list and the candidate groups crossed by the ray.
// Inlined into its callers on purpose: as a called function it would take
// the scene view and the best hit through the stack (scratch memory), which
// the compiler does for the all-shape kernels if left to decide.
template <typename T, int SH = kShapesAll>
__device__ __forceinline__ void find_nearest(const SceneView<T>& S, V3<double> O, V3<double> D, int prev_vol,
                                                   int prev_face, int prev_side, Best<T>& b) {
  b.t = tinf<T>(); b.vol = -1; b.face = -1; b.s = 0.0; b.tp = tinf<double>(); b.tie = S.eps_tie;
  const V3<T> d = to_t<T>(D);
  Mailbox mb{prev_vol, -1, -1, -1};
  V3<T> inv = inv_dir(d);
  const V3<T> o = to_t<T>(O);
  Cands<T> c;
  c.n = 0;
  // the volume just left first: photons bouncing inside a cone or between
  // facets usually meet it (or its neighbour) next
  if (prev_vol >= 0) gather<T, SH>(S, c, prev_vol, o, inv, O, D, d, prev_vol, prev_face, prev_side, b);
  for (int i = 0; i < S.n_always; ++i) {
    int vid = S.always[i];
    if (vid != prev_vol) gather<T, SH>(S, c, vid, o, inv, O, D, d, prev_vol, prev_face, prev_side, b);
  }
  // candidate groups: walk each group's grid over the stretch of the ray that
  // lies inside the group's z-slab (in the group frame)
  for (int gi = 0; gi < S.n_grp; ++gi) {
    const GroupRec<T>& G = S.groups[gi];
    T rx = (T)(O.x - (double)G.c[0]), ry = (T)(O.y - (double)G.c[1]), rz = (T)(O.z - (double)G.c[2]);
    // the slab first: most searches cross only some groups' slabs
    T goz = G.Q[6] * rx + G.Q[7] * ry + G.Q[8] * rz, gdz = G.Q[6] * d.x + G.Q[7] * d.y + G.Q[8] * d.z;
    T ta = T(0), tb = b.t;
    if (gdz != T(0)) {
      T iz = frcp(gdz);
      T t1 = (G.zmin - goz) * iz, t2 = (G.zmax - goz) * iz;
      ta = dmax(ta, dmin(t1, t2)); tb = dmin(tb, dmax(t1, t2));
    } else if (goz < G.zmin || goz > G.zmax) {
      continue;
    }
    if (!(ta <= tb)) continue;
    V3<T> go = {G.Q[0] * rx + G.Q[1] * ry + G.Q[2] * rz, G.Q[3] * rx + G.Q[4] * ry + G.Q[5] * rz, goz};
    V3<T> gd = {G.Q[0] * d.x + G.Q[1] * d.y + G.Q[2] * d.z, G.Q[3] * d.x + G.Q[4] * d.y + G.Q[5] * d.z, gdz};
    T gx1 = G.x0 + T(G.nx) * G.cell, gy1 = G.y0 + T(G.ny) * G.cell;
    T ix_ = T(0), iy_ = T(0);
    if (gd.x != T(0)) {
      ix_ = frcp(gd.x);
      T t1 = (G.x0 - go.x) * ix_, t2 = (gx1 - go.x) * ix_;
      ta = dmax(ta, dmin(t1, t2)); tb = dmin(tb, dmax(t1, t2));
    } else if (go.x < G.x0 || go.x > gx1) {
      continue;
    }
    if (gd.y != T(0)) {
      iy_ = frcp(gd.y);
      T t1 = (G.y0 - go.y) * iy_, t2 = (gy1 - go.y) * iy_;
      ta = dmax(ta, dmin(t1, t2)); tb = dmin(tb, dmax(t1, t2));
    } else if (go.y < G.y0 || go.y > gy1) {
      continue;
    }
    if (!(ta <= tb)) continue;
    T px = go.x + ta * gd.x, py = go.y + ta * gd.y;
    int ix = (int)dfloor((px - G.x0) * G.inv_cell), iy = (int)dfloor((py - G.y0) * G.inv_cell);
    ix = ix < 0 ? 0 : (ix >= G.nx ? G.nx - 1 : ix);
    iy = iy < 0 ? 0 : (iy >= G.ny ? G.ny - 1 : iy);
    int sx = gd.x > T(0) ? 1 : -1, sy = gd.y > T(0) ? 1 : -1;
    T tmx = gd.x != T(0) ? (G.x0 + T(ix + (gd.x > T(0) ? 1 : 0)) * G.cell - go.x) * ix_ : tinf<T>();
    T tmy = gd.y != T(0) ? (G.y0 + T(iy + (gd.y > T(0) ? 1 : 0)) * G.cell - go.y) * iy_ : tinf<T>();
    T tdx = gd.x != T(0) ? G.cell * dabs(ix_) : tinf<T>();
    T tdy = gd.y != T(0) ? G.cell * dabs(iy_) : tinf<T>();
    int guard = G.nx + G.ny + 2;
    while (guard-- > 0) {
      uint32_t cell = G.start + (uint32_t)(iy * G.nx + ix);
      uint32_t i0 = S.cell_start[cell], i1 = S.cell_start[cell + 1];
      for (uint32_t k = i0; k < i1; ++k) {
        int vid = S.items[k];
        if (!mb.seen(vid)) {
          mb.put(vid);
          gather<T, SH>(S, c, vid, o, inv, O, D, d, prev_vol, prev_face, prev_side, b);
        }
      }
      T tn = dmin(tmx, tmy);
      if (tn > tb || tn >= b.t) break;
      if (tmx < tmy) { ix += sx; tmx += tdx; if (ix < 0 || ix >= G.nx) break; }
      else { iy += sy; tmy += tdy; if (iy < 0 || iy >= G.ny) break; }
    }
  }
  run_cands<T, SH>(S, c, O, D, d, prev_vol, prev_face, prev_side, b);
}

// Front normal (world, double) of the face hit at world point X (double):
// local point, gradient and normalisation in double from the record.
template <typename T, int SH = kShapesAll>
__device__ __forceinline__ V3<double> front_normal(const DVol<T>& v, int face, V3<double> X,
                                                                        double s) {
  double rx = X.x - (double)v.c[0], ry = X.y - (double)v.c[1], rz = X.z - (double)v.c[2];
  double Q[9];
#pragma unroll
  for (int i = 0; i < 9; ++i) Q[i] = (double)v.Q[i];
  V3<double> x = {Q[0] * rx + Q[1] * ry + Q[2] * rz, Q[3] * rx + Q[4] * ry + Q[5] * rz,
                  Q[6] * rx + Q[7] * ry + Q[8] * rz};
  V3<double> g = local_grad<double, T, SH>(v, face, x, s);
  V3<double> w = {Q[0] * g.x + Q[3] * g.y + Q[6] * g.z, Q[1] * g.x + Q[4] * g.y + Q[7] * g.z,
                  Q[2] * g.x + Q[5] * g.y + Q[8] * g.z};
  return scl(rsqrt_d(dot(w, w)), w);
}

template <typename T> __device__ __forceinline__ T fresnel_R(T cos_i, T n1, T n2, T& cos_t) {
  T eta = n1 / n2;
  T s2 = eta * eta * (T(1) - cos_i * cos_i);
  if (s2 >= T(1)) { cos_t = T(0); return T(1); }
  cos_t = dsqrt(T(1) - s2);
  T rs = (n1 * cos_i - n2 * cos_t) / (n1 * cos_i + n2 * cos_t);
  T rp = (n2 * cos_i - n1 * cos_t) / (n2 * cos_i + n1 * cos_t);
  return T(0.5) * (rs * rs + rp * rp);
}

enum { ACT_REFLECT = 0, ACT_REFRACT = 1, ACT_STOP = 2 };

// Index of a lens volume's medium for a photon of wavelength lam (metres;
// 0: the photon carries none): the lens's dispersion law A + B / lam^2 when
// it has one and the kernel carries wavelengths, else its fixed index.
template <int SH, typename T> __device__ __forceinline__ double lens_index(const DVol<T>& v, double lam) {
  if constexpr ((SH & kLambda) != 0) {
    if (lam > 0.0 && v.p[11] != T(0)) return (double)v.p[10] + (double)v.p[11] / (lam * lam);
  }
  return (double)v.n_in;
}

// Apply the interaction of the event at X on (vol, face).  Updates d, ncur,
// fate; returns the action.  `back` is set from the side the photon came from;
// seg is the length of the segment that ends at this event.
template <typename C, typename T> __device__ __forceinline__ int interact(const DVol<T>& v, V3<C> n, V3<C>& d,
                                                                          C& ncur, int& fate, int& back,
                                                                          uint64_t seed, uint64_t id, int k,
                                                                          double seg, C nlens) {
  C dn = dot(d, n);
  back = dn < C(0) ? 0 : 1;
  switch (v.role) {
    case FOCAL: fate = back ? ABSORBED : FOCUSED; return ACT_STOP;
    case OBSCURATION: fate = ABSORBED; return ACT_STOP;
    case MIRROR: {
      if (back) { fate = ABSORBED; return ACT_STOP; }
      if (!v.always_reflect) {
        uint32_t u = philox_word(seed, id, k);
        if (u >= v.thr) { fate = ABSORBED; return ACT_STOP; }
      }
      d = fma3(C(-2) * dn, n, d);
      return ACT_REFLECT;
    }
    case LENS: {
      // bulk absorption: a photon reaching the face from inside survived the
      // segment through the glass with probability exp(-seg / absl)
      if (back && v.absl > T(0) && bulk_absorbed(seed, id, k, seg, (double)v.absl)) {
        fate = ABSORBED;
        return ACT_STOP;
      }
      C n1 = back ? nlens : C(1), n2 = back ? C(1) : nlens;
      V3<C> no = back ? scl(C(-1), n) : n;
      C cos_i = -dot(d, no), cos_t;
      C R = fresnel_R(cos_i, n1, n2, cos_t);
      uint32_t u = philox_word(seed, id, k);
      if (C(u >> 8) * C(1.0 / 16777216.0) < R) {
        d = fma3(C(-2) * dot(d, no), no, d);
        return ACT_REFLECT;
      }
      C eta = n1 / n2;
      d = fma3(eta * cos_i - cos_t, no, scl(eta, d));
      ncur = n2;
      return ACT_REFRACT;
    }
  }
  fate = FAILED;
  return ACT_STOP;
}

template <typename T> struct PhotonOut {
  int fate, nev, last_vol;
  V3<T> pos, dir;
  T opl;
  uint64_t hash;
};

// State of a photon between interactions.  Position and direction are kept
// in double; every search uses their rounding to T.
struct PhotonState {
  V3<double> o, d;
  double ncur, opl, lam;   // lam: the photon's wavelength (0: none)
  uint64_t hash, id;
  int k, prev_v, prev_f, prev_side, fate, last_vol;
};

template <typename T> __device__ __forceinline__ void photon_init(PhotonState& p, V3<T> o, V3<T> d, uint64_t id,
                                                                  double lam = 0.0) {
  p.o = {(double)o.x, (double)o.y, (double)o.z};
  p.d = {(double)d.x, (double)d.y, (double)d.z};
  p.ncur = 1.0; p.opl = 0.0; p.lam = lam; p.hash = 0xcbf29ce484222325ull; p.id = id;
  p.k = 0; p.prev_v = -1; p.prev_f = -1; p.prev_side = 0; p.fate = 0; p.last_vol = -1;
  // directions must be unit vectors (to rounding): a photon with any other
  // ends FAILED rather than being traced with wrong path lengths and angles
  if (!finite3(o) || !finite3(d) || !(dabs(dot(d, d) - T(1)) <= T(1e-5))) p.fate = FAILED;
}

// One interaction of the non-sequential transport: nearest surface, then the
// role of its volume.  Returns the event code (vol << 8 | face << 4 | action)
// of the interaction, or 0xffffffff when the photon ends without one.
// SH: the shape set of the calling kernel (a scene holding only those shapes).
template <typename T, int SH = kShapesAll>
__device__ __forceinline__ uint32_t photon_step(const SceneView<T>& S, PhotonState& p) {
  if (p.k == S.max_events) { p.fate = SUSPENDED; return 0xffffffffu; }
  Best<T> b;
  find_nearest<T, SH>(S, p.o, p.d, p.prev_v, p.prev_f, p.prev_side, b);
  if (b.vol < 0) { p.fate = EXITED; return 0xffffffffu; }
  const DVol<T>& v = S.vol[b.vol];
  V3<double> X = {p.o.x + b.tp * p.d.x, p.o.y + b.tp * p.d.y, p.o.z + b.tp * p.d.z};
  p.opl += p.ncur * b.tp;
  V3<double> n = front_normal<T, SH>(v, b.face, X, b.s);
  int back, fate = 0;
  int act = interact<double>(v, n, p.d, p.ncur, fate, back, S.seed, p.id, p.k, b.tp, lens_index<SH>(v, p.lam));
  p.hash = (p.hash ^ (((uint64_t)b.vol << 4) | ((uint64_t)b.face << 1) | (uint64_t)back)) * 0x100000001b3ull;
  p.last_vol = b.vol;
  uint32_t code = ((uint32_t)b.vol << 8) | ((uint32_t)b.face << 4) | (uint32_t)act;
  p.o = X;
  p.prev_v = b.vol; p.prev_f = b.face;
  // side of the face just left: reflection keeps the photon on the side it
  // came from, refraction moves it across
  p.prev_side = back ^ (act == ACT_REFRACT ? 1 : 0);
  ++p.k;
  if (fate) p.fate = fate;
  else if (!finite3(p.d)) p.fate = FAILED;
  return code;
}

template <typename T> __device__ __forceinline__ PhotonOut<T> photon_out(const PhotonState& p) {
  PhotonOut<T> r;
  r.fate = p.fate; r.nev = p.k; r.last_vol = p.last_vol;
  r.pos = to_t<T>(p.o); r.dir = to_t<T>(p.d); r.opl = (T)p.opl; r.hash = p.hash;
  return r;
}

// Full non-sequential transport of one photon.  If `codes` is non-null the
// event codes are written to it (at most MAXLOG).
template <typename T, int MAXLOG, int SH = kShapesAll>
__device__ __forceinline__ PhotonOut<T> trace_photon(const SceneView<T>& S, V3<T> o, V3<T> d, uint64_t id,
                                                     uint32_t* codes, double lam = 0.0) {
  PhotonState p;
  photon_init(p, o, d, id, lam);
  while (!p.fate) {
    int k = p.k;
    uint32_t code = photon_step<T, SH>(S, p);
    if (codes && code != 0xffffffffu && k < MAXLOG) codes[k] = code;
  }
  return photon_out<T>(p);
}

}  // namespace robast
