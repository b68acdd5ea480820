// Device-side adjoint of one photon (shared by the backward kernel).
#pragma once
#include <hip/hip_runtime.h>

#include "device_trace.hpp"
#include "kernels.hpp"

namespace robast {

struct GradSink {
  double* acc;   // LDS or global
  __device__ __forceinline__ void add(int i, double v) {
    if (v != 0.0) atomicAdd(acc + i, v);
  }
};

template <typename T> __device__ __forceinline__ V3<T> qT(const DVol<T>& v, V3<T> a) {
  return {v.Q[0] * a.x + v.Q[3] * a.y + v.Q[6] * a.z, v.Q[1] * a.x + v.Q[4] * a.y + v.Q[7] * a.z,
          v.Q[2] * a.x + v.Q[5] * a.y + v.Q[8] * a.z};
}
template <typename T> __device__ __forceinline__ V3<T> qm(const DVol<T>& v, V3<T> a) {
  return {v.Q[0] * a.x + v.Q[1] * a.y + v.Q[2] * a.z, v.Q[3] * a.x + v.Q[4] * a.y + v.Q[5] * a.z,
          v.Q[6] * a.x + v.Q[7] * a.y + v.Q[8] * a.z};
}

// Apply a recorded action at a hit with front normal n (no random draw),
// in double like the forward interaction.
template <typename T> __device__ __forceinline__ void apply_action(const DVol<T>& v, V3<double> n, int act,
                                                                   V3<double>& d, int& back) {
  double dn = dot(d, n);
  back = dn < 0.0 ? 0 : 1;
  if (act == ACT_REFLECT) {
    d = fma3(-2.0 * dn, n, d);
  } else if (act == ACT_REFRACT) {
    double nin = (double)v.n_in;
    double n1 = back ? nin : 1.0, n2 = back ? 1.0 : nin;
    V3<double> no = back ? scl(-1.0, n) : n;
    double cos_i = -dot(d, no);
    double eta = n1 / n2;
    double s2 = eta * eta * (1.0 - cos_i * cos_i);
    double cos_t = dsqrt(dmax(1.0 - s2, 0.0));
    d = fma3(eta * cos_i - cos_t, no, scl(eta, d));
  }
}

// Exact root of the recorded (vol, face) from state (O, d); false if the
// volume no longer yields that face (cannot happen for an unchanged scene).
template <typename T>
__device__ __forceinline__ bool replay_root(const SceneView<T>& S, int vid, int face, V3<double> O, V3<double> dd,
                                            int pv, int pf, int ps, double& t, double& s) {
  Best<T> b;
  b.t = tinf<T>(); b.vol = -1; b.face = -1; b.s = T(0); b.tp = 0.0;
  V3<T> d = to_t<T>(dd);
  test_volume(S.vol[vid], vid, O, to_t<T>(O), d, inv_dir(d), pv, pf, ps, S.eps_self, b);
  if (b.vol != vid || b.face != face) return false;
  t = b.tp; s = (double)b.s;
  return true;
}

// Bernstein cubic helpers for the cone walls
template <typename T> __device__ __forceinline__ void bez2(const T* p, T s, T& rho, T& z, T& dr, T& dz, T& ddr,
                                                           T& ddz) {
  bez_eval(p, s, rho, z, dr, dz);
  T b0 = T(6) - T(6) * s, b1 = T(-12) + T(18) * s, b2 = T(6) - T(18) * s, b3 = T(6) * s;
  ddr = b0 * p[0] + b1 * p[2] + b2 * p[4] + b3 * p[6];
  ddz = b0 * p[1] + b1 * p[3] + b2 * p[5] + b3 * p[7];
}

// Volume record in double (for the FP64 pull-back of FP32 scenes).
template <typename T> __device__ __forceinline__ DVol<double> promote(const DVol<T>& v) {
  DVol<double> r;
  r.role = v.role; r.shape = v.shape; r.outline = v.outline; r.nfaces = v.nfaces;
  r.sparam = v.sparam; r.tparam = v.tparam; r.always_reflect = v.always_reflect; r.thr = v.thr;
#pragma unroll
  for (int i = 0; i < 9; ++i) r.Q[i] = (double)v.Q[i];
#pragma unroll
  for (int i = 0; i < 3; ++i) r.c[i] = (double)v.c[i];
#pragma unroll
  for (int i = 0; i < 12; ++i) r.p[i] = (double)v.p[i];
  r.n_in = (double)v.n_in;
  return r;
}

// Pull back the cotangents of one event.  In: Xb (cotangent of the hit point,
// i.e. of the next origin) and db (cotangent of the outgoing direction, or of
// the entering direction for the terminal event).  Out: cotangents of the
// entering origin and direction; parameter partials go to the sink.
template <typename T>
__device__ __forceinline__ void event_adjoint(const DVol<T>& v, const DTilt* tilt, int face, int act,
                                              V3<double> O, V3<T> d, T t, T s, V3<T>& Xb, V3<T>& db,
                                              GradSink& gs) {
  V3<double> Xw = adv(O, t, d);
  V3<T> xl = loc_pd(v, Xw);
  V3<T> Gl = local_grad(v, face, xl, s);
  V3<T> m = qT(v, Gl);
  T mn = dsqrt(dot(m, m));
  V3<T> n = scl(T(1) / mn, m);

  // 1. interaction
  V3<T> dbar = {T(0), T(0), T(0)}, nbar = {T(0), T(0), T(0)};
  if (act == ACT_REFLECT) {
    T dn = dot(d, n), bn = dot(db, n);
    dbar = fma3(T(-2) * bn, n, db);
    nbar = add(scl(T(-2) * bn, d), scl(T(-2) * dn, db));
  } else if (act == ACT_REFRACT) {
    int back = dot(d, n) < T(0) ? 0 : 1;
    T sg = back ? T(-1) : T(1);
    V3<T> no = scl(sg, n);
    T n1 = back ? v.n_in : T(1), n2 = back ? T(1) : v.n_in;
    T eta = n1 / n2;
    T cos_i = -dot(d, no);
    T cos_t = dsqrt(dmax(T(1) - eta * eta * (T(1) - cos_i * cos_i), T(1e-30)));
    T k = eta * cos_i - cos_t;
    dbar = scl(eta, db);
    T kb = dot(db, no);
    V3<T> nob = scl(k, db);
    T cib = kb * (eta - eta * eta * cos_i / cos_t);
    dbar = fma3(-cib, no, dbar);
    nob = fma3(-cib, d, nob);
    nbar = scl(sg, nob);
  } else {
    dbar = db;
  }

  // 2. normal n = m / |m|, m = Q^T G(x_l)
  V3<T> mbar = scl(T(1) / mn, fma3(-dot(nbar, n), n, nbar));
  V3<T> Gb = qm(v, mbar);
  V3<T> xlb = {T(0), T(0), T(0)};
  T sbar = T(0);
  const int sp = v.sparam;
  switch (v.shape) {
    case SPHERE: {
      T c = v.p[0];
      xlb = scl(-c, Gb);                                   // Hessian -c I
      if (sp >= 0) {
        T cbar = -dot(Gb, xl);                             // dG/dc = -x_l
        // root term added below; radius R = 1/c
        gs.add(sp, (double)(cbar * (-c * c)));
      }
      break;
    }
    case ASPHERE: {
      T ir = v.p[9];
      T u = (xl.x * xl.x + xl.y * xl.y) * ir;
      T S, dS;
      sag_eval(v.p, u, S, dS);
      T d2 = T(56) * v.p[8];
      for (int i = 7; i >= 2; --i) d2 = d2 * u + T(i * (i - 1)) * v.p[i];
      T k = T(2) * ir * dS;
      T proj = xl.x * Gb.x + xl.y * Gb.y;
      T h = T(4) * ir * ir * d2 * proj;
      xlb = {-k * Gb.x - h * xl.x, -k * Gb.y - h * xl.y, T(0)};
      if (sp >= 0) {
        // dG/db_i = -2 ir i u^{i-1} (x, y, 0)
        T up = T(1);
        for (int i = 1; i <= 8; ++i) {
          gs.add(sp + i - 1, (double)(T(-2) * ir * T(i) * up * proj));
          up *= u;
        }
      }
      break;
    }
    case CYLINDER: xlb = {Gb.x, Gb.y, T(0)}; break;
    case HEXCONE: {
      T rho, z, dr, dz, ddr, ddz;
      bez2(v.p, s, rho, z, dr, dz, ddr, ddz);
      T nx, ny;
      wall_dir(face, nx, ny);
      sbar = -ddz * (Gb.x * nx + Gb.y * ny) + ddr * Gb.z;
      if (sp >= 0) {
        T a = T(1) - s;
        T B1p = T(3) * a * a - T(6) * a * s, B2p = T(6) * a * s - T(3) * s * s;
        T gxy = Gb.x * nx + Gb.y * ny;
        gs.add(sp + 0, (double)(Gb.z * B1p));   // rho1: dG/drho1 = (0, 0, B1')
        gs.add(sp + 1, (double)(-gxy * B1p));   // z1:   dG/dz1 = (-B1' n, 0)
        gs.add(sp + 2, (double)(Gb.z * B2p));
        gs.add(sp + 3, (double)(-gxy * B2p));
      }
      break;
    }
    default: break;
  }
  const bool tilted = v.tparam >= 0;
  V3<T> a1 = {T(0), T(0), T(0)}, a2 = a1, Xp = a1;
  if (tilted) {
    const DTilt& tl = tilt[0];
    a1 = {(T)tl.a1[0], (T)tl.a1[1], (T)tl.a1[2]};
    a2 = {(T)tl.a2[0], (T)tl.a2[1], (T)tl.a2[2]};
    Xp = {(T)(Xw.x - tl.pivot[0]), (T)(Xw.y - tl.pivot[1]), (T)(Xw.z - tl.pivot[2])};
  }
  T tb1 = T(0), tb2 = T(0);
  if (tilted) {
    // explicit rotation of m, and the frame dependence of x_l at fixed X
    V3<T> qx = qT(v, xlb);
    tb1 += dot(mbar, cross(a1, m)) - dot(qx, cross(a1, Xp));
    tb2 += dot(mbar, cross(a2, m)) - dot(qx, cross(a2, Xp));
  }

  // 3. hit point X = O + t d (x_l = Q (X - c))
  V3<T> Xt = add(Xb, qT(v, xlb));
  V3<T> obar = Xt;
  dbar = fma3(t, Xt, dbar);
  T tbar = dot(Xt, d);

  // 4. implicit root
  if (v.shape == HEXCONE) {
    T rho, z, dr, dz, ddr, ddz;
    bez2(v.p, s, rho, z, dr, dz, ddr, ddz);
    T nx, ny;
    wall_dir(face, nx, ny);
    V3<T> dl = loc_d(v, d);
    T du = dl.x * nx + dl.y * ny, dzl = dl.z;
    T det = du * dz - dr * dzl;
    T mu1 = (sbar * dzl + dz * tbar) / det;
    T mu2 = (-dr * tbar - du * sbar) / det;
    V3<T> olb = {-mu1 * nx, -mu1 * ny, -mu2};
    V3<T> ow = qT(v, olb);
    obar = add(obar, ow);
    dbar = fma3(t, ow, dbar);
    if (sp >= 0) {
      T a = T(1) - s;
      T B1 = T(3) * a * a * s, B2 = T(3) * a * s * s;
      gs.add(sp + 0, (double)(mu1 * B1));
      gs.add(sp + 1, (double)(mu2 * B1));
      gs.add(sp + 2, (double)(mu1 * B2));
      gs.add(sp + 3, (double)(mu2 * B2));
    }
  } else {
    T gt = dot(m, d);
    T lam = gt != T(0) ? -tbar / gt : T(0);
    obar = fma3(lam, m, obar);
    dbar = fma3(lam * t, m, dbar);
    if (sp >= 0) {
      if (v.shape == SPHERE) {
        T c = v.p[0];
        gs.add(sp, (double)(lam * (T(-0.5) * dot(xl, xl)) * (-c * c)));
      } else if (v.shape == ASPHERE) {
        T u = (xl.x * xl.x + xl.y * xl.y) * v.p[9];
        T up = u;
        for (int i = 1; i <= 8; ++i) {
          gs.add(sp + i - 1, (double)(-lam * up));
          up *= u;
        }
      }
    }
    if (tilted) {
      tb1 -= lam * dot(m, cross(a1, Xp));
      tb2 -= lam * dot(m, cross(a2, Xp));
    }
  }
  if (tilted) {
    gs.add(v.tparam, (double)tb1);
    gs.add(v.tparam + 1, (double)tb2);
  }
  Xb = obar;
  db = dbar;
}

// Reverse sweep along a photon's recorded sequence of `nev` events (codes
// vol << 8 | face << 4 | action) from its initial ray.  The state entering
// event e is recomputed by replaying events 0..e-1 (one exact intersection
// each, no search).  The objective's cotangents start at the last event:
// those of the final position (rounded to T like the photon's record) and of
// the sign of its final direction.  Returns false if a replayed intersection
// no longer yields the recorded (volume, face), which an unchanged scene
// cannot produce; the photon then adds nothing further.
template <typename T>
__device__ __forceinline__ bool reverse_sweep(const SceneView<T>& L, const AdjView& A, GradSink& gs,
                                              const double* cf, V3<T> o0, V3<T> d0, const uint32_t* codes,
                                              int nev) {
  const V3<double> O0 = {(double)o0.x, (double)o0.y, (double)o0.z};
  const V3<double> D0 = {(double)d0.x, (double)d0.y, (double)d0.z};
  V3<double> Xb = {0.0, 0.0, 0.0}, db = {0.0, 0.0, 0.0};
  for (int e = nev - 1; e >= 0; --e) {
    // state entering event e, replayed along the recorded sequence
    V3<double> O = O0;
    V3<double> d = D0;
    int pv = -1, pf = -1, ps = 0;
    for (int j = 0; j < e; ++j) {
      const int vid = (int)(codes[j] >> 8), face = (int)((codes[j] >> 4) & 15u), act = (int)(codes[j] & 15u);
      double t, s;
      if (!replay_root(L, vid, face, O, d, pv, pf, ps, t, s)) return false;
      const DVol<T>& v = L.vol[vid];
      V3<double> X = {O.x + t * d.x, O.y + t * d.y, O.z + t * d.z};
      V3<double> nrm = front_normal(v, face, X, s);
      int back;
      apply_action(v, nrm, act, d, back);
      O = X; pv = vid; pf = face; ps = back ^ (act == ACT_REFRACT ? 1 : 0);
    }
    const int vid = (int)(codes[e] >> 8), face = (int)((codes[e] >> 4) & 15u), act = (int)(codes[e] & 15u);
    double t, s;
    if (!replay_root(L, vid, face, O, d, pv, pf, ps, t, s)) return false;
    if (e == nev - 1) {
      const V3<double> X = {O.x + t * d.x, O.y + t * d.y, O.z + t * d.z};
      V3<double> dout = d;
      if (act == ACT_REFLECT || act == ACT_REFRACT) {
        int back;
        apply_action(L.vol[vid], front_normal(L.vol[vid], face, X, s), act, dout, back);
      }
      Xb = {cf[0] * ((double)(T)X.x - cf[1]), cf[0] * ((double)(T)X.y - cf[2]), 0.0};
      db = {0.0, 0.0, (T)dout.z >= T(0) ? cf[3] : -cf[3]};
    }
    // the pull-back runs in FP64 from the replayed state: the per-photon
    // partials are summed with cancellation (centroid-subtracted
    // cotangents), which FP32 arithmetic would not resolve
    DVol<double> vd = promote(L.vol[vid]);
    event_adjoint<double>(vd, A.tilt + vid, face, act, O, d, t, s, Xb, db, gs);
  }
  return true;
}

// Adjoint of one photon whose sequence is not recorded: its forward search
// is run again with the same draws (so its fate and sequence equal the
// forward ones) and the sequence is swept in reverse.  Photons that are not
// FOCUSED add nothing.
template <typename T, int MAXE>
__device__ __forceinline__ void adjoint_photon(const SceneView<T>& L, const RaysView<T>& R, int64_t i,
                                               const AdjView& A, GradSink& gs) {
  const int g = R.grp(i);
  if ((unsigned)g >= (unsigned)L.n_groups) return;
  const double* cf = A.coef + 4 * g;
  if ((T)cf[0] == T(0) && (T)cf[3] == T(0)) return;
  T oa[3], da[3];
  R.load(i, oa, da);
  const V3<T> o0 = {oa[0], oa[1], oa[2]};
  const V3<T> d0 = {da[0], da[1], da[2]};
  uint32_t codes[MAXE];
  PhotonOut<T> r = trace_photon<T, MAXE>(L, o0, d0, R.id_base + (uint64_t)R.src(i), codes);
  if (r.fate != FOCUSED || r.nev > MAXE) return;
  (void)reverse_sweep<T>(L, A, gs, cf, o0, d0, codes, r.nev);
}

#ifndef ROBAST_PATH_SWEEP
#define ROBAST_PATH_SWEEP 1
#endif

// State entering an event of a recorded path: origin, direction, and the
// root (distance, cone wall parameter) of the event's intersection.
struct PathState {
  V3<double> O, d;
  double t, s;
};

// Adjoint of one photon from its path record (see kPathSlots): no search.
// The states entering the (at most kPathSlots) events are replayed once,
// forward, and kept in registers; the reverse sweep then reads them back.
template <typename T>
__device__ __forceinline__ void adjoint_photon_path(const SceneView<T>& L, const RaysView<T>& R, int64_t i,
                                                    const AdjView& A, GradSink& gs, uint4 w) {
  const int g = R.grp(i);
  if ((unsigned)g >= (unsigned)L.n_groups) return;
  const double* cf = A.coef + 4 * g;
  if ((T)cf[0] == T(0) && (T)cf[3] == T(0)) return;
  T oa[3], da[3];
  R.load(i, oa, da);
  const uint32_t codes[kPathSlots] = {w.x, w.y, w.z, w.w};
  const int nev = w.y == kPathEnd ? 1 : w.z == kPathEnd ? 2 : w.w == kPathEnd ? 3 : 4;
#if ROBAST_PATH_SWEEP == 0
  (void)reverse_sweep<T>(L, A, gs, cf, V3<T>{oa[0], oa[1], oa[2]}, V3<T>{da[0], da[1], da[2]}, codes, nev);
#else
  PathState st[kPathSlots];
  V3<double> O = {(double)oa[0], (double)oa[1], (double)oa[2]};
  V3<double> d = {(double)da[0], (double)da[1], (double)da[2]};
  int pv = -1, pf = -1, ps = 0;
#pragma unroll
  for (int e = 0; e < kPathSlots; ++e) {
    if (e < nev) {
      const int vid = (int)(codes[e] >> 8), face = (int)((codes[e] >> 4) & 15u), act = (int)(codes[e] & 15u);
      double t, s;
      // a replayed intersection that no longer yields the recorded face
      // (impossible for an unchanged scene): the photon adds nothing
      if (!replay_root(L, vid, face, O, d, pv, pf, ps, t, s)) return;
      st[e] = PathState{O, d, t, s};
      const DVol<T>& v = L.vol[vid];
      const V3<double> X = {O.x + t * d.x, O.y + t * d.y, O.z + t * d.z};
      if (act == ACT_REFLECT || act == ACT_REFRACT) {
        int back;
        apply_action(v, front_normal(v, face, X, s), act, d, back);
        ps = back ^ (act == ACT_REFRACT ? 1 : 0);
      } else {
        ps = dot(d, front_normal(v, face, X, s)) < 0.0 ? 0 : 1;
      }
      O = X; pv = vid; pf = face;
    }
  }
  // cotangents of the final position (rounded to T like the photon's record)
  // and of the sign of the final direction
  V3<double> Xb = {cf[0] * ((double)(T)O.x - cf[1]), cf[0] * ((double)(T)O.y - cf[2]), 0.0};
  V3<double> db = {0.0, 0.0, (T)d.z >= T(0) ? cf[3] : -cf[3]};
#if ROBAST_PATH_SWEEP == 1
#pragma unroll
  for (int e = kPathSlots - 1; e >= 0; --e) {
    if (e < nev) {
      const int vid = (int)(codes[e] >> 8), face = (int)((codes[e] >> 4) & 15u), act = (int)(codes[e] & 15u);
      DVol<double> vd = promote(L.vol[vid]);
      event_adjoint<double>(vd, A.tilt + vid, face, act, st[e].O, st[e].d, st[e].t, st[e].s, Xb, db, gs);
    }
  }
#else
  for (int e = nev - 1; e >= 0; --e) {
    PathState c = st[0];
#pragma unroll
    for (int k = 1; k < kPathSlots; ++k)
      if (e == k) c = st[k];
    const uint32_t code = e == 0 ? codes[0] : e == 1 ? codes[1] : e == 2 ? codes[2] : codes[3];
    const int vid = (int)(code >> 8), face = (int)((code >> 4) & 15u), act = (int)(code & 15u);
    DVol<double> vd = promote(L.vol[vid]);
    event_adjoint<double>(vd, A.tilt + vid, face, act, c.O, c.d, c.t, c.s, Xb, db, gs);
  }
#endif
#endif
}

}  // namespace robast
