// Device-side adjoint of one photon (shared by the backward kernel).
#pragma once
#include <hip/hip_runtime.h>

#include "device_trace.hpp"
#include "kernels.hpp"

namespace robast {

// Group coefficients of a photon outside every group (or of a call without
// a figure objective): no figure term.
static __device__ const double kNoCoef[4] = {0.0, 0.0, 0.0, 0.0};

// The cotangent coefficients of photon i's group, and its own cotangent of
// the exit state (or null).
template <typename T>
__device__ __forceinline__ void photon_cots(const SceneView<T>& L, const RaysView<T>& R, int64_t i, const AdjView& A,
                                            const double*& cf, const double*& pc) {
  const int g = R.grp(i);
  cf = (A.coef && (unsigned)g < (unsigned)L.n_groups) ? A.coef + 4 * g : kNoCoef;
  pc = A.pcot ? A.pcot + 6 * R.src(i) : nullptr;
}

// Cotangents of a FOCUSED photon's exit state (position X rounded to T like
// its record, direction d): the figure terms of its group -- RMS about the
// group centroid, a (x - xbar, y - ybar, 0); weighted collection, b sign(u_z)
// on u_z -- plus its own cotangent.
template <typename T>
__device__ __forceinline__ void seed_cots(const double* cf, const double* pc, V3<double> X, V3<double> d,
                                          V3<double>& Xb, V3<double>& db) {
  Xb = {cf[0] * ((double)(T)X.x - cf[1]), cf[0] * ((double)(T)X.y - cf[2]), 0.0};
  db = {0.0, 0.0, (T)d.z >= T(0) ? cf[3] : -cf[3]};
  if (pc) {
    Xb.x += pc[0]; Xb.y += pc[1]; Xb.z += pc[2];
    db.x += pc[3]; db.y += pc[4]; db.z += pc[5];
  }
}

struct GradSink {
  double* acc;   // LDS or global; null: partials are dropped
  __device__ __forceinline__ void add(int i, double v) {
    if (v != 0.0 && acc) atomicAdd(acc + i, v);
  }
};

// A volume's local frame (rotation Q, origin c) converted once to the
// compute type C; Q^T a, Q a and local coordinates of a world point held in
// double (offset from the origin formed in double).
template <typename C> struct FrameC {
  C q[9];
  double c[3];
  template <typename T> __device__ __forceinline__ explicit FrameC(const DVol<T>& v) {
#pragma unroll
    for (int i = 0; i < 9; ++i) q[i] = (C)v.Q[i];
#pragma unroll
    for (int i = 0; i < 3; ++i) c[i] = (double)v.c[i];
  }
  __device__ __forceinline__ V3<C> qT(V3<C> a) const {
    return {q[0] * a.x + q[3] * a.y + q[6] * a.z, q[1] * a.x + q[4] * a.y + q[7] * a.z,
            q[2] * a.x + q[5] * a.y + q[8] * a.z};
  }
  __device__ __forceinline__ V3<C> qm(V3<C> a) const {
    return {q[0] * a.x + q[1] * a.y + q[2] * a.z, q[3] * a.x + q[4] * a.y + q[5] * a.z,
            q[6] * a.x + q[7] * a.y + q[8] * a.z};
  }
  __device__ __forceinline__ V3<C> local(V3<double> x) const {
    return qm({(C)(x.x - c[0]), (C)(x.y - c[1]), (C)(x.z - c[2])});
  }
};

// Apply a recorded action at a hit with front normal n (no random draw),
// in double like the forward interaction; nin: the lens medium's index for
// this photon.
template <typename T> __device__ __forceinline__ void apply_action(const DVol<T>& v, V3<double> n, int act,
                                                                   V3<double>& d, int& back, double nin) {
  double dn = dot(d, n);
  back = dn < 0.0 ? 0 : 1;
  if (act == ACT_REFLECT) {
    d = fma3(-2.0 * dn, n, d);
  } else if (act == ACT_REFRACT) {
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
template <typename T, int SH = kShapesAll>
__device__ __forceinline__ bool replay_root(const SceneView<T>& S, int vid, int face, V3<double> O, V3<double> dd,
                                            int pv, int pf, int ps, double& t, double& s) {
  Best<T> b;
  b.t = tinf<T>(); b.vol = -1; b.face = -1; b.s = 0.0; b.tp = tinf<double>(); b.tie = S.eps_tie;
  V3<T> d = to_t<T>(dd);
  test_volume<T, SH>(S.vol[vid], vid, O, dd, to_t<T>(O), d, inv_dir(d), pv, pf, ps, S.eps_self, b);
  if (b.vol != vid || b.face != face) return false;
  t = b.tp; s = b.s;
  return true;
}

// Bernstein cubic of the cone walls with its first and second derivatives,
// in C from the record's control points.
template <typename C, typename P> __device__ __forceinline__ void bez2(const P* p, C s, C& rho, C& z, C& dr, C& dz, C& ddr,
                                                                       C& ddz) {
  bez_eval(p, s, rho, z, dr, dz);
  C b0 = C(6) - C(6) * s, b1 = C(-12) + C(18) * s, b2 = C(6) - C(18) * s, b3 = C(6) * s;
  ddr = b0 * (C)p[0] + b1 * (C)p[2] + b2 * (C)p[4] + b3 * (C)p[6];
  ddz = b0 * (C)p[1] + b1 * (C)p[3] + b2 * (C)p[5] + b3 * (C)p[7];
}

// Pull back the cotangents of one event, computing in C from the volume
// record (fields converted as they are read).  In: Xb (cotangent of the hit
// point, i.e. of the next origin) and db (cotangent of the outgoing
// direction, or of the entering direction for the terminal event).  Out:
// cotangents of the entering origin and direction; parameter partials go to
// the sink.
template <typename C, typename T, int SH = kShapesAll>
__device__ __forceinline__ void event_adjoint(const DVol<T>& v, const DTilt* tilt, int face, int act,
                                              V3<double> O, V3<C> d, C t, C s, V3<C>& Xb, V3<C>& db,
                                              GradSink& gs, C nin) {
  const FrameC<C> F(v);
  V3<double> Xw = adv(O, t, d);
  V3<C> xl = F.local(Xw);
  V3<C> Gl = local_grad<C, T, SH>(v, face, xl, s);
  V3<C> m = F.qT(Gl);
  C mn = dsqrt(dot(m, m));
  V3<C> n = scl(C(1) / mn, m);

  // 1. interaction
  V3<C> dbar = {C(0), C(0), C(0)}, nbar = {C(0), C(0), C(0)};
  if (act == ACT_REFLECT) {
    C dn = dot(d, n), bn = dot(db, n);
    dbar = fma3(C(-2) * bn, n, db);
    nbar = add(scl(C(-2) * bn, d), scl(C(-2) * dn, db));
  } else if (act == ACT_REFRACT) {
    int back = dot(d, n) < C(0) ? 0 : 1;
    C sg = back ? C(-1) : C(1);
    V3<C> no = scl(sg, n);
    C n1 = back ? nin : C(1), n2 = back ? C(1) : nin;
    C eta = n1 / n2;
    C cos_i = -dot(d, no);
    C cos_t = dsqrt(dmax(C(1) - eta * eta * (C(1) - cos_i * cos_i), C(1e-30)));
    C k = eta * cos_i - cos_t;
    dbar = scl(eta, db);
    C kb = dot(db, no);
    V3<C> nob = scl(k, db);
    C cib = kb * (eta - eta * eta * cos_i / cos_t);
    dbar = fma3(-cib, no, dbar);
    nob = fma3(-cib, d, nob);
    nbar = scl(sg, nob);
  } else {
    dbar = db;
  }

  // 2. normal n = m / |m|, m = Q^T G(x_l)
  V3<C> mbar = scl(C(1) / mn, fma3(-dot(nbar, n), n, nbar));
  V3<C> Gb = F.qm(mbar);
  V3<C> xlb = {C(0), C(0), C(0)};
  C sbar = C(0);
  const int sp = v.sparam;
  switch (v.shape) {
    case SPHERE: {
      C c = (C)v.p[0];
      xlb = scl(-c, Gb);                                   // Hessian -c I
      if (sp >= 0) {
        C cbar = -dot(Gb, xl);                             // dG/dc = -x_l
        // root term added below; radius R = 1/c
        gs.add(sp, (double)(cbar * (-c * c)));
      }
      break;
    }
    case ASPHERE: {
      C ir = (C)v.p[9];
      C u = (xl.x * xl.x + xl.y * xl.y) * ir;
      C S, dS;
      sag_eval(v.p, u, S, dS);
      C d2 = C(56) * (C)v.p[8];
      for (int i = 7; i >= 2; --i) d2 = d2 * u + C(i * (i - 1)) * (C)v.p[i];
      C k = C(2) * ir * dS;
      C proj = xl.x * Gb.x + xl.y * Gb.y;
      C h = C(4) * ir * ir * d2 * proj;
      xlb = {-k * Gb.x - h * xl.x, -k * Gb.y - h * xl.y, C(0)};
      if (sp >= 0) {
        // dG/db_i = -2 ir i u^{i-1} (x, y, 0)
        C up = C(1);
        for (int i = 1; i <= 8; ++i) {
          gs.add(sp + i - 1, (double)(C(-2) * ir * C(i) * up * proj));
          up *= u;
        }
      }
      break;
    }
    case CYLINDER: xlb = {Gb.x, Gb.y, C(0)}; break;
    case HEXCONE: {
      if constexpr (!((SH >> HEXCONE) & 1)) break;
      C rho, z, dr, dz, ddr, ddz;
      bez2(v.p, s, rho, z, dr, dz, ddr, ddz);
      C nx, ny;
      wall_dir(face, nx, ny);
      sbar = -ddz * (Gb.x * nx + Gb.y * ny) + ddr * Gb.z;
      if (sp >= 0) {
        C a = C(1) - s;
        C B1p = C(3) * a * a - C(6) * a * s, B2p = C(6) * a * s - C(3) * s * s;
        C gxy = Gb.x * nx + Gb.y * ny;
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
  V3<C> a1 = {C(0), C(0), C(0)}, a2 = a1, Xp = a1;
  if (tilted) {
    const DTilt& tl = tilt[0];
    a1 = {(C)tl.a1[0], (C)tl.a1[1], (C)tl.a1[2]};
    a2 = {(C)tl.a2[0], (C)tl.a2[1], (C)tl.a2[2]};
    Xp = {(C)(Xw.x - tl.pivot[0]), (C)(Xw.y - tl.pivot[1]), (C)(Xw.z - tl.pivot[2])};
  }
  C tb1 = C(0), tb2 = C(0);
  if (tilted) {
    // explicit rotation of m, and the frame dependence of x_l at fixed X
    V3<C> qx = F.qT(xlb);
    tb1 += dot(mbar, cross(a1, m)) - dot(qx, cross(a1, Xp));
    tb2 += dot(mbar, cross(a2, m)) - dot(qx, cross(a2, Xp));
  }

  // 3. hit point X = O + t d (x_l = Q (X - c))
  V3<C> Xt = add(Xb, F.qT(xlb));
  V3<C> obar = Xt;
  dbar = fma3(t, Xt, dbar);
  C tbar = dot(Xt, d);

  // 4. implicit root
  if (v.shape == HEXCONE) {
    C rho, z, dr, dz, ddr, ddz;
    bez2(v.p, s, rho, z, dr, dz, ddr, ddz);
    C nx, ny;
    wall_dir(face, nx, ny);
    V3<C> dl = F.qm(d);
    C du = dl.x * nx + dl.y * ny, dzl = dl.z;
    C det = du * dz - dr * dzl;
    C mu1 = (sbar * dzl + dz * tbar) / det;
    C mu2 = (-dr * tbar - du * sbar) / det;
    V3<C> olb = {-mu1 * nx, -mu1 * ny, -mu2};
    V3<C> ow = F.qT(olb);
    obar = add(obar, ow);
    dbar = fma3(t, ow, dbar);
    if (sp >= 0) {
      C a = C(1) - s;
      C B1 = C(3) * a * a * s, B2 = C(3) * a * s * s;
      gs.add(sp + 0, (double)(mu1 * B1));
      gs.add(sp + 1, (double)(mu2 * B1));
      gs.add(sp + 2, (double)(mu1 * B2));
      gs.add(sp + 3, (double)(mu2 * B2));
    }
  } else {
    C gt = dot(m, d);
    C lam = gt != C(0) ? -tbar / gt : C(0);
    obar = fma3(lam, m, obar);
    dbar = fma3(lam * t, m, dbar);
    if (sp >= 0) {
      if (v.shape == SPHERE) {
        C c = (C)v.p[0];
        gs.add(sp, (double)(lam * (C(-0.5) * dot(xl, xl)) * (-c * c)));
      } else if (v.shape == ASPHERE) {
        C u = (xl.x * xl.x + xl.y * xl.y) * (C)v.p[9];
        C up = u;
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

// State entering an event of a recorded path: origin, direction, and the
// root (distance, cone wall parameter) of the event's intersection.
struct PathState {
  V3<double> O, d;
  double t, s;
};

// Reverse sweep along a photon's recorded sequence of `nev` <= MAXE events
// (codes vol << 8 | face << 4 | action) from its initial ray.  The sequence
// is replayed forward once (one exact intersection per event, no search)
// and the states entering the events are kept in a lane-local array, so the
// sweep costs one replay per event however long the path (a many-bounce
// concentrator photon).  The objective's cotangents start at the last event:
// those of the final position (rounded to T like the photon's record) and of
// the sign of its final direction.  Returns false if a replayed intersection
// no longer yields the recorded (volume, face), which an unchanged scene
// cannot produce; the photon then adds nothing.
template <typename T, int MAXE, int SH = kShapesAll>
__device__ __forceinline__ bool reverse_sweep(const SceneView<T>& L, const AdjView& A, GradSink& gs,
                                              const double* cf, const double* pc, V3<T> o0, V3<T> d0,
                                              const uint32_t* codes, int nev, double lam) {
  PathState st[MAXE];
  V3<double> O = {(double)o0.x, (double)o0.y, (double)o0.z};
  V3<double> d = {(double)d0.x, (double)d0.y, (double)d0.z};
  int pv = -1, pf = -1, ps = 0;
  for (int e = 0; e < nev; ++e) {
    const int vid = (int)(codes[e] >> 8), face = (int)((codes[e] >> 4) & 15u), act = (int)(codes[e] & 15u);
    double t, s;
    if (!replay_root<T, SH>(L, vid, face, O, d, pv, pf, ps, t, s)) return false;
    st[e] = PathState{O, d, t, s};
    const DVol<T>& v = L.vol[vid];
    const V3<double> X = {O.x + t * d.x, O.y + t * d.y, O.z + t * d.z};
    if (act == ACT_REFLECT || act == ACT_REFRACT) {
      int back;
      apply_action(v, front_normal<T, SH>(v, face, X, s), act, d, back, lens_index<SH>(v, lam));
      ps = back ^ (act == ACT_REFRACT ? 1 : 0);
    } else {
      ps = dot(d, front_normal<T, SH>(v, face, X, s)) < 0.0 ? 0 : 1;
    }
    O = X; pv = vid; pf = face;
  }
  // the final position and direction: O and d after the last event
  V3<double> Xb, db;
  seed_cots<T>(cf, pc, O, d, Xb, db);
  for (int e = nev - 1; e >= 0; --e) {
    const int vid = (int)(codes[e] >> 8), face = (int)((codes[e] >> 4) & 15u), act = (int)(codes[e] & 15u);
    // the pull-back runs in FP64 from the replayed state: the per-photon
    // partials are summed with cancellation (centroid-subtracted
    // cotangents), which FP32 arithmetic would not resolve
    event_adjoint<double, T, SH>(L.vol[vid], A.tilt + vid, face, act, st[e].O, st[e].d, st[e].t, st[e].s, Xb, db, gs,
                                 lens_index<SH>(L.vol[vid], lam));
  }
  return true;
}

// Adjoint of one photon whose sequence is not recorded: its forward search
// is run again with the same draws (so its fate and sequence equal the
// forward ones) and the sequence is swept in reverse.  Photons that are not
// FOCUSED add nothing.  With A.check_hash every photon's sequence hash is
// compared with the forward one (a count of differences in A.mismatch).
template <typename T, int MAXE, int SH = kShapesAll>
__device__ __forceinline__ void adjoint_photon(const SceneView<T>& L, const RaysView<T>& R, int64_t i,
                                               const AdjView& A, GradSink& gs) {
  const double *cf, *pc;
  photon_cots(L, R, i, A, cf, pc);
  const bool want = cf[0] != 0.0 || cf[3] != 0.0 || pc;
  if (!want && !A.check_hash) return;
  T oa[3], da[3];
  R.load(i, oa, da);
  const V3<T> o0 = {oa[0], oa[1], oa[2]};
  const V3<T> d0 = {da[0], da[1], da[2]};
  uint32_t codes[MAXE];
  const double lam = R.template wavelength<SH>(i);
  PhotonOut<T> r = trace_photon<T, MAXE, SH>(L, o0, d0, R.id_base + (uint64_t)R.src(i), codes, lam);
  if (A.check_hash && A.check_hash[R.src(i)] != r.hash) atomicAdd(A.mismatch, 1u);
  if (!want || r.fate != FOCUSED || r.nev > MAXE) return;
  (void)reverse_sweep<T, MAXE, SH>(L, A, gs, cf, pc, o0, d0, codes, r.nev, lam);
}

// Volume record in double (the pull-back then reads no FP32 field).
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
  r.absl = (double)v.absl;
  return r;
}

// Adjoint of one photon from its path record (see kPathSlots): no search.
// The states entering its events (at most NS <= kPathSlots of them: the
// caller passes only records that short) are replayed once, forward, and
// kept in registers; the reverse sweep then reads them back.  NS sizes the
// register arrays: a sweep over 3 slots needs no spills, over 4 it does.
// PROMOTE: convert each event's volume record to double once (fewer
// instructions) rather than field by field as read (fewer registers); which
// is faster depends on the register pressure of the calling kernel.
template <typename T, bool PROMOTE, int NS = kPathSlots, int SH = kShapesAll>
__device__ __forceinline__ void adjoint_photon_path(const SceneView<T>& L, const RaysView<T>& R, int64_t i,
                                                    const AdjView& A, GradSink& gs, uint4 w) {
  static_assert(NS >= 1 && NS <= kPathSlots, "slots of a path record");
  const double *cf, *pc;
  photon_cots(L, R, i, A, cf, pc);
  if (cf[0] == 0.0 && cf[3] == 0.0 && !pc) return;
  T oa[3], da[3];
  R.load(i, oa, da);
  const uint32_t codes[kPathSlots] = {w.x, w.y, w.z, w.w};
  const double lam = R.template wavelength<SH>(i);
  const int nev = w.y == kPathEnd ? 1 : w.z == kPathEnd ? 2 : w.w == kPathEnd ? 3 : 4;
  PathState st[NS];
  V3<double> O = {(double)oa[0], (double)oa[1], (double)oa[2]};
  V3<double> d = {(double)da[0], (double)da[1], (double)da[2]};
  int pv = -1, pf = -1, ps = 0;
#pragma unroll
  for (int e = 0; e < NS; ++e) {
    if (e < nev) {
      const int vid = (int)(codes[e] >> 8), face = (int)((codes[e] >> 4) & 15u), act = (int)(codes[e] & 15u);
      double t, s;
      // a replayed intersection that no longer yields the recorded face
      // (impossible for an unchanged scene): the photon adds nothing
      if (!replay_root<T, SH>(L, vid, face, O, d, pv, pf, ps, t, s)) return;
      st[e] = PathState{O, d, t, s};
      const DVol<T>& v = L.vol[vid];
      const V3<double> X = {O.x + t * d.x, O.y + t * d.y, O.z + t * d.z};
      if (act == ACT_REFLECT || act == ACT_REFRACT) {
        int back;
        apply_action(v, front_normal<T, SH>(v, face, X, s), act, d, back, lens_index<SH>(v, lam));
        ps = back ^ (act == ACT_REFRACT ? 1 : 0);
      } else {
        ps = dot(d, front_normal<T, SH>(v, face, X, s)) < 0.0 ? 0 : 1;
      }
      O = X; pv = vid; pf = face;
    }
  }
  V3<double> Xb, db;
  seed_cots<T>(cf, pc, O, d, Xb, db);
#pragma unroll
  for (int e = NS - 1; e >= 0; --e) {
    if (e < nev) {
      const int vid = (int)(codes[e] >> 8), face = (int)((codes[e] >> 4) & 15u), act = (int)(codes[e] & 15u);
      if constexpr (PROMOTE) {
        const DVol<double> vd = promote(L.vol[vid]);
        event_adjoint<double, double, SH>(vd, A.tilt + vid, face, act, st[e].O, st[e].d, st[e].t, st[e].s, Xb, db, gs,
                                          lens_index<SH>(L.vol[vid], lam));
      } else {
        event_adjoint<double, T, SH>(L.vol[vid], A.tilt + vid, face, act, st[e].O, st[e].d, st[e].t, st[e].s, Xb, db,
                                 gs, lens_index<SH>(L.vol[vid], lam));
      }
    }
  }
}

}  // namespace robast
