// Boundary (fate-flip) terms of the gradient of the collection efficiency.
//
// A photon count has no pathwise gradient: with the photon's sequence held
// fixed its fate never changes.  Its derivative is carried by the photons
// whose fate flips as the geometry moves, i.e. by the discontinuities of the
// fate over the space of photons: the edges of the faces a path meets (a
// cone wall's seams with its neighbours, its exit and entrance rims, the
// exit aperture's hexagon) and the Fresnel decision at a lens face.  Written
// with a signed distance delta(x; p) to such an edge (zero on it), the
// boundary term of d eta / dp is the flux of photons across delta = 0:
//   d eta / dp = E[ Dirac(delta) (d delta / dp) (f(delta > 0) - f(delta < 0)) ].
// It is estimated by edge sampling in a band: every event that lies within
// band / 2 of an edge of its face (delta measured on the photon's own side
// of the edge, in the edge's own units) adds
//   (sides' / band) (d delta / dp) (f_own - f_other)
// per launched photon, where f_own - f_other is the jump of the fate at the
// edge: the fates of the photon moved to just inside and just outside it
// (its initial origin shifted along the gradient of delta, so that its
// whole path up to the event moves with it: replayed along the recorded
// sequence up to the event and traced on from there with the same draws;
// comparing two photons a hair apart keeps earlier and later, unrelated
// edges out of the difference), or at a Fresnel decision the photon's own fate
// and that of the other decision; sides' is 1 for edges whose other side
// also produces such events (seams, exit rim and aperture edge, Fresnel
// decisions) and 2 for an
// edge seen from one side only (the entrance rim, shared by neighbouring
// cones: beyond it a photon simply enters the next cone).  d delta / dp is
// the total derivative along the photon's fixed path: the edge's own motion
// at a fixed hit point plus the hit point's motion, obtained by a reverse
// sweep seeded at the event.  The estimate is unbiased as band -> 0; its
// noise grows as 1 / sqrt(N band).
#pragma once
#include <hip/hip_runtime.h>

#include "adjoint_device.hpp"
#include "device_trace.hpp"

namespace robast {

struct BndView {
  const double* w;     // per group: c_g / (N_g band), 0 when the group adds nothing
  double band;         // band width, in each edge's own distance units
  double push;         // distance across the edge at which the other fate is traced (same units)
  const DTilt* tilt;
  double* grad;
  int n_params;
};

// An edge of the face an event lies on, near the hit.  delta >= 0 is the
// distance to it on the photon's side (zero on the edge); gX its gradient
// with respect to the hit point (world), gp with respect to the cone's
// control points (rho1, z1, rho2, z2) at a fixed hit point.
enum EdgeKind { EDGE_NONE = 0, EDGE_SEAM = 1, EDGE_EXIT_RIM = 2, EDGE_ENTRANCE_RIM = 3, EDGE_APERTURE = 4 };

struct EdgeNear {
  double delta;
  V3<double> gX;
  double gp[4];
  int kind;
  int sides;   // 2: the other side produces such events too; 1: only this side
};

// Distance to the edge of the given kind (EDGE_NONE: the nearest edge of the
// face) of the face hit at X (world) with cone wall parameter s.  Cone
// walls: to the seams with the two neighbouring walls, 1 - sqrt(3) |v| /
// rho(s) (v the lateral coordinate along the wall), to the exit rim, s, and
// to the entrance rim, 1 - s.  Exit apertures (focal hexagons): 1 - max_k
// |x . n_k| / a.  kind stays EDGE_NONE for faces without such edges.
template <typename T, int SH>
__device__ __forceinline__ EdgeNear edge_eval(const DVol<T>& v, int face, V3<double> X, double s, int want) {
  EdgeNear E;
  E.kind = EDGE_NONE;
  E.sides = 2;
  E.delta = 1e300;
  E.gp[0] = E.gp[1] = E.gp[2] = E.gp[3] = 0.0;
  const FrameC<double> F(v);
  const V3<double> xl = F.local(X);
  V3<double> gl = {0.0, 0.0, 0.0};
  if constexpr (((SH >> HEXCONE) & 1) != 0) {
    if (v.shape == HEXCONE && v.role == MIRROR) {
      double rho, z, dr, dz;
      bez_eval(v.p, s, rho, z, dr, dz);
      if (dz == 0.0) return E;
      double nx, ny;
      wall_dir(face, nx, ny);
      const double sq3 = 1.7320508075688772;
      const double vt = -xl.x * ny + xl.y * nx, av = dabs(vt), sg = vt >= 0.0 ? 1.0 : -1.0;
      const double dseam = 1.0 - sq3 * av / rho, dbot = s, dtop = 1.0 - s;
      const double a = 1.0 - s, B[2] = {3.0 * a * a * s, 3.0 * a * s * s};
      int k = want;
      if (k == EDGE_NONE) {
        const double m = dmin(dseam, dmin(dbot, dtop));
        k = dseam == m ? EDGE_SEAM : dbot == m ? EDGE_EXIT_RIM : EDGE_ENTRANCE_RIM;
      }
      if (k == EDGE_SEAM) {
        // s follows the local height: ds/dz_l = 1/z'(s), ds/dz_k = -B_k/z'(s)
        const double c = sq3 * av / (rho * rho);
        gl = {sq3 * sg * ny / rho, -sq3 * sg * nx / rho, c * dr / dz};
        for (int j = 0; j < 2; ++j) {
          E.gp[2 * j] = c * B[j];
          E.gp[2 * j + 1] = -c * dr * B[j] / dz;
        }
        E.delta = dseam;
      } else if (k == EDGE_EXIT_RIM) {
        gl = {0.0, 0.0, 1.0 / dz};
        for (int j = 0; j < 2; ++j) E.gp[2 * j + 1] = -B[j] / dz;
        E.delta = dbot;
      } else if (k == EDGE_ENTRANCE_RIM) {
        gl = {0.0, 0.0, -1.0 / dz};
        for (int j = 0; j < 2; ++j) E.gp[2 * j + 1] = B[j] / dz;
        E.delta = dtop;
        E.sides = 1;
      } else {
        return E;
      }
      E.kind = k;
      E.gX = F.qT(gl);
      return E;
    }
  }
  if (v.shape == PLANE && v.role == FOCAL && v.outline == OL_HEX && (want == EDGE_NONE || want == EDGE_APERTURE)) {
    const double h = 0.8660254037844386, a = (double)v.o[0];
    const double q[3] = {xl.x, 0.5 * xl.x + h * xl.y, -0.5 * xl.x + h * xl.y};
    const double nk[3][2] = {{1.0, 0.0}, {0.5, h}, {-0.5, h}};
    int k = 0;
    for (int j = 1; j < 3; ++j)
      if (dabs(q[j]) > dabs(q[k])) k = j;
    E.delta = 1.0 - dabs(q[k]) / a;
    const double sg = q[k] >= 0.0 ? 1.0 : -1.0;
    gl = {-sg * nk[k][0] / a, -sg * nk[k][1] / a, 0.0};
    E.gX = F.qT(gl);
    E.kind = EDGE_APERTURE;
  }
  return E;
}

// Derivative of the unpolarised Fresnel reflectance with respect to the
// cosine of incidence (no total internal reflection).
__device__ __forceinline__ double fresnel_dR(double ci, double n1, double n2) {
  const double eta = n1 / n2;
  const double ct = dsqrt(1.0 - eta * eta * (1.0 - ci * ci));
  const double dct = eta * eta * ci / ct;
  const double ds_ = n1 * ci + n2 * ct, dp_ = n2 * ci + n1 * ct;
  const double rs = (n1 * ci - n2 * ct) / ds_, rp = (n2 * ci - n1 * ct) / dp_;
  const double num = 2.0 * n1 * n2 * (ct - ci * dct);
  return rs * num / (ds_ * ds_) + rp * num / (dp_ * dp_);
}

// State of a photon entering event e of its recorded sequence, replayed from
// its initial ray (medium index ncur included).
struct ReplayState {
  V3<double> O, d;
  double ncur;
  int pv, pf, ps;
};

template <typename T, int SH>
__device__ __forceinline__ bool replay_event(const SceneView<T>& L, uint32_t code, ReplayState& st, double lam,
                                             double& t, double& s) {
  const int vid = (int)(code >> 8), face = (int)((code >> 4) & 15u), act = (int)(code & 15u);
  if (!replay_root<T, SH>(L, vid, face, st.O, st.d, st.pv, st.pf, st.ps, t, s)) return false;
  const DVol<T>& v = L.vol[vid];
  const V3<double> X = {st.O.x + t * st.d.x, st.O.y + t * st.d.y, st.O.z + t * st.d.z};
  const V3<double> n = front_normal<T, SH>(v, face, X, s);
  int back = dot(st.d, n) < 0.0 ? 0 : 1;
  if (act == ACT_REFLECT || act == ACT_REFRACT) {
    const double nin = lens_index<SH>(v, lam);
    apply_action(v, n, act, st.d, back, nin);
    if (act == ACT_REFRACT) st.ncur = back ? 1.0 : nin;
  }
  st.ps = back ^ (act == ACT_REFRACT ? 1 : 0);
  st.O = X;
  st.pv = vid;
  st.pf = face;
  return true;
}

// Reverse sweep seeded at event e0 (Xb: cotangent of its hit point, db: of
// its outgoing direction) down to the initial ray.  One forward replay keeps
// the state entering each event and its root in a lane-local stack (linear
// in e0; replaying from the start for every event would be quadratic), then
// the events are swept in reverse.  On return Xb and db hold the cotangents
// of the initial origin and direction; if the recorded sequence no longer
// holds, nothing is changed.  A sink without an array (acc null) collects
// no parameter partials.
template <typename T, int MAXE, int SH>
__device__ __forceinline__ void sweep_from(const SceneView<T>& L, const DTilt* tilt, GradSink& gs, V3<T> o0, V3<T> d0,
                                           const uint32_t* codes, int e0, V3<double>& Xb, V3<double>& db,
                                           double lam) {
  if (e0 < 0 || e0 >= MAXE) return;
  V3<double> O[MAXE], D[MAXE];
  double tr[MAXE], sr[MAXE];
  ReplayState st = {{(double)o0.x, (double)o0.y, (double)o0.z}, {(double)d0.x, (double)d0.y, (double)d0.z}, 1.0,
                    -1, -1, 0};
  for (int e = 0; e <= e0; ++e) {
    O[e] = st.O;
    D[e] = st.d;
    double t = 0.0, s = 0.0;
    if (e < e0) {
      if (!replay_event<T, SH>(L, codes[e], st, lam, t, s)) return;
    } else {
      const int vid = (int)(codes[e] >> 8), face = (int)((codes[e] >> 4) & 15u);
      if (!replay_root<T, SH>(L, vid, face, st.O, st.d, st.pv, st.pf, st.ps, t, s)) return;
    }
    tr[e] = t;
    sr[e] = s;
  }
  for (int e = e0; e >= 0; --e) {
    const int vid = (int)(codes[e] >> 8), face = (int)((codes[e] >> 4) & 15u), act = (int)(codes[e] & 15u);
    event_adjoint<double, T, SH>(L.vol[vid], tilt + vid, face, act, O[e], D[e], tr[e], sr[e], Xb, db, gs,
                                 lens_index<SH>(L.vol[vid], lam));
  }
}

// Distance delta to the edge of the given kind at event e of the photon
// started from origin O (direction d0), its path replayed along the
// recorded sequence; false if the sequence no longer holds before or at e.
template <typename T, int SH>
__device__ __forceinline__ bool delta_at(const SceneView<T>& L, const uint32_t* codes, int e, V3<double> O,
                                         V3<double> D, double lam, int kind, double& delta) {
  ReplayState st = {O, D, 1.0, -1, -1, 0};
  double t = 0.0, s = 0.0;
  for (int j = 0; j < e; ++j)
    if (!replay_event<T, SH>(L, codes[j], st, lam, t, s)) return false;
  const int vid = (int)(codes[e] >> 8), face = (int)((codes[e] >> 4) & 15u);
  if (!replay_root<T, SH>(L, vid, face, st.O, st.d, st.pv, st.pf, st.ps, t, s)) return false;
  const V3<double> X = {st.O.x + t * st.d.x, st.O.y + t * st.d.y, st.O.z + t * st.d.z};
  delta = edge_eval<T, SH>(L.vol[vid], face, X, s, kind).delta;
  return true;
}

// Fate of a photon continued from state p until it ends.
template <typename T, int SH>
__device__ __forceinline__ int finish_fate(const SceneView<T>& L, PhotonState p) {
  while (!p.fate) (void)photon_step<T, SH>(L, p);
  return p.fate;
}

template <typename T, int SH>
__device__ __forceinline__ PhotonState state_at(const ReplayState& st, int k, uint64_t id, double lam) {
  PhotonState p;
  p.o = st.O; p.d = st.d; p.ncur = st.ncur; p.opl = 0.0; p.lam = lam; p.hash = 0ull; p.id = id;
  p.k = k; p.prev_v = st.pv; p.prev_f = st.pf; p.prev_side = st.ps; p.fate = 0; p.last_vol = -1;
  return p;
}

// Fate of the photon started from origin O (direction D): its recorded
// sequence replayed up to event e (exclusive; no search, the same actions,
// so the same draws), then traced on from there.  If the sequence no longer
// holds before e, the photon is traced from its start instead.
template <typename T, int SH>
__device__ __forceinline__ int fate_from(const SceneView<T>& L, const uint32_t* codes, int e, V3<double> O,
                                         V3<double> D, uint64_t id, double lam) {
  const ReplayState s0 = {O, D, 1.0, -1, -1, 0};
  ReplayState st = s0;
  double t = 0.0, s = 0.0;
  for (int j = 0; j < e; ++j)
    if (!replay_event<T, SH>(L, codes[j], st, lam, t, s)) return finish_fate<T, SH>(L, state_at<T, SH>(s0, 0, id, lam));
  return finish_fate<T, SH>(L, state_at<T, SH>(st, e, id, lam));
}

// Boundary terms of one photon (see the top of this file).  f_own: the
// photon's own fate, used at Fresnel decisions.
template <typename T, int MAXE, int SH>
__device__ __forceinline__ void boundary_photon(const SceneView<T>& L, const RaysView<T>& R, int64_t i,
                                                const BndView& B, GradSink& gs) {
  const int g = R.grp(i);
  if ((unsigned)g >= (unsigned)L.n_groups) return;
  const double w = B.w[g];
  if (w == 0.0) return;
  T oa[3], da[3];
  R.load(i, oa, da);
  const V3<T> o0 = {oa[0], oa[1], oa[2]};
  const V3<T> d0 = {da[0], da[1], da[2]};
  const uint64_t id = R.id_base + (uint64_t)R.src(i);
  const double lam = R.template wavelength<SH>(i);
  uint32_t codes[MAXE];
  const PhotonOut<T> r = trace_photon<T, MAXE, SH>(L, o0, d0, id, codes, lam);
  if (r.nev > MAXE) return;
  const double f_own = r.fate == FOCUSED ? 1.0 : 0.0;
  ReplayState st = {{(double)o0.x, (double)o0.y, (double)o0.z}, {(double)d0.x, (double)d0.y, (double)d0.z}, 1.0, -1,
                    -1, 0};
  for (int e = 0; e < r.nev; ++e) {
    const uint32_t code = codes[e];
    const int vid = (int)(code >> 8), face = (int)((code >> 4) & 15u), act = (int)(code & 15u);
    double t, s;
    if (!replay_root<T, SH>(L, vid, face, st.O, st.d, st.pv, st.pf, st.ps, t, s)) return;
    const DVol<T>& v = L.vol[vid];
    const V3<double> X = {st.O.x + t * st.d.x, st.O.y + t * st.d.y, st.O.z + t * st.d.z};
    const V3<double> n = front_normal<T, SH>(v, face, X, s);
    const EdgeNear E = edge_eval<T, SH>(v, face, X, s, EDGE_NONE);
    if (E.kind != EDGE_NONE && E.delta < 0.5 * B.band) {
      // the photon moved to just inside and just outside the edge: its
      // initial origin shifted along the gradient G of delta with respect to
      // it (a first sweep, which collects no parameter partials), so that
      // its whole path up to the event moves with it.  The inside point is
      // found by Newton steps on delta along G, replaying the sequence (the
      // linear step alone misses by the curvature of delta across the
      // band); the outside one lies 2 push beyond it.
      V3<double> G = E.gX, Gd = {0.0, 0.0, 0.0};
      GradSink none{nullptr};
      sweep_from<T, MAXE, SH>(L, B.tilt, none, o0, d0, codes, e, G, Gd, lam);
      const double gg = dot(G, G);
      const V3<double> D0 = {(double)d0.x, (double)d0.y, (double)d0.z};
      V3<double> Oin = {(double)o0.x, (double)o0.y, (double)o0.z};
      double dcur = E.delta;
      bool ok = gg > 0.0;
      for (int it = 0; ok && it < 4; ++it) {
        Oin = fma3(-(dcur - B.push) / gg, G, Oin);
        ok = delta_at<T, SH>(L, codes, e, Oin, D0, lam, E.kind, dcur);
        if (ok && dabs(dcur - B.push) < 0.1 * B.push) break;
      }
      ok = ok && dabs(dcur - B.push) < 0.5 * B.push;
      if (ok) {
        const V3<double> Oout = fma3(-2.0 * B.push / gg, G, Oin);
        const double f_in = fate_from<T, SH>(L, codes, e, Oin, D0, id, lam) == FOCUSED ? 1.0 : 0.0;
        const double f_out = fate_from<T, SH>(L, codes, e, Oout, D0, id, lam) == FOCUSED ? 1.0 : 0.0;
        const double c = (E.sides == 1 ? 2.0 : 1.0) * w * (f_in - f_out);
        if (c != 0.0) {
          if (v.sparam >= 0 && v.shape == HEXCONE)
            for (int k = 0; k < 4; ++k) gs.add(v.sparam + k, c * E.gp[k]);
          V3<double> Xb = scl(c, E.gX), db = {0.0, 0.0, 0.0};
          sweep_from<T, MAXE, SH>(L, B.tilt, gs, o0, d0, codes, e, Xb, db, lam);
        }
      }
    }
    if (v.role == LENS && (act == ACT_REFLECT || act == ACT_REFRACT) && e > 0) {
      // the Fresnel decision: reflect iff u < R(cos_i); delta = R - u on the
      // reflecting side, u - R on the other, through the incoming direction
      const int back = dot(st.d, n) < 0.0 ? 0 : 1;
      const double nin = lens_index<SH>(v, lam);
      const double n1 = back ? nin : 1.0, n2 = back ? 1.0 : nin;
      const V3<double> no = back ? scl(-1.0, n) : n;
      const double ci = -dot(st.d, no);
      const double eta = n1 / n2;
      if (eta * eta * (1.0 - ci * ci) < 1.0) {
        double ct;
        const double Rf = fresnel_R(ci, n1, n2, ct);
        const double u = (double)(philox_word(L.seed, id, e) >> 8) * (1.0 / 16777216.0);
        const bool refl = act == ACT_REFLECT;
        const double delta = refl ? Rf - u : u - Rf;
        if (delta < 0.5 * B.band) {
          // the other decision at this event, then the rest of the path
          PhotonState p = state_at<T, SH>(st, e + 1, id, lam);
          p.o = X;
          p.prev_v = vid;
          p.prev_f = face;
          if (refl) {
            p.d = fma3(eta * ci - ct, no, scl(eta, st.d));
            p.ncur = n2;
            p.prev_side = back ^ 1;
          } else {
            p.d = fma3(-2.0 * dot(st.d, no), no, st.d);
            p.prev_side = back;
          }
          const double f_alt = finish_fate<T, SH>(L, p) == FOCUSED ? 1.0 : 0.0;
          const double c = w * (f_own - f_alt);
          if (c != 0.0) {
            // d delta / d d_in = +-(dR/dcos_i) (-n_o): seeded on the outgoing
            // direction of the previous event
            V3<double> Xb = {0.0, 0.0, 0.0}, db = scl(-(refl ? 1.0 : -1.0) * c * fresnel_dR(ci, n1, n2), no);
            sweep_from<T, MAXE, SH>(L, B.tilt, gs, o0, d0, codes, e - 1, Xb, db, lam);
          }
        }
      }
    }
    double t2, s2;
    if (!replay_event<T, SH>(L, code, st, lam, t2, s2)) return;
  }
}

}  // namespace robast
