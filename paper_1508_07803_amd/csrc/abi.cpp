// C ABI of the tracer: argument validation, the scene compiler and launches.
//
// The scene compiler turns the caller's volume descriptors (roles and shapes
// of §2.1/§2.2) into device records in the kernel precision, computes
// conservative local and world bounds for each volume, and builds an XY
// uniform grid of candidate lists used by the non-sequential search.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/robast.h"
#include "kernels.hpp"
#include "scene_layout.hpp"

using namespace robast;

namespace {

thread_local std::string g_err;

int fail(int code, const std::string& msg) {
  g_err = msg;
  return code;
}
int hip_fail(hipError_t e, const char* what) {
  g_err = std::string(what) + ": " + hipGetErrorString(e);
  return ROBAST_EHIP;
}

bool finite_all(const double* a, int n) {
  for (int i = 0; i < n; ++i)
    if (!std::isfinite(a[i])) return false;
  return true;
}

// ------------------------------------------------------------------ small host algebra
void rodrigues(const double e[3], double ang, double R[9]) {
  double c = std::cos(ang), s = std::sin(ang), C = 1.0 - c;
  double K[9] = {0, -e[2], e[1], e[2], 0, -e[0], -e[1], e[0], 0};
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) R[3 * i + j] = (i == j ? c : 0.0) + s * K[3 * i + j] + C * e[i] * e[j];
}
void matmul(const double* A, const double* B, double* C) {
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      double s = 0;
      for (int k = 0; k < 3; ++k) s += A[3 * i + k] * B[3 * k + j];
      C[3 * i + j] = s;
    }
}
bool inv3(const double* M, double* I) {
  double a = M[0], b = M[1], c = M[2], d = M[3], e = M[4], f = M[5], g = M[6], h = M[7], k = M[8];
  double det = a * (e * k - f * h) - b * (d * k - f * g) + c * (d * h - e * g);
  if (!(std::fabs(det) > 1e-12)) return false;
  double id = 1.0 / det;
  I[0] = (e * k - f * h) * id; I[1] = (c * h - b * k) * id; I[2] = (b * f - c * e) * id;
  I[3] = (f * g - d * k) * id; I[4] = (a * k - c * g) * id; I[5] = (c * d - a * f) * id;
  I[6] = (d * h - e * g) * id; I[7] = (b * g - a * h) * id; I[8] = (a * e - b * d) * id;
  return true;
}

double sag_asph(const double* b, double u) {
  double s = b[7];
  for (int i = 6; i >= 0; --i) s = s * u + b[i];
  return s * u;
}
double dsag_asph(const double* b, double u) {
  double s = 8.0 * b[7];
  for (int i = 6; i >= 0; --i) s = s * u + (i + 1) * b[i];
  return s;
}

double outline_rmin(const robast_volume_desc& v) {
  return (v.outline == ROBAST_ANNULUS || v.outline == ROBAST_SECTOR) ? v.o[0] : 0.0;
}
double outline_rmax(const robast_volume_desc& v) {
  switch (v.outline) {
    case ROBAST_DISC: return v.o[0];
    case ROBAST_ANNULUS: case ROBAST_SECTOR: return v.o[1];
    case ROBAST_RECT: return std::hypot(v.o[0], v.o[1]);
    case ROBAST_HEX: return v.o[0] * 2.0 / std::sqrt(3.0);
  }
  return 0.0;
}

// ------------------------------------------------------------------ validation
int validate(const robast_scene_desc* d, const double* params, int64_t n_params) {
  if (!d) return fail(ROBAST_EINVAL, "desc is NULL");
  if (d->n_volumes < 0 || d->n_volumes > 65535) return fail(ROBAST_EINVAL, "n_volumes out of range 0..65535");
  if (d->n_volumes > 0 && !d->volumes) return fail(ROBAST_EINVAL, "volumes is NULL");
  if (d->precision != 32 && d->precision != 64) return fail(ROBAST_EINVAL, "precision must be 32 or 64");
  if (d->max_events < 1 || d->max_events > 255) return fail(ROBAST_EINVAL, "max_events out of range 1..255");
  if (d->n_groups < 1 || d->n_groups > 4096) return fail(ROBAST_EINVAL, "n_groups out of range 1..4096");
  if (!(d->l_ref > 0.0) || !std::isfinite(d->l_ref)) return fail(ROBAST_EINVAL, "l_ref must be finite and > 0");
  if (n_params < 0 || (n_params > 0 && !params)) return fail(ROBAST_EINVAL, "params NULL or n_params < 0");
  if (n_params > 0 && !finite_all(params, (int)n_params)) return fail(ROBAST_EINVAL, "non-finite parameter");
  for (int i = 0; i < d->n_volumes; ++i) {
    const robast_volume_desc& v = d->volumes[i];
    std::string at = " (volume " + std::to_string(i) + ")";
    if (v.role < ROBAST_MIRROR || v.role > ROBAST_OBSCURATION) return fail(ROBAST_EINVAL, "unknown role" + at);
    if (v.shape < ROBAST_PLANE || v.shape > ROBAST_HEXCONE) return fail(ROBAST_EINVAL, "unknown shape" + at);
    if (v.outline < 0 || v.outline > ROBAST_SECTOR) return fail(ROBAST_EINVAL, "unknown outline" + at);
    if (!finite_all(v.Q, 9) || !finite_all(v.c, 3) || !finite_all(v.p, 16) || !finite_all(v.o, 4) ||
        !std::isfinite(v.reflectivity) || !std::isfinite(v.n_inside) || !finite_all(v.Q0, 9) ||
        !finite_all(v.c0, 3) || !finite_all(v.pivot, 3) || !finite_all(v.e1, 3) || !finite_all(v.e2, 3))
      return fail(ROBAST_EINVAL, "non-finite descriptor value" + at);
    double I[9];
    if (!inv3(v.Q, I)) return fail(ROBAST_EINVAL, "singular frame Q" + at);
    bool sagged = v.shape == ROBAST_PLANE || v.shape == ROBAST_SPHERE || v.shape == ROBAST_ASPHERE;
    if (sagged) {
      if (v.outline == ROBAST_OUTLINE_NONE) return fail(ROBAST_EINVAL, "sag surface needs an outline" + at);
      const double* o = v.o;
      bool ok = true;
      switch (v.outline) {
        case ROBAST_DISC: ok = o[0] > 0; break;
        case ROBAST_ANNULUS: ok = o[0] >= 0 && o[1] > o[0]; break;
        case ROBAST_RECT: ok = o[0] > 0 && o[1] > 0; break;
        case ROBAST_HEX: ok = o[0] > 0; break;
        case ROBAST_SECTOR: ok = o[0] >= 0 && o[1] > o[0] && o[3] > o[2] && o[3] - o[2] <= 2 * M_PI + 1e-12; break;
      }
      if (!ok) return fail(ROBAST_EINVAL, "degenerate outline" + at);
    }
    if (v.shape == ROBAST_SPHERE && std::fabs(v.p[0]) * outline_rmax(v) >= 1.0)
      return fail(ROBAST_EINVAL, "sphere aperture reaches its equator" + at);
    if (v.shape == ROBAST_ASPHERE && !(v.p[0] > 0)) return fail(ROBAST_EINVAL, "asphere rn must be > 0" + at);
    if (v.shape == ROBAST_CYLINDER && !(v.p[0] > 0 && v.p[1] > 0)) return fail(ROBAST_EINVAL, "cylinder size" + at);
    if (v.shape == ROBAST_BOX && !(v.p[0] > 0 && v.p[1] > 0 && v.p[2] > 0)) return fail(ROBAST_EINVAL, "box size" + at);
    if (v.shape == ROBAST_HEXCONE) {
      for (int k = 0; k < 4; ++k)
        if (!(v.p[2 * k] > 0)) return fail(ROBAST_EINVAL, "cone profile radius must be > 0" + at);
    }
    if (v.role == ROBAST_MIRROR && !(v.reflectivity >= 0.0 && v.reflectivity <= 1.0))
      return fail(ROBAST_EINVAL, "reflectivity outside [0, 1]" + at);
    if (v.role == ROBAST_LENS && !(v.n_inside > 0.0)) return fail(ROBAST_EINVAL, "lens index must be > 0" + at);
    if (v.role == ROBAST_LENS && v.shape != ROBAST_BOX)
      return fail(ROBAST_EUNSUPPORTED, "lenses must be closed solids (BOX)" + at);
    int ns = v.shape == ROBAST_SPHERE ? 1 : v.shape == ROBAST_ASPHERE ? 8 : v.shape == ROBAST_HEXCONE ? 4 : 0;
    if (v.shape_param >= 0 && (ns == 0 || v.shape_param + ns > n_params))
      return fail(ROBAST_EINVAL, "shape_param out of range" + at);
    if (v.tilt_param >= 0 && v.tilt_param + 2 > n_params) return fail(ROBAST_EINVAL, "tilt_param out of range" + at);
    if (v.shape_param < -1 || v.tilt_param < -1) return fail(ROBAST_EINVAL, "negative parameter index" + at);
  }
  return ROBAST_OK;
}

}  // namespace

struct robast_scene {
  int precision = 32, n_vol = 0, n_groups = 1, max_events = 16;
  uint64_t seed = 0;
  double l_ref = 1.0;
  std::vector<robast_volume_desc> desc;
  std::vector<double> params;
  void* d_blob = nullptr;
  size_t blob_bytes = 0;
  DTilt* d_tilt = nullptr;
  double* d_coef = nullptr;    // n_groups * 4 backward coefficients
  SceneView<float> sf{};
  SceneView<double> sd{};
  LaunchCfg cfg{};
};

namespace {

// Apply the differentiable parameters to a descriptor: radius, sag
// coefficients, cone control points and tilted frame.
void apply_params(robast_volume_desc& v, const std::vector<double>& P) {
  if (v.shape_param >= 0) {
    if (v.shape == ROBAST_SPHERE) v.p[0] = 1.0 / P[v.shape_param];
    else if (v.shape == ROBAST_ASPHERE) for (int i = 0; i < 8; ++i) v.p[1 + i] = P[v.shape_param + i];
    else if (v.shape == ROBAST_HEXCONE) for (int i = 0; i < 4; ++i) v.p[2 + i] = P[v.shape_param + i];
  }
  if (v.tilt_param >= 0) {
    double Ra[9], Rb[9], R[9], Rt[9];
    rodrigues(v.e1, P[v.tilt_param], Ra);
    rodrigues(v.e2, P[v.tilt_param + 1], Rb);
    matmul(Rb, Ra, R);
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) Rt[3 * i + j] = R[3 * j + i];
    matmul(v.Q0, Rt, v.Q);
    for (int i = 0; i < 3; ++i) {
      double s = 0;
      for (int k = 0; k < 3; ++k) s += R[3 * i + k] * (v.pivot[k] - v.c0[k]);
      v.c[i] = v.pivot[i] - s;
    }
  }
}

template <typename T> T q(double x) { return (T)x; }

struct Box3 { double lo[3], hi[3]; };

// Conservative local bounds of the surface of a volume.
Box3 local_bounds(const robast_volume_desc& v, double& slope) {
  Box3 b{};
  slope = 0.0;
  double rmax = outline_rmax(v), rmin = outline_rmin(v);
  double xe = rmax, ye = rmax;
  double x0 = -rmax, x1 = rmax, y0 = -rmax, y1 = rmax;
  if (v.outline == ROBAST_RECT) { xe = v.o[0]; ye = v.o[1]; }
  if (v.outline == ROBAST_HEX) { xe = v.o[0]; ye = v.o[0] * 2.0 / std::sqrt(3.0); }
  x0 = -xe; x1 = xe; y0 = -ye; y1 = ye;
  if (v.outline == ROBAST_SECTOR && v.o[3] - v.o[2] < 2 * M_PI - 1e-12) {
    // box of the annular sector: its four corners plus the axis crossings inside it
    double ra = v.o[0], rb = v.o[1], pa = v.o[2], pb = v.o[3];
    x0 = y0 = 1e300; x1 = y1 = -1e300;
    auto take = [&](double r, double ph) {
      double x = r * std::cos(ph), y = r * std::sin(ph);
      x0 = std::min(x0, x); x1 = std::max(x1, x); y0 = std::min(y0, y); y1 = std::max(y1, y);
    };
    take(ra, pa); take(ra, pb); take(rb, pa); take(rb, pb);
    for (int k = (int)std::floor(pa / (0.5 * M_PI)) - 1; k <= (int)std::ceil(pb / (0.5 * M_PI)) + 1; ++k) {
      double ph = k * 0.5 * M_PI;
      if (ph >= pa && ph <= pb) take(rb, ph);
    }
  }
  switch (v.shape) {
    case ROBAST_PLANE:
      b = {{x0, y0, 0.0}, {x1, y1, 0.0}};
      break;
    case ROBAST_SPHERE: {
      double c = v.p[0];
      auto sag = [&](double r) { return c * r * r / (1.0 + std::sqrt(1.0 - c * c * r * r)); };
      double z0 = sag(rmin), z1 = sag(rmax);
      b = {{x0, y0, std::min(z0, z1)}, {x1, y1, std::max(z0, z1)}};
      slope = std::fabs(c) * rmax / std::sqrt(1.0 - c * c * rmax * rmax);
      break;
    }
    case ROBAST_ASPHERE: {
      const double* bb = v.p + 1;
      double rn2 = v.p[0] * v.p[0];
      double ua = rmin * rmin / rn2, ub = rmax * rmax / rn2;
      const int N = 4096;
      double zmin = 1e300, zmax = -1e300, smax = 0.0, dmax = 0.0;
      for (int i = 0; i <= N; ++i) {
        double u = ua + (ub - ua) * i / N;
        double z = sag_asph(bb, u);
        zmin = std::min(zmin, z); zmax = std::max(zmax, z);
        double ds = std::fabs(dsag_asph(bb, u));
        dmax = std::max(dmax, ds);
        smax = std::max(smax, ds * 2.0 * std::sqrt(u * rn2) / rn2);
      }
      double pad = dmax * (ub - ua) / N;  // Lipschitz bound between samples
      b = {{x0, y0, zmin - pad}, {x1, y1, zmax + pad}};
      slope = smax * 1.01 + 1e-6;
      break;
    }
    case ROBAST_CYLINDER:
      b = {{-v.p[0], -v.p[0], 0.0}, {v.p[0], v.p[0], v.p[1]}};
      break;
    case ROBAST_BOX:
      b = {{-v.p[0], -v.p[1], -v.p[2]}, {v.p[0], v.p[1], v.p[2]}};
      break;
    case ROBAST_HEXCONE: {
      double rm = 0, zl = 1e300, zh = -1e300;
      for (int k = 0; k < 4; ++k) {
        rm = std::max(rm, v.p[2 * k]);
        zl = std::min(zl, v.p[2 * k + 1]); zh = std::max(zh, v.p[2 * k + 1]);
      }
      double R = rm * 2.0 / std::sqrt(3.0);
      b = {{-R, -R, zl}, {R, R, zh}};
      break;
    }
  }
  return b;
}

template <typename T> void fill_record(DVol<T>& r, const robast_volume_desc& v, Box3& world, double l_ref) {
  std::memset(&r, 0, sizeof(r));
  r.role = v.role; r.shape = v.shape; r.outline = v.outline;
  r.nfaces = (v.shape == ROBAST_BOX || v.shape == ROBAST_HEXCONE) ? 6 : 1;
  r.sparam = v.shape_param; r.tparam = v.tilt_param;
  double R = std::min(std::max(v.reflectivity, 0.0), 1.0);
  r.always_reflect = R >= 1.0 ? 1 : 0;
  r.thr = R >= 1.0 ? 0xffffffffu : (uint32_t)std::floor(R * 4294967296.0);
  for (int i = 0; i < 9; ++i) r.Q[i] = q<T>(v.Q[i]);
  for (int i = 0; i < 3; ++i) r.c[i] = q<T>(v.c[i]);
  switch (v.shape) {
    case ROBAST_SPHERE: r.p[0] = q<T>(v.p[0]); break;
    case ROBAST_ASPHERE:
      for (int i = 0; i < 9; ++i) r.p[i] = q<T>(v.p[i]);
      r.p[9] = q<T>(1.0 / ((double)q<T>(v.p[0]) * (double)q<T>(v.p[0])));
      break;
    case ROBAST_CYLINDER: r.p[0] = q<T>(v.p[0]); r.p[1] = q<T>(v.p[1]); break;
    case ROBAST_BOX: for (int i = 0; i < 3; ++i) r.p[i] = q<T>(v.p[i]); break;
    case ROBAST_HEXCONE: for (int i = 0; i < 8; ++i) r.p[i] = q<T>(v.p[i]); break;
    default: break;
  }
  const double* o = v.o;
  switch (v.outline) {
    case ROBAST_DISC: r.o[0] = q<T>(o[0] * o[0]); break;
    case ROBAST_ANNULUS: r.o[0] = q<T>(o[0] * o[0]); r.o[1] = q<T>(o[1] * o[1]); break;
    case ROBAST_RECT: r.o[0] = q<T>(o[0]); r.o[1] = q<T>(o[1]); break;
    case ROBAST_HEX: r.o[0] = q<T>(o[0]); break;
    case ROBAST_SECTOR:
      r.o[0] = q<T>(o[0] * o[0]); r.o[1] = q<T>(o[1] * o[1]);
      r.o[2] = q<T>(std::cos(o[2])); r.o[3] = q<T>(std::sin(o[2]));
      r.o[4] = q<T>(std::cos(o[3])); r.o[5] = q<T>(std::sin(o[3]));
      r.o[6] = (o[3] - o[2] > M_PI) ? T(1) : T(0);
      if (o[3] - o[2] >= 2 * M_PI - 1e-12) { r.outline = ROBAST_ANNULUS; }
      break;
    default: break;
  }
  double slope = 0;
  Box3 lb = local_bounds(v, slope);
  double ext = 0;
  for (int k = 0; k < 3; ++k) ext = std::max(ext, lb.hi[k] - lb.lo[k]);
  double pad = 1e-5 * (ext + l_ref);
  for (int k = 0; k < 3; ++k) { r.lo[k] = q<T>(lb.lo[k] - pad); r.hi[k] = q<T>(lb.hi[k] + pad); }
  r.slope = q<T>(slope);
  r.rout = q<T>(outline_rmax(v) * (1.0 + 1e-6));
  r.n_in = q<T>(v.n_inside);
  // world AABB of the 8 corners, x = c + Q^{-1} x_l
  double I[9];
  inv3(v.Q, I);
  double mn[3] = {1e300, 1e300, 1e300}, mx[3] = {-1e300, -1e300, -1e300};
  for (int m = 0; m < 8; ++m) {
    double xl[3] = {(m & 1) ? lb.hi[0] : lb.lo[0], (m & 2) ? lb.hi[1] : lb.lo[1], (m & 4) ? lb.hi[2] : lb.lo[2]};
    for (int i = 0; i < 3; ++i) {
      double w = v.c[i] + I[3 * i] * xl[0] + I[3 * i + 1] * xl[1] + I[3 * i + 2] * xl[2];
      mn[i] = std::min(mn[i], w); mx[i] = std::max(mx[i], w);
    }
  }
  double wpad = 1e-5 * (ext + l_ref) + 1e-6 * (std::fabs(v.c[0]) + std::fabs(v.c[1]) + std::fabs(v.c[2]));
  for (int i = 0; i < 3; ++i) {
    world.lo[i] = mn[i] - wpad; world.hi[i] = mx[i] + wpad;
    r.bmin[i] = q<T>(world.lo[i]); r.bmax[i] = q<T>(world.hi[i]);
    // rounding to T must not shrink the box
    if ((double)r.bmin[i] > world.lo[i]) r.bmin[i] = std::nextafter(r.bmin[i], (T)-INFINITY);
    if ((double)r.bmax[i] < world.hi[i]) r.bmax[i] = std::nextafter(r.bmax[i], (T)INFINITY);
  }
}

template <typename T> void align_to(std::vector<char>& b, size_t a) {
  while (b.size() % a) b.push_back(0);
}

// Build the blob for precision T and fill the view offsets (host addresses
// are rebased to the device allocation by the caller).
template <typename T>
void compile_blob(const robast_scene& s, std::vector<char>& blob, SceneView<T>& V, std::vector<size_t>& offs) {
  int nv = s.n_vol;
  std::vector<DVol<T>> recs(nv);
  std::vector<Box3> wb(nv);
  for (int i = 0; i < nv; ++i) fill_record<T>(recs[i], s.desc[i], wb[i], s.l_ref);
  // grid over the XY footprints
  std::vector<uint16_t> always;
  std::vector<int> gridv;
  double ux0 = 1e300, uy0 = 1e300, ux1 = -1e300, uy1 = -1e300;
  std::vector<double> areas;
  for (int i = 0; i < nv; ++i) {
    ux0 = std::min(ux0, wb[i].lo[0]); uy0 = std::min(uy0, wb[i].lo[1]);
    ux1 = std::max(ux1, wb[i].hi[0]); uy1 = std::max(uy1, wb[i].hi[1]);
    areas.push_back((wb[i].hi[0] - wb[i].lo[0]) * (wb[i].hi[1] - wb[i].lo[1]));
  }
  int nx = 0, ny = 0;
  double cell = 1.0;
  if (nv > 8) {
    std::vector<double> a2 = areas;
    std::nth_element(a2.begin(), a2.begin() + a2.size() / 2, a2.end());
    cell = std::sqrt(std::max(a2[a2.size() / 2], 1e-30));
    double W = ux1 - ux0, H = uy1 - uy0;
    cell = std::max(cell, std::max(W, H) / 256.0);
    nx = std::max(1, (int)std::ceil(W / cell));
    ny = std::max(1, (int)std::ceil(H / cell));
  }
  std::vector<std::vector<uint16_t>> cells((size_t)nx * ny);
  for (int i = 0; i < nv; ++i) {
    if (nx == 0) { always.push_back((uint16_t)i); continue; }
    int ix0 = (int)std::floor((wb[i].lo[0] - ux0) / cell), ix1 = (int)std::floor((wb[i].hi[0] - ux0) / cell);
    int iy0 = (int)std::floor((wb[i].lo[1] - uy0) / cell), iy1 = (int)std::floor((wb[i].hi[1] - uy0) / cell);
    ix0 = std::max(0, ix0); iy0 = std::max(0, iy0);
    ix1 = std::min(nx - 1, ix1); iy1 = std::min(ny - 1, iy1);
    long span = (long)(ix1 - ix0 + 1) * (iy1 - iy0 + 1);
    if (span > 64 || span > (long)nx * ny / 4) { always.push_back((uint16_t)i); continue; }
    for (int iy = iy0; iy <= iy1; ++iy)
      for (int ix = ix0; ix <= ix1; ++ix) cells[(size_t)iy * nx + ix].push_back((uint16_t)i);
  }
  // layout
  blob.clear();
  offs.assign(4, 0);
  offs[0] = 0;
  blob.resize(sizeof(DVol<T>) * nv);
  if (nv) std::memcpy(blob.data(), recs.data(), sizeof(DVol<T>) * nv);
  align_to<T>(blob, 16);
  offs[1] = blob.size();
  for (uint16_t a : always) { blob.push_back((char)(a & 0xff)); blob.push_back((char)(a >> 8)); }
  align_to<T>(blob, 16);
  offs[2] = blob.size();
  uint32_t acc = 0;
  std::vector<uint32_t> starts;
  for (auto& c : cells) { starts.push_back(acc); acc += (uint32_t)c.size(); }
  starts.push_back(acc);
  size_t p0 = blob.size();
  blob.resize(p0 + 4 * starts.size());
  std::memcpy(blob.data() + p0, starts.data(), 4 * starts.size());
  align_to<T>(blob, 16);
  offs[3] = blob.size();
  for (auto& c : cells)
    for (uint16_t a : c) { blob.push_back((char)(a & 0xff)); blob.push_back((char)(a >> 8)); }
  align_to<T>(blob, 16);
  V.n_vol = nv;
  V.n_always = (int)always.size();
  V.nx = nx; V.ny = ny;
  V.gx0 = q<T>(ux0); V.gy0 = q<T>(uy0);
  V.cell = q<T>(cell); V.inv_cell = q<T>(1.0 / (double)q<T>(cell));
  V.max_events = s.max_events;
  V.n_groups = s.n_groups;
  V.seed = s.seed;
  V.eps_self = q<T>(s.l_ref * (sizeof(T) == 4 ? 1e-5 : 1e-9));
  V.blob_bytes = (uint32_t)blob.size();
}

template <typename T> void rebase(SceneView<T>& V, const std::vector<size_t>& offs, const char* base) {
  V.blob = base;
  V.vol = reinterpret_cast<const DVol<T>*>(base + offs[0]);
  V.always = reinterpret_cast<const uint16_t*>(base + offs[1]);
  V.cell_start = reinterpret_cast<const uint32_t*>(base + offs[2]);
  V.items = reinterpret_cast<const uint16_t*>(base + offs[3]);
}

std::vector<DTilt> tilt_table(const robast_scene& s) {
  std::vector<DTilt> t(s.n_vol);
  for (int i = 0; i < s.n_vol; ++i) {
    const robast_volume_desc& v = s.desc[i];
    std::memset(&t[i], 0, sizeof(DTilt));
    if (v.tilt_param < 0) continue;
    double Rb[9];
    rodrigues(v.e2, s.params[v.tilt_param + 1], Rb);
    for (int k = 0; k < 3; ++k) {
      t[i].pivot[k] = v.pivot[k];
      t[i].a1[k] = Rb[3 * k] * v.e1[0] + Rb[3 * k + 1] * v.e1[1] + Rb[3 * k + 2] * v.e1[2];
      t[i].a2[k] = v.e2[k];
    }
  }
  return t;
}

int upload(robast_scene* s) {
  std::vector<char> blob;
  std::vector<size_t> offs;
  if (s->precision == 32) compile_blob<float>(*s, blob, s->sf, offs);
  else compile_blob<double>(*s, blob, s->sd, offs);
  std::vector<DTilt> tilt = tilt_table(*s);
  if (blob.size() > s->blob_bytes || !s->d_blob) {
    if (s->d_blob) (void)hipFree(s->d_blob);
    s->d_blob = nullptr;
    hipError_t e = hipMalloc(&s->d_blob, std::max<size_t>(blob.size(), 16));
    if (e != hipSuccess) return e == hipErrorOutOfMemory ? fail(ROBAST_ENOMEM, "hipMalloc blob") : hip_fail(e, "hipMalloc blob");
  }
  s->blob_bytes = blob.size();
  hipError_t e = hipMemcpy(s->d_blob, blob.data(), blob.size(), hipMemcpyHostToDevice);
  if (e != hipSuccess) return hip_fail(e, "hipMemcpy blob");
  if (!s->d_tilt) {
    e = hipMalloc(&s->d_tilt, sizeof(DTilt) * std::max(1, s->n_vol));
    if (e != hipSuccess) return hip_fail(e, "hipMalloc tilt");
  }
  if (s->n_vol) {
    e = hipMemcpy(s->d_tilt, tilt.data(), sizeof(DTilt) * s->n_vol, hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(e, "hipMemcpy tilt");
  }
  if (!s->d_coef) {
    e = hipMalloc(&s->d_coef, sizeof(double) * 4 * s->n_groups);
    if (e != hipSuccess) return hip_fail(e, "hipMalloc coef");
  }
  if (s->precision == 32) rebase(s->sf, offs, (const char*)s->d_blob);
  else rebase(s->sd, offs, (const char*)s->d_blob);
  return ROBAST_OK;
}

}  // namespace

extern "C" {

int robast_abi_version(void) { return 1; }

const char* robast_status_string(int st) {
  switch (st) {
    case ROBAST_OK: return "ok";
    case ROBAST_EINVAL: return "invalid argument";
    case ROBAST_ENOMEM: return "out of device memory";
    case ROBAST_EHIP: return "HIP runtime error";
    case ROBAST_EUNSUPPORTED: return "unsupported";
    case ROBAST_EMISMATCH: return "mismatch";
  }
  return "unknown status";
}

const char* robast_last_error(void) { return g_err.c_str(); }

int robast_build_scene(const robast_scene_desc* desc, const double* params, int64_t n_params,
                       robast_scene** out) {
  if (!out) return fail(ROBAST_EINVAL, "out is NULL");
  *out = nullptr;
  int rc = validate(desc, params, n_params);
  if (rc) return rc;
  robast_scene* s = new robast_scene();
  s->precision = desc->precision;
  s->n_vol = desc->n_volumes;
  s->n_groups = desc->n_groups;
  s->max_events = desc->max_events;
  s->seed = desc->seed;
  s->l_ref = desc->l_ref;
  s->desc.assign(desc->volumes, desc->volumes + desc->n_volumes);
  s->params.assign(params, params + n_params);
  s->cfg.lds_cap = 48 * 1024;
  s->cfg.waves_mult = 1;
  s->cfg.max_blocks = 0;
  rc = upload(s);
  if (rc) {
    robast_destroy_scene(s);
    return rc;
  }
  *out = s;
  return ROBAST_OK;
}

int robast_update_params(robast_scene* s, const double* params, int64_t n_params) {
  if (!s || (!params && n_params > 0)) return fail(ROBAST_EINVAL, "NULL scene or params");
  if (n_params != (int64_t)s->params.size()) return fail(ROBAST_EMISMATCH, "parameter count differs from build");
  if (!finite_all(params, (int)n_params)) return fail(ROBAST_EINVAL, "non-finite parameter");
  s->params.assign(params, params + n_params);
  for (auto& v : s->desc) apply_params(v, s->params);
  return upload(s);
}

void robast_destroy_scene(robast_scene* s) {
  if (!s) return;
  if (s->d_blob) (void)hipFree(s->d_blob);
  if (s->d_tilt) (void)hipFree(s->d_tilt);
  if (s->d_coef) (void)hipFree(s->d_coef);
  delete s;
}

int robast_trace(robast_scene* s, const robast_rays* rays, int64_t n, const robast_hits* hits, uint32_t flags,
                 void* stream) {
  (void)flags;
  if (!s || !rays || !hits) return fail(ROBAST_EINVAL, "NULL scene, rays or hits");
  if (n < 0) return fail(ROBAST_EINVAL, "n < 0");
  if (n == 0) return ROBAST_OK;
  if (!rays->ox || !rays->oy || !rays->oz || !rays->dx || !rays->dy || !rays->dz)
    return fail(ROBAST_EINVAL, "NULL ray coordinate array");
  if (hits->x && (!hits->y || !hits->z)) return fail(ROBAST_EINVAL, "x given without y, z");
  if (hits->ux && (!hits->uy || !hits->uz)) return fail(ROBAST_EINVAL, "ux given without uy, uz");
  hipStream_t st = (hipStream_t)stream;
  hipError_t e;
  if (s->precision == 32) {
    RaysView<float> R{(const float*)rays->ox, (const float*)rays->oy, (const float*)rays->oz,
                      (const float*)rays->dx, (const float*)rays->dy, (const float*)rays->dz, rays->group,
                      rays->id_base};
    HitsView<float> H{hits->fate, hits->n_events, hits->last_vol, (float*)hits->x, (float*)hits->y,
                      (float*)hits->z, (float*)hits->ux, (float*)hits->uy, (float*)hits->uz,
                      (float*)hits->opl, hits->seq_hash, hits->group_sums};
    e = launch_trace<float>(s->sf, R, n, H, s->cfg, st);
  } else {
    RaysView<double> R{(const double*)rays->ox, (const double*)rays->oy, (const double*)rays->oz,
                       (const double*)rays->dx, (const double*)rays->dy, (const double*)rays->dz, rays->group,
                       rays->id_base};
    HitsView<double> H{hits->fate, hits->n_events, hits->last_vol, (double*)hits->x, (double*)hits->y,
                       (double*)hits->z, (double*)hits->ux, (double*)hits->uy, (double*)hits->uz,
                       (double*)hits->opl, hits->seq_hash, hits->group_sums};
    e = launch_trace<double>(s->sd, R, n, H, s->cfg, st);
  }
  if (e != hipSuccess) return hip_fail(e, "trace launch");
  return ROBAST_OK;
}

int robast_figures(robast_scene* s, const double* sums, double* fig, void* stream) {
  if (!s || !sums || !fig) return fail(ROBAST_EINVAL, "NULL scene, sums or figures");
  hipError_t e = launch_figures(sums, fig, s->n_groups, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "figures launch");
  return ROBAST_OK;
}

int robast_trace_backward(robast_scene* s, const robast_rays* rays, int64_t n, const double* sums,
                          const double* cot, double* grad, void* stream) {
  if (!s || !rays || !sums || !cot || !grad) return fail(ROBAST_EINVAL, "NULL scene, rays, sums, cot or grad");
  if (n < 0) return fail(ROBAST_EINVAL, "n < 0");
  if (n == 0) return ROBAST_OK;
  if (!rays->ox || !rays->oy || !rays->oz || !rays->dx || !rays->dy || !rays->dz)
    return fail(ROBAST_EINVAL, "NULL ray coordinate array");
  if (s->max_events > 64) return fail(ROBAST_EUNSUPPORTED, "backward supports max_events <= 64");
  hipStream_t st = (hipStream_t)stream;
  hipError_t e = launch_adj_coef(sums, cot, s->d_coef, s->n_groups, st);
  if (e != hipSuccess) return hip_fail(e, "coefficient launch");
  AdjView A{s->d_coef, grad, s->d_tilt, (int)s->params.size()};
  if (s->precision == 32) {
    RaysView<float> R{(const float*)rays->ox, (const float*)rays->oy, (const float*)rays->oz,
                      (const float*)rays->dx, (const float*)rays->dy, (const float*)rays->dz, rays->group,
                      rays->id_base};
    e = launch_backward<float>(s->sf, R, n, A, s->cfg, st);
  } else {
    RaysView<double> R{(const double*)rays->ox, (const double*)rays->oy, (const double*)rays->oz,
                       (const double*)rays->dx, (const double*)rays->dy, (const double*)rays->dz, rays->group,
                       rays->id_base};
    e = launch_backward<double>(s->sd, R, n, A, s->cfg, st);
  }
  if (e != hipSuccess) return hip_fail(e, "backward launch");
  return ROBAST_OK;
}

}  // extern "C"
