// C ABI of the tracer: argument validation, the scene compiler and launches.
//
// The scene compiler turns the caller's volume descriptors (roles and shapes
// of §2.1/§2.2) into device records in the kernel precision, computes
// conservative local and world bounds for each volume, and builds an XY
// uniform grid of candidate lists used by the non-sequential search.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <climits>
#include <cmath>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/robast.h"
#include "batch.hpp"
#include "boundary.hpp"
#include "binning.hpp"
#include "kernels.hpp"
#include "scene_layout.hpp"
#include "update.hpp"

using namespace robast;

// Binning workspace of robast_trace_static, for callers that cannot
// allocate: a fixed array in device memory.  Each GPU the library runs on
// holds its own copy, at its own address, until the process ends; calls on
// one GPU share it.  Host code must not pass `scratch` itself to a kernel
// (the name is a host-side stand-in): it uses the device address found by
// hipGetSymbolAddress on each device.
constexpr size_t kStaticScratchBytes = size_t(64) << 20;
static __device__ __align__(256) char scratch[kStaticScratchBytes];

namespace {

constexpr int kMaxDevices = 64;
void* g_scratch_dev[kMaxDevices] = {};
std::mutex g_scratch_mu;

thread_local std::string g_err;

int fail(int code, const std::string& msg) {
  g_err = msg;
  return code;
}
int hip_fail(hipError_t e, const char* what) {
  g_err = std::string(what) + ": " + hipGetErrorString(e);
  return ROBAST_EHIP;
}

// Device address of the static workspace on the current device, looked up
// once per device (with that device current) on the first call there.
int static_scratch(void** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  if (dev < 0 || dev >= kMaxDevices) return fail(ROBAST_EUNSUPPORTED, "device index beyond the static workspace table");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) return hip_fail(e, "hipGetSymbolAddress(scratch)");
    g_scratch_dev[dev] = p;
  }
  *out = g_scratch_dev[dev];
  return ROBAST_OK;
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
// Checks of one volume descriptor (shape, outline, role, sizes, the
// geometry its parameters give, parameter indices).
int validate_volume(const robast_volume_desc& v, int i, int64_t n_params) {
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
  if (v.role == ROBAST_LENS && !(v.p[15] >= 0.0 && std::isfinite(v.p[15])))
    return fail(ROBAST_EINVAL, "lens absorption length p[15] must be finite and >= 0" + at);
  if (v.role == ROBAST_LENS && v.p[14] != 0.0 && !(v.p[13] > 0.0 && v.p[14] > 0.0))
    return fail(ROBAST_EINVAL, "lens dispersion law needs A = p[13] > 0 and B = p[14] > 0" + at);
  if (v.role == ROBAST_LENS && v.p[14] != 0.0 && v.shape == ROBAST_HEXCONE)
    return fail(ROBAST_EUNSUPPORTED, "dispersive lens faces must not be cones" + at);
  if (v.role == ROBAST_LENS && v.shape != ROBAST_BOX && v.shape != ROBAST_PLANE && v.shape != ROBAST_SPHERE &&
      v.shape != ROBAST_ASPHERE)
    return fail(ROBAST_EUNSUPPORTED, "lens faces must be planes, spheres, aspheres or boxes" + at);
  int ns = v.shape == ROBAST_SPHERE ? 1 : v.shape == ROBAST_ASPHERE ? 8 : v.shape == ROBAST_HEXCONE ? 4 : 0;
  if (v.shape_param >= 0 && (ns == 0 || v.shape_param + ns > n_params))
    return fail(ROBAST_EINVAL, "shape_param out of range" + at);
  if (v.tilt_param >= 0 && v.tilt_param + 2 > n_params) return fail(ROBAST_EINVAL, "tilt_param out of range" + at);
  if (v.shape_param < -1 || v.tilt_param < -1) return fail(ROBAST_EINVAL, "negative parameter index" + at);
  return ROBAST_OK;
}

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
    int rc = validate_volume(d->volumes[i], i, n_params);
    if (rc) return rc;
  }
  return ROBAST_OK;
}

}  // namespace

struct robast_scene {
  int precision = 32, n_vol = 0, n_groups = 1, max_events = 16;
  uint64_t seed = 0;
  double l_ref = 1.0;
  std::vector<robast_volume_desc> desc;
  std::vector<double> params;  // parameters of the last host build (device updates leave them)
  void* d_blob = nullptr;      // two table slots of slot_cap bytes; the view points at the live one
  size_t blob_bytes = 0, slot_cap = 0;
  DTilt* d_tilt = nullptr;     // two tilt-table slots of n_vol records
  double* d_coef = nullptr;    // n_groups * 4 backward coefficients
  int cell_choice = 0;         // index into kCellFactors chosen by the last upload
  void* d_view = nullptr;      // the live view (sf / sd with device pointers), read by every kernel
  // device parameter updates: per-volume and per-group tables of the last
  // host build (UpdVol[n_vol] | UpdGroup[n_grp] | members | z-range scratch),
  // the job record and a one-entry array pointing at it
  void* d_upd = nullptr;
  size_t upd_bytes = 0;
  void* d_job = nullptr;
  void* d_jobptr = nullptr;
  std::vector<int> upd_group;          // filled by the scene compiler
  std::vector<double> upd_gpad;
  std::vector<UpdGroup> upd_groups;
  std::vector<uint16_t> upd_members;
  void* d_check = nullptr;     // sequence-check counter of the backward debug mode
  SceneView<float> sf{};
  SceneView<double> sd{};
  LaunchCfg cfg{};
  robast_tuning tuning{};
  // photon binning: plane z = bin_z, square of side bin_side from (bin_x0, bin_y0)
  double bin_z = 0.0, bin_x0 = 0.0, bin_y0 = 0.0, bin_side = 1.0;
  void* d_work = nullptr;                    // binning workspace
  size_t work_bytes = 0;
  // the binned order kept by a trace call for the next backward call
  bool kept = false;
  robast_rays kept_rays{};
  int64_t kept_n = 0;
  void* kept_records = nullptr;
  // path records of the last trace that kept its order (one-shot, like the
  // order): kPathSlots words per photon, then the long-record list and count
  void* d_path = nullptr;
  int64_t path_cap = 0;
  bool path_ok = false, path_binned = false;
  robast_rays path_rays{};
  int64_t path_n = 0;
};

// LDS a workgroup may use for a scene's tables: three workgroups of four
// waves (the trace kernel's occupancy) share the 160 KiB of a CU.
constexpr int kLdsCu = 160 * 1024;
constexpr int kLdsCap = (kLdsCu / 3) & ~15;

struct robast_batch {
  int precision = 32;
  std::vector<robast_scene*> scenes;
  int64_t n_photons = 0, n_groups = 0, n_params = 0;
  int max_events = 0, max_params = 0, n_items = 0;
  int shapes = 0;                  // bit 1 << shape of every shape in any variant
  uint32_t blob_cap = 0, blob_cap_bwd = 0;
  void* d_vars = nullptr;          // BatchVariant<T>[n_scenes]
  BatchItem* d_items = nullptr;    // n_items
  uint32_t* d_queue = nullptr;     // kQueueCounters counters
  double* d_coef = nullptr;        // n_groups * 4
  // photon binning per variant (fixed at build: geometry, bins, workspace)
  bool bin = false;
  int64_t bins = 0;
  int64_t* d_offsets = nullptr;    // n_scenes + 1
  BinGeom* d_geo = nullptr;        // n_scenes
  void* d_work = nullptr;
  bool kept = false;
  robast_rays kept_rays{};
  // path records of the last forward launch that kept its order (one-shot)
  uint32_t* d_path = nullptr;
  bool path_ok = false;
  robast_rays path_rays{};
  // parameter updates of the variants: their update jobs and parameter offsets
  void* d_jobs = nullptr;          // n_scenes job pointers
  int64_t* d_poff = nullptr;       // n_scenes offsets into the concatenated parameters
  bool repeated = false;           // a scene appears more than once
  // launch shape of the forward launch (robast_autotune_batch may change it)
  std::vector<int64_t> offsets;    // n_scenes + 1 photon offsets
  uint32_t chunk = 0, block = 256;
  size_t items_cap = 0;            // BatchItem slots allocated at d_items
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
  r.absl = v.role == ROBAST_LENS ? q<T>(v.p[15]) : T(0);
  if (v.role == ROBAST_LENS && v.p[14] != 0.0) { r.p[10] = q<T>(v.p[13]); r.p[11] = q<T>(v.p[14]); }
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

// Points on a volume's surface (world), spaced about h apart.
void surface_samples(const robast_volume_desc& v, double h, std::vector<std::array<double, 3>>& out) {
  double I[9];
  inv3(v.Q, I);
  auto emit = [&](double x, double y, double z) {
    std::array<double, 3> w;
    for (int i = 0; i < 3; ++i) w[i] = v.c[i] + I[3 * i] * x + I[3 * i + 1] * y + I[3 * i + 2] * z;
    out.push_back(w);
  };
  double slope;
  Box3 lb = local_bounds(v, slope);
  switch (v.shape) {
    case ROBAST_PLANE: case ROBAST_SPHERE: case ROBAST_ASPHERE: {
      const double* o = v.o;
      auto inside = [&](double x, double y) {
        double r = std::hypot(x, y);
        switch (v.outline) {
          case ROBAST_DISC: return r <= o[0] + h;
          case ROBAST_ANNULUS: return r >= o[0] - h && r <= o[1] + h;
          case ROBAST_RECT: return std::fabs(x) <= o[0] + h && std::fabs(y) <= o[1] + h;
          case ROBAST_HEX:
            for (int k = 0; k < 3; ++k)
              if (std::fabs(x * std::cos(k * M_PI / 3) + y * std::sin(k * M_PI / 3)) > o[0] + h) return false;
            return true;
          case ROBAST_SECTOR: {
            if (r < o[0] - h || r > o[1] + h) return false;
            if (o[3] - o[2] >= 2 * M_PI - 1e-12) return true;
            double ph = std::atan2(y, x) - o[2];
            ph = std::fmod(ph, 2 * M_PI);
            if (ph < 0) ph += 2 * M_PI;
            double tol = r > h ? h / r : M_PI;
            return ph <= o[3] - o[2] + tol || ph >= 2 * M_PI - tol;
          }
        }
        return true;
      };
      auto sag = [&](double x, double y) {
        double r2 = x * x + y * y;
        if (v.shape == ROBAST_SPHERE) {
          double c = v.p[0], q = 1.0 - c * c * r2;
          return q > 0 ? c * r2 / (1.0 + std::sqrt(q)) : 1.0 / c;
        }
        if (v.shape == ROBAST_ASPHERE) return sag_asph(v.p + 1, r2 / (v.p[0] * v.p[0]));
        return 0.0;
      };
      for (double x = lb.lo[0]; x <= lb.hi[0] + h; x += h)
        for (double y = lb.lo[1]; y <= lb.hi[1] + h; y += h) {
          double xx = std::min(x, lb.hi[0]), yy = std::min(y, lb.hi[1]);
          if (inside(xx, yy)) emit(xx, yy, sag(xx, yy));
        }
      break;
    }
    case ROBAST_CYLINDER: {
      int nt = std::max(8, (int)std::ceil(2 * M_PI * v.p[0] / h));
      for (int i = 0; i < nt; ++i)
        for (double z = 0; z <= v.p[1] + h; z += h)
          emit(v.p[0] * std::cos(2 * M_PI * i / nt), v.p[0] * std::sin(2 * M_PI * i / nt), std::min(z, v.p[1]));
      break;
    }
    case ROBAST_BOX: case ROBAST_HEXCONE: default: {
      // the local box (conservative: its points cover the surface's projection)
      for (double x = lb.lo[0]; x <= lb.hi[0] + h; x += h)
        for (double y = lb.lo[1]; y <= lb.hi[1] + h; y += h)
          for (int zz = 0; zz < 2; ++zz)
            emit(std::min(x, lb.hi[0]), std::min(y, lb.hi[1]), zz ? lb.hi[2] : lb.lo[2]);
      break;
    }
  }
}

struct GroupBuild {
  double Q[9], c[3];
  std::vector<int> members;
  double zmin = 1e300, zmax = -1e300, x0 = 1e300, y0 = 1e300, x1 = -1e300, y1 = -1e300, cell = 1.0;
  double zpad = 0.0;          // padding of the z-slab
  int nx = 0, ny = 0;
  std::vector<std::vector<uint16_t>> cells;
  std::vector<double> step;   // surface sampling step of each member's rasterisation
};

void to_group(const GroupBuild& g, const double* w, double* x) {
  double r[3] = {w[0] - g.c[0], w[1] - g.c[1], w[2] - g.c[2]};
  for (int i = 0; i < 3; ++i) x[i] = g.Q[3 * i] * r[0] + g.Q[3 * i + 1] * r[1] + g.Q[3 * i + 2] * r[2];
}

// Partition the volumes into the always-list and candidate groups and
// rasterise each group's members onto its grid.
void build_groups(const robast_scene& s, const std::vector<Box3>& wb, std::vector<uint16_t>& always,
                  std::vector<GroupBuild>& groups, double cell_factor) {
  int nv = s.n_vol;
  always.clear();
  groups.clear();
  if (nv <= 4) {
    for (int i = 0; i < nv; ++i) always.push_back((uint16_t)i);
    return;
  }
  double ux0 = 1e300, uy0 = 1e300, uz0 = 1e300, ux1 = -1e300, uy1 = -1e300, uz1 = -1e300;
  for (int i = 0; i < nv; ++i) {
    ux0 = std::min(ux0, wb[i].lo[0]); uy0 = std::min(uy0, wb[i].lo[1]); uz0 = std::min(uz0, wb[i].lo[2]);
    ux1 = std::max(ux1, wb[i].hi[0]); uy1 = std::max(uy1, wb[i].hi[1]); uz1 = std::max(uz1, wb[i].hi[2]);
  }
  double uarea = (ux1 - ux0) * (uy1 - uy0), uz = uz1 - uz0;
  std::vector<double> fa(nv);
  for (int i = 0; i < nv; ++i) fa[i] = (wb[i].hi[0] - wb[i].lo[0]) * (wb[i].hi[1] - wb[i].lo[1]);
  std::vector<double> fs = fa;
  std::nth_element(fs.begin(), fs.begin() + nv / 2, fs.end());
  double fmed = fs[nv / 2];
  std::vector<int> rest;
  std::vector<char> placed(nv, 0);
  // always-list: volumes covering much of the scene, and long slanted ones
  // (struts) that would merge separate z-layers
  for (int i = 0; i < nv; ++i) {
    double z = wb[i].hi[2] - wb[i].lo[2];
    if (fa[i] > 0.2 * uarea || (uz > 0 && z > 0.5 * uz && fa[i] > 10.0 * fmed)) {
      always.push_back((uint16_t)i);
      placed[i] = 1;
    }
  }
  // panels sharing one untilted frame: a group in that frame
  for (int i = 0; i < nv; ++i) {
    const robast_volume_desc& v = s.desc[i];
    if (placed[i] || v.tilt_param < 0) continue;
    GroupBuild g;
    std::memcpy(g.Q, v.Q0, sizeof g.Q);
    std::memcpy(g.c, v.c0, sizeof g.c);
    for (int j = i; j < nv; ++j) {
      const robast_volume_desc& u = s.desc[j];
      if (placed[j] || u.tilt_param < 0) continue;
      if (std::memcmp(u.Q0, v.Q0, sizeof u.Q0) == 0 && std::memcmp(u.c0, v.c0, sizeof u.c0) == 0) {
        g.members.push_back(j);
        placed[j] = 1;
      }
    }
    if (g.members.size() >= 2) groups.push_back(g);
    else for (int j : g.members) placed[j] = 0;
    if (g.members.size() < 2) rest.push_back(i), placed[i] = 1;
  }
  for (int i = 0; i < nv; ++i)
    if (!placed[i]) rest.push_back(i);
  // world-frame layers of overlapping z-extent
  std::sort(rest.begin(), rest.end(), [&](int a, int b) { return wb[a].lo[2] < wb[b].lo[2]; });
  for (size_t k = 0; k < rest.size();) {
    GroupBuild g;
    const double I[9] = {1, 0, 0, 0, 1, 0, 0, 0, 1};
    std::memcpy(g.Q, I, sizeof g.Q);
    g.c[0] = g.c[1] = g.c[2] = 0.0;
    double top = wb[rest[k]].hi[2];
    size_t j = k;
    while (j < rest.size() && wb[rest[j]].lo[2] <= top) {
      top = std::max(top, wb[rest[j]].hi[2]);
      g.members.push_back(rest[j]);
      ++j;
    }
    k = j;
    if (g.members.size() >= 2) groups.push_back(g);
    else always.push_back((uint16_t)g.members[0]);
  }
  // rasterise
  for (GroupBuild& g : groups) {
    std::vector<double> areas;
    for (int m : g.members) {
      double slope;
      Box3 lb = local_bounds(s.desc[m], slope);
      double I[9];
      inv3(s.desc[m].Q, I);
      double mx0 = 1e300, my0 = 1e300, mx1 = -1e300, my1 = -1e300;
      for (int cc = 0; cc < 8; ++cc) {
        double xl[3] = {(cc & 1) ? lb.hi[0] : lb.lo[0], (cc & 2) ? lb.hi[1] : lb.lo[1], (cc & 4) ? lb.hi[2] : lb.lo[2]};
        double w[3], x[3];
        for (int i = 0; i < 3; ++i)
          w[i] = s.desc[m].c[i] + I[3 * i] * xl[0] + I[3 * i + 1] * xl[1] + I[3 * i + 2] * xl[2];
        to_group(g, w, x);
        g.zmin = std::min(g.zmin, x[2]); g.zmax = std::max(g.zmax, x[2]);
        mx0 = std::min(mx0, x[0]); mx1 = std::max(mx1, x[0]); my0 = std::min(my0, x[1]); my1 = std::max(my1, x[1]);
      }
      g.x0 = std::min(g.x0, mx0); g.x1 = std::max(g.x1, mx1); g.y0 = std::min(g.y0, my0); g.y1 = std::max(g.y1, my1);
      areas.push_back(std::max((mx1 - mx0) * (my1 - my0), 1e-30));
    }
    double zp = 1e-5 * (g.zmax - g.zmin + s.l_ref);
    g.zpad = zp;
    g.zmin -= zp; g.zmax += zp;
    double xp = 1e-5 * (g.x1 - g.x0 + g.y1 - g.y0 + s.l_ref);
    g.x0 -= xp; g.y0 -= xp; g.x1 += xp; g.y1 += xp;
    // cell: cell_factor x the side of the median footprint of the members
    // that have one (walls seen edge-on have none), at least 1/256 of the
    // group's extent
    double W = g.x1 - g.x0, H = g.y1 - g.y0;
    std::vector<double> real;
    for (double a : areas)
      if (a > 1e-4 * W * H) real.push_back(a);
    if (real.empty()) real.push_back(W * H / 16.0);
    std::nth_element(real.begin(), real.begin() + real.size() / 2, real.end());
    g.cell = cell_factor * std::sqrt(real[real.size() / 2]);
    g.cell = std::max(g.cell, std::max(W, H) / 256.0);
    g.nx = std::max(1, (int)std::ceil((g.x1 - g.x0) / g.cell));
    g.ny = std::max(1, (int)std::ceil((g.y1 - g.y0) / g.cell));
    g.cells.assign((size_t)g.nx * g.ny, {});
    std::vector<std::array<double, 3>> pts;
    std::vector<int> mark((size_t)g.nx * g.ny, -1);
    for (int m : g.members) {
      double slope;
      Box3 lb = local_bounds(s.desc[m], slope);
      double ext = std::max(std::max(lb.hi[0] - lb.lo[0], lb.hi[1] - lb.lo[1]), lb.hi[2] - lb.lo[2]);
      double h = std::max(g.cell / 6.0, ext / 256.0);
      g.step.push_back(h);
      pts.clear();
      surface_samples(s.desc[m], h, pts);
      double pad = h + 1e-5 * s.l_ref;
      for (auto& w : pts) {
        double x[3];
        to_group(g, w.data(), x);
        for (int q = 0; q < 5; ++q) {
          double px = x[0] + (q == 1 ? pad : q == 2 ? -pad : 0.0), py = x[1] + (q == 3 ? pad : q == 4 ? -pad : 0.0);
          int ix = (int)std::floor((px - g.x0) / g.cell), iy = (int)std::floor((py - g.y0) / g.cell);
          if (ix < 0 || iy < 0 || ix >= g.nx || iy >= g.ny) continue;
          size_t ci = (size_t)iy * g.nx + ix;
          if (mark[ci] != m) { mark[ci] = m; g.cells[ci].push_back((uint16_t)m); }
        }
      }
    }
  }
}

// Build the blob for precision T and fill the view offsets (host addresses
// are rebased to the device allocation by the caller).
// Binning frame: the xy extent of the mirrors and lenses (of every volume
// if there are none) on the plane through their lowest point.
void set_bin_frame(robast_scene& s, const std::vector<Box3>& wb) {
  double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
  for (int pass = 0; pass < 2 && !(lo[0] <= hi[0]); ++pass)
    for (int i = 0; i < s.n_vol; ++i) {
      const int role = s.desc[i].role;
      if (pass == 0 && role != ROBAST_MIRROR && role != ROBAST_LENS) continue;
      for (int k = 0; k < 3; ++k) {
        lo[k] = std::min(lo[k], wb[i].lo[k]);
        hi[k] = std::max(hi[k], wb[i].hi[k]);
      }
    }
  if (!(lo[0] <= hi[0]) || !std::isfinite(lo[0] + lo[1] + lo[2] + hi[0] + hi[1])) {
    s.bin_z = 0.0; s.bin_x0 = -1.0; s.bin_y0 = -1.0; s.bin_side = 2.0;
    return;
  }
  s.bin_z = lo[2];
  s.bin_side = std::max({hi[0] - lo[0], hi[1] - lo[1], 1e-9 * s.l_ref});
  s.bin_x0 = 0.5 * (lo[0] + hi[0]) - 0.5 * s.bin_side;
  s.bin_y0 = 0.5 * (lo[1] + hi[1]) - 0.5 * s.bin_side;
}

template <typename T>
void compile_blob(robast_scene& s, std::vector<char>& blob, SceneView<T>& V, std::vector<size_t>& offs,
                  double cell_factor) {
  int nv = s.n_vol;
  std::vector<DVol<T>> recs(nv);
  std::vector<Box3> wb(nv);
  for (int i = 0; i < nv; ++i) fill_record<T>(recs[i], s.desc[i], wb[i], s.l_ref);
  set_bin_frame(s, wb);
  std::vector<uint16_t> always;
  std::vector<GroupBuild> groups;
  build_groups(s, wb, always, groups, cell_factor);
  // what device parameter updates need of the groups: frames, slab padding,
  // members, and how far a member's surface may move across its group before
  // it could leave the cells it is listed in (samples every h, each padded by
  // h + 1e-5 L_ref: a quarter of h is covered)
  s.upd_group.assign(nv, -1);
  s.upd_gpad.assign(nv, -1.0);
  s.upd_groups.clear();
  s.upd_members.clear();
  for (size_t gi = 0; gi < groups.size(); ++gi) {
    const GroupBuild& g = groups[gi];
    UpdGroup ug{};
    std::memcpy(ug.Q, g.Q, sizeof ug.Q);
    std::memcpy(ug.c, g.c, sizeof ug.c);
    ug.zpad = g.zpad;
    ug.first = (int32_t)s.upd_members.size();
    ug.count = (int32_t)g.members.size();
    for (size_t k = 0; k < g.members.size(); ++k) {
      const int m = g.members[k];
      s.upd_members.push_back((uint16_t)m);
      s.upd_group[m] = (int)gi;
      s.upd_gpad[m] = 0.25 * g.step[k];
    }
    s.upd_groups.push_back(ug);
  }
  std::vector<GroupRec<T>> grecs(groups.size());
  std::vector<uint32_t> starts;
  std::vector<uint16_t> items;
  for (size_t gi = 0; gi < groups.size(); ++gi) {
    const GroupBuild& g = groups[gi];
    GroupRec<T>& r = grecs[gi];
    std::memset(&r, 0, sizeof r);
    for (int i = 0; i < 9; ++i) r.Q[i] = q<T>(g.Q[i]);
    for (int i = 0; i < 3; ++i) r.c[i] = q<T>(g.c[i]);
    r.zmin = std::nextafter(q<T>(g.zmin), (T)-INFINITY); r.zmax = std::nextafter(q<T>(g.zmax), (T)INFINITY);
    r.x0 = std::nextafter(q<T>(g.x0), (T)-INFINITY); r.y0 = std::nextafter(q<T>(g.y0), (T)-INFINITY);
    r.cell = q<T>(g.cell); r.inv_cell = q<T>(1.0 / (double)r.cell);
    r.nx = g.nx; r.ny = g.ny;
    r.start = (uint32_t)starts.size();
    for (auto& c : g.cells) { starts.push_back((uint32_t)items.size()); items.insert(items.end(), c.begin(), c.end()); }
  }
  starts.push_back((uint32_t)items.size());
  // layout: volumes | groups | always | cell_start | items
  blob.clear();
  offs.assign(5, 0);
  blob.resize(sizeof(DVol<T>) * nv);
  if (nv) std::memcpy(blob.data(), recs.data(), sizeof(DVol<T>) * nv);
  align_to<T>(blob, 16);
  offs[4] = blob.size();
  size_t p0 = blob.size();
  blob.resize(p0 + sizeof(GroupRec<T>) * grecs.size());
  if (!grecs.empty()) std::memcpy(blob.data() + p0, grecs.data(), sizeof(GroupRec<T>) * grecs.size());
  align_to<T>(blob, 16);
  offs[1] = blob.size();
  for (uint16_t a : always) { blob.push_back((char)(a & 0xff)); blob.push_back((char)(a >> 8)); }
  align_to<T>(blob, 16);
  offs[2] = blob.size();
  p0 = blob.size();
  blob.resize(p0 + 4 * starts.size());
  std::memcpy(blob.data() + p0, starts.data(), 4 * starts.size());
  align_to<T>(blob, 16);
  offs[3] = blob.size();
  for (uint16_t a : items) { blob.push_back((char)(a & 0xff)); blob.push_back((char)(a >> 8)); }
  align_to<T>(blob, 16);
  V.n_vol = nv;
  V.shapes = 0;
  V.dispersive = 0;
  for (const auto& v : s.desc) {
    V.shapes |= 1 << v.shape;
    if (v.role == ROBAST_LENS && v.p[14] != 0.0) V.dispersive = 1;
  }
  V.n_always = (int)always.size();
  V.n_grp = (int)grecs.size();
  V.max_events = s.max_events;
  V.n_groups = s.n_groups;
  V.seed = s.seed;
  V.eps_self = q<T>(s.l_ref * (sizeof(T) == 4 ? 1e-5 : 1e-9));
  V.eps_tie = 1e-12 * s.l_ref;
  V.blob_bytes = (uint32_t)blob.size();
}

template <typename T> void rebase(SceneView<T>& V, const std::vector<size_t>& offs, const char* base) {
  V.blob = base;
  V.vol = reinterpret_cast<const DVol<T>*>(base + offs[0]);
  V.groups = reinterpret_cast<const GroupRec<T>*>(base + offs[4]);
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

// Candidate-grid cells of the scene compiler: the finest of these factors
// (cell side = factor x the side of the median member footprint) whose blob
// still lets the trace kernel keep four workgroups per CU with the tables in
// LDS.  Finer cells list fewer candidates per cell, so a search makes fewer
// box tests and exact tests of neighbouring panels (Schwarzschild-Couder:
// trace 21.7 ms at 0.5, 19.0 ms at 0.14); the coarsest is used when none fits.
constexpr double kCellFactors[] = {0.14, 0.18, 0.25, 0.35, 0.5};

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// The device tables of a volume for parameter updates (its descriptor with
// the current parameters applied).
UpdVol upd_vol(const robast_scene& s, int i) {
  const robast_volume_desc& v = s.desc[i];
  UpdVol u{};
  std::memcpy(u.Q, v.Q, sizeof u.Q);
  std::memcpy(u.c, v.c, sizeof u.c);
  std::memcpy(u.Q0, v.Q0, sizeof u.Q0);
  std::memcpy(u.c0, v.c0, sizeof u.c0);
  std::memcpy(u.pivot, v.pivot, sizeof u.pivot);
  std::memcpy(u.e1, v.e1, sizeof u.e1);
  std::memcpy(u.e2, v.e2, sizeof u.e2);
  std::memcpy(u.p, v.p, sizeof u.p);
  double slope;
  const Box3 lb = local_bounds(v, slope);
  for (int k = 0; k < 3; ++k) { u.lb_lo[k] = lb.lo[k]; u.lb_hi[k] = lb.hi[k]; }
  u.rmin = outline_rmin(v);
  u.rmax = outline_rmax(v);
  u.gpad = s.upd_gpad.empty() ? -1.0 : s.upd_gpad[i];
  u.shape = v.shape; u.outline = v.outline; u.sparam = v.shape_param; u.tparam = v.tilt_param;
  u.group = s.upd_group.empty() ? -1 : s.upd_group[i];
  u.role = v.role;
  return u;
}

template <typename T> int set_job(robast_scene* s, const SceneView<T>& V) {
  char* base = (char*)s->d_upd;
  const size_t ov = 0, og = align256(sizeof(UpdVol) * s->n_vol), om = og + align256(sizeof(UpdGroup) * V.n_grp),
               oz = om + align256(sizeof(uint16_t) * s->upd_members.size()),
               op = oz + align256(sizeof(double) * 2 * std::max(1, s->n_vol));
  UpdJob<T> j{};
  j.view = (SceneView<T>*)s->d_view;
  j.slot[0] = (char*)s->d_blob;
  j.slot[1] = (char*)s->d_blob + s->slot_cap;
  j.tilt[0] = s->d_tilt;
  j.tilt[1] = s->d_tilt + std::max(1, s->n_vol);
  j.vols = (const UpdVol*)(base + ov);
  j.groups = (const UpdGroup*)(base + og);
  j.members = (const uint16_t*)(base + om);
  j.zr = (double*)(base + oz);
  j.pn = (double*)(base + op);
  j.n_vol = s->n_vol;
  j.n_grp = V.n_grp;
  j.n_params = (int32_t)s->params.size();
  j.blob_bytes = (uint32_t)s->blob_bytes;
  j.l_ref = s->l_ref;
  hipError_t e = hipMemcpy(s->d_job, &j, sizeof j, hipMemcpyHostToDevice);
  return e == hipSuccess ? ROBAST_OK : hip_fail(e, "hipMemcpy update job");
}

// Host build of the scene's device tables (a new scene, or new parameters
// by robast_set_params): compile, then write slot 0, the tilt table, the
// view and the tables of device updates.  Called with no kernel of the
// scene in flight (robast_set_params synchronises the device first).
int upload(robast_scene* s) {
  std::vector<char> blob;
  std::vector<size_t> offs;
  const size_t sums_lds = (size_t)s->n_groups * 64 <= 16384 ? (size_t)s->n_groups * 64 : 0;
  const size_t budget = ((size_t)kLdsCu / 4 - sums_lds) & ~(size_t)15;
  // a parameter update starts from the previous choice (the tables change
  // little), a new scene from the finest
  const int n_f = (int)(sizeof(kCellFactors) / sizeof(kCellFactors[0]));
  for (int k = s->cell_choice; k < n_f; ++k) {
    blob.clear();
    offs.clear();
    if (s->precision == 32) compile_blob<float>(*s, blob, s->sf, offs, kCellFactors[k]);
    else compile_blob<double>(*s, blob, s->sd, offs, kCellFactors[k]);
    s->cell_choice = k;
    if (blob.size() <= budget) break;
  }
  std::vector<DTilt> tilt = tilt_table(*s);
  const size_t need = align256(std::max<size_t>(blob.size(), 16));
  hipError_t e = hipSuccess;
  if (need > s->slot_cap || !s->d_blob) {
    if (s->d_blob) (void)hipFree(s->d_blob);
    s->d_blob = nullptr;
    s->slot_cap = 0;
    e = hipMalloc(&s->d_blob, 2 * need);
    if (e != hipSuccess) return e == hipErrorOutOfMemory ? fail(ROBAST_ENOMEM, "hipMalloc blob") : hip_fail(e, "hipMalloc blob");
    s->slot_cap = need;
  }
  s->blob_bytes = blob.size();
  e = hipMemcpy(s->d_blob, blob.data(), blob.size(), hipMemcpyHostToDevice);
  if (e != hipSuccess) return hip_fail(e, "hipMemcpy blob");
  const int nt = std::max(1, s->n_vol);
  if (!s->d_tilt) {
    e = hipMalloc(&s->d_tilt, 2 * sizeof(DTilt) * nt);
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
  if (!s->d_view) {
    e = hipMalloc(&s->d_view, sizeof(SceneView<double>));
    if (e != hipSuccess) return hip_fail(e, "hipMalloc view");
  }
  if (s->precision == 32) {
    rebase(s->sf, offs, (const char*)s->d_blob);
    s->sf.self = (const SceneView<float>*)s->d_view;
    s->sf.tilt = s->d_tilt;
    e = hipMemcpy(s->d_view, &s->sf, sizeof(SceneView<float>), hipMemcpyHostToDevice);
  } else {
    rebase(s->sd, offs, (const char*)s->d_blob);
    s->sd.self = (const SceneView<double>*)s->d_view;
    s->sd.tilt = s->d_tilt;
    e = hipMemcpy(s->d_view, &s->sd, sizeof(SceneView<double>), hipMemcpyHostToDevice);
  }
  if (e != hipSuccess) return hip_fail(e, "hipMemcpy view");
  // tables of device parameter updates
  const int n_grp = (int)s->upd_groups.size();
  std::vector<char> upd(align256(sizeof(UpdVol) * s->n_vol) + align256(sizeof(UpdGroup) * n_grp) +
                        align256(sizeof(uint16_t) * s->upd_members.size()) + align256(sizeof(double) * 2 * nt) +
                        align256(sizeof(double) * std::max<size_t>(1, s->params.size())));
  for (int i = 0; i < s->n_vol; ++i) {
    const UpdVol u = upd_vol(*s, i);
    std::memcpy(upd.data() + sizeof(UpdVol) * i, &u, sizeof u);
  }
  const size_t og = align256(sizeof(UpdVol) * s->n_vol), om = og + align256(sizeof(UpdGroup) * n_grp);
  if (n_grp) std::memcpy(upd.data() + og, s->upd_groups.data(), sizeof(UpdGroup) * n_grp);
  if (!s->upd_members.empty())
    std::memcpy(upd.data() + om, s->upd_members.data(), sizeof(uint16_t) * s->upd_members.size());
  if (upd.size() > s->upd_bytes || !s->d_upd) {
    if (s->d_upd) (void)hipFree(s->d_upd);
    s->d_upd = nullptr;
    s->upd_bytes = 0;
    e = hipMalloc(&s->d_upd, std::max<size_t>(upd.size(), 256));
    if (e != hipSuccess) return hip_fail(e, "hipMalloc update tables");
    s->upd_bytes = upd.size();
  }
  e = hipMemcpy(s->d_upd, upd.data(), upd.size(), hipMemcpyHostToDevice);
  if (e != hipSuccess) return hip_fail(e, "hipMemcpy update tables");
  if (!s->d_job) {
    e = hipMalloc(&s->d_job, std::max(sizeof(UpdJob<float>), sizeof(UpdJob<double>)));
    if (e == hipSuccess) e = hipMalloc(&s->d_jobptr, sizeof(void*));
    if (e == hipSuccess) e = hipMemcpy(s->d_jobptr, &s->d_job, sizeof(void*), hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(e, "hipMalloc update job");
  }
  return s->precision == 32 ? set_job<float>(s, s->sf) : set_job<double>(s, s->sd);
}

template <typename T> RaysView<T> rays_view(const robast_rays* r) {
  RaysView<T> R{(const T*)r->ox, (const T*)r->oy, (const T*)r->oz, (const T*)r->dx, (const T*)r->dy,
                (const T*)r->dz, r->group, r->id_base};
  R.lam = (const T*)r->lambda;
  return R;
}

template <typename T> HitsView<T> hits_view(const robast_hits* h) {
  HitsView<T> H{h->fate, h->n_events, h->last_vol, (T*)h->x, (T*)h->y, (T*)h->z, (T*)h->ux, (T*)h->uy,
                (T*)h->uz, (T*)h->opl, h->seq_hash, h->group_sums};
  H.seq_log = h->seq_log;
  return H;
}

int check_rays(const robast_rays* rays) {
  if (!rays->ox || !rays->oy || !rays->oz || !rays->dx || !rays->dy || !rays->dz)
    return fail(ROBAST_EINVAL, "NULL ray coordinate array");
  return ROBAST_OK;
}

// Wavelengths are traced for scenes whose dispersive lenses sit beside
// shapes other than cones (the kernels carry them in those instances only).
int check_lambda(const robast_scene* s, const robast_rays* rays) {
  if (!rays->lambda) return ROBAST_OK;
  const int shapes = s->precision == 32 ? s->sf.shapes : s->sd.shapes;
  if (shapes & ~kShapesNoCone)
    return fail(ROBAST_EUNSUPPORTED, "per-photon wavelengths are not traced in scenes with hexagonal cones");
  return ROBAST_OK;
}

int check_hits(const robast_hits* hits) {
  if (hits->x && (!hits->y || !hits->z)) return fail(ROBAST_EINVAL, "x given without y, z");
  if (hits->ux && (!hits->uy || !hits->uz)) return fail(ROBAST_EINVAL, "ux given without uy, uz");
  return ROBAST_OK;
}

template <typename T> BatchView<T> batch_view(const robast_batch* b) {
  return BatchView<T>{(const BatchVariant<T>*)b->d_vars, b->d_items, b->d_queue, b->n_items, b->max_events,
                      b->max_params, b->blob_cap, b->blob_cap_bwd, b->shapes, (int)b->block};
}

template <typename T> std::vector<BatchVariant<T>> variant_table(const robast_batch& b, const int64_t* offsets) {
  std::vector<BatchVariant<T>> t(b.scenes.size());
  int64_t goff = 0, poff = 0;
  for (size_t v = 0; v < b.scenes.size(); ++v) {
    const robast_scene* s = b.scenes[v];
    t[v] = BatchVariant<T>{(const SceneView<T>*)s->d_view, offsets[v], (int32_t)goff, (int32_t)poff,
                           (int32_t)s->params.size(), 0};
    goff += s->n_groups;
    poff += (int64_t)s->params.size();
  }
  return t;
}

constexpr int64_t kBinMin = 32768;

void apply_tuning(robast_scene* s) {
  s->cfg.waves_mult = (int)s->tuning.waves_mult;
  s->cfg.block = s->tuning.block ? (int)s->tuning.block : 256;
}

bool block_valid(uint32_t b) { return b == 0 || b == 64 || b == 128 || b == 192 || b == 256; }
bool dirs_valid(uint32_t d) { return d == 0 || d == 1 || d == 4 || d == 16 || d == 64; }
uint32_t bin_dirs(const robast_tuning& t) { return t.bin_dirs ? t.bin_dirs : 1u; }

// Cells per side of the binning grid: about `target` photons per cell over
// G groups x `dirs` direction sectors, within the key range.
int bin_cells(int64_t n, int G, uint32_t target, uint32_t dirs) {
  const double per_cell = (double)std::max<int64_t>(n, 1) / ((double)G * (double)dirs * (double)target);
  const int nc = (int)std::floor(std::sqrt(std::max(1.0, per_cell)));
  const int nc_max = (int)std::floor(std::sqrt((double)kBinsMax / ((double)G * (double)dirs)));
  return std::max(1, std::min({nc, 1024, nc_max}));
}

int tuning_valid(const robast_tuning& t) {
  return t.bin_target >= 1 && t.bin_target <= 65536 && t.waves_mult >= 1 && t.waves_mult <= 64 &&
         block_valid(t.block) && dirs_valid(t.bin_dirs);
}


// The view of the photons a launch reads: the caller's arrays, or their
// binned copy (with the permutation back to the caller's order).
bool same_rays(const robast_rays& a, const robast_rays& b) {
  return a.ox == b.ox && a.oy == b.oy && a.oz == b.oz && a.dx == b.dx && a.dy == b.dy && a.dz == b.dz &&
         a.group == b.group && a.id_base == b.id_base;
}

// The kept binned order is used by any call given the same arrays and n;
// afterwards it stays kept only if `keep` (a backward call passes false).
// With `ext` (a workspace of ext_bytes the caller supplies) the binning uses
// it instead of the scene's own, keeps nothing and allocates nothing.
template <typename T>
int binned_view(robast_scene* s, const robast_rays* rays, int64_t n, hipStream_t st, RaysView<T>& out,
                bool keep, bool* reused = nullptr, void* ext = nullptr, size_t ext_bytes = 0) {
  const RaysView<T> R = rays_view<T>(rays);
  out = R;
  if (reused) *reused = false;
  if (!s->tuning.bin_photons || n < kBinMin || n > (int64_t)UINT32_MAX) return ROBAST_OK;
  if (!ext && s->kept && s->kept_n == n && same_rays(s->kept_rays, *rays)) {
    s->kept = keep;
    if (reused) *reused = true;
    out = binned_rays<T>((const BinRecord<T>*)s->kept_records, rays->group != nullptr, rays->id_base);
    out.lam = R.lam;
    return ROBAST_OK;
  }
  s->kept = false;   // the workspace is about to be overwritten
  const int G = s->n_groups;
  const uint32_t dirs = bin_dirs(s->tuning);
  const int nc = bin_cells(n, G, s->tuning.bin_target, dirs);
  const int64_t bins = (int64_t)G * dirs * nc * nc;
  const BinPlan plan = bin_plan<T>(n, bins);
  if (ext) {
    if (plan.bytes > ext_bytes)
      return fail(ROBAST_EINVAL, "binning " + std::to_string(n) + " photons needs " + std::to_string(plan.bytes) +
                                     " bytes of workspace, more than the " + std::to_string(ext_bytes) +
                                     " bytes of the static workspace (about " +
                                     std::to_string(ext_bytes / (2 * sizeof(BinRecord<T>) + 8)) + " photons)");
    const BinWork<T> W = bin_carve<T>(plan, ext);
    const BinGeom geo{s->bin_z, s->bin_x0, s->bin_y0, (double)nc / s->bin_side, nc, G, 0u, dirs};
    hipError_t e = launch_binning<T>(R, n, geo, BinMulti{nullptr, nullptr, 0}, plan, W, st);
    if (e != hipSuccess) return hip_fail(e, "binning launch");
    out = binned_rays<T>(W.out, rays->group != nullptr, rays->id_base);
    out.lam = R.lam;
    return ROBAST_OK;
  }
  if (plan.bytes > s->work_bytes) {
    if (s->d_work) (void)hipFree(s->d_work);
    s->d_work = nullptr;
    s->work_bytes = 0;
    hipError_t e = hipMalloc(&s->d_work, plan.bytes);
    if (e != hipSuccess) return e == hipErrorOutOfMemory ? fail(ROBAST_ENOMEM, "hipMalloc binning workspace")
                                                         : hip_fail(e, "hipMalloc binning workspace");
    s->work_bytes = plan.bytes;
  }
  const BinWork<T> W = bin_carve<T>(plan, s->d_work);
  const BinGeom geo{s->bin_z, s->bin_x0, s->bin_y0, (double)nc / s->bin_side, nc, G, 0u, dirs};
  hipError_t e = launch_binning<T>(R, n, geo, BinMulti{nullptr, nullptr, 0}, plan, W, st);
  if (e != hipSuccess) return hip_fail(e, "binning launch");
  out = binned_rays<T>(W.out, rays->group != nullptr, rays->id_base);
  out.lam = R.lam;
  if (keep) {
    s->kept = true;
    s->kept_rays = *rays;
    s->kept_n = n;
    s->kept_records = W.out;
  }
  return ROBAST_OK;
}

// Path-record buffer for n photons: records, long-record list, the list of
// four-event records, their two counts.
size_t path_bytes(int64_t n) {
  return align256((size_t)n * kPathSlots * 4) + 2 * align256((size_t)n * 4) + 256;
}

PathView path_view(const robast_scene* s) {
  char* base = (char*)s->d_path;
  const size_t rec = align256((size_t)s->path_cap * kPathSlots * 4);
  const size_t list = align256((size_t)s->path_cap * 4);
  return PathView{(const uint32_t*)base, (uint32_t*)(base + rec), (uint32_t*)(base + rec + 2 * list),
                  (uint32_t*)(base + rec + list)};
}

int ensure_path(robast_scene* s, int64_t n) {
  if (n <= s->path_cap) return ROBAST_OK;
  if (s->d_path) (void)hipFree(s->d_path);
  s->d_path = nullptr;
  s->path_cap = 0;
  hipError_t e = hipMalloc(&s->d_path, path_bytes(n));
  if (e != hipSuccess) return e == hipErrorOutOfMemory ? fail(ROBAST_ENOMEM, "hipMalloc path records")
                                                       : hip_fail(e, "hipMalloc path records");
  s->path_cap = n;
  return ROBAST_OK;
}

template <typename T>
int trace_t(robast_scene* s, const SceneView<T>& V, const robast_rays* rays, int64_t n, const robast_hits* hits,
            bool keep, hipStream_t st) {
  s->path_ok = false;
  RaysView<T> R;
  int rc = binned_view<T>(s, rays, n, st, R, keep);
  if (rc) return rc;
  HitsView<T> H = hits_view<T>(hits);
  if (keep && n <= (int64_t)UINT32_MAX) {
    rc = ensure_path(s, n);
    if (rc) return rc;
    H.path = const_cast<uint32_t*>(path_view(s).rec);
  }
  hipError_t e = launch_trace<T>(V, R, n, H, s->cfg, st);
  if (e != hipSuccess) return hip_fail(e, "trace launch");
  if (H.path) {
    s->path_ok = true;
    s->path_binned = R.perm != nullptr;
    s->path_rays = *rays;
    s->path_n = n;
  }
  return ROBAST_OK;
}

// The trace of robast_trace_static: binning (if the tuning asks for it) in
// the static workspace, no path records, nothing kept.
template <typename T>
int trace_static_t(robast_scene* s, const SceneView<T>& V, const robast_rays* rays, int64_t n,
                   const robast_hits* hits, void* work, hipStream_t st) {
  s->path_ok = false;
  s->kept = false;
  RaysView<T> R;
  int rc = binned_view<T>(s, rays, n, st, R, false, nullptr, work, kStaticScratchBytes);
  if (rc) return rc;
  hipError_t e = launch_trace<T>(V, R, n, hits_view<T>(hits), s->cfg, st);
  if (e != hipSuccess) return hip_fail(e, "trace launch");
  return ROBAST_OK;
}

// The backward call replays the path records of the preceding trace when
// that trace kept its order for the same arrays (and the photons are read
// in that same order); otherwise it traces the photons again.
template <typename T>
int backward_t(robast_scene* s, const SceneView<T>& V, const robast_rays* rays, int64_t n, const AdjView& A,
               hipStream_t st) {
  RaysView<T> R;
  bool reused = false;
  int rc = binned_view<T>(s, rays, n, st, R, false, &reused);
  if (rc) return rc;
  const bool binned = R.perm != nullptr;
  const bool use_path = s->path_ok && s->path_n == n && same_rays(s->path_rays, *rays) &&
                        binned == s->path_binned && (!binned || reused);
  s->path_ok = false;
  const PathView P = use_path ? path_view(s) : PathView{};
  hipError_t e = launch_backward<T>(V, R, n, A, s->cfg, st, use_path ? &P : nullptr);
  if (e != hipSuccess) return hip_fail(e, "backward launch");
  return ROBAST_OK;
}

// The photons a batched launch reads: the caller's arrays or their binned
// copy (kept order reused when given the same arrays).
int batch_binned_view(robast_batch* b, const robast_rays* rays, hipStream_t st, bool keep, RaysView<float>& out,
                      bool* reused = nullptr) {
  out = rays_view<float>(rays);
  if (reused) *reused = false;
  if (!b->bin) return ROBAST_OK;
  const BinPlan plan = bin_plan<float>(b->n_photons, b->bins);
  const BinWork<float> W = bin_carve<float>(plan, b->d_work);
  if (reused) *reused = b->kept && same_rays(b->kept_rays, *rays);
  if (!(b->kept && same_rays(b->kept_rays, *rays))) {
    const BinMulti multi{b->d_offsets, b->d_geo, (int)b->scenes.size()};
    hipError_t e = launch_binning<float>(out, b->n_photons, BinGeom{}, multi, plan, W, st);
    if (e != hipSuccess) return hip_fail(e, "batched binning launch");
  }
  b->kept = keep;
  b->kept_rays = *rays;
  out = binned_rays<float>(W.out, rays->group != nullptr, rays->id_base);
  return ROBAST_OK;
}

void free_batch(robast_batch* b) {
  if (b->d_vars) (void)hipFree(b->d_vars);
  if (b->d_items) (void)hipFree(b->d_items);
  if (b->d_queue) (void)hipFree(b->d_queue);
  if (b->d_coef) (void)hipFree(b->d_coef);
  if (b->d_offsets) (void)hipFree(b->d_offsets);
  if (b->d_geo) (void)hipFree(b->d_geo);
  if (b->d_work) (void)hipFree(b->d_work);
  if (b->d_path) (void)hipFree(b->d_path);
  if (b->d_jobs) (void)hipFree(b->d_jobs);
  if (b->d_poff) (void)hipFree(b->d_poff);
  delete b;
}

}  // namespace

// The boundary gradient over the binned order (a kept order of the same
// arrays is reused and stays kept; else the bundle is binned and kept, and
// path records of an earlier order are dropped): the photons of a wave then
// replay similar paths, as in the trace.
template <typename T>
int boundary_t(robast_scene* s, const SceneView<T>& V, const robast_rays* rays, int64_t n, const double* group_sums,
               const double* group_cot, double band, double* grad, hipStream_t st) {
  RaysView<T> R;
  bool reused = false;
  int rc = binned_view<T>(s, rays, n, st, R, true, &reused);
  if (rc) return rc;
  if (R.perm && !reused) s->path_ok = false;
  hipError_t e = launch_boundary<T>(V, R, n, group_sums, group_cot, s->d_coef, band, grad, (int)s->params.size(),
                                    s->cfg.lds_cap, st);
  if (e != hipSuccess) return hip_fail(e, "boundary gradient launch");
  return ROBAST_OK;
}

extern "C" {

int robast_abi_version(void) { return 2; }

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
  s->cfg.lds_cap = kLdsCap;
  s->cfg.max_blocks = 0;
  s->cfg.block = 256;
  s->tuning = robast_tuning{1u, 128u, 4u, 256u, 1u};
  apply_tuning(s);
  rc = upload(s);
  if (rc) {
    robast_destroy_scene(s);
    return rc;
  }
  *out = s;
  return ROBAST_OK;
}

int robast_set_params(robast_scene* s, const double* params, int64_t n_params) {
  if (!s || (!params && n_params > 0)) return fail(ROBAST_EINVAL, "NULL scene or params");
  if (n_params != (int64_t)s->params.size()) return fail(ROBAST_EMISMATCH, "parameter count differs from build");
  if (!finite_all(params, (int)n_params)) return fail(ROBAST_EINVAL, "non-finite parameter");
  // the new geometry is checked before anything changes: on failure the
  // scene keeps its parameters and tables
  std::vector<double> P(params, params + n_params);
  std::vector<robast_volume_desc> nd = s->desc;
  for (auto& v : nd) apply_params(v, P);
  for (int i = 0; i < (int)nd.size(); ++i) {
    int rc = validate_volume(nd[i], i, n_params);
    if (rc) return rc;
  }
  hipError_t e = hipDeviceSynchronize();
  if (e != hipSuccess) return hip_fail(e, "hipDeviceSynchronize before a rebuild");
  s->params.swap(P);
  s->desc.swap(nd);
  s->kept = false;
  s->path_ok = false;
  return upload(s);
}

int robast_update_params(robast_scene* s, const double* d_params, int32_t* d_status, void* stream) {
  if (!s || !d_params) return fail(ROBAST_EINVAL, "NULL scene or params");
  s->kept = false;
  s->path_ok = false;
  hipStream_t st = (hipStream_t)stream;
  // the kernel writes params only in its gradient-step form (not this one)
  double* P = const_cast<double*>(d_params);
  hipError_t e = s->precision == 32
                     ? launch_update_params<float>((const UpdJob<float>* const*)s->d_jobptr, 1, P, nullptr, d_status, st)
                     : launch_update_params<double>((const UpdJob<double>* const*)s->d_jobptr, 1, P, nullptr, d_status,
                                                    st);
  if (e != hipSuccess) return hip_fail(e, "parameter update launch");
  return ROBAST_OK;
}

int robast_gd_step(robast_scene* s, double* d_params, const double* d_grad, const double* d_lr, int32_t* d_status,
                   void* stream) {
  if (!s || !d_params || !d_grad || !d_lr) return fail(ROBAST_EINVAL, "NULL scene, params, grad or lr");
  s->kept = false;
  s->path_ok = false;
  hipStream_t st = (hipStream_t)stream;
  hipError_t e = s->precision == 32
                     ? launch_update_params<float>((const UpdJob<float>* const*)s->d_jobptr, 1, d_params, nullptr,
                                                   d_status, st, d_grad, d_lr)
                     : launch_update_params<double>((const UpdJob<double>* const*)s->d_jobptr, 1, d_params, nullptr,
                                                    d_status, st, d_grad, d_lr);
  if (e != hipSuccess) return hip_fail(e, "gradient step launch");
  return ROBAST_OK;
}

void robast_destroy_scene(robast_scene* s) {
  if (!s) return;
  if (s->d_blob) (void)hipFree(s->d_blob);
  if (s->d_tilt) (void)hipFree(s->d_tilt);
  if (s->d_coef) (void)hipFree(s->d_coef);
  if (s->d_view) (void)hipFree(s->d_view);
  if (s->d_work) (void)hipFree(s->d_work);
  if (s->d_path) (void)hipFree(s->d_path);
  if (s->d_check) (void)hipFree(s->d_check);
  if (s->d_upd) (void)hipFree(s->d_upd);
  if (s->d_job) (void)hipFree(s->d_job);
  if (s->d_jobptr) (void)hipFree(s->d_jobptr);
  delete s;
}

int robast_trace(robast_scene* s, const robast_rays* rays, int64_t n, const robast_hits* hits, uint32_t flags,
                 void* stream) {
  if (!s || !rays || !hits) return fail(ROBAST_EINVAL, "NULL scene, rays or hits");
  if (flags & ~(uint32_t)ROBAST_TRACE_KEEP_ORDER) return fail(ROBAST_EINVAL, "unknown trace flag");
  if (n < 0) return fail(ROBAST_EINVAL, "n < 0");
  if (n == 0) return ROBAST_OK;
  int rc = check_rays(rays);
  if (!rc) rc = check_lambda(s, rays);
  if (!rc) rc = check_hits(hits);
  if (rc) return rc;
  hipStream_t st = (hipStream_t)stream;
  const bool keep = (flags & ROBAST_TRACE_KEEP_ORDER) != 0;
  if (s->precision == 32) return trace_t<float>(s, s->sf, rays, n, hits, keep, st);
  return trace_t<double>(s, s->sd, rays, n, hits, keep, st);
}

int robast_trace_static(robast_scene* s, const robast_rays* rays, int64_t n, const robast_hits* hits,
                        void* stream) {
  if (!s || !rays || !hits) return fail(ROBAST_EINVAL, "NULL scene, rays or hits");
  if (n < 0) return fail(ROBAST_EINVAL, "n < 0");
  if (n == 0) return ROBAST_OK;
  int rc = check_rays(rays);
  if (!rc) rc = check_lambda(s, rays);
  if (!rc) rc = check_hits(hits);
  if (rc) return rc;
  void* work = nullptr;
  rc = static_scratch(&work);
  if (rc) return rc;
  hipStream_t st = (hipStream_t)stream;
  if (s->precision == 32) return trace_static_t<float>(s, s->sf, rays, n, hits, work, st);
  return trace_static_t<double>(s, s->sd, rays, n, hits, work, st);
}

int robast_figures(robast_scene* s, const double* sums, double* fig, void* stream) {
  if (!s || !sums || !fig) return fail(ROBAST_EINVAL, "NULL scene, sums or figures");
  hipError_t e = launch_figures(sums, fig, s->n_groups, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "figures launch");
  return ROBAST_OK;
}

int robast_arrival_figures(robast_scene* s, const robast_rays* rays, const robast_hits* hits, int64_t n,
                           double* out, void* stream) {
  if (!s || !rays || !hits || !out) return fail(ROBAST_EINVAL, "NULL scene, rays, hits or out");
  if (!hits->fate || !hits->opl) return fail(ROBAST_EINVAL, "hits need fate and opl");
  if (n < 0) return fail(ROBAST_EINVAL, "n < 0");
  hipError_t e = s->precision == 32
                     ? launch_arrival<float>(hits->fate, (const float*)hits->opl, rays->group, n, s->n_groups, out,
                                             (hipStream_t)stream)
                     : launch_arrival<double>(hits->fate, (const double*)hits->opl, rays->group, n, s->n_groups,
                                              out, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "arrival figures launch");
  return ROBAST_OK;
}

int robast_trace_backward(robast_scene* s, const robast_rays* rays, int64_t n, const robast_hits* fwd,
                          const double* group_cot, const double* photon_cot, double* grad, uint32_t flags,
                          void* stream) {
  if (!s || !rays || !grad) return fail(ROBAST_EINVAL, "NULL scene, rays or grad");
  if (flags & ~(uint32_t)ROBAST_BACKWARD_CHECK_SEQ) return fail(ROBAST_EINVAL, "unknown backward flag");
  const bool check = (flags & ROBAST_BACKWARD_CHECK_SEQ) != 0;
  if (group_cot && (!fwd || !fwd->group_sums))
    return fail(ROBAST_EINVAL, "a group cotangent needs the forward group sums (fwd->group_sums)");
  if (check && (!fwd || !fwd->seq_hash))
    return fail(ROBAST_EINVAL, "the sequence check needs the forward hashes (fwd->seq_hash)");
  if (n < 0) return fail(ROBAST_EINVAL, "n < 0");
  if (n == 0) return ROBAST_OK;
  int rc = check_rays(rays);
  if (!rc) rc = check_lambda(s, rays);
  if (rc) return rc;
  if (s->max_events > 64) return fail(ROBAST_EUNSUPPORTED, "backward supports max_events <= 64");
  hipStream_t st = (hipStream_t)stream;
  AdjView A{nullptr, grad, s->d_tilt, (int)s->params.size()};
  if (group_cot) {
    hipError_t e = launch_adj_coef(fwd->group_sums, group_cot, s->d_coef, s->n_groups, st);
    if (e != hipSuccess) return hip_fail(e, "coefficient launch");
    A.coef = s->d_coef;
  }
  A.pcot = photon_cot;
  if (check) {
    // debug mode: every photon is searched again (no path record replay) and
    // its sequence hash compared with the forward one; synchronous
    if (!s->d_check) {
      hipError_t e = hipMalloc(&s->d_check, 256);
      if (e != hipSuccess) return hip_fail(e, "hipMalloc check counter");
    }
    hipError_t e = hipMemsetAsync(s->d_check, 0, sizeof(uint32_t), st);
    if (e != hipSuccess) return hip_fail(e, "hipMemsetAsync check counter");
    A.check_hash = fwd->seq_hash;
    A.mismatch = (uint32_t*)s->d_check;
    s->path_ok = false;
  }
  rc = s->precision == 32 ? backward_t<float>(s, s->sf, rays, n, A, st) : backward_t<double>(s, s->sd, rays, n, A, st);
  if (rc || !check) return rc;
  uint32_t bad = 0;
  hipError_t e = hipStreamSynchronize(st);
  if (e == hipSuccess) e = hipMemcpy(&bad, s->d_check, sizeof(bad), hipMemcpyDeviceToHost);
  if (e != hipSuccess) return hip_fail(e, "sequence check readback");
  if (bad) return fail(ROBAST_EMISMATCH, std::to_string(bad) + " photons' surface sequences differ from the forward pass");
  return ROBAST_OK;
}

int robast_boundary_grad(robast_scene* s, const robast_rays* rays, int64_t n, const double* group_sums,
                         const double* group_cot, double band, double* grad, void* stream) {
  if (!s || !rays || !group_sums || !group_cot || !grad)
    return fail(ROBAST_EINVAL, "NULL scene, rays, group sums, cotangents or grad");
  if (n < 0) return fail(ROBAST_EINVAL, "n < 0");
  if (!(band > 0.0 && band < 1.0)) return fail(ROBAST_EINVAL, "band must lie in (0, 1)");
  int rc = check_rays(rays);
  if (rc) return rc;
  if (rays->lambda) return fail(ROBAST_EUNSUPPORTED, "the boundary gradient takes no per-photon wavelengths");
  if (s->max_events > kBndMaxEvents) return fail(ROBAST_EUNSUPPORTED, "the boundary gradient supports max_events <= 32");
  hipStream_t st = (hipStream_t)stream;
  return s->precision == 32 ? boundary_t<float>(s, s->sf, rays, n, group_sums, group_cot, band, grad, st)
                            : boundary_t<double>(s, s->sd, rays, n, group_sums, group_cot, band, grad, st);
}

int robast_bin_photons(robast_scene* s, const robast_rays* rays, int64_t n, void* stream) {
  if (!s || !rays) return fail(ROBAST_EINVAL, "NULL scene or rays");
  if (n < 0) return fail(ROBAST_EINVAL, "n < 0");
  if (n == 0) return ROBAST_OK;
  int rc = check_rays(rays);
  if (!rc) rc = check_lambda(s, rays);
  if (rc) return rc;
  s->kept = false;
  s->path_ok = false;
  hipStream_t st = (hipStream_t)stream;
  if (s->precision == 32) {
    RaysView<float> R;
    return binned_view<float>(s, rays, n, st, R, true);
  }
  RaysView<double> R;
  return binned_view<double>(s, rays, n, st, R, true);
}

int robast_get_tuning(const robast_scene* s, robast_tuning* out) {
  if (!s || !out) return fail(ROBAST_EINVAL, "NULL scene or tuning");
  *out = s->tuning;
  return ROBAST_OK;
}

int robast_set_tuning(robast_scene* s, const robast_tuning* t) {
  if (!s || !t) return fail(ROBAST_EINVAL, "NULL scene or tuning");
  if (!tuning_valid(*t)) return fail(ROBAST_EINVAL, "tuning field out of range");
  s->tuning = *t;
  apply_tuning(s);
  s->path_ok = false;
  return ROBAST_OK;
}

int robast_autotune(robast_scene* s, const robast_rays* rays, int64_t n, robast_tuning* best, void* stream) {
  if (!s || !rays) return fail(ROBAST_EINVAL, "NULL scene or rays");
  if (n < 1) return fail(ROBAST_EINVAL, "n < 1");
  int rc = check_rays(rays);
  if (!rc) rc = check_lambda(s, rays);
  if (rc) return rc;
  hipStream_t st = (hipStream_t)stream;
  s->kept = false;
  s->path_ok = false;
  double* sums = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t e = hipMalloc(&sums, sizeof(double) * 8 * s->n_groups);
  if (e == hipSuccess) e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  const robast_tuning saved = s->tuning;
  robast_tuning win = saved;
  float win_ms = INFINITY;
  robast_hits hits{};
  hits.group_sums = sums;
  // times one candidate (the first of two runs warms up) and keeps the fastest
  auto time_one = [&](const robast_tuning& t) {
    if (e != hipSuccess || rc) return;
    s->tuning = t;
    apply_tuning(s);
    float ms = 0.0f;
    for (int rep = 0; rep < 2 && e == hipSuccess && !rc; ++rep) {
      e = hipMemsetAsync(sums, 0, sizeof(double) * 8 * s->n_groups, st);
      if (e == hipSuccess) e = hipEventRecord(e0, st);
      if (e == hipSuccess) rc = robast_trace(s, rays, n, &hits, 0, stream);
      if (e == hipSuccess && !rc) e = hipEventRecord(e1, st);
      if (e == hipSuccess && !rc) e = hipEventSynchronize(e1);
      if (e == hipSuccess && !rc) e = hipEventElapsedTime(&ms, e0, e1);
    }
    if (e == hipSuccess && !rc && ms < win_ms) {
      win_ms = ms;
      win = s->tuning;
    }
  };
  for (uint32_t bin = 0; bin < 2; ++bin)
    for (uint32_t target : {32u, 128u, 512u})
      for (uint32_t mult : {1u, 4u, 8u})
        for (uint32_t block : {128u, 256u})
          if (bin || target == 128u) time_one(robast_tuning{bin, target, mult, block, 1u});
  // direction sectors, with the launch shape found so far
  const robast_tuning shape = win;
  for (uint32_t dirs : {4u, 16u})
    for (uint32_t target : {16u, 32u, 128u}) time_one(robast_tuning{1u, target, shape.waves_mult, shape.block, dirs});
  s->tuning = (e == hipSuccess && !rc) ? win : saved;
  apply_tuning(s);
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (sums) (void)hipFree(sums);
  if (rc) return rc;
  if (e != hipSuccess) return hip_fail(e, "autotune");
  if (best) *best = win;
  return ROBAST_OK;
}

// ---- batched design sweeps

int robast_build_batch(robast_scene* const* scenes, int32_t n_scenes, const int64_t* offsets, uint32_t chunk,
                       robast_batch** out) {
  if (!out) return fail(ROBAST_EINVAL, "out is NULL");
  *out = nullptr;
  if (!scenes || !offsets) return fail(ROBAST_EINVAL, "NULL scenes or offsets");
  if (n_scenes < 1) return fail(ROBAST_EINVAL, "n_scenes < 1");
  if (chunk == 0 || chunk > (1u << 30)) return fail(ROBAST_EINVAL, "chunk must be in [1, 2^30]");
  if (offsets[0] != 0) return fail(ROBAST_EINVAL, "offsets[0] != 0");
  for (int v = 0; v < n_scenes; ++v) {
    if (!scenes[v]) return fail(ROBAST_EINVAL, "NULL scene in batch");
    if (offsets[v + 1] < offsets[v]) return fail(ROBAST_EINVAL, "offsets decrease");
    if (scenes[v]->precision != scenes[0]->precision) return fail(ROBAST_EINVAL, "scenes of different precision");
  }
  if (scenes[0]->precision != 32) return fail(ROBAST_EUNSUPPORTED, "batches are built for FP32 scenes");
  std::vector<BatchItem> items;
  for (int v = 0; v < n_scenes; ++v)
    for (int64_t st = offsets[v]; st < offsets[v + 1]; st += chunk)
      items.push_back(BatchItem{st, (int32_t)std::min<int64_t>(chunk, offsets[v + 1] - st), v});
  if (items.size() > (size_t)INT32_MAX - 65536) return fail(ROBAST_EINVAL, "too many work items: raise chunk");
  robast_batch* b = new robast_batch();
  b->precision = scenes[0]->precision;
  b->scenes.assign(scenes, scenes + n_scenes);
  b->n_photons = offsets[n_scenes];
  b->n_items = (int)items.size();
  b->offsets.assign(offsets, offsets + n_scenes + 1);
  b->chunk = chunk;
  b->items_cap = std::max<size_t>(1, items.size());
  size_t max_blob = 0;
  for (robast_scene* s : b->scenes) {
    b->n_groups += s->n_groups;
    b->n_params += (int64_t)s->params.size();
    b->max_events = std::max(b->max_events, s->max_events);
    b->max_params = std::max(b->max_params, (int)s->params.size());
    max_blob = std::max(max_blob, s->blob_bytes);
    for (const auto& v : s->desc) b->shapes |= 1 << v.shape;
  }
  if (b->n_groups > INT32_MAX || b->n_params > INT32_MAX) {
    free_batch(b);
    return fail(ROBAST_EINVAL, "too many groups or parameters");
  }
  // LDS reserved per workgroup for a variant's tables, with room for the
  // tables to grow under parameter updates; a variant that outgrows it is
  // read from global memory instead.
  const size_t lds_cap = (size_t)scenes[0]->cfg.lds_cap;
  if (max_blob <= lds_cap) b->blob_cap = (uint32_t)std::min(lds_cap, ((max_blob * 3 / 2) + 15) & ~(size_t)15);
  // the adjoint also keeps the gradient sums in LDS (up to 16 KiB); within
  // the same budget per workgroup a variant whose tables do not fit what is
  // left is traced from global memory rather than lowering the occupancy of
  // every variant
  {
    const size_t gbytes = batch_grad_lds_bytes(b->max_params);
    const size_t left = gbytes < lds_cap ? (lds_cap - gbytes) & ~(size_t)15 : 0;
    b->blob_cap_bwd = (uint32_t)std::min<size_t>(b->blob_cap, left);
  }
  const size_t vbytes = sizeof(BatchVariant<float>);
  hipError_t e = hipMalloc(&b->d_vars, vbytes * n_scenes);
  if (e == hipSuccess) e = hipMalloc(&b->d_items, sizeof(BatchItem) * std::max<size_t>(1, items.size()));
  if (e == hipSuccess) e = hipMalloc(&b->d_queue, kQueueCounters * sizeof(uint32_t));
  if (e == hipSuccess) e = hipMalloc(&b->d_coef, sizeof(double) * 4 * std::max<int64_t>(1, b->n_groups));
  if (e == hipSuccess && b->n_photons <= (int64_t)UINT32_MAX)
    e = hipMalloc(&b->d_path, (size_t)std::max<int64_t>(1, b->n_photons) * kPathSlots * sizeof(uint32_t));
  if (e != hipSuccess) {
    free_batch(b);
    return fail(ROBAST_ENOMEM, "hipMalloc batch tables");
  }
  {
    auto t = variant_table<float>(*b, offsets);
    e = hipMemcpy(b->d_vars, t.data(), vbytes * n_scenes, hipMemcpyHostToDevice);
  }
  // the variants' update jobs and parameter offsets (for robast_update_params_batch)
  if (e == hipSuccess) {
    std::vector<void*> jobs(n_scenes);
    std::vector<int64_t> poff(n_scenes);
    int64_t acc = 0;
    for (int v = 0; v < n_scenes; ++v) {
      jobs[v] = scenes[v]->d_job;
      poff[v] = acc;
      acc += (int64_t)scenes[v]->params.size();
      for (int u = 0; u < v; ++u) b->repeated = b->repeated || scenes[u] == scenes[v];
    }
    e = hipMalloc(&b->d_jobs, sizeof(void*) * n_scenes);
    if (e == hipSuccess) e = hipMalloc(&b->d_poff, sizeof(int64_t) * n_scenes);
    if (e == hipSuccess) e = hipMemcpy(b->d_jobs, jobs.data(), sizeof(void*) * n_scenes, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(b->d_poff, poff.data(), sizeof(int64_t) * n_scenes, hipMemcpyHostToDevice);
  }
  if (e == hipSuccess && !items.empty())
    e = hipMemcpy(b->d_items, items.data(), sizeof(BatchItem) * items.size(), hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    free_batch(b);
    return hip_fail(e, "hipMemcpy batch tables");
  }
  // per-variant photon binning, sized from the variant photon counts
  if (scenes[0]->tuning.bin_photons && b->n_photons >= kBinMin && b->n_photons <= (int64_t)UINT32_MAX) {
    std::vector<BinGeom> geo(n_scenes);
    int64_t base = 0;
    for (int v = 0; v < n_scenes; ++v) {
      const robast_scene* sv = scenes[v];
      const int64_t cnt = offsets[v + 1] - offsets[v];
      const int G = sv->n_groups;
      const uint32_t dirs = bin_dirs(sv->tuning);
      const int nc = bin_cells(cnt, G, sv->tuning.bin_target, dirs);
      geo[v] = BinGeom{sv->bin_z, sv->bin_x0, sv->bin_y0, (double)nc / sv->bin_side, nc, G, (uint32_t)base, dirs};
      base += (int64_t)G * dirs * nc * nc;
    }
    if (base <= kBinsMax) {
      b->bins = base;
      const BinPlan plan = bin_plan<float>(b->n_photons, b->bins);
      e = hipMalloc(&b->d_offsets, sizeof(int64_t) * (n_scenes + 1));
      if (e == hipSuccess) e = hipMalloc(&b->d_geo, sizeof(BinGeom) * n_scenes);
      if (e == hipSuccess) e = hipMalloc(&b->d_work, plan.bytes);
      if (e == hipSuccess)
        e = hipMemcpy(b->d_offsets, offsets, sizeof(int64_t) * (n_scenes + 1), hipMemcpyHostToDevice);
      if (e == hipSuccess) e = hipMemcpy(b->d_geo, geo.data(), sizeof(BinGeom) * n_scenes, hipMemcpyHostToDevice);
      if (e != hipSuccess) {
        free_batch(b);
        return e == hipErrorOutOfMemory ? fail(ROBAST_ENOMEM, "hipMalloc batch binning workspace")
                                        : hip_fail(e, "batch binning tables");
      }
      b->bin = true;
    }
  }
  *out = b;
  return ROBAST_OK;
}

int robast_trace_batch(robast_batch* b, const robast_rays* rays, const robast_hits* hits, uint32_t flags,
                       void* stream) {
  if (!b || !rays || !hits) return fail(ROBAST_EINVAL, "NULL batch, rays or hits");
  if (flags & ~(uint32_t)ROBAST_TRACE_KEEP_ORDER) return fail(ROBAST_EINVAL, "unknown trace flag");
  if (hits->seq_log) return fail(ROBAST_EINVAL, "seq_log is written by robast_trace only");
  if (b->n_photons == 0) return ROBAST_OK;
  int rc = check_rays(rays);
  if (!rc && rays->lambda) rc = fail(ROBAST_EUNSUPPORTED, "batches trace no per-photon wavelengths");
  if (!rc) rc = check_hits(hits);
  if (rc) return rc;
  const bool keep = (flags & ROBAST_TRACE_KEEP_ORDER) != 0;
  b->path_ok = false;
  RaysView<float> R;
  rc = batch_binned_view(b, rays, (hipStream_t)stream, keep, R);
  if (rc) return rc;
  HitsView<float> H = hits_view<float>(hits);
  if (keep) H.path = b->d_path;
  hipError_t e = launch_trace_batch(batch_view<float>(b), R, H, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "batched trace launch");
  if (H.path) {
    b->path_ok = true;
    b->path_rays = *rays;
  }
  return ROBAST_OK;
}

int robast_figures_batch(robast_batch* b, const double* sums, double* fig, void* stream) {
  if (!b || !sums || !fig) return fail(ROBAST_EINVAL, "NULL batch, sums or figures");
  hipError_t e = launch_figures(sums, fig, (int)b->n_groups, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "figures launch");
  return ROBAST_OK;
}

int robast_trace_backward_batch(robast_batch* b, const robast_rays* rays, const double* sums, const double* cot,
                                double* grad, void* stream) {
  if (!b || !rays || !sums || !cot || !grad) return fail(ROBAST_EINVAL, "NULL batch, rays, sums, cot or grad");
  if (b->n_photons == 0) return ROBAST_OK;
  int rc = check_rays(rays);
  if (!rc && rays->lambda) rc = fail(ROBAST_EUNSUPPORTED, "batches trace no per-photon wavelengths");
  if (rc) return rc;
  if (b->max_events > 32) return fail(ROBAST_EUNSUPPORTED, "batched backward supports max_events <= 32");
  hipStream_t st = (hipStream_t)stream;
  hipError_t e = launch_adj_coef(sums, cot, b->d_coef, (int)b->n_groups, st);
  if (e != hipSuccess) return hip_fail(e, "coefficient launch");
  RaysView<float> R;
  bool reused = false;
  rc = batch_binned_view(b, rays, st, false, R, &reused);
  if (rc) return rc;
  // replay the path records of the preceding forward launch if it kept its
  // order for these arrays (and the photons are read in that order)
  const bool use_path = b->path_ok && same_rays(b->path_rays, *rays) && (!b->bin || reused);
  b->path_ok = false;
  e = launch_backward_batch(batch_view<float>(b), R, b->d_coef, grad, st, use_path ? b->d_path : nullptr);
  if (e != hipSuccess) return hip_fail(e, "batched backward launch");
  return ROBAST_OK;
}

int robast_update_params_batch(robast_batch* b, const double* d_params, int32_t* d_status, void* stream) {
  if (!b || !d_params) return fail(ROBAST_EINVAL, "NULL batch or params");
  if (b->repeated) return fail(ROBAST_EUNSUPPORTED, "a scene appears more than once in the batch");
  for (robast_scene* s : b->scenes) {
    s->kept = false;
    s->path_ok = false;
  }
  b->path_ok = false;
  hipError_t e = launch_update_params<float>((const UpdJob<float>* const*)b->d_jobs, (int)b->scenes.size(),
                                             const_cast<double*>(d_params), b->d_poff, d_status, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "batched parameter update launch");
  return ROBAST_OK;
}

int robast_gd_step_batch(robast_batch* b, double* d_params, const double* d_grad, const double* d_lr,
                         int32_t* d_status, void* stream) {
  if (!b || !d_params || !d_grad || !d_lr) return fail(ROBAST_EINVAL, "NULL batch, params, grad or lr");
  if (b->repeated) return fail(ROBAST_EUNSUPPORTED, "a scene appears more than once in the batch");
  for (robast_scene* s : b->scenes) {
    s->kept = false;
    s->path_ok = false;
  }
  b->path_ok = false;
  hipError_t e = launch_update_params<float>((const UpdJob<float>* const*)b->d_jobs, (int)b->scenes.size(), d_params,
                                             b->d_poff, d_status, (hipStream_t)stream, d_grad, d_lr);
  if (e != hipSuccess) return hip_fail(e, "batched gradient step launch");
  return ROBAST_OK;
}

namespace {
// The batch's work items for another chunk size, into d_items (grown when
// needed).  Called with no launch of the batch in flight.
int set_batch_chunk(robast_batch* b, uint32_t chunk) {
  std::vector<BatchItem> items;
  const int nv = (int)b->scenes.size();
  for (int v = 0; v < nv; ++v)
    for (int64_t st = b->offsets[v]; st < b->offsets[v + 1]; st += chunk)
      items.push_back(BatchItem{st, (int32_t)std::min<int64_t>(chunk, b->offsets[v + 1] - st), v});
  if (items.size() > (size_t)INT32_MAX - 65536) return fail(ROBAST_EINVAL, "too many work items: raise chunk");
  hipError_t e = hipSuccess;
  if (items.size() > b->items_cap) {
    BatchItem* d = nullptr;
    e = hipMalloc(&d, sizeof(BatchItem) * items.size());
    if (e != hipSuccess) return fail(ROBAST_ENOMEM, "hipMalloc batch items");
    (void)hipFree(b->d_items);
    b->d_items = d;
    b->items_cap = items.size();
  }
  if (!items.empty()) e = hipMemcpy(b->d_items, items.data(), sizeof(BatchItem) * items.size(), hipMemcpyHostToDevice);
  if (e != hipSuccess) return hip_fail(e, "hipMemcpy batch items");
  b->n_items = (int)items.size();
  b->chunk = chunk;
  return ROBAST_OK;
}
}  // namespace

int robast_autotune_batch(robast_batch* b, const robast_rays* rays, uint32_t* best_chunk, uint32_t* best_block,
                          void* stream) {
  if (!b || !rays) return fail(ROBAST_EINVAL, "NULL batch or rays");
  if (b->n_photons == 0) return ROBAST_OK;
  int rc = check_rays(rays);
  if (rc) return rc;
  if (rays->lambda) return fail(ROBAST_EUNSUPPORTED, "batched launches take no per-photon wavelengths");
  hipStream_t st = (hipStream_t)stream;
  (void)hipStreamSynchronize(st);
  b->kept = false;
  b->path_ok = false;
  double* sums = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t e = hipMalloc(&sums, sizeof(double) * 8 * std::max<int64_t>(1, b->n_groups));
  if (e == hipSuccess) e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  const uint32_t saved_chunk = b->chunk, saved_block = b->block;
  uint32_t win_chunk = saved_chunk, win_block = saved_block;
  float win_ms = INFINITY;
  robast_hits hits{};
  hits.group_sums = sums;
  for (uint32_t chunk : {2048u, 8192u, 32768u, 131072u})
    for (uint32_t block : {128u, 256u}) {
      if (e != hipSuccess || rc) continue;
      rc = set_batch_chunk(b, chunk);
      b->block = block;
      float ms = 0.0f;
      for (int rep = 0; rep < 2 && e == hipSuccess && !rc; ++rep) {   // first run warms up
        e = hipMemsetAsync(sums, 0, sizeof(double) * 8 * b->n_groups, st);
        if (e == hipSuccess) e = hipEventRecord(e0, st);
        if (e == hipSuccess) rc = robast_trace_batch(b, rays, &hits, 0, stream);
        if (e == hipSuccess && !rc) e = hipEventRecord(e1, st);
        if (e == hipSuccess && !rc) e = hipEventSynchronize(e1);
        if (e == hipSuccess && !rc) e = hipEventElapsedTime(&ms, e0, e1);
      }
      if (e == hipSuccess && !rc && ms < win_ms) {
        win_ms = ms;
        win_chunk = chunk;
        win_block = block;
      }
    }
  if (e == hipSuccess && !rc) {
    rc = set_batch_chunk(b, win_chunk);
    b->block = win_block;
  } else {
    (void)set_batch_chunk(b, saved_chunk);
    b->block = saved_block;
  }
  b->kept = false;
  b->path_ok = false;
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (sums) (void)hipFree(sums);
  if (rc) return rc;
  if (e != hipSuccess) return hip_fail(e, "batch autotune");
  if (best_chunk) *best_chunk = win_chunk;
  if (best_block) *best_block = win_block;
  return ROBAST_OK;
}

int robast_batch_sizes(const robast_batch* b, int64_t* n_photons, int64_t* n_groups, int64_t* n_params) {
  if (!b) return fail(ROBAST_EINVAL, "NULL batch");
  if (n_photons) *n_photons = b->n_photons;
  if (n_groups) *n_groups = b->n_groups;
  if (n_params) *n_params = b->n_params;
  return ROBAST_OK;
}

void robast_destroy_batch(robast_batch* b) {
  if (b) free_batch(b);
}

}  // extern "C"
