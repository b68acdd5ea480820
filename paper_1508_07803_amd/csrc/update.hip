// Parameter updates of compiled scenes on the device (see update.hpp).
//
// One workgroup per scene.  It copies the live slot's tables to the other
// slot, rebuilds there every volume record from the new parameters (the
// frame of a tilted body, a sphere's curvature, an asphere's sag
// coefficients, a cone profile's control points; then the surface's local
// and world bounds, as the host scene compiler forms them) and each
// candidate group's z-slab, checks the new geometry, and only then points
// the scene's view at that slot.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "../../include/robast.h"
#include "kernels.hpp"
#include "scene_layout.hpp"
#include "update.hpp"

namespace robast {

constexpr int kUpdBlock = 256;
constexpr int kAsphereSamples = 4096;   // sag samples per asphere for its z-range (as the host compiler)

__device__ __forceinline__ void rot_axis(const double e[3], double ang, double R[9]) {
  const double c = cos(ang), s = sin(ang), C = 1.0 - c;
  const double K[9] = {0.0, -e[2], e[1], e[2], 0.0, -e[0], -e[1], e[0], 0.0};
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) R[3 * i + j] = (i == j ? c : 0.0) + s * K[3 * i + j] + C * e[i] * e[j];
}

__device__ __forceinline__ void mat3(const double* A, const double* B, double* C) {
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) C[3 * i + j] = A[3 * i] * B[j] + A[3 * i + 1] * B[3 + j] + A[3 * i + 2] * B[6 + j];
}

// x = c + Q^T xl (the frames are orthonormal)
__device__ __forceinline__ void to_world(const double* Q, const double* c, const double* xl, double* x) {
#pragma unroll
  for (int i = 0; i < 3; ++i) x[i] = c[i] + Q[i] * xl[0] + Q[3 + i] * xl[1] + Q[6 + i] * xl[2];
}

template <typename T> __device__ __forceinline__ T round_down(double x) {
  T f = (T)x;
  return (double)f > x ? nextafter(f, -__builtin_huge_valf()) : f;
}
template <typename T> __device__ __forceinline__ T round_up(double x) {
  T f = (T)x;
  return (double)f < x ? nextafter(f, __builtin_huge_valf()) : f;
}

__device__ __forceinline__ double sag_sphere(double c, double r) {
  return c * r * r / (1.0 + sqrt(1.0 - c * c * r * r));
}

template <typename T>
__global__ void __launch_bounds__(kUpdBlock) k_update_params(const UpdJob<T>* const* jobs, double* params,
                                                             const int64_t* poff, int32_t* status,
                                                             const double* grad, const double* lr) {
  const UpdJob<T>& J = *jobs[blockIdx.x];
  const int64_t po = poff ? poff[blockIdx.x] : 0;
  const double* P = params + po;
  if (grad) {
    // gradient-descent step: the candidate parameters go to the job's
    // scratch; params takes them only if the update is applied
    for (int i = threadIdx.x; i < J.n_params; i += blockDim.x) J.pn[i] = P[i] - lr[po + i] * grad[po + i];
    __syncthreads();
    P = J.pn;
  }
  __shared__ int s_bad;
  __shared__ const char* s_src;
  if (threadIdx.x == 0) {
    s_bad = 0;
    s_src = J.view->blob;
  }
  __syncthreads();
  const char* src = s_src;
  const int live = src == J.slot[0] ? 0 : 1;
  char* dst = J.slot[1 - live];
  DTilt* tdst = J.tilt[1 - live];
  // the grid tables are unchanged: copy the whole live slot first
  for (uint32_t i = threadIdx.x; i < J.blob_bytes / 16u; i += blockDim.x)
    reinterpret_cast<uint4*>(dst)[i] = reinterpret_cast<const uint4*>(src)[i];
  __syncthreads();
  DVol<T>* recs = reinterpret_cast<DVol<T>*>(dst);
  for (int v = threadIdx.x; v < J.n_vol; v += blockDim.x) {
    const UpdVol& U = J.vols[v];
    DVol<T> r = recs[v];
    bool ok = true;
    // frame
    double Q[9], c[3];
#pragma unroll
    for (int i = 0; i < 9; ++i) Q[i] = U.Q[i];
#pragma unroll
    for (int i = 0; i < 3; ++i) c[i] = U.c[i];
    DTilt tl = {};
    if (U.tparam >= 0) {
      const double a = P[U.tparam], b = P[U.tparam + 1];
      ok = ok && isfinite(a) && isfinite(b);
      double Ra[9], Rb[9], R[9], Rt[9];
      rot_axis(U.e1, a, Ra);
      rot_axis(U.e2, b, Rb);
      mat3(Rb, Ra, R);
#pragma unroll
      for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) Rt[3 * i + j] = R[3 * j + i];
      mat3(U.Q0, Rt, Q);
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        const double s = R[3 * i] * (U.pivot[0] - U.c0[0]) + R[3 * i + 1] * (U.pivot[1] - U.c0[1]) +
                         R[3 * i + 2] * (U.pivot[2] - U.c0[2]);
        c[i] = U.pivot[i] - s;
        tl.pivot[i] = U.pivot[i];
        tl.a1[i] = Rb[3 * i] * U.e1[0] + Rb[3 * i + 1] * U.e1[1] + Rb[3 * i + 2] * U.e1[2];
        tl.a2[i] = U.e2[i];
      }
    }
    // shape and local bounds; dsag: largest move of the surface along its
    // local z (sag surfaces) or across the axis (cone walls) since the build
    double lo[3] = {U.lb_lo[0], U.lb_lo[1], U.lb_lo[2]}, hi[3] = {U.lb_hi[0], U.lb_hi[1], U.lb_hi[2]};
    double slope = (double)r.slope, dsag = 0.0, dlat = 0.0;
    if (U.sparam >= 0 && U.shape == SPHERE) {
      const double R = P[U.sparam], cv = 1.0 / R;
      ok = ok && isfinite(R) && R != 0.0 && fabs(cv) * U.rmax < 1.0;
      if (ok) {
        const double z0 = sag_sphere(cv, U.rmin), z1 = sag_sphere(cv, U.rmax);
        lo[2] = fmin(z0, z1); hi[2] = fmax(z0, z1);
        slope = fabs(cv) * U.rmax / sqrt(1.0 - cv * cv * U.rmax * U.rmax);
        dsag = fabs(z1 - sag_sphere(U.p[0], U.rmax));
        r.p[0] = (T)cv;
      }
    } else if (U.sparam >= 0 && U.shape == ASPHERE) {
      double b[8];
      for (int i = 0; i < 8; ++i) {
        b[i] = P[U.sparam + i];
        ok = ok && isfinite(b[i]);
      }
      if (ok) {
        const double rn2 = U.p[0] * U.p[0], ua = U.rmin * U.rmin / rn2, ub = U.rmax * U.rmax / rn2;
        double zmin = 1e300, zmax = -1e300, smax = 0.0, dmax = 0.0;
        for (int k = 0; k <= kAsphereSamples; ++k) {
          const double u = ua + (ub - ua) * k / kAsphereSamples;
          double s = b[7], ds = 8.0 * b[7];
          for (int i = 6; i >= 0; --i) { s = s * u + b[i]; ds = ds * u + (i + 1) * b[i]; }
          const double z = s * u;
          zmin = fmin(zmin, z); zmax = fmax(zmax, z);
          dmax = fmax(dmax, fabs(ds));
          smax = fmax(smax, fabs(ds) * 2.0 * sqrt(u * rn2) / rn2);
        }
        const double pad = dmax * (ub - ua) / kAsphereSamples;
        lo[2] = zmin - pad; hi[2] = zmax + pad;
        slope = smax * 1.01 + 1e-6;
        double up = 1.0;
        for (int i = 0; i < 8; ++i) {
          up *= ub;
          dsag += fabs(b[i] - U.p[1 + i]) * up;
          r.p[1 + i] = (T)b[i];
        }
      }
    } else if (U.sparam >= 0 && U.shape == HEXCONE) {
      double q[8];
      for (int i = 0; i < 8; ++i) q[i] = U.p[i];
      for (int i = 0; i < 4; ++i) {
        q[2 + i] = P[U.sparam + i];
        ok = ok && isfinite(q[2 + i]);
      }
      ok = ok && q[2] > 0.0 && q[4] > 0.0;
      if (ok) {
        double rm = 0.0, zl = 1e300, zh = -1e300;
        for (int k = 0; k < 4; ++k) {
          rm = fmax(rm, q[2 * k]);
          zl = fmin(zl, q[2 * k + 1]); zh = fmax(zh, q[2 * k + 1]);
        }
        const double Rr = rm * 2.0 / sqrt(3.0);
        lo[0] = lo[1] = -Rr; hi[0] = hi[1] = Rr;
        lo[2] = zl; hi[2] = zh;
        dlat = fmax(fabs(q[2] - U.p[2]), fabs(q[4] - U.p[4])) * 2.0 / sqrt(3.0);
        dsag = fmax(fabs(q[3] - U.p[3]), fabs(q[5] - U.p[5]));
        for (int i = 2; i < 6; ++i) r.p[i] = (T)q[i];
      }
    }
    if (!ok) {
      atomicMax(&s_bad, 2);
      continue;
    }
    // record: frame, bounds padded as the host compiler pads them
    double ext = 0.0;
    for (int k = 0; k < 3; ++k) ext = fmax(ext, hi[k] - lo[k]);
    const double pad = 1e-5 * (ext + J.l_ref);
#pragma unroll
    for (int i = 0; i < 9; ++i) r.Q[i] = (T)Q[i];
#pragma unroll
    for (int i = 0; i < 3; ++i) r.c[i] = (T)c[i];
#pragma unroll
    for (int k = 0; k < 3; ++k) { r.lo[k] = (T)(lo[k] - pad); r.hi[k] = (T)(hi[k] + pad); }
    r.slope = (T)slope;
    double mn[3] = {1e300, 1e300, 1e300}, mx[3] = {-1e300, -1e300, -1e300};
    double gz0 = 1e300, gz1 = -1e300, disp = 0.0;
    const UpdGroup* G = U.group >= 0 ? J.groups + U.group : nullptr;
    for (int m = 0; m < 8; ++m) {
      const double xl[3] = {(m & 1) ? hi[0] : lo[0], (m & 2) ? hi[1] : lo[1], (m & 4) ? hi[2] : lo[2]};
      double w[3];
      to_world(Q, c, xl, w);
#pragma unroll
      for (int i = 0; i < 3; ++i) { mn[i] = fmin(mn[i], w[i]); mx[i] = fmax(mx[i], w[i]); }
      if (G) {
        const double rr[3] = {w[0] - G->c[0], w[1] - G->c[1], w[2] - G->c[2]};
        const double gz = G->Q[6] * rr[0] + G->Q[7] * rr[1] + G->Q[8] * rr[2];
        gz0 = fmin(gz0, gz); gz1 = fmax(gz1, gz);
        // rigid displacement of this corner point since the build, across the group
        double wb[3];
        to_world(U.Q, U.c, xl, wb);
        const double dd[3] = {w[0] - wb[0], w[1] - wb[1], w[2] - wb[2]};
        const double gx = G->Q[0] * dd[0] + G->Q[1] * dd[1] + G->Q[2] * dd[2];
        const double gy = G->Q[3] * dd[0] + G->Q[4] * dd[1] + G->Q[5] * dd[2];
        disp = fmax(disp, sqrt(gx * gx + gy * gy));
      }
    }
    const double wpad = pad + 1e-6 * (fabs(c[0]) + fabs(c[1]) + fabs(c[2]));
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      r.bmin[i] = round_down<T>(mn[i] - wpad);
      r.bmax[i] = round_up<T>(mx[i] + wpad);
    }
    if (G) {
      // a move along the local z axis shows across the group as much as that
      // axis leans in the group frame
      const double lx = G->Q[0] * Q[6] + G->Q[1] * Q[7] + G->Q[2] * Q[8];
      const double ly = G->Q[3] * Q[6] + G->Q[4] * Q[7] + G->Q[5] * Q[8];
      disp += dsag * sqrt(lx * lx + ly * ly) + dlat;
      if (!(disp <= U.gpad)) atomicMax(&s_bad, 1);
      J.zr[2 * v] = gz0;
      J.zr[2 * v + 1] = gz1;
    }
    recs[v] = r;
    tdst[v] = tl;
  }
  __syncthreads();
  if (s_bad) {
    if (threadIdx.x == 0 && status) status[blockIdx.x] = s_bad == 2 ? ROBAST_EINVAL : ROBAST_EUNSUPPORTED;
    return;
  }
  // group slabs from their members' new z ranges
  const SceneView<T> cur = *J.view;
  GroupRec<T>* grecs = reinterpret_cast<GroupRec<T>*>(dst + (reinterpret_cast<const char*>(cur.groups) - src));
  for (int g = threadIdx.x; g < J.n_grp; g += blockDim.x) {
    const UpdGroup& G = J.groups[g];
    double z0 = 1e300, z1 = -1e300;
    for (int k = 0; k < G.count; ++k) {
      const int v = J.members[G.first + k];
      z0 = fmin(z0, J.zr[2 * v]);
      z1 = fmax(z1, J.zr[2 * v + 1]);
    }
    grecs[g].zmin = round_down<T>(z0 - G.zpad);
    grecs[g].zmax = round_up<T>(z1 + G.zpad);
  }
  if (grad)
    for (int i = threadIdx.x; i < J.n_params; i += blockDim.x) params[po + i] = J.pn[i];
  __syncthreads();
  if (threadIdx.x == 0) {
    SceneView<T> nv = cur;
    const ptrdiff_t shift = dst - src;
    nv.blob = cur.blob + shift;
    nv.vol = reinterpret_cast<const DVol<T>*>(reinterpret_cast<const char*>(cur.vol) + shift);
    nv.always = reinterpret_cast<const uint16_t*>(reinterpret_cast<const char*>(cur.always) + shift);
    nv.cell_start = reinterpret_cast<const uint32_t*>(reinterpret_cast<const char*>(cur.cell_start) + shift);
    nv.items = reinterpret_cast<const uint16_t*>(reinterpret_cast<const char*>(cur.items) + shift);
    nv.groups = reinterpret_cast<const GroupRec<T>*>(reinterpret_cast<const char*>(cur.groups) + shift);
    nv.tilt = tdst;
    *J.view = nv;
    if (status) status[blockIdx.x] = ROBAST_OK;
  }
}

template <typename T>
hipError_t launch_update_params(const UpdJob<T>* const* jobs, int n_jobs, double* params, const int64_t* poff,
                                int32_t* status, hipStream_t st, const double* grad, const double* lr) {
  if (n_jobs < 1) return hipSuccess;
  hipLaunchKernelGGL(k_update_params<T>, dim3(n_jobs), dim3(kUpdBlock), 0, st, jobs, params, poff, status, grad, lr);
  return hipGetLastError();
}

template hipError_t launch_update_params<float>(const UpdJob<float>* const*, int, double*, const int64_t*, int32_t*,
                                                hipStream_t, const double*, const double*);
template hipError_t launch_update_params<double>(const UpdJob<double>* const*, int, double*, const int64_t*,
                                                 int32_t*, hipStream_t, const double*, const double*);

}  // namespace robast
