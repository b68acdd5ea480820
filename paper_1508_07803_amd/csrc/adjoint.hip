// Reverse-mode (adjoint) kernels: gradients of focal-plane figures with
// respect to the scene parameters along each photon's fixed surface sequence.
//
// For each photon the forward search is run again with the same draws, so its
// fate and (volume, face, action) sequence equal the forward ones, and the
// sequence is recorded.  FOCUSED photons are then swept in reverse: the state
// entering event e is recomputed by replaying events 0..e-1 of the recorded
// sequence (one exact intersection each, no search), and the cotangents of
// the hit point and outgoing direction are pulled back through the
// interaction (reflection / refraction), the surface normal, the hit point
// x = o + t d and the implicit root g(x(t); theta) = 0 to the parameters:
// radii of curvature, aspheric sag coefficients, Bezier control points and
// panel / facet tilt angles (infinitesimal rotations about the recorded tilt
// axes through the pivot).  Per-photon partials are summed per workgroup in
// LDS in FP64 and added to the global gradient once per workgroup.
#include <hip/hip_runtime.h>

#include "adjoint_device.hpp"
#include "device_trace.hpp"
#include "kernels.hpp"

namespace robast {

constexpr int kBlockAdj = 256;

// per-group coefficients of the objective L = sum_g w_rms RMS_g + w_eff effw_g:
//   dL/dx_p = a_g (x_p - xbar_g), dL/dy_p = a_g (y_p - ybar_g), dL/d|uz_p| = b_g
__global__ void k_adj_coef(const double* sums, const double* cot, double* coef, int n_groups) {
  int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= n_groups) return;
  const double* s = sums + g * 8;
  double nl = s[0], nf = s[1];
  double cx = nf > 0 ? s[2] / nf : 0.0, cy = nf > 0 ? s[3] / nf : 0.0;
  double var = nf > 0 ? (s[4] / nf - cx * cx) + (s[5] / nf - cy * cy) : 0.0;
  double rms = var > 0 ? sqrt(var) : 0.0;
  double a = (nf > 0 && rms > 0) ? cot[2 * g] / (nf * rms) : 0.0;
  double b = nl > 0 ? cot[2 * g + 1] / nl : 0.0;
  coef[4 * g + 0] = a; coef[4 * g + 1] = cx; coef[4 * g + 2] = cy; coef[4 * g + 3] = b;
}

// FP32 kernels with up to 16 events are held to 3 waves per SIMD (<= 168
// VGPRs, no spills; the unconstrained allocation gives 2).
template <typename T, int MAXE, bool USE_LDS>
__global__ void __launch_bounds__(kBlockAdj)
__attribute__((amdgpu_waves_per_eu((sizeof(T) == 4 && MAXE <= 16) ? 3 : 1, 8))) k_backward(SceneView<T> S, RaysView<T> R, int64_t n, AdjView A,
                                                         int grad_in_lds) {
  extern __shared__ __align__(16) char lds[];
  SceneView<T> L;
  L = S;
  if (USE_LDS) {
    const uint4* src = reinterpret_cast<const uint4*>(S.blob);
    uint4* dst = reinterpret_cast<uint4*>(lds);
    for (uint32_t i = threadIdx.x; i < S.blob_bytes / 16u; i += blockDim.x) dst[i] = src[i];
    const char* base = S.blob;
    L.vol = reinterpret_cast<const DVol<T>*>(lds);
    L.always = reinterpret_cast<const uint16_t*>(lds + (reinterpret_cast<const char*>(S.always) - base));
    L.cell_start = reinterpret_cast<const uint32_t*>(lds + (reinterpret_cast<const char*>(S.cell_start) - base));
    L.items = reinterpret_cast<const uint16_t*>(lds + (reinterpret_cast<const char*>(S.items) - base));
  L.groups = reinterpret_cast<const GroupRec<T>*>(lds + (reinterpret_cast<const char*>(S.groups) - base));
  }
  double* gacc = reinterpret_cast<double*>(lds + (USE_LDS ? ((S.blob_bytes + 15u) & ~15u) : 0u));
  if (grad_in_lds)
    for (int i = threadIdx.x; i < A.n_params; i += blockDim.x) gacc[i] = 0.0;
  __syncthreads();
  GradSink gs{grad_in_lds ? gacc : A.grad};

  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    adjoint_photon<T, MAXE>(L, R, i, A, gs);
  }
  if (grad_in_lds) {
    __syncthreads();
    for (int i = threadIdx.x; i < A.n_params; i += blockDim.x)
      if (gacc[i] != 0.0) atomicAdd(A.grad + i, gacc[i]);
  }
}

hipError_t launch_adj_coef(const double* sums, const double* cot, double* coef, int n_groups, hipStream_t st) {
  hipLaunchKernelGGL(k_adj_coef, dim3((n_groups + 63) / 64), dim3(64), 0, st, sums, cot, coef, n_groups);
  return hipGetLastError();
}

template <typename T, int MAXE, bool USE_LDS>
static hipError_t launch_bwd_l(const SceneView<T>& S, const RaysView<T>& R, int64_t n, const AdjView& A,
                               const LaunchCfg& cfg, hipStream_t st) {
  int dev = 0, ncu = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
  if (e != hipSuccess) return e;
  const bool use_lds = USE_LDS;
  size_t gbytes = (size_t)A.n_params * sizeof(double);
  bool grad_lds = gbytes <= 16384;
  size_t shmem = (use_lds ? ((S.blob_bytes + 15u) & ~15u) : 0u) + (grad_lds ? gbytes : 0);
  int per_cu = 0;
  e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_backward<T, MAXE, USE_LDS>, kBlockAdj, shmem);
  if (e != hipSuccess || per_cu < 1) per_cu = 1;
  int64_t want = (n + kBlockAdj - 1) / kBlockAdj;
  int64_t cap = (int64_t)ncu * per_cu * (cfg.waves_mult > 0 ? cfg.waves_mult : 1);
  int blocks = (int)std::max<int64_t>(1, std::min(want, cap));
  hipLaunchKernelGGL((k_backward<T, MAXE, USE_LDS>), dim3(blocks), dim3(kBlockAdj), shmem, st, S, R, n, A,
                     grad_lds ? 1 : 0);
  return hipGetLastError();
}

template <typename T, int MAXE>
static hipError_t launch_bwd(const SceneView<T>& S, const RaysView<T>& R, int64_t n, const AdjView& A,
                             const LaunchCfg& cfg, hipStream_t st) {
  if (cfg.lds_cap > 0 && S.blob_bytes <= (uint32_t)cfg.lds_cap) return launch_bwd_l<T, MAXE, true>(S, R, n, A, cfg, st);
  return launch_bwd_l<T, MAXE, false>(S, R, n, A, cfg, st);
}

template <typename T>
hipError_t launch_backward(const SceneView<T>& S, const RaysView<T>& R, int64_t n, const AdjView& A,
                           const LaunchCfg& cfg, hipStream_t st) {
  if (S.max_events <= 16) return launch_bwd<T, 16>(S, R, n, A, cfg, st);
  if (S.max_events <= 32) return launch_bwd<T, 32>(S, R, n, A, cfg, st);
  return launch_bwd<T, 64>(S, R, n, A, cfg, st);
}

template hipError_t launch_backward<float>(const SceneView<float>&, const RaysView<float>&, int64_t,
                                           const AdjView&, const LaunchCfg&, hipStream_t);
template hipError_t launch_backward<double>(const SceneView<double>&, const RaysView<double>&, int64_t,
                                            const AdjView&, const LaunchCfg&, hipStream_t);

}  // namespace robast
