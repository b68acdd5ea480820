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

// Stages the scene blob into LDS (when USE_LDS) and returns the view of it.
template <typename T, bool USE_LDS>
__device__ __forceinline__ void stage_adj_scene(const SceneView<T>& S, SceneView<T>& L, char* lds) {
  L = S;
  if (!USE_LDS) return;
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

// Gradient partials of a workgroup are summed in LDS in `copies` (a power of
// two) interleaved copies of the parameter vector, `pstride` doubles apart:
// lane l adds to copy l mod copies, so lanes of a wave that hit the same
// surface (the common case once photons are binned) contend for one address
// copies times less.  copies == 0: partials go straight to global memory.
struct GradLds {
  int copies, pstride;
};

__device__ __forceinline__ GradSink grad_begin(double* gacc, const GradLds& G, const AdjView& A) {
  if (G.copies > 0)
    for (int i = threadIdx.x; i < G.copies * G.pstride; i += blockDim.x) gacc[i] = 0.0;
  __syncthreads();
  return GradSink{G.copies > 0 ? gacc + (threadIdx.x & (G.copies - 1)) * G.pstride : A.grad};
}

__device__ __forceinline__ void grad_end(const double* gacc, const GradLds& G, const AdjView& A) {
  if (G.copies == 0) return;
  __syncthreads();
  for (int i = threadIdx.x; i < A.n_params; i += blockDim.x) {
    double v = 0.0;
    for (int c = 0; c < G.copies; ++c) v += gacc[c * G.pstride + i];
    if (v != 0.0) atomicAdd(A.grad + i, v);
  }
}

// FP32 kernels with up to 32 events are held to 3 waves per SIMD (<= 168
// VGPRs; the unconstrained allocation gives 2): at 16 events this needs no
// spills, at 32 (the concentrator) the extra wave is worth its spills
// (adjoint 99 -> 89 ms on 91 x 1e6 photons).  With `list` the
// kernel takes only the photons at the positions list[0 .. *count) (those
// whose path record was too long); otherwise every photon of the bundle.
// SH (all kernels here): the shape set compiled in, as for the trace.
template <typename T, int MAXE, bool USE_LDS, int SH>
__global__ void __launch_bounds__(kBlockAdj)
__attribute__((amdgpu_waves_per_eu((sizeof(T) == 4 && MAXE <= 32) ? 3 : 1, 8)))
k_backward(const SceneView<T>* Sp, RaysView<T> R, int64_t n, AdjView A, GradLds G, const uint32_t* list,
           const uint32_t* count) {
  extern __shared__ __align__(16) char lds[];
  const SceneView<T> S = *Sp;
  A.tilt = S.tilt;
  SceneView<T> L;
  stage_adj_scene<T, USE_LDS>(S, L, lds);
  double* gacc = reinterpret_cast<double*>(lds + (USE_LDS ? ((S.blob_bytes + 15u) & ~15u) : 0u));
  GradSink gs = grad_begin(gacc, G, A);
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t m = list ? (int64_t)*count : n;
  for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < m; j += stride) {
    const int64_t i = list ? (int64_t)list[j] : j;
    adjoint_photon<T, MAXE, SH>(L, R, i, A, gs);
  }
  grad_end(gacc, G, A);
}

// Appends position i of the lanes where `take` holds to list / *count, one
// atomic per wave.  Reached by every active lane.
__device__ __forceinline__ void wave_append(bool take, uint32_t i, uint32_t* list, uint32_t* count) {
  const uint64_t mask = __ballot(take);
  if (!mask) return;
  const int leader = __ffsll((unsigned long long)mask) - 1;
  uint32_t base = 0;
  if ((int)__lane_id() == leader) base = atomicAdd(count, (uint32_t)__popcll(mask));
  base = __shfl(base, leader);
  const uint32_t below = __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
  if (take) list[base + below] = i;
}

// Adjoint from the forward trace's path records, main pass: photons with at
// most kPathSlots - 1 recorded events are swept here without a search (a
// sweep over three slots fits the registers without spills); those with
// exactly kPathSlots events go to list4 for k_backward_path4, those whose
// record is too long to the list for k_backward.
template <typename T, bool USE_LDS, int SH>
__global__ void __launch_bounds__(kBlockAdj)
__attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 ? 3 : 1, 8)))
k_backward_path(const SceneView<T>* Sp, RaysView<T> R, int64_t n, AdjView A, GradLds G, PathView P) {
  extern __shared__ __align__(16) char lds[];
  const SceneView<T> S = *Sp;
  A.tilt = S.tilt;
  SceneView<T> L;
  stage_adj_scene<T, USE_LDS>(S, L, lds);
  double* gacc = reinterpret_cast<double*>(lds + (USE_LDS ? ((S.blob_bytes + 15u) & ~15u) : 0u));
  GradSink gs = grad_begin(gacc, G, A);
  const uint4* rec = reinterpret_cast<const uint4*>(P.rec);
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    const uint4 w = rec[i];
    const bool full = w.x < kPathLong && w.w != kPathEnd;
    wave_append(w.x == kPathLong, (uint32_t)i, P.list, P.count);
    wave_append(full, (uint32_t)i, P.list4, P.count + 1);
    if (w.x >= kPathLong || full) continue;
    adjoint_photon_path<T, true, kPathSlots - 1, SH>(L, R, i, A, gs, w);
  }
  grad_end(gacc, G, A);
}

// The photons of list4 (records of exactly kPathSlots events), swept from
// their records like the main pass.
template <typename T, bool USE_LDS, int SH>
__global__ void __launch_bounds__(kBlockAdj)
__attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 ? 3 : 1, 8)))
k_backward_path4(const SceneView<T>* Sp, RaysView<T> R, AdjView A, GradLds G, PathView P) {
  extern __shared__ __align__(16) char lds[];
  const SceneView<T> S = *Sp;
  A.tilt = S.tilt;
  SceneView<T> L;
  stage_adj_scene<T, USE_LDS>(S, L, lds);
  double* gacc = reinterpret_cast<double*>(lds + (USE_LDS ? ((S.blob_bytes + 15u) & ~15u) : 0u));
  GradSink gs = grad_begin(gacc, G, A);
  const uint4* rec = reinterpret_cast<const uint4*>(P.rec);
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t m = (int64_t)P.count[1];
  for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < m; j += stride) {
    const int64_t i = (int64_t)P.list4[j];
    adjoint_photon_path<T, true, kPathSlots, SH>(L, R, i, A, gs, rec[i]);
  }
  grad_end(gacc, G, A);
}

__global__ void k_clear_u32(uint32_t* p, int n) {
  if ((int)threadIdx.x < n) p[threadIdx.x] = 0u;
}

hipError_t launch_adj_coef(const double* sums, const double* cot, double* coef, int n_groups, hipStream_t st) {
  hipLaunchKernelGGL(k_adj_coef, dim3((n_groups + 63) / 64), dim3(64), 0, st, sums, cot, coef, n_groups);
  return hipGetLastError();
}

// LDS bytes of a launch: the scene blob (when staged) and the gradient
// copies, as many (up to 16) as fit beside the blob within the LDS cap, at
// least one while the parameter vector is at most 16 KiB.
static size_t grad_layout(size_t blob_lds, int n_params, int lds_cap, GradLds& G) {
  G.pstride = n_params | 1;   // odd: the copies start in different banks
  const size_t one = (size_t)G.pstride * sizeof(double);
  G.copies = 0;
  if ((size_t)n_params * sizeof(double) <= 16384) {
    G.copies = 1;
    while (G.copies < 16 && blob_lds + 2 * G.copies * one <= (size_t)lds_cap) G.copies *= 2;
  }
  return blob_lds + (size_t)G.copies * one;
}

template <typename K>
static hipError_t grid_for(K kernel, size_t shmem, int64_t n, const LaunchCfg& cfg, int& blocks) {
  int dev = 0, ncu = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
  if (e != hipSuccess) return e;
  int per_cu = 0;
  e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, kBlockAdj, shmem);
  if (e != hipSuccess || per_cu < 1) per_cu = 1;
  const int64_t want = (n + kBlockAdj - 1) / kBlockAdj;
  const int64_t cap = (int64_t)ncu * per_cu * (cfg.waves_mult > 0 ? cfg.waves_mult : 1);
  blocks = (int)std::max<int64_t>(1, std::min(want, cap));
  return hipSuccess;
}

template <typename T, int MAXE, bool USE_LDS, int SH>
static hipError_t launch_bwd_s(const SceneView<T>& S, const RaysView<T>& R, int64_t n, const AdjView& A,
                               const LaunchCfg& cfg, hipStream_t st, const PathView* P) {
  GradLds G;
  const size_t shmem = grad_layout(USE_LDS ? ((S.blob_bytes + 15u) & ~15u) : 0u, A.n_params, cfg.lds_cap, G);
  int blocks = 0;
  hipError_t e;
  if (P) {
    hipLaunchKernelGGL(k_clear_u32, dim3(1), dim3(64), 0, st, P->count, 2);
    e = grid_for(k_backward_path<T, USE_LDS, SH>, shmem, n, cfg, blocks);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_backward_path<T, USE_LDS, SH>), dim3(blocks), dim3(kBlockAdj), shmem, st, S.self, R, n, A, G,
                       *P);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    e = grid_for(k_backward_path4<T, USE_LDS, SH>, shmem, n, cfg, blocks);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_backward_path4<T, USE_LDS, SH>), dim3(blocks), dim3(kBlockAdj), shmem, st, S.self, R, A, G,
                       *P);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  e = grid_for(k_backward<T, MAXE, USE_LDS, SH>, shmem, n, cfg, blocks);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_backward<T, MAXE, USE_LDS, SH>), dim3(blocks), dim3(kBlockAdj), shmem, st, S.self, R, n, A, G,
                     P ? P->list : nullptr, P ? P->count : nullptr);
  return hipGetLastError();
}

template <typename T, int MAXE, bool USE_LDS>
static hipError_t launch_bwd_l(const SceneView<T>& S, const RaysView<T>& R, int64_t n, const AdjView& A,
                               const LaunchCfg& cfg, hipStream_t st, const PathView* P) {
  if (R.lam && S.dispersive) return launch_bwd_s<T, MAXE, USE_LDS, kShapesNoCone | kLambda>(S, R, n, A, cfg, st, P);
  if (S.shapes & ~kShapesNoCone) return launch_bwd_s<T, MAXE, USE_LDS, kShapesAll>(S, R, n, A, cfg, st, P);
  return launch_bwd_s<T, MAXE, USE_LDS, kShapesNoCone>(S, R, n, A, cfg, st, P);
}

template <typename T, int MAXE>
static hipError_t launch_bwd(const SceneView<T>& S, const RaysView<T>& R, int64_t n, const AdjView& A,
                             const LaunchCfg& cfg, hipStream_t st, const PathView* P) {
  if (cfg.lds_cap > 0 && S.blob_bytes <= (uint32_t)cfg.lds_cap)
    return launch_bwd_l<T, MAXE, true>(S, R, n, A, cfg, st, P);
  return launch_bwd_l<T, MAXE, false>(S, R, n, A, cfg, st, P);
}

template <typename T>
hipError_t launch_backward(const SceneView<T>& S, const RaysView<T>& R, int64_t n, const AdjView& A,
                           const LaunchCfg& cfg, hipStream_t st, const PathView* P) {
  if (S.max_events <= 16) return launch_bwd<T, 16>(S, R, n, A, cfg, st, P);
  if (S.max_events <= 32) return launch_bwd<T, 32>(S, R, n, A, cfg, st, P);
  return launch_bwd<T, 64>(S, R, n, A, cfg, st, P);
}

template hipError_t launch_backward<float>(const SceneView<float>&, const RaysView<float>&, int64_t,
                                           const AdjView&, const LaunchCfg&, hipStream_t, const PathView*);
template hipError_t launch_backward<double>(const SceneView<double>&, const RaysView<double>&, int64_t,
                                            const AdjView&, const LaunchCfg&, hipStream_t, const PathView*);

}  // namespace robast
