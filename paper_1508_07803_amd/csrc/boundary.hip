// Boundary (fate-flip) gradient kernel: edge sampling of the collection
// efficiency's discontinuities (see boundary_device.hpp).  Each lane takes
// one photon at a time over a grid-stride loop: its path is traced again
// with the same draws, every event near an edge of its face is moved across
// the edge and traced on, and where the fate differs a reverse sweep from
// that event adds the edge's flux to the gradient (FP64 atomics; such
// events are a small fraction of all).
#include <hip/hip_runtime.h>

#include <algorithm>

#include "boundary.hpp"
#include "boundary_device.hpp"

namespace robast {

constexpr int kBlockBnd = 256;

// per-group weights c_g / (N_g band) from the forward group sums
__global__ void k_bnd_coef(const double* sums, const double* cot, double* w, int n_groups, double band) {
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= n_groups) return;
  const double nl = sums[8 * g];
  w[g] = nl > 0.0 ? cot[g] / (nl * band) : 0.0;
}

// The FP32 kernel is held to 3 waves per SIMD (<= 168 VGPRs, the rest
// spilled): the unconstrained allocation takes 256 registers and runs one
// wave per SIMD, which leaves the latency of its searches and replays
// exposed (measured twice as slow on the concentrator; 2 and 4 waves were
// slower than 3).  The FP64 kernel keeps the compiler's allocation.
template <typename T, bool USE_LDS>
__global__ void __launch_bounds__(kBlockBnd) __attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 ? 3 : 1, 8))) k_boundary(const SceneView<T>* Sp, RaysView<T> R, int64_t n, BndView B) {
  extern __shared__ __align__(16) char lds[];
  const SceneView<T> S = *Sp;
  B.tilt = S.tilt;
  SceneView<T> L = S;
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
  __syncthreads();
  GradSink gs{B.grad};
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
    boundary_photon<T, kBndMaxEvents, kShapesAll>(L, R, i, B, gs);
}

template <typename T>
hipError_t launch_boundary(const SceneView<T>& S, const RaysView<T>& R, int64_t n, const double* sums,
                           const double* cot, double* w, double band, double* grad, int n_params, int lds_cap,
                           hipStream_t st) {
  hipLaunchKernelGGL(k_bnd_coef, dim3((S.n_groups + 63) / 64), dim3(64), 0, st, sums, cot, w, S.n_groups, band);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || n == 0) return e;
  int dev = 0, ncu = 0;
  e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
  if (e != hipSuccess) return e;
  BndView B{w, band, kBndPush, nullptr, grad, n_params};
  const bool use_lds = lds_cap > 0 && S.blob_bytes <= (uint32_t)lds_cap;
  const size_t shmem = use_lds ? ((S.blob_bytes + 15u) & ~15u) : 0u;
  int per_cu = 0;
  if (use_lds)
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_boundary<T, true>, kBlockBnd, shmem);
  else
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_boundary<T, false>, kBlockBnd, shmem);
  if (e != hipSuccess || per_cu < 1) per_cu = 1;
  const int blocks = (int)std::max<int64_t>(1, std::min<int64_t>((n + kBlockBnd - 1) / kBlockBnd, (int64_t)ncu * per_cu * 4));
  if (use_lds)
    hipLaunchKernelGGL((k_boundary<T, true>), dim3(blocks), dim3(kBlockBnd), shmem, st, S.self, R, n, B);
  else
    hipLaunchKernelGGL((k_boundary<T, false>), dim3(blocks), dim3(kBlockBnd), shmem, st, S.self, R, n, B);
  return hipGetLastError();
}

template hipError_t launch_boundary<float>(const SceneView<float>&, const RaysView<float>&, int64_t, const double*,
                                           const double*, double*, double, double*, int, int, hipStream_t);
template hipError_t launch_boundary<double>(const SceneView<double>&, const RaysView<double>&, int64_t, const double*,
                                            const double*, double*, double, double*, int, int, hipStream_t);

}  // namespace robast
