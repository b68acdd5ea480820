// Batched adjoint: the reverse sweep of many scene variants in one
// persistent launch.
//
// Each photon is processed exactly as by the single-scene adjoint kernel
// (forward search replayed with the same draws, reverse sweep along the
// recorded sequence), with the variant's photons indexed and numbered from
// its first photon.  Gradients are summed per workgroup in LDS (FP64) and
// added to the variant's slice of the concatenated gradient when the
// workgroup moves to another variant.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "adjoint_device.hpp"
#include "batch_device.hpp"
#include "device_trace.hpp"
#include "kernels.hpp"

namespace robast {

constexpr uint32_t kGradLdsMax = 16384;

template <bool USE_LDS, int MAXE>
__global__ void __launch_bounds__(kBlockB) __attribute__((amdgpu_waves_per_eu(MAXE <= 16 ? 3 : 1, 8)))
k_backward_batch(const BatchVariant<float>* vars, const BatchItem* items, int n_items, uint32_t* queue,
                 uint32_t blob_cap, int grad_in_lds, RaysView<float> R, const double* coef, double* grad) {
  extern __shared__ __align__(16) char lds[];
  __shared__ int s_item;
  SceneView<float> S = {};
  SceneView<float> L;
  lds_view(L, lds);
  double* gacc = reinterpret_cast<double*>(lds + (USE_LDS ? blob_cap : 0u));
  bool mine = false;
  int cur_v = -1, np = 0;
  int64_t off = 0;
  double* gdst = grad;
  AdjView A{coef, grad, nullptr, 0};
  RaysView<float> Rv = R;
  uint32_t* counter = queue + (USE_LDS ? 2 : 3);
  while (true) {
    const int item = next_item(counter, &s_item);
    if (item >= n_items) break;
    const BatchItem it = items[item];
    if (it.v != cur_v) {
      if (grad_in_lds && mine) {
        for (int i = threadIdx.x; i < np; i += blockDim.x)
          if (gacc[i] != 0.0) atomicAdd(gdst + i, gacc[i]);
        __syncthreads();
      }
      const BatchVariant<float> bv = vars[it.v];
      S = *bv.S;
      mine = fits_lds(S, blob_cap) == USE_LDS;
      np = bv.n_params;
      gdst = grad + bv.poff;
      if (mine) {
        if (USE_LDS) stage_variant<float>(S, L, lds);
        if (grad_in_lds)
          for (int i = threadIdx.x; i < np; i += blockDim.x) gacc[i] = 0.0;
      }
      A = AdjView{coef + (int64_t)bv.goff * 4, gdst, bv.tilt, np};
      // the variant's photons, indexed and numbered from its first photon
      off = bv.off;
      Rv = R;
      const int64_t k = off * R.stride, u = off * R.ustride;
      Rv.ox = R.ox + k; Rv.oy = R.oy + k; Rv.oz = R.oz + k;
      Rv.dx = R.dx + k; Rv.dy = R.dy + k; Rv.dz = R.dz + k;
      Rv.group = R.group ? R.group + u : nullptr;
      // binned photons carry their index in the whole bundle: number them
      // from the variant's first photon
      if (R.perm) {
        Rv.perm = R.perm + u;
        Rv.id_base = R.id_base - (uint64_t)off;
      }
      cur_v = it.v;
      __syncthreads();
    }
    if (!mine) continue;
    GradSink gs{grad_in_lds ? gacc : gdst};
    const int64_t lo = it.start - off, hi = it.start - off + it.count;
    for (int64_t i = lo + threadIdx.x; i < hi; i += blockDim.x)
      adjoint_photon<float, MAXE>(USE_LDS ? L : S, Rv, i, A, gs);
    // a change of variant overwrites LDS: every wave must be done with it
    __syncthreads();
  }
  if (grad_in_lds && mine)
    for (int i = threadIdx.x; i < np; i += blockDim.x)
      if (gacc[i] != 0.0) atomicAdd(gdst + i, gacc[i]);
}

// ------------------------------------------------------------------ launcher
template <bool USE_LDS, int MAXE>
static hipError_t backward_batch_k(const BatchView<float>& B, const RaysView<float>& R, const double* coef,
                                   double* grad, int ncu, hipStream_t st) {
  const size_t gbytes = (size_t)B.max_params * sizeof(double);
  const bool grad_lds = gbytes <= kGradLdsMax;
  const size_t shmem = (USE_LDS ? B.blob_cap : 0) + (grad_lds ? gbytes : 0);
  int per_cu = 0;
  hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_backward_batch<USE_LDS, MAXE>, kBlockB,
                                                              shmem);
  if (e != hipSuccess || per_cu < 1) per_cu = 1;
  const int blocks = std::max(1, std::min(B.n_items, ncu * per_cu));
  hipLaunchKernelGGL((k_backward_batch<USE_LDS, MAXE>), dim3(blocks), dim3(kBlockB), shmem, st, B.vars, B.items,
                     B.n_items, B.queue, B.blob_cap, grad_lds ? 1 : 0, R, coef, grad);
  return hipGetLastError();
}

template <int MAXE>
static hipError_t backward_batch_e(const BatchView<float>& B, const RaysView<float>& R, const double* coef,
                                   double* grad, int ncu, hipStream_t st) {
  hipError_t e = hipSuccess;
  if (B.blob_cap > 0) e = backward_batch_k<true, MAXE>(B, R, coef, grad, ncu, st);
  if (e == hipSuccess) e = backward_batch_k<false, MAXE>(B, R, coef, grad, ncu, st);
  return e;
}

hipError_t launch_backward_batch(const BatchView<float>& B, const RaysView<float>& R, const double* coef,
                                 double* grad, hipStream_t st) {
  int dev = 0, ncu = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
  if (e != hipSuccess) return e;
  if (B.max_events > 32) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_batch_reset, dim3(1), dim3(64), 0, st, B.queue, 2, 2);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (B.max_events <= 16) return backward_batch_e<16>(B, R, coef, grad, ncu, st);
  return backward_batch_e<32>(B, R, coef, grad, ncu, st);
}

}  // namespace robast
