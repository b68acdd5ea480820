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

constexpr uint32_t kGradLdsMax = 16384;   // gradient sums kept in LDS up to this size

// Per-variant state (view, tilt table, slices) is re-derived from the
// variant table for every item rather than carried across items, which
// keeps it out of the registers the adjoint itself needs.
template <bool USE_LDS, int MAXE>
__global__ void __launch_bounds__(kBlockB) __attribute__((amdgpu_waves_per_eu(MAXE <= 16 ? 3 : 1, 8)))
k_backward_batch(const BatchVariant<float>* vars, const BatchItem* items, int n_items, uint32_t* queue,
                 uint32_t blob_cap, int grad_in_lds, RaysView<float> R, const double* coef, double* grad) {
  extern __shared__ __align__(16) char lds[];
  __shared__ int s_item;
  double* gacc = reinterpret_cast<double*>(lds + (USE_LDS ? blob_cap : 0u));
  int cur_v = -1;   // variant whose partial gradient sits in gacc (-1: none)
  uint32_t* counter = queue + (USE_LDS ? 2 : 3);
  while (true) {
    const int item = next_item(counter, &s_item);
    const BatchItem it = item < n_items ? load_uniform(items + item) : BatchItem{0, 0, -1};
    if (it.v != cur_v) {
      if (grad_in_lds && cur_v >= 0) {
        const BatchVariant<float> pv = load_uniform(vars + cur_v);
        for (int i = threadIdx.x; i < pv.n_params; i += blockDim.x)
          if (gacc[i] != 0.0) atomicAdd(grad + pv.poff + i, gacc[i]);
      }
      __syncthreads();
      cur_v = -1;
    }
    if (item >= n_items) break;
    const BatchVariant<float> bv = load_uniform(vars + it.v);
    const SceneView<float> S = load_uniform(bv.S);
    if (fits_lds(S, blob_cap) != USE_LDS) continue;
    SceneView<float> L;
    if (USE_LDS) lds_view(L, lds);
    if (it.v != cur_v) {
      if (USE_LDS) stage_variant<float>(S, L, lds);
      if (grad_in_lds)
        for (int i = threadIdx.x; i < bv.n_params; i += blockDim.x) gacc[i] = 0.0;
      cur_v = it.v;
      __syncthreads();
    } else if (USE_LDS) {
      stage_variant_view<float>(S, L, lds);   // tables already in LDS: rebuild the view only
    }
    const AdjView A{coef + (int64_t)bv.goff * 4, grad + bv.poff, bv.tilt, bv.n_params};
    GradSink gs{grad_in_lds ? gacc : grad + bv.poff};
    // the variant's photons, indexed and numbered from its first photon;
    // binned photons carry their index in the whole bundle
    const int64_t off = bv.off;
    RaysView<float> Rv = R;
    const int64_t k = off * R.stride, u = off * R.ustride;
    Rv.ox = R.ox + k; Rv.oy = R.oy + k; Rv.oz = R.oz + k;
    Rv.dx = R.dx + k; Rv.dy = R.dy + k; Rv.dz = R.dz + k;
    Rv.group = R.group ? R.group + u : nullptr;
    if (R.perm) {
      Rv.perm = R.perm + u;
      Rv.id_base = R.id_base - (uint64_t)off;
    }
    const int64_t lo = it.start - off, hi = it.start - off + it.count;
    for (int64_t i = lo + threadIdx.x; i < hi; i += blockDim.x)
      adjoint_photon<float, MAXE>(USE_LDS ? L : S, Rv, i, A, gs);
    // a change of variant overwrites LDS: every wave must be done with it
    __syncthreads();
  }
}

// ------------------------------------------------------------------ launcher
template <bool USE_LDS, int MAXE>
static hipError_t backward_batch_k(const BatchView<float>& B, const RaysView<float>& R, const double* coef,
                                   double* grad, int ncu, hipStream_t st) {
  const size_t gbytes = (size_t)B.max_params * sizeof(double);
  const bool grad_lds = gbytes <= kGradLdsMax;
  const size_t shmem = (USE_LDS ? B.blob_cap_bwd : 0) + (grad_lds ? gbytes : 0);
  int per_cu = 0;
  hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_backward_batch<USE_LDS, MAXE>, kBlockB,
                                                              shmem);
  if (e != hipSuccess || per_cu < 1) per_cu = 1;
  const int blocks = std::max(1, std::min(B.n_items, ncu * per_cu));
  hipLaunchKernelGGL((k_backward_batch<USE_LDS, MAXE>), dim3(blocks), dim3(kBlockB), shmem, st, B.vars, B.items,
                     B.n_items, B.queue, B.blob_cap_bwd, grad_lds ? 1 : 0, R, coef, grad);
  return hipGetLastError();
}

template <int MAXE>
static hipError_t backward_batch_e(const BatchView<float>& B, const RaysView<float>& R, const double* coef,
                                   double* grad, int ncu, hipStream_t st) {
  hipError_t e = hipSuccess;
  if (B.blob_cap_bwd > 0) e = backward_batch_k<true, MAXE>(B, R, coef, grad, ncu, st);
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
