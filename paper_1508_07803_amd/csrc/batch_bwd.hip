// Batched adjoint: the reverse sweep of many scene variants in one
// persistent launch.
//
// Each photon is processed exactly as by the single-scene adjoint kernels
// (replayed from the forward launch's path record, or its forward search
// run again with the same draws, then the reverse sweep along the sequence),
// with the variant's photons indexed and numbered from its first photon.
// Gradients are summed per workgroup in LDS (FP64) and added to the
// variant's slice of the concatenated gradient when the
// workgroup moves to another variant.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "adjoint_device.hpp"
#include "batch_device.hpp"
#include "device_trace.hpp"
#include "kernels.hpp"

namespace robast {

constexpr uint32_t kGradLdsMax = 16384;   // LDS bytes for the gradient sums of a workgroup

// Gradient sums of variant v in LDS: `copies` interleaved copies of its
// parameter vector (a power of two, as many as fit in grad_bytes, at most
// 16), `pstride` doubles apart (odd: the copies start in different banks);
// lane l adds to copy l mod copies, so lanes of a wave that hit the same
// surface contend for one address copies times less.
struct GradCopies {
  int copies, pstride;
  __device__ __forceinline__ GradCopies(int n_params, uint32_t grad_bytes) {
    pstride = n_params | 1;
    copies = 1;
    while (copies < 16 && (uint32_t)(2 * copies * pstride) * 8u <= grad_bytes) copies *= 2;
  }
};

// Photon selection of a batched adjoint launch: every photon, searched
// again (kSearchAll); only the photons whose path record the replay leaves
// (searched_again), searched again (kSearchLong; the launch ends at once
// when the forward launch flagged none); every photon whose record holds
// at most kPathSlots - 1 events, replayed from it (kReplay).
constexpr int kSearchAll = 0, kSearchLong = 1, kReplay = 2;

// Records the replay pass leaves to the search pass: too long, or holding
// all kPathSlots events (the replay keeps at most kPathSlots - 1 states in
// registers, which fits without spills).
__device__ __forceinline__ bool searched_again(uint4 w) {
  return w.x == kPathLong || (w.x < kPathLong && w.w != kPathEnd);
}

// Per-variant state (view, tilt table, slices) is re-derived from the
// variant table for every item rather than carried across items, which
// keeps it out of the registers the adjoint itself needs.
// SH: the shape set compiled in (the union over the variants).
template <bool USE_LDS, int MAXE, int MODE, int SH>
__global__ void __launch_bounds__(kBlockB) __attribute__((amdgpu_waves_per_eu(MAXE <= 16 ? 3 : 1, 8)))
k_backward_batch(const BatchVariant<float>* vars, const BatchItem* items, int n_items, uint32_t* queue,
                 uint32_t blob_cap, uint32_t grad_bytes, RaysView<float> R, const double* coef, double* grad,
                 const uint32_t* path) {
  extern __shared__ __align__(16) char lds[];
  __shared__ int s_item;
  if (MODE == kSearchLong && queue[kQLongFlag] == 0u) return;
  double* gacc = reinterpret_cast<double*>(lds + (USE_LDS ? blob_cap : 0u));
  int cur_v = -1;   // variant whose partial gradient sits in gacc (-1: none)
  uint32_t* counter = queue + (MODE == kSearchLong ? (USE_LDS ? kQLongLds : kQLongGlobal)
                                                   : (USE_LDS ? kQBwdLds : kQBwdGlobal));
  while (true) {
    const int item = next_item(counter, &s_item);
    const BatchItem it = item < n_items ? load_uniform(items + item) : BatchItem{0, 0, -1};
    if (it.v != cur_v) {
      if (grad_bytes && cur_v >= 0) {
        const BatchVariant<float> pv = load_uniform(vars + cur_v);
        const GradCopies gc(pv.n_params, grad_bytes);
        for (int i = threadIdx.x; i < pv.n_params; i += blockDim.x) {
          double sum = 0.0;
          for (int c = 0; c < gc.copies; ++c) sum += gacc[c * gc.pstride + i];
          if (sum != 0.0) atomicAdd(grad + pv.poff + i, sum);
        }
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
    const GradCopies gc(bv.n_params, grad_bytes);
    if (it.v != cur_v) {
      if (USE_LDS) stage_variant<float>(S, L, lds);
      if (grad_bytes)
        for (int i = threadIdx.x; i < gc.copies * gc.pstride; i += blockDim.x) gacc[i] = 0.0;
      cur_v = it.v;
      __syncthreads();
    } else if (USE_LDS) {
      stage_variant_view<float>(S, L, lds);   // tables already in LDS: rebuild the view only
    }
    const AdjView A{coef + (int64_t)bv.goff * 4, grad + bv.poff, S.tilt, bv.n_params};
    GradSink gs{grad_bytes ? gacc + (threadIdx.x & (gc.copies - 1)) * gc.pstride : grad + bv.poff};
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
    for (int64_t i = lo + threadIdx.x; i < hi; i += blockDim.x) {
      // path records are indexed by position in the whole bundle
      if (MODE == kReplay) {
        const uint4 w = reinterpret_cast<const uint4*>(path)[off + i];
        if (w.x < kPathLong && w.w == kPathEnd)
          adjoint_photon_path<float, false, kPathSlots - 1, SH>(USE_LDS ? L : S, Rv, i, A, gs, w);
      } else if (MODE == kSearchAll || searched_again(reinterpret_cast<const uint4*>(path)[off + i])) {
        adjoint_photon<float, MAXE, SH>(USE_LDS ? L : S, Rv, i, A, gs);
      }
    }
    // a change of variant overwrites LDS: every wave must be done with it
    __syncthreads();
  }
}

// ------------------------------------------------------------------ launcher
uint32_t batch_grad_lds_bytes(int max_params) {
  const uint32_t one = (uint32_t)(max_params | 1) * 8u;
  return one <= kGradLdsMax ? std::min<uint32_t>(kGradLdsMax, 16u * one) : 0u;
}

template <bool USE_LDS, int MAXE, int MODE, int SH>
static hipError_t backward_batch_k(const BatchView<float>& B, const RaysView<float>& R, const double* coef,
                                   double* grad, int ncu, hipStream_t st, const uint32_t* path) {
  const uint32_t gbytes = batch_grad_lds_bytes(B.max_params);
  const size_t shmem = (USE_LDS ? B.blob_cap_bwd : 0) + gbytes;
  int per_cu = 0;
  hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_backward_batch<USE_LDS, MAXE, MODE, SH>,
                                                              kBlockB, shmem);
  if (e != hipSuccess || per_cu < 1) per_cu = 1;
  const int blocks = std::max(1, std::min(B.n_items, ncu * per_cu));
  hipLaunchKernelGGL((k_backward_batch<USE_LDS, MAXE, MODE, SH>), dim3(blocks), dim3(kBlockB), shmem, st, B.vars,
                     B.items, B.n_items, B.queue, B.blob_cap_bwd, gbytes, R, coef, grad, path);
  return hipGetLastError();
}

template <int MAXE, int MODE, int SH>
static hipError_t backward_batch_e(const BatchView<float>& B, const RaysView<float>& R, const double* coef,
                                   double* grad, int ncu, hipStream_t st, const uint32_t* path) {
  hipError_t e = hipSuccess;
  if (B.blob_cap_bwd > 0) e = backward_batch_k<true, MAXE, MODE, SH>(B, R, coef, grad, ncu, st, path);
  if (e == hipSuccess) e = backward_batch_k<false, MAXE, MODE, SH>(B, R, coef, grad, ncu, st, path);
  return e;
}

template <int MAXE, int SH>
static hipError_t backward_batch_s(const BatchView<float>& B, const RaysView<float>& R, const double* coef,
                                   double* grad, int ncu, hipStream_t st, const uint32_t* path) {
  if (!path) return backward_batch_e<MAXE, kSearchAll, SH>(B, R, coef, grad, ncu, st, nullptr);
  hipError_t e = backward_batch_e<16, kReplay, SH>(B, R, coef, grad, ncu, st, path);
  if (e == hipSuccess) e = backward_batch_e<MAXE, kSearchLong, SH>(B, R, coef, grad, ncu, st, path);
  return e;
}

template <int MAXE>
static hipError_t backward_batch_m(const BatchView<float>& B, const RaysView<float>& R, const double* coef,
                                   double* grad, int ncu, hipStream_t st, const uint32_t* path) {
  if (B.shapes & ~kShapesNoCone) return backward_batch_s<MAXE, kShapesAll>(B, R, coef, grad, ncu, st, path);
  return backward_batch_s<MAXE, kShapesNoCone>(B, R, coef, grad, ncu, st, path);
}

hipError_t launch_backward_batch(const BatchView<float>& B, const RaysView<float>& R, const double* coef,
                                 double* grad, hipStream_t st, const uint32_t* path) {
  int dev = 0, ncu = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
  if (e != hipSuccess) return e;
  if (B.max_events > 32) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_batch_reset, dim3(1), dim3(64), 0, st, B.queue, kQBwdLds, kQLongGlobal - kQBwdLds + 1);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (B.max_events <= 16) return backward_batch_m<16>(B, R, coef, grad, ncu, st, path);
  return backward_batch_m<32>(B, R, coef, grad, ncu, st, path);
}

}  // namespace robast
