// Device helpers shared by the batched forward and adjoint kernels.
//
// Work items (variant, first photon, count) are sorted by variant and pulled
// by persistent workgroups from a device-side counter.  Two kernels split
// the items of one call: the LDS kernel takes the items of variants whose
// tables fit the LDS reservation and stages those tables once per change of
// variant; the global kernel takes the rest (normally none: a variant only
// outgrows the reservation if a parameter update enlarges its tables after
// the batch was built) and reads the tables from global memory.  Both walk
// the whole list, so each item is traced exactly once whichever kernel
// takes it.
#pragma once
#include <hip/hip_runtime.h>

#include "batch.hpp"
#include "scene_layout.hpp"

namespace robast {

constexpr int kBlockB = 256;

// Clears the counters [first, first + count); a kernel rather than a memset
// so that a captured graph replays it like any other node.
__global__ void k_batch_reset(uint32_t* q, int first, int count);

// Next work item of the workgroup, uniform across it (kept in scalar
// registers, together with everything loaded through it).
__device__ __forceinline__ int next_item(uint32_t* counter, int* s_item) {
  if (threadIdx.x == 0) *s_item = (int)atomicAdd(counter, 1u);
  __syncthreads();
  const int item = __builtin_amdgcn_readfirstlane(*s_item);
  __syncthreads();
  return item;
}

// Loads a workgroup-uniform record into scalar registers.  The tables are
// read through pointers the compiler cannot prove unaliased by the kernel's
// stores, so it would keep them in vector registers; taking every word
// through readfirstlane marks them uniform.
template <typename T> __device__ __forceinline__ T load_uniform(const T* p) {
  static_assert(sizeof(T) % 4 == 0, "records of whole words");
  T out;
  const uint32_t* src = reinterpret_cast<const uint32_t*>(p);
  uint32_t* dst = reinterpret_cast<uint32_t*>(&out);
#pragma unroll
  for (int k = 0; k < (int)(sizeof(T) / 4); ++k) dst[k] = __builtin_amdgcn_readfirstlane(src[k]);
  return out;
}

template <typename T> __device__ __forceinline__ bool fits_lds(const SceneView<T>& S, uint32_t blob_cap) {
  return blob_cap > 0 && S.blob_bytes <= blob_cap;
}

// A view whose table pointers all point into LDS (so that the search
// addresses them as LDS from the start).
template <typename T> __device__ __forceinline__ void lds_view(SceneView<T>& L, char* lds) {
  L = SceneView<T>{};
  L.vol = reinterpret_cast<const DVol<T>*>(lds);
  L.always = reinterpret_cast<const uint16_t*>(lds);
  L.cell_start = reinterpret_cast<const uint32_t*>(lds);
  L.items = reinterpret_cast<const uint16_t*>(lds);
  L.groups = reinterpret_cast<const GroupRec<T>*>(lds);
}

// The view of a variant's tables held in LDS: the pointers are rebuilt from
// the LDS array.
template <typename T>
__device__ __forceinline__ void stage_variant_view(const SceneView<T>& S, SceneView<T>& L, char* lds) {
  const char* base = S.blob;
  L = S;
  L.vol = reinterpret_cast<const DVol<T>*>(lds);
  L.always = reinterpret_cast<const uint16_t*>(lds + (reinterpret_cast<const char*>(S.always) - base));
  L.cell_start = reinterpret_cast<const uint32_t*>(lds + (reinterpret_cast<const char*>(S.cell_start) - base));
  L.items = reinterpret_cast<const uint16_t*>(lds + (reinterpret_cast<const char*>(S.items) - base));
  L.groups = reinterpret_cast<const GroupRec<T>*>(lds + (reinterpret_cast<const char*>(S.groups) - base));
}

// Copies the variant's tables into LDS and builds their view.  Reached by
// the whole workgroup; the caller synchronises before the tables are read.
template <typename T>
__device__ __forceinline__ void stage_variant(const SceneView<T>& S, SceneView<T>& L, char* lds) {
  const uint4* src = reinterpret_cast<const uint4*>(S.blob);
  uint4* dst = reinterpret_cast<uint4*>(lds);
  for (uint32_t i = threadIdx.x; i < S.blob_bytes / 16u; i += blockDim.x) dst[i] = src[i];
  stage_variant_view<T>(S, L, lds);
}

}  // namespace robast
