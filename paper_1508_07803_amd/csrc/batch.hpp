// Device tables of a batch of scene variants and the batched launchers.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

#include "kernels.hpp"
#include "scene_layout.hpp"

namespace robast {

// One variant of the batch.  The scene view is read through a pointer to the
// scene's own device copy, so parameter updates of the scene (which rewrite
// that copy) are seen by later launches, including graph replays.
template <typename T> struct BatchVariant {
  const SceneView<T>* S;   // device (its tilt table: S->tilt)
  int64_t off;             // first photon of the variant in the concatenated bundle
  int32_t goff;            // first group of the variant in the concatenated sums
  int32_t poff;            // first parameter of the variant in the concatenated gradient
  int32_t n_params;
  int32_t pad;
};

// A work item: `count` photons of variant `v` starting at global index `start`.
struct BatchItem {
  int64_t start;
  int32_t count;
  int32_t v;
};

// Device counters of a batch: work queues of the forward kernels (LDS,
// global), a flag set by the forward launch when some photon's path record
// is too long (kPathLong), and the work queues of the adjoint kernels (LDS,
// global) and of its pass over the long records (LDS, global).  The forward
// launch clears [kQFwdLds, kQLongFlag], the adjoint [kQBwdLds, kQLongGlobal].
constexpr int kQFwdLds = 0, kQFwdGlobal = 1, kQLongFlag = 2;
constexpr int kQBwdLds = 3, kQBwdGlobal = 4, kQLongLds = 5, kQLongGlobal = 6;
constexpr int kQueueCounters = 8;

template <typename T> struct BatchView {
  const BatchVariant<T>* vars;   // device
  const BatchItem* items;        // device, sorted by variant
  uint32_t* queue;               // device, kQueueCounters counters
  int n_items;
  int max_events;                // largest max_events over the variants
  int max_params;                // largest n_params over the variants
  uint32_t blob_cap;             // LDS bytes reserved for a variant's tables (0: read from global memory)
  uint32_t blob_cap_bwd;         // the same for the adjoint, whose LDS also holds the gradient sums
  int shapes;                    // bit 1 << shape of every shape in any variant
  int block;                     // threads per workgroup of the forward launch (64..256)
};

// Batched launches are built for FP32 scenes (the sweep precision).
hipError_t launch_trace_batch(const BatchView<float>& B, const RaysView<float>& R, const HitsView<float>& H,
                              hipStream_t st);
// With `path` (the forward launch's path records, non-null) the sequences
// are replayed from the records; photons whose record is too long are
// found again by a search.
// LDS bytes the batched adjoint keeps for gradient sums (0: they go
// straight to global memory), from the largest parameter count.
uint32_t batch_grad_lds_bytes(int max_params);
hipError_t launch_backward_batch(const BatchView<float>& B, const RaysView<float>& R, const double* coef,
                                 double* grad, hipStream_t st, const uint32_t* path = nullptr);

}  // namespace robast
