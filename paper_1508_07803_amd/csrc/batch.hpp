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
  const SceneView<T>* S;   // device
  const DTilt* tilt;       // device, n_vol entries
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

// Work counters: forward (LDS kernel, global kernel), adjoint (LDS, global).
constexpr int kQueueCounters = 4;

template <typename T> struct BatchView {
  const BatchVariant<T>* vars;   // device
  const BatchItem* items;        // device, sorted by variant
  uint32_t* queue;               // device, kQueueCounters counters
  int n_items;
  int max_events;                // largest max_events over the variants
  int max_params;                // largest n_params over the variants
  uint32_t blob_cap;             // LDS bytes reserved for a variant's tables (0: read from global memory)
  uint32_t blob_cap_bwd;         // the same for the adjoint, whose LDS also holds the gradient sums
};

// Batched launches are built for FP32 scenes (the sweep precision).
hipError_t launch_trace_batch(const BatchView<float>& B, const RaysView<float>& R, const HitsView<float>& H,
                              hipStream_t st);
hipError_t launch_backward_batch(const BatchView<float>& B, const RaysView<float>& R, const double* coef,
                                 double* grad, hipStream_t st);

}  // namespace robast
