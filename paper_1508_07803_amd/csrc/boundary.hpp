// Launcher of the boundary (fate-flip) gradient kernel.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

#include "kernels.hpp"
#include "scene_layout.hpp"

namespace robast {

// Longest photon path the boundary kernel follows (events).
constexpr int kBndMaxEvents = 32;
// Distance (in each edge's own units) at which the fates on either side of
// an edge are taken: above the rounding of the FP32 search (hit points to
// about 1e-7 of the scene size), far below any band.
constexpr double kBndPush = 2e-5;

// Writes the per-group weights w[g] = cot[g] / (N_g band) from the forward
// group sums, then adds the boundary terms of photons [0, n) to grad.
template <typename T>
hipError_t launch_boundary(const SceneView<T>& S, const RaysView<T>& R, int64_t n, const double* sums,
                           const double* cot, double* w, double band, double* grad, int n_params, int lds_cap,
                           hipStream_t st);

}  // namespace robast
