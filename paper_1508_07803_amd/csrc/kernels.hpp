// Host-visible views of device buffers and the kernel launchers.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

#include "scene_layout.hpp"

namespace robast {

template <typename T> struct RaysView {
  const T *ox, *oy, *oz, *dx, *dy, *dz;
  const uint32_t* group;
  uint64_t id_base;
};

template <typename T> struct HitsView {
  uint8_t* fate;
  uint8_t* nev;
  int32_t* last_vol;
  T *x, *y, *z, *ux, *uy, *uz, *opl;
  uint64_t* hash;
  double* sums;
};

struct LaunchCfg {
  int lds_cap;      // stage the scene blob in LDS when it is at most this many bytes
  int waves_mult;   // persistent grid = CUs x resident blocks per CU x waves_mult
  int max_blocks;   // 0 = no cap
};

// Backward-pass inputs: per-group cotangent coefficients of the objective
// (a_g, xbar_g, ybar_g, b_g) and the output gradient.
struct AdjView {
  const double* coef;     // n_groups * 4
  double* grad;           // n_params, accumulated
  const DTilt* tilt;      // n_vol (valid where tparam >= 0)
  int n_params;
};

template <typename T>
hipError_t launch_trace(const SceneView<T>& S, const RaysView<T>& R, int64_t n, const HitsView<T>& H,
                        const LaunchCfg& cfg, hipStream_t st);
hipError_t launch_figures(const double* sums, double* fig, int n_groups, hipStream_t st);
hipError_t launch_adj_coef(const double* sums, const double* cot, double* coef, int n_groups,
                           hipStream_t st);
template <typename T>
hipError_t launch_backward(const SceneView<T>& S, const RaysView<T>& R, int64_t n, const AdjView& A,
                           const LaunchCfg& cfg, hipStream_t st);

}  // namespace robast
