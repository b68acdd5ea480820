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
  // When set, photon i of these arrays is photon perm[i] of the caller's
  // bundle: it is numbered id_base + perm[i] and its results go to perm[i].
  const uint32_t* perm = nullptr;
  // Elements between consecutive photons: 1 for the caller's separate
  // arrays; binned copies interleave each photon into one record.
  int64_t stride = 1;    // in T
  int64_t ustride = 1;   // in uint32_t (group, perm)
  // Wavelength of each photon (metres), in the caller's order (indexed by
  // src(i), also for binned copies), or null.
  const T* lam = nullptr;

  __device__ __forceinline__ void load(int64_t i, T o[3], T d[3]) const {
    const int64_t k = i * stride;
    o[0] = ox[k]; o[1] = oy[k]; o[2] = oz[k];
    d[0] = dx[k]; d[1] = dy[k]; d[2] = dz[k];
  }
  __device__ __forceinline__ int grp(int64_t i) const { return group ? (int)group[i * ustride] : 0; }
  // index of photon i in the caller's bundle
  __device__ __forceinline__ int64_t src(int64_t i) const { return perm ? (int64_t)perm[i * ustride] : i; }
  // wavelength of photon i when the kernel carries wavelengths (SH has kLambda), else 0
  template <int SH> __device__ __forceinline__ double wavelength(int64_t i) const {
    if constexpr ((SH & kLambda) != 0) return (double)lam[src(i)];
    else return 0.0;
  }
};

// Path record of a photon, written by a forward trace for the adjoint that
// follows it: four words per photon, indexed by the photon's position in the
// traced order.  A FOCUSED photon with at most kPathSlots events stores its
// event codes (vol << 8 | face << 4 | action) followed by kPathEnd; any other
// photon stores kPathSkip (not FOCUSED: no gradient) or kPathLong (FOCUSED
// with more events: its sequence is found again by a full trace) in word 0.
constexpr int kPathSlots = 4;
constexpr uint32_t kPathEnd = 0xffffffffu;
constexpr uint32_t kPathSkip = 0xfffffffeu;
constexpr uint32_t kPathLong = 0xfffffffdu;

template <typename T> struct HitsView {
  uint8_t* fate;
  uint8_t* nev;
  int32_t* last_vol;
  T *x, *y, *z, *ux, *uy, *uz, *opl;
  uint64_t* hash;
  double* sums;
  uint32_t* path = nullptr;      // kPathSlots words per photon, or null
  uint32_t* seq_log = nullptr;   // max_events event codes per photon (caller's order), or null
};

struct LaunchCfg {
  int lds_cap;      // stage the scene blob in LDS when it is at most this many bytes
  int waves_mult;   // persistent grid = CUs x resident blocks per CU x waves_mult
  int max_blocks;   // 0 = no cap
  int block;        // threads per workgroup of the forward trace (64..256, a multiple of 64; 0 = 256)
};

// Backward-pass inputs: per-group cotangent coefficients of the objective
// (a_g, xbar_g, ybar_g, b_g), per-photon cotangents of the exit state, and
// the output gradient; optionally the forward sequence hashes to check.
struct AdjView {
  const double* coef;     // n_groups * 4, or null (no figure term)
  double* grad;           // n_params, accumulated
  const DTilt* tilt;      // n_vol (valid where tparam >= 0)
  int n_params;
  const double* pcot = nullptr;          // 6 per photon (caller's order): dL/d(exit x, y, z, ux, uy, uz), or null
  const uint64_t* check_hash = nullptr;  // forward sequence hash per photon (caller's order), or null
  uint32_t* mismatch = nullptr;          // photons whose sequence hash differs from check_hash
};

// Path records of the forward trace for the adjoint, and two lists filled
// by the adjoint's main pass (positions in the traced order, with their
// counts, cleared by the backward launch): the photons whose record holds
// exactly kPathSlots events (list4, count[1]) and those whose record is
// kPathLong (list, count[0]).
struct PathView {
  const uint32_t* rec;
  uint32_t* list;
  uint32_t* count;   // 2 counters
  uint32_t* list4;
};

template <typename T>
hipError_t launch_trace(const SceneView<T>& S, const RaysView<T>& R, int64_t n, const HitsView<T>& H,
                        const LaunchCfg& cfg, hipStream_t st);
hipError_t launch_figures(const double* sums, double* fig, int n_groups, hipStream_t st);
// Arrival-time spread per group from per-photon records (see
// robast_arrival_figures): out[4 g .. 4 g + 3] = {FOCUSED photons, mean
// optical path, RMS optical path spread, 0}.
template <typename T>
hipError_t launch_arrival(const uint8_t* fate, const T* opl, const uint32_t* group, int64_t n, int n_groups,
                          double* out, hipStream_t st);
hipError_t launch_adj_coef(const double* sums, const double* cot, double* coef, int n_groups,
                           hipStream_t st);
// With `P` (non-null) the photons' sequences are read from the forward
// trace's path records instead of being found again by a search.
template <typename T>
hipError_t launch_backward(const SceneView<T>& S, const RaysView<T>& R, int64_t n, const AdjView& A,
                           const LaunchCfg& cfg, hipStream_t st, const PathView* P = nullptr);

}  // namespace robast
