// Parameter updates of compiled scenes on the device.
//
// A scene's tables live in one of two slots of device memory; the scene's
// device view points at the live one.  An update rebuilds the volume and
// group records from new parameter values into the other slot and then
// switches the view, in stream order and without the host, so that a
// gradient-descent step can run inside a captured graph and kernels still
// running on the old slot never see half-written tables.  The candidate
// grid (which cells list which volume) is kept: an update is applied only if
// no surface moves, across the group's grid, by more than the margin the
// grid was rasterised with; otherwise the scene keeps its tables and the
// caller rebuilds it on the host.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

#include "scene_layout.hpp"

namespace robast {

// A volume as the last host build saw it (FP64): what the device needs to
// rebuild its record from new parameter values.
struct UpdVol {
  double Q[9], c[3];                            // frame of the last build
  double Q0[9], c0[3], pivot[3], e1[3], e2[3];  // untilted frame, pivot, tilt axes
  double p[16];                                 // shape parameters of the last build
  double lb_lo[3], lb_hi[3];                    // local box of the surface at the last build
  double rmin, rmax;                            // outline radii
  double gpad;                                  // surface displacement (group frame, lateral) the grid
                                                // tolerates; < 0: the volume is in no group
  int32_t shape, outline, sparam, tparam, group, role;
};

// A candidate group: its frame and z-slab padding as built, and its members.
struct UpdGroup {
  double Q[9], c[3];
  double zpad;
  int32_t first, count;   // members[first .. first + count)
};

// Everything one scene's update touches (device memory, owned by the scene).
template <typename T> struct UpdJob {
  SceneView<T>* view;      // the scene's device view (read, then switched)
  char* slot[2];           // table slots (blob_bytes each, 256-byte aligned)
  DTilt* tilt[2];          // tilt-table slots (n_vol each)
  const UpdVol* vols;      // n_vol
  const UpdGroup* groups;  // n_grp
  const uint16_t* members;
  double* zr;              // scratch, 2 per volume: group-frame z range
  double* pn;              // scratch, n_params: the parameters of a gradient step
  int32_t n_vol, n_grp, n_params;
  uint32_t blob_bytes;
  double l_ref;
};

// Updates job j (j < n_jobs) from params + (poff ? poff[j] : 0); status[j]
// (if status) becomes 0 when applied, ROBAST_EINVAL for parameters that make
// a surface invalid, ROBAST_EUNSUPPORTED when a surface would leave its
// grid cells; in both cases the scene keeps its tables.
// With grad and lr (same offsets as params), a gradient-descent step: the
// new parameters are params - lr * grad, and params takes them where the
// update is applied (and keeps its values where it is not).
template <typename T>
hipError_t launch_update_params(const UpdJob<T>* const* jobs, int n_jobs, double* params, const int64_t* poff,
                                int32_t* status, hipStream_t st, const double* grad = nullptr,
                                const double* lr = nullptr);

}  // namespace robast
