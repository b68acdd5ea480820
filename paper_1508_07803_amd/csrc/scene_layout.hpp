// Device scene layout shared by the host scene compiler and the kernels.
//
// A compiled scene is one contiguous blob (staged into LDS by each workgroup
// when it fits):
//   [DVol<T> x n_vol] [u16 always-list] [u32 cell_start x (ncell + 1)] [u16 cell items]
// The XY uniform grid lists, per cell, every volume whose world AABB overlaps
// the cell's column; volumes too large for the grid go on the always-list and
// are tested for every photon.  The grid is only a candidate filter: a
// volume's exact intersection is always computed in its own frame.
#pragma once
#include <cstdint>

namespace robast {

enum Role { MIRROR = 1, LENS = 2, FOCAL = 3, OBSCURATION = 4 };
enum Shape { PLANE = 1, SPHERE = 2, ASPHERE = 3, CYLINDER = 4, BOX = 5, HEXCONE = 6 };
enum Outline { OL_NONE = 0, OL_DISC = 1, OL_ANNULUS = 2, OL_RECT = 3, OL_HEX = 4, OL_SECTOR = 5 };
enum Fate { FOCUSED = 1, ABSORBED = 2, EXITED = 3, SUSPENDED = 4, FAILED = 5 };

// Shape sets the tracing kernels are compiled for (bit 1 << shape): every
// shape, or every shape but the hex cone, for scenes without hex cones (the
// cone's root solver, the largest, then stays out of the kernel and its
// register allocation); the forward trace has a third set, mirrors and
// focal surfaces only (no cylinder or box: telescopes without masts or a
// camera body), whose search keeps fewer values in scratch.
constexpr int kShapesAll = (1 << PLANE) | (1 << SPHERE) | (1 << ASPHERE) | (1 << CYLINDER) | (1 << BOX) | (1 << HEXCONE);
constexpr int kShapesNoCone = kShapesAll & ~(1 << HEXCONE);
constexpr int kShapesMirrors = (1 << PLANE) | (1 << SPHERE) | (1 << ASPHERE);
// Kernel option joined to a shape set: photons carry their own wavelengths
// and dispersive lenses refract them with n(lambda).
constexpr int kLambda = 1 << 16;

// Per-volume record, precision T.
//   p (shape, derived): SPHERE {c}; ASPHERE {rn, b1..b8, 1/rn^2}; CYLINDER {rho, h};
//     BOX {hx, hy, hz}; HEXCONE {rho0 z0 rho1 z1 rho2 z2 rho3 z3}
//   o (outline, derived): DISC {r^2}; ANNULUS {rin^2, rout^2}; RECT {hx, hy};
//     HEX {a}; SECTOR {rin^2, rout^2, cos phi0, sin phi0, cos phi1, sin phi1, wide}
//   lo/hi: local-frame box of the surface (asphere z-slab for bracketing)
//   bmin/bmax: world AABB; slope: max |grad sag| of a sag surface on its outline
//   absl: lenses: absorption length of the medium on the back side (0: none)
//   lenses also keep their dispersion law in p[10] = A, p[11] = B (n = A + B / lambda^2; B = 0: none)
template <typename T> struct alignas(16) DVol {
  T bmin[3], bmax[3];    // world AABB first: the candidate test reads only these and `shape`
  int32_t shape, role;
  int32_t outline, nfaces, sparam, tparam, always_reflect;
  uint32_t thr;          // mirrors: absorb iff draw >= thr (unless always_reflect)
  T Q[9];
  T c[3];
  T p[12];
  T o[8];
  T lo[3], hi[3];
  T n_in, slope, rout, absl;
};

// Tilt data used only by the adjoint: pivot and the two world rotation axes
// a1 = Rot(e2, beta) e1, a2 = e2 of the current tilt.
struct DTilt {
  double pivot[3], a1[3], a2[3];
};

// A candidate group: volumes whose surfaces lie in the slab zmin <= z <= zmax
// of the group frame (x_g = Q (x - c)), with a uniform grid over (x_g, y_g)
// listing per cell the members whose surface projects into that cell.
// Groups are formed by the scene compiler: panels sharing one untilted frame
// (a segmented mirror) form a group in that frame; the remaining volumes are
// split into world-frame layers by their z extent.
template <typename T> struct alignas(16) GroupRec {
  T Q[9];
  T c[3];
  T zmin, zmax, x0, y0, cell, inv_cell;
  int32_t nx, ny;
  uint32_t start;   // index of this group's first cell in cell_start
  uint32_t pad;
};

template <typename T> struct SceneView {
  // device address of the scene's live view: kernels read the view through
  // it, so parameter updates (which rewrite it) reach later launches and
  // graph replays
  const SceneView<T>* self;
  const DVol<T>* vol;
  const uint16_t* always;
  const uint32_t* cell_start;
  const uint16_t* items;
  const GroupRec<T>* groups;
  int32_t n_vol, n_always, n_grp, shapes;   // shapes: bit 1 << shape of every shape present
  int32_t dispersive;                       // some lens has a dispersion law
  int32_t max_events, n_groups;
  uint64_t seed;
  T eps_self;                      // self-intersection guard for the face just left
  double eps_tie;                  // candidates this close are tied (lower volume, then face, wins)
  uint32_t blob_bytes;             // size of the blob (for LDS staging)
  const char* blob;                // start of the blob (== vol)
  const DTilt* tilt;               // n_vol tilt records of the adjoint (beside the blob)
};

}  // namespace robast
