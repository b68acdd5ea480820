// Spatial binning of photon bundles (ordering for wave coherence).
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

#include "kernels.hpp"

namespace robast {

// Bin geometry: an nc x nc grid of cells of size 1 / inv_cell from (x0, y0)
// on the plane z = z_ref, per photon group and per sector of the direction's
// azimuth (dirs sectors of 2 pi / dirs; 1: direction not used); the bins
// are numbered from base.
struct BinGeom {
  double z_ref, x0, y0, inv_cell;
  int nc, n_groups;
  uint32_t base, dirs;
};

// Photons of several bundles binned together (a batch of scene variants):
// bundle v holds photons [offsets[v], offsets[v+1]) and is binned with
// geo[v], whose bins follow those of bundle v - 1, so every photon stays in
// its bundle's range.
struct BinMulti {
  const int64_t* offsets;   // device, n_var + 1
  const BinGeom* geo;       // device, n_var
  int n_var;
};

// Binned photons, one record per photon: 6 coordinates (ox, oy, oz, dx, dy,
// dz), then the group and the photon's index in the caller's bundle (uint32),
// padded to 32 bytes (FP32) or 64 bytes (FP64) so that a photon is written
// with whole 16-byte stores.
template <typename T> struct BinRecord;
template <> struct alignas(16) BinRecord<float> { float c[6]; uint32_t group, src; };
template <> struct alignas(16) BinRecord<double> { double c[6]; uint32_t group, src, pad[2]; };

// Workspace of one binning (two-level counting sort, see binning.hip).
struct BinPlan {
  int shift;            // fine digit = key & ((1 << shift) - 1), coarse = key >> shift
  int n_coarse;         // coarse buckets
  int n_tiles;          // photon tiles of the coarse pass
  int64_t tile;         // photons per tile
  int64_t cnt_entries;  // n_coarse * n_tiles per-tile counts
  int64_t parts;        // scan partials
  size_t key_off, tkey_off, tmp_off, out_off, cnt_off, part_off, bytes;
};

// Largest bin count a binning supports (keys are 32-bit; the coarse pass
// keeps one LDS counter per coarse bucket and the fine pass one per bin of a
// bucket).
constexpr int64_t kBinsMax = int64_t(1) << 24;

template <typename T> BinPlan bin_plan(int64_t n, int64_t bins);

template <typename T> struct BinWork {
  uint32_t* key;         // n: key per photon (caller order)
  uint32_t* tkey;        // n: key per photon (coarse order)
  BinRecord<T>* tmp;     // n: records in coarse order
  BinRecord<T>* out;     // n: records in key order (the result)
  uint32_t* cnt;         // cnt_entries: per (coarse bucket, tile) counts, then offsets
  uint32_t* part;        // scan partials
};

template <typename T> BinWork<T> bin_carve(const BinPlan& plan, void* base);

// The view of binned records as photon arrays.
template <typename T> RaysView<T> binned_rays(const BinRecord<T>* rec, bool has_group, uint64_t id_base) {
  const T* c = rec->c;
  const uint32_t* u = &rec->group;
  RaysView<T> R{c, c + 1, c + 2, c + 3, c + 4, c + 5, has_group ? u : nullptr, id_base, u + 1};
  R.stride = (int64_t)(sizeof(BinRecord<T>) / sizeof(T));
  R.ustride = (int64_t)(sizeof(BinRecord<T>) / sizeof(uint32_t));
  return R;
}

// One bundle (geo) or several (multi.n_var > 0); bins = total bin count
// (<= kBinsMax), n <= 2^32 - 1; plan = bin_plan<T>(n, bins).
template <typename T>
hipError_t launch_binning(const RaysView<T>& R, int64_t n, const BinGeom& geo, const BinMulti& multi,
                          const BinPlan& plan, const BinWork<T>& W, hipStream_t st);

}  // namespace robast
