// Spatial binning of a photon bundle before tracing.
//
// Photons whose paths start close together meet the same surfaces, visit the
// same grid cells and take the same branches, so a wave of such photons
// diverges far less than a wave of photons drawn at random over the
// aperture.  The bundle is ordered by a key made of the photon's group and
// the cell (row-major in a square grid) where its line crosses a reference
// plane z = z_ref, by a counting sort: count per bin (the atomic's return
// value is the photon's rank inside its bin), exclusive scan of the counts,
// scatter.  The permutation is kept: the trace numbers each photon by its
// original index (its random draws and its result do not depend on the
// order) and writes per-photon results back at that index.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "binning.hpp"

namespace robast {

constexpr int kBinBlock = 256;
constexpr int kScanPerThread = 4;
constexpr int kScanTile = kBinBlock * kScanPerThread;   // bins per scan block

__global__ void k_fill_u32(uint32_t* p, int64_t n, uint32_t v) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

// bundle of photon i: the last v with offsets[v] <= i (offsets ascending)
__device__ __forceinline__ int bundle_of(const int64_t* offsets, int n_var, int64_t i) {
  int lo = 0, hi = n_var - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (offsets[mid] <= i) lo = mid; else hi = mid - 1;
  }
  return lo;
}

template <typename T, bool MULTI>
__global__ void __launch_bounds__(kBinBlock) k_bin_count(RaysView<T> R, int64_t n, BinGeom geo1, BinMulti multi,
                                                         uint32_t* key, uint32_t* rank, uint32_t* hist) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const BinGeom geo = MULTI ? multi.geo[bundle_of(multi.offsets, multi.n_var, i)] : geo1;
    T o[3], d[3];
    R.load(i, o, d);
    double ox = (double)o[0], oy = (double)o[1];
    const double oz = (double)o[2], dx = (double)d[0], dy = (double)d[1], dz = (double)d[2];
    // where the line crosses the reference plane (the origin itself for
    // lines nearly parallel to it)
    if (fabs(dz) > 1e-3) {
      const double s = (geo.z_ref - oz) / dz;
      ox += s * dx;
      oy += s * dy;
    }
    uint32_t g = (uint32_t)R.grp(i);
    if (g >= (uint32_t)geo.n_groups) g = 0u;
    const double fx = (ox - geo.x0) * geo.inv_cell, fy = (oy - geo.y0) * geo.inv_cell;
    const int ix = (int)fmin(fmax(fx, 0.0), (double)(geo.nc - 1));
    const int iy = (int)fmin(fmax(fy, 0.0), (double)(geo.nc - 1));
    const uint32_t k = geo.base + (g * (uint32_t)geo.nc + (uint32_t)iy) * (uint32_t)geo.nc + (uint32_t)ix;
    key[i] = k;
    rank[i] = atomicAdd(hist + k, 1u);
  }
}

// Exclusive scan of the bin counts in place, in three passes: tiles of
// kScanTile bins scanned in LDS (tile totals to `part`), the tile totals
// scanned by one workgroup, the tile offsets added back.
__device__ __forceinline__ uint32_t block_exclusive_scan(uint32_t v, uint32_t* sh, uint32_t& total) {
  const int t = threadIdx.x;
  sh[t] = v;
  __syncthreads();
  for (int o = 1; o < kBinBlock; o <<= 1) {
    uint32_t add = t >= o ? sh[t - o] : 0u;
    __syncthreads();
    sh[t] += add;
    __syncthreads();
  }
  total = sh[kBinBlock - 1];
  const uint32_t incl = sh[t];
  __syncthreads();
  return incl - v;
}

__global__ void __launch_bounds__(kBinBlock) k_scan_tiles(uint32_t* hist, int64_t bins, uint32_t* part) {
  __shared__ uint32_t sh[kBinBlock];
  const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanPerThread;
  uint32_t v[kScanPerThread];
  uint32_t s = 0;
#pragma unroll
  for (int k = 0; k < kScanPerThread; ++k) {
    v[k] = base + k < bins ? hist[base + k] : 0u;
    s += v[k];
  }
  uint32_t total;
  uint32_t run = block_exclusive_scan(s, sh, total);
#pragma unroll
  for (int k = 0; k < kScanPerThread; ++k) {
    if (base + k < bins) hist[base + k] = run;
    run += v[k];
  }
  if (threadIdx.x == 0) part[blockIdx.x] = total;
}

__global__ void __launch_bounds__(kBinBlock) k_scan_parts(uint32_t* part, int n_parts) {
  __shared__ uint32_t sh[kBinBlock];
  uint32_t carry = 0;
  for (int base = 0; base < n_parts; base += kBinBlock) {
    const int i = base + threadIdx.x;
    const uint32_t v = i < n_parts ? part[i] : 0u;
    uint32_t total;
    const uint32_t ex = block_exclusive_scan(v, sh, total);
    if (i < n_parts) part[i] = carry + ex;
    carry += total;
  }
}

__global__ void __launch_bounds__(kBinBlock) k_scan_add(uint32_t* hist, int64_t bins, const uint32_t* part) {
  const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanPerThread;
  const uint32_t add = part[blockIdx.x];
#pragma unroll
  for (int k = 0; k < kScanPerThread; ++k)
    if (base + k < bins) hist[base + k] += add;
}

template <typename T>
__global__ void __launch_bounds__(kBinBlock) k_bin_scatter(RaysView<T> R, int64_t n, const uint32_t* key,
                                                           const uint32_t* rank, const uint32_t* offs,
                                                           BinRecord<T>* out) {
  static_assert(sizeof(BinRecord<T>) % 16 == 0, "records are written as 16-byte words");
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    BinRecord<T> r{};
    R.load(i, r.c, r.c + 3);
    r.group = (uint32_t)R.grp(i);
    r.src = (uint32_t)i;
    const uint32_t slot = offs[key[i]] + rank[i];
    const uint4* from = reinterpret_cast<const uint4*>(&r);
    uint4* to = reinterpret_cast<uint4*>(out + slot);
#pragma unroll
    for (int k = 0; k < (int)(sizeof(BinRecord<T>) / 16); ++k) to[k] = from[k];
  }
}

static int grid_for(int64_t n) {
  return (int)std::max<int64_t>(1, std::min<int64_t>((n + kBinBlock - 1) / kBinBlock, 8192));
}

int64_t bin_scan_parts(int64_t bins) { return (bins + kScanTile - 1) / kScanTile; }

template <typename T>
hipError_t launch_binning(const RaysView<T>& R, int64_t n, const BinGeom& geo, const BinMulti& multi,
                          int64_t bins, const BinWork<T>& W, hipStream_t st) {
  const int64_t parts = bin_scan_parts(bins);
  hipLaunchKernelGGL(k_fill_u32, dim3(grid_for(bins)), dim3(kBinBlock), 0, st, W.hist, bins, 0u);
  if (multi.n_var > 0)
    hipLaunchKernelGGL((k_bin_count<T, true>), dim3(grid_for(n)), dim3(kBinBlock), 0, st, R, n, geo, multi, W.key,
                       W.rank, W.hist);
  else
    hipLaunchKernelGGL((k_bin_count<T, false>), dim3(grid_for(n)), dim3(kBinBlock), 0, st, R, n, geo, multi, W.key,
                       W.rank, W.hist);
  hipLaunchKernelGGL(k_scan_tiles, dim3((unsigned)parts), dim3(kBinBlock), 0, st, W.hist, bins, W.part);
  hipLaunchKernelGGL(k_scan_parts, dim3(1), dim3(kBinBlock), 0, st, W.part, (int)parts);
  hipLaunchKernelGGL(k_scan_add, dim3((unsigned)parts), dim3(kBinBlock), 0, st, W.hist, bins, W.part);
  hipLaunchKernelGGL(k_bin_scatter<T>, dim3(grid_for(n)), dim3(kBinBlock), 0, st, R, n, W.key, W.rank, W.hist,
                     W.out);
  return hipGetLastError();
}

template hipError_t launch_binning<float>(const RaysView<float>&, int64_t, const BinGeom&, const BinMulti&, int64_t,
                                          const BinWork<float>&, hipStream_t);
template hipError_t launch_binning<double>(const RaysView<double>&, int64_t, const BinGeom&, const BinMulti&,
                                           int64_t, const BinWork<double>&, hipStream_t);

}  // namespace robast
