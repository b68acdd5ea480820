// Spatial binning of a photon bundle before tracing.
//
// Photons whose paths start close together meet the same surfaces, visit the
// same grid cells and take the same branches, so a wave of such photons
// diverges far less than a wave of photons drawn at random over the
// aperture.  The bundle is ordered by a key made of the photon's group and
// the cell (row-major in a square grid) where its line crosses a reference
// plane z = z_ref, optionally preceded by the sector of the direction's
// azimuth (photons that enter together but in different directions part at
// once).  The permutation is kept: the trace numbers each photon by
// its original index (its random draws and its result do not depend on the
// order) and writes per-photon results back at that index.
//
// The sort is a two-level counting sort that needs no per-photon global
// atomics: (1) each tile of photons counts its keys' coarse digits in LDS and
// writes one count per (coarse bucket, tile); (2) an exclusive scan of those
// counts, bucket-major, gives every (bucket, tile) its output range, and the
// tile scatters its photons there (LDS cursors); (3) one workgroup per coarse
// bucket counts the fine digits in LDS, scans them and scatters the bucket's
// photons into key order.  Order within a (bucket, tile) or within a bin is
// whatever the LDS atomics give: it changes only which lane traces which
// photon.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "binning.hpp"

namespace robast {

constexpr int kBinBlock = 256;
// The scatters run one large workgroup per CU (the LDS request below keeps a
// second one off the CU): fewer output streams open at once per XCD, so more
// of the partially written lines are completed in L2 before write-back.
constexpr int kCoarseBlock = 1024;                      // threads of a keys / coarse-pass workgroup
constexpr int kFineBlock = 1024;                        // threads of a fine-pass workgroup
constexpr size_t kScatterLds = 90 * 1024;               // LDS requested by each scatter workgroup
constexpr int kUnroll = 4;                              // photons in flight per thread in the scatters
                                                        // (the fine pass is written out for 4)
constexpr int kScanPerThread = 4;
constexpr int kScanTile = kBinBlock * kScanPerThread;   // entries per scan block
constexpr int kMaxCoarse = 2048;                        // LDS counters of the coarse pass
constexpr int kMaxFineShift = 13;                       // LDS counters of the fine pass: 2^13
constexpr int64_t kTileMax = int64_t(1) << 21;          // photons per tile of the coarse pass, at most
constexpr int64_t kTileMin = 4096;                      // and at least
constexpr int64_t kTilesWanted = 512;                   // two rounds of one workgroup per CU (256 and
                                                        // 1024 were 0.1-0.2 ms slower on 1.6e8 photons)
// staged fine scatter (FP32 records): buckets of at most kStagedMaxFine bins,
// kChunk photons at a time through LDS (fits the kScatterLds request)
constexpr int kStagedMaxFine = 1024;
constexpr int kChunk = 2 * kFineBlock;
static_assert((3 * kStagedMaxFine + kChunk + 4) * 4 + kChunk * 32 <= (int)kScatterLds,
              "staged fine scatter exceeds its LDS");

// bundle of photon i: the last v with offsets[v] <= i (offsets ascending)
__device__ __forceinline__ int bundle_of(const int64_t* offsets, int n_var, int64_t i) {
  int lo = 0, hi = n_var - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (offsets[mid] <= i) lo = mid; else hi = mid - 1;
  }
  return lo;
}

template <typename T>
__device__ __forceinline__ uint32_t photon_key(const RaysView<T>& R, int64_t i, const BinGeom& geo) {
  T o[3], d[3];
  R.load(i, o, d);
  double ox = (double)o[0], oy = (double)o[1];
  const double oz = (double)o[2], dx = (double)d[0], dy = (double)d[1], dz = (double)d[2];
  // where the line crosses the reference plane (the origin itself for lines
  // nearly parallel to it)
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
  uint32_t gs = g;
  if (geo.dirs > 1u) {
    // sector of atan2(dy, dx) in [-pi, pi]; single precision is enough, the
    // order only groups photons
    const float a = atan2f((float)dy, (float)dx) + 3.14159265f;
    const int k = (int)(a * (float)geo.dirs * 0.159154943f);
    gs = g * geo.dirs + (uint32_t)(k < 0 ? 0 : (k >= (int)geo.dirs ? (int)geo.dirs - 1 : k));
  }
  return geo.base + (gs * (uint32_t)geo.nc + (uint32_t)iy) * (uint32_t)geo.nc + (uint32_t)ix;
}

// (1) keys and per-tile coarse counts; cnt is bucket-major: cnt[c * n_tiles + tile]
template <typename T, bool MULTI>
__global__ void __launch_bounds__(kCoarseBlock) k_bin_keys(RaysView<T> R, int64_t n, BinGeom geo1, BinMulti multi,
                                                        int shift, int n_coarse, int n_tiles, int64_t tile,
                                                        uint32_t* key, uint32_t* cnt) {
  extern __shared__ uint32_t hist[];
  for (int c = threadIdx.x; c < n_coarse; c += blockDim.x) hist[c] = 0u;
  __syncthreads();
  const int64_t lo = (int64_t)blockIdx.x * tile, hi = lo + tile < n ? lo + tile : n;
  if constexpr (MULTI) {
    // a thread's photons only move forward through the bundles: find its
    // first bundle once, then step past bundle ends (offsets[n_var] = n ends
    // every step) and load a bundle's geometry only when it changes
    int64_t i = lo + threadIdx.x;
    if (i < hi) {
      int v = bundle_of(multi.offsets, multi.n_var, i);
      int64_t v_end = multi.offsets[v + 1];
      BinGeom geo = multi.geo[v];
      for (; i < hi; i += blockDim.x) {
        if (i >= v_end) {
          while (i >= v_end) v_end = multi.offsets[++v + 1];
          geo = multi.geo[v];
        }
        const uint32_t k = photon_key<T>(R, i, geo);
        key[i] = k;
        atomicAdd(hist + (k >> shift), 1u);
      }
    }
  } else {
    for (int64_t i = lo + threadIdx.x; i < hi; i += blockDim.x) {
      const uint32_t k = photon_key<T>(R, i, geo1);
      key[i] = k;
      atomicAdd(hist + (k >> shift), 1u);
    }
  }
  __syncthreads();
  for (int c = threadIdx.x; c < n_coarse; c += blockDim.x) cnt[(int64_t)c * n_tiles + blockIdx.x] = hist[c];
}

// (2) each tile scatters its photons to its range of every coarse bucket
template <typename T>
__global__ void __launch_bounds__(kCoarseBlock) k_bin_coarse(RaysView<T> R, int64_t n, int shift, int n_coarse,
                                                          int n_tiles, int64_t tile, const uint32_t* key,
                                                          const uint32_t* offs, uint32_t* tkey, BinRecord<T>* tmp) {
  static_assert(sizeof(BinRecord<T>) % 16 == 0, "records are written as 16-byte words");
  extern __shared__ uint32_t cursor[];
  for (int c = threadIdx.x; c < n_coarse; c += blockDim.x) cursor[c] = offs[(int64_t)c * n_tiles + blockIdx.x];
  __syncthreads();
  const int64_t lo = (int64_t)blockIdx.x * tile, hi = lo + tile < n ? lo + tile : n;
  // kUnroll photons per thread at a time: all their loads are issued before
  // the first store, so that each thread keeps several in flight
  for (int64_t base = lo + threadIdx.x; base < hi; base += (int64_t)blockDim.x * kUnroll) {
    uint32_t k[kUnroll], pos[kUnroll];
    BinRecord<T> r[kUnroll];
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
      const int64_t i = base + (int64_t)u * blockDim.x;
      if (i < hi) {
        k[u] = key[i];
        R.load(i, r[u].c, r[u].c + 3);
        r[u].group = (uint32_t)R.grp(i);
        r[u].src = (uint32_t)i;
      }
    }
#pragma unroll
    for (int u = 0; u < kUnroll; ++u)
      if (base + (int64_t)u * blockDim.x < hi) pos[u] = atomicAdd(cursor + (k[u] >> shift), 1u);
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
      if (base + (int64_t)u * blockDim.x < hi) {
        const uint4* from = reinterpret_cast<const uint4*>(&r[u]);
        uint4* to = reinterpret_cast<uint4*>(tmp + pos[u]);
#pragma unroll
        for (int w = 0; w < (int)(sizeof(BinRecord<T>) / 16); ++w) to[w] = from[w];
        tkey[pos[u]] = k[u];
      }
    }
  }
}

template <int NT> __device__ __forceinline__ uint32_t block_exclusive_scan(uint32_t v, uint32_t* sh, uint32_t& total);

// Inclusive scan across the 64 lanes of a wave.
__device__ __forceinline__ uint32_t wave_inclusive_scan(uint32_t v) {
  const int lane = (int)__lane_id();
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t t = __shfl_up(v, o, 64);
    if (lane >= o) v += t;
  }
  return v;
}

// Exclusive scan across a workgroup of NT threads (NT / 64 <= 64 waves) with
// two barriers: each wave scans its lanes, one wave scans the wave totals
// (sh: NT / 64 words of LDS, free again after the second barrier's readers).
template <int NT> __device__ __forceinline__ uint32_t block_exclusive_scan_waves(uint32_t v, uint32_t* sh) {
  static_assert(NT % 64 == 0 && NT / 64 <= 64, "one wave scans the wave totals");
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const uint32_t incl = wave_inclusive_scan(v);
  if (lane == 63) sh[w] = incl;
  __syncthreads();
  if (w == 0) {
    const uint32_t x = lane < NT / 64 ? sh[lane] : 0u;
    const uint32_t xi = wave_inclusive_scan(x);
    if (lane < NT / 64) sh[lane] = xi - x;
  }
  __syncthreads();
  return incl - v + sh[w];
}

// (3) one workgroup per coarse bucket: fine counting sort into key order
template <typename T>
__global__ void __launch_bounds__(kFineBlock) k_bin_fine(int64_t n, int shift, int n_coarse, int n_tiles,
                                                         const uint32_t* offs, const uint32_t* tkey,
                                                         const BinRecord<T>* tmp, BinRecord<T>* out) {
  extern __shared__ __align__(16) uint32_t fine[];
  __shared__ uint32_t sh[kFineBlock];
  const int c = blockIdx.x;
  const int nf = 1 << shift;
  const uint32_t mask = (uint32_t)nf - 1u;
  const int64_t start = offs[(int64_t)c * n_tiles];
  const int64_t end = c + 1 < n_coarse ? (int64_t)offs[(int64_t)(c + 1) * n_tiles] : n;
  for (int f = threadIdx.x; f < nf; f += blockDim.x) fine[f] = 0u;
  __syncthreads();
  for (int64_t base = start + threadIdx.x; base < end; base += (int64_t)blockDim.x * kUnroll) {
    uint32_t k[kUnroll];
#pragma unroll
    for (int u = 0; u < kUnroll; ++u)
      if (base + (int64_t)u * blockDim.x < end) k[u] = tkey[base + (int64_t)u * blockDim.x];
#pragma unroll
    for (int u = 0; u < kUnroll; ++u)
      if (base + (int64_t)u * blockDim.x < end) atomicAdd(fine + (k[u] & mask), 1u);
  }
  __syncthreads();
  // exclusive scan of the fine counts: contiguous runs per thread, then the
  // run totals across the workgroup
  const int per = (nf + kFineBlock - 1) / kFineBlock;
  const int f0 = threadIdx.x * per;
  uint32_t run = 0;
  for (int k = 0; k < per; ++k)
    if (f0 + k < nf) run += fine[f0 + k];
  uint32_t total;
  uint32_t acc = block_exclusive_scan<kFineBlock>(run, sh, total);
  for (int k = 0; k < per; ++k)
    if (f0 + k < nf) {
      const uint32_t v = fine[f0 + k];
      fine[f0 + k] = acc;
      acc += v;
    }
  __syncthreads();
  // FP32 records: kUnroll photons per thread at a time, all loads issued
  // before the first store, their 16-byte words in named registers (past
  // the end the last photon is loaded again and never stored)
  const uint4* src = reinterpret_cast<const uint4*>(tmp);
  uint4* dst = reinterpret_cast<uint4*>(out);
  const int64_t step = blockDim.x;
  if constexpr (sizeof(BinRecord<T>) == 32) {
    if (nf <= kStagedMaxFine) {
      // staged: chunks of kChunk photons are put in fine-digit order in LDS,
      // then written out slot by slot, so that consecutive lanes write
      // consecutive records of one bin (runs of whole lines) instead of
      // 32-byte pieces scattered over all the bins
      uint32_t* lc = fine + nf;   // the chunk's count per digit
      uint32_t* ls = fine + 2 * nf;   // and its exclusive scan
      uint32_t* dig = fine + 3 * nf;   // digit of each LDS slot
      uint4* rec = reinterpret_cast<uint4*>(fine + ((3 * nf + kChunk + 3) & ~3));
      const int tid = threadIdx.x;
      for (int64_t cb = start; cb < end; cb += kChunk) {
        const int cnt = (int)std::min<int64_t>(kChunk, end - cb);
        for (int f = tid; f < nf; f += kFineBlock) lc[f] = 0u;
        __syncthreads();
        const int s0 = tid, s1 = tid + kFineBlock;
        const bool h0 = s0 < cnt, h1 = s1 < cnt;
        uint32_t f0 = 0u, f1 = 0u, r0 = 0u, r1 = 0u;
        uint4 a0 = {}, a1 = {}, b0 = {}, b1 = {};
        if (h0) { f0 = tkey[cb + s0] & mask; a0 = src[2 * (cb + s0)]; a1 = src[2 * (cb + s0) + 1]; }
        if (h1) { f1 = tkey[cb + s1] & mask; b0 = src[2 * (cb + s1)]; b1 = src[2 * (cb + s1) + 1]; }
        if (h0) r0 = atomicAdd(lc + f0, 1u);
        if (h1) r1 = atomicAdd(lc + f1, 1u);
        __syncthreads();
        const uint32_t ex = block_exclusive_scan_waves<kFineBlock>(tid < nf ? lc[tid] : 0u, sh);
        if (tid < nf) ls[tid] = ex;
        __syncthreads();
        // slots: ls[f] + rank covers [0, cnt) once
        if (h0) { const uint32_t q = ls[f0] + r0; rec[2 * q] = a0; rec[2 * q + 1] = a1; dig[q] = f0; }
        if (h1) { const uint32_t q = ls[f1] + r1; rec[2 * q] = b0; rec[2 * q + 1] = b1; dig[q] = f1; }
        __syncthreads();
        for (int q = tid; q < cnt; q += kFineBlock) {
          const uint32_t f = dig[q];
          const int64_t p = start + (int64_t)fine[f] + (int64_t)(q - (int)ls[f]);
          dst[2 * p] = rec[2 * q];
          dst[2 * p + 1] = rec[2 * q + 1];
        }
        __syncthreads();
        for (int f = tid; f < nf; f += kFineBlock) fine[f] += lc[f];
        __syncthreads();
      }
      return;
    }
    for (int64_t i0 = start + threadIdx.x; i0 < end; i0 += step * kUnroll) {
      const int64_t i1 = i0 + step, i2 = i0 + 2 * step, i3 = i0 + 3 * step;
      const int64_t j1 = i1 < end ? i1 : end - 1, j2 = i2 < end ? i2 : end - 1, j3 = i3 < end ? i3 : end - 1;
      const uint32_t k0 = tkey[i0], k1 = tkey[j1], k2 = tkey[j2], k3 = tkey[j3];
      const uint4 a0 = src[2 * i0], a1 = src[2 * i0 + 1], b0 = src[2 * j1], b1 = src[2 * j1 + 1];
      const uint4 c0 = src[2 * j2], c1 = src[2 * j2 + 1], d0 = src[2 * j3], d1 = src[2 * j3 + 1];
      const int64_t p0 = start + atomicAdd(fine + (k0 & mask), 1u);
      dst[2 * p0] = a0;
      dst[2 * p0 + 1] = a1;
      if (i1 < end) {
        const int64_t p = start + atomicAdd(fine + (k1 & mask), 1u);
        dst[2 * p] = b0;
        dst[2 * p + 1] = b1;
      }
      if (i2 < end) {
        const int64_t p = start + atomicAdd(fine + (k2 & mask), 1u);
        dst[2 * p] = c0;
        dst[2 * p + 1] = c1;
      }
      if (i3 < end) {
        const int64_t p = start + atomicAdd(fine + (k3 & mask), 1u);
        dst[2 * p] = d0;
        dst[2 * p + 1] = d1;
      }
    }
  } else {
    constexpr int W = (int)(sizeof(BinRecord<T>) / 16);
    for (int64_t i = start + threadIdx.x; i < end; i += step) {
      const int64_t p = start + atomicAdd(fine + (tkey[i] & mask), 1u);
#pragma unroll
      for (int q = 0; q < W; ++q) dst[p * W + q] = src[i * W + q];
    }
  }
}

// Exclusive scan across a workgroup of NT threads (sh: NT words of LDS).
template <int NT> __device__ __forceinline__ uint32_t block_exclusive_scan(uint32_t v, uint32_t* sh, uint32_t& total) {
  const int t = threadIdx.x;
  sh[t] = v;
  __syncthreads();
  for (int o = 1; o < NT; o <<= 1) {
    uint32_t add = t >= o ? sh[t - o] : 0u;
    __syncthreads();
    sh[t] += add;
    __syncthreads();
  }
  total = sh[NT - 1];
  const uint32_t incl = sh[t];
  __syncthreads();
  return incl - v;
}

// Exclusive scan of the bin counts in place, in three passes: tiles of
// kScanTile bins scanned in LDS (tile totals to `part`), the tile totals
// scanned by one workgroup, the tile offsets added back.
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
  uint32_t run = block_exclusive_scan<kBinBlock>(s, sh, total);
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
    const uint32_t ex = block_exclusive_scan<kBinBlock>(v, sh, total);
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

static int grid_for(int64_t n) {
  return (int)std::max<int64_t>(1, std::min<int64_t>((n + kBinBlock - 1) / kBinBlock, 8192));
}

static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

template <typename T> BinPlan bin_plan(int64_t n, int64_t bins) {
  BinPlan p{};
  int shift = 0;
  while ((bins + (int64_t(1) << shift) - 1) >> shift > kMaxCoarse) ++shift;
  p.shift = shift;
  p.n_coarse = (int)((bins + (int64_t(1) << shift) - 1) >> shift);
  p.tile = std::min(kTileMax, std::max(kTileMin, ((n + kTilesWanted - 1) / kTilesWanted + 255) / 256 * 256));
  p.n_tiles = (int)((n + p.tile - 1) / p.tile);
  p.cnt_entries = (int64_t)p.n_coarse * p.n_tiles;
  p.parts = (p.cnt_entries + kScanTile - 1) / kScanTile;
  size_t off = 0;
  p.key_off = off; off += align256((size_t)n * 4);
  p.tkey_off = off; off += align256((size_t)n * 4);
  p.tmp_off = off; off += align256((size_t)n * sizeof(BinRecord<T>));
  p.out_off = off; off += align256((size_t)n * sizeof(BinRecord<T>));
  p.cnt_off = off; off += align256((size_t)p.cnt_entries * 4);
  p.part_off = off; off += align256((size_t)p.parts * 4);
  p.bytes = off;
  return p;
}

template <typename T> BinWork<T> bin_carve(const BinPlan& p, void* base) {
  char* b = (char*)base;
  BinWork<T> W;
  W.key = (uint32_t*)(b + p.key_off);
  W.tkey = (uint32_t*)(b + p.tkey_off);
  W.tmp = (BinRecord<T>*)(b + p.tmp_off);
  W.out = (BinRecord<T>*)(b + p.out_off);
  W.cnt = (uint32_t*)(b + p.cnt_off);
  W.part = (uint32_t*)(b + p.part_off);
  return W;
}

template <typename T>
hipError_t launch_binning(const RaysView<T>& R, int64_t n, const BinGeom& geo, const BinMulti& multi,
                          const BinPlan& p, const BinWork<T>& W, hipStream_t st) {
  if (p.shift > kMaxFineShift || p.n_coarse > kMaxCoarse) return hipErrorInvalidValue;
  const size_t coarse_lds = (size_t)p.n_coarse * 4, fine_lds = ((size_t)1 << p.shift) * 4;
  if (multi.n_var > 0)
    hipLaunchKernelGGL((k_bin_keys<T, true>), dim3(p.n_tiles), dim3(kCoarseBlock), coarse_lds, st, R, n, geo, multi,
                       p.shift, p.n_coarse, p.n_tiles, p.tile, W.key, W.cnt);
  else
    hipLaunchKernelGGL((k_bin_keys<T, false>), dim3(p.n_tiles), dim3(kCoarseBlock), coarse_lds, st, R, n, geo, multi,
                       p.shift, p.n_coarse, p.n_tiles, p.tile, W.key, W.cnt);
  hipLaunchKernelGGL(k_scan_tiles, dim3((unsigned)p.parts), dim3(kBinBlock), 0, st, W.cnt, p.cnt_entries, W.part);
  hipLaunchKernelGGL(k_scan_parts, dim3(1), dim3(kBinBlock), 0, st, W.part, (int)p.parts);
  hipLaunchKernelGGL(k_scan_add, dim3((unsigned)p.parts), dim3(kBinBlock), 0, st, W.cnt, p.cnt_entries, W.part);
  hipLaunchKernelGGL(k_bin_coarse<T>, dim3(p.n_tiles), dim3(kCoarseBlock), std::max(coarse_lds, kScatterLds), st, R, n, p.shift, p.n_coarse,
                     p.n_tiles, p.tile, W.key, W.cnt, W.tkey, W.tmp);
  hipLaunchKernelGGL(k_bin_fine<T>, dim3(p.n_coarse), dim3(kFineBlock), std::max(fine_lds, kScatterLds), st, n, p.shift, p.n_coarse,
                     p.n_tiles, W.cnt, W.tkey, W.tmp, W.out);
  return hipGetLastError();
}

template BinPlan bin_plan<float>(int64_t, int64_t);
template BinPlan bin_plan<double>(int64_t, int64_t);
template BinWork<float> bin_carve<float>(const BinPlan&, void*);
template BinWork<double> bin_carve<double>(const BinPlan&, void*);
template hipError_t launch_binning<float>(const RaysView<float>&, int64_t, const BinGeom&, const BinMulti&,
                                          const BinPlan&, const BinWork<float>&, hipStream_t);
template hipError_t launch_binning<double>(const RaysView<double>&, int64_t, const BinGeom&, const BinMulti&,
                                           const BinPlan&, const BinWork<double>&, hipStream_t);

}  // namespace robast
