// Batched forward trace: many scene variants in one persistent launch.
//
// Inside a work item each lane traces whole photons exactly like the
// single-scene kernel and numbers them from the variant's first photon, so
// every photon's result (and path record) equals that of a single-scene call
// on its variant.  Per-lane FP64 figure sums are reduced across the wave per group
// after every work item, before one atomic per wave and sum.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "batch_device.hpp"
#include "device_trace.hpp"
#include "kernels.hpp"

namespace robast {

constexpr int kNSumB = 7;   // launched, focused, x, y, x^2, y^2, |u_z|

__global__ void k_batch_reset(uint32_t* q, int first, int count) {
  if ((int)threadIdx.x < count) q[first + threadIdx.x] = 0u;
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Adds each lane's sums (group ag, values a) into target[group * 8 + k]: the
// lanes holding the group of the lowest holding lane reduce across the wave
// and that lane issues the atomics; repeated until no lane holds sums.  Must
// be reached by the whole wave.
__device__ __forceinline__ void wave_flush(double* target, int& ag, double* a) {
  while (true) {
    const unsigned long long m = __ballot(ag >= 0);
    if (m == 0ull) break;
    const int lead = __ffsll((unsigned long long)m) - 1;
    const int gsel = __shfl(ag, lead, 64);
    const bool mine = ag == gsel;
#pragma unroll
    for (int k = 0; k < kNSumB; ++k) {
      const double v = wave_sum(mine ? a[k] : 0.0);
      if ((int)(threadIdx.x & 63) == lead && v != 0.0) atomicAdd(target + gsel * 8 + k, v);
    }
    if (mine) {
#pragma unroll
      for (int k = 0; k < kNSumB; ++k) a[k] = 0.0;
      ag = -1;
    }
  }
}

// Traces photons [start, end) of one variant whose first photon is `off`, a
// whole photon per lane (consecutive lanes, consecutive binned photons).
// The lanes' sums stay in registers within the item; a lane whose next
// photon is of another group (an item across a group boundary) adds its
// sums directly.  Reached by the whole workgroup.  long_seen (uniform across the wave) records that some
// photon needs the adjoint's search pass; the kernel publishes it once per
// wave at its end, not once per photon on one contended address.
template <bool RECORD, int SH>
__device__ __forceinline__ void trace_item(const SceneView<float>& L, int64_t start, int64_t end, int64_t off,
                                           const RaysView<float>& R, const HitsView<float>& H, double* target,
                                           int& ag, double* a, bool& long_seen) {
  for (int64_t cur = start + threadIdx.x; cur < end; cur += blockDim.x) {
    float oa[3], da[3];
    R.load(cur, oa, da);
    int g = R.grp(cur);
    if ((unsigned)g >= (unsigned)L.n_groups) g = -1;
    PhotonState ps;
    photon_init(ps, V3<float>{oa[0], oa[1], oa[2]}, V3<float>{da[0], da[1], da[2]},
                R.id_base + (uint64_t)(R.src(cur) - off));
    uint4 rec = {kPathEnd, kPathEnd, kPathEnd, kPathEnd};   // path record, written once
    while (!ps.fate) {
      const int k = ps.k;
      const uint32_t code = photon_step<float, SH>(L, ps);
      if (H.path) {
        rec.x = k == 0 ? code : rec.x;
        rec.y = k == 1 ? code : rec.y;
        rec.z = k == 2 ? code : rec.z;
        rec.w = k == 3 ? code : rec.w;
      }
    }
    PhotonOut<float> r = photon_out<float>(ps);
    if (H.path) {
      const bool is_long = r.fate == FOCUSED && r.nev > kPathSlots;
      if (r.fate != FOCUSED) rec.x = kPathSkip;
      else if (is_long) rec.x = kPathLong;
      reinterpret_cast<uint4*>(H.path)[cur] = rec;
      // the batched adjoint replays records of up to kPathSlots - 1 events;
      // the rest are found again by its search pass, which the flag enables
      long_seen = long_seen || __ballot(r.fate == FOCUSED && r.nev >= kPathSlots) != 0ull;
    }
    if (RECORD) {
      const int64_t q = R.src(cur);
      if (H.fate) H.fate[q] = (uint8_t)r.fate;
      if (H.nev) H.nev[q] = (uint8_t)r.nev;
      if (H.last_vol) H.last_vol[q] = r.last_vol;
      if (H.x) { H.x[q] = r.pos.x; H.y[q] = r.pos.y; H.z[q] = r.pos.z; }
      if (H.ux) { H.ux[q] = r.dir.x; H.uy[q] = r.dir.y; H.uz[q] = r.dir.z; }
      if (H.opl) H.opl[q] = r.opl;
      if (H.hash) H.hash[q] = r.hash;
    }
    if (target && g >= 0) {
      if (ag >= 0 && g != ag) {
#pragma unroll
        for (int k = 0; k < kNSumB; ++k) {
          if (a[k] != 0.0) atomicAdd(target + ag * 8 + k, a[k]);
          a[k] = 0.0;
        }
      }
      ag = g;
      a[0] += 1.0;
      if (r.fate == FOCUSED) {
        double x = (double)r.pos.x, y = (double)r.pos.y;
        a[1] += 1.0; a[2] += x; a[3] += y; a[4] += x * x; a[5] += y * y;
        a[6] += (double)dabs(r.dir.z);
      }
    }
  }
}

// USE_LDS: the items of variants that fit the LDS reservation; otherwise the
// items of the others.  Per-variant state is re-derived from the variant
// table for every item rather than carried across items (only the staged
// variant and the lanes' sums are).  The LDS form is held to 3 waves per SIMD
// (<= 168 VGPRs); 4 measured slower.
// SH: the shape set compiled in (the union over the variants).
template <bool USE_LDS, bool RECORD, int SH>
__global__ void __launch_bounds__(kBlockB) __attribute__((amdgpu_waves_per_eu(USE_LDS ? 3 : 1, USE_LDS ? 3 : 8)))
k_trace_batch(const BatchVariant<float>* vars, const BatchItem* items, int n_items, uint32_t* queue,
              uint32_t blob_cap, RaysView<float> R, HitsView<float> H) {
  extern __shared__ __align__(16) char lds[];
  __shared__ int s_item;
  int staged_v = -1;   // variant whose tables are in LDS
  double a[kNSumB];
#pragma unroll
  for (int k = 0; k < kNSumB; ++k) a[k] = 0.0;
  int ag = -1;
  bool long_seen = false;
  uint32_t* counter = queue + (USE_LDS ? kQFwdLds : kQFwdGlobal);
  while (true) {
    const int item = next_item(counter, &s_item);
    const BatchItem it = item < n_items ? load_uniform(items + item) : BatchItem{0, 0, -1};
    if (item >= n_items) break;
    const BatchVariant<float> bv = load_uniform(vars + it.v);
    const SceneView<float> S = load_uniform(bv.S);
    if (fits_lds(S, blob_cap) != USE_LDS) continue;
    SceneView<float> L;
    if (USE_LDS) {
      lds_view(L, lds);
      if (it.v != staged_v) {
        stage_variant<float>(S, L, lds);
        staged_v = it.v;
        __syncthreads();
      } else {
        stage_variant_view<float>(S, L, lds);
      }
    }
    double* target = H.sums ? H.sums + (int64_t)bv.goff * 8 : nullptr;
    trace_item<RECORD, SH>(USE_LDS ? L : S, it.start, it.start + it.count, bv.off, R, H, target, ag, a,
                       long_seen);
    // a workgroup's next item is usually far along the bundle (another group
    // or variant): reduce the lanes' sums now, one atomic per wave and sum,
    // rather than per lane later on a few contended addresses
    if (target) wave_flush(target, ag, a);
    // a change of variant overwrites LDS: every wave must be done with it
    __syncthreads();
  }
  if (long_seen && __lane_id() == 0) atomicOr(queue + kQLongFlag, 1u);
}

// ------------------------------------------------------------------ launcher
static hipError_t cu_count(int& ncu) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  return hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
}

template <bool USE_LDS, bool RECORD, int SH>
static hipError_t trace_batch_k(const BatchView<float>& B, const RaysView<float>& R, const HitsView<float>& H,
                                int ncu, hipStream_t st) {
  const size_t shmem = USE_LDS ? B.blob_cap : 0;
  const int blk = B.block > 0 ? B.block : kBlockB;
  int per_cu = 0;
  hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_trace_batch<USE_LDS, RECORD, SH>, blk,
                                                              shmem);
  if (e != hipSuccess || per_cu < 1) per_cu = 1;
  const int blocks = std::max(1, std::min(B.n_items, ncu * per_cu));
  hipLaunchKernelGGL((k_trace_batch<USE_LDS, RECORD, SH>), dim3(blocks), dim3(blk), shmem, st, B.vars, B.items,
                     B.n_items, B.queue, B.blob_cap, R, H);
  return hipGetLastError();
}

template <bool RECORD, int SH>
static hipError_t trace_batch_s(const BatchView<float>& B, const RaysView<float>& R, const HitsView<float>& H,
                                int ncu, hipStream_t st) {
  hipError_t e = hipSuccess;
  if (B.blob_cap > 0) e = trace_batch_k<true, RECORD, SH>(B, R, H, ncu, st);
  if (e == hipSuccess) e = trace_batch_k<false, RECORD, SH>(B, R, H, ncu, st);
  return e;
}

template <bool RECORD>
static hipError_t trace_batch_r(const BatchView<float>& B, const RaysView<float>& R, const HitsView<float>& H,
                                int ncu, hipStream_t st) {
  if (B.shapes & ~kShapesNoCone) return trace_batch_s<RECORD, kShapesAll>(B, R, H, ncu, st);
  return trace_batch_s<RECORD, kShapesNoCone>(B, R, H, ncu, st);
}

hipError_t launch_trace_batch(const BatchView<float>& B, const RaysView<float>& R, const HitsView<float>& H,
                              hipStream_t st) {
  int ncu = 0;
  hipError_t e = cu_count(ncu);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_batch_reset, dim3(1), dim3(64), 0, st, B.queue, kQFwdLds, kQLongFlag - kQFwdLds + 1);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  const bool rec = H.fate || H.nev || H.last_vol || H.x || H.ux || H.opl || H.hash;
  return rec ? trace_batch_r<true>(B, R, H, ncu, st) : trace_batch_r<false>(B, R, H, ncu, st);
}

}  // namespace robast
