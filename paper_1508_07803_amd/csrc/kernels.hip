// Forward trace kernels and the figures kernel (gfx950, wave64).
//
// One lane traces one photon at a time, start to finish (the event loop of
// the non-sequential trace, §2.1), over a persistent grid-stride loop.  Each
// workgroup stages the scene blob (volume records + candidate grid) into LDS
// once and reuses it for every photon it traces.  Per-group figure sums are
// kept per lane in FP64 registers, flushed wave-synchronously into LDS when
// any lane's group changes, and added to global memory once per workgroup.
#include <hip/hip_runtime.h>

#include "device_trace.hpp"
#include "kernels.hpp"

namespace robast {

constexpr int kBlock = 256;
constexpr int kNSum = 7;  // launched, focused, x, y, x^2, y^2, |u_z|

// With USE_LDS the scene pointers are derived from the LDS array only, so the
// compiler addresses them as LDS (ds_read) rather than through flat loads.
template <typename T, bool USE_LDS>
__device__ __forceinline__ void stage_scene(const SceneView<T>& S, SceneView<T>& L, char* lds) {
  L = S;
  if (!USE_LDS) return;
  const uint4* src = reinterpret_cast<const uint4*>(S.blob);
  uint4* dst = reinterpret_cast<uint4*>(lds);
  uint32_t n16 = S.blob_bytes / 16u;
  for (uint32_t i = threadIdx.x; i < n16; i += blockDim.x) dst[i] = src[i];
  const char* base = S.blob;
  L.vol = reinterpret_cast<const DVol<T>*>(lds);
  L.always = reinterpret_cast<const uint16_t*>(lds + (reinterpret_cast<const char*>(S.always) - base));
  L.cell_start = reinterpret_cast<const uint32_t*>(lds + (reinterpret_cast<const char*>(S.cell_start) - base));
  L.items = reinterpret_cast<const uint16_t*>(lds + (reinterpret_cast<const char*>(S.items) - base));
  L.groups = reinterpret_cast<const GroupRec<T>*>(lds + (reinterpret_cast<const char*>(S.groups) - base));
}

__device__ __forceinline__ void flush_lane(double* acc_lds, int g, const double* a) {
  if (g < 0) return;
#pragma unroll
  for (int k = 0; k < kNSum; ++k)
    if (a[k] != 0.0) atomicAdd(acc_lds + g * 8 + k, a[k]);
}

// Per-photon results of a finished photon: its records (RECORD), its path
// record, and its share of the group sums, added to the lane's running sums
// (flushed when the lane moves on to another group).
template <typename T, bool RECORD, bool SUMS>
__device__ __forceinline__ void finish_photon(const RaysView<T>& R, const HitsView<T>& H, int64_t cur, int g,
                                              const PhotonState& ps, uint4 rec, double* a, int& ag,
                                              double* acc_target) {
  PhotonOut<T> r = photon_out<T>(ps);
  if (H.path) {
    if (r.fate != FOCUSED) rec.x = kPathSkip;
    else if (r.nev > kPathSlots) rec.x = kPathLong;
    reinterpret_cast<uint4*>(H.path)[cur] = rec;
  }
  if (RECORD) {
    const int64_t o = R.src(cur);
    if (H.fate) H.fate[o] = (uint8_t)r.fate;
    if (H.nev) H.nev[o] = (uint8_t)r.nev;
    if (H.last_vol) H.last_vol[o] = r.last_vol;
    if (H.x) { H.x[o] = r.pos.x; H.y[o] = r.pos.y; H.z[o] = r.pos.z; }
    if (H.ux) { H.ux[o] = r.dir.x; H.uy[o] = r.dir.y; H.uz[o] = r.dir.z; }
    if (H.opl) H.opl[o] = r.opl;
    if (H.hash) H.hash[o] = r.hash;
  }
  if (SUMS && g >= 0) {
    if (g != ag && ag >= 0) {
      flush_lane(acc_target, ag, a);
#pragma unroll
      for (int k = 0; k < kNSum; ++k) a[k] = 0.0;
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

// One interaction of the lane's photon, logged (seq_log) and kept in the
// photon's path record (its first kPathSlots event codes).
template <typename T, bool RECORD, int SH>
__device__ __forceinline__ void step_photon(const SceneView<T>& L, const RaysView<T>& R, const HitsView<T>& H,
                                            int64_t cur, PhotonState& ps, uint4& rec) {
  const int k = ps.k;
  const uint32_t code = photon_step<T, SH>(L, ps);
  if (RECORD && H.seq_log && code != 0xffffffffu) H.seq_log[R.src(cur) * L.max_events + k] = code;
  if (H.path) {
    rec.x = k == 0 ? code : rec.x;
    rec.y = k == 1 ? code : rec.y;
    rec.z = k == 2 ? code : rec.z;
    rec.w = k == 3 ? code : rec.w;
  }
}

template <typename T>
__device__ __forceinline__ int start_photon(const SceneView<T>& L, const RaysView<T>& R, int64_t cur,
                                            PhotonState& ps, uint4& rec) {
  T oa[3], da[3];
  R.load(cur, oa, da);
  int g = R.grp(cur);
  if ((unsigned)g >= (unsigned)L.n_groups) g = -1;
  photon_init(ps, V3<T>{oa[0], oa[1], oa[2]}, V3<T>{da[0], da[1], da[2]}, R.id_base + (uint64_t)R.src(cur), 0.0);
  rec = uint4{kPathEnd, kPathEnd, kPathEnd, kPathEnd};
  return g;
}

// FP32 kernels are held to 4 waves per SIMD (<= 128 VGPRs, a few spills):
// measured faster than the 3 waves the unconstrained allocation gives, as
// the extra wave hides LDS and memory latency of the search.
// SH: the shape set compiled in (kShapesMirrors for scenes of mirrors and
// focal surfaces only, kShapesNoCone for other scenes without hex cones,
// else kShapesAll).
template <typename T, bool RECORD, bool SUMS, bool USE_LDS, int SH>
__global__ void __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 ? 4 : 1, 8))) k_trace(const SceneView<T>* Sp, RaysView<T> R, int64_t n, HitsView<T> H,
                                                  int sums_in_lds) {
  extern __shared__ __align__(16) char lds[];
  const SceneView<T> S = *Sp;
  SceneView<T> L;
  stage_scene<T, USE_LDS>(S, L, lds);
  double* acc = reinterpret_cast<double*>(lds + (USE_LDS ? ((S.blob_bytes + 15u) & ~15u) : 0u));
  if (SUMS && sums_in_lds) {
    for (int i = threadIdx.x; i < S.n_groups * 8; i += blockDim.x) acc[i] = 0.0;
  }
  __syncthreads();

  double a[kNSum];
#pragma unroll
  for (int k = 0; k < kNSum; ++k) a[k] = 0.0;
  int ag = -1;
  double* acc_target = (SUMS && sums_in_lds) ? acc : H.sums;

  // One lane traces one photon start to finish (the event loop, §2.1), over
  // a persistent grid-stride walk of the (binned) bundle: consecutive lanes
  // take consecutive photons, which binning makes spatially close, so a
  // wave's photons follow similar paths event by event.  (Handing a lane the
  // wave's next photon as soon as its own ends was measured slower, on the
  // telescopes and on the many-bounce concentrator alike: lanes then sit at
  // different events of their photons and diverge within each event.)
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t cur = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; cur < n; cur += stride) {
    PhotonState ps;
    uint4 rec;
    const int g = start_photon<T>(L, R, cur, ps, rec);
    ps.lam = R.template wavelength<SH>(cur);
    while (!ps.fate) step_photon<T, RECORD, SH>(L, R, H, cur, ps, rec);
    finish_photon<T, RECORD, SUMS>(R, H, cur, g, ps, rec, a, ag, acc_target);
  }
  if (SUMS) {
    flush_lane(acc_target, ag, a);
    if (sums_in_lds) {
      __syncthreads();
      for (int i = threadIdx.x; i < S.n_groups * 8; i += blockDim.x)
        if (acc[i] != 0.0) atomicAdd(H.sums + i, acc[i]);
    }
  }
}

// Figures per group from the accumulated sums (§3: spot RMS, efficiency).
__global__ void k_figures(const double* sums, double* fig, int n_groups) {
  int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= n_groups) return;
  const double* s = sums + g * 8;
  double nl = s[0], nf = s[1];
  double cx = nf > 0 ? s[2] / nf : 0.0, cy = nf > 0 ? s[3] / nf : 0.0;
  double var = nf > 0 ? (s[4] / nf - cx * cx) + (s[5] / nf - cy * cy) : 0.0;
  double* f = fig + g * 8;
  f[0] = nl; f[1] = nf; f[2] = cx; f[3] = cy;
  f[4] = var > 0 ? sqrt(var) : 0.0;
  f[5] = nl > 0 ? nf / nl : 0.0;
  f[6] = nl > 0 ? s[6] / nl : 0.0;
  f[7] = 0.0;
}

// Arrival-time spread (isochronicity) of the FOCUSED photons of each group
// from the per-photon records, in two passes over them: PASS 0 sums the
// count and the optical path lengths, PASS 1 the squared deviations from
// the group's mean (kept apart so that a spread of millimetres over paths
// of tens of metres is not lost to cancellation).  Each lane sums the
// photons it visits for one group at a time and adds them to LDS when its
// group changes; LDS is added to out once per workgroup.
template <typename T, int PASS>
__global__ void __launch_bounds__(kBlock) k_arrival(const uint8_t* fate, const T* opl, const uint32_t* group,
                                                    int64_t n, int n_groups, double* out, int in_lds) {
  extern __shared__ __align__(16) char lds[];
  double* acc = reinterpret_cast<double*>(lds);
  if (in_lds)
    for (int i = threadIdx.x; i < 2 * n_groups; i += blockDim.x) acc[i] = 0.0;
  __syncthreads();
  double* target = in_lds ? acc : nullptr;
  int ag = -1;
  double c = 0.0, v = 0.0;
  auto flush = [&]() {
    if (ag < 0) return;
    if (in_lds) {
      if (PASS == 0) atomicAdd(target + 2 * ag, c);
      atomicAdd(target + 2 * ag + 1, v);
    } else {
      if (PASS == 0) atomicAdd(out + 4 * ag, c);
      atomicAdd(out + 4 * ag + 1 + PASS, v);
    }
    c = 0.0;
    v = 0.0;
  };
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    if (fate[i] != FOCUSED) continue;
    const int g = group ? (int)group[i] : 0;
    if (g < 0 || g >= n_groups) continue;
    if (g != ag) {
      flush();
      ag = g;
    }
    const double p = (double)opl[i];
    if (PASS == 0) {
      c += 1.0;
      v += p;
    } else {
      const double dv = p - out[4 * g + 1];
      v += dv * dv;
    }
  }
  flush();
  if (in_lds) {
    __syncthreads();
    for (int i = threadIdx.x; i < 2 * n_groups; i += blockDim.x) {
      const int g = i >> 1, k = i & 1;
      if (acc[i] == 0.0) continue;
      if (k == 0 && PASS == 0) atomicAdd(out + 4 * g, acc[i]);
      if (k == 1) atomicAdd(out + 4 * g + 1 + PASS, acc[i]);
    }
  }
}

// Clears out (a kernel, so that a captured graph can replay it), or turns
// the pass sums into the mean (PASS 0) and the RMS spread (PASS 1).
template <int PASS>
__global__ void k_arrival_step(double* out, int n_groups) {
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= n_groups) return;
  double* o = out + 4 * g;
  if (PASS < 0) {
    o[0] = o[1] = o[2] = o[3] = 0.0;
  } else if (PASS == 0) {
    o[1] = o[0] > 0.0 ? o[1] / o[0] : 0.0;
  } else {
    o[2] = o[0] > 0.0 ? sqrt(o[2] / o[0]) : 0.0;
  }
}

// ------------------------------------------------------------------ launchers
static int g_num_cu = 0;

static hipError_t device_cus(int& ncu) {
  if (g_num_cu == 0) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    e = hipDeviceGetAttribute(&g_num_cu, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return e;
  }
  ncu = g_num_cu;
  return hipSuccess;
}

template <typename T, bool RECORD, bool SUMS, bool USE_LDS, int SH>
static hipError_t launch_one_s(const SceneView<T>& S, const RaysView<T>& R, int64_t n, const HitsView<T>& H,
                               const LaunchCfg& cfg, hipStream_t st) {
  int ncu = 0;
  hipError_t e = device_cus(ncu);
  if (e != hipSuccess) return e;
  const bool use_lds = USE_LDS;
  size_t sums_bytes = (size_t)S.n_groups * 8 * sizeof(double);
  bool sums_lds = SUMS && sums_bytes <= 16384;
  size_t shmem = (use_lds ? ((S.blob_bytes + 15u) & ~15u) : 0u) + (sums_lds ? sums_bytes : 0);
  const int blk = cfg.block > 0 ? cfg.block : kBlock;
  int per_cu = 0;
  e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_trace<T, RECORD, SUMS, USE_LDS, SH>, blk, shmem);
  if (e != hipSuccess || per_cu < 1) per_cu = 1;
  int64_t want = (n + blk - 1) / blk;
  int64_t cap = (int64_t)ncu * per_cu * (cfg.waves_mult > 0 ? cfg.waves_mult : 1);
  if (cfg.max_blocks > 0) cap = std::min<int64_t>(cap, cfg.max_blocks);
  int blocks = (int)std::max<int64_t>(1, std::min(want, cap));
  hipLaunchKernelGGL((k_trace<T, RECORD, SUMS, USE_LDS, SH>), dim3(blocks), dim3(blk), shmem, st, S.self, R, n, H,
                     sums_lds ? 1 : 0);
  return hipGetLastError();
}

template <typename T, bool RECORD, bool SUMS, bool USE_LDS>
static hipError_t launch_one_l(const SceneView<T>& S, const RaysView<T>& R, int64_t n, const HitsView<T>& H,
                               const LaunchCfg& cfg, hipStream_t st) {
  // wavelengths matter only for dispersive lenses (the caller rejects them
  // for scenes with cones)
  if (R.lam && S.dispersive)
    return launch_one_s<T, RECORD, SUMS, USE_LDS, kShapesNoCone | kLambda>(S, R, n, H, cfg, st);
  if (S.shapes & ~kShapesNoCone) return launch_one_s<T, RECORD, SUMS, USE_LDS, kShapesAll>(S, R, n, H, cfg, st);
  if (!(S.shapes & ~kShapesMirrors)) return launch_one_s<T, RECORD, SUMS, USE_LDS, kShapesMirrors>(S, R, n, H, cfg, st);
  return launch_one_s<T, RECORD, SUMS, USE_LDS, kShapesNoCone>(S, R, n, H, cfg, st);
}

template <typename T, bool RECORD, bool SUMS>
static hipError_t launch_one(const SceneView<T>& S, const RaysView<T>& R, int64_t n, const HitsView<T>& H,
                             const LaunchCfg& cfg, hipStream_t st) {
  bool use_lds = cfg.lds_cap > 0 && S.blob_bytes <= (uint32_t)cfg.lds_cap;
  if (use_lds) return launch_one_l<T, RECORD, SUMS, true>(S, R, n, H, cfg, st);
  return launch_one_l<T, RECORD, SUMS, false>(S, R, n, H, cfg, st);
}

template <typename T>
hipError_t launch_trace(const SceneView<T>& S, const RaysView<T>& R, int64_t n, const HitsView<T>& H,
                        const LaunchCfg& cfg, hipStream_t st) {
  bool rec = H.fate || H.nev || H.last_vol || H.x || H.ux || H.opl || H.hash || H.seq_log;
  bool sums = H.sums != nullptr;
  if (rec && sums) return launch_one<T, true, true>(S, R, n, H, cfg, st);
  if (rec) return launch_one<T, true, false>(S, R, n, H, cfg, st);
  if (sums) return launch_one<T, false, true>(S, R, n, H, cfg, st);
  return launch_one<T, true, false>(S, R, n, H, cfg, st);
}

hipError_t launch_figures(const double* sums, double* fig, int n_groups, hipStream_t st) {
  hipLaunchKernelGGL(k_figures, dim3((n_groups + 63) / 64), dim3(64), 0, st, sums, fig, n_groups);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_arrival(const uint8_t* fate, const T* opl, const uint32_t* group, int64_t n, int n_groups,
                          double* out, hipStream_t st) {
  int ncu = 0;
  hipError_t e = device_cus(ncu);
  if (e != hipSuccess) return e;
  const size_t lds = (size_t)n_groups * 2 * sizeof(double);
  const int in_lds = lds <= 16384 ? 1 : 0;
  const int blocks = (int)std::max<int64_t>(1, std::min<int64_t>((n + kBlock - 1) / kBlock, (int64_t)ncu * 8));
  const dim3 gsteps((n_groups + 63) / 64);
  hipLaunchKernelGGL(k_arrival_step<-1>, gsteps, dim3(64), 0, st, out, n_groups);
  hipLaunchKernelGGL((k_arrival<T, 0>), dim3(blocks), dim3(kBlock), in_lds ? lds : 0, st, fate, opl, group, n,
                     n_groups, out, in_lds);
  hipLaunchKernelGGL(k_arrival_step<0>, gsteps, dim3(64), 0, st, out, n_groups);
  hipLaunchKernelGGL((k_arrival<T, 1>), dim3(blocks), dim3(kBlock), in_lds ? lds : 0, st, fate, opl, group, n,
                     n_groups, out, in_lds);
  hipLaunchKernelGGL(k_arrival_step<1>, gsteps, dim3(64), 0, st, out, n_groups);
  return hipGetLastError();
}

template hipError_t launch_arrival<float>(const uint8_t*, const float*, const uint32_t*, int64_t, int, double*,
                                          hipStream_t);
template hipError_t launch_arrival<double>(const uint8_t*, const double*, const uint32_t*, int64_t, int, double*,
                                           hipStream_t);

template hipError_t launch_trace<float>(const SceneView<float>&, const RaysView<float>&, int64_t,
                                        const HitsView<float>&, const LaunchCfg&, hipStream_t);
template hipError_t launch_trace<double>(const SceneView<double>&, const RaysView<double>&, int64_t,
                                         const HitsView<double>&, const LaunchCfg&, hipStream_t);

}  // namespace robast
