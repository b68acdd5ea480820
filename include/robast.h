/* robast.h -- C ABI of the MI355X non-sequential photon tracer.
 *
 * The interface follows the paper's statement of the problem (Okumura, Noda,
 * Rulten, ROBAST, ICRC 2015):
 *   - a scene is a set of volumes, each with an optical role -- lens, mirror,
 *     focal surface, or absorbing obscuration (§2.1) -- and a shape: plane,
 *     sphere cap, cylinder, box, aspheric disc, or a hexagonal cone whose wall
 *     profile is a Bezier curve (the Winston / Okumura cones, §2.2);
 *   - photons are given by position and momentum direction (§2.1);
 *   - the trace is non-sequential: no surface order is fixed in advance, so
 *     multiple reflections on segmented mirrors and inside concentrators
 *     arise by themselves (§1, §2.1, §3);
 *   - mirrors reflect (or absorb, by their reflectivity); lenses refract
 *     with Fresnel reflection and total internal reflection, and may absorb
 *     in their bulk (§2.1: refraction by lenses);
 *   - each photon leaves with an exit state: detected on a focal surface,
 *     absorbed, or escaped, plus its exit position and direction and its
 *     optical path (the arrival time of §3's timing-sensitive telescopes).
 * On top of the paper's forward trace the library returns the focal-plane
 * figures of §3 (spot RMS per field angle, cosine-weighted collection per
 * incidence angle, arrival-time spread) and their gradients with respect to
 * the scene's parameters, by reverse mode along each photon's fixed surface
 * sequence, and traces many scene variants (a design sweep, a spectrum of
 * wavelengths) in one batched launch.
 *
 * Conventions
 *   - Every function returns robast_status (0 = OK, < 0 = error) and never
 *     throws.  robast_last_error() gives a thread-local message.
 *   - Host pointers are marked [host]; device pointers [device].  The caller
 *     allocates and owns every ray, hit, sum and gradient buffer; the library
 *     never frees them.  A scene owns its device tables until
 *     robast_destroy_scene.
 *   - Calls that take a stream validate on the host, enqueue on that HIP
 *     stream (NULL = the null stream) and return without waiting.  A device
 *     fault surfaces at the caller's next synchronisation.
 *   - Floating-point ray/hit arrays are float (precision 32) or double
 *     (precision 64), matching the scene.
 */
#ifndef ROBAST_H
#define ROBAST_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  ROBAST_OK = 0,
  ROBAST_EINVAL = -1,       /* invalid argument; nothing was launched */
  ROBAST_ENOMEM = -2,       /* device allocation failed */
  ROBAST_EHIP = -3,         /* a HIP runtime call failed (message in robast_last_error) */
  ROBAST_EUNSUPPORTED = -4, /* valid request with no kernel for it */
  ROBAST_EMISMATCH = -5     /* inconsistent inputs (e.g. buffer sizes of two calls) */
} robast_status;

/* optical roles (§2.1) */
enum { ROBAST_MIRROR = 1, ROBAST_LENS = 2, ROBAST_FOCAL = 3, ROBAST_OBSCURATION = 4 };

/* shapes (§2.2).  Each face has a front side: plane / sphere / asphere front
 * is local +z; cylinder and box front is outside; cone walls front inside.
 *   PLANE    z_l = 0, bounded by the outline
 *   SPHERE   z_l = c r^2 / (1 + sqrt(1 - c^2 r^2)), p[0] = c = 1/R (signed)
 *   ASPHERE  z_l = sum_{i=1..8} b_i u^i, u = r^2/rn^2; p[0] = rn, p[1..8] = b_i
 *   CYLINDER x_l^2 + y_l^2 = p[0]^2, 0 <= z_l <= p[1] (lateral surface)
 *   BOX      |x_l| <= p[0], |y_l| <= p[1], |z_l| <= p[2]; six faces,
 *            face k = 2*axis + (negative side)
 *   HEXCONE  six walls k = 0..5 with outward direction n_k = (cos k60, sin k60):
 *            {rho(s) n_k + v m_k + z(s) e_z : 0<=s<=1, |v| <= rho(s)/sqrt(3)},
 *            (rho, z)(s) the cubic Bezier with control points
 *            p[0..7] = rho0 z0 rho1 z1 rho2 z2 rho3 z3                       */
enum { ROBAST_PLANE = 1, ROBAST_SPHERE = 2, ROBAST_ASPHERE = 3, ROBAST_CYLINDER = 4,
       ROBAST_BOX = 5, ROBAST_HEXCONE = 6 };

/* outlines of plane / sphere / asphere faces, on local (x, y):
 *   DISC r <= o[0];  ANNULUS o[0] <= r <= o[1];  RECT |x| <= o[0], |y| <= o[1];
 *   HEX |x cos a + y sin a| <= o[0] for a = 0, 60, 120 deg;
 *   SECTOR o[0] <= r <= o[1], o[2] <= phi <= o[3] (o[3] - o[2] <= 2 pi)       */
enum { ROBAST_OUTLINE_NONE = 0, ROBAST_DISC = 1, ROBAST_ANNULUS = 2, ROBAST_RECT = 3,
       ROBAST_HEX = 4, ROBAST_SECTOR = 5 };

/* photon fates */
enum { ROBAST_FOCUSED = 1, ROBAST_ABSORBED = 2, ROBAST_EXITED = 3, ROBAST_SUSPENDED = 4,
       ROBAST_FAILED = 5 };

/* One volume.  Local frame x_l = Q (x - c), Q row-major.  Differentiable
 * parameters: shape_param indexes the first of the shape's parameters in the
 * scene's parameter vector (SPHERE: radius R; ASPHERE: b_1..b_8; HEXCONE:
 * rho1 z1 rho2 z2), tilt_param the two tilt angles (alpha, beta) of a body
 * whose frame is the untilted (Q0, c0) rotated about `pivot` by
 * Rot(e2, beta) Rot(e1, alpha); -1 = none.  Layout: 6 int32 then 55 double
 * (464 bytes), identical to a packed C struct on x86-64. */
typedef struct {
  int32_t role, shape, outline, shape_param, tilt_param, flags;
  double Q[9], c[3];
  double p[16], o[4];
  double reflectivity; /* mirrors: absorb iff Philox word >= floor(R 2^32) */
  double n_inside;     /* lenses: refractive index on the back side of each face
                        * (inside a BOX), 1 on the front side.  A lens PLANE,
                        * SPHERE or ASPHERE is one refracting face of a solid
                        * that the caller closes with its other faces (e.g. an
                        * aspheric front, a plane back with its front side
                        * facing out, an absorbing CYLINDER rim); CYLINDER and
                        * HEXCONE lenses are EUNSUPPORTED.  p[15] of a lens
                        * volume: absorption length (m, >= 0; 0 = none) of
                        * the medium on its back side: a photon that reaches
                        * the face from that side after a segment of length
                        * t is absorbed iff its bulk draw (Philox tag 2, see
                        * robast_rays) w / 2^32 >= exp(-t / p[15]).
                        * p[13], p[14] of a lens volume: its dispersion law
                        * (see robast_rays.lambda; both 0 = none). */
  double Q0[9], c0[3], pivot[3], e1[3], e2[3];
} robast_volume_desc;

typedef struct {
  const robast_volume_desc* volumes; /* [host] n_volumes entries */
  int32_t n_volumes;                 /* 0 .. 65535 */
  int32_t precision;                 /* 32 (float) or 64 (double) */
  int32_t max_events;                /* 1 .. 255; photons still alive after it: SUSPENDED */
  int32_t n_groups;                  /* 1 .. 4096 photon groups (field angles) */
  uint64_t seed;                     /* Philox4x32-10 key */
  double l_ref;                      /* scene length scale (> 0), sets self-hit epsilons */
} robast_scene_desc;

/* Structure-of-arrays photon bundle.  Photon i has id id_base + i: its
 * random draws are Philox4x32-10 with key = seed and counter =
 * (id lo, id hi, event >> 2, tag), word event & 3, tag 1 for the draw of an
 * interaction and tag 2 for bulk absorption in a lens -- so a photon's result
 * never depends on launch shape or on which other photons share the launch. */
typedef struct {
  const void *ox, *oy, *oz, *dx, *dy, *dz; /* [device] n each, float or double; (dx, dy, dz)
                                            * a unit vector: a photon whose |d|^2 is off 1
                                            * by more than 1e-5 (or with a non-finite
                                            * coordinate) is not traced and ends FAILED */
  const uint32_t* group;                   /* [device] n, < n_groups; NULL = all group 0 */
  uint64_t id_base;
  const void* lambda;  /* [device] n wavelengths (metres, float or double), or NULL.  A
                        * lens volume whose descriptor gives a dispersion law
                        * (p[13] = A > 0, p[14] = B > 0: n = A + B / lambda^2)
                        * refracts each photon with its own n(lambda); without
                        * wavelengths, or for a lens without the law, n_inside.
                        * EUNSUPPORTED in batches and in scenes with HEXCONE
                        * volumes. */
} robast_rays;

/* Per-photon exit records; any pointer may be NULL (not written).
 * group_sums [device] n_groups * ROBAST_GROUP_STRIDE doubles, ACCUMULATED
 * (+=): per group {launched, focused, sum x, sum y, sum x^2, sum y^2,
 * sum |u_z|, 0} over FOCUSED photons (x, y world focal-surface coordinates,
 * u_z the exit direction's z component). */
#define ROBAST_GROUP_STRIDE 8
typedef struct {
  uint8_t* fate;     /* [device] n */
  uint8_t* n_events; /* [device] n, interactions including the terminal one */
  int32_t* last_vol; /* [device] n, volume of the last interaction or -1 */
  void *x, *y, *z;   /* [device] exit position (focal hit, absorption point, last point) */
  void *ux, *uy, *uz;/* [device] exit direction */
  void* opl;         /* [device] optical path length sum n_medium * segment */
  uint64_t* seq_hash;/* [device] hash of the (volume, face, side) sequence: h0 =
                        0xcbf29ce484222325, h = (h ^ (vol<<4 | face<<1 | back)) *
                        0x100000001b3 per interaction */
  double* group_sums;
  uint32_t* seq_log; /* [device] n * max_events event codes (vol << 8 | face << 4 |
                        action; action 0 reflect, 1 refract, 2 stop), photon i's
                        at [i * max_events, i * max_events + n_events[i]), the
                        rest untouched; robast_trace only (a debug log) */
} robast_hits;

/* Figures per group (§3: spot diagrams, collection efficiency), 8 doubles:
 * {launched, focused, centroid x, centroid y, RMS spot radius, efficiency
 *  focused/launched, weighted collection sum|u_z|/launched, 0}. */
#define ROBAST_FIGURE_STRIDE 8

typedef struct robast_scene robast_scene;

/* Validate the descriptors, compile the device tables (volume records, an XY
 * uniform grid with per-cell volume lists for the non-sequential candidate
 * search) and upload them.  `params` [host] n_params values of the
 * differentiable parameters (may be NULL if n_params == 0); every
 * shape_param/tilt_param index must lie inside it.  EINVAL on: NULL desc or
 * out, n_volumes out of range, unknown role / shape / outline, non-finite
 * values, non-positive sizes, a sphere whose aperture passes its equator,
 * precision not 32/64, max_events outside 1..255, n_groups outside 1..4096,
 * l_ref <= 0, a parameter index out of range.  Synchronous. */
int robast_build_scene(const robast_scene_desc* desc, const double* params, int64_t n_params,
                       robast_scene** out);

/* robast_trace flag: keep the binned photon order this call used (see
 * robast_tuning) for the next calls on the scene.  A kept order is used,
 * instead of binning again, by a trace or backward call given the same ray
 * pointers, id_base and n; the caller guarantees that the photon arrays were
 * not written in between.  It stays kept after a trace call with this flag
 * and is dropped by any other call that bins, by a backward call that used
 * it, by a parameter update and by the autotuner.
 * The call also records each photon's path (its surface sequence, when
 * FOCUSED with at most 4 events; 24 bytes per photon of scene-owned memory,
 * grown by hipMalloc like the binning workspace, n < 2^32).  The next
 * backward call, if it is the next call on the scene after this trace and is
 * given the same arrays, id_base and n, replays the recorded sequences
 * instead of searching for them again (longer sequences are still found by
 * a search).  Any other call drops the record: trace, bin, update, tuning,
 * autotune, and the backward call that used it. */
#define ROBAST_TRACE_KEEP_ORDER 1u

/* Trace photons [0, n).  rays/hits as above; n == 0 is a no-op.  EINVAL on
 * NULL scene/rays/hits, n < 0, a NULL ray coordinate array, an unknown flag
 * (flags: 0 or ROBAST_TRACE_KEEP_ORDER).
 * Calls on one scene (trace, backward, update) must not overlap in time:
 * they share the scene's photon counter and binning workspace, so issue them
 * on one stream or order them.  With binning on (robast_tuning), a call with
 * more photons than any before it on the scene grows the workspace
 * (hipMalloc, 72 bytes per photon in FP32, 136 in FP64): capture a call in a HIP graph only
 * after an eager call of at least the same size. */
int robast_trace(robast_scene* scene, const robast_rays* rays, int64_t n, const robast_hits* hits,
                 uint32_t flags, void* hip_stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the trace
 * of robast_trace with flags 0, whose photon binning (when the scene's
 * tuning bins photons and 32768 <= n <= 2^32 - 1) runs in a fixed 64 MiB
 * workspace in device memory that the library holds per GPU until the
 * process ends, instead of the scene's own growable one.  Calls no hipMalloc
 * or hipFree (the workspace's device address is looked up once per GPU, on
 * the first call there).  Results equal those of robast_trace.  Binning
 * needs 72 bytes per photon in FP32 (136 in FP64) plus per-bin counts:
 * EINVAL, before any launch, when that exceeds the workspace (about 9e5
 * FP32 photons) -- binning off (robast_set_tuning) lifts the limit.  Keeps
 * no binned order and no path records, and drops those of earlier calls on
 * the scene.  Every call on one GPU shares the workspace: calls that overlap
 * in time on one GPU (two streams) race.  Other errors as robast_trace. */
int robast_trace_static(robast_scene* scene, const robast_rays* rays, int64_t n, const robast_hits* hits,
                        void* hip_stream);

/* Figures from accumulated group sums (device -> device, n_groups * 8 doubles). */
int robast_figures(robast_scene* scene, const double* d_group_sums, double* d_figures,
                   void* hip_stream);

/* Arrival-time spread (isochronicity) per group, from the per-photon
 * records of a trace of photons [0, n): over the FOCUSED photons of group g
 * (rays->group, or group 0 when NULL), d_out[4 g .. 4 g + 3] = {count, mean
 * optical path length from the start point to the focal surface, RMS
 * spread of that length, 0} (FP64, metres; arrival time x c).  The optical
 * path is the one the trace records per photon (sum of n x distance over
 * the events; the paper's segmented-dish models, section on CTA
 * telescopes, differ in it: a parabolic dish is isochronous on axis, a
 * Davies-Cotton dish is not).  Reads hits->fate and hits->opl (the scene's
 * precision), indexed like the rays; d_out [device] n_groups * 4 doubles,
 * overwritten.  EINVAL on NULL scene, rays, hits, fate, opl or d_out, n < 0.
 * Two passes over the records (mean, then squared deviations). */
int robast_arrival_figures(robast_scene* scene, const robast_rays* rays, const robast_hits* hits, int64_t n,
                           double* d_out, void* hip_stream);

/* robast_trace_backward flag: debug check that the backward pass follows
 * the forward surface sequences.  Every photon is traced again by the
 * search (no path record replay) and its sequence hash compared with
 * fwd->seq_hash; the call then synchronises the stream and returns
 * ROBAST_EMISMATCH (gradient still accumulated) if any photon differs. */
#define ROBAST_BACKWARD_CHECK_SEQ 1u

/* Reverse mode along each photon's fixed surface sequence: the pathwise
 * gradient of the paper's focal-plane figures (§3: spot size of the
 * segmented telescopes, collection of the concentrators) with respect to
 * the scene parameters, each photon's fate and (volume, face) sequence held
 * fixed.  Sequences are re-derived with the same draws (so they equal the
 * forward ones) or read from the path record of the preceding
 * ROBAST_TRACE_KEEP_ORDER trace; the gradient is the same either way up to
 * FP64 summation order.  The objective is
 *   L = sum_g ( w_rms[g] RMS_g + w_eff[g] effw_g )
 *       + sum_{FOCUSED p} c_p . (x_p, y_p, z_p, ux_p, uy_p, uz_p)
 * with (x, y, z) a photon's focal-surface hit and u its exit direction.
 *   fwd          [device pointers] the forward records of the same photons:
 *                group_sums (needed with d_group_cot) and seq_hash (needed
 *                with ROBAST_BACKWARD_CHECK_SEQ); other fields unused; may
 *                be NULL when neither is needed
 *   d_group_cot  [device] n_groups * 2 doubles {w_rms, w_eff}, or NULL
 *   d_photon_cot [device] n * 6 doubles, c_p of photon p (caller's order),
 *                or NULL; photons that are not FOCUSED contribute nothing
 *   d_grad       [device] n_params doubles, ACCUMULATED (+=)
 *   flags        0 or ROBAST_BACKWARD_CHECK_SEQ
 * EINVAL on NULL scene / rays / grad, n < 0, an unknown flag, a group
 * cotangent without fwd->group_sums, the check without fwd->seq_hash;
 * EUNSUPPORTED when max_events > 64; EMISMATCH as described above. */
int robast_trace_backward(robast_scene* scene, const robast_rays* rays, int64_t n, const robast_hits* fwd,
                          const double* d_group_cot, const double* d_photon_cot, double* d_grad, uint32_t flags,
                          void* hip_stream);

/* Boundary (fate-flip) terms of the gradient of the collection efficiency
 * eta_g = N_FOCUSED,g / N_launched,g (§3: the concentrators' collection;
 * the count changes only through photons whose fate flips as the geometry
 * moves, so robast_trace_backward, which holds every fate fixed, gives it no
 * gradient).  Estimated by edge sampling: every event of a photon's path
 * that lies within band / 2 of an edge of its face -- a cone wall's seams
 * with its neighbours, its exit rim and its entrance rim, an exit
 * aperture's hexagon (focal surfaces with a hexagonal outline), and the
 * Fresnel decision at a lens face (distance R - u in probability) -- is
 * moved just across that edge and traced on with the same draws; where the
 * fate differs, the edge's flux (d delta / dp by a reverse sweep from that
 * event, plus the edge's own motion) is added.  Objective
 * L = sum_g cot[g] eta_g; the estimate is unbiased as band -> 0, its noise
 * grows as 1 / sqrt(N band).  Edges of other faces (telescope facet edges,
 * shadow edges) are not sampled.
 *   d_group_sums [device] the forward trace's group sums of the same photons
 *                (for N_launched,g)
 *   d_group_cot  [device] n_groups doubles cot[g]
 *   band         band width in (0, 1), in each edge's own distance units
 *                (fraction of the wall's lateral half-width at a seam, of
 *                the wall's parameter at its rims, of the aperture's
 *                inradius, of probability at a Fresnel decision)
 *   d_grad       [device] n_params doubles, ACCUMULATED (+=)
 * With binning on (robast_tuning) the photons are processed in binned
 * order: a kept order of the same arrays is reused and stays kept, else the
 * bundle is binned into the scene's workspace (allocated on first need) and
 * kept, and path records of an earlier order are dropped.  EINVAL on NULL
 * arguments, n < 0, band outside (0, 1); EUNSUPPORTED for per-photon
 * wavelengths or max_events > 32. */
int robast_boundary_grad(robast_scene* scene, const robast_rays* rays, int64_t n, const double* d_group_sums,
                         const double* d_group_cot, double band, double* d_grad, void* hip_stream);

/* Bin photons [0, n) now and keep the order, as a trace call with
 * ROBAST_TRACE_KEEP_ORDER would (a no-op when binning is off or n is outside
 * the binning range).  Lets a caller time the binning apart from the trace,
 * or bin once for a forward and a backward call.  EINVAL as robast_trace. */
int robast_bin_photons(robast_scene* scene, const robast_rays* rays, int64_t n, void* hip_stream);

/* ---- launch tuning ------------------------------------------------------
 * Per-scene launch parameters.  They change the order in which photons are
 * processed, never a photon's result (each photon keeps its id, draws and
 * search); group sums and gradients change only in FP64 summation order. */
typedef struct robast_tuning {
  /* nonzero: before each trace / backward call of at least 32768 photons
   * (and at most 2^32 - 1), order the photons by group and by the cell of a
   * square grid where their line crosses the scene's entrance plane (the
   * lowest z of its mirrors and lenses), by a counting sort into scene-owned
   * workspace, so that the photons of one wave take similar paths */
  uint32_t bin_photons;
  uint32_t bin_target;   /* photons per cell aimed at when sizing that grid, 1..65536 */
  uint32_t waves_mult;   /* workgroups launched per resident workgroup slot, 1..64 */
  uint32_t block;        /* threads per workgroup of the forward trace: 64, 128, 192 or 256
                            (0 reads as 256); each workgroup stages the scene's tables into
                            LDS once, so smaller workgroups stage more often */
  uint32_t bin_dirs;     /* azimuth sectors of the photon direction in the binning key: 1, 4,
                            16 or 64 (0 reads as 1).  Above 1, photons of a group are ordered
                            by the sector of atan2(dy, dx) first, then by cell (the grid then
                            has bin_dirs times fewer cells per sector, so a cell still aims at
                            bin_target photons): for bundles whose directions vary within a
                            group (a concentrator lit from all azimuths), where photons that
                            start together but leave in different directions diverge */
} robast_tuning;

/* Defaults: bin_photons 1, bin_target 128, waves_mult 4, block 256, bin_dirs 1. */
int robast_get_tuning(const robast_scene* scene, robast_tuning* out);
/* EINVAL on NULL arguments or a field out of range. */
int robast_set_tuning(robast_scene* scene, const robast_tuning* tuning);

/* Autotuner: traces photons [0, n) of `rays` (group sums only, into its own
 * scratch) under candidate tunings (binning off; binning with 32, 128 or 512
 * photons per cell; grid multiplier 1, 4 or 8; workgroups of 128 or 256
 * threads; then, with the best grid multiplier and workgroup size so far,
 * 4 or 16 direction sectors at 16, 32 or 128 photons per cell), times each with
 * HIP events on the stream, keeps the fastest in the scene and returns it in
 * *best (may be NULL).  Synchronous; allocates;
 * EINVAL as robast_trace or n < 1.  Iteration caps of the root solvers are
 * not tuned: they decide results, which no tuning may change. */
int robast_autotune(robast_scene* scene, const robast_rays* rays, int64_t n, robast_tuning* best,
                    void* hip_stream);

/* Gradient-descent steps on the device (a design optimised as in §3):
 * replace the differentiable parameters with d_params [device, n_params
 * doubles], in stream order, without the host.  A kernel rebuilds every
 * volume record (tilted frames, sphere curvature, asphere coefficients,
 * cone control points, their bounds) and the candidate groups' slabs into
 * the scene's second table slot and then switches the scene's device view
 * to it, so launches queued after it on the stream (and replays of a HIP
 * graph that captured it) trace the new geometry, while kernels still
 * running on the old slot are never given half-written tables.  The
 * candidate grid is kept: the update is applied only if no surface moves,
 * across its group's grid, by more than a quarter of the sampling step the
 * grid was built with (ample for optimisation steps; large changes need
 * robast_set_params).  *d_status [device, may be NULL] becomes 0 when the
 * update is applied, ROBAST_EINVAL when the new parameters make a surface
 * invalid (non-finite value, a sphere whose aperture reaches its equator,
 * a non-positive cone radius), ROBAST_EUNSUPPORTED when a surface would
 * leave its grid cells; in both cases the scene keeps its previous tables.
 * Updates on one scene must not overlap in time with other calls on it from
 * another stream.  Drops the kept binned order and path records.  EINVAL on
 * NULL scene or d_params (host-side, nothing launched). */
int robast_update_params(robast_scene* scene, const double* d_params, int32_t* d_status, void* hip_stream);

/* One gradient-descent step on the device (the optimisation of §3, with
 * the gradient of robast_trace_backward): the candidate parameters
 * p - lr * g (elementwise, FP64) are applied as by robast_update_params.
 *   d_params [device, n_params doubles] the current parameters p; where the
 *            update is applied they are overwritten with the new ones, else
 *            they keep their values (so they always describe the scene)
 *   d_grad   [device, n_params] the gradient g
 *   d_lr     [device, n_params] the step per parameter
 *   d_status [device, may be NULL] as for robast_update_params
 * Stream-ordered and graph-capturable (no host work, no allocation), so a
 * whole optimisation step -- trace, figures, backward, this step -- can be
 * replayed from one HIP graph.  EINVAL on NULL arguments. */
int robast_gd_step(robast_scene* scene, double* d_params, const double* d_grad, const double* d_lr,
                   int32_t* d_status, void* hip_stream);

/* Replace the differentiable parameters from the host [host, n_params] and
 * rebuild the scene's tables on the host, grid included (any change).  The
 * new geometry is checked first (the checks of robast_build_scene): EINVAL
 * and nothing changed on failure; EMISMATCH when n_params differs from the
 * build.  Synchronous: waits for the device to be idle before it rewrites
 * the tables.  The tables may grow: re-capture HIP graphs that launch on the
 * scene after this call. */
int robast_set_params(robast_scene* scene, const double* params, int64_t n_params);

void robast_destroy_scene(robast_scene* scene);

/* ---- batched design sweeps --------------------------------------------
 * Many design variants (scenes of one precision) traced in one persistent
 * launch (the event loop of §2.1 run over a parameter sweep of the kind used
 * for the designs of §3).  The photons of variant v are rays
 * [offsets[v], offsets[v+1]) of one concatenated bundle and are numbered from
 * offsets[v] (photon id = rays->id_base + index - offsets[v]), so every
 * photon's result equals that of robast_trace on variant v alone with the
 * same id_base.  The work is cut into items of at most `chunk` photons,
 * sorted by variant, which persistent workgroups pull from a device-side
 * counter; a workgroup stages a variant's tables into LDS only when its next
 * item belongs to another variant.
 * Concatenated layouts, in variant order: group sums n_groups_v * 8 doubles,
 * cotangents n_groups_v * 2, figures n_groups_v * 8, gradient n_params_v.
 * The work list is fixed at build time and the calls make no host-device
 * copies or allocations, so they can be captured in a HIP graph; parameter
 * updates of member scenes (robast_update_params, outside any capture) are
 * seen by later calls and replays.  The scenes must outlive the batch; a
 * scene may belong to several batches.  Calls on one batch that overlap in
 * time (two streams) race on its work counters.
 * Errors: EINVAL on NULL arguments, n_scenes < 1, offsets not
 * non-decreasing from 0, chunk == 0 or > 2^30, scenes of different precision;
 * EUNSUPPORTED for FP64 scenes (batches are built for FP32, the precision of
 * the sweeps); ENOMEM when the device tables cannot be allocated. */
typedef struct robast_batch robast_batch;

/* scenes: [host] n_scenes handles (a scene may appear more than once);
 * offsets: [host] n_scenes + 1 photon offsets, offsets[0] == 0;
 * chunk: photons per work item (a few thousand: large enough to amortise
 * the item fetch, small enough to balance the tail). */
int robast_build_batch(robast_scene* const* scenes, int32_t n_scenes, const int64_t* offsets, uint32_t chunk,
                       robast_batch** out);

/* Forward trace of the whole bundle: hits as for robast_trace, indexed by the
 * global photon index; hits->group_sums is the concatenated sums (+=).
 * Photon binning (per variant, within its range) follows the tuning of the
 * first scene at build time; its workspace (72 bytes per photon) is
 * allocated by robast_build_batch, so calls allocate nothing.  flags: 0 or
 * ROBAST_TRACE_KEEP_ORDER, with the meaning it has for robast_trace (the kept
 * order belongs to the batch). */
int robast_trace_batch(robast_batch* batch, const robast_rays* rays, const robast_hits* hits, uint32_t flags,
                       void* hip_stream);

/* Figures of every variant's groups from concatenated sums (as robast_figures). */
int robast_figures_batch(robast_batch* batch, const double* d_group_sums, double* d_figures, void* hip_stream);

/* Adjoint of the whole bundle (as robast_trace_backward per variant):
 * d_group_sums and d_cot concatenated, d_grad concatenated and accumulated
 * (+=).  EUNSUPPORTED when a variant has max_events > 32. */
int robast_trace_backward_batch(robast_batch* batch, const robast_rays* rays, const double* d_group_sums,
                                const double* d_cot, double* d_grad, void* hip_stream);

/* robast_update_params for every variant of the batch in one launch (one
 * workgroup per variant): d_params [device] the concatenated parameters,
 * d_status [device, n_scenes int32, may be NULL] one status per variant as
 * for robast_update_params.  Graph-capturable.  EUNSUPPORTED when a scene
 * appears more than once in the batch. */
int robast_update_params_batch(robast_batch* batch, const double* d_params, int32_t* d_status, void* hip_stream);

/* robast_gd_step for every variant of the batch in one launch: d_params,
 * d_grad and d_lr concatenated in variant order (n_params doubles each),
 * d_status [device, n_scenes int32, may be NULL].  Graph-capturable.
 * EINVAL on NULL arguments; EUNSUPPORTED when a scene appears more than once
 * in the batch. */
int robast_gd_step_batch(robast_batch* batch, double* d_params, const double* d_grad, const double* d_lr,
                         int32_t* d_status, void* hip_stream);

/* Autotuner of a batch's forward launch: traces the whole bundle (group
 * sums only, into its own scratch) with work items of 2048, 8192, 32768 or
 * 131072 photons and workgroups of 128 or 256 threads, times each with HIP
 * events, keeps the fastest in the batch (the work list is rebuilt for it)
 * and returns it in *best_chunk / *best_block (may be NULL).  Results do not
 * depend on either (only FP64 summation order does).  Synchronous;
 * allocates; re-capture graphs of the batch afterwards.  EINVAL as
 * robast_trace_batch. */
int robast_autotune_batch(robast_batch* batch, const robast_rays* rays, uint32_t* best_chunk, uint32_t* best_block,
                          void* hip_stream);

/* Totals of the concatenated layouts: photons, groups, parameters. */
int robast_batch_sizes(const robast_batch* batch, int64_t* n_photons, int64_t* n_groups, int64_t* n_params);

void robast_destroy_batch(robast_batch* batch);

const char* robast_status_string(int status);
const char* robast_last_error(void);
/* Version of this interface's layouts: 2 (robast_tuning has bin_dirs). */
int robast_abi_version(void);

#ifdef __cplusplus
}
#endif
#endif /* ROBAST_H */
