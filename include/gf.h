/*
 * gf.h -- C ABI of libgf.so: SU(3) and SU(2) lattice gauge fixing on AMD
 * Instinct MI355X (gfx950) by checkerboard overrelaxation and simulated
 * annealing.
 *
 * Method: M. Schroeck and H. Vogt, "Coulomb, Landau and Maximally Abelian
 * Gauge Fixing in Lattice QCD with Multi-GPUs", arXiv:1212.5221.
 *   - gauge functionals F and precisions theta: Sec. 2.1;
 *   - local updates (relaxation, overrelaxation, microcanonical, stochastic
 *     relaxation): Sec. 2.2, App. A;
 *   - simulated annealing with heatbath updates: Sec. 2.3;
 *   - the even/odd sweep, Alg. 1: Sec. 2.4;
 *   - 12-real compression and reprojection: Sec. 4.2, Sec. 4.5.
 *
 * Conventions
 *   - Every function returns a status: GF_OK (0), a warning (> 0) or an error
 *     (< 0).  No exception crosses the ABI.  gf_last_error() describes the
 *     last non-OK status of a handle.
 *   - A handle belongs to one host thread at a time.  All device work is
 *     enqueued on the handle's HIP stream; host outputs are valid when the
 *     call returns.
 *   - The library never allocates device memory: the caller allocates one
 *     workspace (gf_workspace_size / gf_bind_workspace) and owns it.
 *   - Links exchanged with the caller are in the natural order (Sec. 4.2.1,
 *     "StandardPattern"): t, x, y, z, mu, i, j, re/im with z fastest, 18
 *     doubles per link (gauge group SU(2): 8), mu = 0 the time direction.
 *     Boundaries are periodic.
 *   - Common errors: a NULL handle or a NULL required pointer (the outputs of
 *     gf_measure, gf_measure_timeslices, gf_unitarity, gf_autotune and
 *     gf_sweep's sweeps_done may be NULL and are then not written), an
 *     instance number out of range or a value outside its documented range
 *     gives GF_E_INVALID;
 *     a call that needs a bound workspace before gf_bind_workspace, or a
 *     configuration call after it, gives GF_E_STATE; a failing HIP call
 *     gives GF_E_HIP with the runtime's message.  Host pointers passed in
 *     are only read or written during the call; the library keeps none.
 */
#ifndef GF_H
#define GF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct gf_ctx *gf_handle;

/* status codes */
#define GF_OK 0
#define GF_NOT_CONVERGED 1 /* some instance or time-slice hit max_sweeps */
#define GF_E_INVALID (-1)  /* bad argument (null pointer, value out of range) */
#define GF_E_DIMS (-2)     /* lattice extent odd, < 2, or too large */
#define GF_E_STATE (-3)    /* call not allowed in the current state */
#define GF_E_HIP (-4)      /* a HIP runtime error; the message names it */
#define GF_E_NOMEM (-5)    /* workspace too small or misaligned */
#define GF_E_NONFINITE (-6) /* F or theta is not finite */

/* gauges (Sec. 2.1) */
#define GF_LANDAU 0
#define GF_COULOMB 1
#define GF_MAG 2

/* update types (Sec. 2.2, 2.3) */
#define GF_OR 0       /* overrelaxation g -> g^omega to first order; omega = 1 is relaxation */
#define GF_MICRO 1    /* microcanonical step, g -> g^2 */
#define GF_ANNEAL 2   /* the annealing schedule of gf_set_anneal */
#define GF_SR 3       /* stochastic relaxation: g^2 with probability p, else g */
#define GF_HEATBATH 4 /* heatbath sweeps at the fixed temperature of gf_set_temperature */

/* link storage on the device (Sec. 4.2) */
#define GF_F64_R18 0       /* double, all 18 reals */
#define GF_F64_R12 1       /* double, first two rows; third row = (u x v)^* */
#define GF_MIXED_F32_R12 2 /* float, first two rows; G applied, reductions and reprojection in FP64 */
#define GF_F32_R12 3       /* float, first two rows; all arithmetic of the sweep in FP32, reductions and
                              reprojection in FP64 (the single precision of Sec. 4.5) */

/* gf_download flags */
#define GF_DL_REUNITARISE 1 /* reproject every link to SU(3) (SU(2)) in FP64 while converting */

/* Create a handle on HIP device `hip_device`.  `hip_stream` is a hipStream_t
   of that device (for example torch.cuda.current_stream().cuda_stream);
   NULL means the default stream.  *out receives the handle. */
int gf_create(gf_handle *out, int hip_device, void *hip_stream);

/* Destroy a handle.  Frees host state only; the workspace stays the caller's. */
void gf_destroy(gf_handle h);

/* Message of the last non-OK status on `h` (or, when h is NULL, of the
   calling thread's last failed gf_create or gf_measure_noalloc); valid until
   the next call on that handle (that thread). */
const char *gf_last_error(gf_handle h);

/* Add a lattice instance of extents dims = {Nt, Nx, Ny, Nz}.  Every extent
   must be even and >= 2 (checkerboard with periodic boundaries) and the
   instance below 2^29 sites (half-site indices fit 28 bits); otherwise
   GF_E_DIMS.  *inst receives the instance number (0, 1, ...).  Only before
   gf_bind_workspace.  Instances are independent problems (Gribov copies,
   uneven lattices) swept together with per-instance stopping. */
int gf_add_instance(gf_handle h, const int32_t dims[4], int32_t *inst);

/* Gauge for all instances (Sec. 2.1): GF_LANDAU, GF_COULOMB or GF_MAG.
   Coulomb gauge treats every time-slice as its own problem with its own
   stopping (Sec. 2.1.1) and applies the accumulated transformation to the
   temporal links at the end of each gf_sweep (Sec. 5).  Only before binding. */
int gf_set_gauge(gf_handle h, int gauge);

/* Gauge group SU(nc), nc = 3 (default) or 2 (else GF_E_INVALID).  For SU(2)
   the local update acts on the whole group (Sec. 2.2.1 eq. localsolution,
   Sec. 2.2.2 eq. upMatrix) instead of iterating over subgroups, links are
   exchanged as 2x2 complex matrices (8 doubles, natural order) and stored
   as their 4 Cayley-Klein components [[u0 + i u3, u2 + i u1],
   [-u2 + i u1, u0 - i u3]], read from the first row on upload; F and theta
   are normalised with N_c = 2 (Sec. 2.1).  Storages for SU(2): GF_F64_R18
   and GF_F64_R12 both mean the 4 components in FP64; GF_MIXED_F32_R12 keeps
   them in FP32 with the same precision policy as for SU(3) (g normalised
   and applied in FP64, optional FP64 tail); GF_F32_R12 keeps them in FP32
   and applies g in FP32 too (single precision).  Every gauge and update
   type is available; one wavefront per site group.  Only before binding. */
int gf_set_group(gf_handle h, int nc);

/* Storage (GF_F64_R18, GF_F64_R12, GF_MIXED_F32_R12, GF_F32_R12), reprojection interval
   (inside gf_sweep, reproject the links of every unit still running after
   every `reunit_every` sweeps; 0 = never, Sec. 4.5) and, for mixed storage,
   the threshold below which the local update is computed in FP64 instead of
   FP32 (the "final iterations" of a run): compute in FP64 once the last
   measured theta of a unit is below `fp64_tail_theta` (0 = never, >= 1e300 =
   always; mixed storage only).  Mixed storage always applies the product G of a site's three
   subgroup elements to its links in FP64, after reprojecting a G built in
   FP32 to SU(3), and rounds the result to FP32.  Heatbath sweeps on FP32
   storage (SU(3)) compute the local algebra in FP32 and draw the sample in
   FP64 (FP64 throughout with fp64_tail_theta >= 1e300); stochastic
   relaxation computes in FP64.  12-real storages store a
   left-multiplied link after one first-order renormalisation of its two rows
   (without it, rebuilding the third row lets their norm defect grow under
   large updates).  With FP32 storage (GF_MIXED_F32_R12, GF_F32_R12) and
   reunit_every > 0, gf_sweep delivers reprojected links: a unit stops only
   on a check of links reprojected in FP64 (see gf_sweep).  Only before
   binding. */
int gf_set_precision(gf_handle h, int storage, int32_t reunit_every, double fp64_tail_theta);

/* Bytes of device workspace the bound configuration needs. */
int gf_workspace_size(gf_handle h, size_t *bytes);

/* Bind the caller's device workspace: 256-byte aligned, at least
   gf_workspace_size bytes (else GF_E_NOMEM).  After binding no instance,
   gauge or precision can change.  The workspace holds the links in the
   library's internal layout; its previous contents are ignored. */
int gf_bind_workspace(gf_handle h, void *dev_ptr, size_t bytes);

/* Copy time-slices [t0, t0+nt) of instance `inst` from `links` (natural
   layout, nt*Nx*Ny*Nz*4*18 doubles, SU(2): *8) into the device storage,
   converting precision and dropping the third row for 12-real storage (the
   second row for SU(2)).  on_device != 0:
   `links` is a device pointer, else a host pointer (staged through the
   workspace).  Enqueued on the handle's stream; returns after the copy. */
int gf_upload(gf_handle h, int32_t inst, const double *links, int32_t t0, int32_t nt, int on_device);

/* The inverse of gf_upload (the third row reconstructed in FP64 for 12-real
   storage).  flags: GF_DL_REUNITARISE to reproject in FP64 while converting. */
int gf_download(gf_handle h, int32_t inst, double *links, int32_t t0, int32_t nt, int on_device, int flags);

/* Overrelaxation parameter omega in [1, 2) (Sec. 2.2.3); 1 = relaxation. */
int gf_set_overrelax(gf_handle h, double omega);

/* Probability p in [0, 1] of the microcanonical step in stochastic
   relaxation (Sec. 2.2.5). */
int gf_set_stochastic(gf_handle h, double p);

/* Seed of the random streams of GF_HEATBATH, GF_SR and GF_ANNEAL sweeps
   (Philox4x64-10 keyed by (seed, instance)); default 0. */
int gf_set_seed(gf_handle h, uint64_t seed);

/* Fixed heatbath temperature T > 0 for GF_HEATBATH sweeps (Sec. 2.3). */
int gf_set_temperature(gf_handle h, double T);

/* Annealing schedule for GF_ANNEAL (Sec. 2.3): for k = 0..nsteps-1,
   T_k = T0 + (T1 - T0) k / (nsteps - 1); one heatbath sweep at T_k followed
   by nmicro microcanonical sweeps.  `seed` keys the random streams
   (Philox4x64-10 keyed by (seed, instance), counter (sweep index, site,
   subgroup, draw)).  T0, T1 > 0, nsteps >= 1, nmicro >= 0. */
int gf_set_anneal(gf_handle h, double T0, double T1, int32_t nsteps, int32_t nmicro, uint64_t seed);

/* Run Alg. 1 with update `update`.
   GF_OR, GF_MICRO, GF_SR, GF_HEATBATH: measure theta on the input and after
   every `check_every` sweeps; a unit (instance; Coulomb: time-slice) stops
   at the first check with theta < theta_tol; stop when every unit stopped
   (GF_OK) or after max_sweeps sweeps (GF_NOT_CONVERGED).
   FP32 storage with reunit_every > 0 (Sec. 4.5): once every unit has
   stopped, the links (and the Coulomb accumulator) of every unit are
   reprojected to SU(3) in FP64 and rounded back to FP32, and theta is
   measured again; units whose theta is no longer below theta_tol run on in
   chunks of check_every sweeps (within max_sweeps) until a check passes,
   and are then reprojected and checked again.  So the delivered links are
   reprojected and satisfy theta < theta_tol.
   Coulomb: the U_0 fix-up follows at the end.  Stopped units are neither
   swept nor reprojected by the periodic reprojection: a unit keeps the
   links its stopping check measured.  Later checks read only the units
   still running (a stopped unit's F and theta stay those of its stopping
   check), with cache groups (gf_set_cache_budget) a group whose units
   have all stopped is no longer launched, and a launch in which only some
   units work runs in the linear tile order (the working tiles spread over
   all XCDs) whatever the shape's tile order.
   GF_ANNEAL: run the schedule of gf_set_anneal (no stopping; max_sweeps,
   theta_tol, check_every ignored).
   sweeps_done (host, may be NULL): per instance (Landau/MAG) or per
   instance and time-slice, instance-major (Coulomb), the sweeps each unit ran.
   Synchronises the stream before returning. */
int gf_sweep(gf_handle h, int update, int32_t max_sweeps, double theta_tol, int32_t check_every,
             int32_t *sweeps_done);

/* One half-sweep (the sites of one parity of every instance) without any
   check: for tests of single updates.  parity: 0 even, 1 odd (Coulomb: the
   3D parity inside each time-slice).  Uses the global sweep index as the
   random counter and does not advance it. */
int gf_halfsweep(gf_handle h, int update, int parity);

/* F and theta of instance `inst` (Sec. 2.1) reduced in FP64 at the current
   state, normalised with the N_c of the gauge group (3 or 2); MAG: F is the
   practical form (1/(N_c N_d V)) sum |U_ii|^2.  Coulomb: averages over the
   time-slices.  GF_E_NONFINITE if either is not finite. */
int gf_measure(gf_handle h, int32_t inst, double *F, double *theta);

/* Coulomb: per time-slice F_t, theta_t (Nt values each). */
int gf_measure_timeslices(gf_handle h, int32_t inst, double *F_t, double *theta_t);

/* For callers that cannot allocate device memory (code under HIP graph
   capture, tight serving loops, harnesses that forbid hipMalloc): the F and
   theta of gf_measure for an SU(3) field the caller holds on device
   `hip_device`, without a handle or workspace.  links: device pointer to the
   field in the natural layout (V*4*18 doubles, V = dims[0]*dims[1]*dims[2]*
   dims[3]); gauge: GF_LANDAU, GF_COULOMB or GF_MAG (Coulomb: the averages
   over the time-slices, as gf_measure); out: device pointer, receives
   out[0] = F and out[1] = theta (no finiteness check).  Every extent even and
   >= 2, at most GF_NOALLOC_MAX_SITES sites, else GF_E_DIMS.  The work is
   enqueued on `hip_stream` (a stream of that device, NULL the default
   stream) and the call returns without waiting; it allocates nothing and
   needs no synchronisation, so it can be captured in a HIP graph.  The
   partial sums go to a fixed array of 16 KiB in the library (2048 doubles,
   one pair per reduction block) that each device holds for the life of the
   process; every call on a device uses the same array, so calls that
   overlap on one device (on different streams, or from several threads)
   race and give wrong values.  Errors are reported by gf_last_error(NULL). */
#define GF_NOALLOC_MAX_SITES ((int64_t)1 << 29)
int gf_measure_noalloc(int hip_device, void *hip_stream, int gauge, const int32_t dims[4], const double *links,
                       double *out);

/* Mean and maximum of |1 - det U| over the links of `inst` (Sec. 4.5). */
int gf_unitarity(gf_handle h, int32_t inst, double *mean, double *max);

/* Reproject every link (and the Coulomb accumulator) to SU(3) in FP64
   (SU(2): normalise the 4 components). */
int gf_reunitarise(gf_handle h);

/* Global sweep index of instance `inst`, the random-stream counter
   (checkpoint / resume of annealing runs). */
int gf_get_sweep_index(gf_handle h, int32_t inst, uint64_t *index);
int gf_set_sweep_index(gf_handle h, int32_t inst, uint64_t index);

/* Kernel configuration (launch shapes).  The half-sweep kernels come in
   three tables: GF_KERNELS_FP32 (update computed in FP32: mixed and single
   storage), GF_KERNELS_FP64 (update in FP64: FP64 storage, the FP64 tail of
   mixed storage, stochastic relaxation) and GF_KERNELS_HEATBATH (heatbath
   and annealing).  A shape is:
   - waves_per_site: wavefronts sharing a group of 64 sites, each holding
     8/waves_per_site (Coulomb 6/waves_per_site) of the adjacent links, with
     the partial sums exchanged through LDS (the eight-threads-per-site idea
     of Sec. 4.3 at wavefront granularity): 1, 2 or 4 (Coulomb 1 or 2; SU(2)
     1);
   - block: threads per workgroup, 64, 128, 256 or 512, at least
     64*waves_per_site (a block updates block/waves_per_site sites);
   - flags: GF_SHAPE_NONTEMPORAL loads and stores the links with the
     non-temporal (streaming) cache policy (overrelaxation and
     microcanonical kernels; SU(3) only), GF_SHAPE_LINEAR_TILES hands tile b
     to block b instead of giving every XCD a contiguous range of tiles
     (inside gf_sweep a launch in which only some units work always uses
     the linear order).
   The default is waves_per_site 1 for the FP32 update, 4 (or the largest
   available) for the FP64 update, for the heatbath 1 on FP32 storage, 2 on
   FP64-12, 4 on FP64-18; block 256; no flags.  Results do not depend on the
   shape beyond rounding.
   gf_set_launch sets waves_per_site and block (0 = default) on every table
   that has such a variant, without flags (GF_E_INVALID if none has);
   gf_set_shape sets one table (GF_E_INVALID for a variant that is not
   built); gf_get_shape reads one. */
#define GF_KERNELS_FP32 0
#define GF_KERNELS_FP64 1
#define GF_KERNELS_HEATBATH 2
#define GF_SHAPE_NONTEMPORAL 1
#define GF_SHAPE_LINEAR_TILES 2
int gf_set_launch(gf_handle h, int waves_per_site, int block);
int gf_set_shape(gf_handle h, int kernels, int waves_per_site, int block, int flags);
int gf_get_shape(gf_handle h, int kernels, int *waves_per_site, int *block, int *flags);

/* Autotuning (Sec. 4.3, 4.4: the paper picks threads per site and block
   size by measurement).  gf_autotune times every shape of the tables the
   OR sweeps of the bound configuration use (FP32 and/or FP64 update) and
   keeps the fastest; gf_autotune_heatbath does the same for the heatbath
   table at the temperature of gf_set_temperature.  A visit to a shape
   runs one untimed sweep and then times n back-to-back sweeps between two
   events, group by group as gf_sweep runs them (gf_set_cache_budget).
   Screening: `reps` rounds visit every shape in turn (n = 3); the 4 shapes
   with the smallest medians then get max(reps, 3) rounds of visits with
   n = 12, and the smallest median of those wins.  The trial sweeps
   run on the bound links; the links, the Coulomb accumulators, the sweep
   indices and counts and the stop flags are saved to host memory before
   and written back after, so the caller's state is unchanged (GF_E_NOMEM
   if the host memory for that copy cannot be allocated).
   *waves_per_site and *block (may be NULL) receive the choice (of the
   precision doing most sweeps).  With a tuning cache (gf_set_tune_cache)
   a table whose key is in the cache takes the stored shape without timing,
   and new choices are added to the file.  Key: device architecture, gauge
   group, gauge, storage, kernel table and the size class of the bound
   configuration (half-sites over all units and the number of units, each
   rounded to a power of two). */
int gf_autotune(gf_handle h, int reps, int *waves_per_site, int *block);
int gf_autotune_heatbath(gf_handle h, int reps, int *waves_per_site, int *block);

/* File of persisted autotuning choices (one "key W B nt xcd" line each),
   read now if it exists and rewritten (via a temporary file and rename)
   after each tuning that adds a choice; NULL or "" turns the cache off.
   GF_E_INVALID if the file cannot be written when a choice is added. */
int gf_set_tune_cache(gf_handle h, const char *path);

/* Kernel timing: every: 0 off; n >= 1 times half-sweep launches with HIP
   events that the launch itself records on the handle's stream.  Inside
   gf_sweep, the launches of every n-th chunk of check_every sweeps are timed
   (plain launches; the other chunks replay their HIP graphs as usual);
   elsewhere every launch is timed.  n = 1: every launch, no graphs.
   GF_E_INVALID for every < 0.
   gf_kernel_time returns the number of timed half-sweep launches and their
   mean duration in milliseconds since timing was last set; which: 0 all
   launches, 1 launches computing the update in FP32, 2 in FP64. */
int gf_set_timing(gf_handle h, int every);
int gf_kernel_time(gf_handle h, int which, int64_t *launches, double *mean_ms);

/* Infinity-Cache grouping (an MI355X device has a 256 MB last-level cache
   in front of HBM).  Inside gf_sweep, consecutive units (instances, or
   Coulomb time-slices) whose working sets add up to at most `bytes` form a
   group, and each group runs the whole chunk of check_every sweeps before
   the next group starts, so a group's links stay in the cache across its
   sweeps.  Units are independent, so every unit goes through the same
   sweeps and checks as without grouping and the results are identical; a
   unit larger than the budget is a group of its own.  Working set of a unit:
   8 link planes over its half-sites (Coulomb: 6 spatial planes and the 2
   accumulator planes), 48 / 96 / 144 bytes per link.  bytes = 0 turns
   grouping off; default 224 MiB.  GF_E_INVALID for bytes < 0.  Annealing
   (GF_ANNEAL) is never grouped.  gf_cache_groups returns the number of
   groups of the bound configuration. */
int gf_set_cache_budget(gf_handle h, int64_t bytes);
int gf_cache_groups(gf_handle h, int32_t *groups);

/* HIP graph capture of the sweep loop between checks (1 = on, default):
   each chunk of check_every sweeps is captured once per launch pattern
   (update, waves per site group, FP64-update variants, position relative to
   the reprojection interval) and replayed. */
int gf_set_graph(gf_handle h, int enable);

/* Streaming ceiling (measurement only, no part of the method): the plain
   memory traffic one half-sweep is compared with.  kind GF_STREAM_COPY*:
   copy `bytes` from `src` to `dst` (device pointers, 16-byte aligned, bytes
   a multiple of 16), 16-byte loads and stores, optionally non-temporal;
   dst == src is allowed and makes an in-place pass (every 16 bytes read and
   written back, the traffic of an in-place update; other overlaps are not);
   GF_STREAM_READ: read `bytes` of `src` and write the sum of each 16 KiB
   block as one float to `dst` (gf_stream_blocks gives the count; dst must
   hold that many).
   Enqueued on `hip_stream`; returns without waiting.  GF_E_INVALID for bad
   arguments, GF_E_HIP if the launch fails. */
#define GF_STREAM_COPY 0
#define GF_STREAM_COPY_NT_LOAD 1
#define GF_STREAM_COPY_NT_STORE 2
#define GF_STREAM_COPY_NT 3
#define GF_STREAM_READ 4
int gf_stream(void *hip_stream, int kind, void *dst, const void *src, size_t bytes);
int gf_stream_blocks(size_t bytes, int64_t *blocks);

#ifdef __cplusplus
}
#endif

#endif /* GF_H */
