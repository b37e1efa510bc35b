/*
 * pmfmm.h - C ABI of the short-range PM-FMM gravity library for MI355X.
 *
 * The library evaluates the short-range part of the Gaussian-split gravity
 * of the PM-FMM method (Wang & Meng, "PhotoNs-GPU", arXiv 2107.14008):
 * particles in a periodic cube, split radius r_s (Sec. 2: r_s = 1.2 of the
 * PM cell), a cutoff radius (Sec. 2: the kernel is truncated there), the
 * leaf size MAXLEAF of the ORB tree (Sec. 2) and the expansion order p of
 * the truncated M2L (Sec. 2, M2L equation) in; the short-range
 * accelerations out.
 *
 * Per particle i the result is
 *     a_i = G sum_j m_j T(|d_ij| / 2 r_s) d_ij / |d_ij|^3,  0 < |d_ij|^2 < r_cut^2,
 * with d_ij the periodic displacement from i to j and
 * T(x) = erfc(x) + (2x / sqrt(pi)) exp(-x^2) (Sec. 2, Eq. (tr)).  Pairs of
 * ORB leaves within the cutoff are summed directly (P2P, Sec. 3.2 Alg. 1 and
 * Alg. 2); with the far field on, well separated cell pairs lying wholly
 * inside the cutoff go through P2M, M2M, M2L, L2L and L2P instead (Sec. 2).
 *
 * Conventions for every call:
 *   - return value: PMFMM_OK (0) or a negative pmfmm_status; no C++
 *     exception crosses the ABI; pmfmm_last_error() gives the message of the
 *     last failure on the calling thread;
 *   - arrays of particles are in the caller's order, positions as (n, 3)
 *     row-major float64, masses (n) float64, accelerations (n, 3) float64;
 *   - a "device" pointer is HIP device memory of the current device; a
 *     "host" pointer is ordinary host memory;
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream);
 *     device work is enqueued on it and the call returns without waiting,
 *     except where stated;
 *   - a context is used by one thread at a time; contexts are independent.
 */
#ifndef PMFMM_H
#define PMFMM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum pmfmm_status {
    PMFMM_OK = 0,
    PMFMM_EINVAL = -1,       /* bad argument or parameter                  */
    PMFMM_ENOMEM = -2,       /* host or device allocation failed           */
    PMFMM_EDEVICE = -3,      /* a HIP call failed (no device, launch error) */
    PMFMM_ESTATE = -4,       /* call out of order (e.g. forward before build) */
    PMFMM_EUNSUPPORTED = -5  /* valid request this build does not provide   */
} pmfmm_status;

/* Arithmetic of the pair force (Sec. 4 compares single and double). */
enum { PMFMM_FP64 = 0, PMFMM_FP32 = 1 };
/* Truncation factor T: library erfc/exp, the Taylor table of Eq. (int), or
 * a table of the whole radial factor T(r) / r^3 over polynomial segments
 * in r^2 (not in the paper): r^2 is scaled so that r_cut^2 = 2^11, and each
 * octave of the scaled r^2 is cut into table_size equal segments, each
 * holding the polynomial of degree table_level that approximates
 * T(r) / r^3 on it (Chebyshev interpolation); zero beyond r_cut.  Float32
 * covers the octaves [2^-35, 2^11) with degree 1 or 2; float64 covers
 * [2^-5, 2^11) with degree 4 to 6 and takes pairs closer than that (below
 * r_cut / 256) through the library erfc/exp.  It needs one r_cut / r_s for
 * all boxes of a plan. */
enum { PMFMM_TRUNC_EXACT = 0, PMFMM_TRUNC_TABLE = 1, PMFMM_TRUNC_R2 = 2 };
/* M2L acceptance against the cutoff (Sec. 2 truncates the kernel at
 * r_cut; where a cell pair straddles r_cut the paper does not say).
 * INSIDE: a MAC-accepted cell pair goes to M2L only when the whole pair
 * lies inside r_cut (|(|R| + h_t + h_u)|^2 < r_cut^2 (1 - 2^-40)), else it
 * is refined, down to per-pair truncated P2P, so the FMM converges to the
 * truncated pair sum.  CENTRE: the literal reading, the kernel derivatives
 * f_(n)(|R|) are zero beyond r_cut by centre distance: a MAC-accepted cell
 * pair goes to M2L when |R|^2 < r_cut^2 and is dropped otherwise. */
enum { PMFMM_M2L_INSIDE = 0, PMFMM_M2L_CENTRE = 1 };
/* Table node choice for x: nearest node or the node below x. */
enum { PMFMM_ROUND_NEAREST = 0, PMFMM_ROUND_FLOOR = 1 };
/* Accumulation of the float32 pair sums of each work item: each j leaf's
 * float32 sum added into float64 (default), or into a float32 sum with a
 * float32 compensation term by Knuth's TwoSum (the error-free sum of two
 * floats; the pair is added in float64 at the end of the item).  Sec. 4
 * compares single against double precision; the compensated float32 sum is
 * the all-single-precision variant with the rounding of the running sum
 * recovered. */
enum { PMFMM_ACCUM_FP64 = 0, PMFMM_ACCUM_FP32_TWOSUM = 1 };

typedef struct pmfmm_params {
    /* geometry and force split (Sec. 2) */
    double box;          /* side L of the periodic cube, > 0                     */
    double r_s;          /* split radius, > 0                                     */
    double r_cut;        /* cutoff radius, 0 < r_cut < box / 2                    */
    double G;            /* gravitational constant multiplying every force        */
    double theta;        /* opening angle of the M2L acceptance test
                            (r_A + r_B) < theta |R|; 0 turns the far field off  */
    int32_t max_leaf;    /* MAXLEAF of the ORB tree, 1..64                        */
    int32_t order;       /* expansion order p, 0..6; < 0 turns the far field off  */
    int32_t m2l_cut;     /* PMFMM_M2L_INSIDE (default) or PMFMM_M2L_CENTRE         */
    /* evaluation of the pair force (Sec. 3.3) */
    int32_t precision;   /* PMFMM_FP64 or PMFMM_FP32                              */
    int32_t trunc;       /* PMFMM_TRUNC_EXACT, _TABLE or _R2                       */
    int32_t table_size;  /* TABLE: nodes on x in [0, 3], 16..2048 (FP64) or
                            16..4096 (FP32); R2: segments per octave of r^2,
                            FP32 degree 2: 16, 32, 64 or 128; FP32 degree 1:
                            64, 128, 256 or 512; FP64: 16, 32 or 64          */
    int32_t table_level; /* TABLE: Taylor terms kept, 0..4 (T_[0] .. T_[4]);
                            R2: polynomial degree, FP32 2 or 1 (the linear
                            table covers r >= 2^-9.5 r_cut; closer pairs are
                            evaluated exactly), FP64 4, 5 or 6               */
    int32_t table_round; /* TABLE: PMFMM_ROUND_NEAREST or PMFMM_ROUND_FLOOR       */
    /* scheduling of the P2P work (no effect on results) */
    int32_t chunk;       /* j-leaves per work item, 0 = automatic                 */
    int32_t wg_waves;    /* wavefronts per workgroup of the P2P and adjoint launches,
                            0 = auto; the float64 exact P2P and every float64
                            adjoint run at most 4 (larger values use 4)       */
    int32_t grid_wgs;    /* workgroups of the persistent launch, 0 = auto         */
    int32_t timing;      /* 1: time each phase with HIP events (see get_timings)  */
    int32_t threads;     /* host threads of the host planner, 0 = all             */
    int32_t planner;     /* pmfmm_build: 0 = plan on the GPU, 1 = on the host     */
    int32_t accum;       /* PMFMM_ACCUM_FP64 (default) or PMFMM_ACCUM_FP32_TWOSUM
                            (float32 forms only; the adjoint always adds in
                            float64)                                           */
} pmfmm_params;

typedef struct pmfmm_ctx pmfmm_ctx;

/* Fill *p with defaults: box 100, r_s 3.75, r_cut 4.5 r_s, G 1, theta 0,
 * max_leaf 64, order 4, M2L inside the cutoff, FP64, exact T, 2048-node
 * table, level 4, nearest, float64 accumulation. */
void pmfmm_params_init(pmfmm_params* p);

/* Validate and copy *p into a new context.  *out receives the context, to be
 * released by pmfmm_destroy.  No device memory is taken yet.
 * Errors: EINVAL for any parameter outside the ranges above, ENOMEM. */
int pmfmm_create(const pmfmm_params* p, pmfmm_ctx** out);

/* Release the context and all host and device memory it owns (waits for
 * the device work it enqueued).  NULL is accepted. */
void pmfmm_destroy(pmfmm_ctx* ctx);

/* Message of the last failed call on this thread ("" if none). */
const char* pmfmm_last_error(void);

/* Host-only planning (Sec. 2 ORB tree; Sec. 3 dual walk and task lists;
 * Sec. 3.2 TaskGroup / GroupIdx).  `pos` (n, 3) and `mass` (n) are host
 * pointers, copied.  Positions are wrapped into [0, box).  Builds the tree,
 * the P2P list (i leaf, j leaf, image shift) sorted by (i, j, shift), the
 * M2L list sorted by (target, source, shift) and the work items; touches no
 * GPU.  Errors: EINVAL (n < 1, NaN/Inf position, negative mass), ENOMEM. */
int pmfmm_plan(pmfmm_ctx* ctx, int64_t n, const double* pos,
               const double* mass);

/* Several independent boxes in one plan (one persistent launch later).
 * Box b holds counts[b] >= 1 particles, stored consecutively in `pos` and
 * `mass` (host pointers) in box order; per_box[b] gives its geometry, split,
 * cutoff, G, max_leaf, order and theta; the evaluation fields are the
 * context's.  Errors as pmfmm_plan; the message names the first bad box. */
int pmfmm_plan_batch(pmfmm_ctx* ctx, int32_t nbox,
                     const pmfmm_params* per_box, const int64_t* counts,
                     const double* pos, const double* mass);

/* Plan and upload everything the kernels read.  With params.planner = 0
 * (default) the tree, task lists and work items are built on the GPU from
 * the particles (the same lists as pmfmm_plan, integer for integer); with
 * planner = 1 they are built by pmfmm_plan on the host and uploaded.
 * on_device = 0: pos and mass are host pointers (copied to the device);
 * 1: device pointers (the host planner copies them to the host first).  The
 * particles are gathered into leaf order on the device.  Synchronises
 * `stream` before returning (list sizes come back to the host).  With the
 * GPU planner and the far field on, the far field (P2M .. L2P) is started
 * here, on a stream the context owns, as soon as the M2L lists exist; it
 * may still run when the call returns, and the next forward, adjoint or
 * build on any stream waits for it.  The caller may free or change pos and
 * mass when the call returns.
 * Errors: those of pmfmm_plan, EDEVICE, ENOMEM. */
int pmfmm_build(pmfmm_ctx* ctx, int64_t n, const double* pos,
                const double* mass, int32_t on_device, void* stream);

/* pmfmm_plan_batch followed by the upload, as pmfmm_build. */
int pmfmm_build_batch(pmfmm_ctx* ctx, int32_t nbox,
                      const pmfmm_params* per_box, const int64_t* counts,
                      const double* pos, const double* mass,
                      int32_t on_device, void* stream);

/* Change how the pair force is evaluated (precision, trunc, table_*, accum) and
 * how the P2P work is scheduled (chunk, wg_waves, grid_wgs, timing) without
 * rebuilding the tree.  Geometry, split and tree fields of *p are ignored.
 * A change of chunk re-cuts the work items (needs a prior plan; re-uploads
 * them if the context was built).  Errors: EINVAL. */
int pmfmm_set_eval(pmfmm_ctx* ctx, const pmfmm_params* p);

/* Short-range accelerations of the built particles.  `acc` is a device
 * pointer to (n_total, 3) float64, written in the caller's particle order
 * (boxes consecutive for a batch).  Enqueues: far field (if on and not
 * already started by the build; otherwise a wait for it), the persistent
 * P2P kernel (Alg. 1 / Alg. 2), the ordered reduction of the work-item
 * partials, all on `stream`.  Results are bitwise reproducible run to run.
 * Errors: ESTATE (not built), EDEVICE. */
int pmfmm_forward(pmfmm_ctx* ctx, double* acc, void* stream);

/* pmfmm_forward for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc).
 * Same arguments, kernels and results (bit for bit) as pmfmm_forward; the
 * queue counters and the work items' partial sums live in a static device
 * array of the library instead of the context's buffers: 64 MiB per GPU,
 * held from the first use on that GPU until the process ends, room for
 * 43,688 work items (about 4e5 particles of clustered input at leaf 64).
 * The call allocates nothing, records no timing events and, unlike
 * pmfmm_forward, never builds or uploads the truncation table: the build
 * uploads it, and after a pmfmm_set_eval that changes the evaluation this
 * call refuses until pmfmm_forward (or a build) has run once.  Every call on
 * one GPU shares that GPU's array (the counters are cleared by a kernel at
 * the start of each call): calls that overlap on one GPU, on any streams or
 * contexts, race and give wrong results; order them on one stream or with
 * events.  Errors: ESTATE (not built, or the table is not current), EINVAL
 * (more work items than the array holds: use pmfmm_forward), EDEVICE. */
int pmfmm_forward_static(pmfmm_ctx* ctx, double* acc, void* stream);

/* Gradient of loss = sum_i w_i . a_i with respect to positions and masses
 * (not in the paper; the transpose of the pair sum of Eq. (tr) and, with
 * the far field on, of the Sec. 2 operators P2M, M2M, M2L, L2L, L2P, with
 * the tree, the task lists and the expansion centres of the last build
 * held fixed).  w, grad_pos: device (n_total, 3); grad_mass: device
 * (n_total); caller order.  The almost-everywhere gradient: the step of the
 * hard cutoff is left out.  Pairs are evaluated in the context's
 * precision: with the exact T (erfc and exp), except in the float32 r^2
 * form (PMFMM_FP32 with PMFMM_TRUNC_R2), where g = T / r^3 and
 * h = g'(r) / r come from quadratic tables in r^2 (32 segments per octave,
 * built and uploaded on the first adjoint of a context, with a stream
 * synchronisation).  Errors: ESTATE, EDEVICE. */
int pmfmm_adjoint(pmfmm_ctx* ctx, const double* w, double* grad_pos,
                  double* grad_mass, void* stream);

/* Long-range accelerations of the force split (Sec. 2; not the short-range
 * hot path): the Newtonian force minus the short-range pair force of
 * Eq. (tr), on a periodic mesh of n_pm^3 nodes at g L / n_pm.  Cloud in cell
 * assignment; phi(k) = -4 pi G rho(k) exp(-k^2 r_s^2) / k^2 divided by the
 * squared CIC window prod_a sinc^2(k_a L / 2 n_pm) (the transform of
 * erf(r / 2 r_s) / r; k = 0 dropped, the mean density subtracted);
 * a(k) = -i k phi(k) with each Nyquist component zeroed; cloud in cell
 * interpolation.  Uses the context's box, r_s and G (one box; no build
 * needed).  pos (n, 3), mass (n), acc (n, 3): device float64, caller
 * order; acc is overwritten.  Enqueued on `stream`; the mesh and the FFT
 * plans (hipFFT) are allocated on the first call for a given n_pm and kept.
 * The deposit adds with float64 atomics: results agree run to run to
 * rounding, not bit for bit.  Errors: EINVAL (n_pm odd or outside
 * [4, 1024], n < 0), EDEVICE. */
int pmfmm_long_range(pmfmm_ctx* ctx, int32_t n_pm, int64_t n, const double* pos,
                     const double* mass, double* acc, void* stream);

/* Time stepping around the force (the paper's runs of Sec. 4 take time
 * steps without naming the integrator; a kick-drift-kick leapfrog is the
 * reading here; not the short-range hot path).  pmfmm_kick:
 * vel += acc dt; pmfmm_drift: pos += vel dt, then wrapped into [0, box).
 * pos, vel, acc: device (n, 3) float64, caller order; enqueued on `stream`.
 * One KDK step of length dt is kick(dt / 2) with a(t), drift(dt), a new
 * force, kick(dt / 2).  Errors: EINVAL (null, n < 0, dt not finite,
 * box <= 0), EDEVICE. */
int pmfmm_kick(int64_t n, double* vel, const double* acc, double dt, void* stream);
int pmfmm_drift(int64_t n, double* pos, const double* vel, double dt, double box, void* stream);

/* Host views of the plan, valid until the next plan/build or destroy.
 * Particle and leaf indices are global over the batch; `perm[k]` is the
 * caller index of the particle stored k-th (leaf order). */
typedef struct pmfmm_lists {
    int64_t n;                 /* particles over all boxes                */
    int64_t n_boxes, n_leaves, n_cells, n_p2p, n_m2l, n_items;
    int64_t candidate_pairs;   /* sum over P2P tasks of n_i * n_j         */
    const int32_t* perm;       /* (n)                                     */
    const int32_t* box_first_leaf; /* (n_boxes + 1)                        */
    const int32_t* box_first_cell; /* (n_boxes + 1)                        */
    const int32_t* leaf_first; /* (n_leaves) first particle, leaf order   */
    const int32_t* leaf_count; /* (n_leaves)                              */
    const int32_t* leaf_cell;  /* (n_leaves) cell of each leaf            */
    const int32_t* cell_first; /* (n_cells)                               */
    const int32_t* cell_count; /* (n_cells)                               */
    const int32_t* cell_child; /* (n_cells, 2), -1 for a leaf             */
    const double* cell_lo;     /* (n_cells, 3)                            */
    const double* cell_hi;     /* (n_cells, 3)                            */
    const int32_t* p2p_row;    /* (n_leaves + 1) CSR rows of i leaves     */
    const int32_t* p2p_j;      /* (n_p2p) source leaf                     */
    const int32_t* p2p_shift;  /* (n_p2p) (sx+1) + 3 (sy+1) + 9 (sz+1)   */
    const int32_t* m2l_row;    /* (n_cells + 1) CSR rows of target cells  */
    const int32_t* m2l_src;    /* (n_m2l) source cell                     */
    const int32_t* m2l_shift;  /* (n_m2l)                                 */
} pmfmm_lists;

/* Fill *out with views of the current plan.  Errors: ESTATE (no plan). */
int pmfmm_get_lists(const pmfmm_ctx* ctx, pmfmm_lists* out);

/* Phase times of the last forward/adjoint, in milliseconds, measured with
 * HIP events recorded on the call's stream (only when params.timing = 1;
 * this call waits for those events). */
typedef struct pmfmm_timings {
    double far_ms;       /* P2M .. L2P (with the GPU planner the far
                            field runs during pmfmm_build, on a stream
                            of the library's beside the work items)  */
    double p2p_ms;       /* the persistent P2P kernel alone          */
    double reduce_ms;    /* ordered reduction + write-back           */
    double total_ms;     /* whole forward                            */
    double adjoint_ms;   /* adjoint P2P kernel alone                 */
} pmfmm_timings;

/* Errors: ESTATE (timing off or nothing timed yet), EDEVICE. */
int pmfmm_get_timings(const pmfmm_ctx* ctx, pmfmm_timings* out);

/* One schedule of the persistent P2P launch and its measured time. */
typedef struct pmfmm_schedule {
    int32_t chunk;       /* j leaves per work item, 0 = automatic              */
    int32_t wg_waves;    /* wavefronts per workgroup, 0 = automatic            */
    int32_t grid_wgs;    /* persistent workgroups, 0 = as many as fit          */
    int32_t pad;
    double p2p_ms;       /* mean P2P kernel time in ms; < 0: not timed         */
} pmfmm_schedule;

/* Schedule autotuner of the persistent P2P launch (the paper schedules its
 * task groups with a grid-stride loop, Sec. 3.2, Alg. 1; the tuner is this
 * library's).  Every work item writes its own partial sums, added in a
 * fixed order, so wg_waves and grid_wgs leave the results bitwise alone and
 * chunk (which regroups the float64 sums) changes them by rounding only;
 * the schedule sets
 * how the TaskGroup rows are cut into work items, how many wavefronts
 * share a workgroup (and its LDS copy of a table) and how many workgroups
 * the persistent grid has.  On a built context, times each candidate: one
 * untimed pmfmm_forward into `acc` (device (n_total, 3) float64, written),
 * then `repeats` (1..100) forwards with the P2P kernel timed by HIP events
 * on `stream`; applies the fastest as pmfmm_set_eval would (the other
 * evaluation fields and `timing` stay as they were).
 * cands / n_cands: schedules to try; NULL for the default 24 (chunk 0, 8,
 * 16, 32, 64, 2^20 x wg_waves 2, 4, 8, 16, grid automatic; wg_waves above
 * what the form runs, see pmfmm_params, are skipped).  results (optional,
 * n_cands or 24 entries): each schedule with its time (p2p_ms < 0 when it
 * was skipped or not timed).  cache_path (optional): a text file of lines
 * "key chunk wg_waves grid_wgs p2p_ms", key = device architecture, compute
 * units, pair form and a coarse size signature of the plan (boxes, leaves
 * / 1024, sqrt of the P2P task count / 32); on a hit the cached schedule is
 * applied without timing, on a miss the winner is appended.  *best
 * receives the applied schedule.  Synchronises `stream`.
 * Errors: EINVAL (null acc or best, repeats or n_cands out of range, an
 * invalid candidate), ESTATE (not built), EDEVICE. */
int pmfmm_autotune(pmfmm_ctx* ctx, double* acc, const pmfmm_schedule* cands,
                   int32_t n_cands, int32_t repeats, const char* cache_path,
                   pmfmm_schedule* results, pmfmm_schedule* best, void* stream);

/* Library version string. */
const char* pmfmm_version(void);

#ifdef __cplusplus
}
#endif

#endif /* PMFMM_H */
