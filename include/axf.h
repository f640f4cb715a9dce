/*
 * axf.h -- C ABI of the MI355X (gfx950) axisymmetric modal FMM library.
 *
 * The library evaluates, for azimuthal modes n = 0..N, the modal potential
 *
 *     Phi^(n)(r_j, z_j) = sum_i S_i^(n) G^(n)(r_j, r_i, z_j - z_i)
 *
 * of ring sources at (r_i, z_i) with complex Fourier strengths S_i^(n), at
 * field points (r_j, z_j), where G^(n)(r, r1, x) = Q_{n-1/2}(chi) /
 * (2 pi sqrt(r r1)), chi = (r^2 + r1^2 + x^2) / (2 r r1), is the modal Green's
 * function of Carley, "A Fast Multipole Method for axisymmetric domains"
 * (arXiv 2301.01179), eqs. analysis:gfunc and analysis:sum.  The sum is
 * approximated by the paper's uniform (r, z) quadtree FMM (Algorithm 1):
 * Taylor tables of G built by the Laplace-equation derivative recursion
 * (App. A), moments (eq. analysis:moments), moment shift (eq. analysis:shift),
 * source-to-local operators with the FO/BO/FI/BI reuse (section 2.2,
 * eq. analysis:s2l), local shift (eq. analysis:l2l) and direct near-field
 * sums over the 3x3 neighbour leaves.
 *
 * Conventions (all entry points):
 *   - Every array argument is a DEVICE pointer unless marked "host".
 *   - Complex numbers are interleaved (re, im) doubles (complex128).
 *   - Strengths S: complex128 [nrhs][n_modes][ns]; potentials phi: complex128
 *     [nrhs][n_modes][nf]; both in the caller's point order.
 *   - The caller owns every buffer it passes; the library keeps no reference
 *     to them after the enqueued work completes.  Buffers must stay alive
 *     until the work on `stream` has finished (ordinary stream semantics).
 *   - `stream` is a hipStream_t passed as void* (NULL = default stream).
 *   - A source whose (r, z) equals a field point bit for bit does not act on
 *     it (no self interaction; the log singularity is excluded).
 *   - Errors are returned as status codes and never thrown; axf_last_error()
 *     returns a thread-local description of the last failure.  An argument
 *     error enqueues no work.  Asynchronous kernel failures surface as
 *     AXF_ERR_HIP on a later call.
 *   - A plan must not be used on two streams at the same time.
 */
#ifndef AXF_H
#define AXF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    AXF_OK = 0,
    AXF_ERR_INVALID_ARGUMENT = 1,  /* null pointer, negative size, bad params  */
    AXF_ERR_INVALID_GEOMETRY = 2,  /* r <= 0, or a non-finite coordinate       */
    AXF_ERR_OUT_OF_MEMORY = 3,     /* device allocation failed                 */
    AXF_ERR_UNSUPPORTED = 4,       /* order, modes or depth beyond the limits  */
    AXF_ERR_HIP = 5,               /* a HIP runtime call failed                */
    AXF_ERR_WORKSPACE = 6          /* caller workspace too small or misaligned */
} axf_status;

/* Limits of the library. */
#define AXF_MAX_MODES 64   /* n_modes = N + 1 <= 64                     */
#define AXF_MAX_ORDER 24   /* expansion order M <= 24                   */
#define AXF_MAX_DEPTH 11   /* tree depth d <= 11                        */
#define AXF_MAX_RHS 8      /* right-hand sides per plan                 */
#define AXF_MAX_ANGLES 2048 /* samples per ring of the azimuthal transforms */

/* Plan parameters.
 *   n_modes : N + 1, modes n = 0..N (1 <= n_modes <= AXF_MAX_MODES).
 *   order   : expansion order M of moments and locals; moments S_ij with
 *             i + j <= M, locals Phi_kl with k + l <= M, derivative tables to
 *             total order 2M (0 <= M <= AXF_MAX_ORDER).
 *   depth   : tree depth d (2 <= d <= AXF_MAX_DEPTH), or 0 to choose the
 *             smallest d >= 2 with at most max_leaf sources and at most
 *             max_leaf field points in every leaf (capped at AXF_MAX_DEPTH).
 *   max_leaf: leaf bound used when depth == 0 (>= 1).
 *   nrhs    : right-hand sides sharing the geometry (1..AXF_MAX_RHS).
 *   flags   : the S2L pass contracts, for each interaction-list offset,
 *             one table per radial station and mode against the moments of
 *             several target boxes of that station at once (section 2.2's
 *             operator reuse).  No AXF_TILE flag (the default): on the FP64
 *             matrix cores, up to 16 boxes of a station column per tile.
 *             AXF_TILE(tb), tb = 2, 4 or 8: on the vector units, tb
 *             same-parity boxes per tile.  AXF_NO_OVERLAP: potential
 *             evaluations run the near field after the downward pass on the
 *             caller's stream instead of beside it on a second stream of the
 *             library.  Other bits must be 0. */
#define AXF_TILE_SHIFT 8
#define AXF_TILE_MASK (0xFu << AXF_TILE_SHIFT)
#define AXF_TILE(tb) ((uint32_t)(tb) << AXF_TILE_SHIFT)
#define AXF_NO_OVERLAP (1u << 12)

typedef struct {
    int32_t n_modes;
    int32_t order;
    int32_t depth;
    int32_t max_leaf;
    int32_t nrhs;
    uint32_t flags;
} axf_params;

typedef struct axf_plan axf_plan;   /* opaque; owned by the library */

/* Build a plan for fixed source and field points (Algorithm 1, first two
 * steps, plus the Taylor tables of App. A for every level, radial station
 * and the twelve separations of section 2.2).
 *   r_src, z_src : [ns] source ring radii and axial stations (device).
 *   r_fld, z_fld : [nf] field points (device).  May alias the sources.
 * The plan copies what it needs; the coordinate buffers may be freed after
 * the call returns.  This call synchronises `stream` (it reads back the
 * bounding square and the tree occupancy) and allocates device memory (the
 * library's own, see axf_plan_set_workspace).  The tables are built on an
 * internal stream of the library and may still be in flight when the call
 * returns: every later call that reads them waits for them on its own stream
 * (evaluations just before their first S2L pass).
 *   workspace_bytes : host output (may be NULL), the device bytes that hold
 *          every buffer of this plan (sorted points, tree, work lists,
 *          tables, moments, locals and evaluation scratch), the size that
 *          axf_plan_set_workspace needs.
 * Returns AXF_ERR_INVALID_GEOMETRY if any r <= 0 or any coordinate is not
 * finite; ns >= 1 and nf >= 1 are required. */
axf_status axf_plan_create(const axf_params *params,
                           int64_t ns, const double *r_src, const double *z_src,
                           int64_t nf, const double *r_fld, const double *z_fld,
                           void *stream, axf_plan **out_plan, size_t *workspace_bytes);

/* Move every buffer of the plan into caller-owned device memory, e.g. a
 * uint8 tensor of the caller's allocator: `workspace` (aligned to 256 bytes)
 * of `bytes` >= the workspace_bytes that axf_plan_create reported.  The
 * plan's contents are copied, its device pointers rebased, and the library's
 * own memory for it released; from then on the plan reads and writes only
 * the workspace (and the caller's inputs and outputs).  The caller keeps the
 * workspace alive and untouched until axf_plan_destroy.  Synchronises the
 * device (the plan's tables may still be in flight); no work that uses the
 * plan may be pending.  Once per plan.  Returns AXF_ERR_WORKSPACE if the
 * workspace is too small or misaligned (the plan is then unchanged). */
axf_status axf_plan_set_workspace(axf_plan *plan, void *workspace, size_t bytes);

/* Device memory that the library allocates for itself (plans without a
 * caller workspace, batches) is returned to the runtime when released,
 * unless this per-process cache is enabled: up to `bytes` of released
 * blocks are then kept and reused by later plans of a similar size, so
 * that creating plans in a loop calls no hipMalloc in the steady state.
 * 0 (the default) disables the cache; lowering the limit frees cached
 * blocks at once.  Cached blocks are invisible to other allocators. */
axf_status axf_set_cache_limit(size_t bytes);

/* Release the plan and its device memory (after pending work on the plan's
 * last stream has finished).  NULL is accepted. */
void axf_plan_destroy(axf_plan *plan);

/* FMM evaluation (Algorithm 1: moments, upward pass, downward pass, leaf
 * evaluation).  S: complex128 [nrhs][n_modes][ns]; phi: complex128
 * [nrhs][n_modes][nf], overwritten.  Asynchronous on `stream`; allocates
 * nothing. */
axf_status axf_evaluate(axf_plan *plan, const double *S, double *phi, void *stream);

/* axf_evaluate for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid it): the
 * same passes and the same result bit for bit, with the evaluation scratch
 * (strengths in tree order, moments, locals, S2L partial sums) in a fixed
 * device array of the library of 256 MiB per GPU, held from the library's
 * load until the process ends, instead of the plan's memory.  Allocates
 * nothing, records no timing events.  Returns AXF_ERR_UNSUPPORTED with a
 * message when the plan's evaluation needs more scratch than the array
 * holds (use axf_evaluate), AXF_ERR_INVALID_ARGUMENT when the plan's device
 * is not the current one.  Every call on a GPU shares that GPU's array:
 * calls that overlap on one GPU (other streams, other threads) race. */
axf_status axf_evaluate_noalloc(axf_plan *plan, const double *S, double *phi, void *stream);

/* FMM evaluation that also returns the field gradient at the field points,
 * mode by mode: dphi_dr = dPhi^(n)/dr, dphi_dz = dPhi^(n)/dz and
 * dphi_az = i n Phi^(n) / r, the coefficient of e^(i n theta) in
 * (1/r) dphi/dtheta of the series of eq. analysis:phi; same layout as phi,
 * each may be NULL.  Together they are the cylindrical components of
 * grad phi (the velocity of a potential flow, or with the roles of the
 * source components the Biot-Savart velocity the paper names as the
 * motivation in section 1).  The far field is differentiated through the
 * local expansion, the near field through the first-derivative starting
 * formulas of App. A. */
axf_status axf_evaluate_grad(axf_plan *plan, const double *S, double *phi,
                             double *dphi_dr, double *dphi_dz, double *dphi_az, void *stream);

/* Direct O(ns * nf) modal sum (eq. analysis:sum) on the GPU, same
 * arguments and layout as axf_evaluate.  Uses only the plan's points. */
axf_status axf_evaluate_direct(axf_plan *plan, const double *S, double *phi, void *stream);

/* Adjoint of axf_evaluate for a real loss L(Phi).
 *   gphi : complex128 [nrhs][n_modes][nf], dL/dRe(Phi) + i dL/dIm(Phi).
 *   gS   : complex128 [nrhs][n_modes][ns], overwritten with dL/dRe(S) +
 *          i dL/dIm(S) (the transposed FMM: G is real and symmetric, so this
 *          is the FMM with the roles of sources and field points swapped).
 *   S, g_rsrc, g_zsrc : if g_rsrc or g_zsrc is non-NULL, S must be given and
 *          g_rsrc[ns] = dL/dr_i, g_zsrc[ns] = dL/dz_i of the source rings are
 *          overwritten (summed over modes and right-hand sides).
 * The plan's sources and field points share one tree, so gS is the exact
 * transpose of axf_evaluate up to rounding. */
axf_status axf_adjoint(axf_plan *plan, const double *S, const double *gphi,
                       double *gS, double *g_rsrc, double *g_zsrc, void *stream);

/* Plan introspection (host outputs; any pointer may be NULL). */
axf_status axf_plan_info(const axf_plan *plan, int32_t *depth, int32_t *n_modes,
                         int32_t *order, int32_t *nrhs, int64_t *ns, int64_t *nf,
                         double *square4 /* host [4]: r_lo, z_lo, L, 1/L */,
                         int64_t *n_near_pairs, int64_t *n_s2l_pairs,
                         size_t *device_bytes);

/* Number of occupied source / field boxes at `level` (host outputs). */
axf_status axf_plan_level_info(const axf_plan *plan, int32_t level,
                               int32_t *n_src_boxes, int32_t *n_fld_boxes);

/* Copy one S2L Taylor table to host memory (App. A, eqs. gfunc:gnbar,
 * gfunc:taylor, gfunc:scaled).  The table belongs to `level`, inner radial
 * station `station` (0 <= station < 2^level) and box separation (dr, dz),
 * 0 <= dr, dz <= 3, not both <= 1: with h the box width at the level,
 * r_in = r_lo + (station + 1/2) h, r_out = r_in + dr h and x = dz h,
 *     out[n][a][b][c] = c! * gbar^(n)_{a,b,c}(r_out, r_in, x) * h^(a+b+c)
 * for a, b <= M and a + b + c <= 2M, zero elsewhere; host array of
 * n_modes * (M+1) * (M+1) * (2M+1) doubles owned by the caller.  Tables
 * exist up to the station of the largest ring radius (no S2L operator reads
 * one beyond it); other stations give AXF_ERR_INVALID_ARGUMENT.
 * Synchronous (waits for the plan's tables). */
axf_status axf_plan_table(const axf_plan *plan, int32_t level, int32_t station, int32_t dr,
                          int32_t dz, double *host_out);

/* Phase timing.  When enabled, the library records HIP events on the calling
 * stream around every pass of axf_evaluate / axf_evaluate_grad /
 * axf_evaluate_direct / axf_adjoint and accumulates their durations
 * (milliseconds) and launch counts per phase until read.  Reading
 * synchronises on the recorded events and resets the accumulators.
 * Phases: see AXF_PHASE_*. */
enum {
    AXF_PHASE_GATHER = 0,  /* strengths into tree order                      */
    AXF_PHASE_P2M = 1,     /* leaf moments, eq. analysis:moments             */
    AXF_PHASE_M2M = 2,     /* upward pass, eq. analysis:shift                */
    AXF_PHASE_S2L = 3,     /* downward pass: S2L translations                */
    AXF_PHASE_LEAF = 4,    /* local expansion + near field at the leaves     */
    AXF_PHASE_DIRECT = 5,  /* direct modal sum                               */
    AXF_PHASE_L2L = 6,     /* downward pass: local shifts, eq. analysis:l2l  */
    AXF_PHASE_L2P = 7,     /* local expansions at the field points, added to
                              the near field (potential-only evaluations:
                              their near field runs beside the downward pass
                              and is timed as AXF_PHASE_LEAF)                */
    AXF_NUM_PHASES = 8
};
axf_status axf_plan_set_timing(axf_plan *plan, int32_t enable);
axf_status axf_plan_read_timing(axf_plan *plan, double *ms /* host [AXF_NUM_PHASES] */,
                                int32_t *launches /* host [AXF_NUM_PHASES] */);

/* Algorithmic work of one evaluation (host outputs, any may be NULL):
 * near-field ring pairs, S2L box pairs, S2L units and FP64 operation counts
 * per phase ([AXF_NUM_PHASES], fma = 2).  An S2L unit is a target box with
 * the source boxes at offsets (dr, dz) and (dr, -dz) of its interaction list
 * (section 2.2), either of them occupied: the two share one table (the
 * derivatives' x-parity) and one P x P contraction.  Pair sums: 24 flops per
 * pair + 9 per AGM iteration + 3 per recursion step + (N + 6) per pair on
 * the backward branch + 4 per mode and right-hand side, with the iteration
 * and step counts each pair needs taken from a census of the plan's pairs
 * (sampled to about 3e7 pairs for the direct sum); P2M 4 P C + 2 P per
 * source; separable M2M 24 C(M+3, 3) per parent box and channel, L2L
 * 8 C(M+3, 3) per box and channel (AXF_PHASE_L2L); S2L 4 P^2 per unit and
 * channel; local evaluation 4 P C + 2 P per field point (AXF_PHASE_L2P; the
 * AXF_PHASE_LEAF entry counts the near-field pairs only).  The census runs
 * once, on the first call that asks for flops, and synchronises the device. */
axf_status axf_plan_work(const axf_plan *plan, int64_t *near_pairs, int64_t *s2l_pairs, int64_t *s2l_units,
                         double *flops /* host [AXF_NUM_PHASES] */);

/* The pair census behind the flop model (host outputs, either may be NULL):
 * [pairs, backward-branch pairs, AGM iterations, recursion steps] summed over
 * the near-field pairs, and the same for the direct sum (sampled and
 * scaled).  Runs the census on first use; synchronises the device. */
axf_status axf_plan_census(const axf_plan *plan, double *near_counts /* [4] */,
                           double *direct_counts /* [4] */);

/* ---------------------------------------------------------------------- */
/* Batched launches: many independent problems (uneven sizes, own points,
 * own right-hand-side counts; common n_modes and order) evaluated by one
 * launch sequence of persistent kernels that pull work items from queues
 * built at creation, captured once in a HIP graph and replayed by
 * axf_batch_launch. */
typedef struct {
    int64_t ns, nf;
    const double *r_src, *z_src;   /* device [ns] */
    const double *r_fld, *z_fld;   /* device [nf] */
    const double *S;               /* device complex128 [nrhs][n_modes][ns] */
    double *phi;                   /* device complex128 [nrhs][n_modes][nf] */
    int32_t nrhs;                  /* 1..AXF_MAX_RHS */
    int32_t depth;                 /* 0 = chosen by the autotuner */
    int32_t tile;                  /* S2L tile width 2, 4 or 8; 0 = the batch's choice */
} axf_problem;

typedef struct axf_batch axf_batch;

/* Build the batch: per-problem trees and tables, merged work queues, and
 * the captured graph.  params->nrhs and params->depth are ignored (taken per
 * problem); params->max_leaf is used where a problem's depth is 0 and the
 * autotuner is disabled (flags bit AXF_BATCH_NO_AUTOTUNE).  The autotuner
 * measures, on the device, the seconds per near-field pair, per S2L unit,
 * per shifted box and per point of a probe problem at each S2L tile width
 * (once per process for a given order, mode count and width) and gives
 * every problem of depth 0 the (depth, width) of least modelled time over
 * its exactly counted work; problems of 2,000 points or more then time
 * trial evaluations through the batch kernels (that pair, neighbouring
 * depths at that width, continuing in the direction that improves, then the
 * other widths at the fastest depth) and keep the fastest.  Those trials
 * read S and overwrite phi.  A problem's own `tile` fixes its width (the
 * autotuner then searches depths only); AXF_TILE(tb) in params->flags fixes
 * the width of every problem that names none; otherwise problems with a
 * given depth take the width whose probe S2L ran fastest (4 without the
 * autotuner).  The
 * problem array is host memory and is copied; the S and phi buffers it names
 * must stay valid for every launch.  The graph runs the near field of all
 * problems on a branch beside the downward pass.  Synchronises `stream`. */
#define AXF_BATCH_NO_AUTOTUNE 1u
axf_status axf_batch_create(const axf_params *params, int32_t nprob,
                            const axf_problem *problems, void *stream,
                            axf_batch **out_batch);

/* Evaluate every problem of the batch (replay of the captured graph). */
axf_status axf_batch_launch(axf_batch *batch, void *stream);

/* Evaluate every problem with per-problem plain launches (no graph, no
 * merged queues); the reference the batched path is measured against. */
axf_status axf_batch_launch_plain(axf_batch *batch, void *stream);

/* Depth the batch chose for problem `i` (host output). */
axf_status axf_batch_problem_depth(const axf_batch *batch, int32_t i, int32_t *depth);

/* S2L tile width of problem `i` (host output). */
axf_status axf_batch_problem_tile(const axf_batch *batch, int32_t i, int32_t *tile);

void axf_batch_destroy(axf_batch *batch);

/* ---------------------------------------------------------------------- */
/* Azimuthal analysis and synthesis (section 2): the ring source is a real
 * Fourier series s(theta1) = sum_{n=-N..N} S^(n) e^(i n theta1) with
 * S^(-n) = conj(S^(n)) (eq. analysis:source), and the potential is
 * phi(r, theta, z) = sum_{n=-N..N} Phi^(n)(r, z) e^(i n theta) (eq.
 * analysis:phi), Phi^(n) being what axf_evaluate returns for n = 0..N.
 * Angles are theta_k = 2 pi k / K, k = 0..K-1.  Both calls are
 * asynchronous on `stream`, allocate nothing and need no plan. */

/* S^(n) = (1/K) sum_k s(theta_k) e^(-i n theta_k), n = 0..n_modes-1.
 *   samples : real [nrhs][nrings][K] (each ring's samples contiguous).
 *   S       : complex128 [nrhs][n_modes][nrings], overwritten (the layout of
 *             axf_evaluate's strengths).
 * Exact for a real source of modes |n| <= n_modes - 1, which requires
 * K >= 2 n_modes - 1 (AXF_ERR_INVALID_ARGUMENT otherwise: higher modes would
 * alias); K <= AXF_MAX_ANGLES. */
axf_status axf_azimuthal_analysis(int64_t nrings, int32_t n_angles, int32_t n_modes, int32_t nrhs,
                                  const double *samples, double *S, void *stream);

/* phi(theta_k) = Re Phi^(0) + 2 Re sum_{n=1..n_modes-1} Phi^(n) e^(i n theta_k),
 * the series of eq. analysis:phi with Phi^(-n) = conj(Phi^(n)).
 *   phi : complex128 [nrhs][n_modes][npts] (axf_evaluate's output layout).
 *   out : real [nrhs][npts][K], overwritten.  1 <= K <= AXF_MAX_ANGLES. */
axf_status axf_azimuthal_synthesis(int64_t npts, int32_t n_modes, int32_t nrhs, const double *phi,
                                   int32_t n_angles, double *out, void *stream);

/* ---------------------------------------------------------------------- */
const char *axf_status_string(axf_status status);
const char *axf_last_error(void);   /* thread-local detail of the last error */

#ifdef __cplusplus
}
#endif
#endif /* AXF_H */
