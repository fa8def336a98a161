/*
 * otkm.h -- C-ABI of the MI355X (gfx950) batched Kuhn-Munkres solver.
 *
 * Problem (Eq. (1) of "A Study of Performance of Optimal Transport",
 * Section 1):
 *     minimise <C, X>  subject to  X 1 = r,  X^T 1 = c,  X >= 0,
 * with integer supplies r and demands c (the Hitchcock-Koopmans case); the
 * assignment problem is the case r = c = 1, n = m.
 *
 * Method (Section 2.3.1, "Batched KM"): a Kuhn-Munkres variant that grows
 * alternating trees from all free rows at once, augments the matching along
 * every vertex-disjoint augmenting path it finds among tight edges, and only
 * when none exists adjusts the dual potentials across the cut between the
 * reached and unreached vertices, by the smallest slack, as KM does.
 * Integer transport is reduced to assignment by giving each unit of supply and
 * demand its own vertex (the S = sum r unit expansion of Section 2.3.1).
 *
 * Arithmetic is exact: int32 costs and masses, int64 duals and totals.
 * Every result is optimal; when several optimal plans exist any one of them
 * may be returned (the solver is deterministic for a given input).  The
 * duals always form an LP certificate:
 *     u_i + v_j <= C_ij  for all i, j,
 *     u_i + v_j == C_ij  wherever the plan is positive,
 *     sum_i r_i u_i + sum_j c_j v_j == cost.
 *
 * Conventions shared by every call
 * --------------------------------
 *  * Matrices are row-major; row i is a supply (left) vertex, column j a
 *    demand (right) vertex; entry (i, j) sits at C[i * ld + j] (ld = n or m
 *    unless stated).
 *  * Cost range: max(C) - min(C) must be <= 2^31 - 1 (OT_ERANGE otherwise);
 *    this bounds every reduced cost the solver stores by 2^32.
 *  * Size limit: the on-chip solver holds one instance's row and column state
 *    in a workgroup's LDS, so n (or S = sum r for transport) must be
 *    <= OT_MAX_N (OT_ETOOBIG otherwise).
 *  * Ownership: the caller allocates and owns every input and output buffer.
 *    The library never keeps a caller pointer after a synchronous call
 *    returns; asynchronous (_dev) calls read and write caller buffers until
 *    the work queued on the given stream completes.  Device scratch is owned
 *    by the library (a per-process, per-device pool, freed at exit).
 *  * Errors: every call returns OT_OK (0) or a negative ot_status.  On error,
 *    host outputs are left untouched.  ot_strerror() names a code.
 *  * Threads: calls from several host threads are allowed; each synchronous
 *    call serialises on the library's own stream for the current device.
 */
#ifndef OTKM_H
#define OTKM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define OT_MAX_N 4096

typedef enum ot_status {
    OT_OK = 0,
    OT_EINVAL = -1,       /* null pointer, n <= 0, m <= 0, count < 0, bad option */
    OT_ERANGE = -2,       /* max(C) - min(C) > 2^31 - 1 */
    OT_EUNBALANCED = -3,  /* sum r != sum c, or sum r == 0 */
    OT_ENEGMASS = -4,     /* some r_i < 0 or c_j < 0 */
    OT_ETOOBIG = -5,      /* n (or sum r) > OT_MAX_N, or over the device budget */
    OT_ENOMEM = -6,       /* host or device allocation failed */
    OT_EDEVICE = -7,      /* a HIP runtime call failed */
    OT_ENODEV = -8,       /* no usable gfx950 device */
    OT_EINTERNAL = -9,    /* solver watchdog or invariant check tripped */
    OT_EINFEASIBLE = -10  /* sparse graph: no matching covers every row (Hall's condition fails) */
} ot_status;

/* Per-solve counters (written when a stats pointer is given).  A "level" is
 * one step of the solver: sweep the rows that just joined the forest, take
 * the smallest reduced cost over unreached columns, and settle every column
 * at that value. */
typedef struct ot_stats {
    int64_t levels;        /* solver steps */
    int64_t dual_adjusts;  /* steps that raised the duals across the cut (Section 2.3.1) */
    int64_t aug_events;    /* steps that augmented along at least one path */
    int64_t paths;         /* augmenting paths applied (== n for assignment) */
    int64_t rows_swept;    /* full cost rows read: 2n at initialisation + frontier + re-sweeps */
    int64_t gathers;       /* single cost entries re-read to refresh stale column minima */
    int64_t resweeps;      /* full re-sweeps of the forest */
    int64_t status;        /* device-side ot_status of this solve */
    int64_t t_sweep_ns;    /* device time in each phase of the level loop, */
    int64_t t_select_ns;   /*   measured by the workgroup's first wavefront  */
    int64_t t_settle_ns;   /*   (sweep / minimum selection incl. refreshes /  */
    int64_t t_augment_ns;  /*   settling / augmenting); OT_FLAG_PHASE_TIMERS  */
    int64_t refreshes;     /* steps that recomputed stale column minima */
    int64_t refresh_cols;  /* stale columns recomputed, summed over those steps */
    int64_t t_refresh_ns;  /* part of t_select_ns spent recomputing stale minima */
} ot_stats;

/* Collect the per-phase device times (t_*_ns) in ot_stats; off by default
 * because reading the device clock adds latency to every level. */
#define OT_FLAG_PHASE_TIMERS 1
/* Keep 64-bit column keys even where the cost range lets the solver use its
 * compact 32-bit keys (the same results, more instructions; for tests and
 * comparisons). */
#define OT_FLAG_WIDE_KEYS 2

/* Solver options; pass NULL for the defaults (all zero). */
typedef struct ot_options {
    int32_t max_paths;     /* trees grown at once: 0 = every free row (Batched KM),
                              1 = one tree at a time (classical KM), k = at most k.
                              With a cap the solver's level (the sum of the dual
                              adjustments) grows over the stages; a solve whose level
                              would pass 2^31 - 1 stops with OT_EINTERNAL (random
                              inputs stay near the cost range). */
    int32_t block;         /* workgroup width: 0 = automatic, else 64, 256, 512 or 1024 */
    int32_t flags;         /* OT_FLAG_* bits */
    int32_t scale;         /* cost scaling factor s (Section 2.3.1: one scaling factor turns the
                              costs into small integers): 0 or 1 = exact.  With s > 1 the solver
                              runs on C'_ij = floor(C_ij / s) and returns
                                plan  an optimal plan for C',
                                cost  sum_i C[i, plan[i]] on the ORIGINAL costs,
                                u, v  s * (optimal duals of C'), which are feasible for C
                                      (u_i + v_j <= C_ij), so
                              sum u + sum v <= OPT(C) <= cost <= sum u + sum v + n (s - 1).
                              Square assignment calls only (ot_assign_ex, ot_assign_dev). */
    int32_t wgs;           /* workgroups per instance (single-instance assignment calls):
                              0 = automatic, 1 = one workgroup, 2..16 = the columns split
                              over that many workgroups, which exchange the minimum key
                              and the settled columns through global memory with a grid
                              barrier per step (block then 256 or 512, default 512, at
                              most 4 columns per lane; OT_EINVAL otherwise) */
    int32_t reserved[3];   /* must be zero */
} ot_options;

/* Status text for a code; never NULL. */
const char *ot_strerror(int status);

/* Device check: 0 when a gfx950 device is usable, else OT_ENODEV / OT_EDEVICE. */
int ot_init(void);

/* ------------------------------------------------------------------------ */
/* Host-buffer calls (synchronous)                                           */
/* ------------------------------------------------------------------------ */

/* Assignment (Eq. (1) with r = c = 1).
 *   C    [n*n]  int32 costs (row-major, ld = n)
 *   plan [n]    out: plan[i] = column assigned to row i (a permutation)
 *   cost        out: sum_i C[i, plan[i]]
 *   u [n], v [n] out: optimal duals (may be NULL to skip)
 */
int ot_assign(const int32_t *C, int32_t n, int32_t *plan, int64_t *cost, int64_t *u, int64_t *v);

/* ot_assign with options and counters (opt and stats may be NULL). */
int ot_assign_ex(const int32_t *C, int32_t n, const ot_options *opt, int32_t *plan, int64_t *cost,
                 int64_t *u, int64_t *v, ot_stats *stats);

/* Rectangular assignment (Eq. (1) with unit masses and n != m allowed): every
 * vertex of the smaller side is matched, every vertex of the larger side at
 * most once, at minimum total cost.
 *   C    [n*m]  int32 costs (row-major, ld = m); max(n, m) <= OT_MAX_N
 *   plan [n]    out: column of row i, distinct; -1 for the n - m rows left
 *                    unmatched when n > m
 *   cost        out: sum over matched rows of C[i, plan[i]]
 *   u [n], v [m] out (may be NULL): optimal duals of the rectangular LP:
 *                    u_i + v_j <= C_ij, equality on matched pairs, and the
 *                    larger side's potentials are <= 0 and equal 0 where
 *                    unmatched (v when n <= m, u when n > m), so
 *                    sum u + sum v = cost
 *   opt (may be NULL): max_paths, block and flags as for ot_assign_ex; scale
 *                    must be 0 or 1 (OT_EINVAL otherwise).
 * Solved with the smaller side as the rows (on C^T when n > m), every row a
 * root of the forest and the column duals started at 0; needs 4 n m bytes of
 * device workspace for the transpose.
 * Errors: OT_EINVAL (null pointer, n or m <= 0, bad options), OT_ETOOBIG,
 * OT_ERANGE (max - min over C > 2^31 - 1); outputs untouched on error. */
int ot_assign_rect(const int32_t *C, int32_t n, int32_t m, const ot_options *opt, int32_t *plan,
                   int64_t *cost, int64_t *u, int64_t *v, ot_stats *stats);

/* Scaling factor for a target approximation (Section 2.3.1's single scaling
 * factor; Table 3 fixes the factor of approximation at 1.1, i.e. eps = 0.1).
 * Runs the KM reduction's two sweeps on the device and returns
 *   lower_bound = sum_i u_i + sum_j v_j   (u_i = min_j C_ij, v_j = min_i C_ij - u_i,
 *                                          a feasible dual, so <= OPT)
 *   scale = 1 + floor(eps * lower_bound / n)   (1 when lower_bound <= 0)
 * A solve with ot_options.scale = scale then costs at most
 * OPT + n (scale - 1) <= OPT + eps * lower_bound <= (1 + eps) OPT when the
 * optimum is positive.  C [n*n] host costs; lower_bound may be NULL.
 * Errors as ot_assign, and OT_EINVAL for eps < 0 or NaN. */
int ot_scale_for(const int32_t *C, int32_t n, double eps, int32_t *scale, int64_t *lower_bound);

/* Integer transport (Eq. (1), Hitchcock-Koopmans case).
 *   C [n*m] int32 costs (ld = m); r [n], c [m] int32 masses, >= 0, equal sums S >= 1.
 *   X [n*m] out: int32 optimal plan.   cost out: <C, X>.
 *   u [n], v [m] out: optimal bin duals (may be NULL).  Bins of zero mass get
 *   the tightest feasible dual: a zero-mass row takes min over columns with
 *   mass of C_ij - v_j, then a zero-mass column takes min over rows of C_ij - u_i.
 * Solved by unit expansion (S x S assignment), so S <= OT_MAX_N.
 */
int ot_transport(const int32_t *C, const int32_t *r, const int32_t *c, int32_t n, int32_t m,
                 int32_t *X, int64_t *cost, int64_t *u, int64_t *v);

/* Integer transport on the bins themselves (Eq. (1), Hitchcock-Koopmans
 * case), without expanding units, so the total mass S = sum r may be as large
 * as 2^31 - 1.  The primal-dual (Hungarian) method for transportation in the
 * form of Batched KM (Section 2.3.1): trees grow at once from every supply bin
 * with mass left over tight edges, a column bin is left through every row
 * that already ships to it, a tree that reaches a demand bin with mass left
 * ships the largest amount its path allows, and the duals move across the cut
 * when no tree can grow.
 *   C [n*m] int32 costs (ld = m); r [n], c [m] int32 masses >= 0 with equal
 *   sums S, 1 <= S <= 2^31 - 1; n, m <= OT_MAX_BINS (one workgroup holds both
 *   sides' state in LDS).
 *   X [n*m] out: int32 optimal plan;  cost out: <C, X>.
 *   u [n], v [m] out (may be NULL): optimal bin duals, zero-mass bins by the
 *   convention of ot_transport.  stats (may be NULL): paths = augmentations.
 * Errors: OT_EINVAL, OT_ENEGMASS, OT_EUNBALANCED, OT_ETOOBIG (a side above
 * OT_MAX_BINS or S above 2^31 - 1), OT_ERANGE (max(C) - min(C) over the whole
 * matrix > 2^31 - 1); outputs untouched on error. */
#define OT_MAX_BINS 3072
int ot_transport_bins(const int32_t *C, const int32_t *r, const int32_t *c, int32_t n, int32_t m,
                      int32_t *X, int64_t *cost, int64_t *u, int64_t *v, ot_stats *stats);

/* Many independent assignments in one persistent launch.
 *   C[k] [n[k]*n[k]], plan[k] [n[k]], u[k], v[k] [n[k]] (u, v arrays or their
 *   entries may be NULL); cost [count]; status [count] per-instance ot_status.
 * Returns OT_OK when the batch ran (check status[] per instance), or an error
 * for the whole call.  Instances are scheduled longest-first over persistent
 * workgroups; the workgroup width per instance comes from the size-class
 * schedule (see ot_schedule_*).
 */
int ot_assign_batch(int32_t count, const int32_t *const *C, const int32_t *n, int32_t *const *plan,
                    int64_t *cost, int64_t *const *u, int64_t *const *v, int32_t *status);

/* ------------------------------------------------------------------------ */
/* Device-buffer calls (asynchronous on `stream`, a hipStream_t or NULL for  */
/* the library stream).  All pointers are device pointers; the call only     */
/* validates scalars on the host and reports data-dependent errors (cost    */
/* range, watchdog) in stats->status / status[k] on the device.             */
/* ------------------------------------------------------------------------ */

/* Assignment on device memory.  dC [n*ld] (ld >= n), dplan [n], dcost [1],
 * du [n], dv [n] (du/dv may be NULL), dstats [1] (may be NULL). */
int ot_assign_dev(const int32_t *dC, int32_t n, int32_t ld, const ot_options *opt, int32_t *dplan,
                  int64_t *dcost, int64_t *du, int64_t *dv, ot_stats *dstats, void *stream);

/* Allocation-free variant of ot_assign_dev, for callers that cannot allocate
 * device memory (code under hipGraph capture, tight serving loops, harnesses
 * that forbid hipMalloc).  Same arguments and results as ot_assign_dev, but
 * every call runs on one workgroup over the exact costs: opt->wgs must be 0 or
 * 1 and opt->scale 0 or 1 (OT_EINVAL otherwise), and single stale columns are
 * recomputed from C itself (no transposed copy).  Its scratch (the engine's
 * lists and the reduction sweeps' outputs) is one static device array of
 * OT_NOALLOC_SCRATCH_BYTES bytes per GPU, held until the process ends; the
 * call calls no hipMalloc, hipFree or allocating library routine.  n must be
 * <= OT_MAX_N (OT_ETOOBIG otherwise; every such n fits the array).  Calls
 * that overlap on one GPU share the array and race: serialise them (one
 * stream, or events).  The array keeps the last call's contents; every word
 * a call reads it first writes.  The first call on a device also looks up the
 * array's address there (hipGetSymbolAddress, no stream work); call ot_init()
 * once beforehand where even the library's first set-up must stay out of a
 * capture. */
#define OT_NOALLOC_SCRATCH_BYTES 2244608
int ot_assign_dev_noalloc(const int32_t *dC, int32_t n, int32_t ld, const ot_options *opt,
                          int32_t *dplan, int64_t *dcost, int64_t *du, int64_t *dv, ot_stats *dstats,
                          void *stream);

/* Rectangular assignment on device memory (see ot_assign_rect).  dC [n*ld]
 * (ld >= m), dplan [n], dcost [1], du [n], dv [m] (du/dv may be NULL), dstats
 * [1] (may be NULL; status there).  On a data error (cost range, watchdog)
 * only dstats is written. */
int ot_assign_rect_dev(const int32_t *dC, int32_t n, int32_t m, int32_t ld, const ot_options *opt,
                       int32_t *dplan, int64_t *dcost, int64_t *du, int64_t *dv, ot_stats *dstats,
                       void *stream);

/* Batch on device memory.  Instance k: cost matrix at dC + coff[k] (dense,
 * ld = n[k]), its transpose at dCT + coff[k] (dCT may be NULL: see below),
 * plan/u/v at dplan/du/dv + voff[k]; dcost [count];
 * dstats [count] (may be NULL).  coff, voff, n are DEVICE arrays [count].
 * order (device, may be NULL) lists the nq instances this launch solves, in
 * processing order (longest first is best); NULL solves all count instances
 * in index order.  block selects the workgroup width (64, 256, 512 or 1024;
 * 0 = from max_n via the schedule); max_n bounds n[k] of every queued
 * instance.  Several launches (for example one per size class) may share the
 * same buffers.  The launch resets its device queue head with a kernel, so
 * the call may be captured into a hipGraph and replayed.  With dCT (same size
 * and offsets as dC, filled by ot_transpose_batch_dev) the recomputation of a
 * single stale column reads one contiguous row of the transpose; with NULL it
 * gathers one entry per row of C, which fetches a whole memory line each.
 * (ot_assign_batch_ct_dev makes the transposes inside the launch's pass
 * over the matrices instead, which on MI355X is the faster choice for the
 * embedding batch.) */
int ot_assign_batch_dev(int32_t count, int32_t max_n, const int32_t *dC, const int32_t *dCT,
                        const int64_t *coff, const int32_t *n, const int64_t *voff,
                        const int32_t *order, int32_t nq, int32_t block, int32_t *dplan,
                        int64_t *dcost, int64_t *du, int64_t *dv, ot_stats *dstats, void *stream);

/* ot_assign_batch_dev with the transposes made by the launch itself: dCT is
 * a device workspace as large as dC (same offsets, caller-owned, contents on
 * entry ignored).  The launch's pass over every matrix (the one that picks
 * the key width) also writes the matrix's transpose into dCT + coff[k], and
 * single stale columns are then recomputed from rows of those transposes,
 * which costs one pass of writes and removes the per-entry memory lines of
 * the gathers down C.  Instances solved on one wavefront (block 64 with
 * max_n <= 64) neither need nor write their transposes.  dCT == NULL:
 * OT_EINVAL.  Same queue, graph-capture and output semantics as
 * ot_assign_batch_dev. */
int ot_assign_batch_ct_dev(int32_t count, int32_t max_n, const int32_t *dC, int32_t *dCT,
                           const int64_t *coff, const int32_t *n, const int64_t *voff,
                           const int32_t *order, int32_t nq, int32_t block, int32_t *dplan,
                           int64_t *dcost, int64_t *du, int64_t *dv, ot_stats *dstats, void *stream);

/* dCT + coff[k] = transpose of dC + coff[k] (n[k] x n[k]) for every instance
 * with 1 <= n[k] <= max_n (others are skipped); asynchronous on `stream`,
 * graph-capturable.  dCT must be as large as dC. */
int ot_transpose_batch_dev(int32_t count, int32_t max_n, const int32_t *dC, const int64_t *coff,
                           const int32_t *n, int32_t *dCT, void *stream);

/* Bin-level transport on device memory (see ot_transport_bins): dC [n*ld]
 * (ld >= m), dr [n], dc [m], dX [n*m], dcost [1], du [n], dv [m]; dstats [1]
 * may be NULL.  The masses are checked on the device (OT_ENEGMASS,
 * OT_EUNBALANCED, OT_ETOOBIG and the cost range OT_ERANGE go to
 * dstats->status; the outputs are then not written). */
int ot_transport_bins_dev(const int32_t *dC, const int32_t *dr, const int32_t *dc, int32_t n, int32_t m,
                          int32_t ld, int32_t *dX, int64_t *dcost, int64_t *du, int64_t *dv,
                          ot_stats *dstats, void *stream);

/* Integer transport on device memory (same semantics as ot_transport).
 * dC [n*m], dr [n], dc [m]; dX [n*m]; dcost [1]; du [n]; dv [m];
 * dstats [1] may be NULL.  S = sum r must be passed (the host knows it when
 * it built r) and must equal sum r = sum c; the device checks the masses and
 * reports OT_EUNBALANCED / OT_ENEGMASS in dstats->status. */
int ot_transport_dev(const int32_t *dC, const int32_t *dr, const int32_t *dc, int32_t n, int32_t m,
                     int32_t S, int32_t *dX, int64_t *dcost, int64_t *du, int64_t *dv,
                     ot_stats *dstats, void *stream);

/* ------------------------------------------------------------------------ */
/* Sparse assignment: a cost graph in CSR, missing entries forbidden          */
/* ------------------------------------------------------------------------ */
/* Eq. (1) with unit masses on a bipartite cost graph (the sparse form of the
 * problem; Section 2.3.1's method on the graph's edges only): rows 0..n-1,
 * columns 0..m-1 with 1 <= n <= m <= OT_MAX_N; row i's edges go to columns
 * idx[ptr[i] .. ptr[i+1]) at int32 costs cost[...] (ptr[0] = 0, ptr
 * non-decreasing, nnz = ptr[n]).  Finds a minimum-cost matching that covers
 * every row using edges only; columns may stay free.  Outputs: plan[n] (the
 * column of each row), *total (int64), u[n] and v[m] (may be NULL): optimal
 * duals of the LP, u_i + v_j <= c_e on every edge, equality on the plan,
 * v_j <= 0 and v_j = 0 on the columns left free.  When no matching covers
 * every row, returns OT_EINFEASIBLE.  ot_assign_sparse takes host buffers,
 * checks the graph (offsets, column range, no column twice in a row:
 * OT_EINVAL) and returns once the results are copied back; outputs are
 * untouched on error.  stats may be NULL. */
int ot_assign_sparse(const int64_t *ptr, const int32_t *idx, const int32_t *cost, int32_t n, int32_t m,
                     int32_t *plan, int64_t *total, int64_t *u, int64_t *v, ot_stats *stats);

/* The same on device buffers, asynchronous on stream (NULL: the library's
 * stream).  nnz is the length of idx and cost, at least ptr[n] (it sizes the
 * library's workspace for the graph by columns, which the solve builds first;
 * at most 2^31 - 1, else OT_ETOOBIG).  The device checks the column range and
 * ptr[n] - ptr[0] <= nnz (OT_EINVAL in dstats->status) and reports
 * OT_EINFEASIBLE there;
 * ptr must be a valid offset array.  A column given twice in a row counts at
 * its cheapest copy.  du, dv, dstats may be NULL. */
int ot_assign_sparse_dev(const int64_t *dptr, const int32_t *didx, const int32_t *dcost, int32_t n, int32_t m,
                         int64_t nnz, int32_t *dplan, int64_t *dtotal, int64_t *du, int64_t *dv, ot_stats *dstats,
                         void *stream);

/* One sparse instance of a batch: every pointer is a device pointer. */
typedef struct ot_sparse_desc {
    const int64_t *ptr;
    const int32_t *idx;
    const int32_t *cost;
    int32_t n, m;
    int32_t *plan;
    int64_t *total;
    int64_t *u, *v;        /* may be NULL */
    ot_stats *stats;       /* may be NULL (then errors go unreported) */
} ot_sparse_desc;

/* Many sparse instances in one persistent launch (one workgroup per instance
 * at a time), asynchronous on stream.  ddesc [count] lives in device memory;
 * max_m bounds every instance's m (it sizes the on-chip state; an instance
 * above it reports OT_EINVAL).  Per-instance status in its stats.  count may
 * not exceed the workgroups resident at once for max_m (1,792 at max_m = 512
 * on MI355X; OT_ETOOBIG above): a launch whose workgroups took several
 * instances each faulted the GPU, and that mode stays off until the cause is
 * known. */
int ot_assign_sparse_batch_dev(int32_t count, const ot_sparse_desc *ddesc, int32_t max_m, void *stream);

/* ------------------------------------------------------------------------ */
/* Auction with epsilon-scaling (Section 2.3.3)                              */
/* ------------------------------------------------------------------------ */
/* The auction algorithm on a dense n x n int32 cost matrix (row-major),
 * rows bidding for columns with rewards -C_ij.  Prices and slacks are in
 * units of 1/(n + 1) of a cost, so all arithmetic is exact: the slack runs
 * eps0, eps0 / theta, eps0 / theta^2, ... (integer division, never below
 * eps_final) and each value starts a phase with every row unassigned and
 * the prices kept.  eps_final = 1 is a slack below 1/n of a cost, where the
 * result is an optimal assignment (Section 2.3.3: the plan is within n * eps
 * of the optimum, and the costs are integers); a larger eps_final gives a
 * plan within floor(n * eps_final / (n + 1)) of the optimal cost.  Bidding
 * is parallel (every unassigned row bids in each round), one workgroup per
 * instance with all state on chip.
 * plan[n]: column of each row; cost: sum of C over the plan; price[n] (may
 * be NULL): the final column prices, in the scaled units above.  stats (may
 * be NULL): levels = bidding rounds, aug_events = phases, rows_swept = bids,
 * paths = n, status.
 * Errors: OT_EINVAL (NULL C / plan / cost, n < 1, theta < 2, eps_final < 1,
 * eps0 < eps_final, ld < n), OT_ETOOBIG (n > OT_MAX_N), OT_ERANGE (eps0 >=
 * 2^50, or a price reaching 2^51: reported in status), OT_EINTERNAL (more
 * than 2^22 rounds).  ot_auction copies C from host memory and waits;
 * ot_auction_dev takes device pointers (row stride ld), runs on stream
 * (NULL = the library's stream), allocates no device memory and returns at
 * once. */
int ot_auction(const int32_t *C, int32_t n, int64_t eps0, int32_t theta, int64_t eps_final, int32_t *plan,
               int64_t *cost, int64_t *price, ot_stats *stats);
int ot_auction_dev(const int32_t *dC, int32_t n, int32_t ld, int64_t eps0, int32_t theta, int64_t eps_final,
                   int32_t *dplan, int64_t *dcost, int64_t *dprice, ot_stats *dstats, void *stream);

/* ------------------------------------------------------------------------ */
/* Serving: continuous batching of assignment requests                       */
/* ------------------------------------------------------------------------ */
/* Each request is an assignment between n source and n target points on the
 * integer grid; its cost matrix C_ij = round(sqrt((x_i - x'_j)^2 + (y_i - y'_j)^2))
 * (exact integer rounding, ties cannot occur) is built on the device, so only
 * the points cross PCIe.  A server thread admits queued requests in arrival
 * order while the device bytes of the admitted ones (8 n^2 + 64 n per
 * request: the cost matrix and its transpose) stay within hbm_budget_bytes and a slot is free, and publishes each
 * into one queue in pinned host memory.  One persistent kernel serves every
 * size (one workgroup of 512 threads per request and per CU): its workgroups
 * take requests from the queue while the server keeps appending to it, build
 * the request's matrix from its points, solve it and release the request's
 * completion flag, so a request that arrives while the kernel runs joins it
 * as soon as a workgroup is free (counted in ot_serve_counters.joined) and
 * completes as soon as its own solve does.  The kernel ends after the server
 * has been idle for a short while, and starts again with the next request.
 * Results are identical to a solve of the same request alone (the solver is
 * deterministic).  The kernel's stream is created with a CU mask naming all
 * CUs, which gives it a hardware queue of its own; such a stream is a
 * blocking stream, so work the same process puts on the legacy default
 * stream while the server's kernel runs waits for it. */
typedef struct ot_server ot_server;

/* Device cost builder used by the server, exposed on its own:
 * dC[i*n + j] = round(sqrt((src_i - dst_j)^2)) for int32 grid points
 * dsrc, ddst [2n] (x, y pairs), exact integer rounding.  Asynchronous on stream. */
int ot_grid_cost_dev(const int32_t *dsrc, const int32_t *ddst, int32_t n, int32_t *dC, void *stream);

typedef struct ot_serve_cfg {
    int64_t hbm_budget_bytes;  /* device bytes admitted requests may hold; 0 = 8 GiB */
    int32_t max_inflight;      /* request slots (1..1024); 0 = 256; 1 = one request at a time */
    int32_t streams;           /* 0..8, accepted and unused (the server runs one queue) */
    int32_t max_n;             /* largest n accepted (<= OT_MAX_N); 0 = OT_MAX_N */
    int32_t reserved[5];       /* must be zero */
} ot_serve_cfg;

typedef struct ot_result {
    int32_t *plan;             /* caller buffers [n] filled on completion (each may be NULL) */
    int64_t *u, *v;
    int64_t cost;              /* out */
    int32_t status;            /* out: ot_status of the solve */
    int32_t n;                 /* out */
    double t_submit, t_admit, t_done;  /* out: seconds on the server's monotonic clock */
} ot_result;

typedef struct ot_serve_counters {
    int64_t submitted, admitted, completed;
    int64_t groups;                /* kernel launches (the kernel starts again only after it ended) */
    int64_t peak_inflight_bytes, peak_inflight;
    int64_t joined;                /* requests published while the kernel ran and completed by it */
} ot_serve_counters;

/* Start a server on the current device.  Returns OT_OK and *out, or an error. */
int ot_serve_open(ot_server **out, const ot_serve_cfg *cfg);
/* Queue a request; src, dst are host int32 [2n] (x, y pairs), copied before
 * return.  *req_id receives an id unique within the server. */
int ot_serve_submit(ot_server *s, const int32_t *src, const int32_t *dst, int32_t n, uint64_t *req_id);
/* Wait up to timeout_us (< 0: forever) for request req_id.  OT_OK and *out
 * filled when it completed (the result is then released); 1 when still
 * pending; OT_EINVAL for an unknown id. */
int ot_serve_poll(ot_server *s, uint64_t req_id, ot_result *out, int32_t timeout_us);
/* Counters since open; now = the server clock. */
int ot_serve_stats(ot_server *s, ot_serve_counters *out, double *now);
/* Stop the server once every submitted request has completed; frees its resources. */
int ot_serve_close(ot_server *s);

/* ------------------------------------------------------------------------ */
/* Size-class schedule (autotuner)                                           */
/* ------------------------------------------------------------------------ */

/* The batch path picks a workgroup width per size class: n <= t64 uses one
 * wavefront (64 lanes), n <= t256 uses 256 lanes, larger n uses 512 lanes.
 * ot_schedule_get returns the thresholds in force; ot_schedule_set overrides
 * them (0 restores the default); ot_schedule_tune times synthetic instances
 * on the device and sets them (returns OT_OK or an error).  Each of its probes
 * holds reps times as many instances as the chip has workgroup slots at the
 * narrowest width (their matrices cycle through at most 64 distinct ones), so
 * it ranks widths by throughput; reps < 1 counts as 1. */
int ot_schedule_get(int32_t *t64, int32_t *t256);
int ot_schedule_set(int32_t t64, int32_t t256);
int ot_schedule_tune(int32_t reps);

/* The decision rule of ot_schedule_tune on a timing table, host only (no
 * device needed, nothing is set): sizes [nsizes] strictly increasing, widths
 * [nwidths] each 64, 256 or 512, ms [nsizes * nwidths] (row-major by size)
 * the time of each probe, <= 0 or NaN for a probe that was not run or failed.
 * Per size the fastest width wins (the narrower on a tie); *t64 is the
 * largest size of the contiguous prefix won by 64 lanes (at least 1), *t256
 * that of the prefix won by 64 or 256 lanes (at least *t64), so widths never
 * narrow as n grows.  OT_EINVAL for bad arguments or a size with no
 * successful probe. */
int ot_schedule_rule(int32_t nsizes, const int32_t *sizes, int32_t nwidths, const int32_t *widths,
                     const float *ms, int32_t *t64, int32_t *t256);

/* Single-instance split: an exact single-instance solve (ot_assign,
 * ot_assign_ex, ot_assign_dev, ot_assign_rect*) whose options leave both wgs
 * and block at 0 runs on `wgs` workgroups when n (the longer side) exceeds
 * n_split, else on one.  Defaults measured on MI355X: n_split = 2048, wgs = 8.
 * (Scaled solves split into 2 above n = 256 and into 4 above n = 1024.)  ot_split_set: n_split >= 0,
 * wgs 0 or 2..16, 0 restores a default (OT_EINVAL otherwise); n_split =
 * OT_MAX_N never splits.  ot_split_tune times one exact solve per size of a
 * ladder (1536 .. 4096) at 1, 4 and 8 workgroups on synthetic geometric
 * instances, on a private stream, and sets n_split to the largest size up to
 * which one workgroup stays fastest (a split must win by 2%) and wgs to the
 * count that wins at 4096.  It takes a few seconds. */
int ot_split_get(int32_t *n_split, int32_t *wgs);
int ot_split_set(int32_t n_split, int32_t wgs);
int ot_split_tune(void);

/* The decision rule of ot_split_tune on a timing table, host only: sizes
 * [nsizes] strictly increasing and <= OT_MAX_N, cands [ncands] workgroup
 * counts with cands[0] == 1 and the others in 2..16, ms [nsizes * ncands]
 * (row-major by size) all > 0.  A count wins a size when it is faster than
 * one workgroup by more than 2% and than every other count.  *n_split = the
 * largest size of the contiguous prefix won by one workgroup (sizes[0] - 1
 * when a split wins the smallest size; OT_MAX_N when none wins the largest),
 * *wgs = the count that wins the largest size (0 when none).  OT_EINVAL for
 * bad arguments. */
int ot_split_rule(int32_t nsizes, const int32_t *sizes, int32_t ncands, const int32_t *cands,
                  const float *ms, int32_t *n_split, int32_t *wgs);

#ifdef __cplusplus
}
#endif

#endif /* OTKM_H */
