/*
 * fmm.h -- C ABI of the MI355X (gfx950) fast multipole library for the 3-D
 * Laplace N-body problem of Ltaief & Yokota, "Data-Driven Execution of Fast
 * Multipole Methods" (arXiv:1203.0889).
 *
 * Problem (Sec. 2.1): N bodies with positions x_i and charges q_i; the
 * "solution on the particle" is the potential and field
 *     phi_i = sum_{j : |x_i - x_j| > 0} q_j / |x_i - x_j|
 *     E_i   = -grad phi (x_i) = sum_j q_j (x_i - x_j) / |x_i - x_j|^3
 * (unit Coulomb constant, pairs at zero distance contribute nothing), and the
 * force F_i = q_i E_i.  The FMM approximates these with an adaptive cubic
 * octree (Sec. 2.1, 2.2), a dual tree traversal producing M2L / P2P pair
 * lists (Sec. 4), and the six stages P2M, M2M, M2L, P2P, L2L, L2P (Sec. 2.1,
 * Fig. 1).  The paper's multicore task runtime (Sec. 3) is replaced by a
 * device-side work queue.
 *
 * Conventions for every entry point:
 *   - Every call returns fmm_status; FMM_OK == 0.  No call aborts or exits.
 *   - Pointers documented "device" must point to device memory of the plan's
 *     device; "host" to host memory.  The caller owns every buffer it passes;
 *     the library owns everything inside the plan.
 *   - All device work is enqueued on the plan's stream and is asynchronous
 *     with respect to the host, except where stated.  Host-side argument
 *     checks fail synchronously with FMM_ERR_INVALID_ARG / FMM_ERR_STATE and
 *     leave the plan unchanged.
 *   - Device arrays of vectors are row-major (N, 3) FP64: x0 y0 z0 x1 ...
 *   - Results are in the caller's (input) particle order.
 *   - A plan is not thread safe; one plan per stream.
 */
#ifndef FMM_MI355X_H
#define FMM_MI355X_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    FMM_OK = 0,
    FMM_ERR_INVALID_ARG = -1, /* bad pointer, size or parameter */
    FMM_ERR_STATE = -2,       /* call out of order (see state machine) */
    FMM_ERR_OOM = -3,         /* device allocation failed */
    FMM_ERR_DEVICE = -4,      /* a HIP runtime call failed */
    FMM_ERR_CAPACITY = -5,    /* an internal capacity limit was exceeded */
    FMM_ERR_UNSUPPORTED = -6  /* valid request the library does not provide */
} fmm_status;

typedef enum {
    FMM_PREC_FP64 = 0,  /* every stage in FP64 (the plain GPU path) */
    FMM_PREC_MIXED = 1  /* P2P on FP32 VALU; M2L on bf16 MFMA with split
                           operands (x = x_hi + x_lo, three products, FP32
                           accumulation); tree, P2M, M2M, L2L, L2P and the
                           per-particle / per-cell accumulation in FP64 */
} fmm_precision;

enum {
    FMM_FLAG_USER_BOX = 1u << 0,     /* use params.box_min / box_side for every
                                        instance instead of the tight bounding cube */
    FMM_FLAG_KEEP_TOPOLOGY = 1u << 1, /* a later fmm_build_tree with the same n_inst
                                        and offsets keeps the box, keys, tree and
                                        lists of the previous build and only takes
                                        the new positions and charges (gathered by
                                        the stored sort permutation): a frozen
                                        topology, as finite-difference checks of
                                        the adjoint need */
    FMM_FLAG_DETERMINISTIC = 1u << 3, /* bitwise reproducible results: every
                                        floating-point sum is taken in a fixed
                                        order (each target's sources sorted in
                                        the lists, per-owner FP64 M2L of the
                                        pairs outside the class table without
                                        atomics); the work queue's M2L sums are
                                        in a fixed order in every mode */
    FMM_FLAG_TRACE = 1u << 2,         /* mixed precision: the work queue of
                                        fmm_evaluate records one fmm_task_record
                                        per task it runs (fmm_get_trace) */
    FMM_FLAG_INCREMENTAL = 1u << 4,   /* time stepping: a later fmm_build_tree with
                                        the same n_inst and offsets keeps the
                                        topology (as FMM_FLAG_KEEP_TOPOLOGY) while
                                        every particle, in its stored sort order,
                                        lies inside its old leaf cell widened by
                                        1/8 of the cell's side on every face; it
                                        rebuilds from scratch otherwise.  The
                                        widening scales every cell's radius by
                                        at most 5/4, so an accepted pair's
                                        separation ratio (Sec. 2.1) stays below
                                        5/4 theta: the expansions converge
                                        (needs 5 num < 4 den, else
                                        FMM_ERR_INVALID_ARG at fmm_create) and
                                        the worst-case truncation bound is that
                                        of theta' = 5/4 theta.
                                        fmm_get_build_info counts both kinds of
                                        build */
    FMM_FLAG_COST_REUSE = 1u << 5,    /* mixed precision: the work queue measures
                                        the duration of every P2P task (device
                                        clock, one store per task), and a kept-
                                        topology rebuild (KEEP_TOPOLOGY /
                                        INCREMENTAL, also inside a graph of
                                        fmm_graph_capture_step) orders the next
                                        evaluation's P2P tasks by those
                                        durations instead of the estimated
                                        costs (Sec. 2.2: the previous step's
                                        work as the weights) */
    FMM_FLAG_MUTUAL_M2L = 1u << 6,    /* FP64 precision: the mutual interaction
                                        (Sec. 4) for M2L: each pair listed in
                                        both directions is evaluated once for
                                        both cells, with one set of irregular
                                        harmonics (the reverse direction takes
                                        the sign flip of the odd terms), both
                                        cells' locals added with FP64 atomics;
                                        M2L then runs per pair rather than
                                        over the class tables */
    FMM_FLAG_MUTUAL_P2P = 1u << 7,    /* FP64 precision: the mutual interaction
                                        for P2P: each leaf pair listed in both
                                        directions is evaluated once for both
                                        leaves (one distance and inverse square
                                        root per particle pair), both leaves'
                                        sums added with FP64 atomics */
    FMM_FLAG_MUTUAL = (1u << 6) | (1u << 7) /* both.  Neither is allowed with
                                        FMM_PREC_MIXED or FMM_FLAG_DETERMINISTIC
                                        (FMM_ERR_INVALID_ARG at fmm_create);
                                        fmm_backward is unchanged */
};

typedef struct {
    int32_t p;           /* expansion order: every degree 0..p kept; 0 <= p <= 16 */
    int32_t ncrit;       /* leaf size limit: a cell with more particles is split (Sec. 2.1) */
    int32_t theta_num;   /* multipole acceptance ratio theta = num / den, exact rational, */
    int32_t theta_den;   /*   1 <= num, den <= 100, 0 < theta < 1 (Sec. 2.1, Sec. 4) */
    int32_t max_level;   /* deepest octree level, 1 <= max_level <= 21 (63-bit keys) */
    int32_t precision;   /* fmm_precision */
    uint32_t flags;      /* FMM_FLAG_* */
    double box_min[3];   /* used with FMM_FLAG_USER_BOX */
    double box_side;     /*   (must enclose every particle) */
} fmm_params;

/* Fill *params with defaults: p = 8, ncrit = 64, theta = 1/2,
 * max_level = 21, mixed precision, no flags. */
fmm_status fmm_default_params(fmm_params *params);

typedef struct fmm_plan fmm_plan; /* opaque; owns all device workspaces */

/* Create a plan on HIP device `device` that enqueues on `hip_stream`
 * (a hipStream_t; NULL = the null stream).  params is copied.  Parameters
 * are checked first (FMM_ERR_INVALID_ARG, before any device call); a
 * device index with no device behind it, or one that cannot be selected,
 * is FMM_ERR_DEVICE. */
fmm_status fmm_create(const fmm_params *params, int device, void *hip_stream, fmm_plan **out);

/* Release every device allocation of the plan.  First waits for the plan's
 * stream and for every internal stream of the plan, so no kernel of the
 * plan still runs on its memory.  NULL is accepted. */
fmm_status fmm_destroy(fmm_plan *plan);

/*
 * Build keys, sort, octree and interaction lists (Sec. 2.1, 2.2, 4).
 *   n_inst   number of independent instances (>= 1), batched in one forest
 *   offsets  host int64[n_inst + 1], offsets[0] = 0, non-decreasing;
 *            instance k owns particles [offsets[k], offsets[k+1])
 *   pos      device FP64 (N, 3), N = offsets[n_inst]; finite values
 *   q        device FP64 (N)
 * Copies what it needs; pos and q may be reused once the stream reaches the
 * end of this call.  Synchronises the stream internally (sizes of the tree
 * and lists are read back).  Non-finite coordinates -> FMM_ERR_INVALID_ARG.
 * Empty instances (N_k = 0) are allowed.
 */
fmm_status fmm_build_tree(fmm_plan *plan, int32_t n_inst, const int64_t *offsets,
                          const double *pos, const double *q);

/* Upward pass: P2M at leaves, M2M to the roots (Sec. 2.1).  Requires a
 * built tree. */
fmm_status fmm_upward(fmm_plan *plan);

/*
 * Downward pass and near field: M2L and P2P through the device work queue,
 * then L2L and L2P (Sec. 2.1, Sec. 4).  Requires fmm_upward.  Each output
 * is optional (NULL skips it):
 *   phi     device FP64 (N)      potential
 *   field   device FP64 (N, 3)   E = -grad phi
 *   force   device FP64 (N, 3)   F = q E
 *   energy  device FP64 (n_inst) E_k = 1/2 sum_{i in k} q_i phi_i
 */
fmm_status fmm_evaluate(fmm_plan *plan, double *phi, double *field, double *force, double *energy);

/*
 * fmm_evaluate for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same outputs from the same kernels as fmm_evaluate, with no hipMalloc,
 * hipFree or other allocation.  Every workspace of the plan must already be
 * large enough for the current tree (an earlier fmm_evaluate on the plan
 * sizes them, also for any later smaller tree); otherwise FMM_ERR_STATE,
 * before or while work is enqueued (the outputs are then undefined).  The
 * work queue's claim counters and the energy's chunk partials live in a
 * fixed device array of 1 MiB per GPU (each GPU the library runs on holds it
 * until the process ends): an energy needing more than 131,040 chunk
 * partials (about 1,024 particles each, one chunk at least per instance) is
 * FMM_ERR_CAPACITY.  Calls on one GPU share that array: calls that overlap
 * on one GPU (plans on different streams without ordering between them)
 * race, and must be ordered by the caller.
 */
fmm_status fmm_evaluate_noalloc(fmm_plan *plan, double *phi, double *field, double *force, double *energy);

/*
 * Adjoint: gradient of the FMM total energy, sum_k g_k E_k with
 * E_k = 1/2 q_k^T A q_k, with respect to positions and charges, where A is
 * the matrix the FMM applies (P2M, M2M, M2L, L2L, L2P and P2P over the built
 * lists; not symmetric, since the M2L lists are not, Sec. 4: the mutual
 * flags evaluate the same pairs).  Computed exactly
 * for that A, in the plan's precision: with w = g q and psi = A^T w (a
 * transposed evaluation: L2P^T, L2L^T, M2L^T, P2P^T, M2M^T, P2M^T),
 *   grad_q_i   = (g_i phi_i + psi_i) / 2
 *   grad_pos_i = -q_i (g_i E_i + E^psi_i) / 2,   E^psi = -grad psi.
 * The box and cell geometry are held fixed (the topology of the build).
 * Requires fmm_evaluate on the same plan; its first call after a build also
 * builds the transposed lists.
 *   grad_energy  device FP64 (n_inst) upstream weights g_k
 *   grad_pos     device FP64 (N, 3), input order (NULL skips)
 *   grad_q       device FP64 (N), input order (NULL skips)
 */
fmm_status fmm_backward(fmm_plan *plan, const double *grad_energy, double *grad_pos, double *grad_q);

/*
 * Record the numeric part of a solve into a HIP graph owned by the plan:
 * fmm_upward, fmm_evaluate into the given outputs and, when grad_energy is
 * non-NULL, fmm_backward into grad_pos / grad_q (arguments as for those
 * calls; the pointers are baked into the graph and must stay valid while it
 * is used).  The tree and lists of the last fmm_build_tree are fixed in the
 * graph: a replay recomputes everything downstream of the sorted particle
 * data, e.g. after a frozen-topology fmm_build_tree (FMM_FLAG_KEEP_TOPOLOGY)
 * with new charges or positions.  The build itself is not captured: it reads
 * tree and list sizes back to size its buffers and launches.  Runs the
 * sequence once eagerly (sizing every workspace), synchronises, then
 * captures on the plan's stream.  A full rebuild or fmm_destroy drops the
 * graph.
 */
fmm_status fmm_graph_capture(fmm_plan *plan, double *phi, double *field, double *force, double *energy,
                             const double *grad_energy, double *grad_pos, double *grad_q);

/*
 * Record one whole time step into the plan's graph: the frozen-topology
 * fmm_build_tree from pos / q (device, layouts as for fmm_build_tree; read
 * at every replay, so the caller writes the next step's positions there),
 * fmm_upward and fmm_evaluate into the given outputs.  Needs a built tree
 * and FMM_FLAG_KEEP_TOPOLOGY or FMM_FLAG_INCREMENTAL; with INCREMENTAL a
 * replay also checks that every particle stays inside its widened leaf cell
 * and fmm_sync then returns FMM_ERR_STATE when one left it (the step's
 * outputs are then not to be used: rebuild with fmm_build_tree and capture
 * again).  A non-finite coordinate makes fmm_sync return
 * FMM_ERR_INVALID_ARG.  Runs the step once eagerly, then captures it as
 * fmm_graph_capture does.  N = 0: FMM_ERR_INVALID_ARG.
 */
fmm_status fmm_graph_capture_step(fmm_plan *plan, const double *pos, const double *q, double *phi, double *field,
                                  double *force, double *energy);

/* Replay the captured graph on the plan's stream (asynchronous). */
fmm_status fmm_graph_launch(fmm_plan *plan);

/* Wait for the plan's stream; returns the first device-detected error
 * recorded since the last call (e.g. FMM_ERR_CAPACITY), else FMM_OK. */
fmm_status fmm_sync(fmm_plan *plan);

/* Sizes of the built tree and lists (host outputs; any may be NULL). */
fmm_status fmm_get_counts(const fmm_plan *plan, int64_t *ncell, int64_t *nleaf, int64_t *nm2l,
                          int64_t *np2p);

/* Number of fmm_build_tree calls that built the tree from scratch and of
 * those that kept the previous topology (host outputs; any may be NULL).
 * The eager step of fmm_graph_capture_step counts as a kept build; graph
 * replays are not counted. */
fmm_status fmm_get_build_info(const fmm_plan *plan, int64_t *full_builds, int64_t *kept_builds);

/*
 * Sizes of the work-queue tables of the mixed path after fmm_build_tree
 * (host outputs; any may be NULL): the target cells of the batched M2L
 * (cells owning at least one pair of the class table, Sec. 4 lists regrouped
 * by class), their groups of 256, the M2L tasks (the task size is the
 * paper's granularity knob, Sec. 5), the operator classes in use, and the
 * M2L pairs left to the per-pair FP64 kernel.  The FP64 path reports the
 * same class tables, which its FP64 matrix-core M2L runs over for p <= 12
 * (no P2P tasks; every count is 0 above p = 12 and with
 * FMM_FLAG_MUTUAL_M2L, whose M2L runs per pair).  Before a build:
 * FMM_ERR_STATE.
 */
fmm_status fmm_get_queue_info(const fmm_plan *plan, int64_t *ntarget, int64_t *ngroup, int64_t *ntask,
                              int64_t *nclass, int64_t *nextra);

/*
 * Copy the tree to host memory (synchronous).  Cells are in canonical order:
 * by level, then instance, then Morton prefix.
 *   keys   host uint64[N]: Morton key of every particle, input order
 *   perm   host int64[N]:  perm[r] = input index of the r-th sorted particle
 *   cells  host int64[ncell * 10]: per cell
 *          [level, ix, iy, iz, first, count, child_first, nchild, parent, instance]
 *          (first is a sorted rank; child_first = -1 for leaves)
 * Any pointer may be NULL.
 */
fmm_status fmm_copy_tree(const fmm_plan *plan, uint64_t *keys, int64_t *perm, int64_t *cells);

/*
 * Copy the interaction lists, sorted by (target cell, source cell), as CSR
 * over target cells (synchronous).  host int64 m2l_ptr[ncell + 1],
 * int32 m2l_src[nm2l], p2p_ptr[ncell + 1], p2p_src[np2p].  Any may be NULL.
 * (On the device the lists are grouped by target only; the sources of each
 * target are sorted here, on the host.)
 */
fmm_status fmm_copy_lists(const fmm_plan *plan, int64_t *m2l_ptr, int32_t *m2l_src, int64_t *p2p_ptr,
                          int32_t *p2p_src);

/*
 * Tuning knobs of the work queue and kernels (an autotuner fills them).
 * Results change only within rounding (the M2L sums of a task follow the
 * task size) or not at all (the launch shape).
 */
typedef struct {
    int32_t m2l_task_entries; /* M2L class entries per work-queue task (1..128; default
                                 128 with FMM_PREC_MIXED, 32 with FMM_PREC_FP64, whose
                                 matrix-core M2L runs its tasks as one plain launch) */
    int32_t grid_per_cu;      /* persistent work-queue workgroups per compute unit (1..8) */
    int32_t p2p_per_cu;       /* P2P-only workgroups per compute unit launched beside the
                                 work queue on a second stream of the plan (0..8); with 0
                                 the work-queue workgroups of a compute unit alternate
                                 between starting with M2L and with P2P tasks, otherwise
                                 all of them start with M2L */
    int32_t early_p2p_per_cu; /* of those, workgroups per compute unit started by
                                 fmm_build_tree as soon as the near field's inputs exist
                                 (the P2P lists; Sec. 3: a task runs once its inputs are
                                 ready), beside the upward pass and the far-field build
                                 (0..p2p_per_cu; 0: the near field starts with the work
                                 queue; not with FMM_FLAG_TRACE) */
} fmm_tuning;

fmm_status fmm_get_tuning(const fmm_plan *plan, fmm_tuning *tuning);
/* Takes effect at the next fmm_build_tree (task tables are built there). */
fmm_status fmm_set_tuning(fmm_plan *plan, const fmm_tuning *tuning);

/*
 * Autotuner of the work queue (the paper tunes its task granularity Q,
 * Sec. 5): on the plan's current tree and multipoles (after fmm_upward),
 * times one evaluation (fmm_evaluate without outputs: the queue, the far
 * field that runs beside its P2P tail, the join) for m2l_task_entries in
 * {32, 64, 96, 128} and (grid_per_cu, p2p_per_cu) in {(1, 1), (1, 2),
 * (1, 3), (2, 0), (3, 0), (2, 1), (2, 2)}; early_p2p_per_cu is kept as set
 * (at most p2p_per_cu), since its gain depends on the build it overlaps
 * (the task tables are rebuilt per
 * m2l_task_entries; each setting takes the fastest of `repeats` >= 1 runs,
 * HIP events on the plan's stream), keeps the fastest setting and rebuilds
 * the tables with it.  Outputs (host, may be NULL): the chosen tuning and
 * its time in ms.  Leaves the plan as after fmm_upward (call
 * fmm_evaluate again); drops a captured graph.  The FP64 path has no queue:
 * it times m2l_task_entries in {16, 32, 64, 128} for its matrix-core M2L
 * over the class tables (the other fields kept); where its M2L runs per
 * pair (p > 12, FMM_FLAG_MUTUAL_M2L) the call only reports the current
 * tuning and time -1.
 */
fmm_status fmm_autotune(fmm_plan *plan, int32_t repeats, fmm_tuning *best, double *best_ms);

/* Per-stage device times of the last build / upward / evaluate in ms,
 * measured with HIP events on the plan's stream.  times: host double[16],
 * names: optional host array of 16 const char* filled with stage names. */
fmm_status fmm_get_stage_times(const fmm_plan *plan, double *times, const char **names);

/*
 * Device task trace (the per-task timeline the paper draws for its runtime,
 * Sec. 5): with FMM_FLAG_TRACE, every task the work queue of the last
 * fmm_evaluate ran, in completion order.  Times are ticks of the device's
 * constant 100 MHz real-time clock (s_memrealtime), from the claim of the
 * task to its completion (for an M2L task: all four waves of its workgroup
 * done).  hw_id is the raw HW_ID register of the recording wave: compute
 * unit bits 11:8, SIMD 5:4, shader array 12, shader engine 15:13; xcc is the
 * XCD.
 */
typedef struct {
    uint64_t start, end;
    int32_t kind;    /* 0 = M2L task (one workgroup), 1 = P2P task (one wave) */
    int32_t task;    /* M2L: index in the plan's task table; P2P: target leaf cell */
    int32_t kernel;  /* 0 = k_queue, 1 = k_p2p_side */
    uint32_t hw_id;
    uint32_t xcc;
    uint32_t reserved;
} fmm_task_record;

/* Copy up to cap records of the last traced queue run to host memory
 * (synchronous); *count (host, may be NULL) receives the number recorded.
 * Without FMM_FLAG_TRACE, or before fmm_evaluate, *count = 0.  The FP64
 * path has no queue and records nothing. */
fmm_status fmm_get_trace(const fmm_plan *plan, fmm_task_record *records, int64_t cap, int64_t *count);

const char *fmm_status_string(fmm_status status);
/* Last error message of this plan (host-side detail), never NULL. */
const char *fmm_last_error(const fmm_plan *plan);

#ifdef __cplusplus
}
#endif
#endif /* FMM_MI355X_H */
