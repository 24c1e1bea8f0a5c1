// Internal interface of the mixed-precision near/far field stage: P2P tasks
// (FP32 VALU) and class-batched M2L tasks (split-bf16 MFMA, FP32 accumulation).
#pragma once

#include "../../include/fmm.h"
#include "tree.h"

namespace fmm {

struct NearFarArgs {
    Geometry g;
    int32_t ncell;
    int64_t nleaf, n, nm2l;
    int p;
    const int32_t *m2l_ptr, *m2l_src, *p2p_ptr, *p2p_src;
    const int32_t *leaf_of;
    const double *xs, *ys, *zs, *qs;
    const double *M;   // FP64 multipoles (input)
    double *L;         // FP64 locals (output, overwritten)
    double *phi, *fld; // FP64 near field per sorted particle (output)
    fmm_tuning tuning;
    // Adjoint use: the lists are the transposed ones (owner = forward
    // source), M holds the duals of the locals, L receives the duals of the
    // multipoles, qs the adjoint weights; operators are stored transposed.
    bool transposed = false;
    bool deterministic = false;    // fixed order of every floating-point addition
    // the FP64 path's tables: operators in FP64 for its matrix cores, no
    // P2P task lists (its P2P is the FP64 kernel)
    bool f64 = false;
    HostReader *reader = nullptr;  // fast device-to-host reads (optional)
    int32_t *heads = nullptr;      // 16 claim counters of the queue (null: the state's own)
    const float *leaf_cost = nullptr;   // measured P2P task durations by cell, read for the order (nullable)
    float *cost_out = nullptr;          // the work queue writes its P2P task durations here (nullable)
    // task trace of the queue (optional): records, counter, capacity
    fmm_task_record *trace = nullptr;
    int32_t *trace_count = nullptr;
    int32_t trace_cap = 0;
    // set when build_p2p_leaves already ran on another stream: the build
    // waits for this event instead of building the P2P leaf order itself
    hipEvent_t p2p_ready = nullptr;
};

// Device workspaces of this stage, owned by the plan.  The class operator
// store (slot_of, frags) persists across builds of the same plan.
struct NearFarState {
    DevBuf used, slot_of, nslots, new_keys, frags;
    DevBuf pcode, xcount, tkey, tkey_alt, has, gcount, goff, tcount, toff;
    DevBuf ecls, esrc, gtarget, tasks, xsrc, xptr, leafbuf, leaves, pf, M32, tmp, cnt, centre, gbits, gwpre;
    DevBuf tasks_alt, tkeys, tidx, lists, tmp2;
    DevBuf part;   // per-task FP32 partial locals of the M2L tasks
    DevBuf key_rank;   // deterministic mode: ranks of the marked class keys
    DevBuf frags64, part64;   // FP64 path: FP64 class operators, FP64 task partials
    // streams and events of the P2P side kernels (created on first use):
    // side (launched with the queue), side2 (the deferred tail), side3 (the
    // early near field)
    hipStream_t side = nullptr, side2 = nullptr, side3 = nullptr;
    hipEvent_t fork = nullptr, join = nullptr, after_queue = nullptr, after_side = nullptr;
    bool tail_pending = false;   // a deferred queue whose P2P tail is not launched yet
    bool tail_side = false, tail_early = false;   // what the pending tail joins
    // a P2P side kernel of the current particles was started early
    // (near_far_start_p2p, early_wg workgroups) with these claim counters
    // and not yet joined by a queue
    bool early = false;
    int early_wg = 0;
    const int32_t *early_heads = nullptr;
    hipEvent_t early_fork = nullptr, early_done = nullptr;
    bool f64 = false;            // built for the FP64 path (FP64 operators, no task lists)
    int p = -1;
    int32_t nslot_total = 0, nslot = 0, ngroup = 0, ntarget = 0, nentries = 0, ntask = 0, nextra = 0;
    bool built = false;
};

fmm_tuning default_tuning();
// M2L class entries per task of the FP64 path's matrix-core M2L by default
// (one plain launch over its tasks, so smaller tasks than the work queue's)
constexpr int kFp64TaskEntries = 32;
// Build-time part (after the lists): classes, operators, groups, tasks.
void build_near_far_mixed(NearFarState &st, const NearFarArgs &a, hipStream_t s);
// The P2P leaf order and the cell centres (needs only the tree and the P2P
// lists), for a second stream.
void build_p2p_leaves(NearFarState &st, const NearFarArgs &a, hipStream_t s);
// The P2P leaf order again (a.leaf_cost: measured costs) and the 16 task
// lists, on a kept topology.
void reorder_p2p_leaves(NearFarState &st, const NearFarArgs &a, hipStream_t s);
// Start the near field as soon as its inputs exist (the paper's data-driven
// order: P2P needs neither the upward pass nor the far-field tables): zero
// the claim counters on `from`, then on the side stream the FP32 particles
// and the P2P side kernel.  Needs the P2P leaf order and task lists
// (build_p2p_leaves) and the near-field outputs sized.  The next
// near_far_queue joins the running kernel instead of launching one.
// Returns false (nothing started) without side workgroups or with a trace.
bool near_far_start_p2p(NearFarState &st, const NearFarArgs &a, hipStream_t from);
// Make s wait for an early P2P kernel that no queue joined (before its
// inputs or outputs change); no-op otherwise.
void near_far_drop_early(NearFarState &st, hipStream_t s);
// Evaluate-time part, in stream order: inputs of the queue (bf16 multipoles,
// FP32 particles, zeroed locals), the work-queue kernel (M2L and P2P tasks),
// then the per-pair FP64 M2L of the pairs outside the class table.
void near_far_prepare(NearFarState &st, const NearFarArgs &a, hipStream_t s);
// defer_join: see queue_run; then near_far_join(st, s) before the near
// field is read.  Returns whether the join was deferred.
// *joined_early: the queue joined an early P2P kernel.
bool near_far_queue(NearFarState &st, const NearFarArgs &a, hipStream_t s, bool defer_join = false,
                    bool *joined_early = nullptr);
// The deferred P2P tail: more P2P workgroups once the work queued on s so
// far (the far field) is done, then the join event.
void near_far_tail(NearFarState &st, const NearFarArgs &a, hipStream_t s);
void near_far_join(NearFarState &st, hipStream_t s);
// The stream on which a deferred queue's join is recorded.
hipStream_t near_far_join_stream(const NearFarState &st);
// After the queue (in stream order): the per-pair FP64 M2L of the pairs
// outside the class table added to the locals.
void near_far_rest(NearFarState &st, const NearFarArgs &a, hipStream_t s);
// The FP64 path's M2L over the class tables (built with a.f64): zeroed
// locals, the FP64 matrix-core tasks, their partials summed in task order,
// then the per-pair FP64 M2L of the pairs outside the class table.
void m2l_f64_run(NearFarState &st, const NearFarArgs &a, hipStream_t s);
void release_near_far(NearFarState &st);

}  // namespace fmm
