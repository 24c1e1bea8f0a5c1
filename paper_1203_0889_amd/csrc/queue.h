// Internal interface of the persistent work-queue kernel (M2L + P2P tasks).
#pragma once

#include "../../include/fmm.h"
#include "tree.h"

namespace fmm {

constexpr int kGroupM2L = 256;  // targets per M2L task group (4 waves x 64)
constexpr int kMaxTaskEntries = 128;  // class entries per M2L task (a wave keeps two slots per lane)

struct QueueArgs {
    CellArrays c;
    const double *centre;      // per cell geometric centre (x, y, z), FP64
    // M2L
    const int4 *m2l_tasks;     // (group, entry begin, entry end, partial slot)
    const int32_t *gtarget;    // group x kGroupM2L target cells (-1 = empty slot)
    const int32_t *ecls;       // entry -> operator slot of its class
    const int32_t *esrc;       // entry x kGroupM2L source cells (-1 = absent)
    const uint16_t *ops;       // class operators, split bf16 MFMA blocks (queue_op_elems per class)
    const uint16_t *Mb;        // multipoles, split bf16 rows (queue_mrow_elems per cell),
                               //   plus one all-zero row at index zero_row
    int32_t zero_row;
    float *part;               // per-task FP32 partial locals: slot x P x kGroupM2L
    int P;
    // the pass after k_queue that sums each group's partials into the
    // locals: group task ranges (toff, tcount), group count, FP64 locals
    const int32_t *toff, *tcount;
    int32_t ngroup;
    double *L;
    // P2P
    const int32_t *leaves;     // leaf cells, by XCD, costliest first
    const int32_t *p2p_ptr, *p2p_src;
    const float4 *pf;          // particles: (x, y, z) - own leaf centre, q
    double *phi, *fld;         // FP64 near field per sorted particle
    // queue: 16 task lists, list 2x = M2L tasks of XCD x, list 2x+1 = P2P
    // tasks of XCD x.  lists[L] = (first M2L task, task count, first leaf, 0);
    // P2P task t of a list is leaf first + t.
    const int4 *lists;
    int32_t *heads;            // 16 claim counters (zeroed before launch)
    int32_t role_split;        // set by queue_run
    int32_t m2l_only;          // set by queue_run: k_queue leaves the P2P tasks to k_p2p_side
    // task trace (null: off): records, their counter (zeroed before the
    // launch) and capacity; records past the capacity are dropped
    fmm_task_record *trace;
    int32_t *trace_count;
    int32_t trace_cap;
    // measured P2P task durations (null: off): leaf_cost[leaf] = device
    // clock ticks of the leaf's task, one plain store per task
    float *leaf_cost;
};

bool queue_supported(int p);
// The sum of the FP64 path's per-task partial locals (the same layout in
// FP64): L[gtarget[g][s]][k] = sum_j part[toff[g] + j][k][s] in task order.
void reduce_partials_f64(const double *part, const int32_t *toff, const int32_t *tcount, const int32_t *gtarget,
                         int32_t ngroup, int p, double *L, hipStream_t s);
// Floats of one task's partial locals (P coefficients x kGroupM2L targets).
inline int64_t queue_part_elems(int p) { return (int64_t)ncoef(p) * kGroupM2L; }

// Row tiles of 32 of the M2L operator; the contraction dimension is padded
// to 32 RT as well (2 RT MFMA k-steps of 16).
int queue_row_tiles(int p);
// bf16 elements per class operator: 2 RT k-steps x RT row tiles x 2 pieces
// (hi, lo) x 64 lanes x 8.
int64_t queue_op_elems(int p);
// bf16 elements per multipole row: 2 RT k-steps x 4 (hi, lo for each half
// of the k-step) x 8.
int64_t queue_mrow_elems(int p);
// Split the FP64 multipoles into bf16 (hi, lo) rows; Mb must hold ncell + 1
// rows, row ncell is written as zero.
void queue_split_multipoles(const double *M, int32_t ncell, int p, uint16_t *Mb, hipStream_t s);
// The work queue on stream s: nworkgroups persistent workgroups of k_queue
// followed on s by the sum of the M2L partials into the locals:
// L[gtarget[g][s]][k] = sum_j part[toff[g] + j][k][s], j < tcount[g], in
// task order in FP64 (no atomics, so the locals do not depend on which task
// ends first); cells outside every group keep their locals (zeroed before);
// and, if nside > 0, nside P2P-only workgroups on the stream `side`, forked
// from and joined back into s with the events fork and join.  Without side
// workgroups the k_queue workgroups sharing a compute unit alternate which
// task type they start with; with them every k_queue workgroup starts with
// M2L and the side kernel drains the P2P tasks beside it.
// Streams and events of the side kernels (created by the caller).
struct QueueStreams {
    hipStream_t side = nullptr, side2 = nullptr;
    hipEvent_t fork = nullptr, join = nullptr, after_queue = nullptr, after_side = nullptr;
    // an early P2P kernel (queue_p2p_start) on its own stream, joined with
    // the side kernels (null: none)
    hipStream_t early = nullptr;
    hipEvent_t early_done = nullptr;
};
// defer_join (with side workgroups): k_queue runs the M2L tasks only and the
// side kernel drains the P2P tasks; s does not wait for it: the caller
// queues more work on s, then queue_tail, and waits for the join before it
// reads the near field.
// With qs.early: a P2P kernel already runs there (queue_p2p_start, the
// claim counters zeroed before it); nside more side workgroups join it and
// the join covers both.
// Returns whether the join was deferred.
bool queue_run(const QueueArgs &a, int p, int nworkgroups, int nside, const QueueStreams &qs, hipStream_t s,
               bool defer_join = false);
// The P2P side kernel alone, nside workgroups on stream side: the near
// field started as soon as its inputs exist (the claim counters must be
// zeroed before, in stream order).
void queue_p2p_start(const QueueArgs &a, int nside, hipStream_t side);
// The deferred P2P tail (after queue_run returned true): nworkgroups more
// P2P-only workgroups on side2 once the work queued on s so far is done,
// and the join event recorded after every P2P launch.
void queue_tail(const QueueArgs &a, int nworkgroups, const QueueStreams &qs, hipStream_t s);

}  // namespace fmm
