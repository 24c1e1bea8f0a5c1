// Internal interface of the persistent work-queue kernel (M2L + P2P tasks).
#pragma once

#include "tree.h"

namespace fmm {

constexpr int kGroupM2L = 64;   // targets per M2L task group (one wave, two MFMA column tiles)
constexpr int kMaxTaskEntries = 128;  // class entries per M2L task (the wave keeps two slots per lane)

struct QueueArgs {
    CellArrays c;
    const double *centre;      // per cell geometric centre (x, y, z), FP64
    // M2L
    const int4 *m2l_tasks;     // (group, entry begin, entry end, 0)
    const int32_t *gtarget;    // group x 128 target cells (-1 = empty slot)
    const int32_t *ecls;       // entry -> compact class id
    const int32_t *esrc;       // entry x 128 source cells (-1 = absent)
    const int32_t *slot_of_cid;
    const float *frags;        // class operators, MFMA fragment order
    const float *M32;          // multipoles, FP32, row stride 2 * KS4 (zero padded),
                               //   plus one all-zero row at index zero_row
    int32_t zero_row;
    double *L;                 // FP64 local expansions (accumulated)
    int P;
    // P2P
    const int32_t *leaves;     // leaf cells, costliest first
    int32_t nleaves;
    const int32_t *p2p_ptr, *p2p_src;
    const float4 *pf;          // particles: (x, y, z) - own leaf centre, q
    double *phi, *fld;         // FP64 near field per sorted particle
    // queue: 16 task lists, list 2x = M2L tasks of XCD x, list 2x+1 = P2P
    // tasks of XCD x.  lists[L] = (first M2L task, task count, first leaf, 0);
    // P2P task t of a list is leaf first + t.
    const int4 *lists;
    int32_t *heads;            // 16 claim counters (zeroed before launch)
};

bool queue_supported(int p);
// Row tiles of 32 and padded half-K (multiple of 4) of the MFMA layout.
void queue_layout(int p, int *RT, int *KS4);
// Floats per class operator in the fragment store (padded to whole
// 256-thread float4 loads; the padding is zero).
int64_t queue_frag_floats(int p);
// M32 must hold (ncell + 1) rows of 2 * KS4 floats; row ncell is zero.
void queue_pad_multipoles(const double *M, int32_t ncell, int p, float *M32, hipStream_t s);
void queue_run(const QueueArgs &a, int p, int nworkgroups, hipStream_t s);

}  // namespace fmm
