// Internal launchers of the class-batched MFMA M2L and the FP32 P2P.
#pragma once

#include "../../include/fmm.h"
#include "tree.h"

namespace fmm {

constexpr int kRhoMax = 24;                                  // |rho_i| covered by the dense class table
constexpr int kRhoSpan = 2 * kRhoMax + 1;
constexpr int kDeltaMax = 2;                                 // |delta| covered by the dense class table
constexpr int kDenseKeys = (2 * kDeltaMax + 1) * kRhoSpan * kRhoSpan * kRhoSpan;

// Class code of every pair: its operator slot (>= 0), -1 outside the dense
// table, -2 - key for a class that has no slot yet (its key is marked in
// used); xcount[A] = the owner's pairs outside the table.
void m2l_pair_codes(CellArrays c, int32_t ncell, const int32_t *ptr, const int32_t *src, const int32_t *slot_of,
                    int32_t *pcode, int32_t *used, int32_t *xcount, hipStream_t s);
// Slots for the marked keys (nslots[0] = slots in use, new_keys[0 ..
// nslots[1]) = the keys given one now); clears the marks.
void m2l_alloc_slots(int32_t *used, int32_t *slot_of, int32_t *nslots, int32_t *new_keys, hipStream_t s);
// The same for an empty store (slot_of all -1, nslots zero), with the slots
// given in ascending key order: slot = rank of the key among the marked
// ones, independent of thread timing.  rank holds kDenseKeys + 1 ints, tmp
// scan_tmp_elems(kDenseKeys).
void m2l_alloc_slots_ordered(int32_t *used, int32_t *slot_of, int32_t *nslots, int32_t *new_keys, int32_t *rank,
                             int32_t *tmp, hipStream_t s);
// Split-bf16 operator blocks of the new classes (op_elems bf16 per class,
// RT row tiles, layout as the work queue reads it).  transposed: the keys
// come from transposed pairs (owner = forward source) and each block holds
// the transpose of the forward pair's operator.
void m2l_build_ops(const int32_t *new_keys, int32_t nnew, const int32_t *slot_of, int p, int RT, int64_t op_elems,
                   bool transposed, uint16_t *ops, hipStream_t s);
// The same operators in FP64 for the FP64 path's matrix cores
// (v_mfma_f64_16x16x4f64 A fragments, m2l_f64_op_elems(p) doubles per class).
void m2l_build_ops_f64(const int32_t *new_keys, int32_t nnew, const int32_t *slot_of, int p, int64_t op_elems,
                       bool transposed, double *ops, hipStream_t s);
// ---- m2l_f64.hip: the FP64 path's M2L on the FP64 matrix cores over the
// class-batched tables; part receives FP64 partial locals per task (slot
// task.w, P x kGroupM2L), summed by reduce_partials_f64.
bool m2l_f64_supported(int p);
void m2l_f64_tasks(const int4 *tasks, int32_t ntask, const int32_t *ecls, const int32_t *esrc, const double *ops,
                   const double *M, int p, double *part, hipStream_t s);
inline int64_t m2l_f64_op_elems(int p) {
    const int P = ncoef(p);
    return (int64_t)((P + 3) / 4) * ((P + 15) / 16) * 64;
}
// Sort keys (level, octant, eighth, cell) of the cells with table pairs;
// xptr = exclusive scan of the per-owner counts of pairs outside the table.
void m2l_target_keys(CellArrays c, int32_t ncell, int64_t n, const int32_t *ptr, const int32_t *xptr, uint64_t *tkey,
                     int32_t *has, hipStream_t s);
// Entries of the target groups, one per distinct operator slot: count
// (slot bitmap per group in gbits, ngroup x ceil(nslot/32) words, and word
// prefixes in gwpre), then fill (after goff = exclusive scan of gcount);
// ecls[entry] = the entry's operator slot, esrc[entry][slot] its sources
// (every element written, -1 where the target has no pair of the class).
void m2l_group_count(const uint64_t *tsorted, int32_t ntarget, const int32_t *ptr, const int32_t *pcode,
                     const int32_t *slot_of, int32_t nslot, uint32_t *gbits, uint32_t *gwpre, int32_t *gcount,
                     int chunk, int32_t *tcount, hipStream_t s);
void m2l_group_fill(const uint64_t *tsorted, int32_t ntarget, const int32_t *ptr, const int32_t *src,
                    const int32_t *pcode, const int32_t *slot_of, int32_t nslot, const uint32_t *gbits,
                    const uint32_t *gwpre, const int32_t *goff, const int32_t *gcount, int32_t *ecls, int32_t *esrc,
                    int32_t *gtarget, hipStream_t s);
// *count = the number of targets (keys before the first ~0 of the sorted
// target keys).
void m2l_count_targets(const uint64_t *tsorted, int32_t ncell, int32_t *count, hipStream_t s);
// goff / toff = exclusive scans of gcount / tcount, totals[0..1] their sums;
// zeroes xcd_count[0..8] (tmp: scan scratch for very many groups).
void m2l_group_scans(const int32_t *gcount, const int32_t *tcount, int32_t ngroup, int32_t *goff, int32_t *toff,
                     int32_t *totals, int32_t *xcd_count, int32_t *tmp, hipStream_t s);
// M2L tasks ordered by (XCD, chunk index, task); xcd_count[x] = tasks of XCD x.
// max_entries bounds the entries of a group (it sizes the chunk-index bits).
void m2l_make_tasks(const int32_t *gcount, const int32_t *goff, int32_t ngroup, int chunk, int32_t max_entries,
                    const int32_t *toff,
                    const uint64_t *tsorted, int32_t ntask, int4 *tasks, int4 *tasks_alt, uint64_t *tkeys,
                    uint64_t *tkeys_alt, uint32_t *tidx, uint32_t *tidx_alt, int32_t *xcd_count, int32_t *tmp,
                    hipStream_t s);
// The pairs outside the table as a CSR list (xptr, xsrc), in list order.
void m2l_extra(const int32_t *ptr, int32_t ncell, const int32_t *src, const int32_t *pcode, const int32_t *xptr,
               int32_t *xsrc, hipStream_t s);

// ---- p2p_fp32.hip (preparation of the P2P tasks)
// Leaves ordered by (spatial eighth, cost descending); d_count[0] = number
// of leaves, d_count[1 + x] = leaves in eighth x.
// measured (nullable): per-cell durations of the previous evaluation's P2P
// tasks, used as the cost where positive.
void p2p_leaf_list(CellArrays c, int32_t ncell, int64_t n, const int32_t *p2p_ptr, const int32_t *p2p_src,
                   const float *measured, int32_t *buf, int32_t *leaves, int32_t *tmp, int32_t *d_count,
                   hipStream_t s);
void p2p_prepare(Geometry g, int64_t n, const int32_t *leaf_of, const double *xs, const double *ys,
                 const double *zs, const double *qs, float4 *pf, hipStream_t s);
void cell_centres(Geometry g, int32_t ncell, double *centre, hipStream_t s);

}  // namespace fmm
