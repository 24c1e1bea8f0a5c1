// Internal launchers of the tree, list and expansion kernels.
#pragma once

#include "common.h"

namespace fmm {

// Structure-of-arrays cell table.  Cells are numbered by level, then
// instance, then Morton prefix.
struct CellArrays {
    int32_t *level, *ix, *iy, *iz;  // octree level and integer cell coordinates
    int32_t *first, *count;         // particle range in sorted order
    int32_t *child, *nchild;        // first child (-1 for leaves), number of children
    int32_t *parent, *inst;         // parent cell (-1 for roots), instance
    // The fields the traversal and the class keys read, one 16-byte record
    // per cell (one load instead of six gathers): (ix | level << 24,
    // iy | nchild << 24, iz, child).  Coordinates are below 2^21.
    int4 *rec;
};

__device__ inline int rec_level(int4 r) { return r.x >> 24; }
__device__ inline int rec_ix(int4 r) { return r.x & 0xffffff; }
__device__ inline int rec_iy(int4 r) { return r.y & 0xffffff; }
__device__ inline int rec_iz(int4 r) { return r.z; }
__device__ inline int rec_nchild(int4 r) { return r.y >> 24; }
__device__ inline int rec_child(int4 r) { return r.w; }

// ---- tree.hip
void launch_bbox(const double *pos, int64_t n, const int64_t *d_offsets, int n_inst, unsigned long long *d_ord,
                 int *d_bad, hipStream_t s);
void launch_box_finish(const unsigned long long *d_ord, int n_inst, const int64_t *d_offsets, bool user,
                       const double *ubox, double *d_box, double *d_scale, hipStream_t s);
void launch_keys(const double *pos, int64_t n, const int64_t *d_offsets, int n_inst, const double *d_box,
                 const double *d_scale, uint64_t *keys, uint32_t *idx, hipStream_t s);
void sort_by_instance(uint64_t *keys, uint32_t *idx, uint64_t *kalt, uint32_t *valt, uint32_t *ikey, uint32_t *ialt,
                      uint32_t *rank, uint32_t *ralt, int64_t n, const int64_t *d_offsets, int n_inst, int32_t *tmp,
                      hipStream_t s);
void launch_gather(const double *pos, const double *q, const uint32_t *idx, int64_t n, double *xs, double *ys,
                   double *zs, double *qs, hipStream_t s);
void launch_roots(const int64_t *d_offsets, int n_inst, CellArrays c, hipStream_t s);
void launch_tree_count(CellArrays c, int32_t lb, int32_t le, int ncrit, int max_level, const uint64_t *skeys,
                       int32_t *bounds, int32_t *nch, hipStream_t s);
void launch_tree_write(CellArrays c, int32_t lb, int32_t le, const int32_t *bounds, const int32_t *nch,
                       const int32_t *off, hipStream_t s);
// Device-driven octree levels.  lev[0 .. nlev) are level starts (level l =
// cells [lev[l], lev[l + 1])), lev[nlev] an overflow flag; init sets level 0
// to the n_inst roots.  One level step: child counts, their scan (length
// on the device, in chunks of cells) and the children, with lev[level + 2]
// set on the device; a tree past cap cells sets the flag and stops growing.
// bounds holds 9 cap ints, nch cap + 1, csum (chunk sums) cap + 1, total one.
void launch_tree_levels_init(int32_t *lev, int n_inst, int nlev, hipStream_t s);
void launch_tree_level_dev(CellArrays c, int32_t *lev, int level, int nlev, int ncrit, int max_level,
                           const uint64_t *skeys, int32_t *bounds, int32_t *nch, int32_t *csum, int32_t *total,
                           int32_t cap, hipStream_t s);
// leaf_of[r] = leaf cell of sorted particle r; *nleaf = number of leaves.
void launch_leaf_of(CellArrays c, int32_t ncell, int32_t *leaf_of, int32_t *nleaf, hipStream_t s);
// The cells with children, in cell order: ppos[c] = number of such cells
// before c (ppos[ncell] = all of them; ncell + 1 entries) and
// plist[ppos[c]] = c for each (ncell entries).  The parents of the level
// with cells [lb, le) are plist[ppos[lb] .. ppos[le]).  tmp: scan_tmp_elems(ncell).
void launch_parent_list(CellArrays c, int32_t ncell, int32_t *ppos, int32_t *plist, int32_t *tmp, hipStream_t s);
// After a frozen-topology gather: flag[0] |= 1 if a coordinate is not
// finite; with check_leaf, flag[1] |= 1 if a particle left its leaf cell
// widened by 1/8 of the side on every face (the tree no longer fits it).
void launch_refresh_check(CellArrays c, const int32_t *leaf_of, const double *xs, const double *ys, const double *zs,
                          const double *box, const double *scale, int64_t n, bool check_leaf, int32_t *flag,
                          hipStream_t s);

// ---- lists.hip
struct PairBuf {
    void *m2l;      // keys (target << bits) | source, uint32 if key32 else uint64, unsorted
    void *p2p;
    int32_t cap_m2l, cap_p2p;
    bool key32;
};
// One breadth-first step of the dual tree traversal: consumes the frontier
// whose size is *nf_in, appends accepted M2L / P2P pairs (counters[0],
// counters[1]) and the split pairs of the next frontier (*nf_out).  Counts
// keep growing past capacity so the host can detect overflow and rerun.
void launch_traverse(CellArrays c, const int2 *fin, const int32_t *nf_in, int2 *fout, int32_t *nf_out, int32_t capf,
                     PairBuf pb, int32_t *counters, int bits, uint32_t theta_num, uint32_t theta_den, hipStream_t s);
// counters[2] = number of roots put in the first frontier.
void launch_init_frontier(const int64_t *d_offsets, int n_inst, int2 *front, int32_t *counters, hipStream_t s);
// CSR from pair keys sorted by (target, source).
void launch_csr(const void *sorted, bool key32, int64_t n, int bits, int32_t ncell, int32_t *ptr, int32_t *src,
                hipStream_t s);
// Transposed CSR of a pair list: (ptr, src) lists, per owner cell, its
// partners; (ptr_t, src_t) lists, per partner, its owners (grouped by
// partner; the order within a group is not fixed).  keys and
// alt hold npair keys of 4 (key32) or 8 bytes; tmp radix_tmp_elems(npair).
void transpose_csr(const int32_t *ptr, const int32_t *src, int32_t ncell, int64_t npair, int bits, bool key32,
                   void *keys, void *alt, int32_t *tmp, int32_t *ptr_t, int32_t *src_t, hipStream_t s);

// ---- expansions.hip  (FP64, scaled solid harmonics)
struct Geometry {
    const double *box;    // per instance: min xyz, side
    CellArrays c;
};
void launch_p2m(Geometry g, int32_t ncell, int p, const double *xs, const double *ys, const double *zs,
                const double *qs, double *M, hipStream_t s);
// The parents of one level (cells [lb, le)), as launch_parent_list lists
// them, and a bound on their number that the host knows: the smaller of the
// level's and the next level's cell counts (a parent has at least one child
// there).  The translation kernels take only the parents, so a level's
// leaves cost nothing.
struct LevelParents {
    const int32_t *plist, *ppos;
    int32_t npar_max;
};
// part: scratch of 8 * npar_max * (p+1)^2 doubles.
void launch_m2m_level(Geometry g, int32_t lb, int32_t le, int p, LevelParents lp, const double *ops, double *M,
                      double *part, hipStream_t s);
void launch_l2l_level(Geometry g, int32_t lb, int32_t le, int p, LevelParents lp, const double *ops, double *L,
                      hipStream_t s);
// The outputs of an evaluation, written by the L2P kernel once a particle's
// far field is known: near + far field in input order (perm[r] = input index
// of sorted particle r); force = q E.  Null members are not written; a null
// perm writes none of them.
struct FinalOut {
    const uint32_t *perm = nullptr;
    const double *qs = nullptr, *phi_near = nullptr, *fld_near = nullptr;
    double *phi = nullptr, *field = nullptr, *force = nullptr;
};
// Far field of every sorted particle into phi / fld (and, with out.perm,
// the outputs as described above).
void launch_l2p(Geometry g, int64_t n, int p, const int32_t *leaf_of, const double *xs, const double *ys,
                const double *zs, const double *L, double *phi, double *fld, hipStream_t s,
                const FinalOut &out = FinalOut());
// Host: M2M (dir 0) or L2L (dir 1) operator matrices for the 8 octants,
// column-major P x P each (P = (p+1)^2), acting on the real coefficient layout.
std::vector<double> build_translation_ops(int p, int dir);

// ---- adjoint helpers (expansions.hip)
// Leaf rows of X scaled by s_k / S (dir 0: L2P^T from P2M) or S / s_k
// (dir 1: P2M^T through L2P); s_k = 1 (m = 0), 2 (Re), -2 (Im).
void launch_dual_scale(Geometry g, int32_t ncell, int p, double *X, int dir, hipStream_t s);
// w_i = gE[instance(i)] q_i, sorted order.
void launch_adjoint_weights(Geometry g, int64_t n, const int32_t *leaf_of, const double *gE, const double *qs,
                            double *w, hipStream_t s);
// grad_q = (g phi + psi) / 2, grad_pos = -q (g E + E_psi) / 2, in input order
// (either output may be NULL).
void launch_adjoint_finalize(Geometry g, int64_t n, const uint32_t *perm, const int32_t *leaf_of, const double *gE,
                             const double *qs, const double *phi_near, const double *fld_near, const double *phi_far,
                             const double *fld_far, const double *psi_near, const double *epsi_near,
                             const double *psi_far, const double *epsi_far, double *grad_pos, double *grad_q,
                             hipStream_t s);
// Transposes of the 8 column-major octant matrices (same layout).
std::vector<double> transpose_ops(const std::vector<double> &ops, int p);

// ---- near / far field, FP64 plain path
void launch_p2p_fp64(Geometry g, int32_t ncell, const int32_t *ptr, const int32_t *src, const double *xs,
                     const double *ys, const double *zs, const double *qs, double *phi, double *fld, hipStream_t s);
// The mutual variants (forward only; each target's sources sorted
// ascending): a pair listed in both directions is evaluated once for both
// cells, with FP64 atomics into outputs zeroed first (phi, fld of n sorted
// particles; L of every cell); pairs listed one way only are evaluated
// forward.  The order of the additions is not fixed.
void launch_p2p_fp64_mutual(Geometry g, int32_t ncell, int64_t n, const int32_t *ptr, const int32_t *src,
                            const double *xs, const double *ys, const double *zs, const double *qs, double *phi,
                            double *fld, hipStream_t s);
void launch_m2l_fp64_mutual(Geometry g, int32_t ncell, int p, const int32_t *ptr, const int32_t *src, int64_t npair,
                            const double *M, double *L, hipStream_t s);
// Per-pair FP64 M2L over the CSR list (ptr, src) of npair pairs (target-owned),
// balanced over pairs (FP64 atomics), or with owner_mode one wave per owner
// in list order (no atomics: a fixed order of additions); overwrites L
// (cells without pairs get zero).
void launch_m2l_fp64(Geometry g, int32_t ncell, int p, const int32_t *ptr, const int32_t *src, int64_t npair,
                     const double *M, double *L, bool owner_mode, hipStream_t s);
// Same, adding into L (used for the pairs the MFMA path leaves out).
void launch_m2l_fp64_add(Geometry g, int32_t ncell, int p, const int32_t *ptr, const int32_t *src, int64_t npair,
                         const double *M, double *L, bool owner_mode, hipStream_t s);
// Adjoint of the M2L stage over the transposed list (ptr_t, src_t): for every
// pair (A <- B) of the forward list, Mu_B += T_(A<-B)^T Lam_A, with T the real
// (p+1)^2 x (p+1)^2 matrix the forward kernel applies.  Owner = source cell B.
// add = 0 overwrites Mu (cells without pairs get zero), add = 1 accumulates.
void launch_m2l_fp64_adjoint(Geometry g, int32_t ncell, int p, const int32_t *ptr_t, const int32_t *src_t,
                             int64_t npair, const double *Lam, double *Mu, int add, bool owner_mode, hipStream_t s);

// ---- output
// The outputs (near + far field of every sorted particle) in input order.
void launch_finalize(int64_t n, const uint32_t *perm, const double *qs, const double *phi_near,
                     const double *fld_near, const double *phi_far, const double *fld_far, double *phi, double *field,
                     double *force, hipStream_t s);
// Energy chunk table: chunk_off[k] = first chunk of instance k (size n_inst + 1).
std::vector<int32_t> energy_chunks(const std::vector<int64_t> &offsets);
// With out.perm set (and fld_far), the energy pass also writes the outputs.
void launch_energy(const int64_t *d_offsets, int n_inst, const int32_t *d_chunk_off, int32_t nchunk, const double *qs,
                   const double *phi_near, const double *phi_far, double *part, double *energy, hipStream_t s,
                   const FinalOut &out = FinalOut(), const double *fld_far = nullptr);

}  // namespace fmm
