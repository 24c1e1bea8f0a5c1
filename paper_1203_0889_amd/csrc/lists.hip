// Dual tree traversal (Sec. 4) as a breadth-first, level-synchronous device
// loop.  Every frontier pair gets a pure decision that depends only on the
// two cells, so the resulting sets do not depend on traversal order:
//   A != B and MAC(A, B)            -> M2L (A <- B), target-owned (non-mutual)
//   A and B both leaves             -> P2P (A <- B)
//   B not a leaf and (A is a leaf
//     or A is smaller than B)       -> split the source B
//   otherwise                       -> split the target A (ties split A,
//                                      as in the first traversal step)
// MAC (cell size over distance, Sec. 2.1): with theta = a/b, half-diagonal
// radii and centres in half grid units,
//     3 b^2 (S_A + S_B)^2 < a^2 |C_A - C_B|^2 ,  strict,
// evaluated exactly in 64-bit integers (a, b <= 100 keeps every term below
// 2^63).  Accepted pairs are appended with atomics and sorted afterwards,
// which makes the final lists canonical: sorted by (target, source).
#include "tree.h"

namespace fmm {

namespace {

__device__ inline bool mac_exact(int la, int ax, int ay, int az, int lb, int bx, int by, int bz, uint64_t a,
                                 uint64_t b) {
    int64_t SA = (int64_t)1 << (kLevels - la), SB = (int64_t)1 << (kLevels - lb);
    int64_t dx = (2 * (int64_t)ax + 1) * SA - (2 * (int64_t)bx + 1) * SB;
    int64_t dy = (2 * (int64_t)ay + 1) * SA - (2 * (int64_t)by + 1) * SB;
    int64_t dz = (2 * (int64_t)az + 1) * SA - (2 * (int64_t)bz + 1) * SB;
    uint64_t d2 = (uint64_t)(dx * dx) + (uint64_t)(dy * dy) + (uint64_t)(dz * dz);
    uint64_t s = (uint64_t)(SA + SB);
    return 3ull * b * b * s * s < a * a * d2;
}

// One BFS step, two tree levels deep.  Every frontier pair is decided;
// a pair that is split has its (at most 8) child pairs decided at once, in
// the same thread, and only the child pairs that must be split again go to
// the next frontier.  Compared with one level per step this halves the
// steps and keeps the pairs that resolve at the next level (most of the
// last levels' pairs) out of the frontier buffers.  The frontier size is
// read from device memory (clamped to the buffer capacity), so all steps
// are enqueued without host round trips.  Each workgroup stages its
// accepted pairs and its next-frontier pairs in LDS and reserves global
// space with one atomic per flush: same-address atomics are few, and
// global writes are contiguous.
constexpr int kTravThreads = 256;
constexpr int kTileOut = 8 * kTravThreads;   // most entries one tile adds to one buffer
// Staging sizes: flushes reserve global space with same-address atomics,
// which serialise across the chip, so the buffers are as large as two
// workgroups per compute unit allow (32-bit keys: 80 KB of LDS).
template <class K>
struct TravBuf {
    static constexpr int M = sizeof(K) == 4 ? 4 * kTileOut : kTileOut + 1024;   // M2L keys
    static constexpr int P = sizeof(K) == 4 ? 2 * kTileOut : kTileOut + 1024;   // P2P keys
    static constexpr int F = sizeof(K) == 4 ? 2 * kTileOut - 64 : kTileOut;     // next-frontier pairs
};

// Barrier for LDS traffic only: global loads in flight (the prefetched
// pairs and records of the next tiles) stay in flight.
__device__ inline void lds_barrier() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

template <class K>
__device__ inline void flush_keys(K *__restrict__ buf, int32_t &cnt, K *__restrict__ out, int32_t cap,
                                  int32_t *__restrict__ gcount, int32_t *sh_base) {
    if (threadIdx.x == 0) *sh_base = atomicAdd(gcount, cnt);
    lds_barrier();
    int32_t base = *sh_base;
    for (int j = threadIdx.x; j < cnt; j += kTravThreads)
        if (base + j < cap) out[base + j] = buf[j];
    lds_barrier();
    if (threadIdx.x == 0) cnt = 0;
    lds_barrier();
}

// The pure decision of one pair: M2L, P2P, or split (staged in LDS).
template <class K>
__device__ inline void decide(int32_t A, int32_t B, int4 ra, int4 rb, int bits, uint32_t ta, uint32_t tb,
                              K *__restrict__ bm, int32_t &cm, K *__restrict__ bp, int32_t &cp, bool &split) {
    split = false;
    const K key = ((K)(uint32_t)A << bits) | (K)(uint32_t)B;
    if (A != B && mac_exact(rec_level(ra), rec_ix(ra), rec_iy(ra), rec_iz(ra), rec_level(rb), rec_ix(rb), rec_iy(rb),
                            rec_iz(rb), ta, tb))
        bm[atomicAdd(&cm, 1)] = key;
    else if (rec_child(ra) < 0 && rec_child(rb) < 0)
        bp[atomicAdd(&cp, 1)] = key;
    else
        split = true;
}

// Each thread takes one frontier pair per tile.  The loads are software
// pipelined: while a tile is decided, the records of the next tile and the
// pair of the one after are in flight (indices clamped to the last pair, so
// every load is unconditional and in bounds).
template <class K>
__global__ void __launch_bounds__(kTravThreads) k_traverse(CellArrays c, const int2 *__restrict__ fin,
                                                           const int32_t *__restrict__ nf_in, int2 *__restrict__ fout,
                                                           int32_t *__restrict__ nf_out, int32_t capf,
                                                           K *__restrict__ m2l, K *__restrict__ p2p, int32_t cap_m2l,
                                                           int32_t cap_p2p, int32_t *__restrict__ n_m2l,
                                                           int32_t *__restrict__ n_p2p, int bits, uint32_t ta,
                                                           uint32_t tb) {
    __shared__ K bm[TravBuf<K>::M];
    __shared__ K bp[TravBuf<K>::P];
    __shared__ int2 bf[TravBuf<K>::F];
    __shared__ int32_t cm, cp, cf, base_sh;
    int32_t nf = *nf_in;
    nf = nf < capf ? nf : capf;
    if (nf <= 0) return;
    if (threadIdx.x == 0) cm = cp = cf = 0;
    lds_barrier();
    const int32_t stride = gridDim.x * kTravThreads;
    const int32_t last = nf - 1;
    int32_t i = blockIdx.x * kTravThreads + threadIdx.x;
    int2 pr = fin[i < last ? i : last];
    int4 ra = c.rec[pr.x], rb = c.rec[pr.y];
    int2 pn = fin[i + stride < last ? i + stride : last];
    for (int32_t base = blockIdx.x * kTravThreads; base < nf; base += stride, i += stride) {
        const int4 na = c.rec[pn.x], nb = c.rec[pn.y];
        const int2 pnn = fin[i + 2 * stride < last ? i + 2 * stride : last];
        if (i < nf) {
            const int32_t A = pr.x, B = pr.y;
            bool split;
            decide<K>(A, B, ra, rb, bits, ta, tb, bm, cm, bp, cp, split);
            if (split) {
                // split the source if it is not a leaf and the target is a
                // leaf or smaller; otherwise the target (ties split the target)
                const bool sb = rec_child(rb) >= 0 && (rec_child(ra) < 0 || rec_level(ra) > rec_level(rb));
                const int4 rs = sb ? rb : ra, ro = sb ? ra : rb;
                const int32_t first = rec_child(rs), k = rec_nchild(rs), other = sb ? A : B;
                int4 rc[8];
#pragma unroll
                for (int j = 0; j < 8; j++) rc[j] = c.rec[first + (j < k ? j : k - 1)];
#pragma unroll
                for (int j = 0; j < 8; j++) {
                    if (j < k) {
                        const int32_t X = sb ? other : first + j, Y = sb ? first + j : other;
                        bool again;
                        decide<K>(X, Y, sb ? ro : rc[j], sb ? rc[j] : ro, bits, ta, tb, bm, cm, bp, cp, again);
                        if (again) bf[atomicAdd(&cf, 1)] = make_int2(X, Y);
                    }
                }
            }
        }
        lds_barrier();
        if (cm > TravBuf<K>::M - kTileOut) flush_keys<K>(bm, cm, m2l, cap_m2l, n_m2l, &base_sh);
        if (cp > TravBuf<K>::P - kTileOut) flush_keys<K>(bp, cp, p2p, cap_p2p, n_p2p, &base_sh);
        if (cf > TravBuf<K>::F - kTileOut) flush_keys<int2>(bf, cf, fout, capf, nf_out, &base_sh);
        pr = pn;
        ra = na;
        rb = nb;
        pn = pnn;
    }
    lds_barrier();
    if (cm > 0) flush_keys<K>(bm, cm, m2l, cap_m2l, n_m2l, &base_sh);
    if (cp > 0) flush_keys<K>(bp, cp, p2p, cap_p2p, n_p2p, &base_sh);
    if (cf > 0) flush_keys<int2>(bf, cf, fout, capf, nf_out, &base_sh);
}

// counters: [0] = #M2L, [1] = #P2P, [2 + k] = size of frontier k.
__global__ void k_init_frontier(const int64_t *__restrict__ offsets, int n_inst, int2 *__restrict__ front,
                                int32_t *__restrict__ counters) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    int32_t nf = 0;
    for (int k = 0; k < n_inst; k++)
        if (offsets[k + 1] > offsets[k]) front[nf++] = make_int2(k, k);
    counters[2] = nf;
}

template <class K>
__global__ void k_csr(const K *__restrict__ sorted, int64_t n, int bits, int32_t ncell, int32_t *__restrict__ ptr,
                      int32_t *__restrict__ src) {
    const K mask = (K)(((uint64_t)1 << bits) - 1);
    int64_t tid = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = tid; i < n; i += stride) src[i] = (int32_t)(sorted[i] & mask);
    for (int64_t cidx = tid; cidx <= ncell; cidx += stride) {
        K want = (K)((uint64_t)cidx << bits);
        int64_t a = 0, b = n;
        while (a < b) {
            int64_t mid = (a + b) >> 1;
            if (sorted[mid] < want) a = mid + 1; else b = mid;
        }
        ptr[cidx] = (int32_t)a;
    }
}

// Pair keys of the transposed list: (other << bits) | owner for every entry
// of the CSR list (owner, other).  One wave per owner cell.
template <class K>
__global__ void k_swap_pairs(const int32_t *__restrict__ ptr, const int32_t *__restrict__ src, int32_t ncell, int bits,
                             K *__restrict__ out) {
    const int32_t waves = (int32_t)(gridDim.x * (blockDim.x / 64));
    for (int32_t A = (int32_t)(blockIdx.x * (blockDim.x / 64) + threadIdx.x / 64); A < ncell; A += waves)
        for (int32_t e = ptr[A] + (int32_t)(threadIdx.x & 63); e < ptr[A + 1]; e += 64)
            out[e] = ((K)src[e] << bits) | (K)A;
}

}  // namespace

void transpose_csr(const int32_t *ptr, const int32_t *src, int32_t ncell, int64_t npair, int bits, bool key32,
                   void *keys, void *alt, int32_t *tmp, int32_t *ptr_t, int32_t *src_t, hipStream_t s) {
    bool in_alt = false;   // an odd number of passes leaves the sorted pairs in alt
    if (key32) {
        if (npair > 0) {
            hipLaunchKernelGGL(k_swap_pairs<uint32_t>, dim3(grid_for((int64_t)ncell * 64, 256, 4096)), dim3(256), 0, s,
                               ptr, src, ncell, bits, (uint32_t *)keys);
            FMM_LAUNCH_CHECK();
        }
        radix_sort_u32((uint32_t *)keys, nullptr, (uint32_t *)alt, nullptr, npair, bits, 2 * bits, tmp, s, &in_alt);
    } else {
        if (npair > 0) {
            hipLaunchKernelGGL(k_swap_pairs<uint64_t>, dim3(grid_for((int64_t)ncell * 64, 256, 4096)), dim3(256), 0, s,
                               ptr, src, ncell, bits, (uint64_t *)keys);
            FMM_LAUNCH_CHECK();
        }
        radix_sort_u64((uint64_t *)keys, nullptr, (uint64_t *)alt, nullptr, npair, bits, 2 * bits, tmp, s, &in_alt);
    }
    launch_csr(in_alt ? alt : keys, key32, npair, bits, ncell, ptr_t, src_t, s);
}

void launch_traverse(CellArrays c, const int2 *fin, const int32_t *nf_in, int2 *fout, int32_t *nf_out, int32_t capf,
                     PairBuf pb, int32_t *counters, int bits, uint32_t theta_num, uint32_t theta_den, hipStream_t s) {
    dim3 grid(1024), block(kTravThreads);
    if (pb.key32)
        hipLaunchKernelGGL(k_traverse<uint32_t>, grid, block, 0, s, c, fin, nf_in, fout, nf_out, capf,
                           (uint32_t *)pb.m2l, (uint32_t *)pb.p2p, pb.cap_m2l, pb.cap_p2p, counters, counters + 1, bits,
                           theta_num, theta_den);
    else
        hipLaunchKernelGGL(k_traverse<uint64_t>, grid, block, 0, s, c, fin, nf_in, fout, nf_out, capf,
                           (uint64_t *)pb.m2l, (uint64_t *)pb.p2p, pb.cap_m2l, pb.cap_p2p, counters, counters + 1, bits,
                           theta_num, theta_den);
    FMM_LAUNCH_CHECK();
}

void launch_init_frontier(const int64_t *d_offsets, int n_inst, int2 *front, int32_t *counters, hipStream_t s) {
    hipLaunchKernelGGL(k_init_frontier, dim3(1), dim3(64), 0, s, d_offsets, n_inst, front, counters);
    FMM_LAUNCH_CHECK();
}

void launch_csr(const void *sorted, bool key32, int64_t n, int bits, int32_t ncell, int32_t *ptr, int32_t *src,
                hipStream_t s) {
    int64_t work = n > ncell + 1 ? n : ncell + 1;
    if (key32)
        hipLaunchKernelGGL(k_csr<uint32_t>, dim3(grid_for(work, 256, 16384)), dim3(256), 0, s, (const uint32_t *)sorted, n,
                           bits, ncell, ptr, src);
    else
        hipLaunchKernelGGL(k_csr<uint64_t>, dim3(grid_for(work, 256, 16384)), dim3(256), 0, s, (const uint64_t *)sorted, n,
                           bits, ncell, ptr, src);
    FMM_LAUNCH_CHECK();
}

}  // namespace fmm
