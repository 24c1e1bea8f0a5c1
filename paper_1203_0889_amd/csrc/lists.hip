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

// One BFS step.  The frontier size is read from device memory (clamped to
// the buffer capacity), so all steps are enqueued without host round trips.
// Each workgroup stages its accepted pairs and its next-frontier pairs in
// LDS and reserves global space with one atomic per flush: same-address
// atomics are few, and global writes are contiguous.
constexpr int kTravThreads = 256;
constexpr int kBufM = 2048;   // staged M2L keys
constexpr int kBufP = 1024;   // staged P2P keys
constexpr int kBufF = 4096;   // staged frontier pairs (one tile adds at most 8 per thread)

template <class K>
__device__ inline void flush_keys(K *__restrict__ buf, int32_t &cnt, K *__restrict__ out, int32_t cap,
                                  int32_t *__restrict__ gcount, int32_t *sh_base) {
    if (threadIdx.x == 0) *sh_base = atomicAdd(gcount, cnt);
    __syncthreads();
    int32_t base = *sh_base;
    for (int j = threadIdx.x; j < cnt; j += kTravThreads)
        if (base + j < cap) out[base + j] = buf[j];
    __syncthreads();
    if (threadIdx.x == 0) cnt = 0;
    __syncthreads();
}

template <class K>
__global__ void __launch_bounds__(kTravThreads) k_traverse(CellArrays c, const int2 *__restrict__ fin,
                                                           const int32_t *__restrict__ nf_in, int2 *__restrict__ fout,
                                                           int32_t *__restrict__ nf_out, int32_t capf,
                                                           K *__restrict__ m2l, K *__restrict__ p2p, int32_t cap_m2l,
                                                           int32_t cap_p2p, int32_t *__restrict__ n_m2l,
                                                           int32_t *__restrict__ n_p2p, int bits, uint32_t ta,
                                                           uint32_t tb) {
    __shared__ K bm[kBufM];
    __shared__ K bp[kBufP];
    __shared__ int2 bf[kBufF];
    __shared__ int32_t cm, cp, cf, base_sh;
    int32_t nf = *nf_in;
    nf = nf < capf ? nf : capf;
    if (threadIdx.x == 0) cm = cp = cf = 0;
    __syncthreads();
    const int32_t stride = gridDim.x * kTravThreads;
    for (int32_t base = blockIdx.x * kTravThreads; base < nf; base += stride) {
        int32_t i = base + threadIdx.x;
        if (i < nf) {
            int2 pr = fin[i];
            int32_t A = pr.x, B = pr.y;
            const int4 ra = c.rec[A], rb = c.rec[B];
            int la = rec_level(ra), lb = rec_level(rb);
            int32_t chA = rec_child(ra), chB = rec_child(rb);
            bool leafA = chA < 0, leafB = chB < 0;
            const K key = ((K)(uint32_t)A << bits) | (K)(uint32_t)B;
            if (A != B &&
                mac_exact(la, rec_ix(ra), rec_iy(ra), rec_iz(ra), lb, rec_ix(rb), rec_iy(rb), rec_iz(rb), ta, tb)) {
                bm[atomicAdd(&cm, 1)] = key;
            } else if (leafA && leafB) {
                bp[atomicAdd(&cp, 1)] = key;
            } else if (!leafB && (leafA || la > lb)) {
                int k = rec_nchild(rb);
                int32_t o = atomicAdd(&cf, k);
                for (int j = 0; j < k; j++) bf[o + j] = make_int2(A, chB + j);
            } else {
                int k = rec_nchild(ra);
                int32_t o = atomicAdd(&cf, k);
                for (int j = 0; j < k; j++) bf[o + j] = make_int2(chA + j, B);
            }
        }
        __syncthreads();
        // a tile adds at most 256 keys per list and 2048 frontier pairs
        if (cm > kBufM - kTravThreads) flush_keys<K>(bm, cm, m2l, cap_m2l, n_m2l, &base_sh);
        if (cp > kBufP - kTravThreads) flush_keys<K>(bp, cp, p2p, cap_p2p, n_p2p, &base_sh);
        if (cf > kBufF - 8 * kTravThreads) flush_keys<int2>(bf, cf, fout, capf, nf_out, &base_sh);
    }
    __syncthreads();
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
    if (key32) {
        if (npair > 0) {
            hipLaunchKernelGGL(k_swap_pairs<uint32_t>, dim3(grid_for((int64_t)ncell * 64, 256, 4096)), dim3(256), 0, s,
                               ptr, src, ncell, bits, (uint32_t *)keys);
            FMM_LAUNCH_CHECK();
        }
        radix_sort_u32((uint32_t *)keys, nullptr, (uint32_t *)alt, nullptr, npair, bits, 2 * bits, tmp, s);
    } else {
        if (npair > 0) {
            hipLaunchKernelGGL(k_swap_pairs<uint64_t>, dim3(grid_for((int64_t)ncell * 64, 256, 4096)), dim3(256), 0, s,
                               ptr, src, ncell, bits, (uint64_t *)keys);
            FMM_LAUNCH_CHECK();
        }
        radix_sort_u64((uint64_t *)keys, nullptr, (uint64_t *)alt, nullptr, npair, bits, 2 * bits, tmp, s);
    }
    launch_csr(keys, key32, npair, bits, ncell, ptr_t, src_t, s);
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
