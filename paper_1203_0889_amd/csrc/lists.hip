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

__global__ void k_traverse(CellArrays c, const int2 *__restrict__ fin, int32_t nf, int2 *__restrict__ fout,
                           int32_t capf, PairBuf pb, int32_t *__restrict__ counters, uint32_t ta, uint32_t tb) {
    for (int32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < nf; i += gridDim.x * blockDim.x) {
        int2 pr = fin[i];
        int32_t A = pr.x, B = pr.y;
        int la = c.level[A], lb = c.level[B];
        int32_t chA = c.child[A], chB = c.child[B];
        bool leafA = chA < 0, leafB = chB < 0;
        if (A != B && mac_exact(la, c.ix[A], c.iy[A], c.iz[A], lb, c.ix[B], c.iy[B], c.iz[B], ta, tb)) {
            int32_t slot = atomicAdd(&counters[1], 1);
            if (slot < pb.cap_m2l) pb.m2l[slot] = ((uint64_t)(uint32_t)A << 32) | (uint32_t)B;
        } else if (leafA && leafB) {
            int32_t slot = atomicAdd(&counters[2], 1);
            if (slot < pb.cap_p2p) pb.p2p[slot] = ((uint64_t)(uint32_t)A << 32) | (uint32_t)B;
        } else if (!leafB && (leafA || la > lb)) {
            int k = c.nchild[B];
            int32_t slot = atomicAdd(&counters[0], k);
            for (int j = 0; j < k; j++)
                if (slot + j < capf) fout[slot + j] = make_int2(A, chB + j);
        } else {
            int k = c.nchild[A];
            int32_t slot = atomicAdd(&counters[0], k);
            for (int j = 0; j < k; j++)
                if (slot + j < capf) fout[slot + j] = make_int2(chA + j, B);
        }
    }
}

__global__ void k_init_frontier(const int64_t *__restrict__ offsets, int n_inst, int2 *__restrict__ front,
                                int32_t *__restrict__ counters) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    int32_t nf = 0;
    for (int k = 0; k < n_inst; k++)
        if (offsets[k + 1] > offsets[k]) front[nf++] = make_int2(k, k);
    counters[0] = nf;
    counters[1] = 0;
    counters[2] = 0;
}

__global__ void k_repack(uint64_t *__restrict__ pairs, int64_t n, int bits) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        uint64_t v = pairs[i];
        pairs[i] = ((v >> 32) << bits) | (v & 0xffffffffull);
    }
}

__global__ void k_csr(const uint64_t *__restrict__ sorted, int64_t n, int bits, int32_t ncell, int32_t *__restrict__ ptr,
                      int32_t *__restrict__ src) {
    const uint64_t mask = (1ull << bits) - 1;
    int64_t tid = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = tid; i < n; i += stride) src[i] = (int32_t)(sorted[i] & mask);
    for (int64_t cidx = tid; cidx <= ncell; cidx += stride) {
        uint64_t want = (uint64_t)cidx << bits;
        int64_t a = 0, b = n;
        while (a < b) {
            int64_t mid = (a + b) >> 1;
            if (sorted[mid] < want) a = mid + 1; else b = mid;
        }
        ptr[cidx] = (int32_t)a;
    }
}

}  // namespace

void launch_traverse(CellArrays c, const int2 *fin, int32_t nf, int2 *fout, int32_t capf, PairBuf pb,
                     int32_t *counters, uint32_t theta_num, uint32_t theta_den, hipStream_t s) {
    if (nf <= 0) return;
    hipLaunchKernelGGL(k_traverse, dim3(grid_for(nf, 256, 16384)), dim3(256), 0, s, c, fin, nf, fout, capf, pb, counters,
                       theta_num, theta_den);
    FMM_LAUNCH_CHECK();
}

void launch_init_frontier(const int64_t *d_offsets, int n_inst, int2 *front, int32_t *counters, hipStream_t s) {
    hipLaunchKernelGGL(k_init_frontier, dim3(1), dim3(64), 0, s, d_offsets, n_inst, front, counters);
    FMM_LAUNCH_CHECK();
}

void launch_repack(uint64_t *pairs, int64_t n, int bits, hipStream_t s) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_repack, dim3(grid_for(n, 256, 16384)), dim3(256), 0, s, pairs, n, bits);
    FMM_LAUNCH_CHECK();
}

void launch_csr(const uint64_t *sorted, int64_t n, int bits, int32_t ncell, int32_t *ptr, int32_t *src,
                hipStream_t s) {
    int64_t work = n > ncell + 1 ? n : ncell + 1;
    hipLaunchKernelGGL(k_csr, dim3(grid_for(work, 256, 16384)), dim3(256), 0, s, sorted, n, bits, ncell, ptr, src);
    FMM_LAUNCH_CHECK();
}

}  // namespace fmm
