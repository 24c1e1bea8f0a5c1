// Preparation of the near-field (P2P) tasks of the work queue: the leaf
// list ordered costliest first, FP32 particles relative to their leaf
// centre, and the FP64 centre of every cell.
#include "m2l_mfma.h"

namespace fmm {

namespace {

__device__ inline void centre_of(const Geometry &g, int32_t cell, double *c) {
    int l = g.c.level[cell], k = g.c.inst[cell];
    const double *b = g.box + 4 * k;
    double den = ldexp(1.0, l + 1);
    c[0] = b[0] + ((double)(2 * (int64_t)g.c.ix[cell] + 1) * b[3]) / den;
    c[1] = b[1] + ((double)(2 * (int64_t)g.c.iy[cell] + 1) * b[3]) / den;
    c[2] = b[2] + ((double)(2 * (int64_t)g.c.iz[cell] + 1) * b[3]) / den;
}

__global__ void k_centres(Geometry g, int32_t ncell, double *__restrict__ centre) {
    for (int32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < ncell; i += gridDim.x * blockDim.x) {
        double c[3];
        centre_of(g, i, c);
        centre[3 * i] = c[0];
        centre[3 * i + 1] = c[1];
        centre[3 * i + 2] = c[2];
    }
}

// Leaf cost = targets x sources over its P2P list (one wave per cell).  Sort
// key (16 bits) = (spatial eighth of the particle order) << 13 |
// (8191 - q), q = 1 + min(8190, 200 log2(cost + 1)): ascending order groups
// leaves by eighth (the XCD that runs them) and puts the costliest first
// within each (to the resolution of q; equal keys keep cell order).
// Non-leaves get 0xffff, after every leaf.
// With measured (durations of the previous evaluation's P2P tasks, by
// cell; 0 where none was measured) the measured cost replaces the estimate.
__global__ void k_leaf_cost(CellArrays c, int32_t ncell, int64_t n, const int32_t *__restrict__ ptr,
                            const int32_t *__restrict__ src, const float *__restrict__ measured,
                            uint32_t *__restrict__ key, uint32_t *__restrict__ val) {
    const int lane = threadIdx.x & 63;
    const float inv_n8 = 8.0f / (float)n;
    for (int32_t i = blockIdx.x * blockDim.x / 64 + threadIdx.x / 64; i < ncell; i += gridDim.x * blockDim.x / 64) {
        const bool leaf = c.child[i] < 0 && c.count[i] > 0;
        uint64_t cost = 0;
        if (leaf) {
            // four 64-entry chunks at once (all their loads in flight), then
            // the rest of a long list chunk by chunk
            const int32_t e0 = ptr[i], e1 = ptr[i + 1];
            int32_t sidx[4];
#pragma unroll
            for (int u = 0; u < 4; u++) {
                const int32_t e = e0 + u * 64 + lane;
                sidx[u] = e < e1 ? src[e] : -1;
            }
#pragma unroll
            for (int u = 0; u < 4; u++)
                if (sidx[u] >= 0) cost += (uint64_t)c.count[sidx[u]];
            for (int32_t e = e0 + 256 + lane; e < e1; e += 64) cost += (uint64_t)c.count[src[e]];
        }
#pragma unroll
        for (int d = 32; d > 0; d >>= 1) cost += __shfl_xor(cost, d, 64);
        if (lane == 0) {
            uint32_t k = 0xffffu;
            if (leaf) {
                // an ordering heuristic only: FP32 log2 and a floating-point
                // eighth (a 64-bit integer division or an FP64 log2 costs
                // a wave hundreds of instructions)
                cost *= (uint64_t)c.count[i];
                if (measured && measured[i] > 0.0f) cost = (uint64_t)measured[i];
                int c8 = (int)((float)c.first[i] * inv_n8);
                c8 = c8 > 7 ? 7 : c8;
                const float lq = 200.0f * __log2f((float)cost + 1.0f);
                const uint32_t q = 1u + (uint32_t)(lq < 8190.0f ? lq : 8190.0f);
                k = ((uint32_t)c8 << 13) | (8191u - q);
            }
            key[i] = k;
            val[i] = (uint32_t)i;
        }
    }
}

// From the sorted keys: count[0] = leaves, count[1 + x] = leaves of eighth
// x (lower bounds of the eighth boundaries; no atomics).
__global__ void k_leaf_counts(const uint32_t *__restrict__ skey, int32_t ncell, int32_t *__restrict__ count) {
    __shared__ int32_t lb[9];
    const int x = threadIdx.x;
    if (x < 9) {
        const uint32_t want = x < 8 ? (uint32_t)x << 13 : 0xffffu;   // first key of eighth x; non-leaves
        int32_t a = 0, b = ncell;
        while (a < b) {
            const int32_t mid = a + ((b - a) >> 1);
            if (skey[mid] < want) a = mid + 1; else b = mid;
        }
        lb[x] = a;
    }
    __syncthreads();
    if (x == 0) count[0] = lb[8];
    else if (x < 9) count[x] = lb[x] - lb[x - 1];
}

__global__ void k_p2p_prepare(Geometry g, int64_t n, const int32_t *__restrict__ leaf_of,
                              const double *__restrict__ xs, const double *__restrict__ ys,
                              const double *__restrict__ zs, const double *__restrict__ qs, float4 *__restrict__ pf) {
    for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < n; r += (int64_t)gridDim.x * blockDim.x) {
        double c[3];
        centre_of(g, leaf_of[r], c);
        pf[r] = make_float4((float)(xs[r] - c[0]), (float)(ys[r] - c[1]), (float)(zs[r] - c[2]), (float)qs[r]);
    }
}

}  // namespace

// buf holds 4 * (ncell + 1) ints: keys, values, alternate keys/values.
void p2p_leaf_list(CellArrays c, int32_t ncell, int64_t n, const int32_t *p2p_ptr, const int32_t *p2p_src,
                   const float *measured, int32_t *buf, int32_t *leaves, int32_t *tmp, int32_t *d_count,
                   hipStream_t s) {
    uint32_t *key = (uint32_t *)(buf + (ncell + 1));
    uint32_t *kalt = (uint32_t *)(buf + 2 * (ncell + 1));
    uint32_t *valt = (uint32_t *)(buf + 3 * (ncell + 1));
    uint32_t *val = (uint32_t *)leaves;
    if (ncell <= 0) {
        fill_zero(d_count, 9 * sizeof(int32_t), s);
        return;
    }
    hipLaunchKernelGGL(k_leaf_cost, dim3(grid_for((int64_t)ncell * 64, 256, 16384)), dim3(256), 0, s, c, ncell, n,
                       p2p_ptr, p2p_src, measured, key, val);
    FMM_LAUNCH_CHECK();
    radix_sort_u32(key, val, kalt, valt, ncell, 0, 16, tmp, s);
    hipLaunchKernelGGL(k_leaf_counts, dim3(1), dim3(64), 0, s, key, ncell, d_count);
    FMM_LAUNCH_CHECK();
}

void p2p_prepare(Geometry g, int64_t n, const int32_t *leaf_of, const double *xs, const double *ys,
                 const double *zs, const double *qs, float4 *pf, hipStream_t s) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_p2p_prepare, dim3(grid_for(n, 256, 16384)), dim3(256), 0, s, g, n, leaf_of, xs, ys, zs, qs, pf);
    FMM_LAUNCH_CHECK();
}

void cell_centres(Geometry g, int32_t ncell, double *centre, hipStream_t s) {
    if (ncell <= 0) return;
    hipLaunchKernelGGL(k_centres, dim3(grid_for(ncell, 256, 4096)), dim3(256), 0, s, g, ncell, centre);
    FMM_LAUNCH_CHECK();
}

}  // namespace fmm
