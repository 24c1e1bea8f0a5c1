// Near field (P2P stage of Sec. 2.1) in FP32 on the vector ALUs.
//
// One wave per target leaf.  Target particles sit in registers; source
// particles of the leaf's P2P list are staged through LDS as float4
// (x, y, z relative to the target leaf centre, q).  A leaf holds at most
// ncrit particles, usually fewer than 64, so the wave splits into S = 64 / T
// streams (T = next power of two >= targets): lane = stream * T + target, and
// stream s takes sources s, s + S, ...  The S partial sums of each target are
// combined with cross-lane shuffles, converted to FP64 and written once.
//
// Per interaction (dx = x_t - x_s, r2 = |dx|^2, rinv = 1/sqrt(r2)):
//   phi += q rinv ;  E += q rinv^3 dx
// Pairs at zero distance only occur inside the target's own leaf, so only
// that pass carries the r2 > 0 mask.
#include "m2l_mfma.h"

namespace fmm {

namespace {

constexpr int kTile = 512;   // staged sources per wave

__device__ inline void cell_centre(const Geometry &g, int32_t cell, double *c) {
    int l = g.c.level[cell], k = g.c.inst[cell];
    const double *b = g.box + 4 * k;
    double den = ldexp(1.0, l + 1);
    c[0] = b[0] + ((double)(2 * (int64_t)g.c.ix[cell] + 1) * b[3]) / den;
    c[1] = b[1] + ((double)(2 * (int64_t)g.c.iy[cell] + 1) * b[3]) / den;
    c[2] = b[2] + ((double)(2 * (int64_t)g.c.iz[cell] + 1) * b[3]) / den;
}

__global__ void k_leaf_flag(CellArrays c, int32_t ncell, int32_t *__restrict__ flag) {
    for (int32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < ncell; i += gridDim.x * blockDim.x)
        flag[i] = (c.child[i] < 0 && c.count[i] > 0) ? 1 : 0;
}

__global__ void k_leaf_compact(const int32_t *__restrict__ flag, const int32_t *__restrict__ pos, int32_t ncell,
                               int32_t *__restrict__ leaves) {
    for (int32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < ncell; i += gridDim.x * blockDim.x)
        if (flag[i]) leaves[pos[i]] = i;
}

__global__ void k_p2p_prepare(Geometry g, int64_t n, const int32_t *__restrict__ leaf_of,
                              const double *__restrict__ xs, const double *__restrict__ ys,
                              const double *__restrict__ zs, const double *__restrict__ qs, float4 *__restrict__ pf) {
    for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < n; r += (int64_t)gridDim.x * blockDim.x) {
        double c[3];
        cell_centre(g, leaf_of[r], c);
        pf[r] = make_float4((float)(xs[r] - c[0]), (float)(ys[r] - c[1]), (float)(zs[r] - c[2]), (float)qs[r]);
    }
}

template <bool kMask>
__device__ inline void interact(const float4 *__restrict__ tile, int count, int s, int S, float xt, float yt, float zt,
                                float &ph, float &ex, float &ey, float &ez) {
    int j = s;
    for (; j + 3 * S < count; j += 4 * S) {
#pragma unroll
        for (int u = 0; u < 4; u++) {
            float4 v = tile[j + u * S];
            float dx = xt - v.x, dy = yt - v.y, dz = zt - v.z;
            float r2 = dx * dx + dy * dy + dz * dz;
            float ri = __builtin_amdgcn_rsqf(r2);
            if (kMask) ri = r2 > 0.f ? ri : 0.f;
            float qr = v.w * ri;
            float w = qr * ri * ri;
            ph += qr;
            ex += dx * w;
            ey += dy * w;
            ez += dz * w;
        }
    }
    for (; j < count; j += S) {
        float4 v = tile[j];
        float dx = xt - v.x, dy = yt - v.y, dz = zt - v.z;
        float r2 = dx * dx + dy * dy + dz * dz;
        float ri = __builtin_amdgcn_rsqf(r2);
        if (kMask) ri = r2 > 0.f ? ri : 0.f;
        float qr = v.w * ri;
        float w = qr * ri * ri;
        ph += qr;
        ex += dx * w;
        ey += dy * w;
        ez += dz * w;
    }
}

__global__ void __launch_bounds__(64) k_p2p_fp32(Geometry g, const int32_t *__restrict__ leaves,
                                                 const int32_t *__restrict__ ptr, const int32_t *__restrict__ src,
                                                 const float4 *__restrict__ pf, double *__restrict__ phi,
                                                 double *__restrict__ fld) {
    __shared__ float4 tile[kTile];
    const int lane = threadIdx.x;
    const int32_t A = leaves[blockIdx.x];
    const int32_t tf = g.c.first[A], nt = g.c.count[A];
    double cA[3];
    cell_centre(g, A, cA);
    const int32_t e0 = ptr[A], e1 = ptr[A + 1];
    for (int32_t t0 = 0; t0 < nt; t0 += 64) {
        const int ntc = nt - t0 < 64 ? nt - t0 : 64;
        int T = 1, lgT = 0;
        while (T < ntc) {
            T <<= 1;
            lgT++;
        }
        const int S = 64 >> lgT;
        const int t = lane & (T - 1), s = lane >> lgT;
        const bool active = t < ntc;
        float4 me = active ? pf[tf + t0 + t] : make_float4(0.f, 0.f, 0.f, 0.f);
        float ph = 0.f, ex = 0.f, ey = 0.f, ez = 0.f;
        // own leaf, masked (zero-distance pairs skipped)
        for (int32_t j0 = 0; j0 < nt; j0 += kTile) {
            int cnt = nt - j0 < kTile ? nt - j0 : kTile;
            __syncthreads();
            for (int j = lane; j < cnt; j += 64) tile[j] = pf[tf + j0 + j];
            __syncthreads();
            interact<true>(tile, cnt, s, S, me.x, me.y, me.z, ph, ex, ey, ez);
        }
        // the other leaves of the list, packed into tiles
        int fill = 0;
        __syncthreads();
        for (int32_t e = e0; e < e1; e++) {
            int32_t B = src[e];
            if (B == A) continue;
            double cB[3];
            cell_centre(g, B, cB);
            const float ox = (float)(cB[0] - cA[0]), oy = (float)(cB[1] - cA[1]), oz = (float)(cB[2] - cA[2]);
            const int32_t sf = g.c.first[B], ns = g.c.count[B];
            for (int32_t j0 = 0; j0 < ns; j0 += kTile) {
                int cnt = ns - j0 < kTile ? ns - j0 : kTile;
                if (fill + cnt > kTile) {
                    __syncthreads();
                    interact<false>(tile, fill, s, S, me.x, me.y, me.z, ph, ex, ey, ez);
                    __syncthreads();
                    fill = 0;
                }
                for (int j = lane; j < cnt; j += 64) {
                    float4 v = pf[sf + j0 + j];
                    tile[fill + j] = make_float4(v.x + ox, v.y + oy, v.z + oz, v.w);
                }
                fill += cnt;
            }
        }
        __syncthreads();
        interact<false>(tile, fill, s, S, me.x, me.y, me.z, ph, ex, ey, ez);
        // combine the S streams of each target
        for (int d = T; d < 64; d <<= 1) {
            ph += __shfl_xor(ph, d, 64);
            ex += __shfl_xor(ex, d, 64);
            ey += __shfl_xor(ey, d, 64);
            ez += __shfl_xor(ez, d, 64);
        }
        if (active && s == 0) {
            int64_t r = tf + t0 + t;
            phi[r] = (double)ph;
            fld[3 * r] = (double)ex;
            fld[3 * r + 1] = (double)ey;
            fld[3 * r + 2] = (double)ez;
        }
        __syncthreads();
    }
}

}  // namespace

void p2p_leaf_list(CellArrays c, int32_t ncell, int32_t *flag, int32_t *leaves, int32_t *tmp, int32_t *d_count,
                   hipStream_t s) {
    hipLaunchKernelGGL(k_leaf_flag, dim3(grid_for(ncell, 256, 4096)), dim3(256), 0, s, c, ncell, flag);
    FMM_LAUNCH_CHECK();
    // flag -> positions (flag array is reused: copy then scan)
    FMM_HIP_CHECK(hipMemcpyAsync(flag + ncell + 1, flag, ncell * sizeof(int32_t), hipMemcpyDeviceToDevice, s));
    exclusive_scan_i32(flag + ncell + 1, ncell, d_count, tmp, s);
    hipLaunchKernelGGL(k_leaf_compact, dim3(grid_for(ncell, 256, 4096)), dim3(256), 0, s, flag, flag + ncell + 1, ncell,
                       leaves);
    FMM_LAUNCH_CHECK();
}

void p2p_prepare(Geometry g, int64_t n, const int32_t *leaf_of, const double *xs, const double *ys,
                 const double *zs, const double *qs, float4 *pf, hipStream_t s) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_p2p_prepare, dim3(grid_for(n, 256, 16384)), dim3(256), 0, s, g, n, leaf_of, xs, ys, zs, qs, pf);
    FMM_LAUNCH_CHECK();
}

void p2p_fp32(Geometry g, const int32_t *leaves, int32_t nleaves, const int32_t *ptr, const int32_t *src,
              const float4 *pf, double *phi, double *fld, hipStream_t s) {
    if (nleaves <= 0) return;
    hipLaunchKernelGGL(k_p2p_fp32, dim3(nleaves), dim3(64), 0, s, g, leaves, ptr, src, pf, phi, fld);
    FMM_LAUNCH_CHECK();
}

}  // namespace fmm
