// The device-side work queue of the near/far field stage.
//
// The paper schedules M2L and P2P work as tasks of adjustable granularity
// on a multicore runtime (Sec. 3, 4); here one persistent kernel plays that
// role on the GPU.  Workgroups (4 waves) claim tasks from a global counter
// until the list is exhausted; tasks are ordered largest first.
//   * M2L task: a group of 128 target cells (same level and octant, Morton
//     order) and a range of its class entries.  Per entry the class
//     operator T_c (FP32, pre-swizzled MFMA fragments) is staged in LDS and
//     shared by the 4 waves; each wave owns 32 targets and runs
//     v_mfma_f32_32x32x2_f32 with A = T_c, B = the 32 gathered multipoles.
//     The next entry's operator and multipoles are prefetched into
//     registers while the current one is applied.  Results are added into
//     the FP64 local expansions.
//   * P2P task: 4 target leaves, one per wave.  Sources are staged in the
//     wave's private LDS tile as float4 relative to the target centre.  A
//     leaf of nt targets is covered by one pass per set bit b of nt, with
//     2^b targets x 64/2^b source streams, so every lane works whatever nt
//     is; streams are combined with cross-lane shuffles.
// Target-owned writes (each target cell or particle belongs to one task)
// keep the P2P results deterministic; M2L partial sums of one target may
// come from several tasks and are added with FP64 atomics.
#include "queue.h"

namespace fmm {

namespace {

typedef float f16v __attribute__((ext_vector_type(16)));
typedef float v4f __attribute__((ext_vector_type(4)));

__device__ inline void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// ------------------------------------------------------------------ P2P
constexpr int kP2PTile = 512;  // float4 sources per wave tile (8 KB)

// A leaf of nt <= 64 targets is covered by at most two passes: pass 0
// takes the first T0 = 2^floor(log2 nt) targets, pass 1 the remaining
// r = nt - T0 with T1 = 2^ceil(log2 r) lanes per stream.  A pass with T
// targets runs 64 / T source streams (lane = stream * T + target).
struct Pass {
    int lg;            // log2 of targets per stream (T = 1 << lg); -1 = unused
    int n;             // targets in the pass
    int base;          // first target of the pass within the chunk
    float x, y, z;     // this lane's target (relative to the leaf centre)
    float ph, ex, ey, ez;
};

template <bool kMask>
__device__ inline void p2p_pass(const float4 *__restrict__ tile, int count, Pass &ps, int lane) {
    if (ps.lg < 0) return;
    const int S = 64 >> ps.lg;
    const int s = lane >> ps.lg;
    const float xt = ps.x, yt = ps.y, zt = ps.z;
    float a0 = 0.f, a1 = 0.f, a2 = 0.f, a3 = 0.f;
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
            a0 += qr;
            a1 += dx * w;
            a2 += dy * w;
            a3 += dz * w;
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
        a0 += qr;
        a1 += dx * w;
        a2 += dy * w;
        a3 += dz * w;
    }
    ps.ph += a0;
    ps.ex += a1;
    ps.ey += a2;
    ps.ez += a3;
}

__device__ inline void pass_init(Pass &ps, int n, int base, const float4 *__restrict__ pf, int64_t first, int lane) {
    ps.n = n;
    ps.base = base;
    ps.ph = ps.ex = ps.ey = ps.ez = 0.f;
    ps.x = ps.y = ps.z = 0.f;
    if (n <= 0) {
        ps.lg = -1;
        return;
    }
    int lg = 0;
    while ((1 << lg) < n) lg++;
    ps.lg = lg;
    const int t = lane & ((1 << lg) - 1);
    if (t < n) {
        float4 me = pf[first + base + t];
        ps.x = me.x;
        ps.y = me.y;
        ps.z = me.z;
    }
}

__device__ inline void pass_write(const Pass &ps, const QueueArgs &a, int64_t first, int lane) {
    if (ps.lg < 0) return;
    float p0 = ps.ph, p1 = ps.ex, p2 = ps.ey, p3 = ps.ez;
    for (int d = 1 << ps.lg; d < 64; d <<= 1) {
        p0 += __shfl_xor(p0, d, 64);
        p1 += __shfl_xor(p1, d, 64);
        p2 += __shfl_xor(p2, d, 64);
        p3 += __shfl_xor(p3, d, 64);
    }
    if (lane < ps.n) {
        int64_t r = first + ps.base + lane;
        a.phi[r] = (double)p0;
        a.fld[3 * r] = (double)p1;
        a.fld[3 * r + 1] = (double)p2;
        a.fld[3 * r + 2] = (double)p3;
    }
}

// One target leaf by one wave.
__device__ void p2p_leaf(const QueueArgs &a, int32_t A, float4 *__restrict__ tile, int lane) {
    const int32_t tf = a.c.first[A], nt_all = a.c.count[A];
    const double cax = a.centre[3 * A], cay = a.centre[3 * A + 1], caz = a.centre[3 * A + 2];
    const int32_t e0 = a.p2p_ptr[A], e1 = a.p2p_ptr[A + 1];
    for (int32_t t0 = 0; t0 < nt_all; t0 += 64) {
        const int nt = nt_all - t0 < 64 ? nt_all - t0 : 64;
        int hb = 0;
        while ((2 << hb) <= nt) hb++;
        Pass p0, p1;
        pass_init(p0, 1 << hb, 0, a.pf, tf + t0, lane);
        pass_init(p1, nt - (1 << hb), 1 << hb, a.pf, tf + t0, lane);
        // own leaf: the only place zero distances occur
        for (int32_t j0 = 0; j0 < nt_all; j0 += kP2PTile) {
            int cnt = nt_all - j0 < kP2PTile ? nt_all - j0 : kP2PTile;
            wave_sync();
            for (int j = lane; j < cnt; j += 64) tile[j] = a.pf[tf + j0 + j];
            wave_sync();
            p2p_pass<true>(tile, cnt, p0, lane);
            p2p_pass<true>(tile, cnt, p1, lane);
        }
        // other leaves: 64 list entries at a time; lane j describes entry j
        // (source range, offset to the target centre), a wave prefix sum of
        // the sizes lays them out back to back, and all lanes copy the
        // concatenation into the tile, flushing whenever it is full.
        int fill = 0;
        wave_sync();
        for (int32_t eb = e0; eb < e1; eb += 64) {
            int32_t e = eb + lane;
            int32_t sf = 0, ns = 0;
            float ox = 0.f, oy = 0.f, oz = 0.f;
            if (e < e1) {
                int32_t B = a.p2p_src[e];
                if (B != A) {
                    sf = a.c.first[B];
                    ns = a.c.count[B];
                    ox = (float)(a.centre[3 * B] - cax);
                    oy = (float)(a.centre[3 * B + 1] - cay);
                    oz = (float)(a.centre[3 * B + 2] - caz);
                }
            }
            int inc = ns;
#pragma unroll
            for (int d = 1; d < 64; d <<= 1) {
                int o = __shfl_up(inc, d, 64);
                if (lane >= d) inc += o;
            }
            const int total = __shfl(inc, 63, 64);
            for (int pos0 = 0; pos0 < total;) {
                const int take = kP2PTile - fill < total - pos0 ? kP2PTile - fill : total - pos0;
                // every lane takes part in every shuffle (no divergent lanes)
                for (int k0 = 0; k0 < take; k0 += 64) {
                    const int k = k0 + lane;
                    const bool act = k < take;
                    const int gk = act ? pos0 + k : 0;  // index into the concatenation
                    int lo = 0;                          // first lane whose inclusive prefix exceeds gk
#pragma unroll
                    for (int step = 32; step > 0; step >>= 1) {
                        int v = __shfl(inc, lo + step - 1, 64);
                        if (v <= gk) lo += step;
                    }
                    const int j = lo;
                    const int base = __shfl(inc, j, 64) - __shfl(ns, j, 64);
                    const int32_t sj = __shfl(sf, j, 64);
                    const float sx = __shfl(ox, j, 64), sy = __shfl(oy, j, 64), sz = __shfl(oz, j, 64);
                    if (act) {
                        float4 v = a.pf[sj + (gk - base)];
                        tile[fill + k] = make_float4(v.x + sx, v.y + sy, v.z + sz, v.w);
                    }
                }
                fill += take;
                pos0 += take;
                if (fill == kP2PTile) {
                    wave_sync();
                    p2p_pass<false>(tile, fill, p0, lane);
                    p2p_pass<false>(tile, fill, p1, lane);
                    wave_sync();
                    fill = 0;
                }
            }
        }
        wave_sync();
        p2p_pass<false>(tile, fill, p0, lane);
        p2p_pass<false>(tile, fill, p1, lane);
        wave_sync();
        pass_write(p0, a, tf + t0, lane);
        pass_write(p1, a, tf + t0, lane);
    }
}

// ------------------------------------------------------------------ M2L
// B operand: lane (col, kh) walks row s of the padded multipoles from
// element kh * KS4, one float4 per 4 k-steps, with a 2-deep lookahead that
// runs across entries.  Absent sources point at an all-zero row.
template <int RT, int KS4>
__device__ void m2l_task(const QueueArgs &a, int4 task, float4 *__restrict__ Ts) {
    constexpr int NQ = KS4 / 4;                        // float4 per lane per row tile
    constexpr int PER = (RT * NQ * 64 + 255) / 256;    // operator float4 per thread
    constexpr int NF4P = PER * 256;                    // padded float4 per class operator
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int col = lane & 31, kh = lane >> 5;
    const int PS = 2 * KS4;                            // padded multipole row stride
    const v4f *frag4 = reinterpret_cast<const v4f *>(a.frags) + tid;
    v4f *Tsv = reinterpret_cast<v4f *>(Ts);
    const float4 *m4 = reinterpret_cast<const float4 *>(a.M32) + kh * NQ;
    f16v acc[RT];
#pragma unroll
    for (int r = 0; r < RT; r++)
#pragma unroll
        for (int i = 0; i < 16; i++) acc[r][i] = 0.f;
    v4f tpre[PER];
    // first entry: operator to LDS, multipole window
    {
        const v4f *src = frag4 + (int64_t)a.slot_of_cid[a.ecls[task.y]] * NF4P;
#pragma unroll
        for (int i = 0; i < PER; i++) tpre[i] = src[i * 256];
    }
    int32_t s0 = a.esrc[(int64_t)task.y * kGroupM2L + w * 32 + col];
    const float4 *row = m4 + (int64_t)(s0 < 0 ? a.zero_row : s0) * (PS / 4);
    float4 w0 = row[0], w1 = NQ > 1 ? row[1] : make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
    for (int i = 0; i < PER; i++) Tsv[tid + i * 256] = tpre[i];
    __syncthreads();
    for (int32_t e = task.y; e < task.z; e++) {
        const bool more = e + 1 < task.z;
        const float4 *nrow = row;
        if (more) {
            const v4f *src = frag4 + (int64_t)a.slot_of_cid[a.ecls[e + 1]] * NF4P;
#pragma unroll
            for (int i = 0; i < PER; i++) tpre[i] = src[i * 256];
            int32_t s1 = a.esrc[(int64_t)(e + 1) * kGroupM2L + w * 32 + col];
            nrow = m4 + (int64_t)(s1 < 0 ? a.zero_row : s1) * (PS / 4);
        }
#pragma unroll
        for (int q = 0; q < NQ; q++) {
            const float4 cur = w0;
            w0 = w1;
            if (q + 2 < NQ) w1 = row[q + 2];
            else if (more) w1 = nrow[q + 2 - NQ];
#pragma unroll
            for (int r = 0; r < RT; r++) {
                float4 av = Ts[(r * NQ + q) * 64 + lane];
                acc[r] = __builtin_amdgcn_mfma_f32_32x32x2f32(av.x, cur.x, acc[r], 0, 0, 0);
                acc[r] = __builtin_amdgcn_mfma_f32_32x32x2f32(av.y, cur.y, acc[r], 0, 0, 0);
                acc[r] = __builtin_amdgcn_mfma_f32_32x32x2f32(av.z, cur.z, acc[r], 0, 0, 0);
                acc[r] = __builtin_amdgcn_mfma_f32_32x32x2f32(av.w, cur.w, acc[r], 0, 0, 0);
            }
        }
        row = nrow;
        __syncthreads();
        if (more) {
#pragma unroll
            for (int i = 0; i < PER; i++) Tsv[tid + i * 256] = tpre[i];
        }
        __syncthreads();
    }
    const int32_t A = a.gtarget[(int64_t)task.x * kGroupM2L + w * 32 + col];
    if (A < 0) return;
    double *Lc = a.L + (int64_t)A * a.P;
#pragma unroll
    for (int r = 0; r < RT; r++)
#pragma unroll
        for (int i = 0; i < 16; i++) {
            int row_i = r * 32 + 8 * (i >> 2) + 4 * kh + (i & 3);
            if (row_i < a.P) atomicAdd(&Lc[row_i], (double)acc[r][i]);
        }
}

// ------------------------------------------------------------------ queue
template <int RT, int KS4>
__global__ void __launch_bounds__(256) k_queue(QueueArgs a) {
    constexpr int kTsF4 = ((RT * (KS4 / 4) * 64 + 255) / 256) * 256;
    constexpr int kLdsF4 = kTsF4 > 4 * kP2PTile ? kTsF4 : 4 * kP2PTile;
    __shared__ float4 lds[kLdsF4];
    __shared__ int32_t task_sh;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    for (;;) {
        if (threadIdx.x == 0) task_sh = atomicAdd(a.head, 1);
        __syncthreads();
        const int32_t t = task_sh;
        __syncthreads();
        if (t >= a.ntask) break;
        if (t < a.nm2l_task) {
            m2l_task<RT, KS4>(a, a.m2l_tasks[t], lds);
        } else {
            int32_t li = (t - a.nm2l_task) * 4 + w;
            if (li < a.nleaves) p2p_leaf(a, a.leaves[li], lds + w * kP2PTile, lane);
        }
        __syncthreads();
    }
}

// ------------------------------------------------------------------ prep
__global__ void k_pad_f32(const double *__restrict__ in, int32_t ncell, int P, int PS, float *__restrict__ out) {
    int64_t n = (int64_t)(ncell + 1) * PS;  // row ncell stays zero (absent sources)
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        int64_t c = i / PS;
        int j = (int)(i - c * PS);
        out[i] = (j < P && c < ncell) ? (float)in[c * P + j] : 0.f;
    }
}

}  // namespace

bool queue_supported(int p) { return p >= 0 && p <= 12; }

void queue_layout(int p, int *RT, int *KS4) {
    const int P = ncoef(p);
    *RT = (P + 31) / 32;
    *KS4 = (((P + 1) / 2 + 3) / 4) * 4;
}

int64_t queue_frag_floats(int p) {
    int RT, KS4;
    queue_layout(p, &RT, &KS4);
    int64_t per = ((int64_t)RT * (KS4 / 4) * 64 + 255) / 256;
    return per * 256 * 4;
}

void queue_pad_multipoles(const double *M, int32_t ncell, int p, float *M32, hipStream_t s) {
    int RT, KS4;
    queue_layout(p, &RT, &KS4);
    int64_t n = (int64_t)(ncell + 1) * 2 * KS4;
    hipLaunchKernelGGL(k_pad_f32, dim3(grid_for(n, 256, 16384)), dim3(256), 0, s, M, ncell, ncoef(p), 2 * KS4, M32);
    FMM_LAUNCH_CHECK();
}

void queue_run(const QueueArgs &a, int p, int nworkgroups, hipStream_t s) {
    if (a.ntask <= 0) return;
    FMM_HIP_CHECK(hipMemsetAsync(a.head, 0, sizeof(int32_t), s));
    dim3 grid(nworkgroups), block(256);
#define FMM_Q(PP, R, K)                                                   \
    case PP:                                                              \
        hipLaunchKernelGGL((k_queue<R, K>), grid, block, 0, s, a);        \
        break;
    switch (p) {
        FMM_Q(0, 1, 4) FMM_Q(1, 1, 4) FMM_Q(2, 1, 8) FMM_Q(3, 1, 8) FMM_Q(4, 1, 16) FMM_Q(5, 2, 20)
        FMM_Q(6, 2, 28) FMM_Q(7, 2, 32) FMM_Q(8, 3, 44) FMM_Q(9, 4, 52) FMM_Q(10, 4, 64) FMM_Q(11, 5, 72)
        FMM_Q(12, 6, 88)
        default: throw HipError{hipErrorInvalidValue, "queue: unsupported order"};
    }
#undef FMM_Q
    FMM_LAUNCH_CHECK();
}

}  // namespace fmm
