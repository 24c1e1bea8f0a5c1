// The device-side work queue of the near/far field stage.
//
// The paper schedules M2L and P2P work as tasks of adjustable granularity
// on a multicore runtime (Sec. 3, 4); here one persistent kernel plays that
// role on the GPU.  Every wave is an independent worker: it claims tasks from
// device-side lists with an atomic counter until the lists are exhausted.
// There are no workgroup barriers, so waves of different task types share a
// SIMD and the matrix cores (M2L) overlap the vector ALUs (P2P).
//   * M2L task: a group of 64 target cells (same level and octant, Morton
//     order) and a range of its class entries.  For each entry the wave runs
//     v_mfma_f32_32x32x2_f32 with A = the class operator T_c (FP32,
//     pre-swizzled fragments, one 1 KB line per wave load) and B = the
//     multipoles of the class's sources, two 32-column tiles per operator
//     fragment; operator and multipole loads run two k-steps ahead, across
//     entries.  The targets' local expansions accumulate in FP32 AGPRs and
//     are added into the FP64 locals at the end of the task.
//   * P2P task: one target leaf.  Sources are staged in the wave's LDS tile
//     as float4 relative to the target centre; a leaf of nt targets is
//     covered by at most two passes of 2^b targets x 64/2^b source streams;
//     streams are combined with cross-lane shuffles.
// Lists are kept per XCD (spatially contiguous tasks, so the XCD's L2 holds
// their operators and multipoles); a wave drains its XCD's lists, then steals.
#include "queue.h"

#include <algorithm>

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
constexpr int kP2PTile = 256;  // float4 sources per wave tile (4 KB)

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
__device__ inline void p2p_one(float4 v, float xt, float yt, float zt, float &a0, float &a1, float &a2, float &a3) {
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

// Sources j = s, s + S, ... of the tile against this lane's target.  Eight
// LDS reads are issued before their arithmetic so that their latency
// overlaps (one wait per batch instead of one per source).
template <bool kMask>
__device__ inline void p2p_pass(const float4 *__restrict__ tile, int count, Pass &ps, int lane) {
    if (ps.lg < 0) return;
    const int S = 64 >> ps.lg;
    const int s = lane >> ps.lg;
    const float xt = ps.x, yt = ps.y, zt = ps.z;
    float a0 = 0.f, a1 = 0.f, a2 = 0.f, a3 = 0.f;
    int j = s;
    for (; j + 7 * S < count; j += 8 * S) {
        float4 v[8];
#pragma unroll
        for (int u = 0; u < 8; u++) v[u] = tile[j + u * S];
#pragma unroll
        for (int u = 0; u < 8; u++) p2p_one<kMask>(v[u], xt, yt, zt, a0, a1, a2, a3);
    }
    if (j + 3 * S < count) {
        float4 v[4];
#pragma unroll
        for (int u = 0; u < 4; u++) v[u] = tile[j + u * S];
#pragma unroll
        for (int u = 0; u < 4; u++) p2p_one<kMask>(v[u], xt, yt, zt, a0, a1, a2, a3);
        j += 4 * S;
    }
    for (; j < count; j += S) p2p_one<kMask>(tile[j], xt, yt, zt, a0, a1, a2, a3);
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
// first multipole float4 of this lane's half-row of cell s (s < 0: zero row)
__device__ inline const v4f *mrow(const QueueArgs &a, const v4f *m4, int32_t s, int ps4) {
    return m4 + (int64_t)(s < 0 ? a.zero_row : s) * ps4;
}

// One wave, kGroupM2L = 32 NB targets (NB column tiles of 32).  Lane
// (col = lane % 32, kh = lane / 32) holds, per k-step q, operator element
// T[r * 32 + col][kh * KS4 + 4 q + u] (4 u's in a float4, one per MFMA) and,
// for tile b, multipole element M~_src(b * 32 + col)[kh * KS4 + 4 q + u].
// Each operator fragment feeds NB MFMAs.  Entry metadata never sits on the
// critical path: the operator slots of all the task's entries are loaded
// once (lane l holds entries l and 64 + l, read back with readlane), and the
// source cells of entry e + 2 are loaded while entry e runs.
template <int RT, int KS4>
__device__ void m2l_wave(const QueueArgs &a, int4 task, int lane) {
    constexpr int NQ = KS4 / 4;                        // float4 k-steps per entry
    constexpr int NB = kGroupM2L / 32;                 // column tiles
    static_assert(NQ >= 2, "the load window needs two k-steps per entry");
    constexpr int NF4P = ((RT * NQ * 64 + 255) / 256) * 256;  // padded float4 per class operator
    const int col = lane & 31, kh = lane >> 5;
    const int PS4 = KS4 / 2;                           // float4 per padded multipole row
    const v4f *frag4 = reinterpret_cast<const v4f *>(a.frags) + lane;
    const v4f *m4 = reinterpret_cast<const v4f *>(a.M32) + kh * NQ;
    const int32_t *gsrc = a.esrc + col;
    const int32_t e0 = task.y, ne = task.z - task.y;   // wave-uniform
    // operator slots of the task's entries
    int32_t slot_lo = 0, slot_hi = 0;
    if (lane < ne) slot_lo = a.slot_of_cid[a.ecls[e0 + lane]];
    if (64 + lane < ne) slot_hi = a.slot_of_cid[a.ecls[e0 + 64 + lane]];
    auto slot = [&](int i) {
        return i < 64 ? __builtin_amdgcn_readlane(slot_lo, i) : __builtin_amdgcn_readlane(slot_hi, i - 64);
    };
    f16v acc[RT][NB];
#pragma unroll
    for (int r = 0; r < RT; r++)
#pragma unroll
        for (int b = 0; b < NB; b++)
#pragma unroll
            for (int i = 0; i < 16; i++) acc[r][b][i] = 0.f;
    const v4f *T = frag4 + (int64_t)slot(0) * NF4P;
    const v4f *R[NB];
    int32_t sn[NB];                                    // source cells of entry i + 1
#pragma unroll
    for (int b = 0; b < NB; b++) {
        R[b] = mrow(a, m4, gsrc[(int64_t)e0 * kGroupM2L + b * 32], PS4);
        sn[b] = ne > 1 ? gsrc[(int64_t)(e0 + 1) * kGroupM2L + b * 32] : -1;
    }
    // two-step window: A fragments (RT row tiles) and B fragments (NB
    // column tiles) of steps q and q + 1
    v4f a0[RT], a1[RT], b0[NB], b1[NB];
#pragma unroll
    for (int r = 0; r < RT; r++) {
        a0[r] = T[(r * NQ) * 64];
        a1[r] = T[(r * NQ + 1) * 64];
    }
#pragma unroll
    for (int b = 0; b < NB; b++) {
        b0[b] = R[b][0];
        b1[b] = R[b][1];
    }
    for (int i = 0; i < ne; i++) {
        const bool more = i + 1 < ne;
        const v4f *nT = T;
        const v4f *nR[NB];
#pragma unroll
        for (int b = 0; b < NB; b++) nR[b] = R[b];
        if (more) {
            nT = frag4 + (int64_t)slot(i + 1) * NF4P;
#pragma unroll
            for (int b = 0; b < NB; b++) {
                nR[b] = mrow(a, m4, sn[b], PS4);
                sn[b] = i + 2 < ne ? gsrc[(int64_t)(e0 + i + 2) * kGroupM2L + b * 32] : -1;
            }
        }
#pragma unroll
        for (int q = 0; q < NQ; q++) {
            v4f ca[RT], cb[NB];
#pragma unroll
            for (int r = 0; r < RT; r++) {
                ca[r] = a0[r];
                a0[r] = a1[r];
            }
#pragma unroll
            for (int b = 0; b < NB; b++) {
                cb[b] = b0[b];
                b0[b] = b1[b];
            }
            if (q + 2 < NQ) {
#pragma unroll
                for (int b = 0; b < NB; b++) b1[b] = R[b][q + 2];
#pragma unroll
                for (int r = 0; r < RT; r++) a1[r] = T[(r * NQ + q + 2) * 64];
            } else if (more) {
#pragma unroll
                for (int b = 0; b < NB; b++) b1[b] = nR[b][q + 2 - NQ];
#pragma unroll
                for (int r = 0; r < RT; r++) a1[r] = nT[(r * NQ + q + 2 - NQ) * 64];
            }
            // keep the loads of step q + 2 ahead of the MFMAs of step q (the
            // scheduler would otherwise sink them to their uses)
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int r = 0; r < RT; r++)
#pragma unroll
                for (int b = 0; b < NB; b++) {
                    acc[r][b] = __builtin_amdgcn_mfma_f32_32x32x2f32(ca[r].x, cb[b].x, acc[r][b], 0, 0, 0);
                    acc[r][b] = __builtin_amdgcn_mfma_f32_32x32x2f32(ca[r].y, cb[b].y, acc[r][b], 0, 0, 0);
                    acc[r][b] = __builtin_amdgcn_mfma_f32_32x32x2f32(ca[r].z, cb[b].z, acc[r][b], 0, 0, 0);
                    acc[r][b] = __builtin_amdgcn_mfma_f32_32x32x2f32(ca[r].w, cb[b].w, acc[r][b], 0, 0, 0);
                }
        }
        T = nT;
#pragma unroll
        for (int b = 0; b < NB; b++) R[b] = nR[b];
    }
#pragma unroll
    for (int b = 0; b < NB; b++) {
        const int32_t A = a.gtarget[(int64_t)task.x * kGroupM2L + b * 32 + col];
        if (A < 0) continue;
        double *Lc = a.L + (int64_t)A * a.P;
#pragma unroll
        for (int r = 0; r < RT; r++)
#pragma unroll
            for (int i = 0; i < 16; i++) {
                int row_i = r * 32 + 8 * (i >> 2) + 4 * kh + (i & 3);
                if (row_i < a.P) atomicAdd(&Lc[row_i], (double)acc[r][b][i]);
            }
    }
}

// ------------------------------------------------------------------ queue
template <int RT, int KS4>
__global__ void __launch_bounds__(256) k_queue(QueueArgs a) {
    __shared__ float4 lds[4 * kP2PTile];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    // Workgroups go round-robin over the 8 XCDs.  Waves drain their own
    // XCD's lists first, then steal from other XCDs.  The task type a wave
    // starts with alternates with its wave slot on the SIMD (HW_ID bits 3:0),
    // so the waves sharing a SIMD mix matrix-core and vector work.
    const int x = blockIdx.x & 7;
    const int role = __builtin_amdgcn_s_getreg((4 << 0) | (0 << 6) | (3 << 11)) & 1;
    float4 *tile = lds + w * kP2PTile;
    for (int k = 0; k < 16; k++) {
        const int L = (((x + (k >> 1)) & 7) << 1) | ((k & 1) ^ role);
        const int4 li = a.lists[L];
        for (;;) {
            int32_t t = 0;
            if (lane == 0) t = atomicAdd(&a.heads[L], 1);
            t = __builtin_amdgcn_readfirstlane(t);      // lane 0's claim, wave-uniform
            if (t >= li.y) break;
            if ((L & 1) == 0) m2l_wave<RT, KS4>(a, a.m2l_tasks[li.x + t], lane);
            else p2p_leaf(a, a.leaves[li.z + t], tile, lane);
        }
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
    // at least two float4 k-steps per entry: the M2L load window spans two
    *KS4 = std::max(8, (((P + 1) / 2 + 3) / 4) * 4);
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
    FMM_HIP_CHECK(hipMemsetAsync(a.heads, 0, 16 * sizeof(int32_t), s));
    dim3 grid(nworkgroups), block(256);
#define FMM_Q(PP, R, K)                                                   \
    case PP:                                                              \
        hipLaunchKernelGGL((k_queue<R, K>), grid, block, 0, s, a);        \
        break;
    switch (p) {
        FMM_Q(0, 1, 8) FMM_Q(1, 1, 8) FMM_Q(2, 1, 8) FMM_Q(3, 1, 8) FMM_Q(4, 1, 16) FMM_Q(5, 2, 20)
        FMM_Q(6, 2, 28) FMM_Q(7, 2, 32) FMM_Q(8, 3, 44) FMM_Q(9, 4, 52) FMM_Q(10, 4, 64) FMM_Q(11, 5, 72)
        FMM_Q(12, 6, 88)
        default: throw HipError{hipErrorInvalidValue, "queue: unsupported order"};
    }
#undef FMM_Q
    FMM_LAUNCH_CHECK();
}

}  // namespace fmm
