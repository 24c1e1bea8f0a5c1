// The device-side work queue of the near/far field stage.
//
// The paper schedules M2L and P2P work as tasks of adjustable granularity
// on a multicore runtime (Sec. 3, 4); here one persistent kernel plays that
// role on the GPU.  Workgroups claim tasks from device-side lists with
// atomic counters until the lists are exhausted.
//   * M2L task (one workgroup): a group of 256 target cells (same level and
//     octant, Morton order; 64 per wave) and a range of its class entries.
//     For each entry the waves contract the class operator T_c with the
//     multipoles of the class's sources on the matrix cores
//     (v_mfma_f32_32x32x16_bf16).  Operator and multipoles are each split
//     into two bf16 pieces x = x_hi + x_lo; three products (hi.hi, hi.lo,
//     lo.hi) accumulate in FP32, which keeps about 16 significant bits of
//     every product; the dropped lo.lo term is below 2^-16 of it.  The
//     operator is staged through a three-deep LDS ring shared by the four
//     waves (one barrier per two k-steps); multipoles stream from L2 two
//     k-steps ahead.  The targets' local expansions accumulate in FP32
//     registers and are stored, at the end of the task, in the task's own
//     slot of a partial-locals buffer (plain coalesced stores); one pass after
//     the queue sums each group's task partials in task order into the FP64
//     locals, so the result does not depend on which task ends first.
//   * P2P task (one wave): one target leaf.  Sources are staged in the
//     wave's LDS tile as float4 relative to the target centre; a leaf of nt
//     targets is covered by at most two passes of 2^b targets x 64/2^b
//     source streams; streams are combined with cross-lane shuffles.
// Matrix-core and vector work of waves that share a SIMD do not overlap on
// this chip, so the two task types simply share the machine.  Lists are kept
// per XCD (spatially contiguous tasks, so the XCD's L2 holds their operators
// and multipoles); a workgroup drains its XCD's lists, then steals.  Half
// of the workgroups start with M2L tasks, half with P2P tasks.
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
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));

__device__ inline bf8 as_bf8(v4f v) { return __builtin_bit_cast(bf8, v); }

// LDS barrier that waits only for this wave's LDS traffic (global loads in
// flight stay in flight).
__device__ inline void lds_barrier() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// one multipole k-step for a lane: bf16 pieces hi and lo of its 8 k values
struct MStep {
    v4f h, l;
};

// first float4 of this lane's k-half in multipole row s (s < 0: zero row)
__device__ inline const v4f *mrow(const QueueArgs &a, const v4f *mb4, int32_t s, int nk) {
    return mb4 + (int64_t)(s < 0 ? a.zero_row : s) * nk * 4;
}

__device__ inline MStep mload(const v4f *row, int step) {
    MStep m;
    m.h = row[step * 4];
    m.l = row[step * 4 + 2];
    return m;
}

template <int RT>
constexpr int ring_f4() { return 3 * (2 * RT * 2) * 64; }  // three stages of 2 k-steps x RT tiles x 2 pieces

// One M2L task by the whole workgroup.  Wave w owns target slots
// [64 w, 64 w + 64) as two MFMA column tiles.  Lane (col = lane % 32,
// kh = lane / 32) holds, per k-step s, operator values
// T[r 32 + col][16 s + 8 kh + t] and multipole values M~_src[16 s + 8 kh + t],
// t < 8, each as bf16 hi and lo pieces.
//
// Operator staging: the operator of an entry is 2 RT k-steps, grouped in
// stages of two k-steps (4 RT blocks of 1 KB).  Stage J of the task sits in
// ring buffer J % 3.  At the start of stage J every wave writes its quarter
// of stage J + 1 (loaded into registers one stage earlier) and passes a
// barrier; stage J itself was published by the previous barrier, and the
// buffer written (J + 1) % 3 = (J - 2) % 3 was last read before it.
template <int RT>
__device__ void m2l_group(const QueueArgs &a, int4 task, int w, int lane, v4f *ring) {
    constexpr int NK = 2 * RT;            // k-steps of 16 per entry
    constexpr int SK = 2;                 // k-steps per stage
    constexpr int NS = NK / SK;           // stages per entry (= RT)
    constexpr int SB = SK * RT * 2;       // 1 KB blocks per stage
    constexpr int OB = NK * RT * 2;       // blocks per class operator
    constexpr int NB = 2;                 // column tiles per wave
    const int col = lane & 31, kh = lane >> 5;
    const v4f *ops4 = reinterpret_cast<const v4f *>(a.ops) + lane;
    const v4f *mb4 = reinterpret_cast<const v4f *>(a.Mb) + kh;
    const int32_t *gsrc = a.esrc + w * 64 + col;
    const int32_t e0 = task.y, ne = task.z - task.y;   // workgroup-uniform
    int32_t slot_lo = 0, slot_hi = 0;
    if (lane < ne) slot_lo = a.ecls[e0 + lane];
    if (64 + lane < ne) slot_hi = a.ecls[e0 + 64 + lane];
    auto slot = [&](int i) {
        return i < 64 ? __builtin_amdgcn_readlane(slot_lo, i) : __builtin_amdgcn_readlane(slot_hi, i - 64);
    };
    // this wave's blocks of stage J: w + 4 q, q < RT
    auto stage_src = [&](int J) {
        const int i = J / NS, g = J - i * NS;
        return ops4 + ((int64_t)slot(i) * OB + g * SB + w) * 64;
    };
    const int nstage = ne * NS;
    v4f stg[RT];
    {
        const v4f *src = stage_src(0);
#pragma unroll
        for (int q = 0; q < RT; q++) ring[(w + 4 * q) * 64 + lane] = src[4 * q * 64];
        if (nstage > 1) {
            src = stage_src(1);
#pragma unroll
            for (int q = 0; q < RT; q++) stg[q] = src[4 * q * 64];
        }
    }
    f16v acc[RT][NB];
#pragma unroll
    for (int r = 0; r < RT; r++)
#pragma unroll
        for (int b = 0; b < NB; b++)
#pragma unroll
            for (int i = 0; i < 16; i++) acc[r][b][i] = 0.f;
    // multipole rows of the current and the next entry; sources of entry + 2.
    // live[b]: some target of column tile b has a source in the current
    // entry (wave-uniform); a tile with none skips its MFMAs (at the domain
    // boundary about a fifth of the tiles of an entry are empty).
    const v4f *R[NB], *nR[NB];
    int32_t sn[NB];
    bool live[NB], nlive[NB];
#pragma unroll
    for (int b = 0; b < NB; b++) {
        const int32_t s0 = gsrc[(int64_t)e0 * kGroupM2L + b * 32];
        R[b] = mrow(a, mb4, s0, NK);
        live[b] = __ballot(s0 >= 0) != 0;
        nR[b] = R[b];
        nlive[b] = live[b];
        sn[b] = ne > 1 ? gsrc[(int64_t)(e0 + 1) * kGroupM2L + b * 32] : -1;
    }
    // two-step multipole window
    MStep m0[NB], m1[NB];
#pragma unroll
    for (int b = 0; b < NB; b++) {
        m0[b] = mload(R[b], 0);
        m1[b] = mload(R[b], 1);
    }
    for (int J = 0; J < nstage; J++) {
        const int i = J / NS, g = J - i * NS;
        if (J + 1 < nstage) {
            v4f *dst = ring + ((J + 1) % 3) * SB * 64;
#pragma unroll
            for (int q = 0; q < RT; q++) dst[(w + 4 * q) * 64 + lane] = stg[q];
        }
        lds_barrier();
        if (J + 2 < nstage) {
            const v4f *src = stage_src(J + 2);
#pragma unroll
            for (int q = 0; q < RT; q++) stg[q] = src[4 * q * 64];
        }
        const bool more = i + 1 < ne;
        if (g == 0 && more) {
#pragma unroll
            for (int b = 0; b < NB; b++) {
                nR[b] = mrow(a, mb4, sn[b], NK);
                nlive[b] = __ballot(sn[b] >= 0) != 0;
                sn[b] = i + 2 < ne ? gsrc[(int64_t)(e0 + i + 2) * kGroupM2L + b * 32] : -1;
            }
        }
        const v4f *rb = ring + (J % 3) * SB * 64 + lane;
#pragma unroll
        for (int t = 0; t < SK; t++) {
            const int s = g * SK + t;
            MStep cm[NB];
#pragma unroll
            for (int b = 0; b < NB; b++) {
                cm[b] = m0[b];
                m0[b] = m1[b];
            }
            if (s + 2 < NK) {
#pragma unroll
                for (int b = 0; b < NB; b++) m1[b] = mload(R[b], s + 2);
            } else if (more) {
#pragma unroll
                for (int b = 0; b < NB; b++) m1[b] = mload(nR[b], s + 2 - NK);
            }
            // keep the multipole loads ahead of this step's MFMAs
            __builtin_amdgcn_sched_barrier(0);
            v4f ah[RT], al[RT];
#pragma unroll
            for (int r = 0; r < RT; r++) {
                ah[r] = rb[((t * RT + r) * 2) * 64];
                al[r] = rb[((t * RT + r) * 2 + 1) * 64];
            }
#pragma unroll
            for (int b = 0; b < NB; b++)
                if (live[b])
#pragma unroll
                    for (int r = 0; r < RT; r++) {
                        acc[r][b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(as_bf8(al[r]), as_bf8(cm[b].h), acc[r][b], 0, 0, 0);
                        acc[r][b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(as_bf8(ah[r]), as_bf8(cm[b].l), acc[r][b], 0, 0, 0);
                        acc[r][b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(as_bf8(ah[r]), as_bf8(cm[b].h), acc[r][b], 0, 0, 0);
                    }
        }
        if (g == NS - 1) {
#pragma unroll
            for (int b = 0; b < NB; b++) {
                R[b] = nR[b];
                live[b] = nlive[b];
            }
        }
    }
    // the task's partial locals: part[slot][row][target slot], the 32
    // column lanes of a row write 128 contiguous bytes
    float *out = a.part + (int64_t)task.w * a.P * kGroupM2L + w * 64 + col;
#pragma unroll
    for (int b = 0; b < NB; b++)
#pragma unroll
        for (int r = 0; r < RT; r++)
#pragma unroll
            for (int i = 0; i < 16; i++) {
                const int row_i = r * 32 + 8 * (i >> 2) + 4 * kh + (i & 3);
                if (row_i < a.P) out[(int64_t)row_i * kGroupM2L + b * 32] = acc[r][b][i];
            }
}

// ------------------------------------------------------------------ queue
template <int RT>
constexpr int queue_lds_f4() { return ring_f4<RT>() > 4 * kP2PTile ? ring_f4<RT>() : 4 * kP2PTile; }

// One task record (task trace on): written by one lane.
__device__ inline void trace_task(const QueueArgs &a, int kind, int32_t task, int kernel, uint64_t t0) {
    const uint64_t t1 = __builtin_amdgcn_s_memrealtime();
    const int32_t i = atomicAdd(a.trace_count, 1);
    if (i >= a.trace_cap) return;
    fmm_task_record r;
    r.start = t0;
    r.end = t1;
    r.kind = kind;
    r.task = task;
    r.kernel = kernel;
    r.hw_id = (uint32_t)__builtin_amdgcn_s_getreg((4 << 0) | (0 << 6) | (31 << 11));
    r.xcc = (uint32_t)__builtin_amdgcn_s_getreg((20 << 0) | (0 << 6) | (15 << 11));
    r.reserved = 0;
    a.trace[i] = r;
}

// All P2P tasks this wave can claim, own XCD's list first.
__device__ inline void p2p_phase(const QueueArgs &a, int x, int lane, float4 *__restrict__ tile, int kernel) {
    for (int k = 0; k < 8; k++) {
        const int L = (((x + k) & 7) << 1) | 1;
        const int4 li = a.lists[L];
        for (;;) {
            int32_t t = 0;
            if (lane == 0) t = atomicAdd(&a.heads[L], 1);
            t = __builtin_amdgcn_readfirstlane(t);      // lane 0's claim, wave-uniform
            if (t >= li.y) break;
            const int32_t leaf = a.leaves[li.z + t];
            const bool timed = a.trace || a.leaf_cost;
            const uint64_t t0 = timed ? __builtin_amdgcn_s_memrealtime() : 0;
            p2p_leaf(a, leaf, tile, lane);
            if (a.trace && lane == 0) trace_task(a, 1, leaf, kernel, t0);
            if (a.leaf_cost && lane == 0) a.leaf_cost[leaf] = (float)(__builtin_amdgcn_s_memrealtime() - t0);
        }
    }
}

template <int RT>
__global__ void __launch_bounds__(256, (RT <= 3 ? 2 : 1)) k_queue(QueueArgs a) {
    __shared__ v4f lds[queue_lds_f4<RT>()];
    __shared__ int32_t claim;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    // Workgroups go round-robin over the 8 XCDs.  With role_split the
    // workgroup slot on its compute unit (HW_ID bits 19:16) picks the task
    // type it starts with, so the workgroups sharing a compute unit mix the
    // two types; otherwise every workgroup starts with M2L.
    const int x = blockIdx.x & 7;
    const int role = a.role_split ? (__builtin_amdgcn_s_getreg((4 << 0) | (16 << 6) | (3 << 11)) & 1) : 0;
    for (int ph = 0; ph < 2; ph++) {
        if ((ph ^ role) == 0) {
            // traced: the record of a task is written after the barrier
            // that follows it, when all four waves are done
            int32_t done = -1;
            uint64_t t0 = 0;
            for (int k = 0; k < 8; k++) {
                const int L = ((x + k) & 7) << 1;
                const int4 li = a.lists[L];
                for (;;) {
                    __syncthreads();
                    if (a.trace && done >= 0 && threadIdx.x == 0) trace_task(a, 0, done, 0, t0);
                    done = -1;
                    if (threadIdx.x == 0) claim = atomicAdd(&a.heads[L], 1);
                    __syncthreads();
                    const int32_t t = __builtin_amdgcn_readfirstlane(claim);
                    if (t >= li.y) break;
                    if (a.trace) {
                        t0 = __builtin_amdgcn_s_memrealtime();
                        done = li.x + t;
                    }
                    m2l_group<RT>(a, a.m2l_tasks[li.x + t], w, lane, lds);
                }
            }
        } else if (!a.m2l_only) {
            p2p_phase(a, x, lane, reinterpret_cast<float4 *>(lds) + w * kP2PTile, 0);
        }
        __syncthreads();   // the LDS changes role
    }
}

// P2P tasks only, from the same lists and claim counters as k_queue.  Its
// waves need about half the registers of k_queue's (no MFMA accumulators),
// so launched beside k_queue they give each SIMD more P2P waves to hide
// latency with while the M2L tasks run.
__global__ void __launch_bounds__(256) k_p2p_side(QueueArgs a) {
    __shared__ float4 tiles[4 * kP2PTile];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    p2p_phase(a, blockIdx.x & 7, lane, tiles + w * kP2PTile, 1);
}

// ------------------------------------------------------------------ reduce
// One workgroup per (group, block of kRedRows coefficients): thread s sums
// target slot s over the group's tasks in task order, the block goes
// through LDS so that each target's run of coefficients is written as one
// contiguous piece of its row of L.
constexpr int kRedRows = 16;
template <class T>
__global__ void __launch_bounds__(kGroupM2L) k_reduce_partials(const T *__restrict__ part,
                                                               const int32_t *__restrict__ toff,
                                                               const int32_t *__restrict__ tcount,
                                                               const int32_t *__restrict__ gtarget, int P,
                                                               int nrb, double *__restrict__ L) {
    __shared__ double tile[kRedRows][kGroupM2L + 1];
    __shared__ int32_t tgt[kGroupM2L];
    const int g = blockIdx.x / nrb, k0 = (blockIdx.x % nrb) * kRedRows;
    const int s = threadIdx.x;
    const int nk = P - k0 < kRedRows ? P - k0 : kRedRows;
    const int32_t t0 = toff[g], nt = tcount[g];
    const int64_t ts = (int64_t)P * kGroupM2L;   // one task's partials
    tgt[s] = gtarget[(int64_t)g * kGroupM2L + s];
    const T *base = part + ((int64_t)t0 * P + k0) * kGroupM2L + s;
    for (int k = 0; k < nk; k++) {
        const T *src = base + (int64_t)k * kGroupM2L;
        double acc = 0.0;
        int32_t j = 0;
        for (; j + 4 <= nt; j += 4) {   // four loads in flight, added in task order
            const T v0 = src[j * ts], v1 = src[(j + 1) * ts], v2 = src[(j + 2) * ts], v3 = src[(j + 3) * ts];
            acc += (double)v0;
            acc += (double)v1;
            acc += (double)v2;
            acc += (double)v3;
        }
        for (; j < nt; j++) acc += (double)src[j * ts];
        tile[k][s] = acc;
    }
    __syncthreads();
    for (int i = s; i < nk * kGroupM2L; i += kGroupM2L) {
        const int slot = i / nk, k = i - slot * nk;
        const int32_t A = tgt[slot];
        if (A >= 0) L[(int64_t)A * P + k0 + k] = tile[k][slot];
    }
}

// ------------------------------------------------------------------ prep
__device__ inline uint32_t bf16_bits(float x) {
    const uint32_t u = __float_as_uint(x);
    return (u + 0x7fffu + ((u >> 16) & 1u)) >> 16;
}
__device__ inline float bf16_value(uint32_t h) { return __uint_as_float(h << 16); }

// Row c, k-step s, quarter q (0: hi of k-half 0, 1: hi of k-half 1, 2: lo
// of k-half 0, 3: lo of k-half 1) holds 8 bf16 of k = 16 s + 8 (q & 1) + t.
__global__ void k_split_multipoles(const double *__restrict__ M, int32_t ncell, int P, int NK,
                                   uint4 *__restrict__ Mb) {
    const int64_t n = (int64_t)(ncell + 1) * NK * 4;  // row ncell stays zero (absent sources)
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int q = (int)(i & 3);
        const int64_t cs = i >> 2;
        const int64_t c = cs / NK;
        const int sk = (int)(cs - c * NK);
        uint32_t h[8];
#pragma unroll
        for (int t = 0; t < 8; t++) {
            const int k = 16 * sk + 8 * (q & 1) + t;
            const double v = (c < ncell && k < P) ? M[c * P + k] : 0.0;
            const uint32_t hi = bf16_bits((float)v);
            h[t] = (q & 2) ? bf16_bits((float)(v - (double)bf16_value(hi))) : hi;
        }
        Mb[i] = make_uint4(h[0] | (h[1] << 16), h[2] | (h[3] << 16), h[4] | (h[5] << 16), h[6] | (h[7] << 16));
    }
}

}  // namespace

bool queue_supported(int p) { return p >= 0 && p <= 12; }

void reduce_partials_f64(const double *part, const int32_t *toff, const int32_t *tcount, const int32_t *gtarget,
                         int32_t ngroup, int p, double *L, hipStream_t s) {
    if (ngroup <= 0) return;
    const int P = ncoef(p), nrb = (P + kRedRows - 1) / kRedRows;
    hipLaunchKernelGGL(k_reduce_partials<double>, dim3((unsigned)(ngroup * nrb)), dim3(kGroupM2L), 0, s, part, toff,
                       tcount, gtarget, P, nrb, L);
    FMM_LAUNCH_CHECK();
}

int queue_row_tiles(int p) { return (ncoef(p) + 31) / 32; }

int64_t queue_op_elems(int p) {
    const int RT = queue_row_tiles(p);
    return (int64_t)(2 * RT) * RT * 2 * 64 * 8;
}

int64_t queue_mrow_elems(int p) { return (int64_t)(2 * queue_row_tiles(p)) * 4 * 8; }

void queue_split_multipoles(const double *M, int32_t ncell, int p, uint16_t *Mb, hipStream_t s) {
    const int NK = 2 * queue_row_tiles(p);
    const int64_t n = (int64_t)(ncell + 1) * NK * 4;
    hipLaunchKernelGGL(k_split_multipoles, dim3(grid_for(n, 256, 16384)), dim3(256), 0, s, M, ncell, ncoef(p), NK,
                       reinterpret_cast<uint4 *>(Mb));
    FMM_LAUNCH_CHECK();
}

bool queue_run(const QueueArgs &a_in, int p, int nworkgroups, int nside, const QueueStreams &qs, hipStream_t s,
               bool defer_join) {
    const bool early = qs.early != nullptr;
    const bool any_side = nside > 0 || early;
    if (nworkgroups < 1 || nside < 0 || (nside > 0 && (!qs.side || !qs.fork || !qs.join)) ||
        (early && (!qs.early_done || !qs.join)))
        throw HipError{hipErrorInvalidValue, "queue: bad launch configuration"};
    const bool defer = defer_join && any_side && qs.side2 && qs.after_queue && qs.after_side;
    hipStream_t side = qs.side;
    QueueArgs a = a_in;
    a.role_split = !any_side;
    a.m2l_only = defer ? 1 : 0;
    if (!early) fill_zero(a.heads, 16 * sizeof(int32_t), s);
    if (nside > 0) {
        // fork: the side stream starts after everything queued on s so far
        FMM_HIP_CHECK(hipEventRecord(qs.fork, s));
        FMM_HIP_CHECK(hipStreamWaitEvent(side, qs.fork, 0));
    }
    // k_queue is submitted before the side kernel, so that its workgroups
    // (the larger ones) are placed first and the side kernel fills the rest
    // of each compute unit; the other order can leave no room for k_queue
    // until side workgroups finish
    dim3 grid(nworkgroups), block(256);
#define FMM_Q(PP, R)                                                      \
    case PP:                                                              \
        hipLaunchKernelGGL((k_queue<R>), grid, block, 0, s, a);           \
        break;
    switch (p) {
        FMM_Q(0, 1) FMM_Q(1, 1) FMM_Q(2, 1) FMM_Q(3, 1) FMM_Q(4, 1) FMM_Q(5, 2) FMM_Q(6, 2) FMM_Q(7, 2) FMM_Q(8, 3)
        FMM_Q(9, 4) FMM_Q(10, 4) FMM_Q(11, 5) FMM_Q(12, 6)
        default: throw HipError{hipErrorInvalidValue, "queue: unsupported order"};
    }
#undef FMM_Q
    FMM_LAUNCH_CHECK();
    if (nside > 0) {
        hipLaunchKernelGGL(k_p2p_side, dim3(nside), dim3(256), 0, side, a);
        FMM_LAUNCH_CHECK();
    }
    // the partials of each group summed into the locals, on the slots k_queue
    // frees (before the deferred P2P workgroups below take them)
    if (a.ngroup > 0) {
        const int nrb = (a.P + kRedRows - 1) / kRedRows;
        hipLaunchKernelGGL(k_reduce_partials<float>, dim3((unsigned)(a.ngroup * nrb)), dim3(kGroupM2L), 0, s, a.part,
                           a.toff, a.tcount, a.gtarget, a.P, nrb, a.L);
        FMM_LAUNCH_CHECK();
    }
    if (defer) {
        // the rest of the P2P tail: queue_tail, once the caller has queued
        // what should run first on the compute units k_queue leaves
    } else {
        // join: work queued on s after this waits for the side kernels too
        if (nside > 0) {
            FMM_HIP_CHECK(hipEventRecord(qs.join, side));
            FMM_HIP_CHECK(hipStreamWaitEvent(s, qs.join, 0));
        }
        if (early) {
            FMM_HIP_CHECK(hipEventRecord(qs.early_done, qs.early));
            FMM_HIP_CHECK(hipStreamWaitEvent(s, qs.early_done, 0));
        }
    }
    return defer;
}

void queue_p2p_start(const QueueArgs &a_in, int nside, hipStream_t side) {
    if (nside < 1) throw HipError{hipErrorInvalidValue, "queue: bad launch configuration"};
    QueueArgs a = a_in;
    a.role_split = 0;
    a.m2l_only = 1;
    hipLaunchKernelGGL(k_p2p_side, dim3(nside), dim3(256), 0, side, a);
    FMM_LAUNCH_CHECK();
}

void queue_tail(const QueueArgs &a_in, int nworkgroups, const QueueStreams &qs, hipStream_t s) {
    QueueArgs a = a_in;
    a.role_split = 0;
    a.m2l_only = 1;
    // more P2P workgroups once everything queued on s so far is done
    // (launched with the side kernel they could fill compute units before
    // k_queue's workgroups are placed; launched as soon as k_queue ends they
    // would take the slots it frees from the sum of its partials and the
    // far field behind it); join = the end of all the P2P launches
    FMM_HIP_CHECK(hipEventRecord(qs.after_queue, s));
    FMM_HIP_CHECK(hipStreamWaitEvent(qs.side2, qs.after_queue, 0));
    hipLaunchKernelGGL(k_p2p_side, dim3(nworkgroups), dim3(256), 0, qs.side2, a);
    FMM_LAUNCH_CHECK();
    if (qs.side) {   // the side kernel of this queue, if it launched one
        FMM_HIP_CHECK(hipEventRecord(qs.after_side, qs.side));
        FMM_HIP_CHECK(hipStreamWaitEvent(qs.side2, qs.after_side, 0));
    }
    if (qs.early) {
        FMM_HIP_CHECK(hipEventRecord(qs.early_done, qs.early));
        FMM_HIP_CHECK(hipStreamWaitEvent(qs.side2, qs.early_done, 0));
    }
    FMM_HIP_CHECK(hipEventRecord(qs.join, qs.side2));
}

}  // namespace fmm
