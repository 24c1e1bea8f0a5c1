// M2L of the plain FP64 path as a dense contraction on the FP64 matrix cores
// (v_mfma_f64_16x16x4f64), over the same class-batched tables as the mixed
// path's work queue: for every entry (one operator class) of a group of 256
// target cells, T_c (P x P, FP64) times the FP64 multipoles of the entry's
// sources (one per target, absent ones zero).  One workgroup per (task, row
// pass): wave w owns target slots [64 w, 64 w + 64) as four 16-column
// tiles and a pass of up to kRowTiles 16-row tiles of the output; every
// product and sum is FP64.  Results go to the task's own slot of a partial
// buffer, summed afterwards in task order (no atomics).
#include "m2l_mfma.h"
#include "queue.h"

namespace fmm {

namespace {

typedef double v4d __attribute__((ext_vector_type(4)));

constexpr int kRowTiles = 6;   // 16-row output tiles per pass (24 accumulator tiles per wave)

// Lane l of a wave: column n = l % 16 of its B and D tiles and q = l / 16:
// A holds T[16 r + n][4 s + q], B the multipole coefficient 4 s + q of
// target n's source, and accumulator item i is row 4 i + q of the D tile.
template <int P, int RB>
__global__ void __launch_bounds__(256, 1) k_m2l_f64(const int4 *__restrict__ tasks, const int32_t *__restrict__ ecls,
                                                    const int32_t *__restrict__ esrc, const double *__restrict__ ops,
                                                    const double *__restrict__ M, double *__restrict__ part,
                                                    int npass) {
    constexpr int RT = (P + 15) / 16;          // row tiles of the operator
    constexpr int KS = (P + 3) / 4;            // k-steps of 4
    constexpr int64_t OPE = (int64_t)KS * RT * 64;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int col = lane & 15, q = lane >> 4;
    const int4 task = tasks[blockIdx.x / npass];
    const int r0 = (blockIdx.x % npass) * RB;  // first row tile of this pass
    const int nr = RT - r0 < RB ? RT - r0 : RB;
    v4d acc[RB][4];
#pragma unroll
    for (int r = 0; r < RB; r++)
#pragma unroll
        for (int c = 0; c < 4; c++) acc[r][c] = (v4d){0.0, 0.0, 0.0, 0.0};
    for (int32_t e = task.y; e < task.z; e++) {
        const int32_t slot = __builtin_amdgcn_readfirstlane(ecls[e]);
        const double *op = ops + (int64_t)slot * OPE + lane;
        int32_t src[4];
        bool live[4];
#pragma unroll
        for (int c = 0; c < 4; c++) {
            src[c] = esrc[(int64_t)e * kGroupM2L + w * 64 + c * 16 + col];
            live[c] = __ballot(src[c] >= 0) != 0;
        }
        const double *mrow[4];
#pragma unroll
        for (int c = 0; c < 4; c++) mrow[c] = M + (int64_t)(src[c] >= 0 ? src[c] : 0) * P;
#pragma unroll 6
        for (int s = 0; s < KS; s++) {
            const int k = 4 * s + q;
            double a[RB], b[4];
#pragma unroll
            for (int r = 0; r < RB; r++) a[r] = r < nr ? op[(int64_t)(s * RT + r0 + r) * 64] : 0.0;
#pragma unroll
            for (int c = 0; c < 4; c++) b[c] = (src[c] >= 0 && k < P) ? mrow[c][k] : 0.0;
#pragma unroll
            for (int c = 0; c < 4; c++)
                if (live[c])
#pragma unroll
                    for (int r = 0; r < RB; r++)
                        if (r < nr) acc[r][c] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[r], b[c], acc[r][c], 0, 0, 0);
        }
    }
    double *out = part + (int64_t)task.w * P * kGroupM2L + w * 64 + col;
#pragma unroll
    for (int r = 0; r < RB; r++) {
        if (r >= nr) continue;
#pragma unroll
        for (int c = 0; c < 4; c++)
#pragma unroll
            for (int i = 0; i < 4; i++) {
                const int row = 16 * (r0 + r) + 4 * i + q;
                if (row < P) out[(int64_t)row * kGroupM2L + c * 16] = acc[r][c][i];
            }
    }
}

template <int P>
void launch_p(const int4 *tasks, int32_t ntask, const int32_t *ecls, const int32_t *esrc, const double *ops,
              const double *M, double *part, hipStream_t s) {
    constexpr int RT = (P + 15) / 16;
    constexpr int RB = RT < kRowTiles ? RT : kRowTiles;
    const int npass = (RT + RB - 1) / RB;
    hipLaunchKernelGGL((k_m2l_f64<P, RB>), dim3((unsigned)(ntask * npass)), dim3(256), 0, s, tasks, ecls, esrc, ops,
                       M, part, npass);
    FMM_LAUNCH_CHECK();
}

}  // namespace

bool m2l_f64_supported(int p) { return p >= 0 && p <= 12; }

void m2l_f64_tasks(const int4 *tasks, int32_t ntask, const int32_t *ecls, const int32_t *esrc, const double *ops,
                   const double *M, int p, double *part, hipStream_t s) {
    if (ntask <= 0) return;
    switch (p) {
#define FMM_F64(PP) \
    case PP: launch_p<ncoef(PP)>(tasks, ntask, ecls, esrc, ops, M, part, s); break;
        FMM_F64(0) FMM_F64(1) FMM_F64(2) FMM_F64(3) FMM_F64(4) FMM_F64(5) FMM_F64(6) FMM_F64(7) FMM_F64(8)
        FMM_F64(9) FMM_F64(10) FMM_F64(11) FMM_F64(12)
#undef FMM_F64
        default: throw HipError{hipErrorInvalidValue, "FP64 matrix-core M2L: unsupported order"};
    }
}

}  // namespace fmm
