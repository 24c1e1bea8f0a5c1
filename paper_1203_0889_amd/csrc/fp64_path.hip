// The plain FP64 GPU path of the two dominant stages (Sec. 2.1: M2L and P2P
// take most of the time).  By default target-owned: each workgroup owns one
// target cell and walks its CSR list, so no two workgroups write the same
// data (the non-mutual interaction of Sec. 4); the mutual variants write
// both cells of a pair, with atomics.  This path is the accuracy anchor and
// the baseline the mixed-precision work queue is measured against.
#include "tree.h"

namespace fmm {

namespace {

// ---------------------------------------------------------------- P2P
// One wave per target leaf; source particles of every listed source leaf
// staged through LDS 64 at a time as (x, y, z, q), the slots past the leaf's
// end zero.  A chunk of nt <= 64 targets is covered by two passes: pass 0
// takes the first T0 = 2^floor(log2 nt) targets with 64 / T0 source streams
// (every lane busy), pass 1 the remaining r = nt - T0 with
// T1 = 2^ceil(log2 r) lanes per stream (lane = stream * T + target).  In a
// pass every lane runs the same number of rounds, four sources loaded before
// their arithmetic; a pair at zero distance (coincident particles, or an
// underflowing r^2) is skipped by a select, and the last round (slots past
// the end) is masked.  A pass's streams are added with a fixed butterfly at
// the end.
constexpr int kP2P64Threads = 64;

// 1/sqrt(r2) for r2 > 0: the hardware estimate y refined by one second-order
// step of the series (1 - e)^(-1/2) = 1 + e/2 + 3e^2/8 + ..., with
// e = 1 - r2 y^2, which squares and cubes the estimate's relative error.
__device__ __forceinline__ double rsqrt_fp64(double r2) {
    const double y = __builtin_amdgcn_rsq(r2);
    const double e = fma(-r2, y * y, 1.0);
    return fma(y * e, fma(e, 0.375, 0.5), y);
}

struct Pass64 {
    int lg;           // log2 of targets per stream (T = 1 << lg); -1 = unused
    int n;            // targets in the pass
    int base;         // first target of the pass within the chunk
    double x, y, z;   // this lane's target
    double p, ex, ey, ez;
};

template <bool kMask>
__device__ __forceinline__ void p2p64_one(const double4 &v, Pass64 &a, bool valid) {
    const double dx = a.x - v.x, dy = a.y - v.y, dz = a.z - v.z;
    const double r2 = dx * dx + dy * dy + dz * dz;
    const double inv = ((!kMask || valid) && r2 > 0.0) ? rsqrt_fp64(r2) : 0.0;
    const double qi = v.w * inv;
    const double qi3 = qi * inv * inv;
    a.p += qi;
    a.ex += dx * qi3;
    a.ey += dy * qi3;
    a.ez += dz * qi3;
}

__device__ __forceinline__ void pass64_init(Pass64 &ps, int n, int base, const double *__restrict__ xs,
                                            const double *__restrict__ ys, const double *__restrict__ zs,
                                            int64_t first, int lane) {
    ps.n = n;
    ps.base = base;
    ps.x = ps.y = ps.z = 0.0;
    ps.p = ps.ex = ps.ey = ps.ez = 0.0;
    if (n <= 0) {
        ps.lg = -1;
        return;
    }
    int lg = 0;
    while ((1 << lg) < n) lg++;
    ps.lg = lg;
    const int t = lane & ((1 << lg) - 1);
    if (t < n) {
        ps.x = xs[first + base + t];
        ps.y = ys[first + base + t];
        ps.z = zs[first + base + t];
    }
}

// The staged chunk of ns <= 64 sources against this lane's target of the
// pass: stream s takes sources s, s + S, ...; with K = ceil(ns / S) rounds,
// S K <= 64 (S a power of two), so every slot read is < 64, and the rounds
// before the last read slots < ns only.
__device__ __forceinline__ void pass64_run(const double4 *__restrict__ st, int ns, Pass64 &ps, int lane) {
    if (ps.lg < 0) return;
    const int S = kP2P64Threads >> ps.lg;
    const int s = lane >> ps.lg;
    const int K = (ns + S - 1) / S;
    int i = 0;
    for (; i + 4 <= K - 1; i += 4) {
        const double4 a0 = st[s + S * i], a1 = st[s + S * (i + 1)];
        const double4 a2 = st[s + S * (i + 2)], a3 = st[s + S * (i + 3)];
        p2p64_one<false>(a0, ps, true);
        p2p64_one<false>(a1, ps, true);
        p2p64_one<false>(a2, ps, true);
        p2p64_one<false>(a3, ps, true);
    }
    for (; i < K - 1; i++) p2p64_one<false>(st[s + S * i], ps, true);
    const int j = s + S * (K - 1);   // the last round
    p2p64_one<true>(st[j], ps, j < ns);
}

__device__ __forceinline__ void pass64_write(Pass64 &ps, double *__restrict__ phi, double *__restrict__ fld,
                                             int64_t first, int lane) {
    if (ps.lg < 0) return;
    double p = ps.p, ex = ps.ex, ey = ps.ey, ez = ps.ez;
    for (int o = kP2P64Threads / 2; o >= (1 << ps.lg); o >>= 1) {   // the streams of a target
        p += __shfl_xor(p, o, kP2P64Threads);
        ex += __shfl_xor(ex, o, kP2P64Threads);
        ey += __shfl_xor(ey, o, kP2P64Threads);
        ez += __shfl_xor(ez, o, kP2P64Threads);
    }
    if (lane < ps.n) {   // stream 0, target `lane`
        const int64_t r = first + ps.base + lane;
        phi[r] = p;
        fld[3 * r] = ex;
        fld[3 * r + 1] = ey;
        fld[3 * r + 2] = ez;
    }
}

__global__ void __launch_bounds__(kP2P64Threads)
    k_p2p_fp64(CellArrays c, int32_t ncell, const int32_t *__restrict__ ptr, const int32_t *__restrict__ src,
               const double *__restrict__ xs, const double *__restrict__ ys, const double *__restrict__ zs,
               const double *__restrict__ qs, double *__restrict__ phi, double *__restrict__ fld) {
    __shared__ double4 st[kP2P64Threads];
    int32_t A = blockIdx.x;
    if (A >= ncell || c.child[A] >= 0) return;
    const int lane = threadIdx.x;
    int32_t tf = c.first[A], tc = c.count[A];
    int32_t e0 = ptr[A], e1 = ptr[A + 1];
    for (int32_t t0 = 0; t0 < tc; t0 += kP2P64Threads) {
        const int nt = tc - t0 < kP2P64Threads ? tc - t0 : kP2P64Threads;
        int hb = 0;
        while ((2 << hb) <= nt) hb++;
        Pass64 p0, p1;
        pass64_init(p0, 1 << hb, 0, xs, ys, zs, tf + t0, lane);
        pass64_init(p1, nt - (1 << hb), 1 << hb, xs, ys, zs, tf + t0, lane);
        for (int32_t e = e0; e < e1; e++) {
            const int32_t B = src[e];
            int32_t sf = c.first[B], sc = c.count[B];
            for (int32_t s0 = 0; s0 < sc; s0 += kP2P64Threads) {
                const int ns = sc - s0 < kP2P64Threads ? sc - s0 : kP2P64Threads;
                __syncthreads();
                double4 v = make_double4(0.0, 0.0, 0.0, 0.0);
                if (lane < ns) {
                    const int64_t k = sf + s0 + lane;
                    v = make_double4(xs[k], ys[k], zs[k], qs[k]);
                }
                st[lane] = v;
                __syncthreads();
                pass64_run(st, ns, p0, lane);
                pass64_run(st, ns, p1, lane);
            }
        }
        pass64_write(p0, phi, fld, tf + t0, lane);
        pass64_write(p1, phi, fld, tf + t0, lane);
    }
}

// Is A among the sources of target B?  Each target's sources are sorted
// ascending (the lists are sorted by the whole (target, source) key).
__device__ __forceinline__ bool listed(const int32_t *__restrict__ ptr, const int32_t *__restrict__ src, int32_t B,
                                       int32_t A) {
    int32_t lo = ptr[B], hi = ptr[B + 1];
    while (lo < hi) {
        const int32_t mid = lo + ((hi - lo) >> 1);
        const int32_t v = src[mid];
        if (v == A) return true;
        if (v < A) lo = mid + 1; else hi = mid;
    }
    return false;
}

// The mutual P2P (Sec. 4, the mutual interaction): a leaf pair listed in
// both directions is evaluated once, by the workgroup of the smaller cell
// index, and each particle pair's distance and inverse square root serve
// both leaves.  Pairs listed in one direction only, and a leaf with itself,
// are evaluated forward as in k_p2p_fp64.  The source leaf's sums are
// gathered in LDS with FP64 LDS atomics: in round i lane (t, s) takes source
// s + S ((t + i) mod K), so lanes of one stream mostly hit different
// sources, then added to the source particles with FP64 atomics; the target
// sums are added with atomics as well (other workgroups add to the same
// particles), so phi and fld start at zero and the order of the additions
// is not fixed.
__global__ void __launch_bounds__(kP2P64Threads)
    k_p2p_fp64_mutual(CellArrays c, int32_t ncell, const int32_t *__restrict__ ptr, const int32_t *__restrict__ src,
                      const double *__restrict__ xs, const double *__restrict__ ys, const double *__restrict__ zs,
                      const double *__restrict__ qs, double *__restrict__ phi, double *__restrict__ fld) {
    __shared__ double sx[kP2P64Threads], sy[kP2P64Threads], sz[kP2P64Threads], sq[kP2P64Threads];
    __shared__ double rp[kP2P64Threads], rx[kP2P64Threads], ry[kP2P64Threads], rz[kP2P64Threads];
    int32_t A = blockIdx.x;
    if (A >= ncell || c.child[A] >= 0) return;
    const int lane = threadIdx.x;
    int32_t tf = c.first[A], tc = c.count[A];
    int32_t e0 = ptr[A], e1 = ptr[A + 1];
    for (int32_t t0 = 0; t0 < tc; t0 += kP2P64Threads) {
        const int nt = tc - t0 < kP2P64Threads ? tc - t0 : kP2P64Threads;
        int T = kP2P64Threads;
        while (T / 2 >= nt) T /= 2;
        const int S = kP2P64Threads / T;
        const int t = lane & (T - 1), sidx = lane / T;
        int32_t r = tf + t0 + t;
        bool active = t < nt;
        double xt = active ? xs[r] : 0.0, yt = active ? ys[r] : 0.0, zt = active ? zs[r] : 0.0;
        double qt = active ? qs[r] : 0.0;
        double p = 0.0, ex = 0.0, ey = 0.0, ez = 0.0;
        for (int32_t e = e0; e < e1; e++) {
            const int32_t B = src[e];
            // the same B on every lane: the branches below are uniform
            if (B < A && listed(ptr, src, B, A)) continue;   // taken by B's workgroup
            const bool mutual = B > A && listed(ptr, src, B, A);
            int32_t sf = c.first[B], sc = c.count[B];
            for (int32_t s0 = 0; s0 < sc; s0 += kP2P64Threads) {
                int ns = sc - s0 < kP2P64Threads ? sc - s0 : kP2P64Threads;
                __syncthreads();
                if (lane < ns) {
                    sx[lane] = xs[sf + s0 + lane];
                    sy[lane] = ys[sf + s0 + lane];
                    sz[lane] = zs[sf + s0 + lane];
                    sq[lane] = qs[sf + s0 + lane];
                }
                rp[lane] = rx[lane] = ry[lane] = rz[lane] = 0.0;
                __syncthreads();
                const int K = (ns + S - 1) / S;   // rounds: sources per stream, the last may be past ns
                int u = t % K;
                for (int i = 0; i < K; i++) {
                    const int j = sidx + S * u;
                    u = u + 1 == K ? 0 : u + 1;
                    if (j >= ns) continue;
                    double dx = xt - sx[j], dy = yt - sy[j], dz = zt - sz[j];
                    double r2 = dx * dx + dy * dy + dz * dz;
                    if (r2 > 0.0) {
                        double inv = rsqrt_fp64(r2);
                        double inv2 = inv * inv;
                        double qi = sq[j] * inv;
                        double qi3 = qi * inv2;
                        p += qi;
                        ex += dx * qi3;
                        ey += dy * qi3;
                        ez += dz * qi3;
                        if (mutual && active) {
                            // the target's charge at the source: the field
                            // there points along -d
                            double qj = qt * inv;
                            double qj3 = qj * inv2;
                            atomicAdd(&rp[j], qj);
                            atomicAdd(&rx[j], -dx * qj3);
                            atomicAdd(&ry[j], -dy * qj3);
                            atomicAdd(&rz[j], -dz * qj3);
                        }
                    }
                }
                if (mutual) {
                    __syncthreads();
                    if (lane < ns) {
                        const int64_t k = sf + s0 + lane;
                        atomicAdd(&phi[k], rp[lane]);
                        atomicAdd(&fld[3 * k], rx[lane]);
                        atomicAdd(&fld[3 * k + 1], ry[lane]);
                        atomicAdd(&fld[3 * k + 2], rz[lane]);
                    }
                }
            }
        }
        for (int o = kP2P64Threads / 2; o >= T; o >>= 1) {
            p += __shfl_xor(p, o, kP2P64Threads);
            ex += __shfl_xor(ex, o, kP2P64Threads);
            ey += __shfl_xor(ey, o, kP2P64Threads);
            ez += __shfl_xor(ez, o, kP2P64Threads);
        }
        if (active && sidx == 0) {
            atomicAdd(&phi[r], p);
            atomicAdd(&fld[3 * (int64_t)r], ex);
            atomicAdd(&fld[3 * (int64_t)r + 1], ey);
            atomicAdd(&fld[3 * (int64_t)r + 2], ez);
        }
    }
}

// ---------------------------------------------------------------- M2L
// Per-pair M2L in FP64, balanced over pairs: a wave takes kPairChunk
// consecutive entries of a CSR pair list, finds the owner of its first entry
// by binary search, accumulates while the owner stays the same and adds each
// owner's run into the output with FP64 atomics (so an owner with thousands
// of pairs, like a large leaf facing a dense region, is spread over many
// waves).  In owner mode (deterministic results) a wave takes all pairs of
// one owner instead, in list order, and adds them to the output with plain
// stores: the order of every addition is then fixed.  Per pair, with rho the class offset (c_A - c_B) / S_A and
// delta = l_A - l_B of the forward pair A <- B:
//   forward:  L~_n^m += (-1)^n sum_(k <= p) 2^(delta k) sum_l M~_k^l I_(n+k)^(m+l)(rho)
//   adjoint:  the transpose of that real map (see below), owner = B.
// The irregular solid harmonics (m >= 0, r^2 = |rho|^2, zeta = x + iy)
//   I_0^0 = 1/r,  I_m^m = (2m-1) zeta I_(m-1)^(m-1) / r^2,
//   I_(m+1)^m = (2m+1) z I_m^m / r^2,
//   I_n^m = ((2n-1) z I_(n-1)^m - ((n-1)^2 - m^2) I_(n-2)^m) / r^2,
// I_n^(-m) = (-1)^m conj(I_n^m): lane m evaluates column m into LDS, then
// every lane accumulates its outputs over all input coefficients.
//
// Adjoint.  The forward map on the stored real coefficients is
//   S_n^m = sum_k c_nk sum_(l=-k..k) M~_k^l I_(n+k)^(m+l),  c_nk = (-1)^n 2^(delta k),
// with L_re(n, m) = Re S_n^m and L_im(n, m) = Im S_n^m (m > 0).  Writing the
// dual of L as U_n^m = u_re + i u_im (U_n^0 real), the real inner product
// <u, S(M)> equals <v, M> for
//   V_k^l = sum_(n, m >= 0) c_nk [U_n^m conj(I_(n+k)^(m+l)) + (-1)^l conj(U_n^m) I_(n+k)^(m-l)]
// (l > 0; v_re = Re V, v_im = Im V) and v_re(k, 0) = Re V_k^0 / 2 (the two
// terms coincide for l = 0, where M~_k^0 is real).
constexpr int kM2L64Threads = 64;
constexpr int kPairChunk = 16;

// LDS of one wave (sized by p at launch): the irregular harmonics of the
// current pair for every order m, negative m included (J_n^m at
// n^2 + n + m, n <= 2p), and the source multipole as complex coefficients
// of every order (M_k^l at k^2 + k + l, k <= p).  With the signs of the
// negative orders stored, the inner sums are plain complex products.
__host__ __device__ constexpr int m2l_pairs_lds_doubles(int p) {
    return 2 * (2 * p + 1) * (2 * p + 1) + 2 * (p + 1) * (p + 1);
}
// pair streams per wave (one per half wave when a half holds every output)
__host__ __device__ constexpr int m2l_pairs_streams(int p, bool owner_mode) {
    return (!owner_mode && (p + 1) * (p + 2) / 2 <= 32) ? 2 : 1;
}

// Mutual M2L (Sec. 4, the mutual interaction; forward only, balanced
// mode): a pair listed in both directions is evaluated once, at the entry
// whose owner A has the smaller index, and the reverse pair B <- A reuses the
// harmonics of A <- B.  With rho' = -2^(-delta) rho the reverse offset in
// units of B's side, homogeneity (I_N(lambda x) = lambda^(-N-1) I_N(x)) and
// parity (I_N(-x) = (-1)^N I_N(x)) of the irregular harmonics give
//   reverse:  L~_n^m(B) += 2^(delta (n+1)) sum_k (-1)^k sum_l M~_k^l(A) I_(n+k)^(m+l)(rho),
// the forward sum with the sign flip of the odd terms moved from the output
// degree n to the input degree k.  The reverse sums go to B with FP64
// atomics after every pair.
__host__ __device__ constexpr int m2l_pairs_lds_mutual_doubles(int p, bool mutual) {
    return m2l_pairs_lds_doubles(p) + (mutual ? 2 * (p + 1) * (p + 1) : 0);
}

// The adjoint per pair (the order a launch argument): owner = the forward
// pair's source B, Out its dual multipole.
__global__ void __launch_bounds__(kM2L64Threads)
    k_m2l_pairs_adj(CellArrays c, int32_t ncell, int p, const int32_t *__restrict__ ptr,
                    const int32_t *__restrict__ src, int64_t npair, const double *__restrict__ In,
                    double *__restrict__ Out, int owner_mode) {
    extern __shared__ double lds[];
    const int NJ = (2 * p + 1) * (2 * p + 1), NM = (p + 1) * (p + 1);
    const int P = ncoef(p);
    const int NC = (p + 1) * (p + 2) / 2;
    // H pair streams per wave: with at most 32 outputs (p <= 6) each half
    // of the wave takes every other pair of the chunk, with LDS of its own
    // (owner mode keeps one stream: one owner's pairs in list order)
    const int H = m2l_pairs_streams(p, owner_mode != 0), W = 64 / H;
    const int h = threadIdx.x / W, lane = threadIdx.x - h * W;
    double *base = lds + h * m2l_pairs_lds_doubles(p);
    double *Jre = base, *Jim = base + NJ, *Mre = base + 2 * NJ, *Mim = base + 2 * NJ + NM;
    // this lane's outputs: complex index j = lane, lane + W, lane + 2 W
    int on[3], om[3];
    for (int s = 0; s < 3; s++) {
        int j = lane + W * s;
        on[s] = -1;
        om[s] = 0;
        if (j < NC) {
            int n = 0;
            while ((n + 1) * (n + 2) / 2 <= j) n++;
            on[s] = n;
            om[s] = j - n * (n + 1) / 2;
        }
    }
    const int64_t nchunk = (npair + kPairChunk - 1) / kPairChunk;
    const int64_t nunit = owner_mode ? (int64_t)ncell : nchunk;
    for (int64_t ch = blockIdx.x; ch < nunit; ch += gridDim.x) {
        int64_t e0, e1;
        int32_t O;
        if (owner_mode) {
            O = (int32_t)ch;
            e0 = ptr[O];
            e1 = ptr[O + 1];
            if (e0 == e1) continue;   // uniform over the wave
        } else {
            e0 = ch * kPairChunk;
            e1 = e0 + kPairChunk < npair ? e0 + kPairChunk : npair;
            // owner of this stream's first pair e0 + h (if it has one): the
            // last cell O with ptr[O] <= e0 + h
            const int64_t ef = e0 + h < e1 ? e0 + h : e0;
            int32_t lo = 0, hi = ncell;
            while (lo < hi) {
                int32_t mid = (lo + hi + 1) >> 1;
                if (ptr[mid] <= ef) lo = mid; else hi = mid - 1;
            }
            O = lo;
        }
        const bool any = e0 + h < e1;   // this stream has a pair in the chunk
        double accr[3] = {0, 0, 0}, acci[3] = {0, 0, 0};
        auto flush = [&](int32_t owner) {
            double *out = Out + (int64_t)owner * P;
            for (int s = 0; s < 3; s++) {
                const int n = on[s];
                if (n < 0) continue;
                const int m = om[s];
                double vr = accr[s];
                if (m == 0) vr *= 0.5;
                if (owner_mode) {   // the only wave writing this owner
                    out[cidx_re(n, m)] += vr;
                    if (m > 0) out[cidx_im(n, m)] += acci[s];
                } else {
                    atomicAdd(&out[cidx_re(n, m)], vr);
                    if (m > 0) atomicAdd(&out[cidx_im(n, m)], acci[s]);
                }
                accr[s] = acci[s] = 0.0;
            }
        };
        // the same number of rounds in every stream (the barriers below)
        const int64_t rounds = (e1 - e0 + H - 1) / H;
        for (int64_t t = 0; t < rounds; t++) {
            const int64_t e = e0 + h + H * t;
            const bool act = e < e1;
            if (act && e >= ptr[O + 1]) {
                flush(O);
                while (e >= ptr[O + 1]) O++;
            }
            const int32_t other = act ? src[e] : src[e0];
            const int32_t A = other, B = O;   // the forward pair A <- B
            const int la = c.level[A], lb = c.level[B];
            const int64_t SA = (int64_t)1 << (kLevels - la), SB = (int64_t)1 << (kLevels - lb);
            // rho in units of the target side: (C_A - C_B) / (2 S_A), exact
            const double rx = ldexp((double)((2 * (int64_t)c.ix[A] + 1) * SA - (2 * (int64_t)c.ix[B] + 1) * SB),
                                    -(kLevels - la + 1));
            const double ry = ldexp((double)((2 * (int64_t)c.iy[A] + 1) * SA - (2 * (int64_t)c.iy[B] + 1) * SB),
                                    -(kLevels - la + 1));
            const double rz = ldexp((double)((2 * (int64_t)c.iz[A] + 1) * SA - (2 * (int64_t)c.iz[B] + 1) * SB),
                                    -(kLevels - la + 1));
            const int delta = la - lb;
            __syncthreads();   // the previous pair's readers are done
            // the input coefficients as complex M_k^l, l in [-k, k], with
            // M_k^(-l) = (-1)^l conj(M_k^l)
            for (int i = lane; act && i < NM; i += W) {
                int k = 0;
                while ((k + 1) * (k + 1) <= i) k++;
                const int l = i - k * k - k, al = l < 0 ? -l : l;
                const double *x = In + (int64_t)other * P;
                double re = x[cidx_re(k, al)], im = al > 0 ? x[cidx_im(k, al)] : 0.0;
                if (l < 0) {
                    im = -im;
                    if (al & 1) {
                        re = -re;
                        im = -im;
                    }
                }
                Mre[i] = re;
                Mim[i] = im;
            }
            if (act && lane <= 2 * p) {
                // column m of the harmonics, and its mirror J_n^(-m) =
                // (-1)^m conj(J_n^m)
                int m = lane, nmax = 2 * p;
                const double sg = (m & 1) ? -1.0 : 1.0;
                double r2 = rx * rx + ry * ry + rz * rz;
                double ir2 = 1.0 / r2;
                double mr = 1.0 / sqrt(r2), mi = 0.0;  // I_m^m
                for (int j = 1; j <= m; j++) {
                    double f = (2 * j - 1) * ir2;
                    double nr = (mr * rx - mi * ry) * f, ni = (mr * ry + mi * rx) * f;
                    mr = nr;
                    mi = ni;
                }
                auto put = [&](int n, double re, double im) {
                    Jre[n * n + n + m] = re;
                    Jim[n * n + n + m] = im;
                    if (m > 0) {
                        Jre[n * n + n - m] = sg * re;
                        Jim[n * n + n - m] = -sg * im;
                    }
                };
                put(m, mr, mi);
                double pr = 0, pi = 0, cr = mr, ci = mi;
                for (int n = m + 1; n <= nmax; n++) {
                    double nr, ni;
                    if (n == m + 1) {
                        double f = (2 * m + 1) * rz * ir2;
                        nr = f * cr;
                        ni = f * ci;
                    } else {
                        double aa = (2 * n - 1) * rz, bb = (double)((n - 1) * (n - 1) - m * m);
                        nr = (aa * cr - bb * pr) * ir2;
                        ni = (aa * ci - bb * pi) * ir2;
                    }
                    put(n, nr, ni);
                    pr = cr;
                    pi = ci;
                    cr = nr;
                    ci = ni;
                }
            }
            __syncthreads();
            for (int s = 0; act && s < 3; s++) {
                const int n = on[s];
                if (n < 0) continue;
                const int m = om[s];
                double sr = 0, si = 0;
                {
                    // output (k, l) = (n, m) of this lane; inputs (nu, mu) of the dual
                    const int k = n, l = m;
                    const double fk = ldexp(1.0, delta * k);
                    const double sl = (l & 1) ? -1.0 : 1.0;
                    for (int nu = 0; nu <= p; nu++) {
                        const double cn = (nu & 1) ? -fk : fk;
                        const int nn = nu + k, ub = nu * nu + nu, jb = nn * nn + nn;
                        double tr = 0, ti = 0;
                        for (int mu = 0; mu <= nu; mu++) {
                            const double ur = Mre[ub + mu], ui = Mim[ub + mu];
                            const double i1r = Jre[jb + mu + l], i1i = Jim[jb + mu + l];
                            const double i2r = Jre[jb + mu - l], i2i = Jim[jb + mu - l];
                            // U conj(I1) + sl conj(U) I2
                            tr += (ur * i1r + ui * i1i) + sl * (ur * i2r + ui * i2i);
                            ti += (ui * i1r - ur * i1i) + sl * (ur * i2i - ui * i2r);
                        }
                        sr += cn * tr;
                        si += cn * ti;
                    }
                }
                accr[s] += sr;
                acci[s] += si;
            }
        }
        if (any) flush(O);
    }
}

// The forward per-pair M2L with the order a compile-time constant, harmonics
// and multipoles stored as complex pairs (one 16-byte LDS read per
// coefficient) and the sums over the input coefficients unrolled: for an
// output (n, m) and input degree k both operands of the inner sum are
// contiguous, J_(n+k)^(m+l) and M_k^l for l = -k..k.  With kMutual (balanced
// mode only) a pair listed in both directions is evaluated once, at the
// entry whose owner A has the smaller index, the reverse pair B <- A reusing
// the harmonics of A <- B as described above; its sums go to B with FP64
// atomics after every pair.
template <int PP, bool kMutual>
__global__ void __launch_bounds__(kM2L64Threads)
    k_m2l_pairs_fwd(CellArrays c, int32_t ncell, const int32_t *__restrict__ ptr, const int32_t *__restrict__ src,
                    int64_t npair, const double *__restrict__ In, double *__restrict__ Out, int owner_mode) {
    extern __shared__ double2 lds2[];
    constexpr int p = PP;
    constexpr int NJ = (2 * p + 1) * (2 * p + 1), NM = (p + 1) * (p + 1);
    constexpr int P = ncoef(p);
    constexpr int NC = (p + 1) * (p + 2) / 2;
    constexpr int NS = NJ + (kMutual ? 2 : 1) * NM;   // complex entries per stream
    static_assert(m2l_pairs_lds_mutual_doubles(p, kMutual) == 2 * NS, "LDS layout");
    const int H = m2l_pairs_streams(p, owner_mode != 0), W = 64 / H;
    const int h = threadIdx.x / W, lane = threadIdx.x - h * W;
    double2 *J = lds2 + h * NS;   // J_n^m at n^2 + n + m, |m| <= n <= 2p
    double2 *Mc = J + NJ;         // M_k^l of the source at k^2 + k + l, |l| <= k <= p
    double2 *Ac = Mc + NM;        // mutual: the owner's multipole, same layout
    int on[3], om[3];
    for (int s = 0; s < 3; s++) {
        int j = lane + W * s;
        on[s] = -1;
        om[s] = 0;
        if (j < NC) {
            int n = 0;
            while ((n + 1) * (n + 2) / 2 <= j) n++;
            on[s] = n;
            om[s] = j - n * (n + 1) / 2;
        }
    }
    const int64_t nchunk = (npair + kPairChunk - 1) / kPairChunk;
    const int64_t nunit = owner_mode ? (int64_t)ncell : nchunk;
    for (int64_t ch = blockIdx.x; ch < nunit; ch += gridDim.x) {
        int64_t e0, e1;
        int32_t O;
        if (owner_mode) {
            O = (int32_t)ch;
            e0 = ptr[O];
            e1 = ptr[O + 1];
            if (e0 == e1) continue;   // uniform over the wave
        } else {
            e0 = ch * kPairChunk;
            e1 = e0 + kPairChunk < npair ? e0 + kPairChunk : npair;
            const int64_t ef = e0 + h < e1 ? e0 + h : e0;
            int32_t lo = 0, hi = ncell;
            while (lo < hi) {
                int32_t mid = (lo + hi + 1) >> 1;
                if (ptr[mid] <= ef) lo = mid; else hi = mid - 1;
            }
            O = lo;
        }
        const bool any = e0 + h < e1;
        double accr[3] = {0, 0, 0}, acci[3] = {0, 0, 0};
        double revr[3] = {0, 0, 0}, revi[3] = {0, 0, 0};   // mutual: the reverse pair's sums
        auto flush = [&](int32_t owner) {
            double *out = Out + (int64_t)owner * P;
            for (int s = 0; s < 3; s++) {
                const int n = on[s];
                if (n < 0) continue;
                const int m = om[s];
                if (owner_mode) {
                    out[cidx_re(n, m)] += accr[s];
                    if (m > 0) out[cidx_im(n, m)] += acci[s];
                } else {
                    atomicAdd(&out[cidx_re(n, m)], accr[s]);
                    if (m > 0) atomicAdd(&out[cidx_im(n, m)], acci[s]);
                }
                accr[s] = acci[s] = 0.0;
            }
        };
        const int64_t rounds = (e1 - e0 + H - 1) / H;
        for (int64_t t = 0; t < rounds; t++) {
            const int64_t e = e0 + h + H * t;
            bool act = e < e1;
            if (act && e >= ptr[O + 1]) {
                flush(O);
                while (e >= ptr[O + 1]) O++;
            }
            const int32_t B = act ? src[e] : src[e0];
            const int32_t A = O;
            bool mutual = false;
            if (kMutual && act) {
                // the same (A, B) on every lane of the stream
                const bool both = listed(ptr, src, B, A);
                if (both && B < A) act = false;   // evaluated at the entry owned by B
                mutual = both && B > A;
            }
            const int la = c.level[A], lb = c.level[B];
            const int64_t SA = (int64_t)1 << (kLevels - la), SB = (int64_t)1 << (kLevels - lb);
            const double rx = ldexp((double)((2 * (int64_t)c.ix[A] + 1) * SA - (2 * (int64_t)c.ix[B] + 1) * SB),
                                    -(kLevels - la + 1));
            const double ry = ldexp((double)((2 * (int64_t)c.iy[A] + 1) * SA - (2 * (int64_t)c.iy[B] + 1) * SB),
                                    -(kLevels - la + 1));
            const double rz = ldexp((double)((2 * (int64_t)c.iz[A] + 1) * SA - (2 * (int64_t)c.iz[B] + 1) * SB),
                                    -(kLevels - la + 1));
            const int delta = la - lb;
            __syncthreads();   // the previous pair's readers are done
            for (int i = lane; act && i < NM; i += W) {
                int k = 0;
                while ((k + 1) * (k + 1) <= i) k++;
                const int l = i - k * k - k, al = l < 0 ? -l : l;
                const double *x = In + (int64_t)B * P;
                double re = x[cidx_re(k, al)], im = al > 0 ? x[cidx_im(k, al)] : 0.0;
                if (l < 0) {
                    im = -im;
                    if (al & 1) {
                        re = -re;
                        im = -im;
                    }
                }
                Mc[i] = make_double2(re, im);
                if (kMutual && mutual) {
                    const double *y = In + (int64_t)A * P;
                    double are = y[cidx_re(k, al)], aim = al > 0 ? y[cidx_im(k, al)] : 0.0;
                    if (l < 0) {
                        aim = -aim;
                        if (al & 1) {
                            are = -are;
                            aim = -aim;
                        }
                    }
                    Ac[i] = make_double2(are, aim);
                }
            }
            if (act && lane <= 2 * p) {
                const int m = lane;
                const double sg = (m & 1) ? -1.0 : 1.0;
                const double r2 = rx * rx + ry * ry + rz * rz;
                const double ir2 = 1.0 / r2;
                double mr = 1.0 / sqrt(r2), mi = 0.0;   // I_m^m
                for (int j = 1; j <= m; j++) {
                    const double f = (2 * j - 1) * ir2;
                    const double nr = (mr * rx - mi * ry) * f, ni = (mr * ry + mi * rx) * f;
                    mr = nr;
                    mi = ni;
                }
                auto put = [&](int n, double re, double im) {
                    J[n * n + n + m] = make_double2(re, im);
                    if (m > 0) J[n * n + n - m] = make_double2(sg * re, -sg * im);
                };
                put(m, mr, mi);
                double pr = 0, pi = 0, cr = mr, ci = mi;
                for (int n = m + 1; n <= 2 * p; n++) {
                    double nr, ni;
                    if (n == m + 1) {
                        const double f = (2 * m + 1) * rz * ir2;
                        nr = f * cr;
                        ni = f * ci;
                    } else {
                        const double aa = (2 * n - 1) * rz, bb = (double)((n - 1) * (n - 1) - m * m);
                        nr = (aa * cr - bb * pr) * ir2;
                        ni = (aa * ci - bb * pi) * ir2;
                    }
                    put(n, nr, ni);
                    pr = cr;
                    pi = ci;
                    cr = nr;
                    ci = ni;
                }
            }
            __syncthreads();
#pragma unroll 1
            for (int s = 0; s < 3; s++) {
                const int n = on[s];
                if (!act || n < 0) continue;
                const int m = om[s];
                // S_n^m = sum_k 2^(delta k) sum_l M_k^l J_(n+k)^(m+l); with
                // |m| <= n and |l| <= k every J index lies in row n + k <= 2p
                double sr = 0, si = 0;
                if (kMutual && mutual) {
                    // and the reverse R_n^m = sum_k (-1)^k sum_l A_k^l J_(n+k)^(m+l)
                    double qr = 0, qi = 0;
#pragma unroll
                    for (int k = 0; k <= p; k++) {
                        const int nn = n + k;
                        const double2 *jr = J + (nn * nn + nn + m);
                        const double2 *mk = Mc + (k * k + k);
                        const double2 *ak = Ac + (k * k + k);
                        double tr = 0, ti = 0, ur = 0, ui = 0;
#pragma unroll
                        for (int l = -k; l <= k; l++) {
                            const double2 jv = jr[l], mv = mk[l], av = ak[l];
                            tr = fma(mv.x, jv.x, tr);
                            tr = fma(-mv.y, jv.y, tr);
                            ti = fma(mv.x, jv.y, ti);
                            ti = fma(mv.y, jv.x, ti);
                            ur = fma(av.x, jv.x, ur);
                            ur = fma(-av.y, jv.y, ur);
                            ui = fma(av.x, jv.y, ui);
                            ui = fma(av.y, jv.x, ui);
                        }
                        const double fk = ldexp(1.0, delta * k);
                        sr = fma(fk, tr, sr);
                        si = fma(fk, ti, si);
                        qr += (k & 1) ? -ur : ur;
                        qi += (k & 1) ? -ui : ui;
                    }
                    const double fo = ldexp(1.0, delta * (n + 1));
                    revr[s] = fo * qr;
                    revi[s] = fo * qi;
                } else {
#pragma unroll
                    for (int k = 0; k <= p; k++) {
                        const int nn = n + k;
                        const double2 *jr = J + (nn * nn + nn + m);
                        const double2 *mk = Mc + (k * k + k);
                        double tr = 0, ti = 0;
#pragma unroll
                        for (int l = -k; l <= k; l++) {
                            const double2 mv = mk[l], jv = jr[l];
                            tr = fma(mv.x, jv.x, tr);
                            tr = fma(-mv.y, jv.y, tr);
                            ti = fma(mv.x, jv.y, ti);
                            ti = fma(mv.y, jv.x, ti);
                        }
                        const double fk = ldexp(1.0, delta * k);
                        sr = fma(fk, tr, sr);
                        si = fma(fk, ti, si);
                    }
                }
                if (n & 1) {
                    sr = -sr;
                    si = -si;
                }
                accr[s] += sr;
                acci[s] += si;
            }
            if (kMutual && mutual) {
                double *out = Out + (int64_t)B * P;
                for (int s = 0; s < 3; s++) {
                    const int n = on[s];
                    if (n < 0) continue;
                    const int m = om[s];
                    atomicAdd(&out[cidx_re(n, m)], revr[s]);
                    if (m > 0) atomicAdd(&out[cidx_im(n, m)], revi[s]);
                }
            }
        }
        if (any) flush(O);
    }
}

}  // namespace

namespace {
void launch_pairs(bool adjoint, Geometry g, int32_t ncell, int p, const int32_t *ptr, const int32_t *src, int64_t npair,
                  const double *In, double *Out, bool owner_mode, hipStream_t s, bool mutual = false) {
    if (ncell == 0 || npair <= 0) return;
    if (mutual && (adjoint || owner_mode))
        throw HipError{hipErrorInvalidValue, "mutual M2L: forward, balanced mode only"};
    const int64_t nunit = owner_mode ? (int64_t)ncell : (npair + kPairChunk - 1) / kPairChunk;
    const int grid = (int)(nunit < 65536 ? nunit : 65536);
    const int om = owner_mode ? 1 : 0;
    const size_t lds =
        (size_t)m2l_pairs_streams(p, owner_mode) * m2l_pairs_lds_mutual_doubles(p, mutual) * sizeof(double);
    if (adjoint) {
        hipLaunchKernelGGL(k_m2l_pairs_adj, dim3(grid), dim3(kM2L64Threads), lds, s, g.c, ncell, p, ptr, src, npair,
                           In, Out, om);
    } else {
        switch (p) {
#define FMM_PAIRS(PP)                                                                                             \
    case PP:                                                                                                      \
        if (mutual)                                                                                               \
            hipLaunchKernelGGL((k_m2l_pairs_fwd<PP, true>), dim3(grid), dim3(kM2L64Threads), lds, s, g.c, ncell, ptr, \
                               src, npair, In, Out, om);                                                          \
        else                                                                                                      \
            hipLaunchKernelGGL((k_m2l_pairs_fwd<PP, false>), dim3(grid), dim3(kM2L64Threads), lds, s, g.c, ncell,     \
                               ptr, src, npair, In, Out, om);                                                     \
        break;
            FMM_PAIRS(0) FMM_PAIRS(1) FMM_PAIRS(2) FMM_PAIRS(3) FMM_PAIRS(4) FMM_PAIRS(5) FMM_PAIRS(6)
            FMM_PAIRS(7) FMM_PAIRS(8) FMM_PAIRS(9) FMM_PAIRS(10) FMM_PAIRS(11) FMM_PAIRS(12) FMM_PAIRS(13)
            FMM_PAIRS(14) FMM_PAIRS(15) FMM_PAIRS(16)
#undef FMM_PAIRS
            default: throw HipError{hipErrorInvalidValue, "per-pair M2L: unsupported order"};
        }
    }
    FMM_LAUNCH_CHECK();
}
}  // namespace

void launch_m2l_fp64_adjoint(Geometry g, int32_t ncell, int p, const int32_t *ptr_t, const int32_t *src_t,
                             int64_t npair, const double *Lam, double *Mu, int add, bool owner_mode, hipStream_t s) {
    if (!add) fill_zero(Mu, (size_t)ncell * ncoef(p) * sizeof(double), s);
    launch_pairs(true, g, ncell, p, ptr_t, src_t, npair, Lam, Mu, owner_mode, s);
}

void launch_p2p_fp64(Geometry g, int32_t ncell, const int32_t *ptr, const int32_t *src, const double *xs,
                     const double *ys, const double *zs, const double *qs, double *phi, double *fld, hipStream_t s) {
    if (ncell == 0) return;
    hipLaunchKernelGGL(k_p2p_fp64, dim3(ncell), dim3(kP2P64Threads), 0, s, g.c, ncell, ptr, src, xs, ys, zs, qs, phi,
                       fld);
    FMM_LAUNCH_CHECK();
}

void launch_m2l_fp64(Geometry g, int32_t ncell, int p, const int32_t *ptr, const int32_t *src, int64_t npair,
                     const double *M, double *L, bool owner_mode, hipStream_t s) {
    fill_zero(L, (size_t)ncell * ncoef(p) * sizeof(double), s);
    launch_pairs(false, g, ncell, p, ptr, src, npair, M, L, owner_mode, s);
}

void launch_m2l_fp64_add(Geometry g, int32_t ncell, int p, const int32_t *ptr, const int32_t *src, int64_t npair,
                         const double *M, double *L, bool owner_mode, hipStream_t s) {
    launch_pairs(false, g, ncell, p, ptr, src, npair, M, L, owner_mode, s);
}

void launch_p2p_fp64_mutual(Geometry g, int32_t ncell, int64_t n, const int32_t *ptr, const int32_t *src,
                            const double *xs, const double *ys, const double *zs, const double *qs, double *phi,
                            double *fld, hipStream_t s) {
    if (ncell == 0) return;
    fill_zero(phi, (size_t)n * sizeof(double), s);
    fill_zero(fld, (size_t)n * 3 * sizeof(double), s);
    hipLaunchKernelGGL(k_p2p_fp64_mutual, dim3(ncell), dim3(kP2P64Threads), 0, s, g.c, ncell, ptr, src, xs, ys, zs,
                       qs, phi, fld);
    FMM_LAUNCH_CHECK();
}

void launch_m2l_fp64_mutual(Geometry g, int32_t ncell, int p, const int32_t *ptr, const int32_t *src, int64_t npair,
                            const double *M, double *L, hipStream_t s) {
    fill_zero(L, (size_t)ncell * ncoef(p) * sizeof(double), s);
    launch_pairs(false, g, ncell, p, ptr, src, npair, M, L, false, s, true);
}

}  // namespace fmm
