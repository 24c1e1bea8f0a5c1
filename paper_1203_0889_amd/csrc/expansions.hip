// Multipole and local expansions in scaled solid harmonics, FP64
// (P2M, M2M, L2L, L2P stages of Sec. 2.1).
//
// Basis.  For x = (x, y, z), r^2 = |x|^2, zeta = x + i y, the regular solid
// harmonics R_n^m (m >= 0) satisfy
//   R_0^0 = 1,  R_m^m = R_(m-1)^(m-1) zeta / (2m),  R_(m+1)^m = z R_m^m,
//   R_n^m = ((2n-1) z R_(n-1)^m - r^2 R_(n-2)^m) / ((n+m)(n-m)),
// with R_n^(-m) = (-1)^m conj(R_n^m).  They obey the addition theorem
// R_n^m(a + b) = sum_(k,l) R_k^l(a) R_(n-k)^(m-l)(b) and, with the irregular
// harmonics I_n^m of the M2L kernel, 1/|x - y| = sum conj(R_n^m(y)) I_n^m(x).
//
// Scaling.  A cell of side S with centre c keeps
//   multipole  M~_n^m = sum_j q_j conj(R_n^m((y_j - c) / S))
//   local      phi(x) = (1/S) sum_(n,m) L~_n^m conj(R_n^m((x - c) / S)),
// so that child <-> parent translations are the same 8 matrices on every
// level, and every coefficient stays O(charge) -- the property that lets the
// M2L run in FP32 without range problems.
//   M2M: M~_P,n^m = 2^-n     sum_(k,l) M~_C,k^l conj(R_(n-k)^(m-l)(d))
//   L2L: L~_C,k^l = sum_(n,m) 2^-(n+1) L~_P,n^m conj(R_(n-k)^(m-l)(d))
// with d = (c_child - c_parent) / S_child = (+-1/2, +-1/2, +-1/2).
// Coefficients are stored as (p+1)^2 reals per cell: for each degree n,
// Re(m = 0), then Re, Im for m = 1..n.
#include <complex>

#include "tree.h"

namespace fmm {

namespace {

struct Cplx {
    double re, im;
};
__device__ inline Cplx cmul(Cplx a, Cplx b) { return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re}; }
__device__ inline Cplx cconj(Cplx a) { return {a.re, -a.im}; }

// Geometric centre and side of a cell, FP64: c = min + (2i+1) side / 2^(l+1).
__device__ inline void cell_frame(const Geometry &g, int32_t cell, double *c, double *side_l, int *level) {
    int l = g.c.level[cell], k = g.c.inst[cell];
    const double *b = g.box + 4 * k;
    double side = b[3];
    double den = ldexp(1.0, l + 1);
    c[0] = b[0] + ((double)(2 * (int64_t)g.c.ix[cell] + 1) * side) / den;
    c[1] = b[1] + ((double)(2 * (int64_t)g.c.iy[cell] + 1) * side) / den;
    c[2] = b[2] + ((double)(2 * (int64_t)g.c.iz[cell] + 1) * side) / den;
    *side_l = side;
    *level = l;
}

// P2M: one thread per (cell, order m); non-leaves exit.  Degrees n = m..PP
// are accumulated in registers (PP = p at compile time), with the recurrence
// constants 1/((n+m)(n-m)) computed once per thread.
template <int PP>
__global__ void k_p2m(Geometry g, int32_t ncell, const double *__restrict__ xs, const double *__restrict__ ys,
                      const double *__restrict__ zs, const double *__restrict__ qs, double *__restrict__ M) {
    int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    int32_t cell = (int32_t)(t / (PP + 1));
    const int m = (int)(t % (PP + 1));
    if (cell >= ncell || g.c.child[cell] >= 0) return;
    constexpr int P = ncoef(PP);
    double c[3], side;
    int l;
    cell_frame(g, cell, c, &side, &l);
    const double inv_side = ldexp(1.0 / side, l);
    double dmm = 1.0;  // 1 / (2^m m!)
    for (int i = 1; i <= m; i++) dmm /= 2 * i;
    double inv[PP + 1];
#pragma unroll
    for (int n = 0; n <= PP; n++) inv[n] = n >= m + 2 ? 1.0 / (double)((n + m) * (n - m)) : 0.0;
    double ar[PP + 1], ai[PP + 1];
#pragma unroll
    for (int n = 0; n <= PP; n++) ar[n] = ai[n] = 0.0;
    int32_t f = g.c.first[cell], e = f + g.c.count[cell];
    // the next particle's loads are issued before this one's arithmetic
    double nx = 0.0, ny = 0.0, nz = 0.0, nq = 0.0;
    if (f < e) {
        nx = xs[f];
        ny = ys[f];
        nz = zs[f];
        nq = qs[f];
    }
    for (int32_t r = f; r < e; r++) {
        const double px = nx, py = ny, pz = nz, q = nq;
        if (r + 1 < e) {
            nx = xs[r + 1];
            ny = ys[r + 1];
            nz = zs[r + 1];
            nq = qs[r + 1];
        }
        double ux = (px - c[0]) * inv_side, uy = (py - c[1]) * inv_side, uz = (pz - c[2]) * inv_side;
        double r2 = ux * ux + uy * uy + uz * uz;
        Cplx cur = {dmm, 0.0};
        for (int i = 1; i <= m; i++) cur = cmul(cur, Cplx{ux, uy});
        Cplx prev = {0.0, 0.0};
#pragma unroll
        for (int n = 0; n <= PP; n++) {
            if (n < m) continue;
            if (n == m + 1) {
                prev = cur;
                cur = {uz * cur.re, uz * cur.im};
            } else if (n > m + 1) {
                double a = (2 * n - 1) * uz;
                Cplx nx = {(a * cur.re - r2 * prev.re) * inv[n], (a * cur.im - r2 * prev.im) * inv[n]};
                prev = cur;
                cur = nx;
            }
            ar[n] += q * cur.re;
            ai[n] -= q * cur.im;
        }
    }
    double *out = M + (int64_t)cell * P;
#pragma unroll
    for (int n = 0; n <= PP; n++) {
        if (n < m) continue;
        out[cidx_re(n, m)] = ar[n];
        if (m > 0) out[cidx_im(n, m)] = ai[n];
    }
}

__device__ inline int octant_of(const CellArrays &c, int32_t cell) {
    return (c.ix[cell] & 1) | ((c.iy[cell] & 1) << 1) | ((c.iz[cell] & 1) << 2);
}

// M2M and L2L, octant-major: for each octant o a dense (p+1)^2 x (p+1)^2
// operator (column-major) applied to the vectors of a level's parents; wide
// levels in a register-tiled kernel, levels of at most kSmallLevel parents
// one block per (parent, octant).  A level's parents are listed (cells with
// children, in cell order), so its leaves take no blocks: on an adaptive
// tree most cells of the deep levels are leaves.

__device__ inline int32_t child_in_octant(const CellArrays &c, int32_t parent, int o) {
    int32_t ch = c.child[parent];
    if (ch < 0) return -1;
    int nch = c.nchild[parent];
    for (int k = 0; k < nch; k++)
        if (octant_of(c, ch + k) == o) return ch + k;
    return -1;
}

constexpr int kTransMaxThreads = 320;  // rows_block(p) for p <= 16

// Number of parents of the level with cells [lb, le): at most the host's
// bound, which sizes the grids and the partial sums.
__device__ inline int32_t level_parents(const LevelParents &lp, int32_t lb, int32_t le) {
    const int32_t n = lp.ppos[le] - lp.ppos[lb];
    return n < 0 ? 0 : (n < lp.npar_max ? n : lp.npar_max);
}

__global__ void k_m2m_sum(int32_t lb, int32_t le, int p, LevelParents lp, const double *__restrict__ part,
                          double *__restrict__ M) {
    const int P = ncoef(p);
    const int64_t n = (int64_t)level_parents(lp, lb, le) * P, stride = (int64_t)lp.npar_max * P;
    const int32_t *__restrict__ pl = lp.plist + lp.ppos[lb];
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int32_t par = pl[i / P];
        double s = 0.0;
        for (int o = 0; o < 8; o++) s += part[(int64_t)o * stride + i];
        M[(int64_t)par * P + (i % P)] = s;
    }
}

// Wide levels, register-tiled: block (npb listed parents, octant o), 256 threads;
// a thread owns a tile of kTR rows x kTP parents.  Per chunk of cw columns
// the block stages the operator columns (rows padded to Pp = kTR
// ceil(P / kTR), zeros below P) and the matching rows of the npb input
// vectors in LDS; each k then costs a thread kTR + kTP LDS values for
// kTR kTP FMAs.  Sums run over the columns in order with one accumulator
// per output, like the small-level kernels, so both give the same values.
//   M2M (kL2L = false): input = the octant-o children's M, output
//       part[o][parent's rank in the level][row] (zero without such a child);
//   L2L (kL2L = true): input = the parents' L, output added into the
//       octant-o children's L.
// Measured at p = 8 on the 4,096-parent level (L2L / M2M): 4 x 8 tiles,
// 64 parents per block, 60 KB of LDS: 56 / 83 us; 4 x 4 tiles, 32 parents,
// 36 KB: 45 / 60 us; 4 x 4, 16 parents, 24 KB: 60 / 81 us.  The kernel
// waits on memory about half of its time (SQ_WAIT_ANY).
constexpr int kTR = 4, kTP = 4, kTileThreads = 256;
constexpr int kTileMaxParents = 32;
constexpr int kTileRoomKB = 36;

struct TileShape {
    int Pp, npb, xs, cw;   // padded rows, parents per block, LDS row stride of the inputs, columns per chunk
};

template <bool kL2L>
__global__ void __launch_bounds__(kTileThreads) k_trans_tiled(Geometry g, int32_t lb, int32_t le, int p, TileShape ts,
                                                              LevelParents lp, const double *__restrict__ ops,
                                                              const double *__restrict__ in, double *__restrict__ out) {
    extern __shared__ double dyn[];
    __shared__ int32_t kid[kTileMaxParents], pid[kTileMaxParents];
    const int P = ncoef(p);
    const int Pp = ts.Pp, npb = ts.npb, XS = ts.xs, cw = ts.cw;
    double *opS = dyn;              // cw x Pp, column-major
    double *xS = dyn + cw * Pp;     // cw x XS, k-major
    const int o = blockIdx.y;
    const int32_t npar = level_parents(lp, lb, le);
    const int32_t r0 = blockIdx.x * npb;   // rank of the block's first parent in the level
    if (r0 >= npar) return;                // the grid covers the host's bound on the parents
    const int PG = npb / kTP, RG = Pp / kTR;
    const int rg = threadIdx.x / PG, pg = threadIdx.x - rg * PG;
    const bool active = rg < RG;
    if (threadIdx.x < npb) {
        const int32_t r = r0 + threadIdx.x;
        const int32_t par = r < npar ? lp.plist[lp.ppos[lb] + r] : -1;
        pid[threadIdx.x] = par;
        kid[threadIdx.x] = par >= 0 ? child_in_octant(g.c, par, o) : -1;
    }
    double acc[kTR][kTP];
#pragma unroll
    for (int i = 0; i < kTR; i++)
#pragma unroll
        for (int j = 0; j < kTP; j++) acc[i][j] = 0.0;
    const double *A = ops + (int64_t)o * P * P;
    for (int c0 = 0; c0 < P; c0 += cw) {
        const int w = P - c0 < cw ? P - c0 : cw;
        __syncthreads();   // kid ready; the last chunk's reads done
        // staging: kStageBatch loads in flight per thread before their stores
        constexpr int kStageBatch = 8;
        const int nop = w * Pp, nx = npb * w;
        for (int i0 = threadIdx.x; i0 < nop; i0 += kTileThreads * kStageBatch) {
            double v[kStageBatch];
#pragma unroll
            for (int b = 0; b < kStageBatch; b++) {
                const int i = i0 + b * kTileThreads;
                const int k = i / Pp, r = i - k * Pp;
                v[b] = (i < nop && r < P) ? A[(int64_t)(c0 + k) * P + r] : 0.0;
            }
#pragma unroll
            for (int b = 0; b < kStageBatch; b++)
                if (i0 + b * kTileThreads < nop) opS[i0 + b * kTileThreads] = v[b];
        }
        for (int i0 = threadIdx.x; i0 < nx; i0 += kTileThreads * kStageBatch) {
            double v[kStageBatch];
#pragma unroll
            for (int b = 0; b < kStageBatch; b++) {
                const int i = i0 + b * kTileThreads;
                const int j = i / w, k = i - j * w;   // consecutive threads read consecutive coefficients
                const int32_t src = i >= nx || kid[j] < 0 ? -1 : (kL2L ? pid[j] : kid[j]);
                v[b] = src >= 0 ? in[(int64_t)src * P + c0 + k] : 0.0;
            }
#pragma unroll
            for (int b = 0; b < kStageBatch; b++) {
                const int i = i0 + b * kTileThreads;
                if (i < nx) {
                    const int j = i / w, k = i - j * w;
                    xS[k * XS + j] = v[b];
                }
            }
        }
        __syncthreads();
        if (active)
            for (int k = 0; k < w; k++) {
                double a[kTR], x[kTP];
#pragma unroll
                for (int i = 0; i < kTR; i++) a[i] = opS[k * Pp + kTR * rg + i];
#pragma unroll
                for (int j = 0; j < kTP; j++) x[j] = xS[k * XS + kTP * pg + j];
#pragma unroll
                for (int i = 0; i < kTR; i++)
#pragma unroll
                    for (int j = 0; j < kTP; j++) acc[i][j] += a[i] * x[j];
            }
    }
    if (!active) return;
    if (kL2L) {   // all the children's old values in flight before the adds
        int32_t ch[kTP];
        double old[kTR][kTP];
#pragma unroll
        for (int j = 0; j < kTP; j++) {
            ch[j] = kid[kTP * pg + j];
#pragma unroll
            for (int i = 0; i < kTR; i++) {
                const int r = kTR * rg + i;
                old[i][j] = (ch[j] >= 0 && r < P) ? out[(int64_t)ch[j] * P + r] : 0.0;
            }
        }
#pragma unroll
        for (int j = 0; j < kTP; j++)
#pragma unroll
            for (int i = 0; i < kTR; i++) {
                const int r = kTR * rg + i;
                if (ch[j] >= 0 && r < P) out[(int64_t)ch[j] * P + r] = old[i][j] + acc[i][j];
            }
        return;
    }
#pragma unroll
    for (int j = 0; j < kTP; j++) {
        const int32_t rank = r0 + kTP * pg + j;
        if (rank >= npar) continue;
#pragma unroll
        for (int i = 0; i < kTR; i++) {
            const int r = kTR * rg + i;
            if (r < P) out[((int64_t)o * lp.npar_max + rank) * P + r] = acc[i][j];
        }
    }
}

// Levels with few parents: one block per (parent, octant), a thread per
// row, the operator read straight from global memory (it stays in L2) and
// the one vector in LDS.  A block then waits for about one pass of loads
// instead of a staging round trip per operator chunk, which dominated the
// top levels (tens of microseconds each whatever their size).  The sum runs
// over the columns in the same order with one accumulator, as in the
// register-tiled kernel, so both forms give the same values.
constexpr int32_t kSmallLevel = 256;   // parents per level up to which these are used
constexpr int kMaxCoef = 17 * 17;      // (p + 1)^2 for p <= 16

__global__ void __launch_bounds__(kTransMaxThreads) k_m2m_small(Geometry g, int32_t lb, int32_t le, int p,
                                                                LevelParents lp, const double *__restrict__ ops,
                                                                const double *__restrict__ M, double *__restrict__ part) {
    __shared__ double x[kMaxCoef];
    const int P = ncoef(p);
    const int o = blockIdx.y;
    const int32_t rank = blockIdx.x;
    if (rank >= level_parents(lp, lb, le)) return;
    const int32_t par = lp.plist[lp.ppos[lb] + rank];
    const int row = threadIdx.x;
    const int32_t ch = child_in_octant(g.c, par, o);   // the same in every thread
    double *out = part + ((int64_t)o * lp.npar_max + rank) * P;
    if (ch < 0) {
        if (row < P) out[row] = 0.0;
        return;
    }
    for (int i = threadIdx.x; i < P; i += blockDim.x) x[i] = M[(int64_t)ch * P + i];
    __syncthreads();
    if (row >= P) return;
    const double *A = ops + (int64_t)o * P * P + row;
    double acc = 0.0;
    for (int i = 0; i < P; i++) acc += A[(int64_t)i * P] * x[i];
    out[row] = acc;
}

__global__ void __launch_bounds__(kTransMaxThreads) k_l2l_small(Geometry g, int32_t lb, int32_t le, int p,
                                                                LevelParents lp, const double *__restrict__ ops,
                                                                double *__restrict__ L) {
    __shared__ double x[kMaxCoef];
    const int P = ncoef(p);
    const int o = blockIdx.y;
    const int32_t rank = blockIdx.x;
    if (rank >= level_parents(lp, lb, le)) return;
    const int32_t par = lp.plist[lp.ppos[lb] + rank];
    const int row = threadIdx.x;
    const int32_t ch = child_in_octant(g.c, par, o);
    if (ch < 0) return;
    for (int i = threadIdx.x; i < P; i += blockDim.x) x[i] = L[(int64_t)par * P + i];
    __syncthreads();
    if (row >= P) return;
    const double *B = ops + (int64_t)o * P * P + row;
    double acc = 0.0;
    for (int i = 0; i < P; i++) acc += B[(int64_t)i * P] * x[i];
    L[(int64_t)ch * P + row] += acc;
}

// Local coefficient L~_n^m for any m (negative via conjugate symmetry).
__device__ inline Cplx lget(const double *Lc, int p, int n, int m) {
    if (n > p || m > n || -m > n) return {0.0, 0.0};
    int am = m < 0 ? -m : m;
    Cplx v = {Lc[cidx_re(n, am)], am > 0 ? Lc[cidx_im(n, am)] : 0.0};
    if (m < 0) {
        v.im = -v.im;
        if (am & 1) {
            v.re = -v.re;
            v.im = -v.im;
        }
    }
    return v;
}

// L2P: thread per sorted particle.  Translating the local expansion to the
// particle gives phi from degree 0 and the gradient from degree 1:
//   phi            = (1/S)   sum_(n,m) L~_n^m     conj(R_n^m(u))
//   d/du (z)       = sum     L~_(n+1)^m   conj(R_n^m(u))
//   d/du (x + i y) = sum     L~_(n+1)^(m+1) conj(R_n^m(u))
// and E = -(1/S^2) grad_u.
// At least three waves per SIMD (168 registers instead of 169: 102 -> 96 us at p = 8).
template <int PP>
__global__ void __launch_bounds__(128, 3) k_l2p(Geometry g, int64_t n, const int32_t *__restrict__ leaf_of,
                                             const double *__restrict__ xs, const double *__restrict__ ys,
                                             const double *__restrict__ zs, const double *__restrict__ L,
                                             double *__restrict__ phi, double *__restrict__ fld, FinalOut out) {
    constexpr int p = PP;
    constexpr int P = ncoef(PP);
    for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < n; r += (int64_t)gridDim.x * blockDim.x) {
        int32_t cell = leaf_of[r];
        double c[3], side;
        int l;
        cell_frame(g, cell, c, &side, &l);
        // multiplications by reciprocals (the divisors are compile-time
        // constants after unrolling, or one per particle): FP64 divisions
        // cost about ten instructions each and there are ~90 per particle
        const double inv_side = ldexp(1.0 / side, l);
        double ux = (xs[r] - c[0]) * inv_side;
        double uy = (ys[r] - c[1]) * inv_side;
        double uz = (zs[r] - c[2]) * inv_side;
        double r2 = ux * ux + uy * uy + uz * uz;
        const double *Lc = L + (int64_t)cell * P;
        Cplx zeta = {ux, uy};
        Cplx rmm = {1.0, 0.0};
        Cplx a0 = {0, 0}, gz = {0, 0}, gxy = {0, 0};
#pragma unroll
        for (int m = 0; m <= p; m++) {
            if (m > 0) {
                rmm = cmul(rmm, zeta);
                const double h = 1.0 / (2 * m);
                rmm.re *= h;
                rmm.im *= h;
            }
            Cplx r2m = {0.0, 0.0}, r1m = {0.0, 0.0};
#pragma unroll
            for (int nn = m; nn <= p; nn++) {
                Cplx rn;
                if (nn == m) {
                    rn = rmm;
                } else if (nn == m + 1) {
                    rn = {uz * r1m.re, uz * r1m.im};
                } else {
                    const double a = (2 * nn - 1) * uz, rden = 1.0 / (double)((nn + m) * (nn - m));
                    rn = {(a * r1m.re - r2 * r2m.re) * rden, (a * r1m.im - r2 * r2m.im) * rden};
                }
                r2m = r1m;
                r1m = rn;
                // order +m
                Cplx cr = cconj(rn);
                Cplx t;
                t = cmul(lget(Lc, p, nn, m), cr);
                a0.re += t.re; a0.im += t.im;
                t = cmul(lget(Lc, p, nn + 1, m), cr);
                gz.re += t.re; gz.im += t.im;
                t = cmul(lget(Lc, p, nn + 1, m + 1), cr);
                gxy.re += t.re; gxy.im += t.im;
                if (m > 0) {
                    // order -m: conj(R_n^-m) = (-1)^m R_n^m
                    Cplx cm = (m & 1) ? Cplx{-rn.re, -rn.im} : rn;
                    t = cmul(lget(Lc, p, nn, -m), cm);
                    a0.re += t.re; a0.im += t.im;
                    t = cmul(lget(Lc, p, nn + 1, -m), cm);
                    gz.re += t.re; gz.im += t.im;
                    t = cmul(lget(Lc, p, nn + 1, -m + 1), cm);
                    gxy.re += t.re; gxy.im += t.im;
                }
            }
        }
        double invS = ldexp(1.0 / side, l);
        const double pf = a0.re * invS;
        double e2 = invS * invS;
        const double fx = -gxy.re * e2, fy = -gxy.im * e2, fz = -gz.re * e2;
        phi[r] = pf;
        fld[3 * r] = fx;
        fld[3 * r + 1] = fy;
        fld[3 * r + 2] = fz;
        if (out.perm) {   // uniform: the evaluation's outputs, in input order
            const int64_t i = out.perm[r];
            const double ex = out.fld_near[3 * r] + fx, ey = out.fld_near[3 * r + 1] + fy,
                         ez = out.fld_near[3 * r + 2] + fz;
            if (out.phi) out.phi[i] = out.phi_near[r] + pf;
            if (out.field) {
                out.field[3 * i] = ex;
                out.field[3 * i + 1] = ey;
                out.field[3 * i + 2] = ez;
            }
            if (out.force) {
                const double q = out.qs[r];
                out.force[3 * i] = q * ex;
                out.force[3 * i + 1] = q * ey;
                out.force[3 * i + 2] = q * ez;
            }
        }
    }
}

// ---------------------------------------------------------------- adjoint
// P2M stores C_k(u) = (Re R_n^m(u), -Im R_n^m(u)) per unit charge, and L2P
// evaluates phi = sum_k L_k B_k(u) with B_k = (s_k / S) C_k, s_k = 1 for
// m = 0, 2 for Re and -2 for Im of m > 0 (the +-m terms of a real field).
// Hence the transposed stages reuse those kernels with a diagonal scaling:
//   L2P^T(w) = diag(s_k / S) P2M(w),   P2M^T(mu) = L2P(diag(S / s_k) mu).
// dir = 0 multiplies leaf rows by s_k / S, dir = 1 by S / s_k.
__global__ void k_dual_scale(Geometry g, int32_t ncell, int p, double *__restrict__ X, int dir) {
    const int P = ncoef(p);
    const int64_t total = (int64_t)ncell * P;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
        const int32_t cell = (int32_t)(i / P);
        if (g.c.child[cell] >= 0) continue;
        const int k = (int)(i - (int64_t)cell * P);
        int n = 0;
        while ((n + 1) * (n + 1) <= k) n++;
        const int off = k - n * n;
        const double sk = off == 0 ? 1.0 : ((off & 1) ? 2.0 : -2.0);
        const int l = g.c.level[cell];
        const double S = ldexp(g.box[4 * g.c.inst[cell] + 3], -l);
        X[i] *= dir == 0 ? sk / S : S / sk;
    }
}

// Adjoint weights w_i = g_(instance of i) q_i (sorted order).
__global__ void k_adjoint_weights(int64_t n, const int32_t *__restrict__ leaf_of, const int32_t *__restrict__ inst,
                                  const double *__restrict__ gE, const double *__restrict__ qs, double *__restrict__ w) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        w[i] = gE[inst[leaf_of[i]]] * qs[i];
}

// E = sum_k g_k 1/2 q^T A q per instance, A the FMM's (non-symmetric) matrix:
//   dE/dq_i = 1/2 g q-phi term + 1/2 (A^T w)_i   = 1/2 (g_i phi_i + psi_i)
//   dE/dx_i = 1/2 g_i q_i grad phi(x_i) + 1/2 q_i grad psi(x_i)
//           = -1/2 q_i (g_i E_i + E^psi_i),
// with psi = A^T w (w = g q) and E^psi = -grad psi, both from the transposed
// evaluation.  Written in input order.
__global__ void k_adjoint_finalize(int64_t n, const uint32_t *__restrict__ perm, const int32_t *__restrict__ leaf_of,
                                   const int32_t *__restrict__ inst, const double *__restrict__ gE,
                                   const double *__restrict__ qs, const double *__restrict__ pn,
                                   const double *__restrict__ fn, const double *__restrict__ pf,
                                   const double *__restrict__ ff, const double *__restrict__ sn,
                                   const double *__restrict__ en, const double *__restrict__ sf,
                                   const double *__restrict__ ef, double *__restrict__ grad_pos,
                                   double *__restrict__ grad_q) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const double g = gE[inst[leaf_of[i]]];
        const int64_t o = perm[i];
        if (grad_q) grad_q[o] = 0.5 * (g * (pn[i] + pf[i]) + (sn[i] + sf[i]));
        if (grad_pos) {
            const double hq = -0.5 * qs[i];
            for (int d = 0; d < 3; d++)
                grad_pos[3 * o + d] = hq * (g * (fn[3 * i + d] + ff[3 * i + d]) + (en[3 * i + d] + ef[3 * i + d]));
        }
    }
}

// The outputs from the near and far fields of every sorted particle r, in
// input order (perm[r] = input index of r); force = q E.
__global__ void k_finalize(int64_t n, const uint32_t *__restrict__ perm, const double *__restrict__ qs,
                           const double *__restrict__ pn, const double *__restrict__ fn, const double *__restrict__ pf,
                           const double *__restrict__ ff, double *__restrict__ phi, double *__restrict__ field,
                           double *__restrict__ force) {
    for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < n; r += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = perm[r];
        const double ex = fn[3 * r] + ff[3 * r], ey = fn[3 * r + 1] + ff[3 * r + 1], ez = fn[3 * r + 2] + ff[3 * r + 2];
        if (phi) phi[i] = pn[r] + pf[r];
        if (field) {
            field[3 * i] = ex;
            field[3 * i + 1] = ey;
            field[3 * i + 2] = ez;
        }
        if (force) {
            const double q = qs[r];
            force[3 * i] = q * ex;
            force[3 * i + 1] = q * ey;
            force[3 * i + 2] = q * ez;
        }
    }
}

// E_k = 1/2 sum_(i in k) q_i phi_i in a fixed order: per-chunk partial sums
// (chunks never straddle instances), then per-instance sums of the chunks.
// With out.perm set, the same pass also writes the outputs of its particles
// (near + far, input order; ff = far field), like k_finalize.
constexpr int kEnergyChunk = 1024;

__global__ void __launch_bounds__(256) k_energy_part(const int64_t *__restrict__ offsets, int n_inst,
                                                     const int32_t *__restrict__ chunk_off, const double *__restrict__ qs,
                                                     const double *__restrict__ pn, const double *__restrict__ pf,
                                                     double *__restrict__ part, FinalOut out,
                                                     const double *__restrict__ ff) {
    __shared__ double red[256];
    int j = blockIdx.x;
    // instance of chunk j: largest k with chunk_off[k] <= j
    int lo = 0, hi = n_inst - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (chunk_off[mid] <= j) lo = mid; else hi = mid - 1;
    }
    int64_t b = offsets[lo] + (int64_t)(j - chunk_off[lo]) * kEnergyChunk;
    int64_t e = b + kEnergyChunk < offsets[lo + 1] ? b + kEnergyChunk : offsets[lo + 1];
    double s = 0.0;
    for (int64_t r = b + threadIdx.x; r < e; r += 256) {
        const double ph = pn[r] + pf[r];
        s += qs[r] * ph;
        if (out.perm) {   // uniform
            const int64_t i = out.perm[r];
            const double *fn = out.fld_near;
            const double ex = fn[3 * r] + ff[3 * r], ey = fn[3 * r + 1] + ff[3 * r + 1], ez = fn[3 * r + 2] + ff[3 * r + 2];
            if (out.phi) out.phi[i] = ph;
            if (out.field) {
                out.field[3 * i] = ex;
                out.field[3 * i + 1] = ey;
                out.field[3 * i + 2] = ez;
            }
            if (out.force) {
                const double q = qs[r];
                out.force[3 * i] = q * ex;
                out.force[3 * i + 1] = q * ey;
                out.force[3 * i + 2] = q * ez;
            }
        }
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[j] = red[0];
}

// One wave per instance: lane l sums chunks l, l + 64, ... in order, then
// a fixed butterfly adds the 64 lane sums.
__global__ void __launch_bounds__(64) k_energy_sum(int n_inst, const int32_t *__restrict__ chunk_off,
                                                   const double *__restrict__ part, double *__restrict__ energy) {
    const int k = blockIdx.x;
    if (k >= n_inst) return;
    double s = 0.0;
    for (int j = chunk_off[k] + (int)threadIdx.x; j < chunk_off[k + 1]; j += 64) s += part[j];
#pragma unroll
    for (int d = 32; d > 0; d >>= 1) s += __shfl_xor(s, d, 64);
    if (threadIdx.x == 0) energy[k] = 0.5 * s;
}

}  // namespace

// ---------------------------------------------------------------- host side

namespace {
using cd = std::complex<double>;

// Regular solid harmonics R_n^m(x) for 0 <= m <= n <= p (host, FP64).
std::vector<cd> host_regular(const double *x, int p) {
    std::vector<cd> R((size_t)(p + 1) * (p + 1), cd(0, 0));
    double r2 = x[0] * x[0] + x[1] * x[1] + x[2] * x[2];
    cd zeta(x[0], x[1]);
    auto at = [&](int n, int m) -> cd & { return R[(size_t)n * (p + 1) + m]; };
    at(0, 0) = 1.0;
    for (int m = 0; m <= p; m++) {
        if (m > 0) at(m, m) = at(m - 1, m - 1) * zeta / (2.0 * m);
        if (m + 1 <= p) at(m + 1, m) = x[2] * at(m, m);
        for (int n = m + 2; n <= p; n++)
            at(n, m) = ((2.0 * n - 1) * x[2] * at(n - 1, m) - r2 * at(n - 2, m)) / (double)((n + m) * (n - m));
    }
    return R;
}

cd sym_get(const std::vector<cd> &A, int p, int n, int m) {
    if (n < 0 || n > p || m > n || -m > n) return cd(0, 0);
    if (m >= 0) return A[(size_t)n * (p + 1) + m];
    cd v = std::conj(A[(size_t)n * (p + 1) - m]);
    return (m & 1) ? -v : v;
}
}  // namespace

std::vector<double> build_translation_ops(int p, int dir) {
    const int P = ncoef(p);
    std::vector<double> ops((size_t)8 * P * P, 0.0);
    for (int o = 0; o < 8; o++) {
        double d[3] = {(o & 1) ? 0.5 : -0.5, (o & 2) ? 0.5 : -0.5, (o & 4) ? 0.5 : -0.5};
        std::vector<cd> R = host_regular(d, p);
        for (int col = 0; col < P; col++) {
            // complex input with the real basis vector `col`
            std::vector<cd> in((size_t)(p + 1) * (p + 1), cd(0, 0));
            int nn = 0;
            while ((nn + 1) * (nn + 1) <= col) nn++;
            int off = col - nn * nn;
            int mm = (off + 1) / 2;
            in[(size_t)nn * (p + 1) + mm] = (off == 0 || (off & 1)) ? cd(1, 0) : cd(0, 1);
            std::vector<cd> out((size_t)(p + 1) * (p + 1), cd(0, 0));
            if (dir == 0) {
                for (int n = 0; n <= p; n++)
                    for (int m = 0; m <= n; m++) {
                        cd s(0, 0);
                        for (int k = 0; k <= n; k++)
                            for (int l = -k; l <= k; l++)
                                s += sym_get(in, p, k, l) * std::conj(sym_get(R, p, n - k, m - l));
                        out[(size_t)n * (p + 1) + m] = s * std::ldexp(1.0, -n);
                    }
            } else {
                for (int k = 0; k <= p; k++)
                    for (int l = 0; l <= k; l++) {
                        cd s(0, 0);
                        for (int n = k; n <= p; n++)
                            for (int m = -n; m <= n; m++)
                                s += sym_get(in, p, n, m) * std::conj(sym_get(R, p, n - k, m - l)) *
                                     std::ldexp(1.0, -(n + 1));
                        out[(size_t)k * (p + 1) + l] = s;
                    }
            }
            double *A = ops.data() + (size_t)o * P * P;
            for (int n = 0; n <= p; n++)
                for (int m = 0; m <= n; m++) {
                    cd v = out[(size_t)n * (p + 1) + m];
                    A[(size_t)col * P + cidx_re(n, m)] = v.real();
                    if (m > 0) A[(size_t)col * P + cidx_im(n, m)] = v.imag();
                }
        }
    }
    return ops;
}

void launch_p2m(Geometry g, int32_t ncell, int p, const double *xs, const double *ys, const double *zs,
                const double *qs, double *M, hipStream_t s) {
    int64_t work = (int64_t)ncell * (p + 1);
    if (work == 0) return;
    dim3 grid(grid_for(work, 128, 1 << 30)), block(128);
#define FMM_P2M_CASE(PP)                                                                  \
    case PP:                                                                              \
        hipLaunchKernelGGL(k_p2m<PP>, grid, block, 0, s, g, ncell, xs, ys, zs, qs, M);    \
        break;
    switch (p) {
        FMM_P2M_CASE(0) FMM_P2M_CASE(1) FMM_P2M_CASE(2) FMM_P2M_CASE(3) FMM_P2M_CASE(4) FMM_P2M_CASE(5)
        FMM_P2M_CASE(6) FMM_P2M_CASE(7) FMM_P2M_CASE(8) FMM_P2M_CASE(9) FMM_P2M_CASE(10) FMM_P2M_CASE(11)
        FMM_P2M_CASE(12) FMM_P2M_CASE(13) FMM_P2M_CASE(14) FMM_P2M_CASE(15) FMM_P2M_CASE(16)
        default: throw HipError{hipErrorInvalidValue, "p2m: unsupported order"};
    }
#undef FMM_P2M_CASE
    FMM_LAUNCH_CHECK();
}

static int rows_block(int p) { return ((ncoef(p) + 63) / 64) * 64; }

// Shape of the register-tiled wide-level kernel for order p: as many
// parents per block as 256 threads allow (at most kTileMaxParents), and as
// many columns per chunk as kTileRoomKB of LDS hold (four blocks per CU).
static TileShape tile_shape(int p) {
    TileShape t;
    const int P = ncoef(p);
    t.Pp = ((P + kTR - 1) / kTR) * kTR;
    const int rg = t.Pp / kTR;
    int pg = kTileThreads / rg;
    pg = pg > kTileMaxParents / kTP ? kTileMaxParents / kTP : (pg < 1 ? 1 : pg);
    t.npb = pg * kTP;
    t.xs = t.npb + 2;   // 16-byte aligned rows that fall in different banks
    const int room = (kTileRoomKB * 1024) / (int)sizeof(double);
    int cw = room / (t.Pp + t.xs);
    t.cw = cw > P ? P : (cw < 1 ? 1 : cw);
    return t;
}

static size_t tile_lds(const TileShape &t) { return (size_t)t.cw * (t.Pp + t.xs) * sizeof(double); }

static void allow_lds(const void *fn, size_t bytes) {
    if (bytes > 64 * 1024)
        FMM_HIP_CHECK(hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes));
}

// The grids cover lp.npar_max parents; blocks beyond the level's parent
// count return at once.
void launch_m2m_level(Geometry g, int32_t lb, int32_t le, int p, LevelParents lp, const double *ops, double *M,
                      double *part, hipStream_t s) {
    if (le <= lb || lp.npar_max <= 0) return;
    if (lp.npar_max <= kSmallLevel) {
        hipLaunchKernelGGL(k_m2m_small, dim3(lp.npar_max, 8), dim3(rows_block(p)), 0, s, g, lb, le, p, lp, ops, M,
                           part);
    } else {
        const TileShape t = tile_shape(p);
        const size_t lds = tile_lds(t);
        allow_lds(reinterpret_cast<const void *>(&k_trans_tiled<false>), lds);
        dim3 grid((lp.npar_max + t.npb - 1) / t.npb, 8);
        hipLaunchKernelGGL(k_trans_tiled<false>, grid, dim3(kTileThreads), lds, s, g, lb, le, p, t, lp, ops, M,
                           part);
    }
    FMM_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_m2m_sum, dim3(grid_for((int64_t)lp.npar_max * ncoef(p), 256, 4096)), dim3(256), 0, s, lb, le,
                       p, lp, part, M);
    FMM_LAUNCH_CHECK();
}

void launch_l2l_level(Geometry g, int32_t lb, int32_t le, int p, LevelParents lp, const double *ops, double *L,
                      hipStream_t s) {
    if (le <= lb || lp.npar_max <= 0) return;
    if (lp.npar_max <= kSmallLevel) {
        hipLaunchKernelGGL(k_l2l_small, dim3(lp.npar_max, 8), dim3(rows_block(p)), 0, s, g, lb, le, p, lp, ops, L);
    } else {
        const TileShape t = tile_shape(p);
        const size_t lds = tile_lds(t);
        allow_lds(reinterpret_cast<const void *>(&k_trans_tiled<true>), lds);
        dim3 grid((lp.npar_max + t.npb - 1) / t.npb, 8);
        hipLaunchKernelGGL(k_trans_tiled<true>, grid, dim3(kTileThreads), lds, s, g, lb, le, p, t, lp, ops, L, L);
    }
    FMM_LAUNCH_CHECK();
}

void launch_l2p(Geometry g, int64_t n, int p, const int32_t *leaf_of, const double *xs, const double *ys,
                const double *zs, const double *L, double *phi, double *fld, hipStream_t s, const FinalOut &out) {
    if (n == 0) return;
    dim3 grid(grid_for(n, 128, 1 << 20)), block(128);
#define FMM_L2P_CASE(PP)                                                                             \
    case PP:                                                                                         \
        hipLaunchKernelGGL(k_l2p<PP>, grid, block, 0, s, g, n, leaf_of, xs, ys, zs, L, phi, fld, out); \
        break;
    switch (p) {
        FMM_L2P_CASE(0) FMM_L2P_CASE(1) FMM_L2P_CASE(2) FMM_L2P_CASE(3) FMM_L2P_CASE(4) FMM_L2P_CASE(5)
        FMM_L2P_CASE(6) FMM_L2P_CASE(7) FMM_L2P_CASE(8) FMM_L2P_CASE(9) FMM_L2P_CASE(10) FMM_L2P_CASE(11)
        FMM_L2P_CASE(12) FMM_L2P_CASE(13) FMM_L2P_CASE(14) FMM_L2P_CASE(15) FMM_L2P_CASE(16)
        default: throw HipError{hipErrorInvalidValue, "l2p: unsupported order"};
    }
#undef FMM_L2P_CASE
    FMM_LAUNCH_CHECK();
}

void launch_finalize(int64_t n, const uint32_t *perm, const double *qs, const double *phi_near,
                     const double *fld_near, const double *phi_far, const double *fld_far, double *phi, double *field,
                     double *force, hipStream_t s) {
    if (n == 0 || (!phi && !field && !force)) return;
    hipLaunchKernelGGL(k_finalize, dim3(grid_for(n, 256, 16384)), dim3(256), 0, s, n, perm, qs, phi_near, fld_near,
                       phi_far, fld_far, phi, field, force);
    FMM_LAUNCH_CHECK();
}

void launch_dual_scale(Geometry g, int32_t ncell, int p, double *X, int dir, hipStream_t s) {
    const int64_t total = (int64_t)ncell * ncoef(p);
    if (total == 0) return;
    hipLaunchKernelGGL(k_dual_scale, dim3(grid_for(total, 256, 16384)), dim3(256), 0, s, g, ncell, p, X, dir);
    FMM_LAUNCH_CHECK();
}

void launch_adjoint_weights(Geometry g, int64_t n, const int32_t *leaf_of, const double *gE, const double *qs,
                            double *w, hipStream_t s) {
    if (n == 0) return;
    hipLaunchKernelGGL(k_adjoint_weights, dim3(grid_for(n, 256, 16384)), dim3(256), 0, s, n, leaf_of, g.c.inst, gE, qs,
                       w);
    FMM_LAUNCH_CHECK();
}

void launch_adjoint_finalize(Geometry g, int64_t n, const uint32_t *perm, const int32_t *leaf_of, const double *gE,
                             const double *qs, const double *phi_near, const double *fld_near, const double *phi_far,
                             const double *fld_far, const double *psi_near, const double *epsi_near,
                             const double *psi_far, const double *epsi_far, double *grad_pos, double *grad_q,
                             hipStream_t s) {
    if (n == 0) return;
    hipLaunchKernelGGL(k_adjoint_finalize, dim3(grid_for(n, 256, 16384)), dim3(256), 0, s, n, perm, leaf_of, g.c.inst,
                       gE, qs, phi_near, fld_near, phi_far, fld_far, psi_near, epsi_near, psi_far, epsi_far, grad_pos,
                       grad_q);
    FMM_LAUNCH_CHECK();
}

std::vector<double> transpose_ops(const std::vector<double> &ops, int p) {
    const int P = ncoef(p);
    std::vector<double> t(ops.size());
    for (int o = 0; o < 8; o++)
        for (int r = 0; r < P; r++)
            for (int c = 0; c < P; c++) t[(size_t)o * P * P + (size_t)c * P + r] = ops[(size_t)o * P * P + (size_t)r * P + c];
    return t;
}

std::vector<int32_t> energy_chunks(const std::vector<int64_t> &offsets) {
    std::vector<int32_t> co(offsets.size(), 0);
    for (size_t k = 0; k + 1 < offsets.size(); k++)
        co[k + 1] = co[k] + (int32_t)((offsets[k + 1] - offsets[k] + kEnergyChunk - 1) / kEnergyChunk);
    return co;
}

void launch_energy(const int64_t *d_offsets, int n_inst, const int32_t *d_chunk_off, int32_t nchunk, const double *qs,
                   const double *phi_near, const double *phi_far, double *part, double *energy, hipStream_t s,
                   const FinalOut &out, const double *fld_far) {
    if (nchunk > 0) {
        hipLaunchKernelGGL(k_energy_part, dim3(nchunk), dim3(256), 0, s, d_offsets, n_inst, d_chunk_off, qs, phi_near,
                           phi_far, part, out, fld_far);
        FMM_LAUNCH_CHECK();
    }
    hipLaunchKernelGGL(k_energy_sum, dim3(n_inst), dim3(64), 0, s, n_inst, d_chunk_off, part, energy);
    FMM_LAUNCH_CHECK();
}

}  // namespace fmm
