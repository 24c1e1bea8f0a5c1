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

// P2M: one thread per (leaf, order m); accumulates degrees n = m..p.
__global__ void k_p2m(Geometry g, int32_t ncell, int p, const double *__restrict__ xs, const double *__restrict__ ys,
                      const double *__restrict__ zs, const double *__restrict__ qs, double *__restrict__ M) {
    int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    int32_t cell = (int32_t)(t / (p + 1));
    int m = (int)(t % (p + 1));
    if (cell >= ncell || g.c.child[cell] >= 0) return;
    const int P = ncoef(p);
    double c[3], side;
    int l;
    cell_frame(g, cell, c, &side, &l);
    Cplx acc[kMaxP + 1];
    for (int n = 0; n <= p; n++) acc[n] = {0.0, 0.0};
    int32_t f = g.c.first[cell], e = f + g.c.count[cell];
    for (int32_t r = f; r < e; r++) {
        double ux = ldexp((xs[r] - c[0]) / side, l);
        double uy = ldexp((ys[r] - c[1]) / side, l);
        double uz = ldexp((zs[r] - c[2]) / side, l);
        double r2 = ux * ux + uy * uy + uz * uz;
        Cplx zeta = {ux, uy};
        Cplx rmm = {1.0, 0.0};
        for (int j = 1; j <= m; j++) {
            rmm = cmul(rmm, zeta);
            rmm.re /= 2 * j;
            rmm.im /= 2 * j;
        }
        double q = qs[r];
        Cplx r2m = {0.0, 0.0}, r1m = rmm;  // R_(n-2)^m, R_(n-1)^m
        acc[m].re += q * rmm.re;
        acc[m].im -= q * rmm.im;
        for (int n = m + 1; n <= p; n++) {
            Cplx rn;
            if (n == m + 1) {
                rn = {uz * r1m.re, uz * r1m.im};
            } else {
                double a = (2 * n - 1) * uz, den = (double)((n + m) * (n - m));
                rn = {(a * r1m.re - r2 * r2m.re) / den, (a * r1m.im - r2 * r2m.im) / den};
            }
            acc[n].re += q * rn.re;
            acc[n].im -= q * rn.im;
            r2m = r1m;
            r1m = rn;
        }
    }
    double *out = M + (int64_t)cell * P;
    for (int n = m; n <= p; n++) {
        out[cidx_re(n, m)] = acc[n].re;
        if (m > 0) out[cidx_im(n, m)] = acc[n].im;
    }
}

__device__ inline int octant_of(const CellArrays &c, int32_t cell) {
    return (c.ix[cell] & 1) | ((c.iy[cell] & 1) << 1) | ((c.iz[cell] & 1) << 2);
}

// M2M for the non-leaf cells of one level: thread per (cell, output row).
__global__ void k_m2m(Geometry g, int32_t lb, int32_t le, int p, const double *__restrict__ ops, double *__restrict__ M) {
    const int P = ncoef(p);
    int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    int32_t cell = lb + (int32_t)(t / P);
    int row = (int)(t % P);
    if (cell >= le) return;
    int32_t ch = g.c.child[cell];
    if (ch < 0) return;
    int nch = g.c.nchild[cell];
    double s = 0.0;
    for (int k = 0; k < nch; k++) {
        int32_t cc = ch + k;
        const double *A = ops + (int64_t)octant_of(g.c, cc) * P * P + (int64_t)row * P;
        const double *x = M + (int64_t)cc * P;
        for (int i = 0; i < P; i++) s += A[i] * x[i];
    }
    M[(int64_t)cell * P + row] = s;
}

// L2L for the cells of one level (all have parents): L_child += B L_parent.
__global__ void k_l2l(Geometry g, int32_t lb, int32_t le, int p, const double *__restrict__ ops, double *__restrict__ L) {
    const int P = ncoef(p);
    int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    int32_t cell = lb + (int32_t)(t / P);
    int row = (int)(t % P);
    if (cell >= le) return;
    int32_t par = g.c.parent[cell];
    if (par < 0) return;
    const double *B = ops + (int64_t)octant_of(g.c, cell) * P * P + (int64_t)row * P;
    const double *x = L + (int64_t)par * P;
    double s = 0.0;
    for (int i = 0; i < P; i++) s += B[i] * x[i];
    L[(int64_t)cell * P + row] += s;
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
__global__ void k_l2p(Geometry g, int64_t n, int p, const int32_t *__restrict__ leaf_of, const double *__restrict__ xs,
                      const double *__restrict__ ys, const double *__restrict__ zs, const double *__restrict__ L,
                      double *__restrict__ phi, double *__restrict__ fld) {
    const int P = ncoef(p);
    for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < n; r += (int64_t)gridDim.x * blockDim.x) {
        int32_t cell = leaf_of[r];
        double c[3], side;
        int l;
        cell_frame(g, cell, c, &side, &l);
        double ux = ldexp((xs[r] - c[0]) / side, l);
        double uy = ldexp((ys[r] - c[1]) / side, l);
        double uz = ldexp((zs[r] - c[2]) / side, l);
        double r2 = ux * ux + uy * uy + uz * uz;
        const double *Lc = L + (int64_t)cell * P;
        Cplx zeta = {ux, uy};
        Cplx rmm = {1.0, 0.0};
        Cplx a0 = {0, 0}, gz = {0, 0}, gxy = {0, 0};
        for (int m = 0; m <= p; m++) {
            if (m > 0) {
                rmm = cmul(rmm, zeta);
                rmm.re /= 2 * m;
                rmm.im /= 2 * m;
            }
            Cplx r2m = {0.0, 0.0}, r1m = {0.0, 0.0};
            for (int nn = m; nn <= p; nn++) {
                Cplx rn;
                if (nn == m) {
                    rn = rmm;
                } else if (nn == m + 1) {
                    rn = {uz * r1m.re, uz * r1m.im};
                } else {
                    double a = (2 * nn - 1) * uz, den = (double)((nn + m) * (nn - m));
                    rn = {(a * r1m.re - r2 * r2m.re) / den, (a * r1m.im - r2 * r2m.im) / den};
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
        phi[r] = a0.re * invS;
        double e2 = invS * invS;
        fld[3 * r] = -gxy.re * e2;
        fld[3 * r + 1] = -gxy.im * e2;
        fld[3 * r + 2] = -gz.re * e2;
    }
}

__global__ void k_finalize(int64_t n, const uint32_t *__restrict__ perm, const double *__restrict__ qs,
                           const double *__restrict__ pn, const double *__restrict__ fn, const double *__restrict__ pf,
                           const double *__restrict__ ff, double *__restrict__ phi, double *__restrict__ field,
                           double *__restrict__ force) {
    for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < n; r += (int64_t)gridDim.x * blockDim.x) {
        int64_t i = perm[r];
        double ph = pn[r] + pf[r];
        double ex = fn[3 * r] + ff[3 * r], ey = fn[3 * r + 1] + ff[3 * r + 1], ez = fn[3 * r + 2] + ff[3 * r + 2];
        if (phi) phi[i] = ph;
        if (field) {
            field[3 * i] = ex;
            field[3 * i + 1] = ey;
            field[3 * i + 2] = ez;
        }
        if (force) {
            double q = qs[r];
            force[3 * i] = q * ex;
            force[3 * i + 1] = q * ey;
            force[3 * i + 2] = q * ez;
        }
    }
}

// E_k = 1/2 sum_(i in k) q_i phi_i, one block per instance, fixed order.
__global__ void k_energy(const int64_t *__restrict__ offsets, const double *__restrict__ qs,
                         const double *__restrict__ pn, const double *__restrict__ pf, double *__restrict__ energy) {
    __shared__ double red[256];
    int k = blockIdx.x;
    double s = 0.0;
    for (int64_t r = offsets[k] + threadIdx.x; r < offsets[k + 1]; r += 256) s += qs[r] * (pn[r] + pf[r]);
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) energy[k] = 0.5 * red[0];
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
                    A[(size_t)cidx_re(n, m) * P + col] = v.real();
                    if (m > 0) A[(size_t)cidx_im(n, m) * P + col] = v.imag();
                }
        }
    }
    return ops;
}

void launch_p2m(Geometry g, int32_t ncell, int p, const double *xs, const double *ys, const double *zs,
                const double *qs, double *M, hipStream_t s) {
    int64_t work = (int64_t)ncell * (p + 1);
    if (work == 0) return;
    hipLaunchKernelGGL(k_p2m, dim3(grid_for(work, 128, 1 << 30)), dim3(128), 0, s, g, ncell, p, xs, ys, zs, qs, M);
    FMM_LAUNCH_CHECK();
}

void launch_m2m_level(Geometry g, int32_t lb, int32_t le, int p, const double *ops, double *M, hipStream_t s) {
    int64_t work = (int64_t)(le - lb) * ncoef(p);
    if (work <= 0) return;
    hipLaunchKernelGGL(k_m2m, dim3(grid_for(work, 128, 1 << 30)), dim3(128), 0, s, g, lb, le, p, ops, M);
    FMM_LAUNCH_CHECK();
}

void launch_l2l_level(Geometry g, int32_t lb, int32_t le, int p, const double *ops, double *L, hipStream_t s) {
    int64_t work = (int64_t)(le - lb) * ncoef(p);
    if (work <= 0) return;
    hipLaunchKernelGGL(k_l2l, dim3(grid_for(work, 128, 1 << 30)), dim3(128), 0, s, g, lb, le, p, ops, L);
    FMM_LAUNCH_CHECK();
}

void launch_l2p(Geometry g, int64_t n, int p, const int32_t *leaf_of, const double *xs, const double *ys,
                const double *zs, const double *L, double *phi, double *fld, hipStream_t s) {
    if (n == 0) return;
    hipLaunchKernelGGL(k_l2p, dim3(grid_for(n, 128, 1 << 20)), dim3(128), 0, s, g, n, p, leaf_of, xs, ys, zs, L, phi,
                       fld);
    FMM_LAUNCH_CHECK();
}

void launch_finalize(int64_t n, const uint32_t *perm, const double *qs, const double *phi_near,
                     const double *fld_near, const double *phi_far, const double *fld_far, double *phi, double *field,
                     double *force, hipStream_t s) {
    if (n == 0) return;
    hipLaunchKernelGGL(k_finalize, dim3(grid_for(n, 256, 16384)), dim3(256), 0, s, n, perm, qs, phi_near, fld_near,
                       phi_far, fld_far, phi, field, force);
    FMM_LAUNCH_CHECK();
}

void launch_energy(const int64_t *d_offsets, int n_inst, const double *qs, const double *phi_near,
                   const double *phi_far, double *energy, hipStream_t s) {
    hipLaunchKernelGGL(k_energy, dim3(n_inst), dim3(256), 0, s, d_offsets, qs, phi_near, phi_far, energy);
    FMM_LAUNCH_CHECK();
}

}  // namespace fmm
