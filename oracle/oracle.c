/*
 * oracle.c -- plain, slow, FP64 CPU reference for the 3-D Laplace fast
 * multipole method of Ltaief & Yokota, "Data-Driven Execution of Fast
 * Multipole Methods" (arXiv:1203.0889).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the tests, the smoke check and the CPU-baseline leg
 * of the benchmark do.  It shares no code, header, table or constant with the
 * GPU path.
 *
 * What it computes (paper section in brackets):
 *   - direct sum: phi_i = sum_{j, r_ij > 0} q_j / r_ij,
 *                 E_i   = sum_{j, r_ij > 0} q_j (x_i - x_j) / r_ij^3
 *     [the N-body problem of the introduction and Sec. 2.1; unit Coulomb
 *      constant; pairs at zero distance contribute nothing]
 *   - Morton keys of the cubic octree [Sec. 2.2]
 *   - adaptive octree, leaves hold at most ncrit particles [Sec. 2.1]
 *   - dual tree traversal producing M2L and P2P pair lists, non-mutual
 *     (target-owned) form, well-separatedness by the ratio of cell size to
 *     distance [Sec. 2.1, Sec. 4]
 *   - the six FMM stages P2M, M2M, M2L, P2P, L2L, L2P [Sec. 2.1, Fig. 1], in
 *     Cartesian Taylor form.  The paper defers the operator formulas to its
 *     references; here they are the Taylor expansion of G(r) = 1/|r| written
 *     out with multi-indices (readings listed in the design notes).
 *
 * Readings of points the paper leaves open (all stated once here):
 *   R1  "order p" = every degree 0..p is kept (multi-indices |alpha| <= p).
 *   R2  Bounding cube: per-axis min/max; side = largest extent (1 if zero);
 *       scale = 2^21 / side; ix = min(floor((x - min) * scale), 2^21 - 1).
 *   R3  Key bit 3b+0 = x bit b, 3b+1 = y bit b, 3b+2 = z bit b (63 bits).
 *   R4  Stable sort by (key, original index).
 *   R5  A cell is split iff count > ncrit and level < max_level; only
 *       non-empty octants become children; cells numbered level-major, then
 *       by Morton prefix.
 *   R6  Integer geometry: side S_l = 2^(21-l) grid units, centre in half
 *       units C = (2i+1) S_l, radius = half diagonal.  MAC (theta = a/b):
 *       3 b^2 (S_A + S_B)^2 < a^2 |C_A - C_B|^2, strict, exact integers.
 *   R7  Per-pair decision: A != B and MAC -> M2L(A<-B); else both leaves ->
 *       P2P(A<-B); else split B if B is not a leaf and (A is a leaf or
 *       S_A < S_B), otherwise split A (ties split the target).
 *   R8  Expansion centre = geometric cell centre,
 *       min + (2i+1) * side / 2^(l+1) per axis.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_LEVELS 21

/* ------------------------------------------------------------------------ */
/* Direct sum (the exact result the FMM approximates).                      */
/* ------------------------------------------------------------------------ */

/* For each target t (all N if tidx == NULL, else the nt listed indices):
 * phi[t] and field[3t..3t+2] over every source j with r_tj > 0. */
void orc_direct(int64_t n, const double *pos, const double *q, int64_t nt,
                const int64_t *tidx, double *phi, double *field)
{
    int64_t count = tidx ? nt : n;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t t = 0; t < count; t++) {
        int64_t i = tidx ? tidx[t] : t;
        double xi = pos[3 * i], yi = pos[3 * i + 1], zi = pos[3 * i + 2];
        double p = 0, ex = 0, ey = 0, ez = 0;
        for (int64_t j = 0; j < n; j++) {
            double dx = xi - pos[3 * j], dy = yi - pos[3 * j + 1], dz = zi - pos[3 * j + 2];
            double r2 = dx * dx + dy * dy + dz * dz;
            if (r2 == 0.0) continue;
            double r = sqrt(r2);
            double inv = 1.0 / r;
            p += q[j] * inv;
            double inv3 = inv / r2;
            ex += q[j] * dx * inv3;
            ey += q[j] * dy * inv3;
            ez += q[j] * dz * inv3;
        }
        phi[t] = p;
        field[3 * t] = ex;
        field[3 * t + 1] = ey;
        field[3 * t + 2] = ez;
    }
}

/* ------------------------------------------------------------------------ */
/* Keys, sort, tree (Sec. 2.1 and 2.2).                                      */
/* ------------------------------------------------------------------------ */

/* R2: cube enclosing all points.  box[0..2] = min corner, box[3] = side. */
void orc_bounding_cube(int64_t n, const double *pos, double *box)
{
    double lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
    for (int d = 0; d < 3; d++) {
        lo[d] = n > 0 ? pos[d] : 0.0;
        hi[d] = lo[d];
    }
    for (int64_t i = 0; i < n; i++)
        for (int d = 0; d < 3; d++) {
            double v = pos[3 * i + d];
            if (v < lo[d]) lo[d] = v;
            if (v > hi[d]) hi[d] = v;
        }
    double side = 0;
    for (int d = 0; d < 3; d++) {
        double e = hi[d] - lo[d];
        if (e > side) side = e;
    }
    if (!(side > 0)) side = 1.0;
    box[0] = lo[0];
    box[1] = lo[1];
    box[2] = lo[2];
    box[3] = side;
}

/* R2 + R3: one key per particle.  scale is given by the caller
 * (2^21 / side computed once). */
void orc_morton_keys(int64_t n, const double *pos, const double *box, double scale,
                     uint64_t *keys)
{
    const int64_t top = (1 << ORC_LEVELS) - 1;
    for (int64_t i = 0; i < n; i++) {
        int64_t c[3];
        for (int d = 0; d < 3; d++) {
            volatile double off = pos[3 * i + d] - box[d];
            volatile double s = off * scale;
            double f = floor(s);
            int64_t v = f < 0 ? 0 : (int64_t)f;
            if (v > top) v = top;
            c[d] = v;
        }
        uint64_t k = 0;
        for (int b = 0; b < ORC_LEVELS; b++)
            for (int d = 0; d < 3; d++)
                k |= (uint64_t)((c[d] >> b) & 1) << (3 * b + d);
        keys[i] = k;
    }
}

/* Inverse of the interleave: key prefix at `level` -> integer cell coords. */
static void orc_prefix_coords(uint64_t prefix, int level, int32_t *ix, int32_t *iy, int32_t *iz)
{
    int32_t c[3] = {0, 0, 0};
    for (int b = 0; b < level; b++)
        for (int d = 0; d < 3; d++)
            c[d] |= (int32_t)((prefix >> (3 * b + d)) & 1) << b;
    *ix = c[0];
    *iy = c[1];
    *iz = c[2];
}

static const uint64_t *orc_sort_keys_ref;
static int orc_cmp_idx(const void *a, const void *b)
{
    int64_t i = *(const int64_t *)a, j = *(const int64_t *)b;
    uint64_t ki = orc_sort_keys_ref[i], kj = orc_sort_keys_ref[j];
    if (ki < kj) return -1;
    if (ki > kj) return 1;
    return (i > j) - (i < j);
}

/* R4: perm[r] = original index of the r-th particle in (key, index) order. */
void orc_sort_keys(int64_t n, const uint64_t *keys, int64_t *perm)
{
    for (int64_t i = 0; i < n; i++) perm[i] = i;
    orc_sort_keys_ref = keys;
    qsort(perm, (size_t)n, sizeof(int64_t), orc_cmp_idx);
    orc_sort_keys_ref = NULL;
}

typedef struct {
    int32_t level;
    int32_t ix, iy, iz;       /* integer cell coordinates at `level` */
    int64_t first, count;     /* particle range in sorted order */
    int32_t child_first;      /* index of first child cell, -1 if leaf */
    int32_t nchild;
    int32_t parent;           /* -1 for the root */
} orc_cell;

/* R5: level-major build from sorted keys.  Returns the number of cells, or
 * -1 if `cap` is too small. */
int64_t orc_build_tree(int64_t n, const uint64_t *skeys, int ncrit, int max_level,
                       orc_cell *cells, int64_t cap)
{
    if (cap < 1) return -1;
    int64_t nc = 1;
    cells[0].level = 0;
    cells[0].ix = cells[0].iy = cells[0].iz = 0;
    cells[0].first = 0;
    cells[0].count = n;
    cells[0].child_first = -1;
    cells[0].nchild = 0;
    cells[0].parent = -1;
    int64_t lvl_begin = 0, lvl_end = 1;
    for (int level = 0; level < max_level; level++) {
        for (int64_t c = lvl_begin; c < lvl_end; c++) {
            if (cells[c].count <= ncrit) continue;
            int shift = 3 * (ORC_LEVELS - (level + 1));
            int64_t i = cells[c].first, end = cells[c].first + cells[c].count;
            cells[c].child_first = (int32_t)nc;
            while (i < end) {
                uint64_t pre = skeys[i] >> shift;
                int64_t j = i;
                while (j < end && (skeys[j] >> shift) == pre) j++;
                if (nc >= cap) return -1;
                orc_cell *ch = &cells[nc];
                ch->level = level + 1;
                orc_prefix_coords(pre, level + 1, &ch->ix, &ch->iy, &ch->iz);
                ch->first = i;
                ch->count = j - i;
                ch->child_first = -1;
                ch->nchild = 0;
                ch->parent = (int32_t)c;
                cells[c].nchild++;
                nc++;
                i = j;
            }
        }
        lvl_begin = lvl_end;
        lvl_end = nc;
        if (lvl_begin == lvl_end) break;
    }
    return nc;
}

/* ------------------------------------------------------------------------ */
/* Dual tree traversal (Sec. 4), pure per-pair decision (R6, R7).           */
/* ------------------------------------------------------------------------ */

static int orc_mac(const orc_cell *A, const orc_cell *B, int64_t a, int64_t b)
{
    int64_t SA = (int64_t)1 << (ORC_LEVELS - A->level);
    int64_t SB = (int64_t)1 << (ORC_LEVELS - B->level);
    __int128 d2 = 0;
    int32_t ca[3] = {A->ix, A->iy, A->iz}, cb[3] = {B->ix, B->iy, B->iz};
    for (int d = 0; d < 3; d++) {
        __int128 diff = (__int128)(2 * (int64_t)ca[d] + 1) * SA - (__int128)(2 * (int64_t)cb[d] + 1) * SB;
        d2 += diff * diff;
    }
    __int128 lhs = (__int128)3 * b * b * (__int128)(SA + SB) * (SA + SB);
    __int128 rhs = (__int128)a * a * d2;
    return lhs < rhs;
}

typedef struct {
    int32_t *t, *s;
    int64_t n, cap;
} orc_pairs;

static void orc_push(orc_pairs *p, int32_t t, int32_t s)
{
    if (p->n == p->cap) {
        p->cap = p->cap ? 2 * p->cap : 1024;
        p->t = (int32_t *)realloc(p->t, (size_t)p->cap * sizeof(int32_t));
        p->s = (int32_t *)realloc(p->s, (size_t)p->cap * sizeof(int32_t));
    }
    p->t[p->n] = t;
    p->s[p->n] = s;
    p->n++;
}

static void orc_traverse(const orc_cell *cells, int32_t A, int32_t B, int64_t a, int64_t b,
                         orc_pairs *m2l, orc_pairs *p2p)
{
    const orc_cell *ca = &cells[A], *cb = &cells[B];
    int leafA = ca->child_first < 0, leafB = cb->child_first < 0;
    if (A != B && orc_mac(ca, cb, a, b)) {
        orc_push(m2l, A, B);
    } else if (leafA && leafB) {
        orc_push(p2p, A, B);
    } else if (!leafB && (leafA || ca->level > cb->level)) {
        for (int k = 0; k < cb->nchild; k++)
            orc_traverse(cells, A, cb->child_first + k, a, b, m2l, p2p);
    } else {
        for (int k = 0; k < ca->nchild; k++)
            orc_traverse(cells, ca->child_first + k, B, a, b, m2l, p2p);
    }
}

static const int32_t *orc_pair_t, *orc_pair_s;
static int orc_cmp_pair(const void *x, const void *y)
{
    int64_t i = *(const int64_t *)x, j = *(const int64_t *)y;
    if (orc_pair_t[i] != orc_pair_t[j]) return orc_pair_t[i] < orc_pair_t[j] ? -1 : 1;
    if (orc_pair_s[i] != orc_pair_s[j]) return orc_pair_s[i] < orc_pair_s[j] ? -1 : 1;
    return 0;
}

/* Sort a pair list by (target, source) in place. */
static void orc_sort_pairs(orc_pairs *p)
{
    int64_t *idx = (int64_t *)malloc((size_t)(p->n ? p->n : 1) * sizeof(int64_t));
    for (int64_t i = 0; i < p->n; i++) idx[i] = i;
    orc_pair_t = p->t;
    orc_pair_s = p->s;
    qsort(idx, (size_t)p->n, sizeof(int64_t), orc_cmp_pair);
    int32_t *nt = (int32_t *)malloc((size_t)(p->n ? p->n : 1) * sizeof(int32_t));
    int32_t *ns = (int32_t *)malloc((size_t)(p->n ? p->n : 1) * sizeof(int32_t));
    for (int64_t i = 0; i < p->n; i++) {
        nt[i] = p->t[idx[i]];
        ns[i] = p->s[idx[i]];
    }
    free(p->t);
    free(p->s);
    free(idx);
    p->t = nt;
    p->s = ns;
    p->cap = p->n ? p->n : 1;
}

/* ------------------------------------------------------------------------ */
/* Cartesian Taylor operators (Sec. 2.1 stages).                             */
/* Multi-index alpha = (a0,a1,a2); |alpha| = a0+a1+a2; alpha! = a0!a1!a2!;  */
/* y^alpha = y0^a0 y1^a1 y2^a2.                                              */
/*   P2M: M_alpha(c)  = sum_j q_j (y_j - c)^alpha / alpha!                   */
/*   M2M: M_alpha(c') = sum_{beta<=alpha} M_beta(c) (c-c')^(alpha-beta)/(alpha-beta)! */
/*   M2L: b_gamma(r)  = d^gamma (1/|r|) / gamma!  at r = c_A - c_B,          */
/*        L_beta(c_A) += sum_alpha (-1)^|alpha| (alpha+beta)!/beta!          */
/*                        M_alpha(c_B) b_(alpha+beta)(r)                     */
/*   L2L: L_beta(c')  = sum_{gamma>=beta} L_gamma(c) gamma!/(beta!(gamma-beta)!) */
/*                        (c'-c)^(gamma-beta)                                */
/*   L2P: phi(x) = sum_beta L_beta (x-c)^beta,  E = -grad phi                */
/* The Taylor coefficients b_gamma of 1/|r| obey, for n = |gamma| >= 1,      */
/*   n |r|^2 b_gamma = -(2n-1) sum_k r_k b_(gamma-e_k) - (n-1) sum_k b_(gamma-2e_k) */
/* ------------------------------------------------------------------------ */

typedef struct {
    int p;              /* kept degree */
    int D;              /* 2p + 1: side of the index cube */
    int nk;             /* |K_p| */
    int nk2;            /* |K_2p| */
    int *mi;            /* mi[3*i..3*i+2] = multi-index i of K_2p, ordered by degree */
    int *deg;           /* deg[i] = |mi_i| */
    int *lookup;        /* lookup[(a0*D + a1)*D + a2] = index, or -1 */
    double *ifact;      /* ifact[i] = 1 / alpha_i! */
    double *fact;       /* fact[i] = alpha_i! */
    /* M2L tables over K_p x K_p */
    int *m2l_idx;       /* [beta*nk + alpha] = index of alpha+beta in K_2p */
    double *m2l_coef;   /* (-1)^|alpha| (alpha+beta)! / beta! */
} orc_mi;

static double orc_factorial(int n)
{
    double f = 1;
    for (int i = 2; i <= n; i++) f *= i;
    return f;
}

static int orc_mi_find(const orc_mi *t, int a0, int a1, int a2)
{
    if (a0 < 0 || a1 < 0 || a2 < 0 || a0 >= t->D || a1 >= t->D || a2 >= t->D) return -1;
    return t->lookup[(a0 * t->D + a1) * t->D + a2];
}

static void orc_mi_init(orc_mi *t, int p)
{
    t->p = p;
    t->D = 2 * p + 1;
    int D = t->D;
    t->lookup = (int *)malloc((size_t)D * D * D * sizeof(int));
    for (int i = 0; i < D * D * D; i++) t->lookup[i] = -1;
    int cnt = 0;
    for (int n = 0; n <= 2 * p; n++) cnt += (n + 1) * (n + 2) / 2;
    t->nk2 = cnt;
    t->mi = (int *)malloc((size_t)3 * cnt * sizeof(int));
    t->deg = (int *)malloc((size_t)cnt * sizeof(int));
    t->ifact = (double *)malloc((size_t)cnt * sizeof(double));
    t->fact = (double *)malloc((size_t)cnt * sizeof(double));
    int k = 0;
    for (int n = 0; n <= 2 * p; n++) {
        if (n == p + 1) t->nk = k;
        for (int a0 = n; a0 >= 0; a0--)
            for (int a1 = n - a0; a1 >= 0; a1--) {
                int a2 = n - a0 - a1;
                t->mi[3 * k] = a0;
                t->mi[3 * k + 1] = a1;
                t->mi[3 * k + 2] = a2;
                t->deg[k] = n;
                t->fact[k] = orc_factorial(a0) * orc_factorial(a1) * orc_factorial(a2);
                t->ifact[k] = 1.0 / t->fact[k];
                t->lookup[(a0 * D + a1) * D + a2] = k;
                k++;
            }
    }
    if (p == 0) t->nk = 1;
    int nk = t->nk;
    t->m2l_idx = (int *)malloc((size_t)nk * nk * sizeof(int));
    t->m2l_coef = (double *)malloc((size_t)nk * nk * sizeof(double));
    for (int be = 0; be < nk; be++)
        for (int al = 0; al < nk; al++) {
            const int *A = &t->mi[3 * al], *B = &t->mi[3 * be];
            int g = orc_mi_find(t, A[0] + B[0], A[1] + B[1], A[2] + B[2]);
            t->m2l_idx[be * nk + al] = g;
            double sign = (t->deg[al] & 1) ? -1.0 : 1.0;
            t->m2l_coef[be * nk + al] = sign * t->fact[g] / t->fact[be];
        }
}

static void orc_mi_free(orc_mi *t)
{
    free(t->mi);
    free(t->deg);
    free(t->lookup);
    free(t->ifact);
    free(t->fact);
    free(t->m2l_idx);
    free(t->m2l_coef);
}

/* y^alpha / alpha! for every alpha in K_p (first nk entries). */
static void orc_monomials(const orc_mi *t, const double *y, double *out)
{
    out[0] = 1.0;
    for (int k = 1; k < t->nk; k++) {
        const int *a = &t->mi[3 * k];
        int d = a[0] > 0 ? 0 : (a[1] > 0 ? 1 : 2);
        int prev = orc_mi_find(t, a[0] - (d == 0), a[1] - (d == 1), a[2] - (d == 2));
        out[k] = out[prev] * y[d] / a[d];
    }
}

/* Taylor coefficients b_gamma(r) for gamma in K_2p. */
static void orc_taylor_coeffs(const orc_mi *t, const double *r, double *b)
{
    double r2 = r[0] * r[0] + r[1] * r[1] + r[2] * r[2];
    b[0] = 1.0 / sqrt(r2);
    for (int k = 1; k < t->nk2; k++) {
        const int *g = &t->mi[3 * k];
        int n = t->deg[k];
        double s1 = 0, s2 = 0;
        for (int d = 0; d < 3; d++) {
            int e1 = orc_mi_find(t, g[0] - (d == 0), g[1] - (d == 1), g[2] - (d == 2));
            if (e1 >= 0) s1 += r[d] * b[e1];
            int e2 = orc_mi_find(t, g[0] - 2 * (d == 0), g[1] - 2 * (d == 1), g[2] - 2 * (d == 2));
            if (e2 >= 0) s2 += b[e2];
        }
        b[k] = (-(2.0 * n - 1.0) * s1 - (n - 1.0) * s2) / (n * r2);
    }
}

/* ------------------------------------------------------------------------ */
/* The oracle state: tree, lists and FMM results.                           */
/* ------------------------------------------------------------------------ */

typedef struct {
    int64_t n;
    double box[4];
    double scale;
    uint64_t *keys;      /* input order */
    int64_t *perm;       /* sorted rank -> input index */
    uint64_t *skeys;     /* sorted keys */
    orc_cell *cells;
    int64_t ncell;
    int ncrit, max_level;
    orc_pairs m2l, p2p;
    int have_lists;
} orc_tree;

/* Build keys, sort and tree.  box4 (min xyz, side) may be NULL for R2. */
orc_tree *orc_tree_build(int64_t n, const double *pos, const double *box4, int ncrit,
                         int max_level)
{
    orc_tree *T = (orc_tree *)calloc(1, sizeof(orc_tree));
    T->n = n;
    T->ncrit = ncrit;
    T->max_level = max_level;
    if (box4)
        memcpy(T->box, box4, 4 * sizeof(double));
    else
        orc_bounding_cube(n, pos, T->box);
    T->scale = (double)(1 << ORC_LEVELS) / T->box[3];
    size_t nn = (size_t)(n ? n : 1);
    T->keys = (uint64_t *)malloc(nn * sizeof(uint64_t));
    T->perm = (int64_t *)malloc(nn * sizeof(int64_t));
    T->skeys = (uint64_t *)malloc(nn * sizeof(uint64_t));
    orc_morton_keys(n, pos, T->box, T->scale, T->keys);
    orc_sort_keys(n, T->keys, T->perm);
    for (int64_t i = 0; i < n; i++) T->skeys[i] = T->keys[T->perm[i]];
    int64_t cap = 2 * n + 64;
    for (;;) {
        T->cells = (orc_cell *)malloc((size_t)cap * sizeof(orc_cell));
        T->ncell = orc_build_tree(n, T->skeys, ncrit, max_level, T->cells, cap);
        if (T->ncell >= 0) break;
        free(T->cells);
        cap *= 2;
    }
    return T;
}

void orc_tree_free(orc_tree *T)
{
    if (!T) return;
    free(T->keys);
    free(T->perm);
    free(T->skeys);
    free(T->cells);
    free(T->m2l.t);
    free(T->m2l.s);
    free(T->p2p.t);
    free(T->p2p.s);
    free(T);
}

int64_t orc_tree_ncell(const orc_tree *T) { return T->ncell; }
void orc_tree_box(const orc_tree *T, double *box4, double *scale)
{
    memcpy(box4, T->box, 4 * sizeof(double));
    *scale = T->scale;
}

/* Copy keys (input order), permutation and cells as a flat int64 table:
 * per cell [level, ix, iy, iz, first, count, child_first, nchild, parent]. */
void orc_tree_copy(const orc_tree *T, uint64_t *keys, int64_t *perm, int64_t *cells9)
{
    if (keys) memcpy(keys, T->keys, (size_t)T->n * sizeof(uint64_t));
    if (perm) memcpy(perm, T->perm, (size_t)T->n * sizeof(int64_t));
    if (cells9)
        for (int64_t c = 0; c < T->ncell; c++) {
            const orc_cell *x = &T->cells[c];
            int64_t *o = &cells9[9 * c];
            o[0] = x->level;
            o[1] = x->ix;
            o[2] = x->iy;
            o[3] = x->iz;
            o[4] = x->first;
            o[5] = x->count;
            o[6] = x->child_first;
            o[7] = x->nchild;
            o[8] = x->parent;
        }
}

/* Dual tree traversal from (root, root); lists sorted by (target, source). */
void orc_tree_lists(orc_tree *T, int theta_num, int theta_den, int64_t *nm2l, int64_t *np2p)
{
    T->m2l.n = T->p2p.n = 0;
    if (T->n > 0) orc_traverse(T->cells, 0, 0, theta_num, theta_den, &T->m2l, &T->p2p);
    orc_sort_pairs(&T->m2l);
    orc_sort_pairs(&T->p2p);
    T->have_lists = 1;
    *nm2l = T->m2l.n;
    *np2p = T->p2p.n;
}

void orc_tree_copy_lists(const orc_tree *T, int32_t *m2l_t, int32_t *m2l_s, int32_t *p2p_t,
                         int32_t *p2p_s)
{
    if (m2l_t) memcpy(m2l_t, T->m2l.t, (size_t)T->m2l.n * sizeof(int32_t));
    if (m2l_s) memcpy(m2l_s, T->m2l.s, (size_t)T->m2l.n * sizeof(int32_t));
    if (p2p_t) memcpy(p2p_t, T->p2p.t, (size_t)T->p2p.n * sizeof(int32_t));
    if (p2p_s) memcpy(p2p_s, T->p2p.s, (size_t)T->p2p.n * sizeof(int32_t));
}

/* R8: geometric centre of a cell, FP64. */
static void orc_centre(const orc_tree *T, const orc_cell *c, double *out)
{
    int32_t ic[3] = {c->ix, c->iy, c->iz};
    double den = ldexp(1.0, c->level + 1);
    for (int d = 0; d < 3; d++) out[d] = T->box[d] + ((double)(2 * (int64_t)ic[d] + 1) * T->box[3]) / den;
}

/* Full FMM evaluation at order p on the stored tree and lists.
 * Outputs phi[i], field[3i..3i+2] in input order.  Optional per-stage
 * outputs for tests: mult (ncell x nk) and loc (ncell x nk) may be NULL. */
int orc_fmm_eval(orc_tree *T, const double *pos, const double *q, int p, double *phi,
                 double *field, double *mult_out, double *loc_out)
{
    if (!T->have_lists || T->ncell < 0) return -1;
    int64_t n = T->n, nc = T->ncell;
    orc_mi t;
    orc_mi_init(&t, p);
    int nk = t.nk;
    double *M = (double *)calloc((size_t)nc * nk, sizeof(double));
    double *L = (double *)calloc((size_t)nc * nk, sizeof(double));
    double *ctr = (double *)malloc((size_t)nc * 3 * sizeof(double));
    for (int64_t c = 0; c < nc; c++) orc_centre(T, &T->cells[c], &ctr[3 * c]);

    /* P2M at leaves */
#pragma omp parallel
    {
        double *mono = (double *)malloc((size_t)nk * sizeof(double));
#pragma omp for schedule(dynamic, 8)
        for (int64_t c = 0; c < nc; c++) {
            const orc_cell *cl = &T->cells[c];
            if (cl->child_first >= 0) continue;
            for (int64_t r = cl->first; r < cl->first + cl->count; r++) {
                int64_t i = T->perm[r];
                double y[3] = {pos[3 * i] - ctr[3 * c], pos[3 * i + 1] - ctr[3 * c + 1],
                               pos[3 * i + 2] - ctr[3 * c + 2]};
                orc_monomials(&t, y, mono);
                for (int k = 0; k < nk; k++) M[c * nk + k] += q[i] * mono[k];
            }
        }
        free(mono);
    }

    /* M2M, deepest level first (cells are level-major, so reverse order) */
    {
        double *mono = (double *)malloc((size_t)nk * sizeof(double));
        for (int64_t c = nc - 1; c >= 0; c--) {
            const orc_cell *cl = &T->cells[c];
            for (int k = 0; k < cl->nchild; k++) {
                int64_t ch = cl->child_first + k;
                double d[3] = {ctr[3 * ch] - ctr[3 * c], ctr[3 * ch + 1] - ctr[3 * c + 1],
                               ctr[3 * ch + 2] - ctr[3 * c + 2]};
                orc_monomials(&t, d, mono);
                for (int al = 0; al < nk; al++) {
                    const int *a = &t.mi[3 * al];
                    double s = 0;
                    for (int be = 0; be < nk; be++) {
                        const int *b = &t.mi[3 * be];
                        if (b[0] > a[0] || b[1] > a[1] || b[2] > a[2]) continue;
                        int g = orc_mi_find(&t, a[0] - b[0], a[1] - b[1], a[2] - b[2]);
                        s += M[ch * nk + be] * mono[g];
                    }
                    M[c * nk + al] += s;
                }
            }
        }
        free(mono);
    }

    /* M2L over the list (grouped by target: each target written by one thread) */
    {
        int64_t m = T->m2l.n;
        int64_t *start = (int64_t *)calloc((size_t)nc + 1, sizeof(int64_t));
        for (int64_t e = 0; e < m; e++) start[T->m2l.t[e] + 1]++;
        for (int64_t c = 0; c < nc; c++) start[c + 1] += start[c];
#pragma omp parallel
        {
            double *b = (double *)malloc((size_t)t.nk2 * sizeof(double));
#pragma omp for schedule(dynamic, 4)
            for (int64_t A = 0; A < nc; A++) {
                for (int64_t e = start[A]; e < start[A + 1]; e++) {
                    int64_t B = T->m2l.s[e];
                    double r[3] = {ctr[3 * A] - ctr[3 * B], ctr[3 * A + 1] - ctr[3 * B + 1],
                                   ctr[3 * A + 2] - ctr[3 * B + 2]};
                    orc_taylor_coeffs(&t, r, b);
                    for (int be = 0; be < nk; be++) {
                        double s = 0;
                        const int *gi = &t.m2l_idx[be * nk];
                        const double *cf = &t.m2l_coef[be * nk];
                        for (int al = 0; al < nk; al++) s += cf[al] * M[B * nk + al] * b[gi[al]];
                        L[A * nk + be] += s;
                    }
                }
            }
            free(b);
        }
        free(start);
    }

    /* L2L, shallowest level first */
    {
        double *mono = (double *)malloc((size_t)nk * sizeof(double));
        for (int64_t c = 0; c < nc; c++) {
            const orc_cell *cl = &T->cells[c];
            for (int k = 0; k < cl->nchild; k++) {
                int64_t ch = cl->child_first + k;
                double d[3] = {ctr[3 * ch] - ctr[3 * c], ctr[3 * ch + 1] - ctr[3 * c + 1],
                               ctr[3 * ch + 2] - ctr[3 * c + 2]};
                orc_monomials(&t, d, mono);
                for (int be = 0; be < nk; be++) {
                    const int *b = &t.mi[3 * be];
                    double s = 0;
                    for (int ga = 0; ga < nk; ga++) {
                        const int *g = &t.mi[3 * ga];
                        if (g[0] < b[0] || g[1] < b[1] || g[2] < b[2]) continue;
                        int dg = orc_mi_find(&t, g[0] - b[0], g[1] - b[1], g[2] - b[2]);
                        /* gamma!/(beta!(gamma-beta)!) d^(gamma-beta)
                         *   = (gamma!/beta!) * [d^(gamma-beta)/(gamma-beta)!] */
                        s += L[c * nk + ga] * (t.fact[ga] / t.fact[be]) * mono[dg];
                    }
                    L[ch * nk + be] += s;
                }
            }
        }
        free(mono);
    }

    /* L2P and P2P at leaves; results in input order */
    {
        int64_t m = T->p2p.n;
        int64_t *start = (int64_t *)calloc((size_t)nc + 1, sizeof(int64_t));
        for (int64_t e = 0; e < m; e++) start[T->p2p.t[e] + 1]++;
        for (int64_t c = 0; c < nc; c++) start[c + 1] += start[c];
        for (int64_t i = 0; i < n; i++) {
            phi[i] = 0;
            field[3 * i] = field[3 * i + 1] = field[3 * i + 2] = 0;
        }
#pragma omp parallel for schedule(dynamic, 4)
        for (int64_t A = 0; A < nc; A++) {
            const orc_cell *ca = &T->cells[A];
            if (ca->child_first >= 0) continue;
            for (int64_t r = ca->first; r < ca->first + ca->count; r++) {
                int64_t i = T->perm[r];
                double xi[3] = {pos[3 * i], pos[3 * i + 1], pos[3 * i + 2]};
                /* far field: phi = sum_beta L_beta u^beta; dphi/du_k = sum L_beta beta_k u^(beta-e_k) */
                double u[3] = {xi[0] - ctr[3 * A], xi[1] - ctr[3 * A + 1], xi[2] - ctr[3 * A + 2]};
                double pf = 0, g[3] = {0, 0, 0};
                for (int be = 0; be < nk; be++) {
                    const int *b = &t.mi[3 * be];
                    double l = L[A * nk + be];
                    if (l == 0.0) continue;
                    pf += l * pow(u[0], b[0]) * pow(u[1], b[1]) * pow(u[2], b[2]);
                    for (int d = 0; d < 3; d++) {
                        if (b[d] == 0) continue;
                        int e[3] = {b[0], b[1], b[2]};
                        e[d] -= 1;
                        g[d] += l * b[d] * pow(u[0], e[0]) * pow(u[1], e[1]) * pow(u[2], e[2]);
                    }
                }
                /* near field over the P2P list */
                double pn = 0, en[3] = {0, 0, 0};
                for (int64_t e = start[A]; e < start[A + 1]; e++) {
                    const orc_cell *cb = &T->cells[T->p2p.s[e]];
                    for (int64_t s = cb->first; s < cb->first + cb->count; s++) {
                        int64_t j = T->perm[s];
                        double dx = xi[0] - pos[3 * j], dy = xi[1] - pos[3 * j + 1], dz = xi[2] - pos[3 * j + 2];
                        double r2 = dx * dx + dy * dy + dz * dz;
                        if (r2 == 0.0) continue;
                        double rr = sqrt(r2);
                        double inv = 1.0 / rr, inv3 = inv / r2;
                        pn += q[j] * inv;
                        en[0] += q[j] * dx * inv3;
                        en[1] += q[j] * dy * inv3;
                        en[2] += q[j] * dz * inv3;
                    }
                }
                phi[i] = pf + pn;
                field[3 * i] = -g[0] + en[0];
                field[3 * i + 1] = -g[1] + en[1];
                field[3 * i + 2] = -g[2] + en[2];
            }
        }
        free(start);
    }

    if (mult_out) memcpy(mult_out, M, (size_t)nc * nk * sizeof(double));
    if (loc_out) memcpy(loc_out, L, (size_t)nc * nk * sizeof(double));
    free(M);
    free(L);
    free(ctr);
    orc_mi_free(&t);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Single-operator entry points for tests of the expansions themselves.     */
/* ------------------------------------------------------------------------ */

int orc_nk(int p)
{
    return (p + 1) * (p + 2) * (p + 3) / 6;
}

/* P2M about centre c of m sources -> mult[nk]. */
void orc_p2m(int p, int64_t m, const double *src, const double *q, const double *c, double *mult)
{
    orc_mi t;
    orc_mi_init(&t, p);
    double *mono = (double *)malloc((size_t)t.nk * sizeof(double));
    for (int k = 0; k < t.nk; k++) mult[k] = 0;
    for (int64_t j = 0; j < m; j++) {
        double y[3] = {src[3 * j] - c[0], src[3 * j + 1] - c[1], src[3 * j + 2] - c[2]};
        orc_monomials(&t, y, mono);
        for (int k = 0; k < t.nk; k++) mult[k] += q[j] * mono[k];
    }
    free(mono);
    orc_mi_free(&t);
}

/* Far-field potential and field of a multipole expansion about c, evaluated
 * at m targets:  phi(x) = sum_alpha (-1)^|alpha| M_alpha d^alpha G(x - c). */
void orc_m2p(int p, const double *mult, const double *c, int64_t m, const double *tgt,
             double *phi, double *field)
{
    orc_mi t;
    orc_mi_init(&t, p);
    orc_mi t2;
    orc_mi_init(&t2, p + 1);  /* gradients need degree p+1 coefficients */
    double *b = (double *)malloc((size_t)t2.nk2 * sizeof(double));
    for (int64_t i = 0; i < m; i++) {
        double r[3] = {tgt[3 * i] - c[0], tgt[3 * i + 1] - c[1], tgt[3 * i + 2] - c[2]};
        orc_taylor_coeffs(&t2, r, b);
        double ph = 0, g[3] = {0, 0, 0};
        for (int al = 0; al < t.nk; al++) {
            const int *a = &t.mi[3 * al];
            double sign = (t.deg[al] & 1) ? -1.0 : 1.0;
            int ga = orc_mi_find(&t2, a[0], a[1], a[2]);
            /* d^alpha G = alpha! b_alpha */
            ph += sign * mult[al] * t2.fact[ga] * b[ga];
            for (int d = 0; d < 3; d++) {
                int gd = orc_mi_find(&t2, a[0] + (d == 0), a[1] + (d == 1), a[2] + (d == 2));
                g[d] += sign * mult[al] * t2.fact[gd] * b[gd];
            }
        }
        phi[i] = ph;
        field[3 * i] = -g[0];
        field[3 * i + 1] = -g[1];
        field[3 * i + 2] = -g[2];
    }
    free(b);
    orc_mi_free(&t);
    orc_mi_free(&t2);
}

/* M2M of one expansion from centre c to centre c2. */
void orc_m2m(int p, const double *mult, const double *c, const double *c2, double *out)
{
    orc_mi t;
    orc_mi_init(&t, p);
    double *mono = (double *)malloc((size_t)t.nk * sizeof(double));
    double d[3] = {c[0] - c2[0], c[1] - c2[1], c[2] - c2[2]};
    orc_monomials(&t, d, mono);
    for (int al = 0; al < t.nk; al++) {
        const int *a = &t.mi[3 * al];
        double s = 0;
        for (int be = 0; be < t.nk; be++) {
            const int *bb = &t.mi[3 * be];
            if (bb[0] > a[0] || bb[1] > a[1] || bb[2] > a[2]) continue;
            int g = orc_mi_find(&t, a[0] - bb[0], a[1] - bb[1], a[2] - bb[2]);
            s += mult[be] * mono[g];
        }
        out[al] = s;
    }
    free(mono);
    orc_mi_free(&t);
}

/* M2L of one multipole about cB into a local expansion about cA. */
void orc_m2l(int p, const double *mult, const double *cB, const double *cA, double *loc)
{
    orc_mi t;
    orc_mi_init(&t, p);
    double *b = (double *)malloc((size_t)t.nk2 * sizeof(double));
    double r[3] = {cA[0] - cB[0], cA[1] - cB[1], cA[2] - cB[2]};
    orc_taylor_coeffs(&t, r, b);
    for (int be = 0; be < t.nk; be++) {
        double s = 0;
        for (int al = 0; al < t.nk; al++)
            s += t.m2l_coef[be * t.nk + al] * mult[al] * b[t.m2l_idx[be * t.nk + al]];
        loc[be] = s;
    }
    free(b);
    orc_mi_free(&t);
}

/* L2L of one local expansion from centre c to centre c2. */
void orc_l2l(int p, const double *loc, const double *c, const double *c2, double *out)
{
    orc_mi t;
    orc_mi_init(&t, p);
    double *mono = (double *)malloc((size_t)t.nk * sizeof(double));
    double d[3] = {c2[0] - c[0], c2[1] - c[1], c2[2] - c[2]};
    orc_monomials(&t, d, mono);
    for (int be = 0; be < t.nk; be++) {
        const int *bb = &t.mi[3 * be];
        double s = 0;
        for (int ga = 0; ga < t.nk; ga++) {
            const int *g = &t.mi[3 * ga];
            if (g[0] < bb[0] || g[1] < bb[1] || g[2] < bb[2]) continue;
            int dg = orc_mi_find(&t, g[0] - bb[0], g[1] - bb[1], g[2] - bb[2]);
            s += loc[ga] * (t.fact[ga] / t.fact[be]) * mono[dg];
        }
        out[be] = s;
    }
    free(mono);
    orc_mi_free(&t);
}

/* L2P of one local expansion about c at m targets. */
void orc_l2p(int p, const double *loc, const double *c, int64_t m, const double *tgt,
             double *phi, double *field)
{
    orc_mi t;
    orc_mi_init(&t, p);
    for (int64_t i = 0; i < m; i++) {
        double u[3] = {tgt[3 * i] - c[0], tgt[3 * i + 1] - c[1], tgt[3 * i + 2] - c[2]};
        double pf = 0, g[3] = {0, 0, 0};
        for (int be = 0; be < t.nk; be++) {
            const int *b = &t.mi[3 * be];
            pf += loc[be] * pow(u[0], b[0]) * pow(u[1], b[1]) * pow(u[2], b[2]);
            for (int d = 0; d < 3; d++) {
                if (b[d] == 0) continue;
                int e[3] = {b[0], b[1], b[2]};
                e[d] -= 1;
                g[d] += loc[be] * b[d] * pow(u[0], e[0]) * pow(u[1], e[1]) * pow(u[2], e[2]);
            }
        }
        phi[i] = pf;
        field[3 * i] = -g[0];
        field[3 * i + 1] = -g[1];
        field[3 * i + 2] = -g[2];
    }
    orc_mi_free(&t);
}

/* Taylor coefficients b_gamma(r) for all |gamma| <= order, in the oracle's
 * multi-index order (degree, then a0 descending, then a1 descending). */
void orc_taylor(int order, const double *r, double *b)
{
    /* K_2p with 2p >= order; reuse the table with p = ceil(order/2) */
    int p = (order + 1) / 2;
    orc_mi t;
    orc_mi_init(&t, p);
    double *bb = (double *)malloc((size_t)t.nk2 * sizeof(double));
    orc_taylor_coeffs(&t, r, bb);
    int cnt = (order + 1) * (order + 2) * (order + 3) / 6;
    memcpy(b, bb, (size_t)cnt * sizeof(double));
    free(bb);
    orc_mi_free(&t);
}

int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Threads of later OpenMP regions (timing on a stated number of cores). */
void orc_set_num_threads(int n)
{
#ifdef _OPENMP
    if (n >= 1)
        omp_set_num_threads(n);
#else
    (void)n;
#endif
}
