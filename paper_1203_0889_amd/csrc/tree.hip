// Bounding cube, Morton keys and the adaptive octree (Sec. 2.1, 2.2).
//
// Geometry is integer-exact: a key is 21 bits per axis interleaved (bit 3b+d
// of the key = bit b of axis d), cell (level l, ix, iy, iz) spans
// [i * 2^(21-l), (i+1) * 2^(21-l)) grid units per axis.  The only floating
// point step is the quantisation ix = min(floor((x - min) * scale), 2^21 - 1)
// with scale = 2^21 / side, done with explicitly rounded FP64 operations so
// no fused multiply-add can change a key.
#include "tree.h"

namespace fmm {

namespace {

// Order-preserving map of a double onto uint64 (for atomic min / max).
__device__ inline uint64_t ord_of(double x) {
    uint64_t u = (uint64_t)__double_as_longlong(x);
    return (u >> 63) ? ~u : (u | 0x8000000000000000ull);
}
__device__ inline double double_of_ord(uint64_t u) {
    u = (u >> 63) ? (u & 0x7fffffffffffffffull) : ~u;
    return __longlong_as_double((long long)u);
}

__device__ inline int inst_of(const int64_t *__restrict__ offsets, int n_inst, int64_t i) {
    // largest k with offsets[k] <= i (instances may be empty)
    int lo = 0, hi = n_inst - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (offsets[mid] <= i) lo = mid; else hi = mid - 1;
    }
    return lo;
}

constexpr int kBoxThreads = 256;
constexpr int kBoxItems = 8;

// ord[k*6 + d] = ordered min of axis d, ord[k*6 + 3 + d] = ~(ordered max),
// so that both are reduced with atomicMin.  Also flags non-finite input.
__global__ void __launch_bounds__(kBoxThreads) k_bbox(const double *__restrict__ pos, int64_t n,
                                                      const int64_t *__restrict__ offsets, int n_inst,
                                                      unsigned long long *__restrict__ ord, int *__restrict__ bad) {
    __shared__ uint64_t red[6][kBoxThreads];
    int64_t t0 = (int64_t)blockIdx.x * kBoxThreads * kBoxItems;
    if (t0 >= n) return;
    int64_t t1 = t0 + kBoxThreads * kBoxItems;
    if (t1 > n) t1 = n;
    int k0 = inst_of(offsets, n_inst, t0), k1 = inst_of(offsets, n_inst, t1 - 1);
    uint64_t mn[3] = {~0ull, ~0ull, ~0ull}, mx[3] = {~0ull, ~0ull, ~0ull};
    int my_bad = 0;
    for (int64_t i = t0 + threadIdx.x; i < t1; i += kBoxThreads) {
        int k = k0 == k1 ? k0 : inst_of(offsets, n_inst, i);
        for (int d = 0; d < 3; d++) {
            double v = pos[3 * i + d];
            if (!isfinite(v)) my_bad = 1;
            uint64_t o = ord_of(v);
            if (k0 == k1) {
                mn[d] = o < mn[d] ? o : mn[d];
                mx[d] = ~o < mx[d] ? ~o : mx[d];
            } else {
                atomicMin(&ord[k * 6 + d], (unsigned long long)o);
                atomicMin(&ord[k * 6 + 3 + d], (unsigned long long)~o);
            }
        }
    }
    if (my_bad) atomicOr(bad, 1);
    if (k0 != k1) return;
    for (int d = 0; d < 3; d++) {
        red[d][threadIdx.x] = mn[d];
        red[3 + d][threadIdx.x] = mx[d];
    }
    __syncthreads();
    for (int s = kBoxThreads / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s)
            for (int j = 0; j < 6; j++) {
                uint64_t a = red[j][threadIdx.x], b = red[j][threadIdx.x + s];
                red[j][threadIdx.x] = a < b ? a : b;
            }
        __syncthreads();
    }
    if (threadIdx.x < 6) atomicMin(&ord[k0 * 6 + threadIdx.x], (unsigned long long)red[threadIdx.x][0]);
}

// box[k*4 + 0..2] = min corner, box[k*4 + 3] = side (largest extent, 1 if
// zero); scale[k] = 2^21 / side.  A user box overrides.
__global__ void k_box_finish(const unsigned long long *__restrict__ ord, int n_inst, const int64_t *__restrict__ offsets,
                             int use_user, double ux, double uy, double uz, double us, double *__restrict__ box,
                             double *__restrict__ scale) {
    int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n_inst) return;
    double lo[3], side = 0.0;
    if (use_user) {
        lo[0] = ux;
        lo[1] = uy;
        lo[2] = uz;
        side = us;
    } else if (offsets[k + 1] > offsets[k]) {
        for (int d = 0; d < 3; d++) {
            lo[d] = double_of_ord(ord[k * 6 + d]);
            double hi = double_of_ord(~ord[k * 6 + 3 + d]);
            double e = __dsub_rn(hi, lo[d]);
            side = e > side ? e : side;
        }
    } else {
        lo[0] = lo[1] = lo[2] = 0.0;
    }
    if (!(side > 0.0)) side = 1.0;
    box[4 * k + 0] = lo[0];
    box[4 * k + 1] = lo[1];
    box[4 * k + 2] = lo[2];
    box[4 * k + 3] = side;
    scale[k] = 2097152.0 / side;  // IEEE division, correctly rounded
}

__device__ inline uint64_t spread21(uint64_t v) {
    v &= 0x1fffffull;
    v = (v | (v << 32)) & 0x1f00000000ffffull;
    v = (v | (v << 16)) & 0x1f0000ff0000ffull;
    v = (v | (v << 8)) & 0x100f00f00f00f00full;
    v = (v | (v << 4)) & 0x10c30c30c30c30c3ull;
    v = (v | (v << 2)) & 0x1249249249249249ull;
    return v;
}

__global__ void k_keys(const double *__restrict__ pos, int64_t n, const int64_t *__restrict__ offsets, int n_inst,
                       const double *__restrict__ box, const double *__restrict__ scale, uint64_t *__restrict__ keys,
                       uint32_t *__restrict__ idx, uint32_t *__restrict__ inst) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        int k = n_inst == 1 ? 0 : inst_of(offsets, n_inst, i);
        double sc = scale[k];
        uint64_t key = 0;
        for (int d = 0; d < 3; d++) {
            double s = __dmul_rn(__dsub_rn(pos[3 * i + d], box[4 * k + d]), sc);
            double f = floor(s);
            int64_t v = f < 0.0 ? 0 : (int64_t)f;
            v = v > 2097151 ? 2097151 : v;
            key |= spread21((uint64_t)v) << d;
        }
        keys[i] = key;
        idx[i] = (uint32_t)i;
        if (inst) inst[i] = (uint32_t)k;
    }
}

// After the instance pass: rank permutation r -> old rank; gather keys/idx.
__global__ void k_inst_keys(const uint32_t *__restrict__ idx, int64_t n, const int64_t *__restrict__ offsets, int n_inst,
                            uint32_t *__restrict__ ikey, uint32_t *__restrict__ rank) {
    for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < n; r += (int64_t)gridDim.x * blockDim.x) {
        ikey[r] = (uint32_t)inst_of(offsets, n_inst, idx[r]);
        rank[r] = (uint32_t)r;
    }
}

__global__ void k_permute_keys(const uint32_t *__restrict__ rank, int64_t n, const uint64_t *__restrict__ kin,
                               const uint32_t *__restrict__ vin, uint64_t *__restrict__ kout, uint32_t *__restrict__ vout) {
    for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < n; r += (int64_t)gridDim.x * blockDim.x) {
        uint32_t s = rank[r];
        kout[r] = kin[s];
        vout[r] = vin[s];
    }
}

__global__ void k_gather(const double *__restrict__ pos, const double *__restrict__ q, const uint32_t *__restrict__ idx,
                         int64_t n, double *__restrict__ xs, double *__restrict__ ys, double *__restrict__ zs,
                         double *__restrict__ qs) {
    for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < n; r += (int64_t)gridDim.x * blockDim.x) {
        uint32_t i = idx[r];
        xs[r] = pos[3 * (int64_t)i];
        ys[r] = pos[3 * (int64_t)i + 1];
        zs[r] = pos[3 * (int64_t)i + 2];
        qs[r] = q[i];
    }
}

__global__ void k_roots(const int64_t *__restrict__ offsets, int n_inst, CellArrays c) {
    int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n_inst) return;
    c.level[k] = 0;
    c.ix[k] = c.iy[k] = c.iz[k] = 0;
    c.first[k] = (int32_t)offsets[k];
    c.count[k] = (int32_t)(offsets[k + 1] - offsets[k]);
    c.child[k] = -1;
    c.nchild[k] = 0;
    c.parent[k] = -1;
    c.inst[k] = k;
}

// For each cell of the current level: octant boundaries of its children
// (lower bounds of each level-(l+1) digit within its sorted key range) and
// the number of non-empty children, or 0 if it stays a leaf.  Eight lanes
// per cell: lane o searches the lower bound of digit o on its own, so the
// seven searches run side by side instead of one after another.
__global__ void k_tree_count(CellArrays c, int32_t lb, int32_t le, int ncrit, int max_level,
                             const uint64_t *__restrict__ skeys, int32_t *__restrict__ bounds,
                             int32_t *__restrict__ nch) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int32_t cell = lb + (int32_t)(t >> 3);
    const int o = (int)(t & 7);
    if (cell >= le) return;   // the 8 lanes of a cell leave together
    const int32_t j = cell - lb;
    const int level = c.level[cell];
    const int32_t first = c.first[cell], count = c.count[cell];
    if (count <= ncrit || level >= max_level) {
        if (o == 0) nch[j] = 0;
        return;
    }
    const int shift = 3 * (kLevels - (level + 1));
    const int32_t end = first + count;
    // first index in [first, end) whose digit is >= o
    int32_t a = first, b = end;
    if (o > 0)
        while (a < b) {
            int32_t mid = a + ((b - a) >> 1);
            int dig = (int)((skeys[mid] >> shift) & 7ull);
            if (dig < o) a = mid + 1; else b = mid;
        }
    bounds[9 * j + o] = a;
    if (o == 7) bounds[9 * j + 8] = end;
    // child o is non-empty iff the next bound is larger
    const int32_t next = __shfl_down(a, 1, 8);
    const bool ne = (o == 7 ? end : next) > a;
    const uint64_t m = __ballot(ne);
    if (o == 0) nch[j] = __popcll((m >> (threadIdx.x & 63 & ~7)) & 0xffull);
}

__global__ void k_tree_write(CellArrays c, int32_t lb, int32_t le, const int32_t *__restrict__ bounds,
                             const int32_t *__restrict__ nch, const int32_t *__restrict__ off) {
    int32_t cell = lb + blockIdx.x * blockDim.x + threadIdx.x;
    if (cell >= le) return;
    int32_t j = cell - lb;
    if (nch[j] == 0) return;
    int32_t dst = le + off[j];
    c.child[cell] = dst;
    c.nchild[cell] = nch[j];
    int level = c.level[cell] + 1;
    int32_t px = c.ix[cell], py = c.iy[cell], pz = c.iz[cell], inst = c.inst[cell];
    for (int o = 0; o < 8; o++) {
        int32_t a = bounds[9 * j + o], b = bounds[9 * j + o + 1];
        if (b <= a) continue;
        c.level[dst] = level;
        c.ix[dst] = 2 * px + (o & 1);
        c.iy[dst] = 2 * py + ((o >> 1) & 1);
        c.iz[dst] = 2 * pz + ((o >> 2) & 1);
        c.first[dst] = a;
        c.count[dst] = b - a;
        c.child[dst] = -1;
        c.nchild[dst] = 0;
        c.parent[dst] = cell;
        c.inst[dst] = inst;
        dst++;
    }
}

// Device-driven levels: the cell range of level l is [lev[l], lev[l + 1]),
// read on the device, so a batch of levels is enqueued without host reads.
__global__ void k_tree_levels_init(int32_t *__restrict__ lev, int n_inst, int nlev) {
    for (int i = threadIdx.x; i < nlev; i += blockDim.x) lev[i] = i == 0 ? 0 : n_inst;   // later levels start empty
    if (threadIdx.x == 0) lev[nlev] = 0;                                        // overflow flag
}

// The per-level scan of child counts works on chunks of kTreeChunk cells:
// the count kernel writes each chunk's sum, one workgroup scans the chunk
// sums, and the write kernel finishes each cell's offset inside its chunk.
constexpr int kTreeChunk = 32;
constexpr int kTreeCountThreads = kTreeChunk * 8;   // 8 lanes per cell
constexpr int kChunkScanThreads = 1024;

// Child ranges of the cells of level `level` (8 lanes per cell, binary
// searches over the sorted keys), their number of non-empty children, and
// the per-chunk sums of those numbers.
__global__ void __launch_bounds__(kTreeCountThreads) k_tree_count_dev(CellArrays c, const int32_t *__restrict__ lev,
                                                                      int level, int ncrit, int max_level,
                                                                      const uint64_t *__restrict__ skeys,
                                                                      int32_t *__restrict__ bounds,
                                                                      int32_t *__restrict__ nch,
                                                                      int32_t *__restrict__ csum) {
    __shared__ int wsum[kTreeCountThreads / 64];
    const int32_t lb = lev[level], le = lev[level + 1];
    const int32_t ncl = le - lb;
    const int32_t nchunk = (ncl + kTreeChunk - 1) / kTreeChunk;
    const int o = threadIdx.x & 7, lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    for (int32_t ci = blockIdx.x; ci < nchunk; ci += gridDim.x) {   // uniform over the workgroup
        const int32_t j = ci * kTreeChunk + (int32_t)(threadIdx.x >> 3);
        int mine = 0;
        if (j < ncl) {
            const int32_t cell = lb + j;
            const int level_c = c.level[cell];
            const int32_t first = c.first[cell], count = c.count[cell];
            if (count <= ncrit || level_c >= max_level) {
                if (o == 0) nch[j] = 0;
            } else {   // uniform over the cell's 8 lanes
                const int shift = 3 * (kLevels - (level_c + 1));
                const int32_t end = first + count;
                int32_t a = first, b = end;
                if (o > 0)
                    while (a < b) {
                        int32_t mid = a + ((b - a) >> 1);
                        int dig = (int)((skeys[mid] >> shift) & 7ull);
                        if (dig < o) a = mid + 1; else b = mid;
                    }
                bounds[9 * j + o] = a;
                if (o == 7) bounds[9 * j + 8] = end;
                const int32_t next = __shfl_down(a, 1, 8);
                const bool ne = (o == 7 ? end : next) > a;
                const uint64_t m = __ballot(ne);
                if (o == 0) {
                    mine = __popcll((m >> (lane & ~7)) & 0xffull);
                    nch[j] = mine;
                }
            }
        }
#pragma unroll
        for (int d = 32; d >= 1; d >>= 1) mine += __shfl_xor(mine, d, 64);
        if (lane == 0) wsum[w] = mine;
        __syncthreads();
        if (threadIdx.x == 0) {
            int t = 0;
#pragma unroll
            for (int i = 0; i < kTreeCountThreads / 64; i++) t += wsum[i];
            csum[ci] = t;
        }
        __syncthreads();
    }
}

// One workgroup: exclusive scan of the chunk sums in place; *total = the
// number of cells of the next level.
__global__ void __launch_bounds__(kChunkScanThreads) k_tree_chunk_scan(const int32_t *__restrict__ lev, int level,
                                                                       int32_t *__restrict__ csum,
                                                                       int32_t *__restrict__ total) {
    constexpr int kItems = 4, kStep = kChunkScanThreads * kItems;
    __shared__ int wsum[kChunkScanThreads / 64];
    const int32_t ncl = lev[level + 1] - lev[level];
    const int32_t nchunk = (ncl + kTreeChunk - 1) / kTreeChunk;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    int carry = 0;
    for (int32_t c0 = 0; c0 < nchunk; c0 += kStep) {
        const int32_t b0 = c0 + threadIdx.x * kItems;
        int v[kItems], sum = 0;
#pragma unroll
        for (int i = 0; i < kItems; i++) {
            v[i] = b0 + i < nchunk ? csum[b0 + i] : 0;
            sum += v[i];
        }
        int inc = sum;
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            int t = __shfl_up(inc, d, 64);
            if (lane >= d) inc += t;
        }
        if (lane == 63) wsum[w] = inc;
        __syncthreads();
        int before = 0, tot = 0;
#pragma unroll
        for (int i = 0; i < kChunkScanThreads / 64; i++) {
            if (i < w) before += wsum[i];
            tot += wsum[i];
        }
        int pre = carry + before + inc - sum;
#pragma unroll
        for (int i = 0; i < kItems; i++) {
            if (b0 + i < nchunk) csum[b0 + i] = pre;
            pre += v[i];
        }
        carry += tot;
        __syncthreads();
    }
    if (threadIdx.x == 0) *total = carry;
}

// Children of level `level`; lev[level + 2] = end of the new level.  A tree
// larger than cap cells stops here: the flag lev[nlev] is set, nothing is
// written past cap, and the new level is left empty.  One thread per cell;
// a chunk's cells sit in consecutive lanes, which scan their child counts.
__global__ void __launch_bounds__(256) k_tree_write_dev(CellArrays c, int32_t *__restrict__ lev, int level, int nlev,
                                                        const int32_t *__restrict__ bounds,
                                                        const int32_t *__restrict__ nch,
                                                        const int32_t *__restrict__ cscan,
                                                        const int32_t *__restrict__ total, int32_t cap) {
    static_assert(256 % kTreeChunk == 0 && kTreeChunk <= 64, "chunks must not straddle waves");
    const int32_t lb = lev[level], le = lev[level + 1];
    const int32_t ncl = le - lb;
    const bool over = (int64_t)le + *total > cap;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        lev[level + 2] = over ? le : le + *total;
        if (over) lev[nlev] = 1;
    }
    if (over) return;
    const int sub = threadIdx.x & (kTreeChunk - 1);
    for (int32_t j0 = blockIdx.x * 256; j0 < ncl; j0 += gridDim.x * 256) {
        const int32_t j = j0 + (int32_t)threadIdx.x;
        const int v = j < ncl ? nch[j] : 0;
        int inc = v;
#pragma unroll
        for (int d = 1; d < kTreeChunk; d <<= 1) {
            int t = __shfl_up(inc, d, kTreeChunk);
            if (sub >= d) inc += t;
        }
        if (v == 0) continue;
        const int32_t cell = lb + j;
        int32_t dst = le + cscan[j / kTreeChunk] + inc - v;
        c.child[cell] = dst;
        c.nchild[cell] = v;
        const int lv = c.level[cell] + 1;
        const int32_t px = c.ix[cell], py = c.iy[cell], pz = c.iz[cell], inst = c.inst[cell];
        for (int o = 0; o < 8; o++) {
            const int32_t a = bounds[9 * j + o], b = bounds[9 * j + o + 1];
            if (b <= a) continue;
            c.level[dst] = lv;
            c.ix[dst] = 2 * px + (o & 1);
            c.iy[dst] = 2 * py + ((o >> 1) & 1);
            c.iz[dst] = 2 * pz + ((o >> 2) & 1);
            c.first[dst] = a;
            c.count[dst] = b - a;
            c.child[dst] = -1;
            c.nchild[dst] = 0;
            c.parent[dst] = cell;
            c.inst[dst] = inst;
            dst++;
        }
    }
}

__global__ void k_leaf_of(CellArrays c, int32_t ncell, int32_t *__restrict__ leaf_of, int32_t *__restrict__ nleaf) {
    for (int32_t cell = blockIdx.x * blockDim.x + threadIdx.x; cell < ncell; cell += gridDim.x * blockDim.x) {
        c.rec[cell] = make_int4(c.ix[cell] | (c.level[cell] << 24), c.iy[cell] | (c.nchild[cell] << 24), c.iz[cell],
                                c.child[cell]);
        if (c.child[cell] >= 0) continue;
        atomicAdd(nleaf, 1);
        int32_t f = c.first[cell], e = f + c.count[cell];
        for (int32_t r = f; r < e; r++) leaf_of[r] = cell;
    }
}

// The cells with children: a flag per cell, scanned in place into each
// parent's rank, then every parent stores its index at its rank.
__global__ void k_parent_flags(const int32_t *__restrict__ child, int32_t ncell, int32_t *__restrict__ flag) {
    for (int32_t cell = blockIdx.x * blockDim.x + threadIdx.x; cell < ncell; cell += gridDim.x * blockDim.x)
        flag[cell] = child[cell] >= 0 ? 1 : 0;
}

__global__ void k_parent_scatter(const int32_t *__restrict__ child, int32_t ncell, const int32_t *__restrict__ ppos,
                                 int32_t *__restrict__ plist) {
    for (int32_t cell = blockIdx.x * blockDim.x + threadIdx.x; cell < ncell; cell += gridDim.x * blockDim.x)
        if (child[cell] >= 0) plist[ppos[cell]] = cell;
}

// A frozen-topology rebuild: every sorted particle's new coordinates are
// finite (flag[0]) and, with check_leaf, still inside its leaf cell widened
// by 1/8 of its side on every face (flag[2] otherwise).  Coordinates in
// grid units of the stored box, as the keys were computed.
__global__ void k_refresh_check(CellArrays c, const int32_t *__restrict__ leaf_of, const double *__restrict__ xs,
                                const double *__restrict__ ys, const double *__restrict__ zs,
                                const double *__restrict__ box, const double *__restrict__ scale, int64_t n,
                                int check_leaf, int32_t *__restrict__ flag) {
    bool bad = false, out = false;
    for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < n; r += (int64_t)gridDim.x * blockDim.x) {
        const double x[3] = {xs[r], ys[r], zs[r]};
        if (!(isfinite(x[0]) && isfinite(x[1]) && isfinite(x[2]))) {
            bad = true;
            continue;
        }
        if (!check_leaf) continue;
        const int32_t A = leaf_of[r];
        const int k = c.inst[A], L = c.level[A];
        const double side = ldexp(1.0, kLevels - L), slack = side * 0.125;
        const int32_t cc[3] = {c.ix[A], c.iy[A], c.iz[A]};
        for (int d = 0; d < 3; d++) {
            const double sg = __dmul_rn(__dsub_rn(x[d], box[4 * k + d]), scale[k]);
            const double lo = cc[d] * side;
            if (!(sg >= lo - slack && sg < lo + side + slack)) out = true;
        }
    }
    if (__ballot(bad) && (threadIdx.x & 63) == 0) atomicOr(&flag[0], 1);
    if (__ballot(out) && (threadIdx.x & 63) == 0) atomicOr(&flag[1], 1);
}

}  // namespace

void launch_refresh_check(CellArrays c, const int32_t *leaf_of, const double *xs, const double *ys, const double *zs,
                          const double *box, const double *scale, int64_t n, bool check_leaf, int32_t *flag,
                          hipStream_t s) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_refresh_check, dim3(grid_for(n, 256, 8192)), dim3(256), 0, s, c, leaf_of, xs, ys, zs, box,
                       scale, n, check_leaf ? 1 : 0, flag);
    FMM_LAUNCH_CHECK();
}

void launch_bbox(const double *pos, int64_t n, const int64_t *d_offsets, int n_inst, unsigned long long *d_ord,
                 int *d_bad, hipStream_t s) {
    FMM_HIP_CHECK(hipMemsetAsync(d_ord, 0xff, sizeof(unsigned long long) * 6 * n_inst, s));
    if (n > 0) {
        int64_t nb = (n + kBoxThreads * kBoxItems - 1) / (kBoxThreads * kBoxItems);
        hipLaunchKernelGGL(k_bbox, dim3((unsigned)nb), dim3(kBoxThreads), 0, s, pos, n, d_offsets, n_inst, d_ord, d_bad);
        FMM_LAUNCH_CHECK();
    }
}

void launch_box_finish(const unsigned long long *d_ord, int n_inst, const int64_t *d_offsets, bool user,
                       const double *ubox, double *d_box, double *d_scale, hipStream_t s) {
    hipLaunchKernelGGL(k_box_finish, dim3(grid_for(n_inst, 64)), dim3(64), 0, s, d_ord, n_inst, d_offsets, user ? 1 : 0,
                       ubox[0], ubox[1], ubox[2], ubox[3], d_box, d_scale);
    FMM_LAUNCH_CHECK();
}

void launch_keys(const double *pos, int64_t n, const int64_t *d_offsets, int n_inst, const double *d_box,
                 const double *d_scale, uint64_t *keys, uint32_t *idx, hipStream_t s) {
    if (n == 0) return;
    hipLaunchKernelGGL(k_keys, dim3(grid_for(n, 256, 8192)), dim3(256), 0, s, pos, n, d_offsets, n_inst, d_box, d_scale,
                       keys, idx, (uint32_t *)nullptr);
    FMM_LAUNCH_CHECK();
}

void sort_by_instance(uint64_t *keys, uint32_t *idx, uint64_t *kalt, uint32_t *valt, uint32_t *ikey, uint32_t *ialt,
                      uint32_t *rank, uint32_t *ralt, int64_t n, const int64_t *d_offsets, int n_inst, int32_t *tmp,
                      hipStream_t s) {
    if (n_inst <= 1 || n <= 1) return;
    hipLaunchKernelGGL(k_inst_keys, dim3(grid_for(n, 256, 8192)), dim3(256), 0, s, idx, n, d_offsets, n_inst, ikey, rank);
    FMM_LAUNCH_CHECK();
    int bits = 0;
    while ((1 << bits) < n_inst) bits++;
    radix_sort_u32(ikey, rank, ialt, ralt, n, 0, bits, tmp, s);
    hipLaunchKernelGGL(k_permute_keys, dim3(grid_for(n, 256, 8192)), dim3(256), 0, s, rank, n, keys, idx, kalt, valt);
    FMM_LAUNCH_CHECK();
    FMM_HIP_CHECK(hipMemcpyAsync(keys, kalt, n * sizeof(uint64_t), hipMemcpyDeviceToDevice, s));
    FMM_HIP_CHECK(hipMemcpyAsync(idx, valt, n * sizeof(uint32_t), hipMemcpyDeviceToDevice, s));
}

void launch_gather(const double *pos, const double *q, const uint32_t *idx, int64_t n, double *xs, double *ys,
                   double *zs, double *qs, hipStream_t s) {
    if (n == 0) return;
    hipLaunchKernelGGL(k_gather, dim3(grid_for(n, 256, 8192)), dim3(256), 0, s, pos, q, idx, n, xs, ys, zs, qs);
    FMM_LAUNCH_CHECK();
}

void launch_roots(const int64_t *d_offsets, int n_inst, CellArrays c, hipStream_t s) {
    hipLaunchKernelGGL(k_roots, dim3(grid_for(n_inst, 64)), dim3(64), 0, s, d_offsets, n_inst, c);
    FMM_LAUNCH_CHECK();
}

void launch_tree_count(CellArrays c, int32_t lb, int32_t le, int ncrit, int max_level, const uint64_t *skeys,
                       int32_t *bounds, int32_t *nch, hipStream_t s) {
    hipLaunchKernelGGL(k_tree_count, dim3(grid_for((int64_t)(le - lb) * 8, 128, 1 << 30)), dim3(128), 0, s, c, lb, le,
                       ncrit, max_level, skeys, bounds, nch);
    FMM_LAUNCH_CHECK();
}

void launch_tree_write(CellArrays c, int32_t lb, int32_t le, const int32_t *bounds, const int32_t *nch,
                       const int32_t *off, hipStream_t s) {
    hipLaunchKernelGGL(k_tree_write, dim3(grid_for(le - lb, 128, 1 << 30)), dim3(128), 0, s, c, lb, le, bounds, nch, off);
    FMM_LAUNCH_CHECK();
}

void launch_tree_levels_init(int32_t *lev, int n_inst, int nlev, hipStream_t s) {
    hipLaunchKernelGGL(k_tree_levels_init, dim3(1), dim3(64), 0, s, lev, n_inst, nlev);
    FMM_LAUNCH_CHECK();
}

void launch_tree_level_dev(CellArrays c, int32_t *lev, int level, int nlev, int ncrit, int max_level,
                           const uint64_t *skeys, int32_t *bounds, int32_t *nch, int32_t *csum, int32_t *total,
                           int32_t cap, hipStream_t s) {
    const int64_t nchunk_max = ((int64_t)cap + kTreeChunk - 1) / kTreeChunk;
    hipLaunchKernelGGL(k_tree_count_dev, dim3(grid_for(nchunk_max, 1, 4096)), dim3(kTreeCountThreads), 0, s, c, lev,
                       level, ncrit, max_level, skeys, bounds, nch, csum);
    FMM_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_tree_chunk_scan, dim3(1), dim3(kChunkScanThreads), 0, s, lev, level, csum, total);
    FMM_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_tree_write_dev, dim3(grid_for(cap, 256, 4096)), dim3(256), 0, s, c, lev, level, nlev, bounds,
                       nch, csum, total, cap);
    FMM_LAUNCH_CHECK();
}

void launch_leaf_of(CellArrays c, int32_t ncell, int32_t *leaf_of, int32_t *nleaf, hipStream_t s) {
    FMM_HIP_CHECK(hipMemsetAsync(nleaf, 0, sizeof(int32_t), s));
    hipLaunchKernelGGL(k_leaf_of, dim3(grid_for(ncell, 256, 8192)), dim3(256), 0, s, c, ncell, leaf_of, nleaf);
    FMM_LAUNCH_CHECK();
}

void launch_parent_list(CellArrays c, int32_t ncell, int32_t *ppos, int32_t *plist, int32_t *tmp, hipStream_t s) {
    if (ncell <= 0) return;
    const dim3 grid(grid_for(ncell, 256, 8192)), block(256);
    hipLaunchKernelGGL(k_parent_flags, grid, block, 0, s, (const int32_t *)c.child, ncell, ppos);
    FMM_LAUNCH_CHECK();
    exclusive_scan_i32(ppos, ncell, ppos + ncell, tmp, s);
    hipLaunchKernelGGL(k_parent_scatter, grid, block, 0, s, (const int32_t *)c.child, ncell, (const int32_t *)ppos,
                       plist);
    FMM_LAUNCH_CHECK();
}

}  // namespace fmm
