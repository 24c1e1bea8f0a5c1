// M2L as a dense contraction on the matrix cores (the multipole-to-local
// stage of Sec. 2.1, applied hundreds of times per cell).
//
// With level-scaled coefficients the M2L operator of a pair (A <- B) depends
// only on its class c = (delta, rho): delta = level(A) - level(B) and rho =
// (C_A - C_B) / min(S_A, S_B), the integer displacement of the centres in
// units of the smaller cell (half grid units C, cell sides S).  The real
// operator T_c ((p+1)^2 x (p+1)^2) is built once per class in FP64 from the
// irregular solid harmonics I_n^m(rho / (2 S_A / S_min)) and stored as two
// bf16 pieces (the rounding of each entry and of its remainder):
//   L~_n^m += (-1)^n sum_k 2^(delta k) sum_l M~_k^l I_(n+k)^(m+l)
// Classes with |delta| <= 2 and |rho_i| <= 24 (all pairs of a uniform tree,
// 99.8% of the 1M-particle Plummer tree at theta = 1/2) index a dense table;
// their operators are cached in the plan across builds.  The rest (deeper
// level differences: a few pairs per class) go to the per-pair FP64 kernel.
//
// Batching: targets are grouped 256 at a time (same level and octant,
// Morton order, so neighbouring targets share their class sets).  A group's
// entries are its distinct classes in the order of their operator slots,
// each with the source cell of every target slot (-1 if absent).  The work
// queue applies each entry's T_c to the gathered multipoles on the matrix
// cores.
#include "m2l_mfma.h"
#include "queue.h"

#include <stdexcept>

namespace fmm {

namespace {

// bf16 bits of x, rounded to nearest even (finite inputs)
__device__ inline uint32_t bf16_bits(float x) {
    const uint32_t u = __float_as_uint(x);
    return (u + 0x7fffu + ((u >> 16) & 1u)) >> 16;
}
__device__ inline float bf16_value(uint32_t h) { return __uint_as_float(h << 16); }

__device__ inline int dense_key(int delta, int rx, int ry, int rz) {
    if (delta < -kDeltaMax || delta > kDeltaMax) return -1;
    if (rx < -kRhoMax || rx > kRhoMax || ry < -kRhoMax || ry > kRhoMax || rz < -kRhoMax || rz > kRhoMax) return -1;
    return (((delta + kDeltaMax) * kRhoSpan + (rx + kRhoMax)) * kRhoSpan + (ry + kRhoMax)) * kRhoSpan +
           (rz + kRhoMax);
}

// Class code of every M2L pair in CSR order (one wave per owner cell): the
// operator slot of its class (>= 0), -1 for a pair outside the dense table,
// or -2 - key for a class without a slot yet, whose key is then marked in
// `used` (read first: a read leaves the cache line shared) for the slot
// allocation; such codes are resolved through slot_of afterwards.  xcount[A]
// counts the owner's pairs outside the table.
__global__ void k_pair_classes(CellArrays c, int32_t ncell, const int32_t *__restrict__ ptr,
                               const int32_t *__restrict__ src, const int32_t *__restrict__ slot_of,
                               int32_t *__restrict__ pcode, int32_t *__restrict__ used, int32_t *__restrict__ xcount) {
    constexpr int U = 8;   // rounds of 64 pairs whose loads are issued together
    const int lane = threadIdx.x & 63;
    for (int32_t A = blockIdx.x * blockDim.x / 64 + threadIdx.x / 64; A < ncell; A += gridDim.x * blockDim.x / 64) {
        int nx = 0;
        const int4 ra = c.rec[A];
        const int la = rec_level(ra);
        const int64_t SA = (int64_t)1 << (kLevels - la);
        const int64_t ca[3] = {(2 * (int64_t)rec_ix(ra) + 1) * SA, (2 * (int64_t)rec_iy(ra) + 1) * SA,
                               (2 * (int64_t)rec_iz(ra) + 1) * SA};
        const int32_t end = ptr[A + 1];
        for (int32_t e0 = ptr[A] + lane; e0 < end; e0 += 64 * U) {
            int32_t B[U];
            int4 rb[U];
#pragma unroll
            for (int u = 0; u < U; u++) B[u] = e0 + 64 * u < end ? src[e0 + 64 * u] : -1;
#pragma unroll
            for (int u = 0; u < U; u++) rb[u] = c.rec[B[u] >= 0 ? B[u] : A];
#pragma unroll
            for (int u = 0; u < U; u++) {
                if (B[u] < 0) continue;
                const int lb = rec_level(rb[u]);
                const int64_t SB = (int64_t)1 << (kLevels - lb);
                // both centres are multiples of the smaller half-size 2^sh:
                // the division by it is an exact arithmetic shift
                const int sh = kLevels - (la > lb ? la : lb);
                const int rx = (int)((ca[0] - (2 * (int64_t)rec_ix(rb[u]) + 1) * SB) >> sh);
                const int ry = (int)((ca[1] - (2 * (int64_t)rec_iy(rb[u]) + 1) * SB) >> sh);
                const int rz = (int)((ca[2] - (2 * (int64_t)rec_iz(rb[u]) + 1) * SB) >> sh);
                const int k = dense_key(la - lb, rx, ry, rz);
                int code = -1;
                if (k >= 0) {
                    code = slot_of[k];
                    if (code < 0) {
                        code = -2 - k;
                        if (!used[k]) used[k] = 1;
                    }
                } else {
                    nx++;
                }
                pcode[e0 + 64 * u] = code;
            }
        }
#pragma unroll
        for (int d = 32; d > 0; d >>= 1) nx += __shfl_xor(nx, d, 64);
        if (lane == 0) xcount[A] = nx;
    }
}

// Marked dense keys get a slot in the operator store; the marks are
// cleared for the next build.
__global__ void k_alloc_slots(int32_t *__restrict__ used, int32_t nkeys, int32_t *__restrict__ slot_of,
                              int32_t *__restrict__ nslots, int32_t *__restrict__ new_keys) {
    for (int32_t k = blockIdx.x * blockDim.x + threadIdx.x; k < nkeys; k += gridDim.x * blockDim.x) {
        if (!used[k]) continue;
        used[k] = 0;
        if (slot_of[k] < 0) {
            int32_t s = atomicAdd(&nslots[0], 1);
            slot_of[k] = s;
            int32_t j = atomicAdd(&nslots[1], 1);
            new_keys[j] = k;
        }
    }
}

// Slots in key order: rank = exclusive scan of the marks, its total in
// rank[nkeys].
__global__ void k_alloc_slots_ordered(int32_t *__restrict__ used, int32_t nkeys, const int32_t *__restrict__ rank,
                                      int32_t *__restrict__ slot_of, int32_t *__restrict__ nslots,
                                      int32_t *__restrict__ new_keys) {
    for (int32_t k = blockIdx.x * blockDim.x + threadIdx.x; k < nkeys; k += gridDim.x * blockDim.x) {
        if (k == 0) nslots[0] = nslots[1] = rank[nkeys];
        if (!used[k]) continue;
        used[k] = 0;
        slot_of[k] = rank[k];
        new_keys[rank[k]] = k;
    }
}

// operator slot of a pair code (-1: outside the table)
__device__ inline int32_t code_slot(int32_t code, const int32_t *__restrict__ slot_of) {
    return code < -1 ? slot_of[-2 - code] : code;
}

// Build the operator fragments of each new class: one workgroup per class.
// Lane m computes column m of I_n^m (n <= 2p) in FP64; the entries are
// stored as split bf16 pieces for the mixed path's matrix cores, or (kF64)
// as FP64 for the FP64 path's.
template <bool kF64>
__global__ void __launch_bounds__(256) k_build_ops(const int32_t *__restrict__ new_keys, int32_t nnew,
                                                   const int32_t *__restrict__ slot_of, int p, int RT,
                                                   int64_t op_elems, int transposed, void *__restrict__ ops) {
    __shared__ double Ire[(2 * kMaxP + 1) * (2 * kMaxP + 2) / 2], Iim[(2 * kMaxP + 1) * (2 * kMaxP + 2) / 2];
    int32_t j = blockIdx.x;
    if (j >= nnew) return;
    int k = new_keys[j];
    int rz = k % kRhoSpan - kRhoMax;
    int t = k / kRhoSpan;
    int ry = t % kRhoSpan - kRhoMax;
    t /= kRhoSpan;
    int rx = t % kRhoSpan - kRhoMax;
    int delta = t / kRhoSpan - kDeltaMax;
    if (transposed) {
        // key of a transposed pair (owner B, partner A): the forward pair
        // A <- B has the opposite level difference and displacement, and the
        // store holds the transpose of its operator
        delta = -delta;
        rx = -rx;
        ry = -ry;
        rz = -rz;
    }
    // rho in units of the target side: (C_A - C_B) / (2 S_A) = r_int * S_min / (2 S_A)
    double sc = delta >= 0 ? 0.5 : ldexp(0.5, delta);  // S_min / S_A = 2^min(0, delta)
    double x = rx * sc, y = ry * sc, z = rz * sc;
    const int nmax = 2 * p;
    auto tri = [](int n, int m) { return n * (n + 1) / 2 + m; };
    if ((int)threadIdx.x <= nmax) {
        int m = threadIdx.x;
        double r2 = x * x + y * y + z * z, ir2 = 1.0 / r2;
        double mr = 1.0 / sqrt(r2), mi = 0.0;
        for (int q = 1; q <= m; q++) {
            double f = (2 * q - 1) * ir2;
            double nr = (mr * x - mi * y) * f, ni = (mr * y + mi * x) * f;
            mr = nr;
            mi = ni;
        }
        Ire[tri(m, m)] = mr;
        Iim[tri(m, m)] = mi;
        double pr = 0, pi = 0, cr = mr, ci = mi;
        for (int n = m + 1; n <= nmax; n++) {
            double nr, ni;
            if (n == m + 1) {
                double f = (2 * m + 1) * z * ir2;
                nr = f * cr;
                ni = f * ci;
            } else {
                double a = (2 * n - 1) * z, b = (double)((n - 1) * (n - 1) - m * m);
                nr = (a * cr - b * pr) * ir2;
                ni = (a * ci - b * pi) * ir2;
            }
            Ire[tri(n, m)] = nr;
            Iim[tri(n, m)] = ni;
            pr = cr;
            pi = ci;
            cr = nr;
            ci = ni;
        }
    }
    __syncthreads();
    const int P = ncoef(p);
    // entry (row, col) of the forward operator: output (n, m, part) and
    // input (kk, l, part) of the real layouts
    auto entry = [&](int row, int col) -> double {
        if (row >= P || col >= P) return 0.0;
        int n = 0;
        while ((n + 1) * (n + 1) <= row) n++;
        int ro = row - n * n, m = (ro + 1) / 2;
        bool out_im = ro > 0 && !(ro & 1);
        int kk = 0;
        while ((kk + 1) * (kk + 1) <= col) kk++;
        int co = col - kk * kk, l = (co + 1) / 2;
        bool in_im = co > 0 && !(co & 1);
        // I_(n+kk)^(mm) with conjugate symmetry for mm < 0
        auto Ig = [&](int mm, double &re, double &im) {
            int nn = n + kk, am = mm < 0 ? -mm : mm;
            re = Ire[tri(nn, am)];
            im = Iim[tri(nn, am)];
            if (mm < 0) {
                im = -im;
                if (am & 1) {
                    re = -re;
                    im = -im;
                }
            }
        };
        double zr, zi;
        if (l == 0) {
            Ig(m, zr, zi);
        } else {
            double ar, ai, br, bi;
            Ig(m + l, ar, ai);
            Ig(m - l, br, bi);
            double sg = (l & 1) ? -1.0 : 1.0;
            if (!in_im) {
                zr = ar + sg * br;
                zi = ai + sg * bi;
            } else {  // i * (a - sg b)
                double dr = ar - sg * br, di = ai - sg * bi;
                zr = -di;
                zi = dr;
            }
        }
        double v = out_im ? zi : zr;
        v *= ldexp(1.0, delta * kk);
        if (n & 1) v = -v;
        return v;
    };
    if (kF64) {
        // FP64 matrix-core fragments (v_mfma_f64_16x16x4f64, A operand):
        // block (s RT + r) of 64 lanes holds T[16 r + lane % 16][4 s + lane / 16]
        const int KS = (P + 3) / 4;
        double *out = static_cast<double *>(ops) + (int64_t)slot_of[k] * op_elems;
        const int total = KS * RT * 64;
        for (int f = threadIdx.x; f < total; f += blockDim.x) {
            const int lane = f & 63, r = (f >> 6) % RT, sk = (f >> 6) / RT;
            const int orow = 16 * r + (lane & 15), ocol = 4 * sk + (lane >> 4);
            out[f] = transposed ? entry(ocol, orow) : entry(orow, ocol);
        }
        return;
    }
    // Block order: block ((s RT + r) 2 + piece) of 64 lanes x 8 bf16; lane
    // holds T[r 32 + lane % 32][16 s + 8 (lane / 32) + t], t < 8, piece 0 =
    // bf16 rounding of the value, piece 1 = bf16 rounding of the remainder.
    const int NK = 2 * RT;
    uint16_t *out = static_cast<uint16_t *>(ops) + (int64_t)slot_of[k] * op_elems;
    const int total = NK * RT * 64 * 8;  // values (each written as two pieces)
    for (int f = threadIdx.x; f < total; f += blockDim.x) {
        const int t = f & 7, lane = (f >> 3) & 63, r = (f >> 9) % RT, sk = (f >> 9) / RT;
        const int orow = r * 32 + (lane & 31), ocol = 16 * sk + 8 * (lane >> 5) + t;
        const double v = transposed ? entry(ocol, orow) : entry(orow, ocol);
        const uint32_t hi = bf16_bits((float)v);
        const uint32_t lo = bf16_bits((float)(v - (double)bf16_value(hi)));
        const int64_t blk = (int64_t)(sk * RT + r) * 2;
        out[((blk * 64) + lane) * 8 + t] = (uint16_t)hi;
        out[(((blk + 1) * 64) + lane) * 8 + t] = (uint16_t)lo;
    }
}

// Sort key of every cell that has batched M2L pairs: (level, octant, spatial
// eighth of the particle order, cell).  Within a level the cells are in
// Morton order, in which the eighth never decreases, so the eighth does not
// change the order (long runs of one octant: fewer classes per group of 256
// than with the eighth above the octant, 16% fewer entries on the uniform
// and Plummer trees); it rides along in bits 32..34, where it later selects
// the XCD whose task list the group joins.
__global__ void k_target_keys(CellArrays c, int32_t ncell, int64_t n, const int32_t *__restrict__ ptr,
                              const int32_t *__restrict__ xptr, uint64_t *__restrict__ tkey,
                              int32_t *__restrict__ has) {
    for (int32_t A = blockIdx.x * blockDim.x + threadIdx.x; A < ncell; A += gridDim.x * blockDim.x) {
        int32_t nb = (ptr[A + 1] - ptr[A]) - (xptr[A + 1] - xptr[A]);
        has[A] = nb > 0;
        int oct = (c.ix[A] & 1) | ((c.iy[A] & 1) << 1) | ((c.iz[A] & 1) << 2);
        int c8 = n > 0 ? (int)(((int64_t)c.first[A] * 8) / n) : 0;
        c8 = c8 > 7 ? 7 : c8;
        tkey[A] = nb > 0 ? (((uint64_t)c.level[A] << 38) | ((uint64_t)oct << 35) | ((uint64_t)c8 << 32) | (uint32_t)A)
                         : ~0ull;
    }
}

// Group entries in three steps, each spread over kSplit workgroups per
// group:  (1) mark the classes of the group's pairs in a global bitmap,
// (2) per group, exclusive popcount prefix over its bitmap words (entry
// rank of every class), (3) write every pair's source into its entry slot.
// In (1) each wave walks the pair lists of whole targets (target slots
// split, split + kSplit, ... go to the waves of the split's workgroup in
// turn).  In (3), spread over kFillSplit workgroups per group, workgroup
// `split` owns 8 consecutive target slots: 32 bytes of every entry row.
// It places its targets' sources in an LDS tile of entry rows and writes
// the tile out row by row, absent sources included (-1), so the entry table
// needs no clearing and no scattered 4-byte writes reach memory.
constexpr int kSplit = 8;
constexpr int kGroupWaves = 4;   // waves per workgroup of a group kernel
constexpr int kFillUnroll = 4;   // rounds of 64 pairs whose loads are issued together
constexpr int kPairUnroll = 4;   // rounds of 64 pairs whose loads are issued together

// Block b of a group kernel -> (group, split).  Workgroups are dispatched
// round-robin over the 8 XCDs (XCD = b mod 8), so mapping the kSplit blocks
// of group g to b = ((g / 8) kSplit + split) 8 + g mod 8 keeps a group on one
// XCD: its entry rows are then written through a single L2, which merges the
// scattered slot writes into whole lines before they go to memory.
template <int Split = kSplit>
__device__ inline void group_split_of(int b, int *g, int *split) {
    const int i = b >> 3;
    *g = (i / Split) * 8 + (b & 7);
    *split = i % Split;
}

inline int group_blocks(int32_t ngroup, int split = kSplit) { return ((ngroup + 7) / 8) * 8 * split; }

// Calls f(slot, source, cid) for the table pairs of the wave's targets
// (cid = operator slot >= 0; source = the pair's source cell if src is
// given, else 0).
template <class F>
__device__ inline void for_group_pairs(const uint64_t *__restrict__ tsorted, int32_t ntarget, int g, int split,
                                       const int32_t *__restrict__ ptr, const int32_t *__restrict__ pcode,
                                       const int32_t *__restrict__ src, const int32_t *__restrict__ slot_of, F &&f) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int t0 = g * kGroupM2L;
    const int nt = ntarget - t0 < kGroupM2L ? ntarget - t0 : kGroupM2L;
    for (int sl = split + kSplit * w; sl < nt; sl += kSplit * kGroupWaves) {   // uniform over the wave
        const int32_t A = (int32_t)(tsorted[t0 + sl] & 0xffffffffull);
        if (A < 0) continue;   // a key without table pairs (never within ntarget)
        const int32_t end = ptr[A + 1];
        for (int32_t e0 = ptr[A] + lane; e0 < end; e0 += 64 * kPairUnroll) {
            int32_t code[kPairUnroll], sv[kPairUnroll];
#pragma unroll
            for (int u = 0; u < kPairUnroll; u++) {
                const bool in = e0 + 64 * u < end;
                code[u] = in ? pcode[e0 + 64 * u] : -1;
                sv[u] = (src && in) ? src[e0 + 64 * u] : 0;
            }
#pragma unroll
            for (int u = 0; u < kPairUnroll; u++) {
                const int32_t cid = code_slot(code[u], slot_of);
                if (cid >= 0) f(sl, sv[u], cid);
            }
        }
    }
}

__global__ void __launch_bounds__(64 * kGroupWaves) k_group_mark(const uint64_t *__restrict__ tsorted,
                                                                 int32_t ntarget, const int32_t *__restrict__ ptr,
                                                                 const int32_t *__restrict__ pcode,
                                                                 const int32_t *__restrict__ slot_of, int nwords,
                                                                 uint32_t *__restrict__ gbits) {
    extern __shared__ uint32_t lbits[];
    int g, split;
    group_split_of(blockIdx.x, &g, &split);
    if (g * kGroupM2L >= ntarget) return;
    for (int w = threadIdx.x; w < nwords; w += blockDim.x) lbits[w] = 0u;
    __syncthreads();
    for_group_pairs(tsorted, ntarget, g, split, ptr, pcode, (const int32_t *)nullptr, slot_of,
                    [&](int, int32_t, int32_t cid) {
        atomicOr(&lbits[cid >> 5], 1u << (cid & 31));
    });
    __syncthreads();
    uint32_t *bits = gbits + (int64_t)g * nwords;
    for (int w = threadIdx.x; w < nwords; w += blockDim.x)
        if (lbits[w]) atomicOr(&bits[w], lbits[w]);
}

// One workgroup per group: gwpre[g][w] = entries before word w; gcount[g]
// and the group's task count tcount[g] (its entries in chunks of `chunk`).
__global__ void __launch_bounds__(256) k_group_prefix(int nwords, const uint32_t *__restrict__ gbits,
                                                      uint32_t *__restrict__ gwpre, int32_t *__restrict__ gcount,
                                                      int chunk, int32_t *__restrict__ tcount) {
    __shared__ int32_t part[257];
    const int g = blockIdx.x;
    const uint32_t *bits = gbits + (int64_t)g * nwords;
    uint32_t *wpre = gwpre + (int64_t)g * nwords;
    const int per = (nwords + 255) / 256;
    int mine = 0;
    for (int w = threadIdx.x * per; w < (int)(threadIdx.x + 1) * per && w < nwords; w++) mine += __popc(bits[w]);
    part[threadIdx.x] = mine;
    __syncthreads();
    if (threadIdx.x == 0) {
        int run = 0;
        for (int i = 0; i < 256; i++) {
            int v = part[i];
            part[i] = run;
            run += v;
        }
        part[256] = run;
        gcount[g] = run;
        tcount[g] = (run + chunk - 1) / chunk;
    }
    __syncthreads();
    int run = part[threadIdx.x];
    for (int w = threadIdx.x * per; w < (int)(threadIdx.x + 1) * per && w < nwords; w++) {
        wpre[w] = run;
        run += __popc(bits[w]);
    }
}

// The number of targets: the sorted target keys end with the ~0 keys of
// the cells without table pairs (their sorted bits hold 31 in the level
// field, above every real level), so "key is ~0" is false then true along
// the array; one thread finds the first ~0 key by binary search (ncell if
// there is none).
__global__ void k_count_targets(const uint64_t *__restrict__ tsorted, int32_t ncell, int32_t *__restrict__ count) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    int32_t lo = 0, hi = ncell;   // the answer lies in [lo, hi]
    while (lo < hi) {
        const int32_t mid = lo + ((hi - lo) >> 1);
        if (tsorted[mid] == ~0ull) hi = mid; else lo = mid + 1;
    }
    *count = lo;
}

// Exclusive scans of the per-group entry and task counts (goff, toff; the
// totals to totals[0..1]) in one workgroup, and zeroed per-XCD task
// counters.  For at most kGroupScanMax groups.
constexpr int kGroupScanThreads = 1024, kGroupScanItems = 8;
constexpr int kGroupScanMax = kGroupScanThreads * kGroupScanItems;
__global__ void __launch_bounds__(kGroupScanThreads) k_group_scans(const int32_t *__restrict__ gcount,
                                                                   const int32_t *__restrict__ tcount, int32_t ngroup,
                                                                   int32_t *__restrict__ goff,
                                                                   int32_t *__restrict__ toff,
                                                                   int32_t *__restrict__ totals,
                                                                   int32_t *__restrict__ xcd_count) {
    __shared__ int32_t ws[2][kGroupScanThreads / 64];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int32_t b0 = threadIdx.x * kGroupScanItems;
    int va[kGroupScanItems], vb[kGroupScanItems], sa = 0, sb = 0;
#pragma unroll
    for (int i = 0; i < kGroupScanItems; i++) {
        va[i] = b0 + i < ngroup ? gcount[b0 + i] : 0;
        vb[i] = b0 + i < ngroup ? tcount[b0 + i] : 0;
        sa += va[i];
        sb += vb[i];
    }
    int ia = sa, ib = sb;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const int ta = __shfl_up(ia, d, 64), tb = __shfl_up(ib, d, 64);
        if (lane >= d) {
            ia += ta;
            ib += tb;
        }
    }
    if (lane == 63) {
        ws[0][w] = ia;
        ws[1][w] = ib;
    }
    __syncthreads();
    int pa = 0, pb = 0, ta = 0, tb = 0;
#pragma unroll
    for (int i = 0; i < kGroupScanThreads / 64; i++) {
        if (i < w) {
            pa += ws[0][i];
            pb += ws[1][i];
        }
        ta += ws[0][i];
        tb += ws[1][i];
    }
    pa += ia - sa;
    pb += ib - sb;
#pragma unroll
    for (int i = 0; i < kGroupScanItems; i++)
        if (b0 + i < ngroup) {
            goff[b0 + i] = pa;
            toff[b0 + i] = pb;
            pa += va[i];
            pb += vb[i];
        }
    if (threadIdx.x == 0) {
        totals[0] = ta;
        totals[1] = tb;
    }
    if (threadIdx.x < 8) xcd_count[threadIdx.x] = 0;
}

constexpr int kFillSplit = 32;                           // workgroups per group in the fill (16: 8% slower)
constexpr int kSlotsPerSplit = kGroupM2L / kFillSplit;   // 8 slots = 32 bytes of an entry row
constexpr int kTileStride = kSlotsPerSplit + 1;      // padded LDS row: rows fall in different banks
constexpr int kFillEntries = 384;                    // entry rows per LDS tile
constexpr size_t kFillTileBytes = (size_t)kFillEntries * kTileStride * 4;

// kLds: the group's class bitmap and word prefixes are staged in LDS (after
// the tile, 2 nwords words) instead of read from global memory per pair.
template <bool kLds>
__global__ void __launch_bounds__(64 * kGroupWaves) k_group_fill(
    const uint64_t *__restrict__ tsorted, int32_t ntarget, const int32_t *__restrict__ ptr,
    const int32_t *__restrict__ src, const int32_t *__restrict__ pcode, const int32_t *__restrict__ slot_of,
    int nwords, const uint32_t *__restrict__ gbits, const uint32_t *__restrict__ gwpre,
    const int32_t *__restrict__ goff, const int32_t *__restrict__ gcount, int32_t *__restrict__ ecls,
    int32_t *__restrict__ esrc, int32_t *__restrict__ gtarget) {
    static_assert(kSlotsPerSplit % kGroupWaves == 0 && 64 * kGroupWaves % kSlotsPerSplit == 0, "tile shape");
    extern __shared__ uint32_t dyn[];
    int32_t *tile = reinterpret_cast<int32_t *>(dyn);
    uint32_t *ltab = dyn + kFillEntries * kTileStride;
    int g, split;
    group_split_of<kFillSplit>(blockIdx.x, &g, &split);
    const int t0 = g * kGroupM2L;
    if (t0 >= ntarget) return;
    const int nt = ntarget - t0 < kGroupM2L ? ntarget - t0 : kGroupM2L;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const uint32_t *gb = gbits + (int64_t)g * nwords;
    const uint32_t *gw = gwpre + (int64_t)g * nwords;
    if (kLds) {
        for (int i = threadIdx.x; i < nwords; i += blockDim.x) {
            ltab[i] = gb[i];
            ltab[nwords + i] = gw[i];
        }
        __syncthreads();
    }
    const uint32_t *bits = kLds ? ltab : gb;
    const uint32_t *wpre = kLds ? ltab + nwords : gw;
    const int32_t base = goff[g], nent = gcount[g];
    if (split == 0) {
        for (int i = threadIdx.x; i < kGroupM2L; i += blockDim.x)
            gtarget[(int64_t)g * kGroupM2L + i] = i < nt ? (int32_t)(tsorted[t0 + i] & 0xffffffffull) : -1;
        for (int i = threadIdx.x; i < nwords; i += blockDim.x) {
            uint32_t b = bits[i];
            int32_t ent = base + (int32_t)wpre[i];
            while (b) {
                int bit = __ffs(b) - 1;
                ecls[ent++] = i * 32 + bit;
                b &= b - 1;
            }
        }
    }
    const int s0 = split * kSlotsPerSplit;
    for (int ec = 0; ec < nent; ec += kFillEntries) {   // uniform over the workgroup
        const int ne = nent - ec < kFillEntries ? nent - ec : kFillEntries;
        for (int i = threadIdx.x; i < ne * kTileStride; i += blockDim.x) tile[i] = -1;
        __syncthreads();
        for (int sl = w; sl < kSlotsPerSplit && s0 + sl < nt; sl += kGroupWaves) {   // uniform over the wave
            const int32_t A = (int32_t)(tsorted[t0 + s0 + sl] & 0xffffffffull);
            if (A < 0) continue;   // a key without table pairs (never within ntarget)
            const int32_t end = ptr[A + 1];
            for (int32_t e0 = ptr[A] + lane; e0 < end; e0 += 64 * kFillUnroll) {
                int32_t code[kFillUnroll], sv[kFillUnroll];
#pragma unroll
                for (int u = 0; u < kFillUnroll; u++) {
                    const bool in = e0 + 64 * u < end;
                    code[u] = in ? pcode[e0 + 64 * u] : -1;
                    sv[u] = in ? src[e0 + 64 * u] : 0;
                }
#pragma unroll
                for (int u = 0; u < kFillUnroll; u++) {
                    const int32_t cid = code_slot(code[u], slot_of);
                    if (cid < 0) continue;
                    const uint32_t wv = bits[cid >> 5] & ((1u << (cid & 31)) - 1u);
                    const int r = (int)wpre[cid >> 5] + __popc(wv) - ec;
                    if (r >= 0 && r < ne) tile[r * kTileStride + sl] = sv[u];
                }
            }
        }
        __syncthreads();
        for (int i = threadIdx.x; i < ne * kSlotsPerSplit; i += blockDim.x) {
            const int r = i / kSlotsPerSplit, c = i % kSlotsPerSplit;
            esrc[(int64_t)(base + ec + r) * kGroupM2L + s0 + c] = tile[r * kTileStride + c];
        }
        __syncthreads();
    }
}

// Tasks: each group's entries split into chunks of `chunk`.
// Tasks of a group: its entries cut into chunks.  Each task also gets a
// sort key (XCD of the group, chunk index, task) so that every XCD runs its
// own groups chunk by chunk: concurrent workgroups then share class
// operators in that XCD's L2.
__global__ void k_make_tasks(const int32_t *__restrict__ gcount, const int32_t *__restrict__ goff, int32_t ngroup,
                             int chunk, int jbits, const int32_t *__restrict__ toff,
                             const uint64_t *__restrict__ tsorted, int4 *__restrict__ tasks,
                             uint64_t *__restrict__ tkeys, uint32_t *__restrict__ tidx,
                             int32_t *__restrict__ xcd_count) {
    for (int32_t g = blockIdx.x * blockDim.x + threadIdx.x; g < ngroup; g += gridDim.x * blockDim.x) {
        int32_t n = gcount[g], t = toff[g];
        int xcd = (int)((tsorted[(int64_t)g * kGroupM2L] >> 32) & 7ull);   // eighth of the first target
        for (int32_t e = 0, j = 0; e < n; e += chunk, j++, t++) {
            // .w: the task's slot in the partial-locals buffer, group-major
            // (the group's tasks are toff[g] .. toff[g] + tcount[g] - 1)
            tasks[t] = make_int4(g, goff[g] + e, goff[g] + (e + chunk < n ? e + chunk : n), t);
            // t is already in (group, chunk) order: a stable sort on the
            // (XCD, chunk index) bits above it yields (XCD, chunk, task)
            tkeys[t] = ((uint64_t)xcd << (32 + jbits)) | ((uint64_t)j << 32) | (uint32_t)t;
            tidx[t] = (uint32_t)t;
            atomicAdd(&xcd_count[xcd], 1);
        }
    }
}

__global__ void k_permute_tasks(const uint32_t *__restrict__ order, int32_t ntask, const int4 *__restrict__ in,
                                int4 *__restrict__ out) {
    for (int32_t t = blockIdx.x * blockDim.x + threadIdx.x; t < ntask; t += gridDim.x * blockDim.x) out[t] = in[order[t]];
}

// The pairs outside the class table, per owner in list order: one wave per
// owner, a ballot and prefix count place each flagged pair at xptr[A] + rank.
__global__ void k_compact_extra(const int32_t *__restrict__ ptr, int32_t ncell, const int32_t *__restrict__ src,
                                const int32_t *__restrict__ pcode, const int32_t *__restrict__ xptr,
                                int32_t *__restrict__ xsrc) {
    const int lane = threadIdx.x & 63;
    for (int32_t A = blockIdx.x * blockDim.x / 64 + threadIdx.x / 64; A < ncell; A += gridDim.x * blockDim.x / 64) {
        if (xptr[A + 1] == xptr[A]) continue;
        int32_t base = xptr[A];
        for (int32_t e0 = ptr[A]; e0 < ptr[A + 1]; e0 += 64) {
            const int32_t e = e0 + lane;
            const bool x = e < ptr[A + 1] && pcode[e] == -1;
            const unsigned long long m = __ballot(x);
            if (x) xsrc[base + __popcll(m & ((1ull << lane) - 1ull))] = src[e];
            base += __popcll(m);
        }
    }
}

}  // namespace

void m2l_pair_codes(CellArrays c, int32_t ncell, const int32_t *ptr, const int32_t *src, const int32_t *slot_of,
                    int32_t *pcode, int32_t *used, int32_t *xcount, hipStream_t s) {
    hipLaunchKernelGGL(k_pair_classes, dim3(grid_for((int64_t)ncell * 64, 256, 16384)), dim3(256), 0, s, c, ncell, ptr,
                       src, slot_of, pcode, used, xcount);
    FMM_LAUNCH_CHECK();
}

void m2l_alloc_slots(int32_t *used, int32_t *slot_of, int32_t *nslots, int32_t *new_keys, hipStream_t s) {
    hipLaunchKernelGGL(k_alloc_slots, dim3(grid_for(kDenseKeys, 256, 4096)), dim3(256), 0, s, used, kDenseKeys, slot_of,
                       nslots, new_keys);
    FMM_LAUNCH_CHECK();
}

void m2l_alloc_slots_ordered(int32_t *used, int32_t *slot_of, int32_t *nslots, int32_t *new_keys, int32_t *rank,
                             int32_t *tmp, hipStream_t s) {
    exclusive_scan_oop(used, rank, kDenseKeys, rank + kDenseKeys, tmp, s);
    hipLaunchKernelGGL(k_alloc_slots_ordered, dim3(grid_for(kDenseKeys, 256, 4096)), dim3(256), 0, s, used, kDenseKeys,
                       rank, slot_of, nslots, new_keys);
    FMM_LAUNCH_CHECK();
}

void m2l_build_ops(const int32_t *new_keys, int32_t nnew, const int32_t *slot_of, int p, int RT, int64_t op_elems,
                   bool transposed, uint16_t *ops, hipStream_t s) {
    if (nnew <= 0) return;
    hipLaunchKernelGGL(k_build_ops<false>, dim3(nnew), dim3(256), 0, s, new_keys, nnew, slot_of, p, RT, op_elems,
                       transposed ? 1 : 0, (void *)ops);
    FMM_LAUNCH_CHECK();
}

void m2l_build_ops_f64(const int32_t *new_keys, int32_t nnew, const int32_t *slot_of, int p, int64_t op_elems,
                       bool transposed, double *ops, hipStream_t s) {
    if (nnew <= 0) return;
    hipLaunchKernelGGL(k_build_ops<true>, dim3(nnew), dim3(256), 0, s, new_keys, nnew, slot_of, p,
                       (ncoef(p) + 15) / 16, op_elems, transposed ? 1 : 0, (void *)ops);
    FMM_LAUNCH_CHECK();
}

void m2l_target_keys(CellArrays c, int32_t ncell, int64_t n, const int32_t *ptr, const int32_t *xptr, uint64_t *tkey,
                     int32_t *has, hipStream_t s) {
    hipLaunchKernelGGL(k_target_keys, dim3(grid_for(ncell, 256, 4096)), dim3(256), 0, s, c, ncell, n, ptr, xptr, tkey,
                       has);
    FMM_LAUNCH_CHECK();
}

void m2l_count_targets(const uint64_t *tsorted, int32_t ncell, int32_t *count, hipStream_t s) {
    if (ncell <= 0) {
        fill_zero(count, sizeof(int32_t), s);
        return;
    }
    hipLaunchKernelGGL(k_count_targets, dim3(1), dim3(64), 0, s, tsorted, ncell, count);
    FMM_LAUNCH_CHECK();
}

void m2l_group_scans(const int32_t *gcount, const int32_t *tcount, int32_t ngroup, int32_t *goff, int32_t *toff,
                     int32_t *totals, int32_t *xcd_count, int32_t *tmp, hipStream_t s) {
    if (ngroup <= kGroupScanMax) {
        hipLaunchKernelGGL(k_group_scans, dim3(1), dim3(kGroupScanThreads), 0, s, gcount, tcount, ngroup, goff, toff,
                           totals, xcd_count);
        FMM_LAUNCH_CHECK();
        return;
    }
    exclusive_scan_oop(gcount, goff, ngroup, totals, tmp, s);
    exclusive_scan_oop(tcount, toff, ngroup, totals + 1, tmp, s);
    fill_zero(xcd_count, 8 * sizeof(int32_t), s);
}

void m2l_group_count(const uint64_t *tsorted, int32_t ntarget, const int32_t *ptr, const int32_t *pcode,
                     const int32_t *slot_of, int32_t nslot, uint32_t *gbits, uint32_t *gwpre, int32_t *gcount,
                     int chunk, int32_t *tcount, hipStream_t s) {
    const int32_t ngroup = (ntarget + kGroupM2L - 1) / kGroupM2L;
    if (ngroup <= 0) return;
    const int nwords = (nslot + 31) / 32;
    FMM_HIP_CHECK(hipMemsetAsync(gbits, 0, (size_t)ngroup * nwords * 4, s));
    if ((size_t)nwords * 4 > 48 * 1024) throw std::runtime_error("too many M2L classes for the group builder");
    hipLaunchKernelGGL(k_group_mark, dim3(group_blocks(ngroup)), dim3(256), (size_t)nwords * 4, s, tsorted, ntarget,
                       ptr, pcode, slot_of, nwords, gbits);
    FMM_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_group_prefix, dim3(ngroup), dim3(256), 0, s, nwords, gbits, gwpre, gcount, chunk, tcount);
    FMM_LAUNCH_CHECK();
}

void m2l_group_fill(const uint64_t *tsorted, int32_t ntarget, const int32_t *ptr, const int32_t *src,
                    const int32_t *pcode, const int32_t *slot_of, int32_t nslot, const uint32_t *gbits,
                    const uint32_t *gwpre, const int32_t *goff, const int32_t *gcount, int32_t *ecls, int32_t *esrc,
                    int32_t *gtarget, hipStream_t s) {
    const int32_t ngroup = (ntarget + kGroupM2L - 1) / kGroupM2L;
    if (ngroup <= 0) return;
    const int nwords = (nslot + 31) / 32;
    const size_t tab = (size_t)2 * nwords * 4;
    if (kFillTileBytes + tab <= 65536)
        hipLaunchKernelGGL(k_group_fill<true>, dim3(group_blocks(ngroup, kFillSplit)), dim3(64 * kGroupWaves), kFillTileBytes + tab,
                           s, tsorted, ntarget, ptr, src, pcode, slot_of, nwords, gbits, gwpre, goff, gcount, ecls,
                           esrc, gtarget);
    else
        hipLaunchKernelGGL(k_group_fill<false>, dim3(group_blocks(ngroup, kFillSplit)), dim3(64 * kGroupWaves), kFillTileBytes, s,
                           tsorted, ntarget, ptr, src, pcode, slot_of, nwords, gbits, gwpre, goff, gcount, ecls, esrc,
                           gtarget);
    FMM_LAUNCH_CHECK();
}

void m2l_make_tasks(const int32_t *gcount, const int32_t *goff, int32_t ngroup, int chunk, int32_t max_entries,
                    const int32_t *toff,
                    const uint64_t *tsorted, int32_t ntask, int4 *tasks, int4 *tasks_alt, uint64_t *tkeys,
                    uint64_t *tkeys_alt, uint32_t *tidx, uint32_t *tidx_alt, int32_t *xcd_count, int32_t *tmp,
                    hipStream_t s) {
    if (ngroup <= 0 || ntask <= 0) return;   // xcd_count was zeroed by m2l_group_scans
    int jbits = 1;
    while ((1 << jbits) <= max_entries / chunk + 1) jbits++;
    hipLaunchKernelGGL(k_make_tasks, dim3(grid_for(ngroup, 256, 4096)), dim3(256), 0, s, gcount, goff, ngroup, chunk,
                       jbits, toff, tsorted, tasks_alt, tkeys, tidx, xcd_count);
    FMM_LAUNCH_CHECK();
    bool in_alt = false;
    radix_sort_u64(tkeys, tidx, tkeys_alt, tidx_alt, ntask, 32, 32 + jbits + 3, tmp, s, &in_alt);
    hipLaunchKernelGGL(k_permute_tasks, dim3(grid_for(ntask, 256, 4096)), dim3(256), 0, s, in_alt ? tidx_alt : tidx,
                       ntask, tasks_alt, tasks);
    FMM_LAUNCH_CHECK();
}

void m2l_extra(const int32_t *ptr, int32_t ncell, const int32_t *src, const int32_t *pcode, const int32_t *xptr,
               int32_t *xsrc, hipStream_t s) {
    if (ncell <= 0) return;
    hipLaunchKernelGGL(k_compact_extra, dim3(grid_for((int64_t)ncell * 64, 256, 16384)), dim3(256), 0, s, ptr, ncell, src,
                       pcode, xptr, xsrc);
    FMM_LAUNCH_CHECK();
}


}  // namespace fmm
