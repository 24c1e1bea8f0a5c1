// Device-wide exclusive scan and stable LSD radix sort (keys of the Morton
// octree, Sec. 2.2, and of the interaction-pair lists).
//
// Radix sort: 8-bit digits; per pass three launches -- per-tile digit
// histograms, a scan of each digit's row of the (digit-major, tile-minor)
// count table with the row totals, and a stable scatter that scans the 256
// digit totals itself.  Inside a tile each wave64 ranks its keys with
// ballot-based peer masks (lanes holding the same digit), so ranks follow the
// input order and the sort is stable.
#include "common.h"

#include <algorithm>
#include <cstring>

namespace fmm {

namespace {

constexpr int kScanThreads = 256;
constexpr int kScanItems = 8;
constexpr int kScanTile = kScanThreads * kScanItems;

__device__ inline int wave_inclusive_scan(int v) {
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        int o = __shfl_up(v, d, 64);
        if (lane >= d) v += o;
    }
    return v;
}

// Exclusive scan of one value per thread across a block of kScanThreads;
// returns the exclusive prefix and writes the block total to *total.
__device__ inline int block_exclusive_scan(int v, int *total) {
    __shared__ int wsum[kScanThreads / 64];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    int inc = wave_inclusive_scan(v);
    if (lane == 63) wsum[w] = inc;
    __syncthreads();
    int base = 0, tot = 0;
#pragma unroll
    for (int i = 0; i < kScanThreads / 64; i++) {
        if (i < w) base += wsum[i];
        tot += wsum[i];
    }
    __syncthreads();
    *total = tot;
    return base + inc - v;
}

// Small inputs (n <= kSmallScan): one workgroup of 1024 threads, 8 items each.
constexpr int kSmallThreads = 1024;
constexpr int kSmallScan = kSmallThreads * kScanItems;

__global__ void __launch_bounds__(kSmallThreads) k_scan_small(const int32_t *__restrict__ in, int32_t *__restrict__ out,
                                                              int64_t n, int32_t *__restrict__ total) {
    __shared__ int wsum[kSmallThreads / 64];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    int64_t base = (int64_t)threadIdx.x * kScanItems;
    int v[kScanItems];
    int s = 0;
#pragma unroll
    for (int i = 0; i < kScanItems; i++) {
        v[i] = base + i < n ? in[base + i] : 0;
        s += v[i];
    }
    int inc = wave_inclusive_scan(s);
    if (lane == 63) wsum[w] = inc;
    __syncthreads();
    int pre = 0, tot = 0;
    for (int i = 0; i < kSmallThreads / 64; i++) {
        if (i < w) pre += wsum[i];
        tot += wsum[i];
    }
    pre += inc - s;
#pragma unroll
    for (int i = 0; i < kScanItems; i++) {
        if (base + i < n) out[base + i] = pre;
        pre += v[i];
    }
    if (threadIdx.x == 0 && total) *total = tot;
}

__global__ void k_scan_reduce(const int32_t *__restrict__ data, int64_t n, int32_t *__restrict__ sums) {
    int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    int s = 0;
#pragma unroll
    for (int i = 0; i < kScanItems; i++)
        if (base + i < n) s += data[base + i];
    int tot;
    block_exclusive_scan(s, &tot);
    if (threadIdx.x == 0) sums[blockIdx.x] = tot;
}

// Single block, 256 threads: exclusive scan of nb block sums in chunks.
__global__ void k_scan_top(int32_t *__restrict__ sums, int64_t nb, int32_t *__restrict__ total) {
    int carry = 0;
    for (int64_t c = 0; c < nb; c += kScanTile) {
        int64_t base = c + (int64_t)threadIdx.x * kScanItems;
        int v[kScanItems];
        int s = 0;
#pragma unroll
        for (int i = 0; i < kScanItems; i++) {
            v[i] = base + i < nb ? sums[base + i] : 0;
            s += v[i];
        }
        int tot;
        int pre = block_exclusive_scan(s, &tot) + carry;
#pragma unroll
        for (int i = 0; i < kScanItems; i++) {
            if (base + i < nb) sums[base + i] = pre;
            pre += v[i];
        }
        carry += tot;
        __syncthreads();
    }
    if (threadIdx.x == 0 && total) *total = carry;
}

__global__ void k_scan_down(const int32_t *__restrict__ in, int32_t *__restrict__ out, int64_t n,
                            const int32_t *__restrict__ sums) {
    int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    int v[kScanItems];
    int s = 0;
#pragma unroll
    for (int i = 0; i < kScanItems; i++) {
        v[i] = base + i < n ? in[base + i] : 0;
        s += v[i];
    }
    int tot;
    int pre = block_exclusive_scan(s, &tot) + sums[blockIdx.x];
#pragma unroll
    for (int i = 0; i < kScanItems; i++) {
        if (base + i < n) out[base + i] = pre;
        pre += v[i];
    }
}

// ---------------------------------------------------------------- radix sort

constexpr int kRsThreads = 256;
constexpr int kRsWaves = kRsThreads / 64;
constexpr int kRsItems = 16;   // keys per thread (tiles of 32 keys per thread were slower)
constexpr int kRsTile = kRsThreads * kRsItems;

// Tile of a workgroup.  Workgroups are dealt to the 8 XCDs in turn, so this
// gives each XCD a contiguous run of tiles: the runs of one digit that
// neighbouring tiles write then meet in one L2.
__device__ inline int rs_tile(int b, int nblocks) {
    const int q = nblocks >> 3, r = nblocks & 7, x = b & 7;
    return x * q + (x < r ? x : r) + (b >> 3);
}

// Per-tile digit counts, digit-major: counts[d * nblocks + tile].
template <class K, int Items>
__global__ void __launch_bounds__(kRsThreads) k_rs_hist(const K *__restrict__ kin, int64_t n, int shift,
                                                        int nbits, int32_t *__restrict__ counts, int nblocks) {
    __shared__ int hist[256];
    hist[threadIdx.x] = 0;
    __syncthreads();
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int mask = (1 << nbits) - 1;
    const int t = rs_tile(blockIdx.x, nblocks);
    const int64_t base = (int64_t)t * (kRsThreads * Items) + (int64_t)w * (64 * Items) + lane;
    int dig[Items];
#pragma unroll
    for (int it = 0; it < Items; it++) {
        const int64_t i = base + it * 64;
        dig[it] = i < n ? (int)((kin[i] >> shift) & (K)mask) : -1;
    }
#pragma unroll
    for (int it = 0; it < Items; it++)
        if (dig[it] >= 0) atomicAdd(&hist[dig[it]], 1);
    __syncthreads();
    counts[(int64_t)threadIdx.x * nblocks + t] = hist[threadIdx.x];
}

// Workgroup d: exclusive scan of digit d's row of the count table (the
// tile-order start of each tile's run within digit d) and the row total.
__global__ void __launch_bounds__(kScanThreads) k_rs_rowscan(int32_t *__restrict__ counts, int nblocks,
                                                             int32_t *__restrict__ totals) {
    int32_t *row = counts + (int64_t)blockIdx.x * nblocks;
    int carry = 0;
    for (int c = 0; c < nblocks; c += kScanTile) {
        const int b0 = c + threadIdx.x * kScanItems;
        int v[kScanItems];
        int sum = 0;
#pragma unroll
        for (int i = 0; i < kScanItems; i++) {
            v[i] = b0 + i < nblocks ? row[b0 + i] : 0;
            sum += v[i];
        }
        int tot;
        int pre = block_exclusive_scan(sum, &tot) + carry;
#pragma unroll
        for (int i = 0; i < kScanItems; i++) {
            if (b0 + i < nblocks) row[b0 + i] = pre;
            pre += v[i];
        }
        carry += tot;
    }
    if (threadIdx.x == 0) totals[blockIdx.x] = carry;
}

// Scatter of one pass.  Each block ranks its tile stably (per wave with
// ballots over the digit bits, then across the waves), places the tile in
// LDS in digit order, and writes it out in that order: consecutive threads
// then write consecutive addresses of one digit run instead of up to 64
// different lines per store.  A digit's global start is the exclusive scan
// of the digit totals (done here, per block) plus the tile's row prefix.
// kVals: values travel with the keys (without them the tile's value
// staging is left out, which leaves LDS for more workgroups per CU).
template <class K, bool kVals, int Items>
__global__ void __launch_bounds__(kRsThreads) k_rs_scatter(const K *__restrict__ kin, const uint32_t *__restrict__ vin,
                                                           K *__restrict__ kout, uint32_t *__restrict__ vout, int64_t n,
                                                           int shift, int nbits, const int32_t *__restrict__ offs,
                                                           const int32_t *__restrict__ totals, int nblocks) {
    constexpr int kTile = kRsThreads * Items;
    __shared__ int wcount[kRsWaves][256];
    __shared__ int wbase[kRsWaves][256];
    __shared__ int lstart[257];
    __shared__ int gbase[256];
    __shared__ int wsum[kRsWaves];
    __shared__ int wtot[kRsWaves];
    __shared__ K skey[kTile];
    __shared__ uint32_t sval[kVals ? kTile : 1];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int mask = (1 << nbits) - 1;
    for (int i = threadIdx.x; i < kRsWaves * 256; i += kRsThreads) (&wcount[0][0])[i] = 0;
    __syncthreads();
    const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    const int t = rs_tile(blockIdx.x, nblocks);
    const int64_t base = (int64_t)t * kTile + (int64_t)w * (64 * Items) + lane;
    K key[Items];
    uint32_t val[Items];
    int rank[Items];
#pragma unroll
    for (int it = 0; it < Items; it++) {
        int64_t i = base + it * 64;
        bool valid = i < n;
        key[it] = valid ? kin[i] : (K)0;
        val[it] = (kVals && valid) ? vin[i] : 0u;
    }
#pragma unroll
    for (int it = 0; it < Items; it++) {
        bool valid = base + it * 64 < n;
        int d = (int)((key[it] >> shift) & (K)mask);
        uint64_t peers = __ballot(valid);
        for (int b = 0; b < nbits; b++) {
            uint64_t m = __ballot((d >> b) & 1);
            peers &= ((d >> b) & 1) ? m : ~m;
        }
        int r = __popcll(peers & lt_mask);
        int cnt = __popcll(peers);
        int prior = valid ? wcount[w][d] : 0;
        if (valid && r == 0) wcount[w][d] = prior + cnt;
        rank[it] = prior + r;
    }
    __syncthreads();
    {
        // thread d: block count of digit d, wave offsets within the digit,
        // then exclusive scans over the 256 digits of the block counts
        // (block-local starts) and of the digit totals (global starts)
        const int d = threadIdx.x;
        int run = 0;
#pragma unroll
        for (int ww = 0; ww < kRsWaves; ww++) {
            wbase[ww][d] = run;
            run += wcount[ww][d];
        }
        const int tot = totals[d];
        int inc = run, tinc = tot;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            int a = __shfl_up(inc, o, 64), b = __shfl_up(tinc, o, 64);
            if (lane >= o) {
                inc += a;
                tinc += b;
            }
        }
        if (lane == 63) {
            wsum[w] = inc;
            wtot[w] = tinc;
        }
        const int row = offs[(int64_t)d * nblocks + t];
        __syncthreads();
        int before = 0, tbefore = 0;
        for (int ww = 0; ww < w; ww++) {
            before += wsum[ww];
            tbefore += wtot[ww];
        }
        lstart[d] = before + inc - run;
        gbase[d] = tbefore + tinc - tot + row;
        if (d == 255) lstart[256] = before + inc;
    }
    __syncthreads();
#pragma unroll
    for (int it = 0; it < Items; it++) {
        int64_t i = base + it * 64;
        if (i < n) {
            int d = (int)((key[it] >> shift) & (K)mask);
            int lp = lstart[d] + wbase[w][d] + rank[it];
            skey[lp] = key[it];
            if (kVals) sval[lp] = val[it];
        }
    }
    __syncthreads();
    const int tile_n = lstart[256];
    for (int lp = threadIdx.x; lp < tile_n; lp += kRsThreads) {
        const K k = skey[lp];
        const int d = (int)((k >> shift) & (K)mask);
        const int pos = gbase[d] + (lp - lstart[d]);
        kout[pos] = k;
        if (kVals) vout[pos] = sval[lp];
    }
}

template <class K, bool kVals>
void radix_passes(K *kin, uint32_t *vin, K *kalt, uint32_t *valt, int64_t n, int bit_lo, int bit_hi, int32_t *d_tmp,
                  hipStream_t s, bool *in_alt) {
    constexpr int Items = kRsItems;
    const int nblocks = (int)((n + kRsTile - 1) / kRsTile);
    int32_t *totals = d_tmp;
    int32_t *counts = d_tmp + 256;
    K *ka = kin, *kb = kalt;
    uint32_t *va = vin, *vb = kVals ? valt : nullptr;
    int passes = 0;
    for (int shift = bit_lo; shift < bit_hi; shift += 8) {
        int nbits = bit_hi - shift < 8 ? bit_hi - shift : 8;
        hipLaunchKernelGGL((k_rs_hist<K, Items>), dim3(nblocks), dim3(kRsThreads), 0, s, ka, n, shift, nbits, counts,
                           nblocks);
        FMM_LAUNCH_CHECK();
        hipLaunchKernelGGL(k_rs_rowscan, dim3(256), dim3(kScanThreads), 0, s, counts, nblocks, totals);
        FMM_LAUNCH_CHECK();
        hipLaunchKernelGGL((k_rs_scatter<K, kVals, Items>), dim3(nblocks), dim3(kRsThreads), 0, s, ka, va, kb, vb, n,
                           shift, nbits, counts, totals, nblocks);
        FMM_LAUNCH_CHECK();
        K *tk = ka;
        ka = kb;
        kb = tk;
        uint32_t *tv = va;
        va = vb;
        vb = tv;
        passes++;
    }
    if (in_alt) {
        *in_alt = (passes & 1) != 0;
    } else if (passes & 1) {
        FMM_HIP_CHECK(hipMemcpyAsync(kin, ka, n * sizeof(K), hipMemcpyDeviceToDevice, s));
        if (kVals) FMM_HIP_CHECK(hipMemcpyAsync(vin, va, n * sizeof(uint32_t), hipMemcpyDeviceToDevice, s));
    }
}

template <class K>
void radix_sort_impl(K *kin, uint32_t *vin, K *kalt, uint32_t *valt, int64_t n, int bit_lo, int bit_hi,
                     int32_t *d_tmp, hipStream_t s, bool *in_alt) {
    if (in_alt) *in_alt = false;
    if (n <= 1 || bit_hi <= bit_lo) return;
    if (vin)
        radix_passes<K, true>(kin, vin, kalt, valt, n, bit_lo, bit_hi, d_tmp, s, in_alt);
    else
        radix_passes<K, false>(kin, vin, kalt, valt, n, bit_lo, bit_hi, d_tmp, s, in_alt);
}

}  // namespace

namespace {
// One thread: the values, then a system-scope fence and the flag.
__global__ void k_host_read(const int32_t *__restrict__ src, int n, int32_t *dst, int32_t seq) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    for (int i = 0; i < n; i++) dst[16 + i] = src[i];
    __threadfence_system();
    __hip_atomic_store(&dst[0], seq, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
}

__global__ void k_fill_zero(uint32_t *__restrict__ p, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0u;
}
}  // namespace

void HostReader::init() {
    if (h) return;
    void *ph = nullptr;
    if (hipHostMalloc(&ph, (16 + kHostReadMax) * sizeof(int32_t), hipHostMallocMapped | hipHostMallocCoherent) !=
        hipSuccess) {
        (void)hipGetLastError();
        return;
    }
    void *pd = nullptr;
    if (hipHostGetDevicePointer(&pd, ph, 0) != hipSuccess) {
        (void)hipGetLastError();
        (void)hipHostFree(ph);
        return;
    }
    h = static_cast<int32_t *>(ph);
    d = static_cast<int32_t *>(pd);
    __atomic_store_n(&h[0], 0, __ATOMIC_RELEASE);
    seq = 0;
}

void HostReader::release() {
    if (h) (void)hipHostFree(h);
    h = d = nullptr;
}

void HostReader::read(void *host, const void *dev, size_t bytes, hipStream_t s) {
    begin(dev, bytes, s);
    end(host, s);
}

void HostReader::begin(const void *dev, size_t bytes, hipStream_t s) {
    pend_dev = dev;
    pend_bytes = bytes;
    pend_fallback = !h || bytes > kHostReadMax * sizeof(int32_t) || (bytes & 3);
    if (pend_fallback) return;   // copied synchronously by end()
    seq = seq == 0x7fffffff ? 1 : seq + 1;
    hipLaunchKernelGGL(k_host_read, dim3(1), dim3(64), 0, s, (const int32_t *)dev, (int)(bytes / 4), d, seq);
    FMM_LAUNCH_CHECK();
}

void HostReader::end(void *host, hipStream_t s) {
    const size_t bytes = pend_bytes;
    if (pend_fallback) {
        FMM_HIP_CHECK(hipMemcpyAsync(host, pend_dev, bytes, hipMemcpyDeviceToHost, s));
        FMM_HIP_CHECK(hipStreamSynchronize(s));
        return;
    }
    for (uint64_t it = 0;; it++) {
        if (__atomic_load_n(&h[0], __ATOMIC_ACQUIRE) == seq) break;
        if ((it & 255) == 255) {
            hipError_t e = hipStreamQuery(s);
            if (e == hipSuccess) {  // the stream drained: the flag is visible by now
                if (__atomic_load_n(&h[0], __ATOMIC_ACQUIRE) == seq) break;
                throw HipError{hipErrorUnknown, "host read: flag missing after the stream drained"};
            }
            if (e != hipErrorNotReady) throw HipError{e, "host read"};
        }
        __builtin_ia32_pause();
    }
    std::memcpy(host, h + 16, bytes);
}

void fill_zero(void *ptr, size_t bytes, hipStream_t s) {
    const int64_t n = (int64_t)(bytes / 4);
    if (n == 0) return;
    hipLaunchKernelGGL(k_fill_zero, dim3(grid_for(n, 256, 16384)), dim3(256), 0, s, (uint32_t *)ptr, n);
    FMM_LAUNCH_CHECK();
}

size_t scan_tmp_elems(int64_t n) {
    int64_t nb = (n + kScanTile - 1) / kScanTile;
    return (size_t)(nb + 1);
}

void exclusive_scan_i32(int32_t *d_data, int64_t n, int32_t *d_total, int32_t *d_tmp, hipStream_t s) {
    exclusive_scan_oop(d_data, d_data, n, d_total, d_tmp, s);
}

void exclusive_scan_oop(const int32_t *d_in, int32_t *d_out, int64_t n, int32_t *d_total, int32_t *d_tmp,
                        hipStream_t s) {
    if (n <= 0) {
        if (d_total) FMM_HIP_CHECK(hipMemsetAsync(d_total, 0, sizeof(int32_t), s));
        return;
    }
    if (n <= kSmallScan) {
        hipLaunchKernelGGL(k_scan_small, dim3(1), dim3(kSmallThreads), 0, s, d_in, d_out, n, d_total);
        FMM_LAUNCH_CHECK();
        return;
    }
    int64_t nb = (n + kScanTile - 1) / kScanTile;
    hipLaunchKernelGGL(k_scan_reduce, dim3((unsigned)nb), dim3(kScanThreads), 0, s, d_in, n, d_tmp);
    FMM_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(kScanThreads), 0, s, d_tmp, nb, d_total);
    FMM_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_scan_down, dim3((unsigned)nb), dim3(kScanThreads), 0, s, d_in, d_out, n, d_tmp);
    FMM_LAUNCH_CHECK();
}

size_t radix_tmp_elems(int64_t n) {
    int64_t nblocks = (n + kRsTile - 1) / kRsTile;
    return (size_t)(256 * nblocks) + 256 + 64;
}

void radix_sort_u64(uint64_t *kin, uint32_t *vin, uint64_t *kalt, uint32_t *valt, int64_t n, int bit_lo,
                    int bit_hi, int32_t *d_tmp, hipStream_t s, bool *in_alt) {
    radix_sort_impl<uint64_t>(kin, vin, kalt, valt, n, bit_lo, bit_hi, d_tmp, s, in_alt);
}

void radix_sort_u32(uint32_t *kin, uint32_t *vin, uint32_t *kalt, uint32_t *valt, int64_t n, int bit_lo,
                    int bit_hi, int32_t *d_tmp, hipStream_t s, bool *in_alt) {
    radix_sort_impl<uint32_t>(kin, vin, kalt, valt, n, bit_lo, bit_hi, d_tmp, s, in_alt);
}

}  // namespace fmm
