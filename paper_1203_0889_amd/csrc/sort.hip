// Device-wide exclusive scan and stable LSD radix sort (keys of the Morton
// octree, Sec. 2.2, and of the interaction-pair lists).
//
// Radix sort: 8-bit digits; per pass three launches -- per-tile digit
// histograms, one exclusive scan over the (digit-major, tile-minor) count
// table, and a stable scatter.  Inside a tile each wave64 ranks its keys with
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

// Scans whose length lives on the device: n = range[1] - range[0] (a level's
// cell range), at most n_max; grids are sized for n_max and blocks past n
// return at once.
__device__ inline int64_t dev_len(const int32_t *range) { return (int64_t)range[1] - range[0]; }

__global__ void k_scan_reduce_dev(const int32_t *__restrict__ data, const int32_t *__restrict__ range,
                                  int32_t *__restrict__ sums) {
    const int64_t n = dev_len(range);
    const int64_t nb = (n + kScanTile - 1) / kScanTile;
    if (blockIdx.x >= nb) return;
    int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    int sum = 0;
#pragma unroll
    for (int i = 0; i < kScanItems; i++)
        if (base + i < n) sum += data[base + i];
    int tot;
    block_exclusive_scan(sum, &tot);
    if (threadIdx.x == 0) sums[blockIdx.x] = tot;
}

__global__ void k_scan_top_dev(int32_t *__restrict__ sums, const int32_t *__restrict__ range,
                               int32_t *__restrict__ total) {
    const int64_t nb = (dev_len(range) + kScanTile - 1) / kScanTile;
    int carry = 0;
    for (int64_t c = 0; c < nb; c += kScanTile) {
        int64_t base = c + (int64_t)threadIdx.x * kScanItems;
        int v[kScanItems];
        int sum = 0;
#pragma unroll
        for (int i = 0; i < kScanItems; i++) {
            v[i] = base + i < nb ? sums[base + i] : 0;
            sum += v[i];
        }
        int tot;
        int pre = block_exclusive_scan(sum, &tot) + carry;
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

__global__ void k_scan_down_dev(const int32_t *__restrict__ in, int32_t *__restrict__ out,
                                const int32_t *__restrict__ range, const int32_t *__restrict__ sums) {
    const int64_t n = dev_len(range);
    const int64_t nb = (n + kScanTile - 1) / kScanTile;
    if (blockIdx.x >= nb) return;
    int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    int v[kScanItems];
    int sum = 0;
#pragma unroll
    for (int i = 0; i < kScanItems; i++) {
        v[i] = base + i < n ? in[base + i] : 0;
        sum += v[i];
    }
    int tot;
    int pre = block_exclusive_scan(sum, &tot) + sums[blockIdx.x];
#pragma unroll
    for (int i = 0; i < kScanItems; i++) {
        if (base + i < n) out[base + i] = pre;
        pre += v[i];
    }
}

// ---------------------------------------------------------------- radix sort

constexpr int kRsThreads = 256;
constexpr int kRsWaves = kRsThreads / 64;
constexpr int kRsItems = 16;
constexpr int kRsTile = kRsThreads * kRsItems;
constexpr int kRsWaveTile = 64 * kRsItems;

template <class K>
__global__ void __launch_bounds__(kRsThreads) k_rs_hist(const K *__restrict__ kin, int64_t n, int shift,
                                                        int nbits, int32_t *__restrict__ counts, int nblocks) {
    __shared__ int hist[256];
    hist[threadIdx.x] = 0;
    __syncthreads();
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int mask = (1 << nbits) - 1;
    int64_t base = (int64_t)blockIdx.x * kRsTile + (int64_t)w * kRsWaveTile + lane;
#pragma unroll 4
    for (int it = 0; it < kRsItems; it++) {
        int64_t i = base + it * 64;
        if (i < n) atomicAdd(&hist[(int)((kin[i] >> shift) & (K)mask)], 1);
    }
    __syncthreads();
    counts[(int64_t)threadIdx.x * nblocks + blockIdx.x] = hist[threadIdx.x];
}

// Scatter of one pass.  Each block ranks its tile stably (per wave with
// ballots over the digit bits, then across the waves), places the tile in
// LDS in digit order, and writes it out in that order: consecutive threads
// then write consecutive addresses of one digit run instead of up to 64
// different lines per store.
// kVals: values travel with the keys (without them the tile's value
// staging is left out, which leaves LDS for more workgroups per CU).
template <class K, bool kVals>
__global__ void __launch_bounds__(kRsThreads) k_rs_scatter(const K *__restrict__ kin, const uint32_t *__restrict__ vin,
                                                           K *__restrict__ kout, uint32_t *__restrict__ vout, int64_t n,
                                                           int shift, int nbits, const int32_t *__restrict__ offs,
                                                           int nblocks) {
    __shared__ int wcount[kRsWaves][256];
    __shared__ int wbase[kRsWaves][256];
    __shared__ int lstart[257];
    __shared__ int gbase[256];
    __shared__ int wsum[kRsWaves];
    __shared__ K skey[kRsTile];
    __shared__ uint32_t sval[kVals ? kRsTile : 1];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int mask = (1 << nbits) - 1;
    for (int i = threadIdx.x; i < kRsWaves * 256; i += kRsThreads) (&wcount[0][0])[i] = 0;
    __syncthreads();
    const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    const int64_t tile0 = (int64_t)blockIdx.x * kRsTile;
    const int64_t base = tile0 + (int64_t)w * kRsWaveTile + lane;
    K key[kRsItems];
    uint32_t val[kRsItems];
    int rank[kRsItems];
#pragma unroll
    for (int it = 0; it < kRsItems; it++) {
        int64_t i = base + it * 64;
        bool valid = i < n;
        K k = valid ? kin[i] : (K)0;
        key[it] = k;
        val[it] = (kVals && valid) ? vin[i] : 0u;
        int d = (int)((k >> shift) & (K)mask);
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
        // then an exclusive scan over the 256 digits (block-local starts)
        const int d = threadIdx.x;
        int run = 0;
#pragma unroll
        for (int ww = 0; ww < kRsWaves; ww++) {
            wbase[ww][d] = run;
            run += wcount[ww][d];
        }
        int inc = run;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            int t = __shfl_up(inc, o, 64);
            if (lane >= o) inc += t;
        }
        if (lane == 63) wsum[w] = inc;
        gbase[d] = offs[(int64_t)d * nblocks + blockIdx.x];
        __syncthreads();
        int before = 0;
        for (int ww = 0; ww < w; ww++) before += wsum[ww];
        lstart[d] = before + inc - run;
        if (d == 255) lstart[256] = before + inc;
    }
    __syncthreads();
#pragma unroll
    for (int it = 0; it < kRsItems; it++) {
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

template <class K>
void radix_sort_impl(K *kin, uint32_t *vin, K *kalt, uint32_t *valt, int64_t n, int bit_lo, int bit_hi,
                     int32_t *d_tmp, hipStream_t s) {
    if (n <= 1 || bit_hi <= bit_lo) return;
    const int nblocks = (int)((n + kRsTile - 1) / kRsTile);
    int32_t *counts = d_tmp;
    int32_t *scan_tmp = d_tmp + (int64_t)256 * nblocks;
    K *ka = kin, *kb = kalt;
    uint32_t *va = vin, *vb = vin ? valt : nullptr;
    int passes = 0;
    for (int shift = bit_lo; shift < bit_hi; shift += 8) {
        int nbits = bit_hi - shift < 8 ? bit_hi - shift : 8;
        hipLaunchKernelGGL(k_rs_hist<K>, dim3(nblocks), dim3(kRsThreads), 0, s, ka, n, shift, nbits, counts, nblocks);
        FMM_LAUNCH_CHECK();
        exclusive_scan_i32(counts, (int64_t)256 * nblocks, nullptr, scan_tmp, s);
        if (va)
            hipLaunchKernelGGL((k_rs_scatter<K, true>), dim3(nblocks), dim3(kRsThreads), 0, s, ka, va, kb, vb, n, shift,
                               nbits, counts, nblocks);
        else
            hipLaunchKernelGGL((k_rs_scatter<K, false>), dim3(nblocks), dim3(kRsThreads), 0, s, ka, va, kb, vb, n, shift,
                               nbits, counts, nblocks);
        FMM_LAUNCH_CHECK();
        K *tk = ka;
        ka = kb;
        kb = tk;
        uint32_t *tv = va;
        va = vb;
        vb = tv;
        passes++;
    }
    if (passes & 1) {
        FMM_HIP_CHECK(hipMemcpyAsync(kin, ka, n * sizeof(K), hipMemcpyDeviceToDevice, s));
        if (vin) FMM_HIP_CHECK(hipMemcpyAsync(vin, va, n * sizeof(uint32_t), hipMemcpyDeviceToDevice, s));
    }
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

void exclusive_scan_dev(const int32_t *d_in, int32_t *d_out, const int32_t *d_range, int64_t n_max,
                        int32_t *d_total, int32_t *d_tmp, hipStream_t s) {
    const int64_t nb = std::max<int64_t>(1, (n_max + kScanTile - 1) / kScanTile);
    hipLaunchKernelGGL(k_scan_reduce_dev, dim3((unsigned)nb), dim3(kScanThreads), 0, s, d_in, d_range, d_tmp);
    FMM_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_scan_top_dev, dim3(1), dim3(kScanThreads), 0, s, d_tmp, d_range, d_total);
    FMM_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_scan_down_dev, dim3((unsigned)nb), dim3(kScanThreads), 0, s, d_in, d_out, d_range, d_tmp);
    FMM_LAUNCH_CHECK();
}

size_t radix_tmp_elems(int64_t n) {
    int64_t nblocks = (n + kRsTile - 1) / kRsTile;
    return (size_t)(256 * nblocks) + scan_tmp_elems(256 * nblocks) + 64;
}

void radix_sort_u64(uint64_t *kin, uint32_t *vin, uint64_t *kalt, uint32_t *valt, int64_t n, int bit_lo,
                    int bit_hi, int32_t *d_tmp, hipStream_t s) {
    radix_sort_impl<uint64_t>(kin, vin, kalt, valt, n, bit_lo, bit_hi, d_tmp, s);
}

void radix_sort_u32(uint32_t *kin, uint32_t *vin, uint32_t *kalt, uint32_t *valt, int64_t n, int bit_lo,
                    int bit_hi, int32_t *d_tmp, hipStream_t s) {
    radix_sort_impl<uint32_t>(kin, vin, kalt, valt, n, bit_lo, bit_hi, d_tmp, s);
}

}  // namespace fmm
