// Internal declarations shared by the HIP sources of the FMM library.
// Nothing here is part of the public C ABI (include/fmm.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <cstdio>
#include <string>
#include <vector>

namespace fmm {

constexpr int kLevels = 21;      // key bits per axis (63-bit Morton keys)
constexpr int kMaxP = 16;        // highest supported expansion order

// Number of real coefficients kept for order p: degrees 0..p, (2n+1) each.
__host__ __device__ constexpr int ncoef(int p) { return (p + 1) * (p + 1); }
// Real layout of degree n, order m >= 0:  m = 0 -> n*n ; m > 0 -> re at
// n*n + 2m - 1, im at n*n + 2m.
__host__ __device__ constexpr int cidx_re(int n, int m) { return m == 0 ? n * n : n * n + 2 * m - 1; }
__host__ __device__ constexpr int cidx_im(int n, int m) { return n * n + 2 * m; }

// Device allocation that only grows.  Contents are not preserved by grow()
// unless grow_keep() is used.
struct DevBuf {
    void *ptr = nullptr;
    size_t bytes = 0;
    hipError_t grow(size_t want);
    hipError_t grow_keep(size_t want, hipStream_t s);
    void release();
    template <class T> T *as() const { return static_cast<T *>(ptr); }
};

struct HipError {
    hipError_t err;
    const char *what;
};

// Device-wide exclusive scan of int32 values in place; writes the total to
// *d_total (device) when non-null.  tmp must hold scan_tmp_elems(n) ints.
size_t scan_tmp_elems(int64_t n);
void exclusive_scan_i32(int32_t *d_data, int64_t n, int32_t *d_total, int32_t *d_tmp, hipStream_t s);
// Out-of-place variant (d_in may equal d_out).  d_total may point at d_out[n].
void exclusive_scan_oop(const int32_t *d_in, int32_t *d_out, int64_t n, int32_t *d_total, int32_t *d_tmp,
                        hipStream_t s);

// Stable LSD radix sort of (key, value) pairs over bits [bit_lo, bit_hi).
// kin/vin and kalt/valt are ping-pong buffers of n elements; the sorted
// result ends in kin/vin.  vin may be null (keys only).  tmp must hold
// radix_tmp_elems(n) ints.
size_t radix_tmp_elems(int64_t n);
// With in_alt given, an odd number of passes leaves the result in kalt/valt
// (*in_alt = true) instead of copying it back.
void radix_sort_u64(uint64_t *kin, uint32_t *vin, uint64_t *kalt, uint32_t *valt, int64_t n, int bit_lo,
                    int bit_hi, int32_t *d_tmp, hipStream_t s, bool *in_alt = nullptr);
void radix_sort_u32(uint32_t *kin, uint32_t *vin, uint32_t *kalt, uint32_t *valt, int64_t n, int bit_lo,
                    int bit_hi, int32_t *d_tmp, hipStream_t s, bool *in_alt = nullptr);

// Small device-to-host reads without a stream synchronisation: a one-thread
// kernel copies the values into pinned, mapped host memory and then raises a
// sequence flag there (system-scope release); the host spins on the flag,
// checking the stream for errors while it waits.  Falls back to a copy and a
// stream synchronisation for reads above kHostReadMax values or when the
// pinned buffer could not be allocated.
constexpr int kHostReadMax = 64;  // int32 values per fast read
struct HostReader {
    int32_t *h = nullptr;  // pinned host: [0] flag, [16 ..] data
    int32_t *d = nullptr;  // device view of h
    int32_t seq = 0;
    void init();           // best effort: on failure reads use the fallback
    void release();
    void read(void *host, const void *dev, size_t bytes, hipStream_t s);  // throws HipError
    // The same in two halves: begin enqueues the copy, end waits for it.
    // Work enqueued on s in between keeps the GPU busy while the host waits
    // (one read outstanding at a time).
    void begin(const void *dev, size_t bytes, hipStream_t s);
    void end(void *host, hipStream_t s);
    const void *pend_dev = nullptr;
    size_t pend_bytes = 0;
    bool pend_fallback = false;
};

// Zero `bytes` bytes (a multiple of 4) at a 4-byte aligned device address
// with a kernel: unlike hipMemsetAsync it may be captured in a HIP graph and
// replayed.
void fill_zero(void *ptr, size_t bytes, hipStream_t s);

inline int grid_for(int64_t n, int threads, int cap = 65535 * 4) {
    int64_t g = (n + threads - 1) / threads;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (int)g;
}

}  // namespace fmm

#define FMM_HIP_CHECK(expr)                                     \
    do {                                                        \
        hipError_t _e = (expr);                                 \
        if (_e != hipSuccess) throw ::fmm::HipError{_e, #expr}; \
    } while (0)

#define FMM_LAUNCH_CHECK() FMM_HIP_CHECK(hipGetLastError())
