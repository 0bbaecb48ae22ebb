// Device exclusive prefix sums (row pointers of the reference rows, cell
// pointers of the cell -> ray transpose).  Three passes: per-tile totals, a
// scan of the tile totals in one workgroup, then per-tile scans with offsets.
#include "uspg_internal.hpp"

namespace uspg {
namespace {

constexpr int kThreads = 256;
constexpr int kItems = 8;
constexpr int kTile = kThreads * kItems;

template <class T>
__device__ T block_exclusive_scan(T v, T *sh, T *total)
{
    // Hillis-Steele in shared memory over 256 values; returns the exclusive
    // prefix of this thread's value and writes the block total.
    const int t = threadIdx.x;
    sh[t] = v;
    __syncthreads();
    for (int off = 1; off < kThreads; off <<= 1) {
        T x = (t >= off) ? sh[t - off] : T(0);
        __syncthreads();
        sh[t] += x;
        __syncthreads();
    }
    T incl = sh[t];
    if (t == kThreads - 1) *total = incl;
    __syncthreads();
    return incl - v;
}

template <class T>
__global__ __launch_bounds__(kThreads) void tile_totals(const uint32_t *in, int64_t n, T *tot)
{
    __shared__ T sh[kThreads];
    __shared__ T total;
    int64_t base = (int64_t)blockIdx.x * kTile + (int64_t)threadIdx.x * kItems;
    T s = 0;
    for (int k = 0; k < kItems; ++k)
        if (base + k < n) s += (T)in[base + k];
    block_exclusive_scan<T>(s, sh, &total);
    if (threadIdx.x == 0) tot[blockIdx.x] = total;
}

template <class T>
__global__ __launch_bounds__(kThreads) void scan_totals(T *tot, int64_t ntiles, T *grand)
{
    __shared__ T sh[kThreads];
    __shared__ T total;
    T carry = 0;
    for (int64_t base = 0; base < ntiles; base += kThreads) {
        int64_t i = base + threadIdx.x;
        T v = (i < ntiles) ? tot[i] : T(0);
        T ex = block_exclusive_scan<T>(v, sh, &total);
        if (i < ntiles) tot[i] = carry + ex;
        carry += total;
        __syncthreads();
    }
    if (threadIdx.x == 0) *grand = carry;
}

template <class T>
__global__ __launch_bounds__(kThreads) void tile_scan(const uint32_t *in, int64_t n, const T *tot, T *out)
{
    __shared__ T sh[kThreads];
    __shared__ T total;
    int64_t base = (int64_t)blockIdx.x * kTile + (int64_t)threadIdx.x * kItems;
    T loc[kItems];
    T s = 0;
    for (int k = 0; k < kItems; ++k) {
        loc[k] = (base + k < n) ? (T)in[base + k] : T(0);
        s += loc[k];
    }
    T ex = block_exclusive_scan<T>(s, sh, &total) + tot[blockIdx.x];
    for (int k = 0; k < kItems; ++k) {
        if (base + k < n) out[base + k] = ex;
        ex += loc[k];
    }
}

template <class T>
int scan_impl(const uint32_t *in, T *out, int64_t n, hipStream_t s)
{
    // out has n + 1 entries; out[n] is the grand total.
    int64_t ntiles = (n + kTile - 1) / kTile;
    if (ntiles == 0) {
        USPG_HIP(hipMemsetAsync(out, 0, sizeof(T), s));
        return USPG_OK;
    }
    T *tot = nullptr;
    if (dev_malloc((void **)&tot, sizeof(T) * ntiles) != hipSuccess) return fail(USPG_E_NOMEM, "device allocation failed");
    hipLaunchKernelGGL(tile_totals<T>, dim3((unsigned)ntiles), dim3(kThreads), 0, s, in, n, tot);
    hipLaunchKernelGGL(scan_totals<T>, dim3(1), dim3(kThreads), 0, s, tot, ntiles, out + n);
    hipLaunchKernelGGL(tile_scan<T>, dim3((unsigned)ntiles), dim3(kThreads), 0, s, in, n, tot, out);
    USPG_HIP(hipGetLastError());
    USPG_HIP(hipStreamSynchronize(s));
    USPG_HIP(dev_free(tot));
    return USPG_OK;
}

}  // namespace

int exclusive_scan_u32_to_i64(const uint32_t *in, int64_t *out, int64_t n, hipStream_t s)
{
    return scan_impl<int64_t>(in, out, n, s);
}

int exclusive_scan_u32(const uint32_t *in, uint32_t *out, int64_t n, hipStream_t s)
{
    return scan_impl<uint32_t>(in, out, n, s);
}

}  // namespace uspg
