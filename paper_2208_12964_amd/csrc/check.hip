// Debug checks around the solver: whether a colour lattice keeps the rays of
// each class cell-disjoint in a view (the condition that makes a class batch
// equal to its rays applied one by one, Sec. III.D), counted independently of
// the conflict map the lattice was chosen from; and whether projection data
// are finite and non-negative (the update of eq. 18 keeps the image positive
// only for such data).
#include <cmath>

#include "uspg_internal.hpp"

namespace uspg {
namespace {

constexpr int kWaves = 4;
constexpr int kBlock = 64 * kWaves;

struct StampArgs {
    const int64_t *rowptr;
    const uint32_t *ids;     // first word of each (id, coefficient) pair
    int stride;              // words per pair
    uint32_t *hits;          // [Wtot] hits of the current class
    unsigned long long *extra;
    uint32_t shift, wtot;
    int U, cu, cw, Ku, Kv, nu, ncls;
};

// One wavefront per ray of the class: every entry adds a hit to its
// (shifted) cell; a hit on a cell already hit counts as one extra.
__global__ __launch_bounds__(kBlock) void stamp_class(StampArgs A)
{
    const int x = (int)(((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6);
    const int lane = threadIdx.x & 63;
    if (x >= A.ncls) return;
    const int w = A.cw + (x / A.nu) * A.Kv;
    const int u = A.cu + (x % A.nu) * A.Ku;
    const int64_t r = (int64_t)w * A.U + u;
    const int64_t beg = A.rowptr[r], n = A.rowptr[r + 1] - beg;
    int m = 0;
    for (int64_t j = lane; j < n; j += 64) {
        uint32_t t = A.ids[(beg + j) * A.stride] + A.shift;
        t = t >= A.wtot ? t - A.wtot : t;
        m += atomicAdd(A.hits + t, 1u) > 0u;
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) m += __shfl_xor(m, off, 64);
    if (lane == 0 && m) atomicAdd(A.extra, (unsigned long long)m);
}

template <class T>
__global__ __launch_bounds__(256) void count_bad(const T *p, int64_t n, unsigned long long *bad)
{
    __shared__ unsigned int sh[256];
    unsigned int m = 0;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
        const T v = p[i];
        m += !(v >= T(0)) || isinf(v);   // NaN, negative or infinite
    }
    sh[threadIdx.x] = m;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0 && sh[0]) atomicAdd(bad, (unsigned long long)sh[0]);
}

}  // namespace
}  // namespace uspg

using namespace uspg;

extern "C" {

int uspg_check_lattice(const uspg_coeffs *c, int32_t view, int32_t ku, int32_t kv, void *stream,
                       int64_t *collisions)
{
    if (!c || !collisions) return fail(USPG_E_ARG, "null argument");
    if (c->segments) return fail(USPG_E_ARG, "segment-record coefficients have no stored rows to check");
    if (view < 0 || view >= c->scan.n_views) return fail(USPG_E_ARG, "view out of range");
    const int U = c->scan.det_u, V = c->scan.det_v;
    if (ku < 1 || kv < 1 || ku > U || kv > V) return fail(USPG_E_ARG, "lattice out of range");
    int rc = check_coeffs(c);
    if (rc != USPG_OK) return rc;
    hipStream_t s = (hipStream_t)stream;
    DevBuf hits, extra;
    if ((rc = hits.alloc(sizeof(uint32_t) * (size_t)c->Wtot)) != USPG_OK) return rc;
    if ((rc = extra.alloc(sizeof(unsigned long long))) != USPG_OK) {
        hits.release();
        return rc;
    }
    StampArgs A{};
    A.rowptr = c->rowptr.as<int64_t>();
    A.ids = c->coef.as<uint32_t>();
    A.stride = (int)((c->scan.coeff_dtype == USPG_F64 ? sizeof(Coef<double>) : sizeof(Coef<float>)) / 4);
    A.hits = hits.as<uint32_t>();
    A.extra = extra.as<unsigned long long>();
    A.shift = (uint32_t)(((int64_t)view * c->Wc) % c->Wtot);
    A.wtot = (uint32_t)c->Wtot;
    A.U = U;
    A.Ku = ku;
    A.Kv = kv;
    unsigned long long total = 0;
    do {
        if (hipMemsetAsync(extra.p, 0, sizeof(unsigned long long), s) != hipSuccess) {
            rc = fail(USPG_E_HIP, "check: memset failed");
            break;
        }
        for (int cl = 0; cl < ku * kv && rc == USPG_OK; ++cl) {
            A.cu = cl % ku;
            A.cw = cl / ku;
            A.nu = (U - A.cu + ku - 1) / ku;
            A.ncls = A.nu * ((V - A.cw + kv - 1) / kv);
            if (A.ncls == 0) continue;
            if (hipMemsetAsync(hits.p, 0, sizeof(uint32_t) * (size_t)c->Wtot, s) != hipSuccess) {
                rc = fail(USPG_E_HIP, "check: memset failed");
                break;
            }
            const unsigned blocks = (unsigned)(((int64_t)A.ncls + kWaves - 1) / kWaves);
            hipLaunchKernelGGL(stamp_class, dim3(blocks), dim3(kBlock), 0, s, A);
            if (hipGetLastError() != hipSuccess) rc = fail(USPG_E_HIP, "check: launch failed");
        }
        if (rc != USPG_OK) break;
        if (hipMemcpyAsync(&total, extra.p, sizeof(total), hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess)
            rc = fail(USPG_E_HIP, "check: reading the count failed");
    } while (0);
    (void)hipStreamSynchronize(s);
    hits.release();
    extra.release();
    if (rc == USPG_OK) *collisions = (int64_t)total;
    return rc;
}

int uspg_check_projections(const uspg_coeffs *c, int32_t dtype, const void *proj, void *stream, int64_t *n_bad)
{
    if (!c || !proj || !n_bad) return fail(USPG_E_ARG, "null argument");
    if (dtype != USPG_F32 && dtype != USPG_F64) return fail(USPG_E_ARG, "dtype");
    int rc = check_coeffs(c);
    if (rc != USPG_OK) return rc;
    hipStream_t s = (hipStream_t)stream;
    const int64_t n = (int64_t)c->scan.n_views * c->nrays;
    DevBuf bad;
    if ((rc = bad.alloc(sizeof(unsigned long long))) != USPG_OK) return rc;
    unsigned long long total = 0;
    const int64_t want = (n + 255) / 256;
    const unsigned blocks = (unsigned)(want < 4096 ? (want > 0 ? want : 1) : 4096);
    if (hipMemsetAsync(bad.p, 0, sizeof(unsigned long long), s) != hipSuccess) rc = fail(USPG_E_HIP, "check: memset failed");
    if (rc == USPG_OK) {
        if (dtype == USPG_F64)
            hipLaunchKernelGGL(count_bad<double>, dim3(blocks), dim3(256), 0, s, (const double *)proj, n,
                               bad.as<unsigned long long>());
        else
            hipLaunchKernelGGL(count_bad<float>, dim3(blocks), dim3(256), 0, s, (const float *)proj, n,
                               bad.as<unsigned long long>());
        if (hipGetLastError() != hipSuccess ||
            hipMemcpyAsync(&total, bad.p, sizeof(total), hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess)
            rc = fail(USPG_E_HIP, "check: counting failed");
    }
    (void)hipStreamSynchronize(s);
    bad.release();
    if (rc == USPG_OK) *n_bad = (int64_t)total;
    return rc;
}

}  // extern "C"
