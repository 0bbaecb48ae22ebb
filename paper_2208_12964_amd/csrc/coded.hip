// Coded rows of a cone-beam coefficient set (coded_rows.hpp): the in-plane
// path of every detector column, then per ray its code, checked against
// the stored row entry by entry.
//
//   col_count / col_fill   one thread walks one column's in-plane line
//   ray_nwords             mask words of each ray from its entry count (scanned)
//   ray_code               one thread codes one ray (the rays of a column on
//                          neighbouring lanes) and writes its bits, or
//                          leaves it explicit
#include <cmath>

#include "coded_rows.hpp"
#include "uspg_internal.hpp"

namespace uspg {

walk::TraceGeo trace_geo(const uspg_coeffs *c);

namespace {

using coded::CodeGeo;
using coded::PieceSink;
using coded::RayCode;

__global__ __launch_bounds__(256) void col_count(walk::TraceGeo G, uint32_t *cnt)
{
    const int u = blockIdx.x * blockDim.x + threadIdx.x;
    if (u >= G.U) return;
    PieceSink s;
    coded::walk_column(G, u, s);
    cnt[u] = (uint32_t)coded::column_records(s);
}

__global__ __launch_bounds__(256) void col_fill(walk::TraceGeo G, const int64_t *colptr, double *t, uint32_t *id0)
{
    const int u = blockIdx.x * blockDim.x + threadIdx.x;
    if (u >= G.U) return;
    PieceSink s;
    s.base = colptr[u];
    s.t = t;
    s.id0 = id0;
    coded::walk_column(G, u, s);
    s.close();
}

template <class TC>
struct StoredRow {
    const Coef<TC> *co;
    __device__ void operator()(int e, uint32_t &id, TC &a) const
    {
        id = co[e].id;
        a = co[e].a;
    }
};

// Mask words of every ray (two per chunk of 64 entries), from its row
// length; explicit rays keep their (unused) slots.
__global__ __launch_bounds__(256) void ray_nwords(int64_t nrays, const uint32_t *cnt, uint32_t *nwords)
{
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= nrays) return;
    nwords[r] = 2 * ((cnt[r] + 63) / 64);
}

// Code of every ray, checked against its stored row; a ray whose row is not
// reproduced gets word = -1 (explicit).  counts[0] += coded rays,
// counts[1] += explicit rays.
template <class TC>
__global__ __launch_bounds__(256) void ray_code(walk::TraceGeo G, CodeGeo Q, int64_t nrays, const int64_t *rowptr,
                                                const Coef<TC> *co, const int64_t *colptr, const double *t,
                                                const uint32_t *id0, int binary, const int64_t *woff,
                                                RayCode *codes, uint64_t *words, unsigned long long *counts)
{
    const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    bool coded_ray = false, explicit_ray = false;
    if (tid < nrays) {
        // the rays of one column on neighbouring lanes: they read the same
        // column records
        const int64_t r = walk::column_major_ray(G, tid, nrays);
        const int n = (int)(rowptr[r + 1] - rowptr[r]);
        RayCode rc{};
        walk::Ray ray;
        bool ok;
        if (!walk::setup_ray(G, r, ray)) {
            ok = n == 0;
            rc.n = n;
        } else {
            const int u = (int)(r % G.U);
            ok = coded::code_ray<TC>(Q, G, ray, t, id0, colptr[u], colptr[u + 1] - 1, StoredRow<TC>{co + rowptr[r]},
                                     n, binary != 0, rc, words + woff[r]);
        }
        rc.word = ok ? (int32_t)woff[r] : -1;
        codes[r] = rc;
        coded_ray = n > 0 && ok;
        explicit_ray = n > 0 && !ok;
    }
    // one atomic per wavefront and count
    const unsigned long long cm = __ballot(coded_ray), em = __ballot(explicit_ray);
    if ((threadIdx.x & 63) == 0) {
        if (cm) atomicAdd(counts, (unsigned long long)__popcll(cm));
        if (em) atomicAdd(counts + 1, (unsigned long long)__popcll(em));
    }
}

// Column records per column (scanned into colptr) and mask-word offsets per
// ray (scanned into woff) from the entry counts of the count pass.
int code_offsets(uspg_coeffs *c, int64_t *colptr, int64_t *woff, hipStream_t s)
{
    const walk::TraceGeo G = trace_geo(c);
    if (!G.kq || !G.hq || !c->pend_cnt.p || !colptr || !woff)
        return fail(USPG_E_INTERNAL, "coded rows: tables or counts not on the device");
    const int U = c->scan.det_u;
    const int64_t nrays = c->nrays;
    int rc;
    DevBuf cnt, nwords;
    if ((rc = cnt.alloc(sizeof(uint32_t) * (U + 1))) != USPG_OK) return rc;
    if ((rc = nwords.alloc(sizeof(uint32_t) * (nrays + 1))) != USPG_OK) return rc;
    hipLaunchKernelGGL(col_count, dim3((U + 255) / 256), dim3(256), 0, s, G, cnt.as<uint32_t>());
    if ((rc = exclusive_scan_u32_to_i64(cnt.as<uint32_t>(), colptr, U, s)) != USPG_OK) return rc;
    hipLaunchKernelGGL(ray_nwords, dim3((unsigned)((nrays + 255) / 256)), dim3(256), 0, s, nrays,
                       c->pend_cnt.as<uint32_t>(), nwords.as<uint32_t>());
    if ((rc = exclusive_scan_u32_to_i64(nwords.as<uint32_t>(), woff, nrays, s)) != USPG_OK) return rc;
    USPG_HIP(hipGetLastError());
    return USPG_OK;
}

template <class TC>
int fill_typed(uspg_coeffs *c, hipStream_t s)
{
    const walk::TraceGeo G = trace_geo(c);
    const uspg_grid *g = c->g;
    CodeGeo Q{g->z0, g->h, g->nz, (uint32_t)c->Cq, (uint32_t)c->Wc};
    const int U = c->scan.det_u;
    const int64_t nrays = c->nrays;
    const int binary = c->scan.weights == USPG_WEIGHTS_BINARY;
    int rc;
    if (!c->rowptr.p || !c->coef.p || !c->d_colptr.p || !c->d_colt.p || !c->d_colid.p || !c->d_codes.p ||
        !c->d_words.p)
        return fail(USPG_E_INTERNAL, "coded rows: rows or code buffers not on the device");
    DevBuf woff, counts;
    if ((rc = counts.alloc(2 * sizeof(unsigned long long))) != USPG_OK) return rc;
    if (c->pend_colptr.p && c->pend_woff.p) {
        // the offsets of the count pass
        USPG_HIP(hipMemcpyAsync(c->d_colptr.p, c->pend_colptr.p, sizeof(int64_t) * (U + 1), hipMemcpyDeviceToDevice,
                                s));
    } else {
        if ((rc = woff.alloc(sizeof(int64_t) * (nrays + 1))) != USPG_OK) return rc;
        if ((rc = code_offsets(c, c->d_colptr.as<int64_t>(), woff.as<int64_t>(), s)) != USPG_OK) return rc;
    }
    const int64_t *wo = woff.p ? woff.as<int64_t>() : c->pend_woff.as<int64_t>();
    hipLaunchKernelGGL(col_fill, dim3((U + 255) / 256), dim3(256), 0, s, G, c->d_colptr.as<int64_t>(),
                       c->d_colt.as<double>(), c->d_colid.as<uint32_t>());
    USPG_HIP(hipMemsetAsync(counts.p, 0, 2 * sizeof(unsigned long long), s));
    hipLaunchKernelGGL(ray_code<TC>, dim3((unsigned)((nrays + 255) / 256)), dim3(256), 0, s, G, Q, nrays,
                       c->rowptr.as<int64_t>(), c->coef.as<Coef<TC>>(), c->d_colptr.as<int64_t>(),
                       c->d_colt.as<double>(), c->d_colid.as<uint32_t>(), binary, wo,
                       c->d_codes.as<RayCode>(), c->d_words.as<uint64_t>(), counts.as<unsigned long long>());
    USPG_HIP(hipGetLastError());
    unsigned long long hc[2] = {0, 0};
    USPG_HIP(hipMemcpyAsync(hc, counts.p, sizeof(hc), hipMemcpyDeviceToHost, s));
    USPG_HIP(hipStreamSynchronize(s));
    c->coded_rays = (int64_t)hc[0];
    c->explicit_rays = (int64_t)hc[1];
    c->coded = true;
    return USPG_OK;
}

}  // namespace

int code_count(uspg_coeffs *c, hipStream_t s)
{
    const int U = c->scan.det_u;
    const int64_t nrays = c->nrays;
    int rc;
    // kept in the handle for the fill, which then needs no second column walk
    DevBuf &colptr = c->pend_colptr, &woff = c->pend_woff;
    if ((rc = colptr.alloc(sizeof(int64_t) * (U + 1))) != USPG_OK) return rc;
    if ((rc = woff.alloc(sizeof(int64_t) * (nrays + 1))) != USPG_OK) return rc;
    if ((rc = code_offsets(c, colptr.as<int64_t>(), woff.as<int64_t>(), s)) != USPG_OK) return rc;
    USPG_HIP(hipMemcpy(&c->pend_nrec, colptr.as<int64_t>() + U, sizeof(int64_t), hipMemcpyDeviceToHost));
    USPG_HIP(hipMemcpy(&c->pend_nwords, woff.as<int64_t>() + nrays, sizeof(int64_t), hipMemcpyDeviceToHost));
    if (c->pend_nrec >= ((int64_t)1 << 31) || c->pend_nwords >= ((int64_t)1 << 31))
        return fail(USPG_E_ARG, "coded rows: more than 2^31 column records or mask words");
    return USPG_OK;
}

int code_fill(uspg_coeffs *c, hipStream_t s)
{
    if (c->scan.coeff_dtype == USPG_F64) return fill_typed<double>(c, s);
    return fill_typed<float>(c, s);
}

}  // namespace uspg
