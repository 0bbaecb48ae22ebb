// Coded rows of a cone-beam coefficient set (coded_rows.hpp): the in-plane
// path of every detector column, then per ray its code, checked against
// the stored row entry by entry.
//
//   col_count / col_fill   one thread walks one column's in-plane line
//   ray_nwords             mask words of each ray from its row length (scanned)
//   ray_code               one thread codes one ray and writes its bits, or
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

// Mask words of every ray (two per chunk of 64 entries), from its stored
// row length; explicit rays keep their (unused) slots.
__global__ __launch_bounds__(256) void ray_nwords(int64_t nrays, const int64_t *rowptr, uint32_t *nwords)
{
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= nrays) return;
    const int64_t n = rowptr[r + 1] - rowptr[r];
    nwords[r] = (uint32_t)(2 * ((n + 63) / 64));
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
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= nrays) return;
    const int n = (int)(rowptr[r + 1] - rowptr[r]);
    RayCode rc{};
    walk::Ray ray;
    bool ok;
    if (!walk::setup_ray(G, r, ray)) {
        ok = n == 0;
        rc.n = n;
    } else {
        const int u = (int)(r % G.U);
        ok = coded::code_ray<TC>(Q, G, ray, t, id0, colptr[u], colptr[u + 1] - 1, StoredRow<TC>{co + rowptr[r]}, n,
                                 binary != 0, rc, words + woff[r]);
    }
    rc.word = ok ? (int32_t)woff[r] : -1;
    codes[r] = rc;
    if (n > 0) atomicAdd(counts + (ok ? 0 : 1), 1ull);
}

template <class TC>
int build_typed(uspg_coeffs *c, hipStream_t s)
{
    const walk::TraceGeo G = trace_geo(c);
    const uspg_grid *g = c->g;
    CodeGeo Q{g->z0, g->h, g->nz, (uint32_t)c->Cq, (uint32_t)c->Wc};
    const int U = c->scan.det_u;
    const int64_t nrays = c->nrays;
    const int binary = c->scan.weights == USPG_WEIGHTS_BINARY;
    int rc = USPG_OK;
    DevBuf cnt, nwords, woff, counts;
    do {
        // column paths
        if ((rc = cnt.alloc(sizeof(uint32_t) * (U + 1))) != USPG_OK) break;
        if ((rc = c->d_colptr.alloc(sizeof(int64_t) * (U + 1))) != USPG_OK) break;
        hipLaunchKernelGGL(col_count, dim3((U + 255) / 256), dim3(256), 0, s, G, cnt.as<uint32_t>());
        if ((rc = exclusive_scan_u32_to_i64(cnt.as<uint32_t>(), c->d_colptr.as<int64_t>(), U, s)) != USPG_OK) break;
        int64_t nrec = 0;
        USPG_HIP(hipMemcpy(&nrec, c->d_colptr.as<int64_t>() + U, sizeof(int64_t), hipMemcpyDeviceToHost));
        if (nrec >= ((int64_t)1 << 31)) { rc = fail(USPG_E_ARG, "coded rows: more than 2^31 column records"); break; }
        if ((rc = c->d_colt.alloc(sizeof(double) * nrec)) != USPG_OK) break;
        if ((rc = c->d_colid.alloc(sizeof(uint32_t) * nrec)) != USPG_OK) break;
        hipLaunchKernelGGL(col_fill, dim3((U + 255) / 256), dim3(256), 0, s, G, c->d_colptr.as<int64_t>(),
                           c->d_colt.as<double>(), c->d_colid.as<uint32_t>());
        USPG_HIP(hipGetLastError());
        // mask words at the offsets of the row lengths, then the codes
        if ((rc = nwords.alloc(sizeof(uint32_t) * (nrays + 1))) != USPG_OK) break;
        if ((rc = woff.alloc(sizeof(int64_t) * (nrays + 1))) != USPG_OK) break;
        const unsigned rb = (unsigned)((nrays + 255) / 256);
        hipLaunchKernelGGL(ray_nwords, dim3(rb), dim3(256), 0, s, nrays, c->rowptr.as<int64_t>(), nwords.as<uint32_t>());
        if ((rc = exclusive_scan_u32_to_i64(nwords.as<uint32_t>(), woff.as<int64_t>(), nrays, s)) != USPG_OK) break;
        int64_t nw = 0;
        USPG_HIP(hipMemcpy(&nw, woff.as<int64_t>() + nrays, sizeof(int64_t), hipMemcpyDeviceToHost));
        if (nw >= ((int64_t)1 << 31)) { rc = fail(USPG_E_ARG, "coded rows: more than 2^31 mask words"); break; }
        if ((rc = c->d_words.alloc(sizeof(uint64_t) * (nw > 0 ? nw : 1))) != USPG_OK) break;
        if ((rc = c->d_codes.alloc(sizeof(RayCode) * nrays)) != USPG_OK) break;
        if ((rc = counts.alloc(2 * sizeof(unsigned long long))) != USPG_OK) break;
        USPG_HIP(hipMemsetAsync(counts.p, 0, 2 * sizeof(unsigned long long), s));
        hipLaunchKernelGGL(ray_code<TC>, dim3(rb), dim3(256), 0, s, G, Q, nrays, c->rowptr.as<int64_t>(),
                           c->coef.as<Coef<TC>>(), c->d_colptr.as<int64_t>(), c->d_colt.as<double>(),
                           c->d_colid.as<uint32_t>(), binary, woff.as<int64_t>(), c->d_codes.as<RayCode>(),
                           c->d_words.as<uint64_t>(), counts.as<unsigned long long>());
        USPG_HIP(hipGetLastError());
        unsigned long long hc[2] = {0, 0};
        USPG_HIP(hipMemcpyAsync(hc, counts.p, sizeof(hc), hipMemcpyDeviceToHost, s));
        USPG_HIP(hipStreamSynchronize(s));
        c->coded_rays = (int64_t)hc[0];
        c->explicit_rays = (int64_t)hc[1];
        c->coded = true;
    } while (0);
    if (rc != USPG_OK) {
        c->d_colptr.release();
        c->d_colt.release();
        c->d_colid.release();
        c->d_codes.release();
        c->d_words.release();
        c->coded = false;
    }
    return rc;
}

}  // namespace

int build_row_codes(uspg_coeffs *c, hipStream_t s)
{
    if (c->scan.coeff_dtype == USPG_F64) return build_typed<double>(c, s);
    return build_typed<float>(c, s);
}

}  // namespace uspg
