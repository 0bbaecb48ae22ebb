// Reference-view tracing on the device (Sec. III.A-B, Alg. 1).
// One thread walks one view-0 ray in FP64 (trace_walk.hpp), the rays of a
// detector column on neighbouring threads.  Two passes with identical
// arithmetic: the first counts entries per ray, the second writes them at
// the scanned offsets.
#include <cmath>

#include "trace_walk.hpp"
#include "uspg_internal.hpp"

namespace uspg {
namespace {

using walk::Ray;
using walk::RowSink;
using walk::TraceGeo;
using walk::Walker;
using walk::setup_ray;

__global__ __launch_bounds__(256) void trace_count(TraceGeo G, int64_t nrays, uint32_t *cnt)
{
    const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (tid >= nrays) return;
    const int64_t r = walk::column_major_ray(G, tid, nrays);
    Ray ray;
    uint32_t n = 0;
    if (setup_ray(G, r, ray)) {
        RowSink<false, float> sink;
        sink.base = 0;
        sink.ids = nullptr;
        sink.a = nullptr;
        sink.binary = false;
        sink.eps = G.eps;
        Walker<RowSink<false, float>> w(G, ray, sink);
        w.run();
        n = (uint32_t)sink.count;
    }
    cnt[r] = n;
}

// Writes each row's (id, coefficient) pairs straight into the coefficient
// array.
template <class TC>
__global__ __launch_bounds__(256) void trace_fill(TraceGeo G, int64_t nrays, const int64_t *rowptr, Coef<TC> *co,
                                                  int binary)
{
    const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (tid >= nrays) return;
    const int64_t r = walk::column_major_ray(G, tid, nrays);
    Ray ray;
    if (!setup_ray(G, r, ray)) return;
    RowSink<true, TC> sink;
    sink.base = rowptr[r];
    sink.ids = &co[0].id;
    sink.a = &co[0].a;
    sink.ids_stride = sizeof(Coef<TC>) / sizeof(uint32_t);
    sink.a_stride = sizeof(Coef<TC>) / sizeof(TC);
    sink.binary = binary != 0;
    sink.eps = G.eps;
    Walker<RowSink<true, TC>> w(G, ray, sink);
    w.run();
}

__global__ void row_lengths_max(const uint32_t *cnt, int64_t n, unsigned int *mx)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) atomicMax(mx, cnt[i]);
}

}  // namespace

// Geometry of the view-0 walk of a coefficient set (device tables).
TraceGeo trace_geo(const uspg_coeffs *c)
{
    const uspg_grid *g = c->g;
    const uspg_scan_desc &sc = c->scan;
    TraceGeo G{};
    G.nr = g->nr; G.nz = g->nz; G.is3d = sc.geometry == USPG_CONE_3D; G.geom = sc.geometry;
    G.R = g->R; G.r = g->r; G.h = g->h; G.z0 = g->z0; G.H = g->H;
    G.ng = g->d_ng.as<int32_t>();
    G.head = g->d_head.as<int64_t>();
    G.cs = g->d_cs.as<double2>();
    G.kq = c->d_kq.as<int32_t>();
    G.hq = c->d_hq.as<int32_t>();
    G.Cq = c->Cq; G.Wc = c->Wc; G.grp = c->grp;
    G.U = sc.det_u; G.V = sc.det_v;
    G.Wu = sc.det_half_u; G.Wv = sc.det_half_v; G.Dso = sc.src_axis; G.Dsd = sc.src_det;
    G.eps = 1e-12 * g->R;
    return G;
}

int trace_count_rows(uspg_coeffs *c, hipStream_t s)
{
    const TraceGeo G = trace_geo(c);
    if (!G.kq || !G.hq) return fail(USPG_E_INTERNAL, "trace: layout tables not on the device");
    const int64_t nrays = c->nrays;
    const unsigned blocks = (unsigned)((nrays + 255) / 256);
    int rc = USPG_OK;
    DevBuf rp, mx;
    do {
        if ((rc = c->pend_cnt.alloc(sizeof(uint32_t) * (nrays + 1))) != USPG_OK) break;
        if ((rc = rp.alloc(sizeof(int64_t) * (nrays + 1))) != USPG_OK) break;
        if ((rc = mx.alloc(sizeof(unsigned int))) != USPG_OK) break;
        uint32_t *cnt = c->pend_cnt.as<uint32_t>();
        hipLaunchKernelGGL(trace_count, dim3(blocks), dim3(256), 0, s, G, nrays, cnt);
        if (hipGetLastError() != hipSuccess) { rc = fail(USPG_E_HIP, "trace_count launch failed"); break; }
        if ((rc = exclusive_scan_u32_to_i64(cnt, rp.as<int64_t>(), nrays, s)) != USPG_OK) break;
        if (hipMemsetAsync(mx.p, 0, sizeof(unsigned int), s) != hipSuccess) { rc = fail(USPG_E_HIP, "memset"); break; }
        hipLaunchKernelGGL(row_lengths_max, dim3(blocks), dim3(256), 0, s, cnt, nrays, mx.as<unsigned int>());
        int64_t nnz = 0;
        unsigned int mrow = 0;
        if (hipMemcpyAsync(&nnz, rp.as<int64_t>() + nrays, sizeof(int64_t), hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipMemcpyAsync(&mrow, mx.p, sizeof(unsigned int), hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess) {
            rc = fail(USPG_E_HIP, "trace: reading the row count failed");
            break;
        }
        if (nnz >= (int64_t)UINT32_MAX) { rc = fail(USPG_E_ARG, "more than 2^32 reference coefficients"); break; }
        c->nnz = nnz;
        c->max_row = (int32_t)mrow;
    } while (0);
    if (rc != USPG_OK) c->pend_cnt.release();
    return rc;
}

int trace_fill_rows(uspg_coeffs *c, hipStream_t s)
{
    const uspg_scan_desc &sc = c->scan;
    const TraceGeo G = trace_geo(c);
    if (!G.kq || !G.hq || !c->pend_cnt.p || !c->rowptr.p || !c->coef.p)
        return fail(USPG_E_INTERNAL, "trace: tables, counts or rows not on the device");
    const int64_t nrays = c->nrays;
    const unsigned blocks = (unsigned)((nrays + 255) / 256);
    int rc = USPG_OK;
    do {
        if ((rc = exclusive_scan_u32_to_i64(c->pend_cnt.as<uint32_t>(), c->rowptr.as<int64_t>(), nrays, s)) != USPG_OK)
            break;
        const int binary = sc.weights == USPG_WEIGHTS_BINARY;
        if (sc.coeff_dtype == USPG_F64)
            hipLaunchKernelGGL(trace_fill<double>, dim3(blocks), dim3(256), 0, s, G, nrays, c->rowptr.as<int64_t>(),
                               c->coef.as<Coef<double>>(), binary);
        else
            hipLaunchKernelGGL(trace_fill<float>, dim3(blocks), dim3(256), 0, s, G, nrays, c->rowptr.as<int64_t>(),
                               c->coef.as<Coef<float>>(), binary);
        const bool launched = hipGetLastError() == hipSuccess;
        const bool synced = hipStreamSynchronize(s) == hipSuccess;
        if (!launched) { rc = fail(USPG_E_HIP, "trace_fill launch failed"); break; }
        if (!synced) { rc = fail(USPG_E_HIP, "trace_fill failed"); break; }
    } while (0);
    return rc;
}

}  // namespace uspg
