// Segment records of the reference view and their colouring (the paper's
// literal scheme, Sec. III.B-C, Alg. 1; see segments.hpp).
//
// Build: one thread per view-0 ray counts its records, a scan places them,
// a second pass writes (slice << 16 | ring, phi_a, phi_b) and, for a record
// in the ring just outside the innermost ring the line reaches, the index of
// the earlier record of the same ring and slice (the line's other pass
// through that ring).  Those two can meet the same sectors, which must count
// once; no other pair of records of a ray can (the grid's sector rule keeps
// the passes through any outer ring more than a sector apart).
//
// Colouring: re-binning by a rotation that is not a whole number of sectors
// changes which rays meet, so the conflict offsets are the union over every
// view of the offsets of rays sharing a cell in that view (rows rebuilt per
// view, then the same cell -> rays transpose as the reference colouring).
#include <algorithm>

#include "segments.hpp"
#include "uspg_internal.hpp"

namespace uspg {
namespace {

using walk::TraceGeo;

using seg::CountSink;
using seg::FillSink;

__global__ __launch_bounds__(256) void seg_count(TraceGeo G, int64_t nrays, uint32_t *cnt)
{
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= nrays) return;
    CountSink sk;
    cnt[r] = (uint32_t)seg::segments_of_ray(G, r, sk);
}

__global__ __launch_bounds__(256) void seg_fill(TraceGeo G, int64_t nrays, const int64_t *segptr, uint32_t *sr,
                                                double *pa, double *pb, int32_t *partner)
{
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= nrays) return;
    FillSink sk{sr, pa, pb, partner, segptr[r]};
    seg::segments_of_ray(G, r, sk);
}

// Quarter tracing (Sec. III.C): the reference view is symmetric under
// y -> -y (detector column u <-> U-1-u: azimuth phi -> 2 pi - phi) and, in
// 3D, under z -> -z (row w <-> V-1-w: slice k -> Nz-1-k).  Only the rays of
// one quadrant (u < ceil(U/2), w < ceil(V/2)) are traced; their records are
// copied to the mirror rays with those maps, in the same order along the
// ray (a mirror keeps the distance from the source).
__device__ inline int mirror_rays(int uq, int wq, int U, int V, int64_t *out)
{
    const int um = U - 1 - uq, wm = V - 1 - wq;
    int n = 0;
    out[n++] = (int64_t)wq * U + uq;
    if (um != uq) out[n++] = (int64_t)wq * U + um;
    if (wm != wq) {
        out[n++] = (int64_t)wm * U + uq;
        if (um != uq) out[n++] = (int64_t)wm * U + um;
    }
    return n;
}

__global__ __launch_bounds__(256) void seg_count_q(TraceGeo G, int uh, int vh, uint32_t *cnt)
{
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= (int64_t)uh * vh) return;
    const int uq = (int)(q % uh), wq = (int)(q / uh);
    CountSink sk;
    const uint32_t n = (uint32_t)seg::segments_of_ray(G, (int64_t)wq * G.U + uq, sk);
    int64_t rays[4];
    const int m = mirror_rays(uq, wq, G.U, G.V, rays);
    for (int j = 0; j < m; ++j) cnt[rays[j]] = n;
}

__global__ __launch_bounds__(256) void seg_fill_q(TraceGeo G, int uh, int vh, const int64_t *segptr, uint32_t *sr,
                                                  double *pa, double *pb, int32_t *partner)
{
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= (int64_t)uh * vh) return;
    const int uq = (int)(q % uh), wq = (int)(q / uh);
    const int64_t r0 = (int64_t)wq * G.U + uq;
    FillSink sk{sr, pa, pb, partner, segptr[r0]};
    const int n = seg::segments_of_ray(G, r0, sk);
    const int um = G.U - 1 - uq, wm = G.V - 1 - wq;
    const int64_t b0 = segptr[r0];
    for (int mir = 1; mir < 4; ++mir) {
        const bool my = mir & 1, mz = mir & 2;
        if ((my && um == uq) || (mz && wm == wq)) continue;
        const int64_t r = (int64_t)(mz ? wm : wq) * G.U + (my ? um : uq);
        const int64_t b = segptr[r];
        for (int j = 0; j < n; ++j) {
            uint32_t x = sr[b0 + j];
            double a = pa[b0 + j], c = pb[b0 + j];
            seg::mirror_record(my, mz, G.nz, x, a, c);
            sr[b + j] = x;
            pa[b + j] = a;
            pb[b + j] = c;
            partner[b + j] = partner[b0 + j];
        }
    }
}

__global__ void max_u32(const uint32_t *v, int64_t n, unsigned int *mx)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) atomicMax(mx, v[i]);
}

// Rows of one view from the records: count pass (ids == nullptr) and fill.
struct RebinArgs {
    const int64_t *segptr;
    const uint32_t *sr;
    const double *pa, *pb;
    const int32_t *partner;
    const int32_t *ng;
    const int64_t *head;
    int64_t c2d, nrays;
    double theta;
};

struct CountEmit {
    __device__ void operator()(int64_t) {}
};

struct WriteEmit {
    uint32_t *ids;
    int64_t at;
    __device__ void operator()(int64_t cell) { ids[at++] = (uint32_t)cell; }
};

__device__ inline int wave_sum_i(int v)
{
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// One wavefront per ray: lane l takes records l, l + 64, ...
__global__ __launch_bounds__(256) void rebin_count(RebinArgs A, uint32_t *cnt)
{
    const int64_t r = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int lane = threadIdx.x & 63;
    if (r >= A.nrays) return;
    const int64_t b = A.segptr[r], n = A.segptr[r + 1] - b;
    int m = 0;
    CountEmit e;
    for (int64_t j = lane; j < n; j += 64)
        m += seg::rebin_record(A.sr + b, A.pa + b, A.pb + b, A.partner + b, j, A.ng, A.head, A.c2d, A.theta, e);
    m = wave_sum_i(m);
    if (lane == 0) cnt[r] = (uint32_t)m;
}

// Same assignment; each chunk of 64 records writes at the row offset plus
// the exclusive prefix of the lanes' counts, so cells stay in record order.
__global__ __launch_bounds__(256) void rebin_fill(RebinArgs A, const int64_t *rowptr, uint32_t *ids)
{
    const int64_t r = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int lane = threadIdx.x & 63;
    if (r >= A.nrays) return;
    const int64_t b = A.segptr[r], n = A.segptr[r + 1] - b;
    int64_t at = rowptr[r];
    for (int64_t j0 = 0; j0 < n; j0 += 64) {
        const int64_t j = j0 + lane;
        CountEmit ce;
        const int m = j < n ? seg::rebin_record(A.sr + b, A.pa + b, A.pb + b, A.partner + b, j, A.ng, A.head, A.c2d,
                                                A.theta, ce)
                            : 0;
        int incl = m;
        for (int off = 1; off < 64; off <<= 1) {
            const int o = __shfl_up(incl, off, 64);
            if (lane >= off) incl += o;
        }
        if (j < n) {
            WriteEmit we{ids, at + incl - m};
            seg::rebin_record(A.sr + b, A.pa + b, A.pb + b, A.partner + b, j, A.ng, A.head, A.c2d, A.theta, we);
        }
        at += __shfl(incl, 63, 64);
    }
}

TraceGeo geometry_of(const uspg_coeffs *c)
{
    const uspg_grid *g = c->g;
    const uspg_scan_desc &sc = c->scan;
    TraceGeo G{};
    G.nr = g->nr; G.nz = g->nz; G.is3d = sc.geometry == USPG_CONE_3D; G.geom = sc.geometry;
    G.R = g->R; G.r = g->r; G.h = g->h; G.z0 = g->z0; G.H = g->H;
    G.ng = g->d_ng.as<int32_t>();
    G.head = g->d_head.as<int64_t>();
    G.U = sc.det_u; G.V = sc.det_v;
    G.Wu = sc.det_half_u; G.Wv = sc.det_half_v; G.Dso = sc.src_axis; G.Dsd = sc.src_det;
    G.eps = 1e-12 * g->R;
    return G;
}

RebinArgs rebin_args(const uspg_coeffs *c, int view)
{
    RebinArgs A{};
    A.segptr = c->segptr.as<int64_t>();
    A.sr = c->seg_sr.as<uint32_t>();
    A.pa = c->seg_pa.as<double>();
    A.pb = c->seg_pb.as<double>();
    A.partner = c->seg_partner.as<int32_t>();
    A.ng = c->g->d_ng.as<int32_t>();
    A.head = c->g->d_head.as<int64_t>();
    A.c2d = c->g->c2d;
    A.nrays = c->nrays;
    A.theta = seg::view_angle(view, c->scan.span, c->scan.n_views);
    return A;
}

}  // namespace

int segments_reference_view(uspg_coeffs *c, hipStream_t s)
{
    const TraceGeo G = geometry_of(c);
    const int64_t nrays = c->nrays;
    const unsigned blocks = (unsigned)((nrays + 255) / 256);
    uint32_t *cnt = nullptr;
    unsigned int *mx = nullptr;
    if (dev_malloc((void **)&cnt, sizeof(uint32_t) * (nrays + 1)) != hipSuccess) return fail(USPG_E_NOMEM, "device allocation failed");
    if (dev_malloc((void **)&mx, sizeof(unsigned int)) != hipSuccess) {
        (void)dev_free(cnt);
        return fail(USPG_E_NOMEM, "segments: allocation failed");
    }
    int rc = USPG_OK;
    do {
        const bool quarter = c->scan.quarter != 0;
        const int uh = (c->scan.det_u + 1) / 2, vh = (c->scan.det_v + 1) / 2;
        const unsigned qblocks = (unsigned)(((int64_t)uh * vh + 255) / 256);
        if (quarter)
            hipLaunchKernelGGL(seg_count_q, dim3(qblocks), dim3(256), 0, s, G, uh, vh, cnt);
        else
            hipLaunchKernelGGL(seg_count, dim3(blocks), dim3(256), 0, s, G, nrays, cnt);
        if (hipGetLastError() != hipSuccess) { rc = fail(USPG_E_HIP, "seg_count launch failed"); break; }
        if ((rc = c->segptr.alloc(sizeof(int64_t) * (nrays + 1))) != USPG_OK) break;
        if ((rc = exclusive_scan_u32_to_i64(cnt, c->segptr.as<int64_t>(), nrays, s)) != USPG_OK) break;
        if (hipMemsetAsync(mx, 0, sizeof(unsigned int), s) != hipSuccess) { rc = fail(USPG_E_HIP, "memset"); break; }
        hipLaunchKernelGGL(max_u32, dim3(blocks), dim3(256), 0, s, cnt, nrays, mx);
        int64_t ns = 0;
        unsigned int mseg = 0;
        if (hipMemcpyAsync(&ns, c->segptr.as<int64_t>() + nrays, sizeof(int64_t), hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipMemcpyAsync(&mseg, mx, sizeof(unsigned int), hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess) {
            rc = fail(USPG_E_HIP, "segments: reading the record count failed");
            break;
        }
        c->nseg = ns;
        c->max_seg = (int32_t)mseg;
        const int64_t n1 = ns > 0 ? ns : 1;
        if ((rc = c->seg_sr.alloc(sizeof(uint32_t) * n1)) != USPG_OK) break;
        if ((rc = c->seg_pa.alloc(sizeof(double) * n1)) != USPG_OK) break;
        if ((rc = c->seg_pb.alloc(sizeof(double) * n1)) != USPG_OK) break;
        if ((rc = c->seg_partner.alloc(sizeof(int32_t) * n1)) != USPG_OK) break;
        if (quarter)
            hipLaunchKernelGGL(seg_fill_q, dim3(qblocks), dim3(256), 0, s, G, uh, vh, c->segptr.as<int64_t>(),
                               c->seg_sr.as<uint32_t>(), c->seg_pa.as<double>(), c->seg_pb.as<double>(),
                               c->seg_partner.as<int32_t>());
        else
            hipLaunchKernelGGL(seg_fill, dim3(blocks), dim3(256), 0, s, G, nrays, c->segptr.as<int64_t>(),
                               c->seg_sr.as<uint32_t>(), c->seg_pa.as<double>(), c->seg_pb.as<double>(),
                               c->seg_partner.as<int32_t>());
        if (hipGetLastError() != hipSuccess) { rc = fail(USPG_E_HIP, "seg_fill launch failed"); break; }
        if (hipStreamSynchronize(s) != hipSuccess) { rc = fail(USPG_E_HIP, "seg_fill failed"); break; }
    } while (0);
    (void)dev_free(cnt);
    (void)dev_free(mx);
    return rc;
}

// (cell, 1) pairs of a re-binned row set, for MART on kept rows.
__global__ __launch_bounds__(256) void ids_to_pairs(const uint32_t *ids, int64_t n, Coef<float> *out)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    Coef<float> e;
    e.id = ids[i];
    e.a = 1.0f;
    out[i] = e;
}

// Re-bins the rows of every view (counts first, for all views), ORs every
// view's conflicts into the mark map and chooses the lattice; with
// view_rows == 0 keeps the rows as (cell, 1) pairs when they fit.
int colour_segments(uspg_coeffs *c, hipStream_t s)
{
    const int U = c->scan.det_u, V = c->scan.det_v, p = c->scan.n_views;
    const int64_t nrays = c->nrays;
    const unsigned wblocks = (unsigned)((nrays * 64 + 255) / 256);   // one wavefront per ray
    c->mark.assign((size_t)U * V, 0);
    c->view_nnz.assign(p, 0);
    uint32_t *cnt = nullptr, *ids = nullptr;
    uint8_t *mark = nullptr;
    int rc = USPG_OK;
    do {
        if (dev_malloc((void **)&cnt, sizeof(uint32_t) * (nrays + 1)) != hipSuccess ||
            dev_malloc((void **)&mark, (size_t)U * V) != hipSuccess) {
            rc = fail(USPG_E_NOMEM, "segment colouring: allocation failed");
            break;
        }
        if ((rc = c->view_rowptr.alloc(sizeof(int64_t) * (size_t)p * (nrays + 1))) != USPG_OK) break;
        int64_t *vrp = c->view_rowptr.as<int64_t>();
        if (hipMemsetAsync(mark, 0, (size_t)U * V, s) != hipSuccess) { rc = fail(USPG_E_HIP, "memset"); break; }
        for (int v = 0; v < p && rc == USPG_OK; ++v) {
            hipLaunchKernelGGL(rebin_count, dim3(wblocks), dim3(256), 0, s, rebin_args(c, v), cnt);
            rc = exclusive_scan_u32_to_i64(cnt, vrp + (int64_t)v * (nrays + 1), nrays, s);
        }
        if (rc != USPG_OK) break;
        std::vector<int64_t> h_rp((size_t)p * (nrays + 1));
        if (hipMemcpyAsync(h_rp.data(), vrp, sizeof(int64_t) * h_rp.size(), hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess) {
            rc = fail(USPG_E_HIP, "segment colouring: reading the row counts failed");
            break;
        }
        int64_t total = 0, longest = 0, widest = 1;
        c->view_start.assign(p + 1, 0);
        for (int v = 0; v < p; ++v) {
            const int64_t *rp = h_rp.data() + (size_t)v * (nrays + 1);
            c->view_nnz[v] = rp[nrays];
            widest = std::max<int64_t>(widest, rp[nrays]);
            for (int64_t r = 0; r < nrays; ++r) longest = std::max<int64_t>(longest, rp[r + 1] - rp[r]);
            total += rp[nrays];
            c->view_start[v + 1] = total;
        }
        const bool keep = c->scan.view_rows == 0 &&
                          total * (int64_t)sizeof(Coef<float>) + (int64_t)c->view_rowptr.bytes <= USPG_VIEW_ROWS_MAX_BYTES;
        if (keep && (rc = c->view_coef.alloc(sizeof(Coef<float>) * (size_t)std::max<int64_t>(total, 1))) != USPG_OK)
            break;
        c->view_max_row = (int32_t)longest;
        if (dev_malloc((void **)&ids, sizeof(uint32_t) * (size_t)widest) != hipSuccess) {
            rc = fail(USPG_E_NOMEM, "segment colouring: allocation failed");
            break;
        }
        for (int v = 0; v < p && rc == USPG_OK; ++v) {
            const int64_t nnz = c->view_nnz[v];
            const int64_t *rowptr = vrp + (int64_t)v * (nrays + 1);
            hipLaunchKernelGGL(rebin_fill, dim3(wblocks), dim3(256), 0, s, rebin_args(c, v), rowptr, ids);
            if (hipGetLastError() != hipSuccess) { rc = fail(USPG_E_HIP, "rebin launch failed"); break; }
            if (keep && nnz > 0)
                hipLaunchKernelGGL(ids_to_pairs, dim3((unsigned)((nnz + 255) / 256)), dim3(256), 0, s, ids, nnz,
                                   c->view_coef.as<Coef<float>>() + c->view_start[v]);
            rc = conflict_marks(rowptr, ids, 1, nrays, nnz, c->g->ncells, U, mark, s);
        }
        if (rc != USPG_OK) break;
        if (hipMemcpy(c->mark.data(), mark, (size_t)U * V, hipMemcpyDeviceToHost) != hipSuccess)
            rc = fail(USPG_E_HIP, "segment colouring: copy failed");
        if (keep && rc == USPG_OK) {
            if ((rc = c->d_view_start.alloc(sizeof(int64_t) * (p + 1))) == USPG_OK &&
                hipMemcpy(c->d_view_start.p, c->view_start.data(), sizeof(int64_t) * (p + 1),
                          hipMemcpyHostToDevice) != hipSuccess)
                rc = fail(USPG_E_HIP, "segment colouring: copy failed");
        }
        if (!keep) c->view_rowptr.release();
    } while (0);
    (void)hipStreamSynchronize(s);
    (void)dev_free(cnt); (void)dev_free(ids); (void)dev_free(mark);
    if (rc != USPG_OK) return rc;
    return choose_lattice(c);
}

int segments_row(const uspg_coeffs *c, int view, int64_t ray, std::vector<int64_t> &cells)
{
    int64_t sp[2];
    USPG_HIP(hipMemcpy(sp, c->segptr.as<int64_t>() + ray, sizeof(sp), hipMemcpyDeviceToHost));
    const int64_t n = sp[1] - sp[0];
    cells.clear();
    if (n == 0) return USPG_OK;
    std::vector<uint32_t> sr(n);
    std::vector<double> pa(n), pb(n);
    std::vector<int32_t> partner(n);
    USPG_HIP(hipMemcpy(sr.data(), c->seg_sr.as<uint32_t>() + sp[0], sizeof(uint32_t) * n, hipMemcpyDeviceToHost));
    USPG_HIP(hipMemcpy(pa.data(), c->seg_pa.as<double>() + sp[0], sizeof(double) * n, hipMemcpyDeviceToHost));
    USPG_HIP(hipMemcpy(pb.data(), c->seg_pb.as<double>() + sp[0], sizeof(double) * n, hipMemcpyDeviceToHost));
    USPG_HIP(hipMemcpy(partner.data(), c->seg_partner.as<int32_t>() + sp[0], sizeof(int32_t) * n,
                       hipMemcpyDeviceToHost));
    const uspg_grid *g = c->g;
    const double theta = seg::view_angle(view, c->scan.span, c->scan.n_views);
    auto emit = [&cells](int64_t cell) { cells.push_back(cell); };
    seg::rebin_cells(sr.data(), pa.data(), pb.data(), partner.data(), n, g->ng.data(), g->head.data(), g->c2d,
                     theta, emit);
    std::sort(cells.begin(), cells.end());
    return USPG_OK;
}

}  // namespace uspg
