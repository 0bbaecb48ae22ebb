// The paper's literal coefficient scheme on the device: MART over rows
// rebuilt per view from the reference view's segment records (Sec. III.B-C,
// the per-view part of Alg. 1, eqs. 10-18; records and re-binning in segments.hpp).
#include <algorithm>

#include "mart_row.hpp"
#include "segments.hpp"
#include "uspg_internal.hpp"

namespace uspg {
namespace {

using row::Bits;
using row::max_rel_change;
using row::xcd_block;

constexpr int kWaves = 4;             // wavefronts per workgroup
constexpr int kBlock = 64 * kWaves;

// The paper's literal variant: one (view, class) batch with each ray's row
// rebuilt from its segment records (segments.hpp).  A record meets a run of
// sectors of one ring and slice, minus those its partner record (the line's
// other pass through that ring and slice) already met.  Binary coefficients:
// Pbar is the sum of f over the row and every cell gets the same factor
// 1 + beta (P / Pbar - 1) (eq. 18 with a_j = a_max = 1).  The image is in the
// paper's numbering.
//
// A group of G lanes (32, 64 or the whole workgroup of 256, picked per
// coefficient set) takes one ray (a wavefront holds 64 / G rays when
// G <= 64); lane l of a group takes records l, l + G, ...  The runs of a lane's first
// kRebinNR records and up to kRebinNS of their gathered values stay in
// registers between the gather and the scatter; what does not fit is
// rebuilt in the second pass.  Every gather of the register part is issued
// before the first wait (invalid entries read cell 0 and are masked).
template <class T>
struct RebinMartArgs {
    const int64_t *segptr;
    const uint32_t *sr;
    const double *pa, *pb;
    const int32_t *partner;
    const int32_t *ng;
    const int64_t *head;
    int64_t c2d;
    const T *P;
    T *f;
    double theta;
    int U, cu, cw, Ku, Kv, nu, ncls, nblk;
    T beta;
};

constexpr int kRebinNR = 2;           // records per lane kept in registers
constexpr int kRebinNS = 4;           // sectors per record kept in registers

template <class T>
struct SumEmit {
    const T *f;
    T acc;
    int m;
    __device__ void operator()(int64_t cell)
    {
        acc += f[cell];
        ++m;
    }
};

template <class T>
struct ScaleEmit {
    T *f;
    T g;
    __device__ void operator()(int64_t cell) { f[cell] = f[cell] * g; }
};

// Sum over a ray's group of G lanes.  G <= 64: xor butterfly inside the
// wavefront.  G = 256 (the workgroup): butterfly per wavefront, then the
// four wavefront sums added in wavefront order through LDS (every lane gets
// the same value; the caller's workgroup reaches the barrier as a whole).
template <class V, int G>
__device__ inline V group_sum(V v, V *lds)
{
    constexpr int W = G < 64 ? G : 64;
#pragma unroll
    for (int off = W / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    if constexpr (G > 64) {
        if ((threadIdx.x & 63) == 0) lds[threadIdx.x >> 6] = v;
        __syncthreads();
        v = lds[0];
#pragma unroll
        for (int w = 1; w < G / 64; ++w) v += lds[w];
    }
    return v;
}

template <class T, int G>
__global__ __launch_bounds__(kBlock) void mart_rebin(RebinMartArgs<T> A)
{
#pragma clang fp contract(off)
    static_assert(G == 32 || G == 64 || G == kBlock, "lanes per ray");
    constexpr int NR = kRebinNR, NS = kRebinNS;
    __shared__ T red_acc[kWaves];
    __shared__ int red_m[kWaves];
    int sub, x;
    if constexpr (G == kBlock) {
        // one ray per workgroup (n is then uniform over the workgroup, so
        // every lane reaches the barriers of group_sum or none does)
        sub = threadIdx.x;
        x = xcd_block(blockIdx.x, A.nblk);
    } else {
        constexpr int RPW = 64 / G;
        const int lane = threadIdx.x & 63;
        sub = lane & (G - 1);
        x = (xcd_block(blockIdx.x, A.nblk) * kWaves + (threadIdx.x >> 6)) * RPW + lane / G;
    }
    int64_t r = 0, b = 0;
    int n = 0;
    if (x < A.ncls) {
        const int w = A.cw + (x / A.nu) * A.Kv;
        const int u = A.cu + (x % A.nu) * A.Ku;
        r = (int64_t)w * A.U + u;
        b = A.segptr[r];
        n = (int)(A.segptr[r + 1] - b);
    }
    if (!__any(n > 0)) return;
    const T Pr = n > 0 ? A.P[r] : T(0);
    const uint32_t *sr = A.sr + b;
    const double *pa = A.pa + b, *pb = A.pb + b;
    const int32_t *pt = A.partner + b;

    seg::RecordRange rr[NR];
    int64_t cell[NR][NS];
    bool ok[NR][NS];
#pragma unroll
    for (int k = 0; k < NR; ++k) {
        const int j = sub + k * G;
        if (j < n) {
            rr[k] = seg::record_range(sr, pa, pb, pt, j, A.ng, A.head, A.c2d, A.theta);
        } else {
            rr[k].first = rr[k].pf = rr[k].pc = 0;
            rr[k].count = 0;
            rr[k].ng = 1;
            rr[k].base = 0;
        }
#pragma unroll
        for (int q = 0; q < NS; ++q) {
            const int s = q < rr[k].count ? seg::range_sector(rr[k], q) : -1;
            ok[k][q] = s >= 0;
            cell[k][q] = s >= 0 ? rr[k].base + s : 0;
        }
    }
    T val[NR][NS];
#pragma unroll
    for (int k = 0; k < NR; ++k)
#pragma unroll
        for (int q = 0; q < NS; ++q) val[k][q] = A.f[cell[k][q]];
    SumEmit<T> se{A.f, T(0), 0};
#pragma unroll
    for (int k = 0; k < NR; ++k)
#pragma unroll
        for (int q = 0; q < NS; ++q)
            if (ok[k][q]) {
                se.acc += val[k][q];
                ++se.m;
            }
    // runs longer than NS, and records beyond the first NR per lane
#pragma unroll
    for (int k = 0; k < NR; ++k)
        if (rr[k].count > NS) seg::emit_range(rr[k], NS, se);
    for (int j = sub + NR * G; j < n; j += G)
        seg::rebin_record(sr, pa, pb, pt, j, A.ng, A.head, A.c2d, A.theta, se);
    const T acc = group_sum<T, G>(se.acc, red_acc);
    const int m = group_sum<int, G>(se.m, red_m);
    if (n == 0 || m == 0 || !(acc > T(0))) return;
    ScaleEmit<T> ue{A.f, T(1) + A.beta * (Pr / acc - T(1))};
#pragma unroll
    for (int k = 0; k < NR; ++k)
#pragma unroll
        for (int q = 0; q < NS; ++q)
            if (ok[k][q]) A.f[cell[k][q]] = val[k][q] * ue.g;
#pragma unroll
    for (int k = 0; k < NR; ++k)
        if (rr[k].count > NS) seg::emit_range(rr[k], NS, ue);
    for (int j = sub + NR * G; j < n; j += G)
        seg::rebin_record(sr, pa, pb, pt, j, A.ng, A.head, A.c2d, A.theta, ue);
}

template <class T>
int run_segments(const uspg_coeffs *c, const T *proj, T *image, void *work, int n_sweeps, double beta,
                 double tol, int32_t *sweeps_done, hipStream_t s)
{
    const uspg_grid *g = c->g;
    const uint32_t ncells = (uint32_t)g->ncells;
    T *f = static_cast<T *>(work);
    T *old = tol > 0 ? f + ncells : nullptr;
    using UB = typename Bits<T>::U;
    UB *mx = tol > 0 ? reinterpret_cast<UB *>(old + ncells) : nullptr;
    USPG_HIP(hipMemcpyAsync(f, image, sizeof(T) * ncells, hipMemcpyDeviceToDevice, s));
    RebinMartArgs<T> A{};
    A.segptr = c->segptr.as<int64_t>();
    A.sr = c->seg_sr.as<uint32_t>();
    A.pa = c->seg_pa.as<double>();
    A.pb = c->seg_pb.as<double>();
    A.partner = c->seg_partner.as<int32_t>();
    A.ng = g->d_ng.as<int32_t>();
    A.head = g->d_head.as<int64_t>();
    A.c2d = g->c2d;
    A.f = f;
    A.U = c->scan.det_u;
    A.Ku = c->Ku; A.Kv = c->Kv;
    A.beta = (T)beta;
    const int K = c->Ku * c->Kv;
    const unsigned pb = (ncells + 255) / 256;
    // Lanes per ray, measured on the paper's scans (Tables 1 and 3; us per
    // launch for 32 / 64 / 256 lanes):
    //  - 256 (one ray per workgroup) when a class has few rays and they are
    //    long: fan scans, 101 rays of 123-490 records (1024^2: 75.2 / 44.7 /
    //    29.2; 256^2: 17.2 at 64, 15.9 at 256); Cu-lump geometry, 1,133 rays
    //    per class of 101 records (16.9 / 10.4 / 10.3);
    //  - 32 when a ray's records fit two per lane on average, a class has
    //    enough rays to fill the chip at two rays per wavefront, and the
    //    image stays in cache: 128^3 cone (20.1 / 24.7 / 40.3);
    //  - else 64: the 256^3 frog geometry (75.8 / 67.2 / 100.2), whose 67 MB
    //    image makes the kernel bound by its scattered line traffic, where
    //    one ray per wavefront keeps the lines of each load together.
    // 16 lanes per ray was slower on every scan.
    const int64_t mean = c->nrays > 0 ? (c->nseg + c->nrays - 1) / c->nrays : 0;
    const int64_t class_rays = c->nrays / K;
    const bool small_image = (int64_t)ncells * (int64_t)sizeof(T) <= (int64_t(32) << 20);
    const int G = class_rays < 2048 && mean > 64                           ? kBlock
                  : mean <= 2 * 32 && class_rays >= 4096 && small_image ? 32
                                                                          : 64;
    const int rays_per_block = G == kBlock ? 1 : kWaves * (64 / G);
    int done = 0;
    const bool timing = mart_timing_on(s) && tol == 0;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    int64_t launches = 0;
    if (timing) {
        USPG_HIP(hipEventCreate(&ev0));
        USPG_HIP(hipEventCreate(&ev1));
        USPG_HIP(hipEventRecord(ev0, s));
    }
    const bool kept = c->view_coef.p != nullptr;
    for (int sw = 0; sw < n_sweeps; ++sw) {
        if (tol > 0) USPG_HIP(hipMemcpyAsync(old, f, sizeof(T) * ncells, hipMemcpyDeviceToDevice, s));
        for (int v = 0; v < c->scan.n_views; ++v) {
            A.P = proj + (int64_t)v * c->nrays;
            A.theta = seg::view_angle(v, c->scan.span, c->scan.n_views);
            if (kept) {
                // the view's re-binned rows, kept as (cell, 1) pairs: the
                // stored-row kernel with no shift (eq. 18 with a_j = a_max = 1)
                const int64_t *rp = c->view_rowptr.as<int64_t>() + (int64_t)v * (c->nrays + 1);
                const Coef<float> *co = c->view_coef.as<Coef<float>>() + c->view_start[v];
                for (int cl = 0; cl < K; ++cl) {
                    const int rc = rows_batch_launch(c, sizeof(T) == sizeof(double) ? USPG_F64 : USPG_F32, A.P, f,
                                                     rp, co, 0u, ncells, cl, beta, c->view_max_row, s);
                    if (rc != USPG_OK) return rc;
                    ++launches;
                }
                continue;
            }
            for (int cl = 0; cl < K; ++cl) {
                A.cu = cl % c->Ku;
                A.cw = cl / c->Ku;
                A.nu = (c->scan.det_u - A.cu + c->Ku - 1) / c->Ku;
                const int nw = (c->scan.det_v - A.cw + c->Kv - 1) / c->Kv;
                A.ncls = A.nu * nw;
                A.nblk = (A.ncls + rays_per_block - 1) / rays_per_block;
                if (A.ncls == 0) continue;
                if (G == 32)
                    hipLaunchKernelGGL((mart_rebin<T, 32>), dim3(A.nblk), dim3(kBlock), 0, s, A);
                else if (G == kBlock)
                    hipLaunchKernelGGL((mart_rebin<T, kBlock>), dim3(A.nblk), dim3(kBlock), 0, s, A);
                else
                    hipLaunchKernelGGL((mart_rebin<T, 64>), dim3(A.nblk), dim3(kBlock), 0, s, A);
                ++launches;
            }
        }
        USPG_HIP(hipGetLastError());
        ++done;
        if (tol > 0) {
            USPG_HIP(hipMemsetAsync(mx, 0, sizeof(UB), s));
            unsigned nb = pb < 4096 ? pb : 4096;
            hipLaunchKernelGGL(max_rel_change<T>, dim3(nb), dim3(256), 0, s, f, old, ncells, mx);
            UB hb = 0;
            USPG_HIP(hipMemcpyAsync(&hb, mx, sizeof(UB), hipMemcpyDeviceToHost, s));
            USPG_HIP(hipStreamSynchronize(s));
            T hv;
            __builtin_memcpy(&hv, &hb, sizeof(hv));
            if ((double)hv <= tol) break;
        }
    }
    if (timing) {
        USPG_HIP(hipEventRecord(ev1, s));
        USPG_HIP(hipEventSynchronize(ev1));
        float ms = 0.f;
        USPG_HIP(hipEventElapsedTime(&ms, ev0, ev1));
        mart_timing_add(s, (int64_t)((double)ms * 1e6), launches);
        (void)hipEventDestroy(ev0);
        (void)hipEventDestroy(ev1);
    }
    USPG_HIP(hipMemcpyAsync(image, f, sizeof(T) * ncells, hipMemcpyDeviceToDevice, s));
    if (sweeps_done) *sweeps_done = done;
    return USPG_OK;
}

}  // namespace

int rebin_launch(const uspg_coeffs *c, int dtype, const void *proj, void *image, void *work, int n_sweeps,
                 double beta, double tol, int32_t *sweeps_done, hipStream_t s)
{
    if (dtype == USPG_F32)
        return run_segments<float>(c, (const float *)proj, (float *)image, work, n_sweeps, beta, tol, sweeps_done, s);
    return run_segments<double>(c, (const double *)proj, (double *)image, work, n_sweeps, beta, tol, sweeps_done, s);
}

}  // namespace uspg
