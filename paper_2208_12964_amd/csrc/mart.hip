// Sp-MART on the device (Sec. III.D, eqs. 17-19).
//
// The image lives in the wedge-major layout during the solve, so the rows of
// view v are the reference rows with every cell id shifted by v * Wc modulo
// the image size (one add and one conditional subtract per coefficient).
// One batch = one (view, colour class): all rays of the class are cell
// disjoint, so each wavefront takes one ray and updates its cells without
// atomics, exactly as if the rays were applied one after another.
//
// Per ray (wavefront of 64 lanes, lane j handles coefficients j, j+64, ...):
//   load ids / coefficients (coalesced), rotate ids, gather f,
//   Pbar = sum a f and a_max by wavefront reductions (fixed order),
//   c = beta (P / Pbar - 1) / a_max,  f_j <- f_j (1 + c a_j)   (eq. 18).
// Rows up to 64 * 16 coefficients (64 * 32 for coefficient sets whose
// longest row needs it) stay in registers between the gather and the
// scatter; longer rows are re-read in a second pass.
#include <algorithm>
#include <atomic>
#include <mutex>
#include <unordered_map>

#include "mart_batch.hpp"
#include "mart_coded.hpp"
#include "mart_row.hpp"
#include "uspg_internal.hpp"

namespace uspg {
namespace {

using row::Bits;
using row::mart_row;
using row::max_rel_change;
using row::xcd_block;
using row::wave_max;
using row::wave_sum;

using batchk::BatchArgs;
using batchk::CodedArgs;
using batchk::mart_batch;
using batchk::mart_coded;
using batchk::mart_explicit;
constexpr int kWaves = batchk::kWaves;
constexpr int kBlock = batchk::kBlock;
// Grid cap of the batch kernels, in workgroups per compute unit: measured on
// the 256-ring cone (43,690 rays per class), 16 per CU (4,096 on 256 CUs)
// gave 122 us per batch against 135 us for one wavefront per ray with
// stored rows, 8, 12, 20, 24 and 32 per CU 128-150 us; with coded rows 16
// per CU gives 79 us, 8 / 12 / 24 per CU 87 / 86 / 94 us.  Classes of fewer
// rays are not capped.
constexpr int kBlocksPerCU = 16;

int grid_cap()
{
    static int cap[64] = {0};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 1 << 30;
    if (!cap[dev]) {
        int cus = 0;
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
            cus = 256;
        cap[dev] = kBlocksPerCU * cus;
    }
    return cap[dev];
}

// Layout maps between the paper's numbering and the wedge-major layout.
struct LayoutArgs {
    const int32_t *ring_of_off, *kq, *hq;
    const int64_t *head;
    uint32_t Cq, Wc, c2d, wtot, grp;
};

// Paper index of device index x, or -1 for a padding slot of the layout.
__device__ inline int64_t native_to_paper(uint32_t x, const LayoutArgs &L)
{
    uint32_t aw = x / L.Wc;
    uint32_t rem = x - aw * L.Wc;
    uint32_t k = rem / L.Cq;
    uint32_t o = rem - k * L.Cq;
    int i = L.ring_of_off[o];
    if (i < 0) return -1;
    uint32_t b = (o - (uint32_t)L.hq[i]) / L.grp;
    uint32_t s = aw * (uint32_t)L.kq[i] + b;
    return (int64_t)k * L.c2d + L.head[i] + s;
}

// Padding slots are set to 1 (never touched by a ray, neutral for eq. 19).
template <class T>
__global__ __launch_bounds__(256) void to_native(LayoutArgs L, const T *paper, T *native)
{
    uint32_t x = blockIdx.x * 256u + threadIdx.x;
    if (x >= L.wtot) return;
    int64_t p = native_to_paper(x, L);
    native[x] = p < 0 ? T(1) : paper[p];
}

template <class T>
__global__ __launch_bounds__(256) void to_paper(LayoutArgs L, const T *native, T *paper)
{
    uint32_t x = blockIdx.x * 256u + threadIdx.x;
    if (x >= L.wtot) return;
    int64_t p = native_to_paper(x, L);
    if (p >= 0) paper[p] = native[x];
}

template <class T, class TC, int NCH, bool NT>
void launch_batch(const BatchArgs<T, TC> &A, hipStream_t s)
{
    hipLaunchKernelGGL((mart_batch<T, TC, NCH, NT>), dim3(A.nblk), dim3(kBlock), 0, s, A);
}

template <class T, class TC, bool NT>
void launch_batch_nch(int nch, const BatchArgs<T, TC> &A, hipStream_t s)
{
    // the instantiation bounds the register path; longer rows stream
    if (nch <= 2) launch_batch<T, TC, 2, NT>(A, s);
    else if (nch <= 4) launch_batch<T, TC, 4, NT>(A, s);
    else if (nch <= 8) launch_batch<T, TC, 8, NT>(A, s);
    else if (nch <= 16) launch_batch<T, TC, 16, NT>(A, s);
    else launch_batch<T, TC, 32, NT>(A, s);
}

template <class T, class TC>
void launch_batch_n(int nch, bool nt, const BatchArgs<T, TC> &A, hipStream_t s)
{
    if (nt) launch_batch_nch<T, TC, true>(nch, A, s);
    else launch_batch_nch<T, TC, false>(nch, A, s);
}

// Coded rows: the instantiation bounds the register path (coded rows have
// at most 16 chunks); the explicit rows of a set, if any, run in a second
// launch per batch with the stored-row cache rule.
template <class T, class TC>
void launch_coded(int nch, const CodedArgs<T, TC> &A, hipStream_t s)
{
    const coded::RayCode *codes = A.K.codes;
    const uint64_t *words = A.K.words;
    const dim3 g(A.B.nblk), blk(kBlock);
    if (nch <= 2) hipLaunchKernelGGL((mart_coded<T, TC, 2>), g, blk, 0, s, A, codes, words, A.B.P);
    else if (nch <= 4) hipLaunchKernelGGL((mart_coded<T, TC, 4>), g, blk, 0, s, A, codes, words, A.B.P);
    else if (nch <= 8) hipLaunchKernelGGL((mart_coded<T, TC, 8>), g, blk, 0, s, A, codes, words, A.B.P);
    else if (nch <= 12) hipLaunchKernelGGL((mart_coded<T, TC, 12>), g, blk, 0, s, A, codes, words, A.B.P);
    else hipLaunchKernelGGL((mart_coded<T, TC, 16>), g, blk, 0, s, A, codes, words, A.B.P);
}

template <class T, class TC, bool NT>
void launch_explicit(int nch, const CodedArgs<T, TC> &A, hipStream_t s)
{
    if (nch <= 4) hipLaunchKernelGGL((mart_explicit<T, TC, 4, NT>), dim3(A.B.nblk), dim3(kBlock), 0, s, A);
    else if (nch <= 16) hipLaunchKernelGGL((mart_explicit<T, TC, 16, NT>), dim3(A.B.nblk), dim3(kBlock), 0, s, A);
    else hipLaunchKernelGGL((mart_explicit<T, TC, 32, NT>), dim3(A.B.nblk), dim3(kBlock), 0, s, A);
}

}  // namespace

batchk::CodeTab code_tab(const uspg_coeffs *c)
{
    batchk::CodeTab K{};
    if (!c->coded) return K;
    K.codes = c->d_codes.as<coded::RayCode>();
    K.words = c->d_words.as<uint64_t>();
    K.t = c->d_colt.as<double>();
    K.id0 = c->d_colid.as<uint32_t>();
    K.Q = coded::CodeGeo{c->g->z0, c->g->h, c->g->nz, (uint32_t)c->Cq, (uint32_t)c->Wc};
    K.binary = c->scan.weights == USPG_WEIGHTS_BINARY;
    return K;
}

namespace {

// Ray order of the coded kernel inside a class: bands of 8 class rows,
// w fastest inside a band, so that the rays in flight on one XCD share
// their columns' in-plane paths (cache-resident) while neighbouring columns
// still share image lines.  Measured on the 256-ring cone (us per batch):
// band 1 (row order) 103, 2: 104, 4: 100, 8: 98, 16: 106, 32: 125, the
// whole class column-major 155.
constexpr int kCodedBand = 8;

template <class T, class TC>
CodedArgs<T, TC> coded_args(const uspg_coeffs *c, const BatchArgs<T, TC> &B)
{
    CodedArgs<T, TC> A{};
    A.B = B;
    A.K = code_tab(c);
    A.band = kCodedBand;
    return A;
}

// One (view, class) batch of a single problem: the coded kernel when the
// coefficient set has coded rows, else the stored-row kernel.
template <class T, class TC>
void launch_step(const uspg_coeffs *c, int nch, bool nt, const BatchArgs<T, TC> &B, hipStream_t s)
{
    if (c->coded) {
        const CodedArgs<T, TC> A = coded_args<T, TC>(c, B);
        launch_coded<T, TC>(std::min(nch, 16), A, s);
        if (c->explicit_rays > 0) {
            if (nt) launch_explicit<T, TC, true>(nch, A, s);
            else launch_explicit<T, TC, false>(nch, A, s);
        }
    } else {
        launch_batch_n<T, TC>(nch, nt, B, s);
    }
}

int pick_nch(int max_row) { return (max_row + 63) / 64; }

// Coefficient loads take the non-temporal hint unless the coefficient set and
// the image together fit comfortably in the 256 MiB last-level cache; then
// the set, read again in every view, stays cached.  Measured (MI355X, FP32,
// same bits either way): 128-ring cone, 110 MB of coefficients and a 27 MB
// image, 19.0 us per batch with the hint and 14.4 without; 256-ring cone,
// 876 MB and 215 MB, 111.2 us with the hint and 121.2 without.  The 192 MiB
// bound between them is a choice, not a measured crossover.
constexpr size_t kCacheResidentBytes = size_t(192) << 20;

// Arguments of batch (view v, class cl) of problem c on the wedge-major
// image f: the class's rays, the view's projections and shift, and the
// capped grid.
template <class T, class TC>
BatchArgs<T, TC> batch_args(const uspg_coeffs *c, const T *proj, T *f, double beta, int v, int cl)
{
    BatchArgs<T, TC> A{};
    A.rowptr = c->rowptr.as<int64_t>();
    A.co = c->coef.as<Coef<TC>>();
    A.f = f;
    A.wtot = (uint32_t)c->Wtot;
    A.U = c->scan.det_u;
    A.Ku = c->Ku; A.Kv = c->Kv;
    A.beta = (T)beta;
    A.P = proj + (int64_t)v * c->nrays;
    A.shift = (uint32_t)(((int64_t)v * c->Wc) % c->Wtot);
    A.cu = cl % c->Ku;
    A.cw = cl / c->Ku;
    A.nu = (c->scan.det_u - A.cu + c->Ku - 1) / c->Ku;
    const int nw = (c->scan.det_v - A.cw + c->Kv - 1) / c->Kv;
    A.ncls = A.nu * nw;
    A.nblk = (A.ncls + kWaves - 1) / kWaves;
    const int cap = grid_cap();
    if (A.nblk > cap) A.nblk = cap;
    return A;
}


template <class T, class TC>
int run_typed(const uspg_coeffs *c, const T *proj, T *image, void *work, int n_sweeps, double beta,
              double tol, int32_t *sweeps_done, hipStream_t s)
{
    const uspg_grid *g = c->g;
    const uint32_t ncells = (uint32_t)c->Wtot;   // device layout, padded
    T *nat = static_cast<T *>(work);
    T *old = tol > 0 ? nat + ncells : nullptr;
    using UB = typename Bits<T>::U;
    UB *mx = tol > 0 ? reinterpret_cast<UB *>(old + ncells) : nullptr;

    LayoutArgs L;
    L.ring_of_off = c->d_ring_of_off.as<int32_t>();
    L.kq = c->d_kq.as<int32_t>();
    L.hq = c->d_hq.as<int32_t>();
    L.head = g->d_head.as<int64_t>();
    L.Cq = (uint32_t)c->Cq; L.Wc = (uint32_t)c->Wc; L.c2d = (uint32_t)g->c2d; L.wtot = ncells;
    L.grp = (uint32_t)c->grp;
    const unsigned pb = (ncells + 255) / 256;
    hipLaunchKernelGGL(to_native<T>, dim3(pb), dim3(256), 0, s, L, image, nat);

    const int nch = pick_nch(c->max_row);
    const bool nt = stream_coefs(c->coef.bytes, sizeof(T) * (size_t)ncells);
    const int K = c->Ku * c->Kv;
    int done = 0;
    const bool timing = mart_timing_on(s) && tol == 0;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    int64_t launches = 0;
    if (timing) {
        USPG_HIP(hipEventCreate(&ev0));
        USPG_HIP(hipEventCreate(&ev1));
        USPG_HIP(hipEventRecord(ev0, s));
    }
    for (int sw = 0; sw < n_sweeps; ++sw) {
        if (tol > 0) USPG_HIP(hipMemcpyAsync(old, nat, sizeof(T) * ncells, hipMemcpyDeviceToDevice, s));
        for (int v = 0; v < c->scan.n_views; ++v) {
            for (int cl = 0; cl < K; ++cl) {
                const BatchArgs<T, TC> A = batch_args<T, TC>(c, proj, nat, beta, v, cl);
                if (A.ncls == 0) continue;
                launch_step<T, TC>(c, nch, nt, A, s);
                ++launches;
            }
        }
        USPG_HIP(hipGetLastError());
        ++done;
        if (tol > 0) {
            USPG_HIP(hipMemsetAsync(mx, 0, sizeof(UB), s));
            unsigned nb = pb < 4096 ? pb : 4096;
            hipLaunchKernelGGL(max_rel_change<T>, dim3(nb), dim3(256), 0, s, nat, old, ncells, mx);
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
    hipLaunchKernelGGL(to_paper<T>, dim3(pb), dim3(256), 0, s, L, nat, image);
    USPG_HIP(hipGetLastError());
    if (sweeps_done) *sweeps_done = done;
    return USPG_OK;
}


}  // namespace

int layout_permute(const uspg_coeffs *c, int dtype, const void *src, void *dst, int to_native_layout,
                   hipStream_t s)
{
    const uspg_grid *g = c->g;
    if (c->segments) {   // segment-record solves work in the paper's numbering
        USPG_HIP(hipMemcpyAsync(dst, src, (dtype == USPG_F64 ? sizeof(double) : sizeof(float)) * (size_t)g->ncells,
                                hipMemcpyDeviceToDevice, s));
        return USPG_OK;
    }
    LayoutArgs L;
    L.ring_of_off = c->d_ring_of_off.as<int32_t>();
    L.kq = c->d_kq.as<int32_t>();
    L.hq = c->d_hq.as<int32_t>();
    L.head = g->d_head.as<int64_t>();
    L.Cq = (uint32_t)c->Cq; L.Wc = (uint32_t)c->Wc; L.c2d = (uint32_t)g->c2d; L.wtot = (uint32_t)c->Wtot;
    L.grp = (uint32_t)c->grp;
    const unsigned pb = (unsigned)((c->Wtot + 255) / 256);
    if (dtype == USPG_F64) {
        if (to_native_layout)
            hipLaunchKernelGGL(to_native<double>, dim3(pb), dim3(256), 0, s, L, (const double *)src, (double *)dst);
        else
            hipLaunchKernelGGL(to_paper<double>, dim3(pb), dim3(256), 0, s, L, (const double *)src, (double *)dst);
    } else {
        if (to_native_layout)
            hipLaunchKernelGGL(to_native<float>, dim3(pb), dim3(256), 0, s, L, (const float *)src, (float *)dst);
        else
            hipLaunchKernelGGL(to_paper<float>, dim3(pb), dim3(256), 0, s, L, (const float *)src, (float *)dst);
    }
    USPG_HIP(hipGetLastError());
    return USPG_OK;
}

bool stream_coefs(size_t coef_bytes, size_t image_bytes) { return coef_bytes + image_bytes > kCacheResidentBytes; }

bool stream_capturing(hipStream_t s)
{
    hipStreamCaptureStatus st = hipStreamCaptureStatusNone;
    return hipStreamIsCapturing(s, &st) == hipSuccess && st != hipStreamCaptureStatusNone;
}

// Calls of the allocation-free entry point on this thread are not timed
// (timing creates events).
thread_local bool t_untimed = false;

UntimedScope::UntimedScope() : prev(t_untimed) { t_untimed = true; }
UntimedScope::~UntimedScope() { t_untimed = prev; }

// Timing records and waits on events, which a stream under graph capture
// cannot do: captured calls are not timed.
// Batch-kernel timing (uspg_mart_timing), kept per stream.
namespace {
struct TimingAcc {
    bool on = false;
    int64_t ns = 0, launches = 0;
};
std::mutex g_timing_mu;
std::unordered_map<hipStream_t, TimingAcc> g_timing;
}  // namespace

bool mart_timing_on(hipStream_t s)
{
    if (t_untimed) return false;
    {
        std::lock_guard<std::mutex> lk(g_timing_mu);
        auto it = g_timing.find(s);
        if (it == g_timing.end() || !it->second.on) return false;
    }
    return !stream_capturing(s);
}

void mart_timing_add(hipStream_t s, int64_t ns, int64_t launches)
{
    std::lock_guard<std::mutex> lk(g_timing_mu);
    TimingAcc &a = g_timing[s];
    a.ns += ns;
    a.launches += launches;
}

int mart_timing(int enable, hipStream_t s, double *batch_ms, int64_t *batch_launches)
{
    std::lock_guard<std::mutex> lk(g_timing_mu);
    TimingAcc &a = g_timing[s];
    if (enable) {
        a.ns = 0;
        a.launches = 0;
    }
    a.on = enable != 0;
    if (batch_ms) *batch_ms = (double)a.ns * 1e-6;
    if (batch_launches) *batch_launches = a.launches;
    if (!enable) g_timing.erase(s);
    return USPG_OK;
}

int rows_batch_launch(const uspg_coeffs *c, int dtype, const void *proj_view, void *f, const int64_t *rowptr,
                      const void *coef, uint32_t shift, uint32_t wtot, int cl, double beta, int max_row,
                      hipStream_t s)
{
    const int nch = pick_nch(max_row);
    const size_t tsz = dtype == USPG_F64 ? sizeof(double) : sizeof(float);
    const bool nt = stream_coefs(c->view_coef.bytes, tsz * (size_t)c->g->ncells);
    auto fill = [&](auto &A) {
        A.rowptr = rowptr;
        A.co = static_cast<const Coef<float> *>(coef);
        A.wtot = wtot;
        A.shift = shift;
        A.U = c->scan.det_u;
        A.Ku = c->Ku;
        A.Kv = c->Kv;
        A.cu = cl % c->Ku;
        A.cw = cl / c->Ku;
        A.nu = (c->scan.det_u - A.cu + c->Ku - 1) / c->Ku;
        A.ncls = A.nu * ((c->scan.det_v - A.cw + c->Kv - 1) / c->Kv);
        A.nblk = std::min((A.ncls + kWaves - 1) / kWaves, grid_cap());
    };
    if (dtype == USPG_F64) {
        BatchArgs<double, float> A{};
        fill(A);
        A.P = static_cast<const double *>(proj_view);
        A.f = static_cast<double *>(f);
        A.beta = beta;
        if (A.ncls) launch_batch_n<double, float>(nch, nt, A, s);
    } else {
        BatchArgs<float, float> A{};
        fill(A);
        A.P = static_cast<const float *>(proj_view);
        A.f = static_cast<float *>(f);
        A.beta = (float)beta;
        if (A.ncls) launch_batch_n<float, float>(nch, nt, A, s);
    }
    return hipGetLastError() == hipSuccess ? USPG_OK : fail(USPG_E_HIP, "batch launch failed");
}

int batch_grid_cap() { return grid_cap(); }

int batch_step(const uspg_coeffs *c, int dtype, const void *proj, void *f, double beta, int v, int cl, hipStream_t s)
{
    if (kept_rows(c)) {
        const size_t tsz = dtype == USPG_F64 ? sizeof(double) : sizeof(float);
        return rows_batch_launch(c, dtype, static_cast<const char *>(proj) + tsz * (size_t)v * c->nrays, f,
                                 c->view_rowptr.as<int64_t>() + (int64_t)v * (c->nrays + 1),
                                 c->view_coef.as<Coef<float>>() + c->view_start[v], 0u, (uint32_t)c->g->ncells, cl,
                                 beta, c->view_max_row, s);
    }
    const int nch = pick_nch(c->max_row);
    const bool cf64 = c->scan.coeff_dtype == USPG_F64;
    const bool nt = stream_coefs(c->coef.bytes, (dtype == USPG_F64 ? sizeof(double) : sizeof(float)) * (size_t)c->Wtot);
    if (dtype == USPG_F64) {
        if (cf64) {
            const auto A = batch_args<double, double>(c, (const double *)proj, (double *)f, beta, v, cl);
            if (A.ncls) launch_step<double, double>(c, nch, nt, A, s);
        } else {
            const auto A = batch_args<double, float>(c, (const double *)proj, (double *)f, beta, v, cl);
            if (A.ncls) launch_step<double, float>(c, nch, nt, A, s);
        }
    } else {
        if (cf64) {
            const auto A = batch_args<float, double>(c, (const float *)proj, (float *)f, beta, v, cl);
            if (A.ncls) launch_step<float, double>(c, nch, nt, A, s);
        } else {
            const auto A = batch_args<float, float>(c, (const float *)proj, (float *)f, beta, v, cl);
            if (A.ncls) launch_step<float, float>(c, nch, nt, A, s);
        }
    }
    return hipGetLastError() == hipSuccess ? USPG_OK : fail(USPG_E_HIP, "batch launch failed");
}

int mart_launch(const uspg_coeffs *c, int dtype, const void *proj, void *image, void *work,
                int n_sweeps, double beta, double tol, int32_t *sweeps_done, hipStream_t s)
{
    if (c->segments) return rebin_launch(c, dtype, proj, image, work, n_sweeps, beta, tol, sweeps_done, s);
    const bool cf64 = c->scan.coeff_dtype == USPG_F64;
    if (dtype == USPG_F32) {
        if (cf64)
            return run_typed<float, double>(c, (const float *)proj, (float *)image, work, n_sweeps, beta, tol, sweeps_done, s);
        return run_typed<float, float>(c, (const float *)proj, (float *)image, work, n_sweeps, beta, tol, sweeps_done, s);
    }
    if (cf64)
        return run_typed<double, double>(c, (const double *)proj, (double *)image, work, n_sweeps, beta, tol, sweeps_done, s);
    return run_typed<double, float>(c, (const double *)proj, (double *)image, work, n_sweeps, beta, tol, sweeps_done, s);
}

}  // namespace uspg
