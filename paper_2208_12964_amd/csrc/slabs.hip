// One cone-beam solve split into z-slabs, the way several devices would
// share it, run on one device.
//
// Slab g owns the cells of slices [begin_g, begin_{g+1}) and, of every
// reference row, the entries that fall in them (a subsequence of the row, in
// row order).  The view shift adds a multiple of Wc = Nz * Cq and so keeps
// every cell in its slice: a slab's rows serve every view.  A (view, class)
// batch of eqs. 17-18 then splits at the ray sum:
//   1. every slab sums a_j f_j over its part of each ray of the class
//      (slab_partial, one launch per slab, as each device would);
//   2. the partial sums are added over the slabs in slab order (the
//      all-reduce of a multi-device run; here each ray's waves read all of
//      them);
//   3. every slab applies f_j <- f_j (1 + beta (P / Pbar - 1) a_j / a_max)
//      to its own cells (slab_apply), with a_max of the whole row.
// With one slab the partial sum is the fused kernel's sum, in the same lane
// order, so the result equals mart_run bit for bit; with more slabs only the
// association of the ray sums changes.
#include <algorithm>
#include <vector>

#include "mart_row.hpp"
#include "uspg_internal.hpp"

struct uspg_slabs {
    const uspg_coeffs *c = nullptr;
    int G = 0;
    int device = 0;
    std::vector<int32_t> begin;     // first slice of each slab, G + 1 entries
    std::vector<int64_t> start;     // first entry of each slab, G + 1 entries
    uspg::DevBuf rowptr;            // int64 [G][nrays + 1], relative to the slab's first entry
    uspg::DevBuf coef;              // Coef<TC> [nnz], slab-major
    uspg::DevBuf amax;              // TC [nrays]: largest coefficient of the whole row
};

namespace uspg {
namespace {

using row::fmadd;
using row::load_coef;
using row::wave_sum;
using row::xcd_block;

constexpr int kWaves = 4;
constexpr int kBlock = 64 * kWaves;

struct SlabGeo {
    uint32_t Wc, Cq;
    const int32_t *slab_of_slice;
};

__device__ inline int slab_of(uint32_t id, const SlabGeo &S) { return S.slab_of_slice[(id % S.Wc) / S.Cq]; }

__device__ inline int wave_sum_int(int v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// One wavefront per (slab, ray): entries of the ray's row in the slab.
template <class TC>
__global__ __launch_bounds__(kBlock) void slab_count(const int64_t *rowptr, const Coef<TC> *co, int64_t nrays,
                                                     int G, SlabGeo S, uint32_t *cnt)
{
    const int64_t w = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int lane = threadIdx.x & 63;
    if (w >= (int64_t)G * nrays) return;
    const int g = (int)(w / nrays);
    const int64_t r = w - (int64_t)g * nrays;
    const int64_t beg = rowptr[r], n = rowptr[r + 1] - beg;
    int m = 0;
    for (int64_t j = lane; j < n; j += 64) m += slab_of(co[beg + j].id, S) == g;
    m = wave_sum_int(m);
    if (lane == 0) cnt[w] = (uint32_t)m;
}

// Same assignment: the slab's entries of the row, written in row order
// (ballot prefix per chunk of 64).
template <class TC>
__global__ __launch_bounds__(kBlock) void slab_fill(const int64_t *rowptr, const Coef<TC> *co, int64_t nrays,
                                                    int G, SlabGeo S, const int64_t *srow, const int64_t *start,
                                                    Coef<TC> *out)
{
    const int64_t w = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int lane = threadIdx.x & 63;
    if (w >= (int64_t)G * nrays) return;
    const int g = (int)(w / nrays);
    const int64_t r = w - (int64_t)g * nrays;
    const int64_t beg = rowptr[r], n = rowptr[r + 1] - beg;
    int64_t at = start[g] + srow[(int64_t)g * (nrays + 1) + r];
    const unsigned long long below = (1ull << lane) - 1ull;
    for (int64_t j0 = 0; j0 < n; j0 += 64) {
        const int64_t j = j0 + lane;
        const bool in = j < n && slab_of(co[beg + j].id, S) == g;
        const unsigned long long mask = __ballot(in);
        if (in) out[at + __popcll(mask & below)] = co[beg + j];
        at += __popcll(mask);
    }
}

// Largest coefficient of every whole row (a_max of eq. 18).
template <class TC>
__global__ __launch_bounds__(kBlock) void row_amax(const int64_t *rowptr, const Coef<TC> *co, int64_t nrays, TC *amax)
{
    const int64_t r = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int lane = threadIdx.x & 63;
    if (r >= nrays) return;
    const int64_t beg = rowptr[r], n = rowptr[r + 1] - beg;
    TC m = TC(0);
    for (int64_t j = lane; j < n; j += 64) m = co[beg + j].a > m ? co[beg + j].a : m;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        const TC o = __shfl_xor(m, off, 64);
        m = o > m ? o : m;
    }
    if (lane == 0) amax[r] = m;
}

template <class T, class TC>
struct SlabArgs {
    const int64_t *rowptr;   // this slab's, [nrays + 1]
    const Coef<TC> *co;      // this slab's first entry
    const TC *amax;          // [nrays]
    const T *P;              // the view's projections
    T *f;                    // device-layout image
    T *part;                 // [G][ncls] partial ray sums of the batch
    int g, G;
    uint32_t shift, wtot;
    int U, cu, cw, Ku, Kv, nu, ncls, nblk;
    T beta;
};

__device__ inline int64_t class_ray(int x, int U, int cu, int cw, int Ku, int Kv, int nu)
{
    const int w = cw + (x / nu) * Kv;
    const int u = cu + (x % nu) * Ku;
    return (int64_t)w * U + u;
}

// Step 1: this slab's part of every ray sum of the batch (zero for an empty
// part).  Lane l adds entries l, l + 64, ... in order, then the wavefront
// reduces, exactly as the fused kernel does for a whole row.
template <class T, class TC>
__global__ __launch_bounds__(kBlock) void slab_partial(SlabArgs<T, TC> A)
{
#pragma clang fp contract(off)
    const int lane = threadIdx.x & 63;
    const int total = A.nblk * kWaves;
    for (int x = xcd_block(blockIdx.x, A.nblk) * kWaves + (threadIdx.x >> 6); x < A.ncls; x += total) {
        const int64_t r = class_ray(x, A.U, A.cu, A.cw, A.Ku, A.Kv, A.nu);
        const int64_t beg = A.rowptr[r];
        const int n = (int)(A.rowptr[r + 1] - beg);
        T acc = T(0);
        for (int j = lane; j < n; j += 64) {
            uint32_t id;
            TC a;
            load_coef(A.co + beg + j, id, a);
            uint32_t t = id + A.shift;
            t = t >= A.wtot ? t - A.wtot : t;
            acc = fmadd((T)a, A.f[t], acc);
        }
        acc = wave_sum(acc);
        if (lane == 0) A.part[(int64_t)A.g * A.ncls + x] = acc;
    }
}

// Steps 2 and 3: the sum of the slabs' partial sums (in slab order), then
// the multiplicative correction of this slab's cells.
template <class T, class TC>
__global__ __launch_bounds__(kBlock) void slab_apply(SlabArgs<T, TC> A)
{
#pragma clang fp contract(off)
    const int lane = threadIdx.x & 63;
    const int total = A.nblk * kWaves;
    for (int x = xcd_block(blockIdx.x, A.nblk) * kWaves + (threadIdx.x >> 6); x < A.ncls; x += total) {
        const int64_t r = class_ray(x, A.U, A.cu, A.cw, A.Ku, A.Kv, A.nu);
        const int64_t beg = A.rowptr[r];
        const int n = (int)(A.rowptr[r + 1] - beg);
        if (n == 0) continue;
        T acc = A.part[x];
        for (int h = 1; h < A.G; ++h) acc += A.part[(int64_t)h * A.ncls + x];
        const T amax = (T)A.amax[r];
        if (!(acc > T(0)) || !(amax > T(0))) continue;
        const T c = A.beta * (A.P[r] / acc - T(1)) / amax;
        for (int j = lane; j < n; j += 64) {
            uint32_t id;
            TC a;
            load_coef(A.co + beg + j, id, a);
            uint32_t t = id + A.shift;
            t = t >= A.wtot ? t - A.wtot : t;
            A.f[t] = A.f[t] * fmadd(c, (T)a, T(1));
        }
    }
}

int max_class_rays(const uspg_coeffs *c)
{
    return (int)(((c->scan.det_u + c->Ku - 1) / c->Ku) * (int64_t)((c->scan.det_v + c->Kv - 1) / c->Kv));
}

size_t part_offset(const uspg_coeffs *c, size_t tsz) { return ((size_t)c->Wtot * tsz + 255) / 256 * 256; }

template <class TC>
int build_rows(uspg_slabs *S, const int32_t *d_slab_of_slice, DevBuf &cnt, DevBuf &d_start, hipStream_t s)
{
    const uspg_coeffs *c = S->c;
    const int G = S->G;
    const int64_t nrays = c->nrays;
    SlabGeo geo{(uint32_t)c->Wc, (uint32_t)c->Cq, d_slab_of_slice};
    const Coef<TC> *co = c->coef.as<Coef<TC>>();
    const int64_t *rp = c->rowptr.as<int64_t>();
    int rc = cnt.alloc(sizeof(uint32_t) * (size_t)G * nrays);
    if (rc == USPG_OK) rc = S->rowptr.alloc(sizeof(int64_t) * (size_t)G * (nrays + 1));
    if (rc == USPG_OK) rc = S->amax.alloc(sizeof(TC) * (size_t)std::max<int64_t>(nrays, 1));
    if (rc == USPG_OK) rc = d_start.alloc(sizeof(int64_t) * (G + 1));
    if (rc != USPG_OK) return rc;
    const int64_t waves = (int64_t)G * nrays;
    const unsigned blocks = (unsigned)((waves + kWaves - 1) / kWaves);
    hipLaunchKernelGGL(slab_count<TC>, dim3(blocks), dim3(kBlock), 0, s, rp, co, nrays, G, geo, cnt.as<uint32_t>());
    USPG_HIP(hipGetLastError());
    for (int g = 0; g < G; ++g)
        if ((rc = exclusive_scan_u32_to_i64(cnt.as<uint32_t>() + (int64_t)g * nrays,
                                            S->rowptr.as<int64_t>() + (int64_t)g * (nrays + 1), nrays, s)) != USPG_OK)
            return rc;
    std::vector<int64_t> part_nnz(G);
    for (int g = 0; g < G; ++g)
        USPG_HIP(hipMemcpyAsync(&part_nnz[g], S->rowptr.as<int64_t>() + (int64_t)g * (nrays + 1) + nrays,
                                sizeof(int64_t), hipMemcpyDeviceToHost, s));
    USPG_HIP(hipStreamSynchronize(s));
    S->start.assign(G + 1, 0);
    for (int g = 0; g < G; ++g) S->start[g + 1] = S->start[g] + part_nnz[g];
    if (S->start[G] != c->nnz) return fail(USPG_E_INTERNAL, "slab rows do not add up to the reference rows");
    if ((rc = S->coef.alloc(sizeof(Coef<TC>) * (size_t)std::max<int64_t>(c->nnz, 1))) != USPG_OK) return rc;
    USPG_HIP(hipMemcpyAsync(d_start.p, S->start.data(), sizeof(int64_t) * (G + 1), hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(slab_fill<TC>, dim3(blocks), dim3(kBlock), 0, s, rp, co, nrays, G, geo,
                       S->rowptr.as<int64_t>(), d_start.as<int64_t>(), S->coef.as<Coef<TC>>());
    const unsigned rblocks = (unsigned)((nrays + kWaves - 1) / kWaves);
    if (nrays > 0)
        hipLaunchKernelGGL(row_amax<TC>, dim3(rblocks), dim3(kBlock), 0, s, rp, co, nrays, S->amax.as<TC>());
    USPG_HIP(hipGetLastError());
    USPG_HIP(hipStreamSynchronize(s));
    return USPG_OK;
}

// Builds the slab rows; the temporaries are freed on every path (after the
// stream has drained).
template <class TC>
int build_typed(uspg_slabs *S, const int32_t *d_slab_of_slice, hipStream_t s)
{
    DevBuf cnt, d_start;
    const int rc = build_rows<TC>(S, d_slab_of_slice, cnt, d_start, s);
    (void)hipStreamSynchronize(s);
    cnt.release();
    d_start.release();
    return rc;
}

template <class T, class TC>
int run_typed(const uspg_slabs *S, const T *proj, T *image, void *work, int n_sweeps, double beta, hipStream_t s)
{
    const uspg_coeffs *c = S->c;
    const int dtype = sizeof(T) == sizeof(double) ? USPG_F64 : USPG_F32;
    T *nat = static_cast<T *>(work);
    T *part = reinterpret_cast<T *>(static_cast<char *>(work) + part_offset(c, sizeof(T)));
    int rc = layout_permute(c, dtype, image, nat, 1, s);
    if (rc != USPG_OK) return rc;
    const int K = c->Ku * c->Kv;
    const int cap = batch_grid_cap();
    SlabArgs<T, TC> A{};
    A.amax = S->amax.as<TC>();
    A.f = nat;
    A.part = part;
    A.G = S->G;
    A.wtot = (uint32_t)c->Wtot;
    A.U = c->scan.det_u;
    A.Ku = c->Ku;
    A.Kv = c->Kv;
    A.beta = (T)beta;
    const int64_t nrays = c->nrays;
    for (int sw = 0; sw < n_sweeps; ++sw) {
        for (int v = 0; v < c->scan.n_views; ++v) {
            A.P = proj + (int64_t)v * nrays;
            A.shift = (uint32_t)(((int64_t)v * c->Wc) % c->Wtot);
            for (int cl = 0; cl < K; ++cl) {
                A.cu = cl % c->Ku;
                A.cw = cl / c->Ku;
                A.nu = (c->scan.det_u - A.cu + c->Ku - 1) / c->Ku;
                A.ncls = A.nu * ((c->scan.det_v - A.cw + c->Kv - 1) / c->Kv);
                if (A.ncls == 0) continue;
                A.nblk = std::min((A.ncls + kWaves - 1) / kWaves, cap);
                for (int g = 0; g < S->G; ++g) {
                    A.g = g;
                    A.rowptr = S->rowptr.as<int64_t>() + (int64_t)g * (nrays + 1);
                    A.co = S->coef.as<Coef<TC>>() + S->start[g];
                    hipLaunchKernelGGL((slab_partial<T, TC>), dim3(A.nblk), dim3(kBlock), 0, s, A);
                }
                for (int g = 0; g < S->G; ++g) {
                    A.g = g;
                    A.rowptr = S->rowptr.as<int64_t>() + (int64_t)g * (nrays + 1);
                    A.co = S->coef.as<Coef<TC>>() + S->start[g];
                    hipLaunchKernelGGL((slab_apply<T, TC>), dim3(A.nblk), dim3(kBlock), 0, s, A);
                }
            }
        }
        USPG_HIP(hipGetLastError());
    }
    return layout_permute(c, dtype, nat, image, 0, s);
}

}  // namespace
}  // namespace uspg

using namespace uspg;

extern "C" {

int uspg_build_slabs(const uspg_coeffs *c, int32_t n_slabs, void *stream, uspg_slabs **out)
{
    if (!c || !out) return fail(USPG_E_ARG, "null argument");
    *out = nullptr;
    if (c->segments) return fail(USPG_E_ARG, "segment-record coefficients run through mart_run only");
    const int nz = c->g->nz;
    if (n_slabs < 1 || n_slabs > nz || n_slabs > USPG_MAX_SLABS)
        return fail(USPG_E_ARG, "n_slabs must lie in [1, min(n_slices, USPG_MAX_SLABS)]");
    int rc = check_device(c->device);
    if (rc != USPG_OK) return rc;
    hipStream_t s = (hipStream_t)stream;
    auto *S = new uspg_slabs();
    S->c = c;
    S->G = n_slabs;
    S->device = c->device;
    S->begin.resize(n_slabs + 1);
    for (int g = 0; g <= n_slabs; ++g) S->begin[g] = (int32_t)((int64_t)g * nz / n_slabs);
    std::vector<int32_t> of(nz);
    for (int g = 0; g < n_slabs; ++g)
        for (int k = S->begin[g]; k < S->begin[g + 1]; ++k) of[k] = g;
    DevBuf d_of;
    rc = d_of.alloc(sizeof(int32_t) * nz);
    if (rc == USPG_OK && hipMemcpyAsync(d_of.p, of.data(), sizeof(int32_t) * nz, hipMemcpyHostToDevice, s) != hipSuccess)
        rc = fail(USPG_E_HIP, "uploading the slab table failed");
    if (rc == USPG_OK)
        rc = c->scan.coeff_dtype == USPG_F64 ? build_typed<double>(S, d_of.as<int32_t>(), s)
                                            : build_typed<float>(S, d_of.as<int32_t>(), s);
    (void)hipStreamSynchronize(s);
    d_of.release();
    if (rc != USPG_OK) {
        uspg_free_slabs(S);
        return rc;
    }
    *out = S;
    return USPG_OK;
}

int uspg_slabs_info(const uspg_slabs *S, int32_t slab, int32_t *slice_begin, int32_t *slice_end, int64_t *nnz)
{
    if (!S) return fail(USPG_E_ARG, "null slabs");
    if (slab < 0 || slab >= S->G) return fail(USPG_E_ARG, "slab out of range");
    if (slice_begin) *slice_begin = S->begin[slab];
    if (slice_end) *slice_end = S->begin[slab + 1];
    if (nnz) *nnz = S->start[slab + 1] - S->start[slab];
    return USPG_OK;
}

size_t uspg_slabs_workspace_bytes(const uspg_slabs *S, int32_t dtype)
{
    if (!S) return 0;
    const size_t tsz = dtype == USPG_F64 ? sizeof(double) : sizeof(float);
    return part_offset(S->c, tsz) + (size_t)S->G * max_class_rays(S->c) * tsz;
}

int mart_run_slabs(const uspg_slabs *S, int32_t dtype, const void *proj, void *image, void *work, size_t work_bytes,
                   int32_t n_sweeps, double beta, void *stream)
{
    if (!S || !proj || !image || !work) return fail(USPG_E_ARG, "null argument");
    if (dtype != USPG_F32 && dtype != USPG_F64) return fail(USPG_E_ARG, "dtype");
    if (n_sweeps < 0 || !(beta > 0)) return fail(USPG_E_ARG, "n_sweeps >= 0 and beta > 0");
    if (work_bytes < uspg_slabs_workspace_bytes(S, dtype)) return fail(USPG_E_NOMEM, "work space too small");
    int rc = check_device(S->device);
    if (rc != USPG_OK) return rc;
    hipStream_t s = (hipStream_t)stream;
    const bool cf64 = S->c->scan.coeff_dtype == USPG_F64;
    if (dtype == USPG_F64)
        return cf64 ? run_typed<double, double>(S, (const double *)proj, (double *)image, work, n_sweeps, beta, s)
                    : run_typed<double, float>(S, (const double *)proj, (double *)image, work, n_sweeps, beta, s);
    return cf64 ? run_typed<float, double>(S, (const float *)proj, (float *)image, work, n_sweeps, beta, s)
                : run_typed<float, float>(S, (const float *)proj, (float *)image, work, n_sweeps, beta, s);
}

void uspg_free_slabs(uspg_slabs *S)
{
    if (!S) return;
    S->rowptr.release();
    S->coef.release();
    S->amax.release();
    delete S;
}

}  // extern "C"
