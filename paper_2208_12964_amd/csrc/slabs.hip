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
//      all-reduce of a multi-device run; here each ray's waves read the
//      parts of the slabs holding entries of the ray, the others being
//      zero);
//   3. every slab applies f_j <- f_j (1 + beta (P / Pbar - 1) a_j / a_max)
//      to its own cells (slab_apply), with a_max of the whole row.
// A slab's launches cover only the rays of the class with entries in the
// slab (lists built with the slab rows).  With one slab the partial sum is
// the fused kernel's sum, in the same lane order, so the result equals
// mart_run bit for bit; with more slabs only the association of the ray sums
// changes.
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
    // Rays of each (slab, class) whose row has entries in the slab, as
    // class-local indices: list (g, c) is xs[lofs[g K + c] .. lofs[g K + c + 1]).
    std::vector<int64_t> lofs;
    uspg::DevBuf xs;                // int32
    uspg::DevBuf mask;              // uint64 [nrays]: bit g set when the ray has entries in slab g
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
    const unsigned long long *mask;  // [nrays]: slabs holding entries of the ray
    const int32_t *xs;       // rays of the class with entries in this slab
    int nx;
    const T *P;              // the view's projections
    T *f;                    // device-layout image
    T *part;                 // [G][ncls] partial ray sums of the batch
    int g, G;
    uint32_t shift, wtot;
    int U, cu, cw, Ku, Kv, nu, ncls, nblk;
    T beta;
};

// Rows of up to 64 * kSlabChunks entries stay in registers between the
// gather and the scatter; longer rows are streamed.
constexpr int kSlabChunks = 8;

__device__ inline int64_t class_ray(int x, int U, int cu, int cw, int Ku, int Kv, int nu)
{
    const int w = cw + (x / nu) * Kv;
    const int u = cu + (x % nu) * Ku;
    return (int64_t)w * U + u;
}

// Loads the (shifted id, coefficient) pairs of a row of 1 <= n <= 64 C
// entries and gathers their image values: every load is issued before the
// first wait; entries past the row repeat its last id with coefficient 0.
template <class T, class TC, int C>
__device__ __forceinline__ void gather_row(const SlabArgs<T, TC> &A, int64_t beg, int n, int lane, uint32_t *id,
                                           T *av, T *fv)
{
    const int last = n - 1;
#pragma unroll
    for (int k = 0; k < C; ++k) {
        const int j = lane + 64 * k;
        uint32_t cid;
        TC ca;
        load_coef(A.co + beg + (j < n ? j : last), cid, ca);
        const uint32_t t = cid + A.shift;
        id[k] = t >= A.wtot ? t - A.wtot : t;
        av[k] = (T)ca * (j < n ? T(1) : T(0));
    }
#pragma unroll
    for (int k = 0; k < C; ++k) fv[k] = A.f[id[k]];
}

// Step 1: this slab's part of the ray sums of the batch, for the rays with
// entries in the slab.  Lane l adds entries l, l + 64, ... in order, then the
// wavefront reduces, exactly as the fused kernel does for a whole row.
template <class T, class TC>
__global__ __launch_bounds__(kBlock) void slab_partial(SlabArgs<T, TC> A)
{
#pragma clang fp contract(off)
    constexpr int C = kSlabChunks;
    const int lane = threadIdx.x & 63;
    const int total = A.nblk * kWaves;
    for (int i = xcd_block(blockIdx.x, A.nblk) * kWaves + (threadIdx.x >> 6); i < A.nx; i += total) {
        const int x = A.xs[i];
        const int64_t r = class_ray(x, A.U, A.cu, A.cw, A.Ku, A.Kv, A.nu);
        const int64_t beg = A.rowptr[r];
        const int n = (int)(A.rowptr[r + 1] - beg);
        T acc = T(0);
        if (n > 0 && n <= 64 * C) {
            uint32_t id[C];
            T av[C], fv[C];
            gather_row<T, TC, C>(A, beg, n, lane, id, av, fv);
#pragma unroll
            for (int k = 0; k < C; ++k) acc = fmadd(av[k], fv[k], acc);
        } else {
            for (int j = lane; j < n; j += 64) {
                uint32_t id;
                TC a;
                load_coef(A.co + beg + j, id, a);
                uint32_t t = id + A.shift;
                t = t >= A.wtot ? t - A.wtot : t;
                acc = fmadd((T)a, A.f[t], acc);
            }
        }
        acc = wave_sum(acc);
        if (lane == 0) A.part[(int64_t)A.g * A.ncls + x] = acc;
    }
}

// Steps 2 and 3: the sum of the partial sums of the slabs holding entries of
// the ray, in slab order (the other slabs' parts are zero), then the
// multiplicative correction of this slab's cells.  The row's loads and
// gathers are issued before the partial sums are read.
template <class T, class TC>
__global__ __launch_bounds__(kBlock) void slab_apply(SlabArgs<T, TC> A)
{
#pragma clang fp contract(off)
    constexpr int C = kSlabChunks;
    const int lane = threadIdx.x & 63;
    const int total = A.nblk * kWaves;
    for (int i = xcd_block(blockIdx.x, A.nblk) * kWaves + (threadIdx.x >> 6); i < A.nx; i += total) {
        const int x = A.xs[i];
        const int64_t r = class_ray(x, A.U, A.cu, A.cw, A.Ku, A.Kv, A.nu);
        const int64_t beg = A.rowptr[r];
        const int n = (int)(A.rowptr[r + 1] - beg);
        if (n == 0) continue;
        const bool in_regs = n <= 64 * C;
        uint32_t id[C];
        T av[C], fv[C];
        if (in_regs) gather_row<T, TC, C>(A, beg, n, lane, id, av, fv);
        unsigned long long m = A.mask[r];
        T acc = T(0);
        bool first = true;
        while (m) {
            const int h = __builtin_ctzll(m);
            m &= m - 1;
            const T p = A.part[(int64_t)h * A.ncls + x];
            acc = first ? p : acc + p;
            first = false;
        }
        const T amax = (T)A.amax[r];
        if (!(acc > T(0)) || !(amax > T(0))) continue;
        const T c = A.beta * (A.P[r] / acc - T(1)) / amax;
        if (in_regs) {
#pragma unroll
            for (int k = 0; k < C; ++k)
                if (lane + 64 * k < n) A.f[id[k]] = fv[k] * fmadd(c, av[k], T(1));
        } else {
            for (int j = lane; j < n; j += 64) {
                uint32_t id1;
                TC a;
                load_coef(A.co + beg + j, id1, a);
                uint32_t t = id1 + A.shift;
                t = t >= A.wtot ? t - A.wtot : t;
                A.f[t] = A.f[t] * fmadd(c, (T)a, T(1));
            }
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
    // per (slab, class): the rays with entries in the slab; per ray: its slabs
    std::vector<uint32_t> h_cnt((size_t)G * nrays);
    USPG_HIP(hipMemcpyAsync(h_cnt.data(), cnt.p, sizeof(uint32_t) * h_cnt.size(), hipMemcpyDeviceToHost, s));
    USPG_HIP(hipStreamSynchronize(s));
    const int K = c->Ku * c->Kv, U = c->scan.det_u, V = c->scan.det_v;
    std::vector<unsigned long long> h_mask(nrays, 0ull);
    for (int g = 0; g < G; ++g)
        for (int64_t r = 0; r < nrays; ++r)
            if (h_cnt[(size_t)g * nrays + r]) h_mask[r] |= 1ull << g;
    std::vector<int32_t> h_xs;
    S->lofs.assign((size_t)G * K + 1, 0);
    for (int g = 0; g < G; ++g)
        for (int cl = 0; cl < K; ++cl) {
            const int cu = cl % c->Ku, cw = cl / c->Ku;
            const int nu = (U - cu + c->Ku - 1) / c->Ku, nw = (V - cw + c->Kv - 1) / c->Kv;
            for (int x = 0; x < nu * nw; ++x) {
                const int64_t r = (int64_t)(cw + (x / nu) * c->Kv) * U + cu + (x % nu) * c->Ku;
                if (h_cnt[(size_t)g * nrays + r]) h_xs.push_back(x);
            }
            S->lofs[(size_t)g * K + cl + 1] = (int64_t)h_xs.size();
        }
    if ((rc = S->xs.alloc(sizeof(int32_t) * std::max<size_t>(h_xs.size(), 1))) != USPG_OK) return rc;
    if ((rc = S->mask.alloc(sizeof(unsigned long long) * (size_t)std::max<int64_t>(nrays, 1))) != USPG_OK) return rc;
    if (!h_xs.empty())
        USPG_HIP(hipMemcpyAsync(S->xs.p, h_xs.data(), sizeof(int32_t) * h_xs.size(), hipMemcpyHostToDevice, s));
    USPG_HIP(hipMemcpyAsync(S->mask.p, h_mask.data(), sizeof(unsigned long long) * nrays, hipMemcpyHostToDevice, s));
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
    A.mask = S->mask.as<unsigned long long>();
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
                // one slab's launch covers only the class's rays with entries in it
                auto set_slab = [&](int g) {
                    const int64_t lo = S->lofs[(size_t)g * K + cl], hi = S->lofs[(size_t)g * K + cl + 1];
                    A.g = g;
                    A.rowptr = S->rowptr.as<int64_t>() + (int64_t)g * (nrays + 1);
                    A.co = S->coef.as<Coef<TC>>() + S->start[g];
                    A.xs = S->xs.as<int32_t>() + lo;
                    A.nx = (int)(hi - lo);
                    A.nblk = std::min((A.nx + kWaves - 1) / kWaves, cap);
                    return A.nx > 0;
                };
                for (int g = 0; g < S->G; ++g)
                    if (set_slab(g)) hipLaunchKernelGGL((slab_partial<T, TC>), dim3(A.nblk), dim3(kBlock), 0, s, A);
                for (int g = 0; g < S->G; ++g)
                    if (set_slab(g)) hipLaunchKernelGGL((slab_apply<T, TC>), dim3(A.nblk), dim3(kBlock), 0, s, A);
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
    int rc = check_coeffs(c);
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
    S->xs.release();
    S->mask.release();
    delete S;
}

}  // extern "C"
