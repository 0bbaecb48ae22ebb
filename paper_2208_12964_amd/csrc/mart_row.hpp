// Per-ray Sp-MART update shared by the single-problem and batched kernels
// (Sec. III.D, eqs. 17-18).  One wavefront handles one ray: coefficients are
// loaded as (id, coefficient) pairs with non-temporal hints, the ids rotated
// to the view by one add and a conditional subtract, the image gathered
// through `img` (global memory or LDS), Pbar and a_max reduced across the
// wavefront in a fixed order, then
//   f_j <- f_j (1 + beta (P / Pbar - 1) a_j / a_max).
// Also the largest relative change of a sweep (eq. 19), shared by the
// stored-row and segment-record solvers.
#pragma once

#include "uspg_internal.hpp"

namespace uspg {
namespace row {

// Workgroups are dispatched round robin over the 8 XCDs; renumber them so
// that each XCD owns one contiguous run of the virtual workgroups 0 .. nb-1
// (neighbouring rays touch neighbouring cells, which then share that XCD's
// L2).  A bijection on [0, nb).
__device__ inline int xcd_block(int b, int nb)
{
    int xcd = b & 7, idx = b >> 3;
    int per = nb >> 3, rem = nb & 7;
    return xcd * per + (xcd < rem ? xcd : rem) + idx;
}

template <class T>
__device__ inline T wave_sum(T v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

template <class T>
__device__ inline T wave_max(T v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        T o = __shfl_xor(v, off, 64);
        v = o > v ? o : v;
    }
    return v;
}

// The per-ray arithmetic is pinned: explicit fused multiply-adds and no
// compiler contraction, so every kernel that runs a row (single problem,
// batched, persistent, engine) produces the same bits for it.
template <class T>
__device__ __forceinline__ T fmadd(T a, T b, T c) { return __builtin_fma(a, b, c); }
template <>
__device__ __forceinline__ float fmadd<float>(float a, float b, float c) { return __builtin_fmaf(a, b, c); }

// Load of one (id, coefficient) pair: one vector load.  NT: with the
// non-temporal hint, for coefficient sets that stream through caches too
// small to hold them; without it, a set that fits the last-level cache
// together with the image stays there from one view to the next.
template <bool NT = true>
__device__ __forceinline__ void load_coef(const Coef<float> *p, uint32_t &id, float &a)
{
    typedef unsigned int u2 __attribute__((ext_vector_type(2)));
    const u2 *q = reinterpret_cast<const u2 *>(p);
    u2 e;
    if constexpr (NT) e = __builtin_nontemporal_load(q);
    else e = *q;
    id = e.x;
    a = __uint_as_float(e.y);
}

template <bool NT = true>
__device__ __forceinline__ void load_coef(const Coef<double> *p, uint32_t &id, double &a)
{
    typedef unsigned int u4 __attribute__((ext_vector_type(4)));
    const u4 *q = reinterpret_cast<const u4 *>(p);
    u4 e;
    if constexpr (NT) e = __builtin_nontemporal_load(q);
    else e = *q;
    id = e.x;
    const unsigned long long bits = ((unsigned long long)e.w << 32) | e.z;
    __builtin_memcpy(&a, &bits, sizeof(a));
}

// One row of C chunks of 64 coefficients, kept in registers.  Indices are
// clamped and coefficients masked instead of branching, so every load of a
// phase is issued before the first wait: the ids and coefficients, then all
// gathers, then the reductions, then the predicated scatter.
template <class T, class TC, int C, bool NT = true, class Img>
__device__ __forceinline__ void row_in_registers(Img img, uint32_t shift, uint32_t wtot, T beta,
                                                 const Coef<TC> *co, int n, T P, int lane)
{
#pragma clang fp contract(off)
    uint32_t id[C];
    T av[C], fv[C];
    const int last = n - 1;
#pragma unroll
    for (int k = 0; k < C; ++k) {
        const int j = lane + 64 * k;
        const int jj = j < n ? j : last;
        // the coefficient stream is read once per view: for large sets
        // non-temporal loads keep it from evicting the image from the caches
        uint32_t cid;
        TC ca;
        load_coef<NT>(co + jj, cid, ca);
        const uint32_t t = cid + shift;
        id[k] = t >= wtot ? t - wtot : t;
        av[k] = (T)ca * (j < n ? T(1) : T(0));   // masked, not branched
    }
#pragma unroll
    for (int k = 0; k < C; ++k) fv[k] = img[id[k]];
    T acc = T(0), amax = T(0);
#pragma unroll
    for (int k = 0; k < C; ++k) {
        acc = fmadd(av[k], fv[k], acc);
        amax = av[k] > amax ? av[k] : amax;
    }
    acc = wave_sum(acc);
    amax = wave_max(amax);
    if (!(acc > T(0)) || !(amax > T(0))) return;
    const T c = beta * (P / acc - T(1)) / amax;
#pragma unroll
    for (int k = 0; k < C; ++k) {
        if (lane + 64 * k < n) img[id[k]] = fv[k] * fmadd(c, av[k], T(1));
    }
}

// Rows longer than the register path: forward pass, then re-read and update.
template <class T, class TC, class Img>
__device__ void row_streamed(Img img, uint32_t shift, uint32_t wtot, T beta, const Coef<TC> *co, int n, T P,
                             int lane)
{
#pragma clang fp contract(off)
    T acc = T(0), amax = T(0);
    for (int j = lane; j < n; j += 64) {
        uint32_t t = co[j].id + shift;
        t = t >= wtot ? t - wtot : t;
        T av = (T)co[j].a;
        acc = fmadd(av, img[t], acc);
        amax = av > amax ? av : amax;
    }
    acc = wave_sum(acc);
    amax = wave_max(amax);
    if (!(acc > T(0)) || !(amax > T(0))) return;
    const T c = beta * (P / acc - T(1)) / amax;
    for (int j = lane; j < n; j += 64) {
        uint32_t t = co[j].id + shift;
        t = t >= wtot ? t - wtot : t;
        img[t] = img[t] * fmadd(c, (T)co[j].a, T(1));
    }
}

// One ray: dispatch on its wave-uniform chunk count to a compile-time
// unrolled register body (rows longer than 64 * MAXC are streamed).
template <class T, class TC, int MAXC, bool NT = true, class Img>
__device__ __forceinline__ void mart_row(Img img, uint32_t shift, uint32_t wtot, T beta, const Coef<TC> *co, int n,
                                         T P, int lane)
{
    const int chunks = (n + 63) >> 6;   // wave-uniform
    if constexpr (MAXC > 16) {
        // 17 .. MAXC chunks: one register body of MAXC chunks, the entries
        // past the row masked (same sums as the streamed loop)
        if (chunks > 16 && chunks <= MAXC) {
            row_in_registers<T, TC, MAXC, NT>(img, shift, wtot, beta, co, n, P, lane);
            return;
        }
    }
    if (chunks > MAXC) {
        row_streamed<T, TC>(img, shift, wtot, beta, co, n, P, lane);
        return;
    }
    switch (chunks) {
#define USPG_ROW_CASE(C)                                                                          \
    case C:                                                                                       \
        if (C <= MAXC)                                                                            \
            row_in_registers<T, TC, (C <= MAXC ? C : 1), NT>(img, shift, wtot, beta, co, n, P, lane); \
        break;
        USPG_ROW_CASE(1) USPG_ROW_CASE(2) USPG_ROW_CASE(3) USPG_ROW_CASE(4)
        USPG_ROW_CASE(5) USPG_ROW_CASE(6) USPG_ROW_CASE(7) USPG_ROW_CASE(8)
        USPG_ROW_CASE(9) USPG_ROW_CASE(10) USPG_ROW_CASE(11) USPG_ROW_CASE(12)
        USPG_ROW_CASE(13) USPG_ROW_CASE(14) USPG_ROW_CASE(15) USPG_ROW_CASE(16)
#undef USPG_ROW_CASE
    default:
        break;
    }
}



// max_j |f_j - g_j| / g_j (eq. 19), values are positive so their bit
// patterns order like unsigned integers.
template <class T> struct Bits;
template <> struct Bits<float> { using U = unsigned int; };
template <> struct Bits<double> { using U = unsigned long long; };

template <class T>
__global__ __launch_bounds__(256) void max_rel_change(const T *f, const T *g, uint32_t n,
                                                      typename Bits<T>::U *out)
{
    __shared__ T sh[256];
    T m = T(0);
    for (uint32_t x = blockIdx.x * 256u + threadIdx.x; x < n; x += gridDim.x * 256u) {
        T d = (f[x] - g[x]) / g[x];
        d = d < T(0) ? -d : d;
        m = d > m ? d : m;
    }
    sh[threadIdx.x] = m;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) sh[threadIdx.x] = sh[threadIdx.x + s] > sh[threadIdx.x] ? sh[threadIdx.x + s] : sh[threadIdx.x];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        T v = sh[0];
        typename Bits<T>::U bits;
        __builtin_memcpy(&bits, &v, sizeof(v));
        atomicMax(out, bits);
    }
}

}  // namespace row
}  // namespace uspg
