// The single-problem batch kernel over coded cone-beam rows: one (view,
// colour class) batch of Sp-MART (Sec. III.C-D, eqs. 17-18), one wavefront
// per ray, with every row entry rebuilt from its column's in-plane path and
// the ray's piece and slice bits (coded_rows.hpp) instead of being read
// from a stored (id, coefficient) stream.  The rebuilt entries equal the
// stored ones bit for bit and take the same lanes, so the ray sums, the
// corrections and the image are the same bits as mart_batch's.  Rays whose
// rows were left explicit run mart_batch's per-ray routine on the stored
// rows.  Launched by mart.hip.
#pragma once

#include "coded_rows.hpp"
#include "mart_batch.hpp"
#include "mart_row.hpp"

namespace uspg {
namespace batchk {

// The codes of one coefficient set (coded_rows.hpp).
struct CodeTab {
    const coded::RayCode *codes;     // per ray
    const uint64_t *words;           // piece / slice bits, two words per 64 entries
    const double *t;                 // column records: piece starts
    const uint32_t *id0;             // column records: slice-0 cell ids
    coded::CodeGeo Q;
    int binary;
};

template <class T, class TC>
struct CodedArgs {
    BatchArgs<T, TC> B;              // class, view, image, stored rows of explicit rays
    CodeTab K;
    int band;                        // ray order: bands of `band` class rows, w fastest inside a band
};

// Two consecutive FP64 column records, 8-byte aligned.
typedef double PieceSpan __attribute__((ext_vector_type(2), aligned(8)));

// One coded row of exactly C chunks of 64 entries, kept in registers as in
// row::row_in_registers (same masking, same reduction order).  Straight-line
// code, so every chunk's table loads, then every gather, are issued before
// the first wait.
template <class T, class TC, int C, class W>
__device__ __forceinline__ void coded_row(const CodeTab &K, W words, T *f, uint32_t shift, uint32_t wtot, T beta,
                                          const coded::RayCode &rc, T P, int lane, double *planes)
{
#pragma clang fp contract(off)
    const int dk = coded::code_dk(rc), kinit = coded::code_kinit(rc), J = coded::code_planes(rc);
    // bounds of the slices the ray crosses, 0 .. J + 1 (t0, the J crossed
    // planes, then the next plane or t1); the previous ray of this
    // wavefront has finished reading the table
    for (int j = lane; j <= J + 1; j += 64) planes[j] = coded::slice_bound(K.Q, kinit, dk, J, rc.t0, rc.t1, rc.ez, j);
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");

    const int n = rc.n;
    // cell of (piece p, slice bound j): id0[p] + (kinit + dk j) Cq + shift,
    // with the uniform part folded (wraps in 32 bits; the sum is < 2 wtot)
    const uint32_t base = (uint32_t)kinit * K.Q.Cq + shift;
    const int step = dk * (int)K.Q.Cq;
    uint32_t pacc = (uint32_t)rc.p0;
    int jacc = coded::code_j0(rc);
    uint32_t id[C];
    T av[C], fv[C];
#pragma unroll
    for (int k = 0; k < C; ++k) {
        // bit i of chunk k's words is entry 64 k + i + 1: the bits below this
        // lane are the entries of the chunk up to this one
        const uint64_t pw = words[rc.word + 2 * k];
        const uint64_t kw = words[rc.word + 2 * k + 1];
        const uint32_t p =
            pacc + __builtin_amdgcn_mbcnt_hi((uint32_t)(pw >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)pw, 0u));
        const int j =
            jacc + (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(kw >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)kw, 0u));
        pacc += (uint32_t)__builtin_popcountll(pw);
        jacc += __builtin_popcountll(kw);
        // the piece's start and end (the next record's start) in one 16-byte load
        const PieceSpan ts = *reinterpret_cast<const PieceSpan *>(K.t + p);
        const double len = coded::entry_length(ts.x, ts.y, planes[j], planes[j + 1], rc.L);
        const TC a = K.binary ? TC(1) : TC(len);
        const uint32_t t = K.id0[p] + base + (uint32_t)__mul24(j, step);
        const uint32_t tw = t - wtot;
        id[k] = tw < t ? tw : t;                        // t mod wtot (t < 2 wtot < 2^32)
        av[k] = lane + 64 * k < n ? (T)a : T(0);       // masked, not branched
    }
#pragma unroll
    for (int k = 0; k < C; ++k) fv[k] = f[id[k]];
    T acc = T(0), amax = T(0);
#pragma unroll
    for (int k = 0; k < C; ++k) {
        acc = row::fmadd(av[k], fv[k], acc);
        amax = av[k] > amax ? av[k] : amax;
    }
    acc = row::wave_sum(acc);
    amax = row::wave_max(amax);
    if (!(acc > T(0)) || !(amax > T(0))) return;
    const T c = beta * (P / acc - T(1)) / amax;
#pragma unroll
    for (int k = 0; k < C; ++k)
        if (lane + 64 * k < n) f[id[k]] = fv[k] * row::fmadd(c, av[k], T(1));
}

// A coded row of any chunk count up to MAXC (at most 16): the straight-line
// body of its exact count.
template <class T, class TC, int MAXC, class W>
__device__ __forceinline__ void coded_row_any(const CodeTab &K, W words, T *f, uint32_t shift, uint32_t wtot, T beta,
                                              const coded::RayCode &rc, T P, int lane, double *planes)
{
    switch ((rc.n + 63) >> 6) {
#define USPG_CODED_CASE(C)                                                                                 \
    case C:                                                                                                \
        if (C <= MAXC) coded_row<T, TC, (C <= MAXC ? C : 1)>(K, words, f, shift, wtot, beta, rc, P, lane, planes); \
        break;
        USPG_CODED_CASE(1) USPG_CODED_CASE(2) USPG_CODED_CASE(3) USPG_CODED_CASE(4)
        USPG_CODED_CASE(5) USPG_CODED_CASE(6) USPG_CODED_CASE(7) USPG_CODED_CASE(8)
        USPG_CODED_CASE(9) USPG_CODED_CASE(10) USPG_CODED_CASE(11) USPG_CODED_CASE(12)
        USPG_CODED_CASE(13) USPG_CODED_CASE(14) USPG_CODED_CASE(15) USPG_CODED_CASE(16)
#undef USPG_CODED_CASE
    default:
        break;
    }
}

// Class position x of the band order: bands of `band` class rows, w
// fastest inside a band.
template <class T, class TC>
__device__ __forceinline__ int64_t class_ray(const CodedArgs<T, TC> &A, int x)
{
    const int nw = A.B.ncls / A.B.nu;
    const int wb = x / (A.band * A.B.nu);
    const int xl = x - wb * A.band * A.B.nu;
    const int h = nw - wb * A.band < A.band ? nw - wb * A.band : A.band;
    const int u = A.B.cu + (xl / h) * A.B.Ku;
    const int w = A.B.cw + (wb * A.band + xl % h) * A.B.Kv;
    return (int64_t)w * A.B.U + u;
}

// One wavefront per ray, each wavefront striding through the class; empty
// rays and explicit rows (run by mart_explicit) are skipped.  MAXC bounds
// the chunk count of the coefficient set's longest row (at most 16).
// The ray headers, bit words and projections come in as their own
// restrict-qualified arguments: their addresses are wavefront-uniform and
// no store of the kernel can alias them, so the compiler reads them with
// scalar loads into scalar registers and counts the bits on the scalar unit
// (116 -> 102 vector registers; 85.9 -> 80.5 us per batch on the 256-ring
// cone).  Each wavefront loads the header and measurement of its next ray
// before it runs the current one, so their latency hides behind it
// (79.1 -> 75.9 us).
template <class T, class TC, int MAXC>
__global__ __launch_bounds__(kBlock) void mart_coded(CodedArgs<T, TC> A, const coded::RayCode *__restrict__ codes,
                                                     const uint64_t *__restrict__ words, const T *__restrict__ Pv)
{
    __shared__ double planes[kWaves][coded::kMaxPlanes + 2];
    const int lane = threadIdx.x & 63;
    const int wv = threadIdx.x >> 6;
    const int total = A.B.nblk * kWaves;
    int x = __builtin_amdgcn_readfirstlane(row::xcd_block(blockIdx.x, A.B.nblk) * kWaves + wv);
    coded::RayCode nx{};   // the next ray's header and measurement
    T np = T(0);
    if (x < A.B.ncls) {
        const int64_t r0 = class_ray(A, x);
        nx = codes[r0];
        np = Pv[r0];
    }
    for (; x < A.B.ncls; x += total) {
        const coded::RayCode rc = nx;
        const T P = np;
        if (x + total < A.B.ncls) {
            const int64_t r1 = class_ray(A, x + total);
            nx = codes[r1];
            np = Pv[r1];
        }
        if (rc.n == 0 || rc.word < 0) continue;
        coded_row_any<T, TC, MAXC>(A.K, words, A.B.f, A.B.shift, A.B.wtot, A.B.beta, rc, P, lane, planes[wv]);
    }
}

// The explicit rows of a class (rays whose rows the code does not
// reproduce), mart_batch's per-ray routine on the stored rows; launched after
// mart_coded for the same batch only when the coefficient set has such rays.
template <class T, class TC, int MAXC, bool NT = true>
__global__ __launch_bounds__(kBlock) void mart_explicit(CodedArgs<T, TC> A)
{
    const int lane = threadIdx.x & 63;
    const int total = A.B.nblk * kWaves;
    for (int x = row::xcd_block(blockIdx.x, A.B.nblk) * kWaves + (threadIdx.x >> 6); x < A.B.ncls; x += total) {
        const int64_t r = class_ray(A, x);
        const coded::RayCode rc = A.K.codes[r];
        if (rc.n == 0 || rc.word >= 0) continue;
        row::mart_row<T, TC, MAXC, NT>(A.B.f, A.B.shift, A.B.wtot, A.B.beta, A.B.co + A.B.rowptr[r], rc.n, A.B.P[r],
                                       lane);
    }
}

}  // namespace batchk
}  // namespace uspg
