// The single-problem batch kernel: one (view, colour class) batch of
// Sp-MART over the reference rows shifted to the view (Sec. III.C-D,
// eqs. 17-18), one wavefront per ray through the per-ray routine of
// mart_row.hpp.  Launched by mart.hip.
#pragma once

#include "mart_row.hpp"

namespace uspg {
namespace batchk {

constexpr int kWaves = 4;             // wavefronts per workgroup
constexpr int kBlock = 64 * kWaves;

template <class T, class TC>
struct BatchArgs {
    const int64_t *rowptr;
    const Coef<TC> *co;
    const T *P;        // projections of the view, [rays]
    T *f;              // wedge-major image
    uint32_t shift;    // v * Wc (mod Wtot)
    uint32_t wtot;
    int U, cu, cw, Ku, Kv, nu, ncls, nblk;
    T beta;
};

// The launcher caps the grid (16 workgroups per CU) and each wavefront
// strides through the class by the grid's wavefront count; the rays of a
// class share no cell, so the assignment changes no result.  NT: load the
// coefficients with the non-temporal hint (the launcher's choice by the
// size of the coefficient set; the same bits either way).
template <class T, class TC, int MAXC, bool NT = true>
__global__ __launch_bounds__(kBlock) void mart_batch(BatchArgs<T, TC> A)
{
    const int lane = threadIdx.x & 63;
    const int total = A.nblk * kWaves;
    for (int x = row::xcd_block(blockIdx.x, A.nblk) * kWaves + (threadIdx.x >> 6); x < A.ncls; x += total) {
        const int w = A.cw + (x / A.nu) * A.Kv;
        const int u = A.cu + (x % A.nu) * A.Ku;
        const int64_t r = (int64_t)w * A.U + u;
        const int64_t beg = A.rowptr[r];
        const int n = (int)(A.rowptr[r + 1] - beg);
        if (n == 0) continue;
        row::mart_row<T, TC, MAXC, NT>(A.f, A.shift, A.wtot, A.beta, A.co + beg, n, A.P[r], lane);
    }
}

}  // namespace batchk
}  // namespace uspg
