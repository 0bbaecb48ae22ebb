// USPG -> Cartesian grid for display (Sec. II.B).
//
// One thread per pixel column (ix, iy) finds the cell once and copies it for
// every slice (reads gather across slices, writes are coalesced per slice).
//   POINT: the cell containing the pixel centre; centres exactly on a
//     diagonal sit at an odd multiple of pi/4 and take the sector of that
//     exact angle.
//   BIJECTION (paper grid, nc = 2 Nr): square ring n and circular ring n hold
//     4(2n - 1) cells each (eq. 1, Fig. 2); the square ring's pixels are
//     ranked anticlockwise from the +x axis in closed form (right edge upper
//     half, top, left, bottom, right edge lower half) and pixel j takes
//     sector j of ring n.
#include <cmath>

#include "uspg_internal.hpp"

// the pixel -> cell decision is floating point deciding an integer: keep the
// arithmetic unfused, as on the host
#pragma clang fp contract(off)

namespace uspg {
namespace {

__device__ int64_t point_cell(int X, int Y, int nc, double R, double r, int nr, const int32_t *ng,
                              const int64_t *head)
{
    double x = X * R / nc, y = Y * R / nc;
    double rho = sqrt(x * x + y * y);
    if (!(rho < R)) return -1;
    int i = (int)floor(rho / r);
    if (i >= nr) i = nr - 1;
    int n = ng[i];
    int s;
    if (X == Y || X == -Y) {
        int oct = (X > 0 && Y > 0) ? 1 : (X < 0 && Y > 0) ? 3 : (X < 0 ? 5 : 7);
        s = (int)(((int64_t)oct * n) / 8);
    } else {
        double phi = atan2(y, x);
        if (phi < 0) phi += kTwoPi;
        s = (int)floor(phi / (kTwoPi / n));
        s = s < 0 ? 0 : (s >= n ? n - 1 : s);
    }
    return head[i] + s;
}

__device__ int64_t bijection_cell(int X, int Y, const int64_t *head)
{
    int ax = X < 0 ? -X : X, ay = Y < 0 ? -Y : Y;
    int M = ax > ay ? ax : ay;      // 2n - 1
    int n = (M + 1) / 2;
    int rank;
    if (X == M && Y > 0) rank = (Y - 1) / 2;                       // right edge, upper half
    else if (Y == M && X < M) rank = n + (M - 2 - X) / 2;           // top edge, leftwards
    else if (X == -M && Y < M) rank = 3 * n - 1 + (M - 2 - Y) / 2;  // left edge, downwards
    else if (Y == -M && X > -M) rank = 5 * n - 2 + (X + M - 2) / 2; // bottom edge, rightwards
    else rank = 7 * n - 3 + (Y + M - 2) / 2;                        // right edge, lower half
    return head[n - 1] + rank;
}

template <class T>
__global__ __launch_bounds__(256) void remap_kernel(const T *img, T *cart, int nc, int mode, double R,
                                                    double r, int nr, int nz, int64_t c2d,
                                                    const int32_t *ng, const int64_t *head)
{
    int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
    int64_t plane = (int64_t)nc * nc;
    if (p >= plane) return;
    int iy = (int)(p / nc), ix = (int)(p % nc);
    int X = 2 * ix + 1 - nc, Y = 2 * iy + 1 - nc;
    int64_t cell = mode == USPG_REMAP_BIJECTION ? bijection_cell(X, Y, head)
                                                : point_cell(X, Y, nc, R, r, nr, ng, head);
    for (int k = 0; k < nz; ++k) cart[k * plane + p] = cell < 0 ? T(0) : img[k * c2d + cell];
}

}  // namespace

int remap_launch(const uspg_grid *g, int dtype, const void *image, void *cart, int nc, int mode,
                 hipStream_t s)
{
    int64_t plane = (int64_t)nc * nc;
    unsigned blocks = (unsigned)((plane + 255) / 256);
    if (dtype == USPG_F32)
        hipLaunchKernelGGL(remap_kernel<float>, dim3(blocks), dim3(256), 0, s, (const float *)image,
                           (float *)cart, nc, mode, g->R, g->r, g->nr, g->nz, g->c2d,
                           g->d_ng.as<int32_t>(), g->d_head.as<int64_t>());
    else
        hipLaunchKernelGGL(remap_kernel<double>, dim3(blocks), dim3(256), 0, s, (const double *)image,
                           (double *)cart, nc, mode, g->R, g->r, g->nr, g->nz, g->c2d,
                           g->d_ng.as<int32_t>(), g->d_head.as<int64_t>());
    USPG_HIP(hipGetLastError());
    return USPG_OK;
}

}  // namespace uspg
