// Lattice colouring of the reference view's rays (fixes MART's ray order).
//
// Two rays may be updated together only if they share no cell.  The
// conflict offsets (du, dw) = (|u1 - u2|, |w1 - w2|) of every pair of view-0
// rays that share a cell are collected on the device from the cell -> rays
// transpose of the reference rows (count, scan, fill, pair sweep).  The
// lattice (Ku, Kv), class (w mod Kv) Ku + (u mod Ku), is valid when no
// conflict offset has Ku | du and Kv | dw; rotating all rays by a view step
// maps cells to cells, so validity for view 0 carries to every view.  The
// smallest valid lattice is searched in order of increasing Ku Kv, ties to
// the smaller Ku.
#include "uspg_internal.hpp"

namespace uspg {
namespace {

__global__ __launch_bounds__(256) void count_cells(const int64_t *rowptr, const uint32_t *ids, int stride,
                                                   int64_t nrays, uint32_t *cnt)
{
    int64_t r = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    int lane = threadIdx.x & 63;
    if (r >= nrays) return;
    for (int64_t j = rowptr[r] + lane; j < rowptr[r + 1]; j += 64) atomicAdd(&cnt[ids[j * stride]], 1u);
}

__global__ __launch_bounds__(256) void fill_cells(const int64_t *rowptr, const uint32_t *ids, int stride,
                                                  int64_t nrays, const uint32_t *cptr,
                                                  uint32_t *cur, uint32_t *rays)
{
    int64_t r = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    int lane = threadIdx.x & 63;
    if (r >= nrays) return;
    for (int64_t j = rowptr[r] + lane; j < rowptr[r + 1]; j += 64) {
        uint32_t c = ids[j * stride];
        uint32_t pos = atomicAdd(&cur[c], 1u);
        rays[cptr[c] + pos] = (uint32_t)r;
    }
}

__global__ __launch_bounds__(256) void pair_offsets(const uint32_t *cptr, const uint32_t *rays,
                                                    int64_t ncells, int U, uint8_t *mark)
{
    int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= ncells) return;
    uint32_t b = cptr[c], e = cptr[c + 1];
    for (uint32_t x = b; x < e; ++x) {
        uint32_t rx = rays[x];
        int ux = (int)(rx % (uint32_t)U), wx = (int)(rx / (uint32_t)U);
        for (uint32_t y = x + 1; y < e; ++y) {
            uint32_t ry = rays[y];
            int uy = (int)(ry % (uint32_t)U), wy = (int)(ry / (uint32_t)U);
            int du = ux > uy ? ux - uy : uy - ux;
            int dw = wx > wy ? wx - wy : wy - wx;
            size_t at = (size_t)dw * U + du;
            if (!mark[at]) mark[at] = 1;
        }
    }
}

bool lattice_ok(const std::vector<uint8_t> &mark, int U, int V, int ku, int kv)
{
    for (int dw = 0; dw < V; dw += kv)
        for (int du = 0; du < U; du += ku)
            if (mark[(size_t)dw * U + du]) return false;
    return true;
}

}  // namespace

int conflict_marks(const int64_t *rowptr, const uint32_t *ids, int stride, int64_t nrays, int64_t nnz,
                   int64_t ncells, int U, uint8_t *mark, hipStream_t s)
{
    uint32_t *cnt = nullptr, *cptr = nullptr, *rays = nullptr;
    int rc = USPG_OK;
    do {
        if (dev_malloc((void **)&cnt, sizeof(uint32_t) * (ncells + 1)) != hipSuccess ||
            dev_malloc((void **)&cptr, sizeof(uint32_t) * (ncells + 1)) != hipSuccess ||
            dev_malloc((void **)&rays, sizeof(uint32_t) * (nnz > 0 ? nnz : 1)) != hipSuccess) {
            rc = fail(USPG_E_NOMEM, "colouring: device allocation failed");
            break;
        }
        if (hipMemsetAsync(cnt, 0, sizeof(uint32_t) * (ncells + 1), s) != hipSuccess) {
            rc = fail(USPG_E_HIP, "colouring: memset failed");
            break;
        }
        const unsigned rb = (unsigned)((nrays * 64 + 255) / 256);
        hipLaunchKernelGGL(count_cells, dim3(rb), dim3(256), 0, s, rowptr, ids, stride, nrays, cnt);
        if ((rc = exclusive_scan_u32(cnt, cptr, ncells, s)) != USPG_OK) break;
        if (hipMemsetAsync(cnt, 0, sizeof(uint32_t) * (ncells + 1), s) != hipSuccess) {
            rc = fail(USPG_E_HIP, "colouring: memset failed");
            break;
        }
        hipLaunchKernelGGL(fill_cells, dim3(rb), dim3(256), 0, s, rowptr, ids, stride, nrays, cptr, cnt, rays);
        hipLaunchKernelGGL(pair_offsets, dim3((unsigned)((ncells + 255) / 256)), dim3(256), 0, s,
                           cptr, rays, ncells, U, mark);
        if (hipGetLastError() != hipSuccess) { rc = fail(USPG_E_HIP, "colouring: launch failed"); break; }
        if (hipStreamSynchronize(s) != hipSuccess) { rc = fail(USPG_E_HIP, "colouring failed"); break; }
    } while (0);
    (void)dev_free(cnt); (void)dev_free(cptr); (void)dev_free(rays);
    return rc;
}

int choose_lattice(uspg_coeffs *c)
{
    const int U = c->scan.det_u, V = c->scan.det_v;
    if (c->scan.colour_u > 0 || c->scan.colour_v > 0) {
        int ku = c->scan.colour_u > 0 ? c->scan.colour_u : 1;
        int kv = c->scan.colour_v > 0 ? c->scan.colour_v : 1;
        if (ku > U || kv > V || !lattice_ok(c->mark, U, V, ku, kv))
            return fail(USPG_E_ARG, "requested colour lattice puts two rays that share a cell in one class");
        c->Ku = ku; c->Kv = kv;
        return USPG_OK;
    }
    const int64_t total = (int64_t)U * V;
    for (int64_t P = 1; P <= total; ++P) {
        for (int64_t ku = 1; ku <= P && ku <= U; ++ku) {
            if (P % ku) continue;
            int64_t kv = P / ku;
            if (kv > V) continue;
            if (lattice_ok(c->mark, U, V, (int)ku, (int)kv)) {
                c->Ku = (int)ku;
                c->Kv = (int)kv;
                return USPG_OK;
            }
        }
    }
    return fail(USPG_E_INTERNAL, "no valid colour lattice");
}

int colour_reference_view(uspg_coeffs *c, hipStream_t s)
{
    const int U = c->scan.det_u, V = c->scan.det_v;
    uint8_t *mark = nullptr;
    c->mark.assign((size_t)U * V, 0);
    if (dev_malloc((void **)&mark, (size_t)U * V) != hipSuccess) return fail(USPG_E_NOMEM, "colouring: allocation");
    int rc = USPG_OK;
    if (hipMemsetAsync(mark, 0, (size_t)U * V, s) != hipSuccess) rc = fail(USPG_E_HIP, "colouring: memset failed");
    // ids live in the device layout, as the first word of each (id,
    // coefficient) pair
    const int stride = (int)((c->scan.coeff_dtype == USPG_F64 ? sizeof(Coef<double>) : sizeof(Coef<float>)) / 4);
    if (rc == USPG_OK)
        rc = conflict_marks(c->rowptr.as<int64_t>(), c->coef.as<uint32_t>(), stride, c->nrays, c->nnz, c->Wtot, U,
                            mark, s);
    if (rc == USPG_OK && hipMemcpy(c->mark.data(), mark, (size_t)U * V, hipMemcpyDeviceToHost) != hipSuccess)
        rc = fail(USPG_E_HIP, "colouring: copy failed");
    (void)dev_free(mark);
    if (rc != USPG_OK) return rc;
    return choose_lattice(c);
}

}  // namespace uspg
