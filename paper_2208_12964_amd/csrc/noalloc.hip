// Allocation-free MART entry point: mart_run with its work space taken from a
// fixed device array of this library instead of a caller buffer, for callers
// that cannot allocate device memory (code under HIP graph capture, serving
// loops that forbid allocation).
//
// The array lives in the code object, so every device the library runs on
// holds its own copy from module load until the process ends.  Host code
// never passes the array's name to a kernel (on the host it is only a
// stand-in symbol): the device address of each device's copy is looked up
// once with hipGetSymbolAddress, with that device current, and used from then
// on.  Every call on one device shares that device's copy, so calls that
// overlap on one device (two streams, two threads) race; the work space is
// fully rewritten by each call (the image permuted into it, the stopping
// rule's maximum cleared every sweep), so nothing carries over between calls.
#include <mutex>

#include "uspg_internal.hpp"

namespace uspg {
namespace {

constexpr int kMaxDevices = 64;

// 64 MiB: the device-layout image of up to 16,777,216 FP32 cells (8,388,608
// FP64 cells), half of that with the stopping rule (two images).
__device__ __align__(256) unsigned char scratch[USPG_NOALLOC_SCRATCH_BYTES];

std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {nullptr};

// Device address of this device's copy of the scratch array (looked up on
// the first call with the device current).
int scratch_address(int dev, void **out)
{
    if (dev < 0 || dev >= kMaxDevices) return fail(USPG_E_ARG, "device ordinal out of range");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(USPG_E_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return USPG_OK;
}

}  // namespace
}  // namespace uspg

using namespace uspg;

extern "C" int mart_run_noalloc(const uspg_coeffs *c, int32_t dtype, const void *proj, void *image,
                                int32_t n_sweeps, double beta, double tol, int32_t *sweeps_done, void *stream)
{
    if (!c || !proj || !image) return fail(USPG_E_ARG, "null argument");
    if (dtype != USPG_F32 && dtype != USPG_F64) return fail(USPG_E_ARG, "dtype");
    if (n_sweeps < 0 || !(beta > 0) || !(tol >= 0)) return fail(USPG_E_ARG, "n_sweeps >= 0, beta > 0, tol >= 0");
    const size_t need = uspg_mart_workspace_bytes(c, dtype, tol);
    if (need > (size_t)USPG_NOALLOC_SCRATCH_BYTES)
        return fail(USPG_E_NOMEM, "mart_run_noalloc: the problem needs " + std::to_string(need) +
                                      " bytes of work space, more than the fixed " +
                                      std::to_string((size_t)USPG_NOALLOC_SCRATCH_BYTES));
    int rc = check_coeffs(c);
    if (rc != USPG_OK) return rc;
    if (tol > 0 && stream_capturing((hipStream_t)stream))
        return fail(USPG_E_ARG, "tol > 0 synchronises the stream once per sweep and cannot be graph-captured");
    void *work = nullptr;
    if ((rc = scratch_address(c->device, &work)) != USPG_OK) return rc;
    UntimedScope untimed;   // timing would create events
    return mart_launch(c, dtype, proj, image, work, n_sweeps, beta, tol, sweeps_done, (hipStream_t)stream);
}
