// Internal declarations of the USPG / USCG MART library (gfx950).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/uspg.h"

namespace uspg {

constexpr double kTwoPi = 6.283185307179586476925286766559;

// Thread-local error message behind uspg_last_error().
void set_error(const std::string &msg);
int fail(int code, const std::string &msg);

#define USPG_HIP(expr)                                                                   \
    do {                                                                                 \
        hipError_t e_ = (expr);                                                          \
        if (e_ != hipSuccess)                                                            \
            return ::uspg::fail(USPG_E_HIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

// One stored coefficient: the cell id in the device layout and the value,
// interleaved so that a row is read with one vector load per entry.
template <class TC> struct Coef;
template <> struct alignas(8) Coef<float> {
    uint32_t id;
    float a;
};
template <> struct alignas(16) Coef<double> {
    uint32_t id;
    uint32_t pad;
    double a;
};

// Counted device allocation and release (every library allocation).
hipError_t dev_malloc(void **p, size_t n);
hipError_t dev_free(void *p);

// Device buffer of a handle: allocated by the library (owned) or a piece of
// a caller's work space (borrowed, never freed here).
struct DevBuf {
    void *p = nullptr;
    size_t bytes = 0;
    bool owned = true;
    DevBuf() = default;
    DevBuf(const DevBuf &) = delete;
    DevBuf &operator=(const DevBuf &) = delete;
    ~DevBuf() { release(); }
    int alloc(size_t n);
    void borrow(void *q, size_t n)
    {
        release();
        p = q;
        bytes = n;
        owned = false;
    }
    void release();
    template <class T> T *as() const { return static_cast<T *>(p); }
};

// Carves 256-byte aligned buffers out of a caller's work space, or only adds
// up their sizes when base is null.
struct Arena {
    char *base = nullptr;
    size_t cap = 0, off = 0;
    static size_t rounded(size_t n) { return ((n ? n : 1) + 255) / 256 * 256; }
    int take(DevBuf &b, size_t n);
};

}  // namespace uspg

// Grid handle: host tables plus their device copies.
struct uspg_grid {
    int nr = 0, nz = 0;
    double R = 0, H = 0, r = 0, h = 0, z0 = 0;
    int rule = 0;
    std::vector<int32_t> ng;     // sectors per ring
    std::vector<int64_t> head;   // ring heads, nr + 1 entries
    int64_t c2d = 0, ncells = 0;
    int device = 0;
    uspg::DevBuf d_ng, d_head;   // int32 [nr], int64 [nr + 1]
    uspg::DevBuf d_cs;           // double2 [c2d]: cos / sin of every sector's lower boundary
};

// Coefficient handle: reference-view rows in the device (wedge-major) cell
// numbering, lattice colouring and the tables of the wedge layout.
//
// Device image layout (trace_walk.hpp, wedge_tables): sector s = a k_i + b of
// ring i in slice k is stored at a * Wc + k * Cq + hq_i + b * grp, so
// rotating by v view steps adds v * Wc modulo Wtot = q * Wc (>= cells: the
// ring groups are padded).
struct uspg_coeffs {
    const uspg_grid *g = nullptr;
    uspg_scan_desc scan{};
    int device = 0;
    int q = 0;
    std::vector<int32_t> kq, hq;  // per ring
    std::vector<int32_t> ring_of_off;  // per within-slice offset (-1: padding)
    int grp = 1;
    int64_t Cq = 0, Wc = 0, Wtot = 0;
    int64_t nrays = 0, nnz = 0;
    int32_t max_row = 0;
    int Ku = 1, Kv = 1;
    std::vector<uint8_t> mark;    // conflict offsets [det_v][det_u]
    uspg::DevBuf rowptr;          // int64 [nrays + 1]
    uspg::DevBuf coef;            // Coef<float or double> [nnz]: (cell id, coefficient) pairs
    uspg::DevBuf d_kq, d_hq;      // int32 [nr]
    uspg::DevBuf d_ring_of_off;   // int32 [Cq]: ring of each within-slice offset, -1 padding
    int64_t device_bytes = 0;
    // Segment-record mode (weights == USPG_WEIGHTS_SEGMENTS): the rows of a
    // view are rebuilt from these records; the image stays in the paper's
    // numbering and rowptr / ids / a and the wedge tables are unused.
    bool segments = false;
    int64_t nseg = 0;             // records
    int32_t max_seg = 0;          // records of the longest ray
    uspg::DevBuf segptr;          // int64 [nrays + 1]
    uspg::DevBuf seg_sr;          // uint32 [nseg]: slice << 16 | ring
    uspg::DevBuf seg_pa, seg_pb;  // double [nseg]: reference azimuths of the two ends
    uspg::DevBuf seg_partner;     // int32 [nseg]: earlier record of the ray in the same ring and slice, -1
    std::vector<int64_t> view_nnz;  // re-binned entries of every view's rows
    // Kept re-binned rows (view_rows == 0 and small enough): per view v the
    // rows rowptr view_rowptr[v (nrays + 1) ...] (relative to the view's first
    // entry view_start[v]) of (paper cell, 1) pairs in view_coef.
    uspg::DevBuf view_rowptr;     // int64 [n_views][nrays + 1]
    uspg::DevBuf view_coef;       // Coef<float> [sum of view_nnz]
    std::vector<int64_t> view_start;
    uspg::DevBuf d_view_start;    // int64 [n_views + 1], device copy of view_start
    int32_t view_max_row = 0;
    // Coded rows (cone beam, coded_rows.hpp): per detector column its
    // in-plane path, per ray its code; mart_run reads these instead of the
    // stored rows (which stay for explicit rays and the other solvers).
    bool coded = false;
    int64_t coded_rays = 0, explicit_rays = 0;
    uspg::DevBuf d_colptr;        // int64 [det_u + 1]: first record of each column
    uspg::DevBuf d_colt;          // double [records]: piece starts (a column closes with its end)
    uspg::DevBuf d_colid;         // uint32 [records]: slice-0 cell id of each piece
    uspg::DevBuf d_codes;         // RayCode [nrays]
    uspg::DevBuf d_words;         // uint64: piece / slice bits of the coded rays
    // Two-call build: after the size query the handle is pending (counts
    // only) until a second call fills the caller's work space.
    bool pending = false;
    bool want_codes = false;
    size_t ws_needed = 0;
    uspg::DevBuf pend_cnt;        // uint32 [nrays + 1]: entries per ray (library memory, until the fill)
    uspg::DevBuf pend_colptr;     // int64 [det_u + 1]: coded rows, column record offsets (until the fill)
    uspg::DevBuf pend_woff;       // int64 [nrays + 1]: coded rows, mask word offsets (until the fill)
    int64_t pend_nrec = 0, pend_nwords = 0;
};

namespace uspg {

// Whether the rows of every view are stored (kept re-binned rows of SEGMENTS
// coefficients) rather than the reference view shifted; the image cells the
// solver works on (device layout for shifted rows, paper numbering for kept
// rows); the longest stored row; and the stored coefficient type.
inline bool kept_rows(const uspg_coeffs *c) { return c->segments && c->view_coef.p != nullptr; }
inline int64_t solve_cells(const uspg_coeffs *c) { return c->segments ? c->g->ncells : c->Wtot; }
inline int32_t stored_max_row(const uspg_coeffs *c) { return c->segments ? c->view_max_row : c->max_row; }
inline int32_t stored_coeff_dtype(const uspg_coeffs *c) { return c->segments ? (int32_t)USPG_F32 : c->scan.coeff_dtype; }

// Rings per group of the blocked device layout.
constexpr int kRingGroup = 4;

// trace.hip: the count pass (pend_cnt, nnz, max_row) and the fill pass
// (into rowptr and coef, already set).
int trace_count_rows(uspg_coeffs *c, hipStream_t s);
int trace_fill_rows(uspg_coeffs *c, hipStream_t s);
// colour.hip
int colour_reference_view(uspg_coeffs *c, hipStream_t s);
// ORs into mark (device, det_u * det_v bytes) the offsets of every pair of
// rays of the CSR that share a cell; entry j's cell id is ids[j * stride]
// (< ncells); synchronises s.
int conflict_marks(const int64_t *rowptr, const uint32_t *ids, int stride, int64_t nrays, int64_t nnz,
                   int64_t ncells, int U, uint8_t *mark, hipStream_t s);
// Smallest valid lattice for c->mark (or the requested one).
int choose_lattice(uspg_coeffs *c);
// segments.hip
int segments_reference_view(uspg_coeffs *c, hipStream_t s);
int colour_segments(uspg_coeffs *c, hipStream_t s);
int segments_row(const uspg_coeffs *c, int view, int64_t ray, std::vector<int64_t> &cells);
// coded.hip: coded rows of a cone-beam coefficient set: the sizes (after the
// count pass: pend_nrec, pend_nwords) and the codes (after tracing, into
// d_colptr, d_colt, d_colid, d_codes, d_words, already set).
int code_count(uspg_coeffs *c, hipStream_t s);
int code_fill(uspg_coeffs *c, hipStream_t s);
// scan.hip
int exclusive_scan_u32_to_i64(const uint32_t *in, int64_t *out, int64_t n, hipStream_t s);
int exclusive_scan_u32(const uint32_t *in, uint32_t *out, int64_t n, hipStream_t s);
// mart.hip
int mart_launch(const uspg_coeffs *c, int dtype, const void *proj, void *image, void *work,
                int n_sweeps, double beta, double tol, int32_t *sweeps_done, hipStream_t s);
int mart_timing(int enable, hipStream_t s, double *batch_ms, int64_t *batch_launches);
// Whether batch timing is on, and adding a timed run of launches to it.
bool stream_capturing(hipStream_t s);
// Whether coefficient loads take the non-temporal hint: true unless the
// coefficient sets and images a launch reads fit the last-level cache.
bool stream_coefs(size_t coef_bytes, size_t image_bytes);
// Device bytes of the coefficient rows a solve reads (kept view rows or the
// stored reference rows).
inline size_t coef_set_bytes(const uspg_coeffs *c) { return c->view_coef.p ? c->view_coef.bytes : c->coef.bytes; }
bool mart_timing_on(hipStream_t s);
// While one lives, mart_launch on this thread records no timing events.
struct UntimedScope {
    bool prev;
    UntimedScope();
    ~UntimedScope();
};
void mart_timing_add(hipStream_t s, int64_t ns, int64_t launches);
// One (view, class) batch of the single-problem kernel over explicit rows
// of (id, coefficient) pairs of float coefficients (shift added mod wtot);
// nch bounds the register path from the longest row.
int rows_batch_launch(const uspg_coeffs *c, int dtype, const void *proj_view, void *f, const int64_t *rowptr,
                      const void *coef, uint32_t shift, uint32_t wtot, int cl, double beta, int max_row,
                      hipStream_t s);
// mart_rebin.hip: mart_run for segment-record coefficients.
int rebin_launch(const uspg_coeffs *c, int dtype, const void *proj, void *image, void *work, int n_sweeps,
                 double beta, double tol, int32_t *sweeps_done, hipStream_t s);
// Grid cap of the single-problem batch kernel, in workgroups.
int batch_grid_cap();
// Batch (view v, class cl) of problem c on its device-layout image f with the
// single-problem kernel (same bits as the lockstep kernel's step).
int batch_step(const uspg_coeffs *c, int dtype, const void *proj, void *f, double beta, int v, int cl,
               hipStream_t s);
// Permute an image between the paper's numbering and the device layout
// (to_native_layout = 1: paper -> device; 0: device -> paper).
int layout_permute(const uspg_coeffs *c, int dtype, const void *src, void *dst, int to_native_layout,
                   hipStream_t s);
// api.hip
int check_device(int want);
// A built (not pending) coefficient handle on the current device.
int check_coeffs(const uspg_coeffs *c);
int current_device_id(int *dev);
// remap.hip
int remap_launch(const uspg_grid *g, int dtype, const void *image, void *cart, int nc, int mode,
                 hipStream_t s);

}  // namespace uspg
