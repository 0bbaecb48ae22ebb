// C ABI entry points: argument checks, handle construction, dispatch.
#include <atomic>
#include <cmath>
#include <cstring>

#include <algorithm>

#include "coded_rows.hpp"
#include "trace_walk.hpp"
#include "uspg_internal.hpp"

namespace uspg {

static thread_local std::string g_last_error;

void set_error(const std::string &msg) { g_last_error = msg; }

int fail(int code, const std::string &msg)
{
    set_error(msg);
    return code;
}

// Device allocations of the library go through these two calls: they keep
// a count of live allocations and can fail on purpose (uspg_debug_alloc),
// so that error paths can be shown to free what they took.
static std::atomic<int64_t> g_live_allocs{0};
static std::atomic<int64_t> g_fail_after{0};

hipError_t dev_malloc(void **p, size_t n)
{
    *p = nullptr;
    if (g_fail_after.load() > 0 && g_fail_after.fetch_sub(1) == 1) return hipErrorOutOfMemory;
    hipError_t e = hipMalloc(p, n);
    if (e == hipSuccess) ++g_live_allocs;
    else *p = nullptr;
    return e;
}

hipError_t dev_free(void *p)
{
    if (!p) return hipSuccess;
    --g_live_allocs;
    return hipFree(p);
}

int DevBuf::alloc(size_t n)
{
    release();
    if (n == 0) n = 1;
    if (dev_malloc(&p, n) != hipSuccess) {
        p = nullptr;
        (void)hipGetLastError();
        return fail(USPG_E_NOMEM, "device allocation of " + std::to_string(n) + " bytes failed");
    }
    bytes = n;
    owned = true;
    return USPG_OK;
}

void DevBuf::release()
{
    if (p && owned) (void)dev_free(p);
    p = nullptr;
    bytes = 0;
    owned = true;
}

int Arena::take(DevBuf &b, size_t n)
{
    const size_t r = rounded(n);
    if (base) {
        if (off + r > cap) return fail(USPG_E_NOMEM, "work space too small");
        b.borrow(base + off, n);
    }
    off += r;
    return USPG_OK;
}

static int current_device(int *dev)
{
    USPG_HIP(hipGetDevice(dev));
    return USPG_OK;
}

int current_device_id(int *dev) { return current_device(dev); }

int check_device(int want)
{
    int dev = -1;
    int rc = current_device(&dev);
    if (rc != USPG_OK) return rc;
    if (dev != want) return fail(USPG_E_ARG, "handle belongs to another device than the current one");
    return USPG_OK;
}

// Sector counts of the grid rules (Sec. II.A, eq. 1).
static int sector_table(const uspg_grid_desc *d, std::vector<int32_t> &ng)
{
    ng.resize(d->n_rings);
    for (int i = 0; i < d->n_rings; ++i) {
        switch (d->sector_rule) {
        case USPG_SECTORS_PAPER:
            ng[i] = 4 * (2 * i + 1);
            break;
        case USPG_SECTORS_MULTIPLE: {
            int m = d->sector_multiple;
            if (m <= 0) return fail(USPG_E_ARG, "sector_multiple must be positive");
            double need = kTwoPi * (i + 0.5) / m;
            ng[i] = m * (int)std::ceil(need);
            break;
        }
        case USPG_SECTORS_EXPLICIT:
            if (!d->sectors) return fail(USPG_E_ARG, "explicit sector rule needs a table");
            ng[i] = d->sectors[i];
            break;
        default:
            return fail(USPG_E_ARG, "unknown sector rule");
        }
        if (ng[i] < 2) return fail(USPG_E_ARG, "every ring needs at least two sectors");
        // a line dipping two rings below ring i spans at least 2 acos((i-1)/i)
        // in azimuth; that must exceed one sector so that only the ring just
        // outside the innermost ring can be entered twice
        if (i >= 2 && std::acos((double)(i - 1) / i) * ng[i] <= M_PI * (1 + 1e-9))
            return fail(USPG_E_ARG, "too few sectors in ring " + std::to_string(i));
    }
    return USPG_OK;
}


// Arguments of a scan, before anything is counted.
static int validate_scan(const uspg_grid *g, const uspg_scan_desc *sc)
{
    const bool cone = sc->geometry == USPG_CONE_3D;
    if (sc->geometry < USPG_PARALLEL_2D || sc->geometry > USPG_CONE_3D) return fail(USPG_E_ARG, "unknown geometry");
    if (sc->n_views <= 0 || !(sc->span > 0) || sc->det_u <= 0 || sc->det_v <= 0 || !(sc->det_half_u > 0))
        return fail(USPG_E_ARG, "views, span, detector size and width must be positive");
    if (!cone && (g->nz != 1 || sc->det_v != 1)) return fail(USPG_E_ARG, "2D scans need a 2D grid and det_v == 1");
    if (cone && !(g->H > 0 && sc->det_half_v > 0)) return fail(USPG_E_ARG, "cone beam needs a cylinder and det_half_v > 0");
    if (sc->geometry != USPG_PARALLEL_2D && !(sc->src_axis > g->R && sc->src_det > 0))
        return fail(USPG_E_ARG, "the source must lie outside the cylinder");
    if (sc->weights != USPG_WEIGHTS_LENGTH && sc->weights != USPG_WEIGHTS_BINARY &&
        sc->weights != USPG_WEIGHTS_SEGMENTS)
        return fail(USPG_E_ARG, "weights");
    if (sc->coeff_dtype != USPG_F32 && sc->coeff_dtype != USPG_F64) return fail(USPG_E_ARG, "coeff_dtype");
    if (sc->row_codes != 0 && sc->row_codes != 1) return fail(USPG_E_ARG, "row_codes must be 0 or 1");
    if ((int64_t)sc->det_u * sc->det_v >= (int64_t)1 << 31) return fail(USPG_E_ARG, "too many rays");
    if (sc->weights == USPG_WEIGHTS_SEGMENTS) {
        if (g->nr >= (1 << 16) || g->nz >= (1 << 16)) return fail(USPG_E_ARG, "segment records need < 65536 rings and slices");
        if (sc->view_rows != 0 && sc->view_rows != 1) return fail(USPG_E_ARG, "view_rows must be 0 or 1");
    }
    return USPG_OK;
}

// Pieces of a stored-row handle's device memory, in work-space order (only
// sizes when the arena has no base).
static int carve_rows(uspg_coeffs *c, Arena &a)
{
    const uspg_grid *g = c->g;
    const size_t pair = c->scan.coeff_dtype == USPG_F64 ? sizeof(Coef<double>) : sizeof(Coef<float>);
    int rc;
    if ((rc = a.take(c->d_kq, sizeof(int32_t) * g->nr)) != USPG_OK ||
        (rc = a.take(c->d_hq, sizeof(int32_t) * (g->nr + 1))) != USPG_OK ||
        (rc = a.take(c->d_ring_of_off, sizeof(int32_t) * c->Cq)) != USPG_OK ||
        (rc = a.take(c->rowptr, sizeof(int64_t) * (c->nrays + 1))) != USPG_OK ||
        (rc = a.take(c->coef, pair * (size_t)std::max<int64_t>(c->nnz, 1))) != USPG_OK)
        return rc;
    if (c->want_codes &&
        ((rc = a.take(c->d_colptr, sizeof(int64_t) * (c->scan.det_u + 1))) != USPG_OK ||
         (rc = a.take(c->d_colt, sizeof(double) * (size_t)c->pend_nrec)) != USPG_OK ||
         (rc = a.take(c->d_colid, sizeof(uint32_t) * (size_t)c->pend_nrec)) != USPG_OK ||
         (rc = a.take(c->d_codes, sizeof(coded::RayCode) * (size_t)c->nrays)) != USPG_OK ||
         (rc = a.take(c->d_words, sizeof(uint64_t) * (size_t)std::max<int64_t>(c->pend_nwords, 1))) != USPG_OK))
        return rc;
    return USPG_OK;
}

// The layout tables of the walk (kq, hq, ring_of_off) on the device, in
// whatever buffers the handle holds for them (allocated here if empty).
static int upload_tables(uspg_coeffs *c)
{
    const uspg_grid *g = c->g;
    int rc;
    if ((!c->d_kq.p && (rc = c->d_kq.alloc(sizeof(int32_t) * g->nr)) != USPG_OK) ||
        (!c->d_hq.p && (rc = c->d_hq.alloc(sizeof(int32_t) * (g->nr + 1))) != USPG_OK) ||
        (!c->d_ring_of_off.p && (rc = c->d_ring_of_off.alloc(sizeof(int32_t) * c->Cq)) != USPG_OK))
        return rc;
    USPG_HIP(hipMemcpy(c->d_kq.p, c->kq.data(), sizeof(int32_t) * g->nr, hipMemcpyHostToDevice));
    USPG_HIP(hipMemcpy(c->d_hq.p, c->hq.data(), sizeof(int32_t) * (g->nr + 1), hipMemcpyHostToDevice));
    USPG_HIP(hipMemcpy(c->d_ring_of_off.p, c->ring_of_off.data(), sizeof(int32_t) * c->Cq, hipMemcpyHostToDevice));
    return USPG_OK;
}

// Size query of stored (LENGTH / BINARY) rows: the view group, the layout
// tables (host), the trace's count pass and, for coded rows, their sizes.
static int count_rows(uspg_coeffs *c, hipStream_t s)
{
    const uspg_grid *g = c->g;
    const uspg_scan_desc *sc = &c->scan;
    // view group: a view step must be a whole number of sectors in every ring
    double qf = sc->n_views * kTwoPi / sc->span;
    int q = (int)std::floor(qf + 0.5);
    if (q <= 0 || std::fabs(qf - q) > 1e-9) return fail(USPG_E_SHIFT, "n_views * 2 pi / span is not an integer");
    for (int i = 0; i < g->nr; ++i)
        if (g->ng[i] % q)
            return fail(USPG_E_SHIFT, "ring " + std::to_string(i) + " has " + std::to_string(g->ng[i]) +
                                          " sectors, not a multiple of " + std::to_string(q));
    c->q = q;
    c->grp = kRingGroup;
    c->kq.resize(g->nr);
    c->hq.resize(g->nr + 1);
    c->Cq = walk::wedge_tables(g->nr, g->ng.data(), q, c->grp, c->kq.data(), c->hq.data(), nullptr);
    c->hq[g->nr] = (int32_t)c->Cq;
    c->ring_of_off.assign(c->Cq, -1);
    walk::wedge_tables(g->nr, g->ng.data(), q, c->grp, c->kq.data(), c->hq.data(), c->ring_of_off.data());
    c->Wc = (int64_t)g->nz * c->Cq;
    c->Wtot = q * c->Wc;
    if (c->Wtot >= (int64_t)1 << 31) return fail(USPG_E_ARG, "device image layout exceeds 2^31 cells");
    // the walk of the count passes reads the layout tables on the device:
    // library copies until the fill moves them into the work space
    int rc;
    if ((rc = upload_tables(c)) != USPG_OK) return rc;
    if ((rc = trace_count_rows(c, s)) != USPG_OK) return rc;
    c->want_codes = sc->geometry == USPG_CONE_3D && sc->row_codes == 0;
    if (c->want_codes && (rc = code_count(c, s)) != USPG_OK) return rc;
    Arena sizing;
    if ((rc = carve_rows(c, sizing)) != USPG_OK) return rc;
    c->ws_needed = sizing.off;
    return USPG_OK;
}

// Fill of stored rows into the caller's work space: layout tables, the
// trace's fill pass, the colouring and the coded rows.
static int fill_rows(uspg_coeffs *c, Arena &a, hipStream_t s)
{
    int rc;
    if ((rc = carve_rows(c, a)) != USPG_OK || (rc = upload_tables(c)) != USPG_OK) return rc;
    if ((rc = trace_fill_rows(c, s)) != USPG_OK || (rc = colour_reference_view(c, s)) != USPG_OK) return rc;
    if (c->want_codes && (rc = code_fill(c, s)) != USPG_OK) return rc;
    c->pend_cnt.release();
    c->pend_colptr.release();
    c->pend_woff.release();
    return USPG_OK;
}

// The literal scheme's device arrays (library memory after the count phase,
// moved into the work space by the fill).
static DevBuf *segment_bufs(uspg_coeffs *c, int k)
{
    DevBuf *b[] = {&c->segptr, &c->seg_sr, &c->seg_pa, &c->seg_pb, &c->seg_partner,
                   &c->view_rowptr, &c->view_coef, &c->d_view_start};
    return k < (int)(sizeof(b) / sizeof(b[0])) ? b[k] : nullptr;
}

// Size query of the literal scheme: its records and (re-binned) view rows
// depend on the whole colouring pass, so the query builds them in library
// memory and the fill moves them.
static int count_segments(uspg_coeffs *c, hipStream_t s)
{
    c->segments = true;
    int rc;
    if ((rc = segments_reference_view(c, s)) != USPG_OK || (rc = colour_segments(c, s)) != USPG_OK) return rc;
    c->nnz = c->nseg;
    c->max_row = c->max_seg;
    size_t need = 0;
    for (int k = 0; DevBuf *b = segment_bufs(c, k); ++k)
        if (b->p) need += Arena::rounded(b->bytes);
    c->ws_needed = need;
    return USPG_OK;
}

static int fill_segments(uspg_coeffs *c, Arena &a, hipStream_t s)
{
    int rc;
    for (int k = 0; DevBuf *b = segment_bufs(c, k); ++k) {
        if (!b->p) continue;
        DevBuf nb;
        if ((rc = a.take(nb, b->bytes)) != USPG_OK) return rc;
        USPG_HIP(hipMemcpyAsync(nb.p, b->p, b->bytes, hipMemcpyDeviceToDevice, s));
        USPG_HIP(hipStreamSynchronize(s));
        b->borrow(nb.p, nb.bytes);   // frees the library copy
    }
    return USPG_OK;
}

int check_coeffs(const uspg_coeffs *c)
{
    if (!c) return fail(USPG_E_ARG, "null coefficients");
    if (c->pending) return fail(USPG_E_ARG, "coefficients are pending: fill them with a second uspg_build_coeffs call");
    return check_device(c->device);
}

}  // namespace uspg

using namespace uspg;

extern "C" {

const char *uspg_last_error(void) { return g_last_error.c_str(); }

int uspg_build_grid(const uspg_grid_desc *desc, uspg_grid **out)
{
    if (!desc || !out) return fail(USPG_E_ARG, "null argument");
    *out = nullptr;
    if (desc->n_rings <= 0 || desc->n_slices <= 0 || !(desc->radius > 0))
        return fail(USPG_E_ARG, "n_rings, n_slices and radius must be positive");
    if (desc->n_slices > 1 && !(desc->height > 0)) return fail(USPG_E_ARG, "height must be positive");
    auto *g = new uspg_grid();
    int rc = sector_table(desc, g->ng);
    if (rc != USPG_OK) { delete g; return rc; }
    g->nr = desc->n_rings;
    g->nz = desc->n_slices;
    g->R = desc->radius;
    g->H = desc->n_slices > 1 ? desc->height : (desc->height > 0 ? desc->height : 0.0);
    g->r = g->R / g->nr;
    g->h = g->nz > 1 || g->H > 0 ? g->H / g->nz : 0.0;
    g->z0 = -g->H / 2;
    g->rule = desc->sector_rule;
    g->head.assign(g->nr + 1, 0);
    for (int i = 0; i < g->nr; ++i) g->head[i + 1] = g->head[i] + g->ng[i];   // eq. 2
    g->c2d = g->head[g->nr];
    g->ncells = g->c2d * g->nz;
    if (g->ncells >= (int64_t)1 << 31) { delete g; return fail(USPG_E_ARG, "more than 2^31 cells"); }
    if ((rc = current_device(&g->device)) != USPG_OK) { delete g; return rc; }
    std::vector<double2> cs(g->c2d);
    for (int i = 0; i < g->nr; ++i)
        for (int b = 0; b < g->ng[i]; ++b) cs[g->head[i] + b] = walk::boundary_dir(b, g->ng[i]);
    if ((rc = g->d_ng.alloc(sizeof(int32_t) * g->nr)) != USPG_OK ||
        (rc = g->d_head.alloc(sizeof(int64_t) * (g->nr + 1))) != USPG_OK ||
        (rc = g->d_cs.alloc(sizeof(double2) * g->c2d)) != USPG_OK) {
        uspg_free_grid(g);
        return rc;
    }
    if (hipMemcpy(g->d_ng.p, g->ng.data(), sizeof(int32_t) * g->nr, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(g->d_head.p, g->head.data(), sizeof(int64_t) * (g->nr + 1), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(g->d_cs.p, cs.data(), sizeof(double2) * g->c2d, hipMemcpyHostToDevice) != hipSuccess) {
        uspg_free_grid(g);
        return fail(USPG_E_HIP, "uploading grid tables failed");
    }
    *out = g;
    return USPG_OK;
}

int uspg_grid_info(const uspg_grid *g, int64_t *n_cells, int64_t *cells_per_slice, int32_t *n_rings,
                   int32_t *n_slices)
{
    if (!g) return fail(USPG_E_ARG, "null grid");
    if (n_cells) *n_cells = g->ncells;
    if (cells_per_slice) *cells_per_slice = g->c2d;
    if (n_rings) *n_rings = g->nr;
    if (n_slices) *n_slices = g->nz;
    return USPG_OK;
}

int uspg_grid_tables(const uspg_grid *g, int32_t *sectors, int64_t *heads)
{
    if (!g) return fail(USPG_E_ARG, "null grid");
    if (sectors) std::memcpy(sectors, g->ng.data(), sizeof(int32_t) * g->nr);
    if (heads) std::memcpy(heads, g->head.data(), sizeof(int64_t) * (g->nr + 1));
    return USPG_OK;
}

void uspg_free_grid(uspg_grid *g)
{
    if (!g) return;
    g->d_ng.release();
    g->d_head.release();
    g->d_cs.release();
    delete g;
}

int uspg_build_coeffs(const uspg_grid *g, const uspg_scan_desc *sc, void *dev_ws, size_t ws_bytes,
                      size_t *ws_needed, void *stream, uspg_coeffs **out)
{
    if (!g || !sc || !out) return fail(USPG_E_ARG, "null argument");
    if (!dev_ws && !ws_needed) return fail(USPG_E_ARG, "a size query needs ws_needed");
    uspg_coeffs *c = *out;
    if (c && (!c->pending || c->g != g || std::memcmp(&c->scan, sc, sizeof(*sc)) != 0))
        return fail(USPG_E_ARG, "*out is not a pending handle of this grid and scan");
    const bool fresh = c == nullptr;
    int rc = check_device(g->device);
    if (rc != USPG_OK) return rc;
    hipStream_t s = (hipStream_t)stream;
    if (fresh) {
        if ((rc = validate_scan(g, sc)) != USPG_OK) return rc;
        c = new uspg_coeffs();
        c->g = g;
        c->scan = *sc;
        c->device = g->device;
        c->nrays = (int64_t)sc->det_u * sc->det_v;
        rc = sc->weights == USPG_WEIGHTS_SEGMENTS ? count_segments(c, s) : count_rows(c, s);
        if (rc != USPG_OK) {
            uspg_free_coeffs(c);
            return rc;
        }
        c->pending = true;
    }
    if (ws_needed) *ws_needed = c->ws_needed;
    if (!dev_ws) {
        *out = c;
        return USPG_OK;
    }
    if (ws_bytes < c->ws_needed) {
        if (fresh) uspg_free_coeffs(c);
        return fail(USPG_E_NOMEM, "work space of " + std::to_string(ws_bytes) + " bytes, " +
                                      std::to_string(c->ws_needed) + " needed");
    }
    Arena a{static_cast<char *>(dev_ws), ws_bytes, 0};
    rc = c->segments ? fill_segments(c, a, s) : fill_rows(c, a, s);
    if (rc != USPG_OK) {
        uspg_free_coeffs(c);
        *out = nullptr;
        return rc;
    }
    c->pending = false;
    c->device_bytes = (int64_t)c->ws_needed;
    *out = c;
    return USPG_OK;
}

int uspg_debug_alloc(int32_t fail_after, int64_t *live)
{
    if (fail_after >= 0) g_fail_after = fail_after;
    if (live) *live = g_live_allocs.load();
    return USPG_OK;
}

int uspg_coeffs_info(const uspg_coeffs *c, int64_t *nnz_ref, int64_t *n_rays, int32_t *colour_u,
                     int32_t *colour_v, int32_t *max_row, int64_t *device_bytes)
{
    if (!c) return fail(USPG_E_ARG, "null coefficients");
    if (nnz_ref) *nnz_ref = c->nnz;
    if (n_rays) *n_rays = c->nrays;
    if (colour_u) *colour_u = c->Ku;
    if (colour_v) *colour_v = c->Kv;
    if (max_row) *max_row = c->max_row;
    if (device_bytes) *device_bytes = c->device_bytes;
    return USPG_OK;
}

int uspg_coeffs_row(const uspg_coeffs *c, int32_t view, int64_t ray, int64_t *cells, double *lengths,
                    int32_t cap, int32_t *n)
{
    if (!c || !n) return fail(USPG_E_ARG, "null argument");
    if (view < 0 || view >= c->scan.n_views || ray < 0 || ray >= c->nrays) return fail(USPG_E_ARG, "view or ray out of range");
    int rc = check_coeffs(c);
    if (rc != USPG_OK) return rc;
    if (c->segments) {
        std::vector<int64_t> row;
        if ((rc = segments_row(c, view, ray, row)) != USPG_OK) return rc;
        *n = (int32_t)row.size();
        if (*n > cap) return fail(USPG_E_NOMEM, "row longer than cap");
        if (*n == 0) return USPG_OK;
        if (!cells || !lengths) return fail(USPG_E_ARG, "null output");
        for (int32_t j = 0; j < *n; ++j) {
            cells[j] = row[j];
            lengths[j] = 1.0;
        }
        return USPG_OK;
    }
    int64_t rp[2];
    USPG_HIP(hipMemcpy(rp, c->rowptr.as<int64_t>() + ray, sizeof(rp), hipMemcpyDeviceToHost));
    int32_t len = (int32_t)(rp[1] - rp[0]);
    *n = len;
    if (len > cap) return fail(USPG_E_NOMEM, "row longer than cap");
    if (len == 0) return USPG_OK;
    if (!cells || !lengths) return fail(USPG_E_ARG, "null output");
    std::vector<uint32_t> ids(len);
    if (c->scan.coeff_dtype == USPG_F64) {
        std::vector<Coef<double>> pr(len);
        USPG_HIP(hipMemcpy(pr.data(), c->coef.as<Coef<double>>() + rp[0], sizeof(Coef<double>) * len,
                           hipMemcpyDeviceToHost));
        for (int j = 0; j < len; ++j) { ids[j] = pr[j].id; lengths[j] = pr[j].a; }
    } else {
        std::vector<Coef<float>> pr(len);
        USPG_HIP(hipMemcpy(pr.data(), c->coef.as<Coef<float>>() + rp[0], sizeof(Coef<float>) * len,
                           hipMemcpyDeviceToHost));
        for (int j = 0; j < len; ++j) { ids[j] = pr[j].id; lengths[j] = pr[j].a; }
    }
    const uspg_grid *g = c->g;
    for (int j = 0; j < len; ++j) {
        int64_t x = ((int64_t)ids[j] + (int64_t)view * c->Wc) % c->Wtot;
        int64_t aw = x / c->Wc, rem = x % c->Wc, k = rem / c->Cq, o = rem % c->Cq;
        int i = c->ring_of_off[o];
        if (i < 0) return fail(USPG_E_INTERNAL, "row entry in layout padding");
        int64_t s = aw * c->kq[i] + (o - c->hq[i]) / c->grp;
        cells[j] = k * g->c2d + g->head[i] + s;
    }
    return USPG_OK;
}

int uspg_coeffs_code_info(const uspg_coeffs *c, int32_t *coded, int64_t *coded_rays, int64_t *explicit_rays,
                          int64_t *code_bytes)
{
    if (!c) return fail(USPG_E_ARG, "null coefficients");
    if (coded) *coded = c->coded ? 1 : 0;
    if (coded_rays) *coded_rays = c->coded_rays;
    if (explicit_rays) *explicit_rays = c->explicit_rays;
    if (code_bytes) {
        int64_t b = 0;
        for (const DevBuf *d : {&c->d_colptr, &c->d_colt, &c->d_colid, &c->d_codes, &c->d_words})
            if (d->p) b += (int64_t)Arena::rounded(d->bytes);
        *code_bytes = b;
    }
    return USPG_OK;
}

int uspg_coeffs_view_nnz(const uspg_coeffs *c, int64_t *nnz_per_view)
{
    if (!c || !nnz_per_view) return fail(USPG_E_ARG, "null argument");
    if (c->pending) return fail(USPG_E_ARG, "pending coefficients");
    for (int v = 0; v < c->scan.n_views; ++v)
        nnz_per_view[v] = c->segments ? c->view_nnz[v] : c->nnz;
    return USPG_OK;
}

int uspg_coeffs_conflicts(const uspg_coeffs *c, uint8_t *mark)
{
    if (!c || !mark) return fail(USPG_E_ARG, "null argument");
    if (c->pending) return fail(USPG_E_ARG, "pending coefficients");
    std::memcpy(mark, c->mark.data(), c->mark.size());
    return USPG_OK;
}

void uspg_free_coeffs(uspg_coeffs *c)
{
    if (!c) return;
    c->rowptr.release();
    c->coef.release();
    c->d_kq.release();
    c->d_hq.release();
    c->d_ring_of_off.release();
    c->segptr.release();
    c->seg_sr.release();
    c->seg_pa.release();
    c->seg_pb.release();
    c->seg_partner.release();
    c->view_rowptr.release();
    c->view_coef.release();
    c->d_view_start.release();
    c->d_colptr.release();
    c->d_colt.release();
    c->d_colid.release();
    c->d_codes.release();
    c->d_words.release();
    delete c;
}

size_t uspg_mart_workspace_bytes(const uspg_coeffs *c, int32_t dtype, double tol)
{
    if (!c) return 0;
    size_t sz = dtype == USPG_F64 ? sizeof(double) : sizeof(float);
    size_t n = (size_t)(c->segments ? c->g->ncells : c->Wtot) * sz;
    return tol > 0 ? 2 * n + 16 : n;
}

int mart_run(const uspg_coeffs *c, int32_t dtype, const void *proj, void *image, void *work,
             size_t work_bytes, int32_t n_sweeps, double beta, double tol, int32_t *sweeps_done,
             void *stream)
{
    if (!c || !proj || !image || !work) return fail(USPG_E_ARG, "null argument");
    if (dtype != USPG_F32 && dtype != USPG_F64) return fail(USPG_E_ARG, "dtype");
    if (n_sweeps < 0 || !(beta > 0) || !(tol >= 0)) return fail(USPG_E_ARG, "n_sweeps >= 0, beta > 0, tol >= 0");
    if (work_bytes < uspg_mart_workspace_bytes(c, dtype, tol)) return fail(USPG_E_NOMEM, "work space too small");
    int rc = check_coeffs(c);
    if (rc != USPG_OK) return rc;
    if (tol > 0 && stream_capturing((hipStream_t)stream))
        return fail(USPG_E_ARG, "tol > 0 synchronises the stream once per sweep and cannot be graph-captured");
    return mart_launch(c, dtype, proj, image, work, n_sweeps, beta, tol, sweeps_done, (hipStream_t)stream);
}

int uspg_mart_timing(int32_t enable, void *stream, double *batch_ms, int64_t *batch_launches)
{
    return mart_timing(enable, (hipStream_t)stream, batch_ms, batch_launches);
}

int uspg_to_cartesian(const uspg_grid *g, int32_t dtype, const void *image, void *cart, int32_t nc,
                      int32_t mode, void *stream)
{
    if (!g || !image || !cart) return fail(USPG_E_ARG, "null argument");
    if (dtype != USPG_F32 && dtype != USPG_F64) return fail(USPG_E_ARG, "dtype");
    if (nc <= 0 || (int64_t)nc * nc >= (int64_t)1 << 31) return fail(USPG_E_ARG, "nc out of range");
    if (mode == USPG_REMAP_BIJECTION) {
        if (nc != 2 * g->nr) return fail(USPG_E_ARG, "bijection needs nc == 2 n_rings");
        for (int i = 0; i < g->nr; ++i)
            if (g->ng[i] != 4 * (2 * i + 1)) return fail(USPG_E_ARG, "bijection needs the paper's sector rule");
    } else if (mode != USPG_REMAP_POINT) {
        return fail(USPG_E_ARG, "unknown remap mode");
    }
    int rc = check_device(g->device);
    if (rc != USPG_OK) return rc;
    return remap_launch(g, dtype, image, cart, nc, mode, (hipStream_t)stream);
}

}  // extern "C"
