/*
 * uspg.h -- C ABI of the MI355X (gfx950) library for MART reconstruction on a
 * Uniformly Sampled Polar / Cylindrical Grid (USPG in 2D, USCG in 3D).
 *
 * Method: Chaudhary, Wahi, Munshi, "Uniformly Sampled Polar and Cylindrical
 * Grid Approach for 2D, 3D Image Reconstruction using Algebraic Algorithm".
 * Coefficients are traced for the first (reference) view only and reused for
 * every other view by rotating the angular cell index (Sec. III.B-C); the
 * image is solved with Sp-MART (Sec. III.D) and mapped to a Cartesian grid for
 * display (Sec. II.B).
 *
 * Conventions shared by every call:
 *  - Every entry point returns USPG_OK (0) or a negative status; no call
 *    aborts or throws.  uspg_last_error() gives a message for the calling
 *    thread's last failure.
 *  - Handles (uspg_grid, uspg_coeffs) are opaque host objects owned by the
 *    library and released with the matching uspg_free_* call.  A handle is
 *    bound to the HIP device that was current when it was built and must be
 *    used with that device current.  Handles are immutable after the build
 *    and may be shared by calls on different streams.
 *  - "stream" is a hipStream_t passed as void* (NULL = the null stream).
 *    Device work is enqueued on it asynchronously unless a call says
 *    otherwise.
 *  - Device buffers passed in (projections, images, work space, Cartesian
 *    output) are owned by the caller and must be device-accessible memory on
 *    the handle's device.  The library owns the device memory inside handles.
 *  - Images are in the paper's numbering: cell (slice k, ring i, sector s) has
 *    index k * C2D + H_i + s, with H_i the ring head (eq. 2), rings 0-based
 *    from the centre and sectors anticlockwise from the +x axis.
 */
#ifndef USPG_H
#define USPG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------ */
#define USPG_OK 0
#define USPG_E_ARG (-1)      /* invalid argument (null, size, range, dtype)       */
#define USPG_E_SHIFT (-2)    /* views are not a whole number of sectors per ring  */
#define USPG_E_NOMEM (-3)    /* device allocation failed or work space too small  */
#define USPG_E_HIP (-4)      /* HIP runtime error (reported at this or a later call) */
#define USPG_E_INTERNAL (-5) /* internal consistency check failed                 */

/* ---- enumerations ------------------------------------------------------- */
enum {
    USPG_SECTORS_PAPER = 0,    /* ring n (1-based) has 4(2n-1) sectors (eq. 1)          */
    USPG_SECTORS_MULTIPLE = 1, /* ring i (0-based) has m * ceil(2 pi (i + 1/2) / m)      */
    USPG_SECTORS_EXPLICIT = 2  /* caller's table                                         */
};
enum {
    USPG_PARALLEL_2D = 0, /* view-0 ray b is the line y = -W + (b + 1/2) 2W / B             */
    USPG_FAN_2D = 1,      /* point source (-D_so, 0), flat detector at x = D_sd - D_so      */
    USPG_CONE_3D = 2      /* point source (-D_so, 0, 0), flat U x V detector at x = D_sd - D_so */
};
enum {
    USPG_WEIGHTS_LENGTH = 0,  /* intersection lengths, view-0 rows shifted per view         */
    USPG_WEIGHTS_BINARY = 1,  /* 1 per traversed cell, view-0 rows shifted per view         */
    USPG_WEIGHTS_SEGMENTS = 2 /* the paper's literal scheme: binary, re-binned per view     */
};
enum { USPG_F32 = 0, USPG_F64 = 1 };
enum { USPG_REMAP_POINT = 0, USPG_REMAP_BIJECTION = 1 };

typedef struct uspg_grid uspg_grid;
typedef struct uspg_coeffs uspg_coeffs;

/* ---- grid (Sec. II.A, eqs. 1-2; Sec. III.A USCG) --------------------------
 * A disk (n_slices == 1) or a cylinder of radius `radius` and height `height`
 * centred on the origin, cut into n_rings rings of equal spacing
 * r = radius / n_rings, each ring into sectors (rule below) and, in 3D, into
 * n_slices slices of thickness height / n_slices.  `sectors` is read only for
 * USPG_SECTORS_EXPLICIT (n_rings host entries, each >= 2).  The rule must give
 * every ring enough sectors that a line cannot dip two rings deep inside one
 * sector (true for the paper and multiple rules); otherwise USPG_E_ARG. */
typedef struct {
    int32_t n_rings;
    int32_t n_slices;       /* 1 for a 2D disk */
    double radius;
    double height;          /* ignored when n_slices == 1 */
    int32_t sector_rule;
    int32_t sector_multiple;
    const int32_t *sectors;
} uspg_grid_desc;

/* Builds the grid tables on the host and uploads them to the current device
 * (synchronous).  *out receives the handle. */
int uspg_build_grid(const uspg_grid_desc *desc, uspg_grid **out);

/* Sizes of a grid.  Any output pointer may be NULL. */
int uspg_grid_info(const uspg_grid *g, int64_t *n_cells, int64_t *cells_per_slice,
                   int32_t *n_rings, int32_t *n_slices);

/* Host copies of the per-ring sector counts (n_rings entries) and heads
 * (n_rings + 1 entries, heads[n_rings] = cells per slice).  NULL skips. */
int uspg_grid_tables(const uspg_grid *g, int32_t *sectors, int64_t *heads);

void uspg_free_grid(uspg_grid *g);

/* ---- scan and coefficients (Sec. III.A-C, Alg. 1) ------------------------
 * View v is the view-0 arrangement rotated anticlockwise about z by
 * v * span / n_views.  q = n_views * 2 pi / span must be an integer that
 * divides every ring's sector count, so that a view step is a whole number of
 * sectors in every ring; otherwise USPG_E_SHIFT.
 * Detector: det_u columns x det_v rows (det_v = 1 in 2D), ray index
 * r = w * det_u + u, pixel centres at -W + (j + 1/2) 2W / count with
 * W = det_half_u (columns) or det_half_v (rows).  Parallel 2D uses only
 * det_u and det_half_u.  src_axis = D_so, src_det = D_sd.
 * weights: LENGTH stores the intersection length of ray and cell, BINARY
 * stores 1 for every traversed cell (Sec. III.B).  SEGMENTS is the paper's
 * literal scheme (Sec. III.B-C, Alg. 1): each view-0 ray is cut only at the
 * cylindrical and axial planes, and each piece is stored as (slice, ring,
 * azimuth at both ends); for view v both azimuths advance by v span /
 * n_views and every sector between them (eqs. 10-16) gets coefficient 1
 * (a cell met by both passes of a line through one ring counts once).  With
 * SEGMENTS any n_views and span are accepted (no USPG_E_SHIFT), the
 * colouring is the union of every view's conflicts, coeff_dtype is ignored
 * (records are FP64; kept view rows are float pairs, so batches and engines
 * take them with the USPG_F32 coefficient type), and batches and engines
 * accept the handle only with its view rows kept (E_ARG otherwise).
 * quarter (SEGMENTS only, else ignored): 1 traces only the rays with
 * u < ceil(det_u / 2) and w < ceil(det_v / 2) and mirrors their records to
 * the other rays (y -> -y maps azimuth phi to 2 pi - phi, z -> -z maps slice
 * k to n_slices - 1 - k; Sec. III.C); 0 traces every ray.  The two agree
 * except for segment ends exactly on a radial plane, where a mirrored
 * azimuth can round to the other side.
 * view_rows (SEGMENTS only, else ignored): the colouring re-bins the rows of
 * every view once; with 0 they are kept on the device as (cell, 1) pairs,
 * 8 bytes per entry plus 8 per ray and view, when that totals at most
 * USPG_VIEW_ROWS_MAX_BYTES, and MART then reads them as stored rows; with 1,
 * or when they do not fit, MART re-bins each view's rows from the records
 * on the fly (the per-view part of Alg. 1).  Both give the same cells; the ray sums
 * may differ in FP32 rounding.
 * coeff_dtype: storage of the coefficients (USPG_F32 or USPG_F64).
 * colour_u, colour_v: 0 = choose the smallest valid lattice; otherwise the
 * lattice is checked and USPG_E_ARG is returned if two rays of one class
 * share a cell. */
typedef struct {
    int32_t geometry;
    int32_t n_views;
    double span;
    int32_t det_u, det_v;
    double det_half_u, det_half_v;
    double src_axis, src_det;
    int32_t weights;
    int32_t coeff_dtype;
    int32_t colour_u, colour_v;
    int32_t quarter;        /* SEGMENTS only: 1 traces one detector quadrant and mirrors it */
    int32_t view_rows;      /* SEGMENTS only: 0 keeps every view's rows when they fit, 1 re-bins per view */
    int32_t row_codes;      /* CONE_3D LENGTH / BINARY: 0 codes the rows (see below), 1 stored rows only */
} uspg_scan_desc;

/* row_codes (CONE_3D with LENGTH or BINARY weights, else ignored): the rays
 * of one detector column share their in-plane path, so with 0 the library
 * also keeps, per column, that path's sector pieces (ray parameter of each
 * piece's start, FP64, and its slice-0 cell; 12 bytes per piece) and, per
 * ray, a 48-byte header plus two bits per entry (next piece, next slice).
 * mart_run then rebuilds every entry from these instead of reading the
 * stored (cell, coefficient) pairs; each rebuilt entry is checked against
 * the stored one when the codes are built, and rays that do not match bit
 * for bit (none on the configured cone-beam scans) keep their stored rows.
 * The solve gives the same bits either way.  1 builds the stored rows only. */

/* Largest size of the kept per-view rows of SEGMENTS coefficients. */
#define USPG_VIEW_ROWS_MAX_BYTES (8LL << 30)

/* Traces every view-0 ray through the grid on the device (FP64 geometry),
 * stores the reference rows (one entry per traversed cell, duplicates merged)
 * and colours the rays into cell-disjoint lattice classes, in two calls:
 *  1. Size query: dev_ws == NULL.  Validates the arguments, runs the count
 *     pass and sets *ws_needed to the bytes of device memory the handle will
 *     hold; *out receives a pending handle (it keeps the counts; every call
 *     except a fill call, uspg_coeffs_info and uspg_free_coeffs refuses it
 *     with USPG_E_ARG).  *out is read on entry: it must be NULL or a
 *     pending handle (then it is returned as is).
 *  2. Fill: dev_ws != NULL, ws_bytes >= the size, *out = the pending handle
 *     of this grid and an equal scan description (or NULL: the counts then
 *     run in this call).  Every device array of the handle is carved out of
 *     dev_ws (256-byte aligned pieces); *out receives the built handle.
 *     ws_needed (nullable) receives the size.  A short work space returns
 *     USPG_E_NOMEM with nothing written to it (a pending handle passed in
 *     stays pending); any other failure frees the handle and sets *out to
 *     NULL.
 * dev_ws is device memory owned by the caller (e.g. a torch tensor, so that
 * the coefficients count in the caller's memory accounting); the handle must
 * not outlive it and uspg_free_coeffs does not free it.  The library's own
 * temporary device memory during the calls is freed before they return.
 * With SEGMENTS the records and kept view rows depend on the whole colouring,
 * so the size query builds them in library memory and the fill moves them
 * into dev_ws.  The grid must outlive the coefficients.  Synchronises
 * `stream` (several times). */
int uspg_build_coeffs(const uspg_grid *g, const uspg_scan_desc *scan, void *dev_ws, size_t ws_bytes,
                      size_t *ws_needed, void *stream, uspg_coeffs **out);

/* Sizes of the reference rows and the chosen lattice (classes are
 * c = (w mod colour_v) * colour_u + (u mod colour_u)).  With SEGMENTS,
 * nnz_ref and max_row count segment records.  device_bytes is the work
 * space the handle occupies.  On a pending handle the lattice is not
 * chosen yet (0).  NULL skips. */
int uspg_coeffs_info(const uspg_coeffs *c, int64_t *nnz_ref, int64_t *n_rays,
                     int32_t *colour_u, int32_t *colour_v, int32_t *max_row,
                     int64_t *device_bytes);

/* Coded rows of a coefficient set (row_codes above): *coded = 1 when
 * mart_run reads them, the rays coded and left explicit (rays that miss the
 * cylinder count in neither) and the device bytes of the codes.  NULL
 * skips. */
int uspg_coeffs_code_info(const uspg_coeffs *c, int32_t *coded, int64_t *coded_rays, int64_t *explicit_rays,
                          int64_t *code_bytes);

/* Host copy of the row of ray `ray` in view `view` (cells in the paper's
 * numbering, rotated to that view; lengths as stored; with SEGMENTS the
 * re-binned row, cells ascending, lengths 1).  Synchronous; for inspection
 * and tests.  *n receives the row length; USPG_E_NOMEM if it exceeds cap
 * (nothing written). */
int uspg_coeffs_row(const uspg_coeffs *c, int32_t view, int64_t ray, int64_t *cells,
                    double *lengths, int32_t cap, int32_t *n);

/* Entries of every view's rows (host, n_views entries): nnz_ref for every
 * view with LENGTH / BINARY; with SEGMENTS the re-binned cells of that view
 * (the MART work per view).  Synchronous. */
int uspg_coeffs_view_nnz(const uspg_coeffs *c, int64_t *nnz_per_view);

/* Host copy of the conflict-offset map used by the colouring:
 * mark[dw * det_u + du] = 1 when two view-0 rays whose detector indices
 * differ by (du, dw) share a cell (with SEGMENTS: in any view).  mark has
 * det_u * det_v bytes. */
int uspg_coeffs_conflicts(const uspg_coeffs *c, uint8_t *mark);

void uspg_free_coeffs(uspg_coeffs *c);

/* ---- MART (Sec. III.D, eqs. 17-19) ---------------------------------------
 * For each sweep, for each view v ascending, for each lattice class c
 * ascending, every ray r of the class is applied (the rays of a class share no
 * cell, so applying them together equals applying them one by one):
 *   Pbar = sum_j a_rj f_j                     (eq. 17, rotated row of view v)
 *   f_j <- f_j (1 - beta (a_rj / a_max,r) (1 - P[v][r] / Pbar))   (eq. 18)
 * Rays with an empty row or Pbar <= 0 are skipped.  With binary weights this
 * is eq. 18 exactly.  beta > 0; positivity of f is kept for beta <= 1.
 * dtype: USPG_F32 or USPG_F64 for proj, image and the arithmetic.
 * proj:  device [n_views][det_v][det_u], non-negative.
 * image: device [n_cells] in the paper's numbering; read as f0 (> 0) and
 *        overwritten with the result.
 * work:  device scratch of at least uspg_mart_workspace_bytes() bytes.
 *        proj, image, work and the coefficient set's work space must not
 *        overlap (the kernels read proj and the codes as read-only data
 *        that no store of theirs can alias).
 * tol:   0 runs exactly n_sweeps sweeps with no host synchronisation; tol > 0
 *        stops after the first sweep with max_j |f_new - f_old| / f_old <= tol
 *        (eq. 19) and synchronises the stream once per sweep.
 * sweeps_done: host, nullable; receives the number of sweeps run (written
 *        before return, so only meaningful after the stream is synchronised
 *        when tol == 0 -- it is then simply n_sweeps).
 * Graph capture: with tol == 0 the call enqueues kernels and device-to-device
 * copies only (no allocation, memset or host wait), so it may be recorded
 * into a HIP graph by capturing `stream`; each replay reads proj and image
 * as they are when it runs.  tol > 0 on a capturing stream returns
 * USPG_E_ARG before anything is enqueued. */
size_t uspg_mart_workspace_bytes(const uspg_coeffs *c, int32_t dtype, double tol);

int mart_run(const uspg_coeffs *c, int32_t dtype, const void *proj, void *image, void *work,
             size_t work_bytes, int32_t n_sweeps, double beta, double tol,
             int32_t *sweeps_done, void *stream);

/* Allocation-free variant of mart_run, for callers that cannot allocate
 * device memory (code under HIP graph capture, serving loops or harnesses
 * that forbid hipMalloc).  Same arguments, semantics and errors as mart_run
 * without work / work_bytes: the work space is a fixed array of
 * USPG_NOALLOC_SCRATCH_BYTES inside the library, one copy per device, held
 * from the library's load until the process ends.  USPG_E_NOMEM (nothing
 * enqueued) when uspg_mart_workspace_bytes(c, dtype, tol) exceeds it.  The
 * call allocates nothing and records no timing (uspg_mart_timing does not see
 * it).  Every call on one device shares that device's array: calls that
 * overlap on one device (on two streams or from two threads) race and must
 * be serialised by the caller.  Each call rewrites the work space before
 * reading it, so nothing carries over from an earlier call. */
#define USPG_NOALLOC_SCRATCH_BYTES (64LL << 20)

int mart_run_noalloc(const uspg_coeffs *c, int32_t dtype, const void *proj, void *image,
                     int32_t n_sweeps, double beta, double tol, int32_t *sweeps_done, void *stream);

/* Timing of mart_run's batch kernels on one stream (profiling aid), kept
 * per stream so that calls on other streams neither add to it nor disturb
 * it.  enable = 1 resets `stream`'s accumulators and turns its timing on:
 * every later mart_run on that stream records one HIP event pair around its
 * sequence of (view, class) batch kernels (nothing between them),
 * synchronises the stream at its end and adds the elapsed time and the
 * number of batch launches (calls under graph capture and
 * mart_run_noalloc calls are not timed).  enable = 0 turns the stream's
 * timing off and forgets it.  batch_ms and batch_launches (host, nullable)
 * receive the stream's totals so far.  Thread-safe. */
int uspg_mart_timing(int32_t enable, void *stream, double *batch_ms, int64_t *batch_launches);

/* ---- USPG -> Cartesian grid (Sec. II.B) -----------------------------------
 * cart: device [n_slices][nc][nc]; pixel (ix, iy) covers the square of side
 * 2R/nc centred at ((2 ix + 1 - nc) R / nc, (2 iy + 1 - nc) R / nc).
 * POINT: the pixel takes the value of the cell containing its centre (0
 *   outside the disk); centres on a diagonal use the exact angle.
 * BIJECTION: paper grid only (sector rule PAPER) with nc = 2 n_rings: square
 *   ring n (pixels with max(|2ix+1-nc|, |2iy+1-nc|) = 2n - 1) and circular
 *   ring n hold the same number of cells and are matched one to one, both
 *   numbered anticlockwise from the +x axis.
 * One kernel on `stream`: the call may be captured into a HIP graph. */
int uspg_to_cartesian(const uspg_grid *g, int32_t dtype, const void *image, void *cart,
                      int32_t nc, int32_t mode, void *stream);

/* ---- many problems run together ------------------------------------------
 * A batch plans MART for n independent problems (each with its own grid,
 * coefficients, projections and image) that run concurrently, each in its
 * own MART order (sweeps > views > colour classes).  Two modes:
 *  - lockstep (1, default): launch t performs step t, one (view, class)
 *    batch, of every unfinished problem, each problem with as many
 *    workgroups as its largest class needs; the whole sequence of launches
 *    is captured once as a HIP graph (re-captured when the step count or
 *    the launch shape changes) and replayed with one graph launch per run;
 *  - persistent (0): one launch, one workgroup per problem for the whole
 *    solve, with workgroup barriers between classes; a problem whose
 *    device-layout image fits the workgroup's LDS keeps it there.
 * Either way the result of every problem is bit for bit the one mart_run
 * gives for it alone (same per-ray arithmetic and order).
 * All coefficient sets must share one coefficient type and the current
 * device.  The batch keeps pointers to the coefficient handles: they must
 * outlive it.  Allocates a small device descriptor table. */
typedef struct uspg_batch uspg_batch;

int uspg_build_batch(int32_t n, const uspg_coeffs *const *coeffs, int32_t dtype, uspg_batch **out);

/* Launch settings: mode (0 persistent, 1 lockstep), threads per workgroup
 * (multiple of 64; 64..1024 persistent, 64..256 lockstep) and whether
 * LDS-resident images are allowed (persistent mode).  Synchronous
 * (re-uploads the descriptor tables). */
int uspg_batch_set(uspg_batch *b, int32_t mode, int32_t block_threads, int32_t use_lds);

/* Current settings; n_lds = problems whose image lives in LDS (persistent
 * mode); lds_bytes = dynamic LDS per workgroup.  NULL skips. */
int uspg_batch_info(const uspg_batch *b, int32_t *mode, int32_t *block_threads, int32_t *use_lds,
                    int32_t *n_lds, int64_t *lds_bytes);

/* Runs every problem: host arrays of n device pointers (proj[i] as for
 * mart_run, image[i] in the paper's numbering, read as f0 and overwritten,
 * work[i] device scratch of work_bytes[i] >= uspg_mart_workspace_bytes(coeffs
 * [i], dtype, 0)), per-problem sweep counts and relaxation.  Fixed sweep
 * counts only (no stopping rule).  Asynchronous on `stream` (a first run,
 * or one with a new step count or grouping, captures the lockstep graph
 * first).  In lockstep mode, problems whose image lines touched per step
 * would together outgrow the last-level cache run in successive groups (in
 * their order, each group from the step where the previous one ends); the
 * results do not depend on the grouping.  The caller must not run the same
 * batch on two streams at once. */
int mart_run_batch(uspg_batch *b, const void *const *proj, void *const *image, void *const *work,
                   const size_t *work_bytes, const int32_t *n_sweeps, const double *beta, void *stream);

/* Autotuner: times probe_sweeps sweeps of the batch for each candidate
 * setting (lockstep with 128 or 256 threads per workgroup; persistent with
 * 256, 512 or 1024 threads, with and without LDS-resident images) on
 * scratch copies of the images made in work[i] (image[i] is only read),
 * keeps the fastest and returns its time in *best_ms (nullable).
 * Synchronous. */
int uspg_batch_autotune(uspg_batch *b, const void *const *proj, const void *const *image,
                        void *const *work, const size_t *work_bytes, int32_t probe_sweeps,
                        const double *beta, void *stream, double *best_ms);

void uspg_free_batch(uspg_batch *b);

/* ---- continuous batching --------------------------------------------------
 * An engine runs MART for problems that arrive and leave at any time, the
 * serving form of the lockstep batch above.  A problem is admitted into a
 * free slot between step calls and starts at the engine's current step;
 * every uspg_engine_step call advances every admitted problem by n_steps
 * steps (one step = one (view, colour class) batch of Sec. III.D, in the
 * problem's own sweep > view > class order), with one launch per step
 * covering all of them, except that a problem whose largest class fills
 * mart_run's capped grid on its own (16 workgroups of 256 threads per
 * compute unit) gets its own mart_run launch per step.  A problem finishes
 * after n_sweeps full sweeps;
 * the result of each problem is bit for bit the one mart_run gives for it
 * alone, whatever else shares the engine.
 * max_slots bounds the problems admitted at once; dtype is the image type
 * (USPG_F32 / USPG_F64), coeff_dtype the coefficient type every admitted
 * coefficient set must have.  Calls on one engine use one stream and one
 * thread; the engine lives on the device current at creation.  Allocates
 * small device descriptor tables and a pinned staging buffer. */
typedef struct uspg_engine uspg_engine;

int uspg_engine_create(int32_t max_slots, int32_t dtype, int32_t coeff_dtype, uspg_engine **out);

/* Admits one problem: proj (device, n_views x rays as for mart_run), image
 * (device, the paper's numbering, read as f0 and overwritten with the
 * result when the problem finishes), work (device scratch of work_bytes >=
 * uspg_mart_workspace_bytes(c, dtype, 0), holding the problem's image
 * while it runs).  c, proj, image and work must stay valid until the step
 * call that reports the slot finished has completed on the stream.
 * Enqueues the layout permutation on `stream`; *slot receives the slot id
 * (nullable).  E_NOMEM when every slot is taken or work is too small;
 * E_ARG for null pointers, n_sweeps <= 0, beta <= 0 or a coefficient type
 * other than the engine's. */
int uspg_engine_admit(uspg_engine *e, const uspg_coeffs *c, const void *proj, void *image, void *work,
                      size_t work_bytes, int32_t n_sweeps, double beta, void *stream, int32_t *slot);

/* Enqueues n_steps steps of every admitted problem on `stream`, then for
 * every problem that has completed its sweeps enqueues the copy of its
 * result into its image and frees its slot.  finished (host, nullable,
 * room for cap ids) receives the freed slot ids, *n_finished their count
 * (which may exceed cap).  The results are ready once the stream reaches
 * this point.  Waits on the host only for the previous call's descriptor
 * upload. */
int uspg_engine_step(uspg_engine *e, int32_t n_steps, void *stream, int32_t *finished, int32_t cap,
                     int32_t *n_finished);

/* Problems currently admitted and steps run so far (nullable outputs). */
int uspg_engine_info(const uspg_engine *e, int32_t *active, int64_t *global_step);

/* Waits for the engine's own uploads and frees it.  Problems still
 * admitted are dropped: their images keep f0, their work buffers hold a
 * partial solve.  The caller synchronizes `stream` before freeing buffers. */
void uspg_engine_destroy(uspg_engine *e);

/* ---- z-slab decomposition --------------------------------------------------
 * One solve split into slabs of whole slices, as several devices would
 * share a cone-beam volume, all run on this device.  Slab g owns the cells
 * of slices [begin_g, begin_{g+1}), begin_g = floor(g n_slices / n_slabs),
 * and of every reference row the entries in those slices (in row order);
 * the view shift keeps a cell in its slice, so one copy serves every view.
 * Each (view, class) batch of eqs. 17-18 runs as: every slab's part of each
 * ray sum (one launch per slab); the sum of the parts in slab order (the
 * all-reduce of a multi-device run); every slab's multiplicative correction
 * with a_max of the whole row (one launch per slab).  One slab gives
 * mart_run's result bit for bit; more slabs change only the association of
 * the ray sums. */
#define USPG_MAX_SLABS 64
typedef struct uspg_slabs uspg_slabs;

/* Builds the slab rows of c (not for SEGMENTS coefficients) with
 * 1 <= n_slabs <= min(n_slices, USPG_MAX_SLABS), else E_ARG.  Allocates
 * the slab rows (as much device memory as c's rows), per slab and colour
 * class the list of rays with entries in the slab (4 bytes per ray and
 * slab it reaches) and per ray the set of its slabs (8 bytes); synchronises
 * `stream`.  c must outlive the handle. */
int uspg_build_slabs(const uspg_coeffs *c, int32_t n_slabs, void *stream, uspg_slabs **out);

/* Slices [*slice_begin, *slice_end) and reference entries of one slab
 * (nullable outputs); E_ARG for a slab out of range. */
int uspg_slabs_info(const uspg_slabs *s, int32_t slab, int32_t *slice_begin, int32_t *slice_end, int64_t *nnz);

/* Work space of mart_run_slabs: the device-layout image plus one partial
 * ray sum per slab and ray of the largest class. */
size_t uspg_slabs_workspace_bytes(const uspg_slabs *s, int32_t dtype);

/* MART as mart_run (same proj, image, n_sweeps, beta and stream; no
 * stopping rule), each batch split over the slabs.  E_NOMEM when work is
 * smaller than uspg_slabs_workspace_bytes. */
int mart_run_slabs(const uspg_slabs *s, int32_t dtype, const void *proj, void *image, void *work,
                   size_t work_bytes, int32_t n_sweeps, double beta, void *stream);

void uspg_free_slabs(uspg_slabs *s);

/* ---- allocation accounting (tests of error paths) --------------------------
 * *live (nullable) receives the number of device allocations the library
 * holds right now (handles' own memory and temporaries; not caller work
 * space).  fail_after > 0 makes the fail_after-th library device allocation
 * from now fail as if the device were out of memory (the call then returns
 * USPG_E_NOMEM); 0 cancels a pending one; < 0 leaves it as it is.
 * Process-wide; meant for tests. */
int uspg_debug_alloc(int32_t fail_after, int64_t *live);

/* ---- debug checks -----------------------------------------------------------
 * Race check of the MART order (Sec. III.D: a class batch equals its rays
 * applied one by one only if the rays of each class share no cell): for view
 * `view` and the lattice (ku, kv), every class c = (w mod kv) ku + (u mod ku)
 * stamps the cells of its rows, and *collisions receives the number of hits
 * on cells another ray of the same class had already hit (0 for a valid
 * lattice).  Independent of the conflict map the lattice was chosen from.
 * Stored rows only (E_ARG for SEGMENTS); E_ARG for a view or lattice out of
 * range.  Allocates a temporary 4-byte counter per device-layout cell and
 * synchronises `stream`. */
int uspg_check_lattice(const uspg_coeffs *c, int32_t view, int32_t ku, int32_t kv, void *stream,
                       int64_t *collisions);

/* Counts the entries of proj (device, n_views x rays of c, dtype
 * USPG_F32 / USPG_F64) that are NaN, infinite or negative: eq. 18 keeps the
 * image positive only for finite, non-negative data.  Synchronises
 * `stream`. */
int uspg_check_projections(const uspg_coeffs *c, int32_t dtype, const void *proj, void *stream, int64_t *n_bad);

/* Message of the calling thread's last failure ("" if none). */
const char *uspg_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* USPG_H */
