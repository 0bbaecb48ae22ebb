/*
 * uspg_oracle.c -- plain FP64 CPU oracle for MART on a Uniformly Sampled
 * Polar / Cylindrical Grid (USPG / USCG).
 *
 * TEST INFRASTRUCTURE ONLY.  This is the slow, obviously correct reference
 * that the tests, the smoke check and the benchmark's CPU-baseline leg compare
 * the HIP library against.  It shares no code, header, table or constant
 * generator with the library, and the library never links or calls it.
 *
 * What it computes (paper: Chaudhary, Wahi, Munshi, "Uniformly Sampled Polar
 * and Cylindrical Grid Approach for 2D, 3D Image Reconstruction using
 * Algebraic Algorithm"):
 *   - the grid: ring sector counts (Sec. II.A, eq. 1) and ring heads (eq. 2);
 *   - the coefficient row of one ray by direct tracing: cylinder clip
 *     (Sec. III.A, eqs. 3-4), axial and cylindrical breakpoints sorted by
 *     distance to the source (Alg. 1), per-segment slice / ring /
 *     azimuth / sector (eqs. 5-10) and the sector range of a segment inside a
 *     ring (eqs. 11-16), with lengths cut at the enumerated radial planes;
 *   - the rows of any view from the reference view by rotating the stored
 *     sector index (Sec. III.C and the rotation part of Alg. 1);
 *   - a lattice colouring of the reference view's rays into cell-disjoint
 *     classes, which fixes MART's ray order;
 *   - Sp-MART (Sec. III.D, eqs. 17-19), one ray at a time;
 *   - the USPG -> Cartesian remap (Sec. II.B).  Parity unpinned: where the
 *     bijection mode's numbering of a square ring starts and which way it
 *     runs (a reading of a figure the text does not describe); its pixel
 *     counts and the one-to-one property are pinned.
 *
 * Readings where the paper is silent or garbled are listed with the functions
 * that take them.  Status codes: 0 ok, -1 bad argument, -2 the grid is not
 * invariant under the view rotation, -3 output capacity too small.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_OK 0
#define ORC_E_ARG (-1)
#define ORC_E_SHIFT (-2)
#define ORC_E_CAP (-3)

#define GEOM_PARALLEL2D 0
#define GEOM_FAN2D 1
#define GEOM_CONE3D 2

static const double TWO_PI = 6.283185307179586476925286766559;
static const double PI = 3.141592653589793238462643383279;

typedef struct {
    /* grid */
    int nr, nz;
    double R, H, r, h, z0;
    int *ng;          /* sectors per ring */
    int64_t *head;    /* ring heads, nr + 1 entries */
    int64_t c2d;      /* cells per slice */
    /* scan */
    int geom, p;
    double span;
    int U, V;
    double Wu, Wv, Dso, Dsd;
    int binary;
    double eps;       /* pieces of length <= eps are dropped */
} orc_t;

/* ------------------------------------------------------------------------ */
/* Grid (Sec. II.A, eqs. 1-2)                                                */
/* ------------------------------------------------------------------------ */

/* Sector counts per ring, 0-based ring i (paper's n = i + 1).
 *   rule 0: the paper's equal-area rule n_g = 4(2n - 1) (eq. 1);
 *   rule 1: m * ceil(2 pi (i + 1/2) / m): cell area close to r^2 and every
 *           count a multiple of m, so rotations by 2 pi / m map the grid onto
 *           itself (reading: needed for the integer view shift);
 *   rule 2: an explicit table.                                            */
int orc_sector_counts(int rule, int m, int nr, const int *table, int *ng)
{
    if (nr <= 0) return ORC_E_ARG;
    for (int i = 0; i < nr; ++i) {
        if (rule == 0) {
            ng[i] = 4 * (2 * (i + 1) - 1);
        } else if (rule == 1) {
            if (m <= 0) return ORC_E_ARG;
            ng[i] = m * (int)ceil(TWO_PI * (i + 0.5) / m);
        } else if (rule == 2) {
            if (!table || table[i] < 2) return ORC_E_ARG;
            ng[i] = table[i];
        } else {
            return ORC_E_ARG;
        }
    }
    return ORC_OK;
}

void *orc_create(int nr, int nz, double R, double H, const int *ng,
                 int geom, int p, double span, int U, int V,
                 double Wu, double Wv, double Dso, double Dsd, int binary)
{
    if (nr <= 0 || nz <= 0 || R <= 0 || p <= 0 || U <= 0 || V <= 0) return NULL;
    if (geom == GEOM_CONE3D && H <= 0) return NULL;
    if (geom != GEOM_CONE3D && (nz != 1 || V != 1)) return NULL;
    orc_t *o = (orc_t *)calloc(1, sizeof(orc_t));
    o->nr = nr; o->nz = nz; o->R = R; o->H = H;
    o->r = R / nr;
    o->h = (geom == GEOM_CONE3D) ? H / nz : 0.0;
    o->z0 = -H / 2;
    o->ng = (int *)malloc(sizeof(int) * nr);
    o->head = (int64_t *)malloc(sizeof(int64_t) * (nr + 1));
    /* eq. 2: H_1 = 0, H_{n+1} = H_n + n_g(n) */
    o->head[0] = 0;
    for (int i = 0; i < nr; ++i) {
        o->ng[i] = ng[i];
        o->head[i + 1] = o->head[i] + ng[i];
    }
    o->c2d = o->head[nr];
    o->geom = geom; o->p = p; o->span = span; o->U = U; o->V = V;
    o->Wu = Wu; o->Wv = Wv; o->Dso = Dso; o->Dsd = Dsd; o->binary = binary;
    o->eps = 1e-12 * R;
    return o;
}

void orc_destroy(void *h)
{
    orc_t *o = (orc_t *)h;
    if (!o) return;
    free(o->ng); free(o->head); free(o);
}

int64_t orc_ncells(void *h) { orc_t *o = (orc_t *)h; return o->c2d * o->nz; }
int64_t orc_nrays(void *h) { orc_t *o = (orc_t *)h; return (int64_t)o->U * o->V; }

void orc_grid_tables(void *h, int *ng, int64_t *head)
{
    orc_t *o = (orc_t *)h;
    for (int i = 0; i < o->nr; ++i) ng[i] = o->ng[i];
    for (int i = 0; i <= o->nr; ++i) head[i] = o->head[i];
}

/* ------------------------------------------------------------------------ */
/* Rays of a view                                                            */
/* ------------------------------------------------------------------------ */

/* Source point S and detector point D of ray `ray` in view `view`.  View v is
 * the reference arrangement rotated anticlockwise about z by v * span / p
 * (Sec. IV: source and detector rotate together; first view at angle 0). */
void orc_ray(void *h, int view, int64_t ray, double *S, double *D)
{
    orc_t *o = (orc_t *)h;
    double th = view * o->span / o->p;
    double c = cos(th), s = sin(th);
    double S0[3], D0[3];
    if (o->geom == GEOM_PARALLEL2D) {
        double t = -o->Wu + (ray + 0.5) * (2.0 * o->Wu / o->U);
        S0[0] = -2.0 * o->R; S0[1] = t; S0[2] = 0.0;
        D0[0] = 2.0 * o->R;  D0[1] = t; D0[2] = 0.0;
    } else {
        int64_t u = ray % o->U, w = ray / o->U;
        double y = -o->Wu + (u + 0.5) * (2.0 * o->Wu / o->U);
        double z = (o->geom == GEOM_CONE3D) ? -o->Wv + (w + 0.5) * (2.0 * o->Wv / o->V) : 0.0;
        S0[0] = -o->Dso; S0[1] = 0.0; S0[2] = 0.0;
        D0[0] = o->Dsd - o->Dso; D0[1] = y; D0[2] = z;
    }
    S[0] = c * S0[0] - s * S0[1]; S[1] = s * S0[0] + c * S0[1]; S[2] = S0[2];
    D[0] = c * D0[0] - s * D0[1]; D[1] = s * D0[0] + c * D0[1]; D[2] = D0[2];
}

/* ------------------------------------------------------------------------ */
/* Direct trace of one ray (Sec. III.A-B, Alg. 1)                            */
/* ------------------------------------------------------------------------ */

typedef struct { double *t; int n, cap; } tvec;

static void tpush(tvec *v, double t)
{
    if (v->n == v->cap) {
        v->cap = v->cap ? 2 * v->cap : 1024;
        v->t = (double *)realloc(v->t, sizeof(double) * v->cap);
    }
    v->t[v->n++] = t;
}

static int cmp_double(const void *a, const void *b)
{
    double x = *(const double *)a, y = *(const double *)b;
    return (x > y) - (x < y);
}

/* eq. 8, with the reading that tan^-1(y/x) is the full-circle azimuth mapped
 * to [0, 2 pi). */
static double azimuth(double x, double y)
{
    double a = atan2(y, x);
    if (a < 0) a += TWO_PI;
    return a;
}

/* The cell containing point (x, y, z): slice by eq. 6 (z measured from the
 * bottom of the cylinder), ring by eq. 7, sector by eq. 10 (with eq. 9's step
 * in radians); the grid number adds the ring head H_n and the slice offset.
 * Indices are clamped to their ranges as a guard only. */
static int64_t cell_of_point(const orc_t *o, double x, double y, double z)
{
    double rho = sqrt(x * x + y * y);
    int i = (int)floor(rho / o->r);
    if (i < 0) i = 0;
    if (i >= o->nr) i = o->nr - 1;
    double dphi = TWO_PI / o->ng[i];
    int s = (int)floor(azimuth(x, y) / dphi);
    if (s < 0) s = 0;
    if (s >= o->ng[i]) s = o->ng[i] - 1;
    int k = 0;
    if (o->geom == GEOM_CONE3D) {
        k = (int)floor((z - o->z0) / o->h);
        if (k < 0) k = 0;
        if (k >= o->nz) k = o->nz - 1;
    }
    return (int64_t)k * o->c2d + o->head[i] + s;
}

typedef struct { int64_t cell; double len; int64_t order; } piece;

static int cmp_piece(const void *a, const void *b)
{
    const piece *x = (const piece *)a, *y = (const piece *)b;
    if (x->cell != y->cell) return (x->cell > y->cell) - (x->cell < y->cell);
    return (x->order > y->order) - (x->order < y->order);
}

static int cmp_order(const void *a, const void *b)
{
    const piece *x = (const piece *)a, *y = (const piece *)b;
    return (x->order > y->order) - (x->order < y->order);
}

/* Parameter of the crossing of the line S + t e with the radial line at
 * azimuth alpha (the plane through the z axis at that angle). */
static int radial_crossing(const double *S, const double *e, double alpha, double *t)
{
    double ca = cos(alpha), sa = sin(alpha);
    double den = e[0] * sa - e[1] * ca;
    if (den == 0.0) return 0;
    *t = (S[1] * ca - S[0] * sa) / den;
    return 1;
}

/* Breakpoints of the line S + t e (e = D - S) inside the grid (Alg. 1 steps
 * 3-4): the chord's ends, its crossings with the cylindrical planes
 * rho = j r (eqs. 3-4) and with the axial planes z = z0 + k h strictly
 * inside it, sorted by distance to the source.  Returns 0 if the line
 * misses the grid; *L is the length per unit t. */
static int line_breakpoints(const orc_t *o, const double *S, const double *D, double *e, double *L,
                            tvec *bp)
{
    const int is3d = (o->geom == GEOM_CONE3D);
    e[0] = D[0] - S[0]; e[1] = D[1] - S[1]; e[2] = is3d ? D[2] - S[2] : 0.0;
    double A = e[0] * e[0] + e[1] * e[1];          /* <S-D', S-D'> */
    *L = sqrt(A + e[2] * e[2]);                    /* length per unit t */
    if (A == 0.0) return 0;

    /* eq. 3: distance d of the XY projection S D' from the axis */
    double sdx = S[0] - D[0], sdy = S[1] - D[1];
    double t = (S[0] * sdx + S[1] * sdy) / A;
    double d2 = (S[0] * S[0] + S[1] * S[1]) - t * t * A;
    if (d2 < 0) d2 = 0;
    if (d2 >= o->R * o->R) return 0;
    /* eq. 4: the line meets the cylinder at S + (t -+ k)(D - S) */
    double k = sqrt((o->R * o->R - d2) / A);
    double t0 = t - k, t1 = t + k;
    if (is3d) {
        /* clip to the slab z0 <= z <= z0 + H (the axial end planes) */
        if (e[2] == 0.0) {
            if (S[2] < o->z0 || S[2] > o->z0 + o->H) return 0;
        } else {
            double ta = (o->z0 - S[2]) / e[2], tb = (o->z0 + o->H - S[2]) / e[2];
            if (ta > tb) { double x = ta; ta = tb; tb = x; }
            if (ta > t0) t0 = ta;
            if (tb < t1) t1 = tb;
        }
        if (t1 <= t0) return 0;
    }

    /* Alg. 1: intersections with the cylindrical planes rho = j r and
     * the axial planes z = z0 + k h strictly inside the chord. */
    tpush(bp, t0);
    tpush(bp, t1);
    for (int j = 1; j < o->nr; ++j) {
        double rj = j * o->r;
        if (rj * rj <= d2) continue;
        double kj = sqrt((rj * rj - d2) / A);
        double ta = t - kj, tb = t + kj;
        if (ta > t0 && ta < t1) tpush(bp, ta);
        if (tb > t0 && tb < t1) tpush(bp, tb);
    }
    if (is3d && e[2] != 0.0) {
        for (int kk = 1; kk < o->nz; ++kk) {
            double tz = (o->z0 + kk * o->h - S[2]) / e[2];
            if (tz > t0 && tz < t1) tpush(bp, tz);
        }
    }
    /* Alg. 1: sort by distance to the source */
    qsort(bp->t, bp->n, sizeof(double), cmp_double);
    return 1;
}

/* Trace the line from S towards D through the grid.  Writes one entry per
 * traversed cell (cell id in the paper's numbering, k * C2D + H_i + s, and the
 * intersection length; 1.0 in binary mode), in order of first entry along the
 * ray.  Returns the entry count, or ORC_E_CAP if `cap` is too small (then the
 * count is stored in *need). */
static int trace_line(const orc_t *o, const double *S, const double *D,
                      int64_t *cells, double *lens, int cap, int *need)
{
    double e[3], L;
    tvec bp = {0, 0, 0};
    *need = 0;
    if (!line_breakpoints(o, S, D, e, &L, &bp)) {
        free(bp.t);
        return 0;
    }

    /* Each segment between consecutive points lies in one ring and one slice.
     * Find the sectors it crosses from the grid numbers of its end points
     * (eqs. 8-10) and the two cases of eqs. 11-16, and cut it at the radial
     * planes between those sectors. */
    tvec all = {0, 0, 0};
    for (int q = 0; q < bp.n; ++q) tpush(&all, bp.t[q]);
    for (int q = 0; q + 1 < bp.n; ++q) {
        double ta = bp.t[q], tb = bp.t[q + 1];
        if ((tb - ta) * L <= o->eps) continue;
        double tm = 0.5 * (ta + tb);                       /* eq. 5 */
        double mx = S[0] + tm * e[0], my = S[1] + tm * e[1];
        int ring = (int)floor(sqrt(mx * mx + my * my) / o->r);   /* eq. 7 */
        if (ring < 0) ring = 0;
        if (ring >= o->nr) ring = o->nr - 1;
        int ng = o->ng[ring];
        double dphi = TWO_PI / ng;                          /* eq. 9 */
        double pa = azimuth(S[0] + ta * e[0], S[1] + ta * e[1]);   /* eq. 8 */
        double pb = azimuth(S[0] + tb * e[0], S[1] + tb * e[1]);
        int Ga = (int)floor(pa / dphi), Gb = (int)floor(pb / dphi); /* eq. 10 */
        if (Ga >= ng) Ga = ng - 1;
        if (Gb >= ng) Gb = ng - 1;
        int Lh, Lt;
        if (fabs(pa - pb) < PI) {
            /* Case 1 (eqs. 11-13): sectors L_h .. L_t; the radial planes
             * between them are at angles (L_h + 1) .. L_t times the step. */
            Lh = Ga < Gb ? Ga : Gb;
            Lt = Ga < Gb ? Gb : Ga;
            for (int s = Lh + 1; s <= Lt; ++s) {
                double tc;
                if (radial_crossing(S, e, s * dphi, &tc) && tc > ta && tc < tb) tpush(&all, tc);
            }
        } else {
            /* Case 2 (eqs. 14-16): the segment crosses the +x axis; walk from
             * the head L_h = max up through the tail of the ring, wrap to
             * index 0 and continue to L_t = min. */
            Lh = Ga < Gb ? Gb : Ga;
            Lt = Ga < Gb ? Ga : Gb;
            for (int s = Lh + 1; s <= ng; ++s) {
                double tc;
                if (radial_crossing(S, e, (s == ng) ? 0.0 : s * dphi, &tc) && tc > ta && tc < tb)
                    tpush(&all, tc);
            }
            for (int s = 1; s <= Lt; ++s) {
                double tc;
                if (radial_crossing(S, e, s * dphi, &tc) && tc > ta && tc < tb) tpush(&all, tc);
            }
        }
    }
    qsort(all.t, all.n, sizeof(double), cmp_double);

    /* Classify every piece by its midpoint (eq. 5) and merge repeated cells
     * (a line can enter one annular sector twice: annular sectors are not
     * convex), keeping the order of first entry. */
    piece *pc = (piece *)malloc(sizeof(piece) * (all.n > 0 ? all.n : 1));
    int np = 0;
    for (int q = 0; q + 1 < all.n; ++q) {
        double ta = all.t[q], tb = all.t[q + 1];
        double len = (tb - ta) * L;
        if (len <= o->eps) continue;
        double tm = 0.5 * (ta + tb);
        pc[np].cell = cell_of_point(o, S[0] + tm * e[0], S[1] + tm * e[1], S[2] + tm * e[2]);
        pc[np].len = len;
        pc[np].order = np;
        ++np;
    }
    qsort(pc, np, sizeof(piece), cmp_piece);
    int nu = 0;
    for (int q = 0; q < np; ++q) {
        if (nu > 0 && pc[nu - 1].cell == pc[q].cell) {
            pc[nu - 1].len += pc[q].len;
        } else {
            pc[nu++] = pc[q];
        }
    }
    qsort(pc, nu, sizeof(piece), cmp_order);
    *need = nu;
    int ret = nu;
    if (nu > cap) {
        ret = ORC_E_CAP;
    } else {
        for (int q = 0; q < nu; ++q) {
            cells[q] = pc[q].cell;
            lens[q] = o->binary ? 1.0 : pc[q].len;
        }
    }
    free(pc); free(bp.t); free(all.t);
    return ret;
}

int orc_trace_line(void *h, const double *S, const double *D, int64_t *cells, double *lens,
                   int cap, int *need)
{
    return trace_line((orc_t *)h, S, D, cells, lens, cap, need);
}

/* Direct trace of every ray of one view into CSR (rowptr has rays + 1
 * entries).  With cells == NULL only rowptr is filled (size query). */
int64_t orc_trace_view(void *h, int view, int64_t *rowptr, int64_t *cells, double *lens,
                       int64_t cap, int nthreads)
{
    orc_t *o = (orc_t *)h;
    int64_t nrays = (int64_t)o->U * o->V;
    int *cnt = (int *)malloc(sizeof(int) * nrays);
    int big = 4 * (o->nr + o->nz + 8) + 64;
    (void)nthreads;
#pragma omp parallel for schedule(dynamic, 16) num_threads(nthreads > 0 ? nthreads : 1)
    for (int64_t r = 0; r < nrays; ++r) {
        double S[3], D[3];
        orc_ray(o, view, r, S, D);
        int cap1 = big, need = 0;
        int64_t *c1 = (int64_t *)malloc(sizeof(int64_t) * cap1);
        double *l1 = (double *)malloc(sizeof(double) * cap1);
        int n = trace_line(o, S, D, c1, l1, cap1, &need);
        if (n == ORC_E_CAP) n = need;
        cnt[r] = n;
        free(c1); free(l1);
    }
    rowptr[0] = 0;
    for (int64_t r = 0; r < nrays; ++r) rowptr[r + 1] = rowptr[r] + cnt[r];
    free(cnt);
    int64_t nnz = rowptr[nrays];
    if (!cells) return nnz;
    if (nnz > cap) return ORC_E_CAP;
#pragma omp parallel for schedule(dynamic, 16) num_threads(nthreads > 0 ? nthreads : 1)
    for (int64_t r = 0; r < nrays; ++r) {
        double S[3], D[3];
        int need = 0;
        orc_ray(o, view, r, S, D);
        trace_line(o, S, D, cells + rowptr[r], lens + rowptr[r],
                   (int)(rowptr[r + 1] - rowptr[r]), &need);
    }
    return nnz;
}

/* ------------------------------------------------------------------------ */
/* Rotation of the stored reference view (Sec. III.C, Alg. 1)               */
/* ------------------------------------------------------------------------ */

/* Number q of view steps in a full turn; the rotation of view v maps sector s
 * of ring i to s + v n_g(i) / q when q divides every n_g(i).  Adding the
 * source angle to the stored azimuths and re-applying eq. 10 is then an exact
 * shift of the sector index. */
static int view_group(const orc_t *o, int *q)
{
    double qf = o->p * TWO_PI / o->span;
    int qi = (int)floor(qf + 0.5);
    if (qi <= 0 || fabs(qf - qi) > 1e-9) return ORC_E_SHIFT;
    for (int i = 0; i < o->nr; ++i)
        if (o->ng[i] % qi) return ORC_E_SHIFT;
    *q = qi;
    return ORC_OK;
}

int orc_shift_ok(void *h)
{
    int q;
    return view_group((orc_t *)h, &q);
}

/* Slice, ring and sector of a cell id (paper numbering). */
static void split_cell(const orc_t *o, int64_t cell, int *k, int *i, int *s)
{
    int64_t kk = cell / o->c2d, rem = cell % o->c2d;
    int lo = 0, hi = o->nr - 1;
    while (lo < hi) {               /* last ring whose head <= rem */
        int mid = (lo + hi + 1) / 2;
        if (o->head[mid] <= rem) lo = mid; else hi = mid - 1;
    }
    *k = (int)kk; *i = lo; *s = (int)(rem - o->head[lo]);
}

/* Map view-0 cells to view `view`: (k, i, s) -> (k, i, (s + v n_g/q) mod n_g). */
int orc_rotate_cells(void *h, int view, const int64_t *cells0, int64_t n, int64_t *out)
{
    orc_t *o = (orc_t *)h;
    int q;
    if (view_group(o, &q) != ORC_OK) return ORC_E_SHIFT;
    for (int64_t j = 0; j < n; ++j) {
        int k, i, s;
        split_cell(o, cells0[j], &k, &i, &s);
        int sh = (int)(((int64_t)view * (o->ng[i] / q)) % o->ng[i]);
        out[j] = (int64_t)k * o->c2d + o->head[i] + (s + sh) % o->ng[i];
    }
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Colouring of the reference view (fixes MART's ray order)                  */
/* ------------------------------------------------------------------------ */

/* Conflict offsets: mark[dw * U + du] = 1 if two distinct reference-view rays
 * (u1, w1), (u2, w2) with |u1-u2| = du, |w1-w2| = dw traverse a common cell.
 * Built from the cell -> rays transpose of the reference CSR. */
int orc_conflict_offsets(void *h, const int64_t *rowptr, const int64_t *cells, uint8_t *mark)
{
    orc_t *o = (orc_t *)h;
    int64_t nrays = (int64_t)o->U * o->V, ncell = o->c2d * o->nz;
    int64_t nnz = rowptr[nrays];
    int64_t *cptr = (int64_t *)calloc(ncell + 1, sizeof(int64_t));
    for (int64_t j = 0; j < nnz; ++j) cptr[cells[j] + 1]++;
    for (int64_t c = 0; c < ncell; ++c) cptr[c + 1] += cptr[c];
    int64_t *fill = (int64_t *)malloc(sizeof(int64_t) * (ncell + 1));
    memcpy(fill, cptr, sizeof(int64_t) * (ncell + 1));
    int64_t *rays = (int64_t *)malloc(sizeof(int64_t) * (nnz > 0 ? nnz : 1));
    for (int64_t r = 0; r < nrays; ++r)
        for (int64_t j = rowptr[r]; j < rowptr[r + 1]; ++j) rays[fill[cells[j]]++] = r;
    memset(mark, 0, (size_t)nrays);
    for (int64_t c = 0; c < ncell; ++c) {
        for (int64_t a = cptr[c]; a < cptr[c + 1]; ++a) {
            for (int64_t b = a + 1; b < cptr[c + 1]; ++b) {
                int64_t ua = rays[a] % o->U, wa = rays[a] / o->U;
                int64_t ub = rays[b] % o->U, wb = rays[b] / o->U;
                int64_t du = ua > ub ? ua - ub : ub - ua;
                int64_t dw = wa > wb ? wa - wb : wb - wa;
                mark[dw * o->U + du] = 1;
            }
        }
    }
    free(cptr); free(fill); free(rays);
    return ORC_OK;
}

/* A lattice colouring assigns ray (u, w) the class (w mod Kv) Ku + (u mod Ku).
 * It is valid when no two rays of one class share a cell, i.e. when no
 * conflict offset has Ku | du and Kv | dw.  Rotation preserves disjointness,
 * so a lattice valid for the reference view is valid for every view.
 * Search: increasing Ku Kv, ties broken by the smaller Ku.  A forced lattice
 * (Ku, Kv > 0 on entry) is only checked. */
int orc_colour(void *h, const uint8_t *mark, int *Ku, int *Kv)
{
    orc_t *o = (orc_t *)h;
    int U = o->U, V = o->V;
    if (*Ku > 0 && *Kv > 0) {
        if (*Ku > U || *Kv > V) return ORC_E_ARG;
        for (int dw = 0; dw < V; dw += *Kv)
            for (int du = 0; du < U; du += *Ku)
                if (mark[(int64_t)dw * U + du]) return ORC_E_ARG;
        return ORC_OK;
    }
    for (int64_t P = 1; P <= (int64_t)U * V; ++P) {
        for (int64_t ku = 1; ku <= P; ++ku) {
            if (P % ku) continue;
            int64_t kv = P / ku;
            if (ku > U || kv > V) continue;
            int ok = 1;
            for (int64_t dw = 0; dw < V && ok; dw += kv)
                for (int64_t du = 0; du < U; du += ku)
                    if (mark[dw * U + du]) { ok = 0; break; }
            if (ok) { *Ku = (int)ku; *Kv = (int)kv; return ORC_OK; }
        }
    }
    return ORC_E_ARG;
}

/* ------------------------------------------------------------------------ */
/* Sp-MART (Sec. III.D, eqs. 17-19)                                          */
/* ------------------------------------------------------------------------ */

/* One ray's update on the cells `ids` with coefficients `a`:
 *   Pbar = sum_j a_j f_j                                   (eq. 17)
 *   rho  = P / Pbar          (reading: the discrepancy of eq. 18 is the ratio)
 *   f_j <- f_j (1 - beta (a_j / a_max) (1 - rho))          (eq. 18)
 * With binary coefficients a_j = a_max = 1 this is eq. 18 exactly; with
 * lengths, a_j / a_max weights the correction by the share of the ray in the
 * cell.  Empty rows and rows with Pbar <= 0 are skipped. */
void orc_mart_ray(const int64_t *ids, const double *a, int64_t n, double P, double *f, double beta)
{
    if (n <= 0) return;
    double pbar = 0.0, amax = 0.0;
    for (int64_t j = 0; j < n; ++j) {
        pbar += a[j] * f[ids[j]];
        if (a[j] > amax) amax = a[j];
    }
    if (!(pbar > 0.0) || !(amax > 0.0)) return;
    double rho = P / pbar;
    for (int64_t j = 0; j < n; ++j)
        f[ids[j]] *= 1.0 - beta * (a[j] / amax) * (1.0 - rho);
}

/* MART over `sweeps` sweeps in the order: views ascending (Alg. 1 loops
 * over the projections), then the lattice classes c = (w mod Kv) Ku +
 * (u mod Ku) ascending, then the rays of the class by ascending index
 * r = w U + u, each ray applied with orc_mart_ray.  The rows of view v are
 * the reference rows with every sector index rotated by v n_g(i) / q (the
 * stored coefficients are reused for all views, Sec. III.C).  The rays of one
 * class share no cell, so spreading them over `nthreads` OpenMP threads gives
 * the same image bit for bit as one thread.  With tol > 0 the sweeps stop
 * after the first sweep with max_j |f_new - f_old| / f_old <= tol (eq. 19). */
int orc_mart(void *h, const int64_t *rowptr, const int64_t *cells, const double *lens,
             int Ku, int Kv, const double *P, double *f, int sweeps, double beta,
             double tol, int *done, int nthreads)
{
    orc_t *o = (orc_t *)h;
    int q;
    if (view_group(o, &q) != ORC_OK) return ORC_E_SHIFT;
    if (Ku <= 0 || Kv <= 0 || sweeps < 0) return ORC_E_ARG;
    const int64_t U = o->U, V = o->V, nrays = U * V, ncell = o->c2d * o->nz;
    const int64_t nnz = rowptr[nrays];
    int *ck = (int *)malloc(sizeof(int) * (nnz > 0 ? nnz : 1));
    int *ci = (int *)malloc(sizeof(int) * (nnz > 0 ? nnz : 1));
    int *cs = (int *)malloc(sizeof(int) * (nnz > 0 ? nnz : 1));
    for (int64_t j = 0; j < nnz; ++j) split_cell(o, cells[j], &ck[j], &ci[j], &cs[j]);
    double *fold = tol > 0 ? (double *)malloc(sizeof(double) * ncell) : NULL;
    const int nth = nthreads > 0 ? nthreads : 1;
    int maxrow = 0;
    for (int64_t r = 0; r < nrays; ++r)
        if (rowptr[r + 1] - rowptr[r] > maxrow) maxrow = (int)(rowptr[r + 1] - rowptr[r]);
    int s_done = 0;
    for (int sw = 0; sw < sweeps; ++sw) {
        if (fold) memcpy(fold, f, sizeof(double) * ncell);
        for (int v = 0; v < o->p; ++v) {
            const double *Pv = P + (int64_t)v * nrays;
            for (int c = 0; c < Ku * Kv; ++c) {
                const int64_t cu = c % Ku, cw = c / Ku;
                const int64_t nu = (U - cu + Ku - 1) / Ku, nw = (V - cw + Kv - 1) / Kv;
#pragma omp parallel num_threads(nth)
                {
                    int64_t *ids = (int64_t *)malloc(sizeof(int64_t) * (maxrow > 0 ? maxrow : 1));
#pragma omp for schedule(dynamic, 64)
                    for (int64_t x = 0; x < nu * nw; ++x) {
                        const int64_t r = (cw + (x / nu) * Kv) * U + cu + (x % nu) * Ku;
                        const int64_t b = rowptr[r], n = rowptr[r + 1] - b;
                        for (int64_t j = 0; j < n; ++j) {
                            const int i = ci[b + j];
                            const int sh = (int)(((int64_t)v * (o->ng[i] / q)) % o->ng[i]);
                            ids[j] = (int64_t)ck[b + j] * o->c2d + o->head[i] + (cs[b + j] + sh) % o->ng[i];
                        }
                        orc_mart_ray(ids, lens + b, n, Pv[r], f, beta);
                    }
                    free(ids);
                }
            }
        }
        ++s_done;
        if (fold) {
            double mx = 0.0;
            for (int64_t j = 0; j < ncell; ++j) {
                double d = fabs((f[j] - fold[j]) / fold[j]);
                if (d > mx) mx = d;
            }
            if (mx <= tol) break;
        }
    }
    if (done) *done = s_done;
    free(ck); free(ci); free(cs); free(fold);
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* The paper's literal variant: segment records re-binned per view          */
/* (Sec. III.B-C, Alg. 1), binary coefficients, any number of views          */
/* ------------------------------------------------------------------------ */

/* Segment records of the line S -> D (Alg. 1, reference-view records): every piece between
 * consecutive cylinder / axial breakpoints longer than eps, in order along the
 * line, with the slice (eq. 6) and ring (eq. 7) of its midpoint (eq. 5) and
 * the azimuths (eq. 8) of its two end points.  No radial plane is crossed:
 * the sectors are found per view from the azimuths.  Returns the count, or
 * ORC_E_CAP with the count in *need. */
static int segments_line(const orc_t *o, const double *S, const double *D, int *slice, int *ring,
                         double *phia, double *phib, int cap, int *need)
{
    double e[3], L;
    tvec bp = {0, 0, 0};
    *need = 0;
    if (!line_breakpoints(o, S, D, e, &L, &bp)) {
        free(bp.t);
        return 0;
    }
    int n = 0;
    for (int q = 0; q + 1 < bp.n; ++q) {
        double ta = bp.t[q], tb = bp.t[q + 1];
        if ((tb - ta) * L <= o->eps) continue;
        if (n < cap) {
            double tm = 0.5 * (ta + tb);                               /* eq. 5 */
            double mx = S[0] + tm * e[0], my = S[1] + tm * e[1], mz = S[2] + tm * e[2];
            int i = (int)floor(sqrt(mx * mx + my * my) / o->r);        /* eq. 7 */
            if (i < 0) i = 0;
            if (i >= o->nr) i = o->nr - 1;
            int k = 0;
            if (o->geom == GEOM_CONE3D) {
                k = (int)floor((mz - o->z0) / o->h);                   /* eq. 6 */
                if (k < 0) k = 0;
                if (k >= o->nz) k = o->nz - 1;
            }
            slice[n] = k;
            ring[n] = i;
            phia[n] = azimuth(S[0] + ta * e[0], S[1] + ta * e[1]);    /* eq. 8 */
            phib[n] = azimuth(S[0] + tb * e[0], S[1] + tb * e[1]);
        }
        ++n;
    }
    free(bp.t);
    *need = n;
    return n > cap ? ORC_E_CAP : n;
}

int orc_segments_line(void *h, const double *S, const double *D, int *slice, int *ring, double *phia,
                      double *phib, int cap, int *need)
{
    return segments_line((orc_t *)h, S, D, slice, ring, phia, phib, cap, need);
}

/* Segment records of every reference-view ray (segptr has rays + 1 entries;
 * with slice == NULL only segptr is filled). */
int64_t orc_segments_view(void *h, int64_t *segptr, int *slice, int *ring, double *phia, double *phib,
                          int64_t cap, int nthreads)
{
    orc_t *o = (orc_t *)h;
    int64_t nrays = (int64_t)o->U * o->V;
    int *cnt = (int *)malloc(sizeof(int) * nrays);
#pragma omp parallel for schedule(dynamic, 16) num_threads(nthreads > 0 ? nthreads : 1)
    for (int64_t r = 0; r < nrays; ++r) {
        double S[3], D[3];
        int need = 0;
        orc_ray(o, 0, r, S, D);
        segments_line(o, S, D, NULL, NULL, NULL, NULL, 0, &need);
        cnt[r] = need;
    }
    segptr[0] = 0;
    for (int64_t r = 0; r < nrays; ++r) segptr[r + 1] = segptr[r] + cnt[r];
    free(cnt);
    int64_t ns = segptr[nrays];
    if (!slice) return ns;
    if (ns > cap) return ORC_E_CAP;
#pragma omp parallel for schedule(dynamic, 16) num_threads(nthreads > 0 ? nthreads : 1)
    for (int64_t r = 0; r < nrays; ++r) {
        double S[3], D[3];
        int need = 0;
        orc_ray(o, 0, r, S, D);
        segments_line(o, S, D, slice + segptr[r], ring + segptr[r], phia + segptr[r], phib + segptr[r],
                      (int)(segptr[r + 1] - segptr[r]), &need);
    }
    return ns;
}

/* Sectors of ring i met by a segment with reference azimuths pa, pb in view
 * `view` (per-view re-binning of Alg. 1).  Both azimuths advance by the source angle
 * theta_v = v span / p and are reduced to [0, 2 pi) (reading: eq. 10 needs
 * an angle inside the turn); eq. 10 gives the grid numbers (without the ring
 * head).  Case 1, |phi_a - phi_b| < pi (eqs. 11-13): sectors L_h = min ..
 * L_t = max.  Case 2 (eqs. 14-16): the segment crosses the +x axis, so the
 * sectors run from L_h = max up to n_g - 1 and on from 0 to L_t = min.
 * Result: first sector and count; the sectors are first, first + 1, ...
 * modulo n_g. */
static void rebin_segment(const orc_t *o, int view, int i, double pa, double pb, int *first, int *count)
{
    const double theta = view * o->span / o->p;
    const int ng = o->ng[i];
    const double dphi = TWO_PI / ng;                                  /* eq. 9 */
    double a = pa + theta, b = pb + theta;                            /* source angle */
    if (a >= TWO_PI) a -= TWO_PI;
    if (b >= TWO_PI) b -= TWO_PI;
    int Ga = (int)floor(a / dphi), Gb = (int)floor(b / dphi);         /* eq. 10 */
    if (Ga >= ng) Ga = ng - 1;
    if (Gb >= ng) Gb = ng - 1;
    int lo = Ga < Gb ? Ga : Gb, hi = Ga < Gb ? Gb : Ga;
    if (fabs(a - b) < PI) {
        *first = lo;                                                  /* eqs. 11-13 */
        *count = hi - lo + 1;
    } else {
        *first = hi;                                                  /* eqs. 14-16 */
        *count = ng - hi + lo + 1;
    }
}

static int cmp_i64(const void *a, const void *b)
{
    int64_t x = *(const int64_t *)a, y = *(const int64_t *)b;
    return (x > y) - (x < y);
}

/* Binary row of one ray in view `view` from its segment records: the union
 * of the cells (k C2D + H_i + s) of every segment's sector range, sorted
 * ascending.  A cell met by two segments (the two passes of a line through
 * the ring just outside the innermost ring it reaches, in one slice) counts
 * once: a binary coefficient marks a traversed cell.  `cells` needs room for
 * the sum of the counts.  Returns the number of distinct cells. */
static int rebin_row(const orc_t *o, int view, int nseg, const int *slice, const int *ring,
                     const double *phia, const double *phib, int64_t *cells)
{
    int n = 0;
    for (int q = 0; q < nseg; ++q) {
        int first, count;
        rebin_segment(o, view, ring[q], phia[q], phib[q], &first, &count);
        int ng = o->ng[ring[q]];
        for (int c = 0; c < count; ++c) {
            int sct = first + c;
            if (sct >= ng) sct -= ng;
            cells[n++] = (int64_t)slice[q] * o->c2d + o->head[ring[q]] + sct;
        }
    }
    qsort(cells, n, sizeof(int64_t), cmp_i64);
    int u = 0;
    for (int q = 0; q < n; ++q)
        if (u == 0 || cells[u - 1] != cells[q]) cells[u++] = cells[q];
    return u;
}

static int rebin_capacity(const orc_t *o, const int64_t *segptr)
{
    /* a segment meets at most n_g(i) sectors of its ring */
    int64_t nrays = (int64_t)o->U * o->V;
    int ngmax = 0;
    for (int i = 0; i < o->nr; ++i) ngmax = o->ng[i] > ngmax ? o->ng[i] : ngmax;
    int64_t mx = 0;
    for (int64_t r = 0; r < nrays; ++r) mx = segptr[r + 1] - segptr[r] > mx ? segptr[r + 1] - segptr[r] : mx;
    return (int)(mx * ngmax + 1);
}

/* Rows of view `view` by re-binning (rowptr has rays + 1 entries; with
 * cells == NULL only rowptr is filled). */
int64_t orc_rebin_view(void *h, int view, const int64_t *segptr, const int *slice, const int *ring,
                       const double *phia, const double *phib, int64_t *rowptr, int64_t *cells,
                       int64_t cap, int nthreads)
{
    orc_t *o = (orc_t *)h;
    int64_t nrays = (int64_t)o->U * o->V;
    int rcap = rebin_capacity(o, segptr);
    int *cnt = (int *)malloc(sizeof(int) * nrays);
#pragma omp parallel num_threads(nthreads > 0 ? nthreads : 1)
    {
        int64_t *tmp = (int64_t *)malloc(sizeof(int64_t) * rcap);
#pragma omp for schedule(dynamic, 16)
        for (int64_t r = 0; r < nrays; ++r) {
            int64_t b = segptr[r];
            cnt[r] = rebin_row(o, view, (int)(segptr[r + 1] - b), slice + b, ring + b, phia + b, phib + b, tmp);
        }
        free(tmp);
    }
    rowptr[0] = 0;
    for (int64_t r = 0; r < nrays; ++r) rowptr[r + 1] = rowptr[r] + cnt[r];
    free(cnt);
    int64_t nnz = rowptr[nrays];
    if (!cells) return nnz;
    if (nnz > cap) return ORC_E_CAP;
#pragma omp parallel num_threads(nthreads > 0 ? nthreads : 1)
    {
        int64_t *tmp = (int64_t *)malloc(sizeof(int64_t) * rcap);
#pragma omp for schedule(dynamic, 16)
        for (int64_t r = 0; r < nrays; ++r) {
            int64_t b = segptr[r];
            int n = rebin_row(o, view, (int)(segptr[r + 1] - b), slice + b, ring + b, phia + b, phib + b, tmp);
            memcpy(cells + rowptr[r], tmp, sizeof(int64_t) * n);
        }
        free(tmp);
    }
    return nnz;
}

/* Conflict offsets of the re-binned rows: the union over all views of the
 * offsets (du, dw) of ray pairs that share a cell in that view.  Re-binning
 * by a rotation that is not a whole number of sectors changes which rays
 * meet, so no single view decides; the union makes one lattice valid for
 * every view. */
int orc_rebin_conflicts(void *h, const int64_t *segptr, const int *slice, const int *ring,
                        const double *phia, const double *phib, uint8_t *mark, int nthreads)
{
    orc_t *o = (orc_t *)h;
    int64_t nrays = (int64_t)o->U * o->V;
    int64_t *rowptr = (int64_t *)malloc(sizeof(int64_t) * (nrays + 1));
    uint8_t *m1 = (uint8_t *)malloc((size_t)nrays);
    memset(mark, 0, (size_t)nrays);
    for (int v = 0; v < o->p; ++v) {
        int64_t nnz = orc_rebin_view(h, v, segptr, slice, ring, phia, phib, rowptr, NULL, 0, nthreads);
        int64_t *cells = (int64_t *)malloc(sizeof(int64_t) * (nnz > 0 ? nnz : 1));
        orc_rebin_view(h, v, segptr, slice, ring, phia, phib, rowptr, cells, nnz, nthreads);
        orc_conflict_offsets(h, rowptr, cells, m1);
        for (int64_t x = 0; x < nrays; ++x) mark[x] |= m1[x];
        free(cells);
    }
    free(rowptr); free(m1);
    return ORC_OK;
}

/* MART with binary coefficients from re-binned segment records, any number
 * of views (the per-view loop of Alg. 1 with Sec. III.D): views ascending, then lattice
 * classes, then the rays of a class ascending; each ray's row is rebuilt for
 * its view and updated by eq. 18 with a_j = a_max = 1.  The lattice must come
 * from orc_rebin_conflicts; the rays of a class then share no cell in any
 * view, so the optional thread parallelism over a class gives the same
 * result bit for bit. */
int orc_mart_rebin(void *h, const int64_t *segptr, const int *slice, const int *ring, const double *phia,
                   const double *phib, int Ku, int Kv, const double *P, double *f, int sweeps, double beta,
                   int nthreads)
{
    orc_t *o = (orc_t *)h;
    if (Ku <= 0 || Kv <= 0 || sweeps < 0) return ORC_E_ARG;
    int64_t nrays = (int64_t)o->U * o->V;
    int rcap = rebin_capacity(o, segptr);
    const int K = Ku * Kv;
    for (int sw = 0; sw < sweeps; ++sw) {
        for (int v = 0; v < o->p; ++v) {
            const double *Pv = P + (int64_t)v * nrays;
            for (int c = 0; c < K; ++c) {
                int cu = c % Ku, cw = c / Ku;
#pragma omp parallel num_threads(nthreads > 0 ? nthreads : 1)
                {
                    int64_t *ids = (int64_t *)malloc(sizeof(int64_t) * rcap);
                    double *ones = (double *)malloc(sizeof(double) * rcap);
                    for (int j = 0; j < rcap; ++j) ones[j] = 1.0;
#pragma omp for schedule(dynamic, 16)
                    for (int64_t r = 0; r < nrays; ++r) {
                        int u = (int)(r % o->U), w = (int)(r / o->U);
                        if (u % Ku != cu || w % Kv != cw) continue;
                        int64_t b = segptr[r];
                        int n = rebin_row(o, v, (int)(segptr[r + 1] - b), slice + b, ring + b, phia + b,
                                          phib + b, ids);
                        orc_mart_ray(ids, ones, n, Pv[r], f, beta);
                    }
                    free(ids); free(ones);
                }
            }
        }
    }
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* USPG -> Cartesian grid (Sec. II.B)                                        */
/* ------------------------------------------------------------------------ */

/* Pixel (ix, iy) of an nc x nc grid covering [-R, R]^2 has centre
 * (X R / nc, Y R / nc) with odd integers X = 2 ix + 1 - nc, Y = 2 iy + 1 - nc.
 *
 * mode 0 (point): the pixel takes the value of the cell containing its centre
 *   (0 outside the disk).  Reading for exact ties: centres on a diagonal
 *   (|X| == |Y|) sit at an odd multiple of pi/4, which can coincide with a
 *   sector boundary; their sector is taken from the exact angle.
 * mode 1 (bijection, Sec. II.B, Fig. 2): for the paper's grid (n_g = 4(2n-1))
 *   with nc = 2 Nr, square ring n (pixels with max(|X|,|Y|) = 2n - 1) has as
 *   many pixels as circular ring n; both are numbered anticlockwise from the
 *   +x axis (reading of Fig. 3; parity unpinned for that start and
 *   direction) and matched one to one.
 * cart is [Nz][nc][nc], row index iy (ascending y), column ix. */
int orc_remap(void *h, const double *f, double *cart, int nc, int mode)
{
    orc_t *o = (orc_t *)h;
    if (nc <= 0) return ORC_E_ARG;
    int64_t plane = (int64_t)nc * nc;
    if (mode == 0) {
        for (int iy = 0; iy < nc; ++iy) {
            for (int ix = 0; ix < nc; ++ix) {
                int X = 2 * ix + 1 - nc, Y = 2 * iy + 1 - nc;
                double x = X * o->R / nc, y = Y * o->R / nc;
                double rho = sqrt(x * x + y * y);
                int64_t cell = -1;
                if (rho < o->R) {
                    int i = (int)floor(rho / o->r);
                    if (i >= o->nr) i = o->nr - 1;
                    int ng = o->ng[i], s;
                    if (X == Y || X == -Y) {
                        /* exact angle oct * pi / 4, sector floor(oct n_g / 8) */
                        int oct = (X > 0 && Y > 0) ? 1 : (X < 0 && Y > 0) ? 3 : (X < 0) ? 5 : 7;
                        s = (int)(((int64_t)oct * ng) / 8);
                    } else {
                        s = (int)floor(azimuth(x, y) / (TWO_PI / ng));
                    }
                    if (s >= ng) s = ng - 1;
                    cell = o->head[i] + s;
                }
                for (int k = 0; k < o->nz; ++k)
                    cart[k * plane + (int64_t)iy * nc + ix] = cell < 0 ? 0.0 : f[k * o->c2d + cell];
            }
        }
        return ORC_OK;
    }
    if (mode == 1) {
        if (nc != 2 * o->nr) return ORC_E_ARG;
        for (int i = 0; i < o->nr; ++i)
            if (o->ng[i] != 4 * (2 * i + 1)) return ORC_E_ARG;
        for (int n = 1; n <= o->nr; ++n) {
            int M = 2 * n - 1, cnt = 0;
            int ringsz = 4 * (2 * n - 1);
            piece *px = (piece *)malloc(sizeof(piece) * ringsz);
            double *ang = (double *)malloc(sizeof(double) * ringsz);
            for (int iy = 0; iy < nc; ++iy)
                for (int ix = 0; ix < nc; ++ix) {
                    int X = 2 * ix + 1 - nc, Y = 2 * iy + 1 - nc;
                    int ax = X < 0 ? -X : X, ay = Y < 0 ? -Y : Y;
                    if ((ax > ay ? ax : ay) != M) continue;
                    px[cnt].cell = (int64_t)iy * nc + ix;
                    px[cnt].order = cnt;
                    ang[cnt] = azimuth((double)X, (double)Y);
                    px[cnt].len = ang[cnt];
                    ++cnt;
                }
            /* sort the ring's pixels by azimuth (insertion sort, rings are small) */
            for (int a = 1; a < cnt; ++a) {
                piece t = px[a];
                int b = a - 1;
                while (b >= 0 && px[b].len > t.len) { px[b + 1] = px[b]; --b; }
                px[b + 1] = t;
            }
            for (int j = 0; j < cnt; ++j)
                for (int k = 0; k < o->nz; ++k)
                    cart[k * plane + px[j].cell] = f[k * o->c2d + o->head[n - 1] + j];
            free(px); free(ang);
        }
        return ORC_OK;
    }
    return ORC_E_ARG;
}
