// Walk of one reference-view ray through the grid (host / device code).
//
// Along a straight line the three kinds of boundaries are met in monotone
// order, so no sort is needed:
//   * cylinders rho = j r: inwards from the outer ring to the innermost ring
//     jmin, then outwards again (crossing parameters tc -+ d_j, the eq. 4
//     form with d from the cross product S x e);
//   * radial planes: inside one ring piece the azimuth moves monotonically in
//     the direction of the ray's angular momentum, so the sectors between the
//     end points' sectors (eq. 10) are visited in order (eqs. 11-16);
//   * axial planes z = z0 + k h: the slice index moves monotonically.
// Pieces shorter than eps are dropped; the rest carry (slice, ring, sector)
// from the walk state.  A line meets an annular sector in at most two
// intervals, separated by a dip inside the sector's inner circle; with the
// sector rules accepted by the grid build such a dip can only stay inside one
// sector for the ring just outside the innermost ring, so the only repeat a
// row can hold is "last inbound piece of ring jmin+1 == first outbound piece"
// and it is merged there.
//
// Compiled by hipcc for the device; a plain C++ compiler can build it for the
// host (used only by the tests to check the walk on the CPU).
#pragma once

#include <cmath>
#include <cstdint>

#if defined(__HIPCC__)
#include <hip/hip_runtime.h>
#define USPG_HD __host__ __device__
#else
#define USPG_HD
struct double2 {
    double x, y;
};
#endif

// Floating point decides integers here (which cell a piece lies in), so the
// arithmetic must be the same on every compiler: no fused multiply-add.
#if defined(__clang__)
#pragma clang fp contract(off)
#endif

namespace uspg {
namespace walk {

constexpr double kTwoPiW = 6.283185307179586476925286766559;
constexpr int kParallel2D = 0;

// Geometry passed to the trace kernels by value.
struct TraceGeo {
    int nr, nz, is3d, geom;
    double R, r, h, z0, H;
    const int32_t *ng;
    const int64_t *head;
    const double2 *cs;
    const int32_t *kq, *hq;
    int64_t Cq, Wc;
    int grp;          // rings per group of the blocked in-plane layout
    int U, V;
    double Wu, Wv, Dso, Dsd;
    double eps;
};

// Ray handled by thread `tid` of a per-ray launch: the rays of one detector
// column (same u, consecutive rows) take neighbouring threads, so the lanes
// of a wavefront share their column's in-plane walk (same ring and sector
// steps, same table entries) and differ only in their slice steps.  A
// bijection of [0, U V); any other ray count keeps the identity.
USPG_HD inline int64_t column_major_ray(const TraceGeo &G, int64_t tid, int64_t nrays)
{
    if (G.U <= 0 || G.V <= 1 || nrays != (int64_t)G.U * G.V) return tid;
    return (tid % G.V) * G.U + tid / G.V;
}

// Device (wedge-major, ring-group blocked) image layout.
//
// With q view steps per turn, ring i holds k_i = n_g(i) / q sectors per
// wedge.  Inside one (wedge, slice) the rings are taken in groups of `grp`;
// a group is stored sector-major, ring-minor, padded to the group's largest
// k_i:  cell (i, b) sits at hq_i + b * grp, hq_i = group base + (i mod grp).
// So one 128-byte line holds 32 / grp sectors of grp neighbouring rings, and
// a line crossing rings radially stays in one line for up to grp cells.
// Whole image: wedge a, slice k at a * Wc + k * Cq, Wc = Nz * Cq; rotating
// by v views adds v * Wc modulo q * Wc.  Padding cells belong to no cell of
// the grid.  ring_of_off[o] is the ring of within-slice offset o, -1 for
// padding.  Returns Cq.
inline int64_t wedge_tables(int nr, const int32_t *ng, int q, int grp, int32_t *kq, int32_t *hq,
                            int32_t *ring_of_off /* may be null */)
{
    int64_t base = 0;
    for (int g0 = 0; g0 < nr; g0 += grp) {
        int kmax = 0;
        for (int i = g0; i < g0 + grp && i < nr; ++i) {
            kq[i] = ng[i] / q;
            kmax = kq[i] > kmax ? kq[i] : kmax;
        }
        for (int i = g0; i < g0 + grp && i < nr; ++i) {
            hq[i] = (int32_t)(base + (i - g0));
            if (ring_of_off) {
                for (int b = 0; b < kmax; ++b)
                    ring_of_off[base + (int64_t)b * grp + (i - g0)] = b < kq[i] ? i : -1;
            }
        }
        if (ring_of_off) {
            for (int j = nr - g0; j < grp; ++j)   // missing rings of a short last group
                for (int b = 0; b < kmax; ++b) ring_of_off[base + (int64_t)b * grp + j] = -1;
        }
        base += (int64_t)grp * kmax;
    }
    return base;
}

// Direction (cos, sin) of the lower boundary of sector b in a ring of ng
// sectors, angle 2 pi b / ng.  Reduced to the first half quadrant so that
// multiples of a quarter turn are exact and mirror-symmetric boundaries get
// mirror-symmetric values.
inline double2 boundary_dir(int b, int ng)
{
    long q4 = (4L * b) / ng;            // quadrant
    long rem = 4L * b - q4 * ng;        // angle (pi/2) rem / ng inside it
    double c, s;
    if (2 * rem <= ng) {
        double t = (kTwoPiW / 4) * (double)rem / ng;
        c = std::cos(t); s = std::sin(t);
    } else {
        double t = (kTwoPiW / 4) * (double)(ng - rem) / ng;
        c = std::sin(t); s = std::cos(t);
    }
    if (rem == 0) { c = 1.0; s = 0.0; }
    switch (q4 & 3) {
    case 0: return double2{c, s};
    case 1: return double2{-s, c};
    case 2: return double2{-c, -s};
    default: return double2{s, -c};
    }
}

struct Entry {
    uint32_t id;
    double len;
    int64_t slot;
};

// Collects a row: counts slots (WRITE = false) or writes them.
template <bool WRITE, class TC>
struct RowSink {
    static constexpr bool kPieces = false;   // takes emitted cell pieces, not whole sector pieces
    int64_t base;          // first output slot of the row
    int64_t count = 0;     // slots reserved so far
    bool pend = false, held = false, armed = false;
    Entry p{}, hd{};
    uint32_t *ids;
    TC *a;
    bool binary;
    double eps;
    // element strides of ids and a (in their own units): 1 for two plain
    // arrays, or the pair size when both point into an array of (id, a)
    // pairs
    int64_t ids_stride = 1, a_stride = 1;

    USPG_HD void flush(const Entry &e)
    {
        if (WRITE) {
            ids[(base + e.slot) * ids_stride] = e.id;
            a[(base + e.slot) * a_stride] = binary ? TC(1) : TC(e.len);
        }
    }
    USPG_HD void emit(uint32_t id, double len)
    {
        if (!(len > eps)) return;
        if (armed) {
            armed = false;
            if (pend) { flush(p); pend = false; }
            if (held && hd.id == id) {
                p = hd;
                p.len += len;
                pend = true;
                held = false;
                return;
            }
            if (held) { flush(hd); held = false; }
        }
        if (pend && p.id == id) {
            p.len += len;
            return;
        }
        if (pend) flush(p);
        p.id = id;
        p.len = len;
        p.slot = count++;
        pend = true;
    }
    USPG_HD void hold()
    {
        if (held) flush(hd);
        held = pend;
        hd = p;
        pend = false;
    }
    USPG_HD void arm() { armed = true; }
    USPG_HD void finish()
    {
        if (pend) flush(p);
        if (held) flush(hd);
        pend = held = false;
    }
};

struct Ray {
    double S[3], e[3];
    double A, L, cr, d2, tc, t0, t1;
};

USPG_HD inline double sq(double x) { return x * x; }

// View-0 source and detector point of ray `ray` (scan description).
USPG_HD inline void ray_points(const TraceGeo &G, int64_t ray, double *S, double *D)
{
    if (G.geom == kParallel2D) {
        double t = -G.Wu + (ray + 0.5) * (2.0 * G.Wu / G.U);
        S[0] = -2.0 * G.R; S[1] = t; S[2] = 0.0;
        D[0] = 2.0 * G.R;  D[1] = t; D[2] = 0.0;
    } else {
        int64_t u = ray % G.U, w = ray / G.U;
        double y = -G.Wu + (u + 0.5) * (2.0 * G.Wu / G.U);
        double z = G.is3d ? -G.Wv + (w + 0.5) * (2.0 * G.Wv / G.V) : 0.0;
        S[0] = -G.Dso; S[1] = 0.0; S[2] = 0.0;
        D[0] = G.Dsd - G.Dso; D[1] = y; D[2] = z;
    }
}

template <class Sink>
struct Walker {
    const TraceGeo &G;
    const Ray &ray;
    Sink &sink;
    // slice state
    int k = 0, dk = 0;
    double tz = INFINITY;   // parameter of the next axial plane in the direction of motion

    USPG_HD Walker(const TraceGeo &g, const Ray &r, Sink &s) : G(g), ray(r), sink(s) {}

    USPG_HD uint32_t cell_id(int i, int s) const
    {
        int kqi = G.kq[i];
        int aw = s / kqi;
        int b = s - aw * kqi;
        return (uint32_t)(aw * G.Wc + (int64_t)k * G.Cq + G.hq[i] + (int64_t)b * G.grp);
    }

    USPG_HD void next_plane()
    {
        // next axial plane strictly inside the cylinder, or none
        int kk = dk > 0 ? k + 1 : k;
        if (dk == 0 || kk <= 0 || kk >= G.nz) {
            tz = INFINITY;
            return;
        }
        tz = (G.z0 + kk * G.h - ray.S[2]) / ray.e[2];
    }

    USPG_HD void init_slices()
    {
        if (!G.is3d) {
            k = 0; dk = 0; tz = INFINITY;
            return;
        }
        double zs = ray.S[2] + ray.t0 * ray.e[2];
        k = (int)floor((zs - G.z0) / G.h);
        k = k < 0 ? 0 : (k >= G.nz ? G.nz - 1 : k);
        dk = ray.e[2] > 0 ? 1 : (ray.e[2] < 0 ? -1 : 0);
        next_plane();
    }

    // Piece [ta, tb] inside one ring and sector, cut at the axial planes.
    // A sink with kPieces set takes the whole sector piece instead (the
    // in-plane path of a detector column, whose rays differ only in z).
    USPG_HD void sector_piece(int i, int s, double ta, double tb)
    {
        if constexpr (Sink::kPieces) {
            sink.piece(cell_id(i, s), ta, tb);
        } else {
            double tcur = ta;
            while (tz < tb) {
                double t = tz > tcur ? tz : tcur;
                sink.emit(cell_id(i, s), (t - tcur) * ray.L);
                tcur = t;
                k += dk;
                if (k < 0 || k >= G.nz) {   // guard only: the chord is clipped to the slab
                    k -= dk;
                    tz = INFINITY;
                    break;
                }
                next_plane();
            }
            sink.emit(cell_id(i, s), (tb - tcur) * ray.L);
        }
    }

    USPG_HD int sector_of(int i, double x, double y) const
    {
        double phi = atan2(y, x);
        if (phi < 0) phi += kTwoPiW;
        int ng = G.ng[i];
        int s = (int)floor(phi / (kTwoPiW / ng));
        return s < 0 ? 0 : (s >= ng ? ng - 1 : s);
    }

    // Piece [ta, tb] inside ring i: walk the radial planes between the end
    // points' sectors in the direction of the angular motion.
    USPG_HD void ring_piece(int i, double ta, double tb)
    {
        if (ta < ray.t0) ta = ray.t0;
        if (tb > ray.t1) tb = ray.t1;
        if (!(tb > ta)) return;
        const double *S = ray.S, *e = ray.e;
        if (ray.cr == 0.0) {
            // the line passes through the axis: constant azimuth on each side
            if (ta < ray.tc && ray.tc < tb) {
                double m1 = 0.5 * (ta + ray.tc), m2 = 0.5 * (ray.tc + tb);
                sector_piece(i, sector_of(i, S[0] + m1 * e[0], S[1] + m1 * e[1]), ta, ray.tc);
                sector_piece(i, sector_of(i, S[0] + m2 * e[0], S[1] + m2 * e[1]), ray.tc, tb);
            } else {
                double m = 0.5 * (ta + tb);
                sector_piece(i, sector_of(i, S[0] + m * e[0], S[1] + m * e[1]), ta, tb);
            }
            return;
        }
        int ng = G.ng[i];
        int sa = sector_of(i, S[0] + ta * e[0], S[1] + ta * e[1]);
        int sb = sector_of(i, S[0] + tb * e[0], S[1] + tb * e[1]);
        int dir = ray.cr > 0 ? 1 : -1;
        int ncross = dir > 0 ? sb - sa : sa - sb;
        if (ncross < 0) ncross += ng;
        const double2 *cs = G.cs + G.head[i];
        int s = sa;
        double tcur = ta;
        for (int c = 0; c < ncross; ++c) {
            int bidx = dir > 0 ? (s + 1 == ng ? 0 : s + 1) : s;   // boundary left behind
            double2 b = cs[bidx];
            double den = e[0] * b.y - e[1] * b.x;
            double t = den != 0.0 ? (S[1] * b.x - S[0] * b.y) / den : tcur;
            t = t < tcur ? tcur : (t > tb ? tb : t);
            sector_piece(i, s, tcur, t);
            tcur = t;
            s = dir > 0 ? (s + 1 == ng ? 0 : s + 1) : (s == 0 ? ng - 1 : s - 1);
        }
        sector_piece(i, s, tcur, tb);
    }

    USPG_HD double dj(int j) const
    {
        // half-chord parameter of circle j (radius j r); circle nr is the rim
        if (j >= G.nr) return sqrt((sq(G.R) - ray.d2) / ray.A);
        return sqrt((sq(j * G.r) - ray.d2) / ray.A);
    }

    USPG_HD void run()
    {
        int nr = G.nr;
        // innermost ring: circles j with (j r)^2 <= d^2 are not crossed
        int jmin = (int)floor(sqrt(ray.d2) / G.r);
        jmin = jmin < 0 ? 0 : (jmin > nr - 1 ? nr - 1 : jmin);
        while (jmin + 1 < nr && sq((jmin + 1) * G.r) <= ray.d2) ++jmin;
        while (jmin > 0 && sq(jmin * G.r) > ray.d2) --jmin;
        init_slices();
        const double tc = ray.tc;
        for (int j = nr - 1; j > jmin; --j) {
            ring_piece(j, tc - dj(j + 1), tc - dj(j));
            if (j == jmin + 1) sink.hold();
        }
        double dm = dj(jmin + 1);
        ring_piece(jmin, tc - dm, tc + dm);
        for (int j = jmin + 1; j < nr; ++j) {
            if (j == jmin + 1) sink.arm();
            ring_piece(j, tc + dj(j), tc + dj(j + 1));
        }
        sink.finish();
    }
};

// Chord of the line from S towards D through the disk / cylinder; false if
// it misses.
USPG_HD inline bool setup_line(const TraceGeo &G, const double *S, const double *D, Ray &ray)
{
    ray.S[0] = S[0]; ray.S[1] = S[1]; ray.S[2] = S[2];
    ray.e[0] = D[0] - ray.S[0];
    ray.e[1] = D[1] - ray.S[1];
    ray.e[2] = G.is3d ? D[2] - ray.S[2] : 0.0;
    ray.A = ray.e[0] * ray.e[0] + ray.e[1] * ray.e[1];
    if (ray.A == 0.0) return false;
    ray.L = sqrt(ray.A + ray.e[2] * ray.e[2]);
    // distance of the XY line from the axis from the cross product S x e
    ray.cr = ray.S[0] * ray.e[1] - ray.S[1] * ray.e[0];
    ray.d2 = ray.cr * ray.cr / ray.A;
    double R2 = G.R * G.R;
    if (ray.d2 >= R2) return false;
    ray.tc = -(ray.S[0] * ray.e[0] + ray.S[1] * ray.e[1]) / ray.A;
    double half = sqrt((R2 - ray.d2) / ray.A);
    ray.t0 = ray.tc - half;
    ray.t1 = ray.tc + half;
    if (G.is3d) {
        double zlo = G.z0, zhi = G.z0 + G.H;
        if (ray.e[2] == 0.0) {
            if (ray.S[2] < zlo || ray.S[2] > zhi) return false;
        } else {
            double ta = (zlo - ray.S[2]) / ray.e[2], tb = (zhi - ray.S[2]) / ray.e[2];
            if (ta > tb) { double x = ta; ta = tb; tb = x; }
            if (ta > ray.t0) ray.t0 = ta;
            if (tb < ray.t1) ray.t1 = tb;
        }
    }
    return ray.t1 > ray.t0;
}

// View-0 ray `r` of the scan.
USPG_HD inline bool setup_ray(const TraceGeo &G, int64_t r, Ray &ray)
{
    double S[3], D[3];
    ray_points(G, r, S, D);
    return setup_line(G, S, D, ray);
}


}  // namespace walk
}  // namespace uspg
