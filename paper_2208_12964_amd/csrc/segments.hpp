// The paper's literal coefficient scheme (host / device code): segment
// records of the reference view re-binned to the sectors of any view.
//
// A line is cut only at the cylindrical planes rho = j r and the axial planes
// z = z0 + k h (Alg. 1, eqs. 3-4).  Each piece longer than eps lies
// in one ring and one slice, found from its midpoint (eqs. 5-7), and is
// stored with the azimuths of its two ends (eq. 8).  For view v both azimuths
// advance by the source angle theta_v = v span / p (Alg. 1); eq. 10
// turns them into sector numbers and the sectors between them (eqs. 11-16,
// two cases) are the cells the piece meets, each with coefficient 1 (binary
// weights, Sec. III.B).  Nothing requires the view step to be a whole number
// of sectors.
//
// The cut points come from three monotone sequences (inbound circles,
// outbound circles, axial planes), merged instead of sorted.  Every quantity
// that decides an integer (ring, slice, sector) is computed in FP64 without
// contraction, from the formulas of eqs. 3-10 as printed.
#pragma once

#include <cmath>
#include <cstdint>

#include "trace_walk.hpp"

#if defined(__clang__)
#pragma clang fp contract(off)
#endif

namespace uspg {
namespace seg {

constexpr double kTwoPiS = 6.283185307179586476925286766559;
constexpr double kPiS = 3.141592653589793238462643383279;

// Records are packed as slice << 16 | ring.
USPG_HD inline uint32_t pack(int slice, int ring) { return ((uint32_t)slice << 16) | (uint32_t)ring; }
USPG_HD inline int ring_of(uint32_t sr) { return (int)(sr & 0xffffu); }
USPG_HD inline int slice_of(uint32_t sr) { return (int)(sr >> 16); }

// eq. 8 as the full-turn azimuth in [0, 2 pi).
USPG_HD inline double azimuth(double x, double y)
{
    double a = atan2(y, x);
    return a < 0 ? a + kTwoPiS : a;
}

// Emits the segments of view-0 ray r in order along the ray:
// sink(slice, ring, phi_a, phi_b).  Returns the number emitted.
template <class Sink>
USPG_HD int segments_of_ray(const walk::TraceGeo &G, int64_t r, Sink &sink)
{
    double S[3], D[3];
    walk::ray_points(G, r, S, D);
    const double e0 = D[0] - S[0], e1 = D[1] - S[1], e2 = G.is3d ? D[2] - S[2] : 0.0;
    const double A = e0 * e0 + e1 * e1;               // <S - D', S - D'>
    const double L = sqrt(A + e2 * e2);
    if (A == 0.0) return 0;
    // eq. 3: d^2 = <S, S> - t^2 <S - D', S - D'>,  t = <S, S - D'> / <S - D', S - D'>
    const double sdx = S[0] - D[0], sdy = S[1] - D[1];
    const double t = (S[0] * sdx + S[1] * sdy) / A;
    double d2 = (S[0] * S[0] + S[1] * S[1]) - t * t * A;
    if (d2 < 0) d2 = 0;
    if (d2 >= G.R * G.R) return 0;
    // eq. 4: the line meets the cylinder at S + (t -+ k)(D - S)
    const double k = sqrt((G.R * G.R - d2) / A);
    double t0 = t - k, t1 = t + k;
    if (G.is3d) {
        if (e2 == 0.0) {
            if (S[2] < G.z0 || S[2] > G.z0 + G.H) return 0;
        } else {
            double ta = (G.z0 - S[2]) / e2, tb = (G.z0 + G.H - S[2]) / e2;
            if (ta > tb) { double x = ta; ta = tb; tb = x; }
            if (ta > t0) t0 = ta;
            if (tb < t1) t1 = tb;
        }
        if (t1 <= t0) return 0;
    }
    // innermost circle crossed: the largest j with (j r)^2 <= d2 is not
    int jlo = 1;
    while (jlo < G.nr && (jlo * G.r) * (jlo * G.r) <= d2) ++jlo;   // first crossed circle
    sink.begin(jlo);
    // circle sequence: j = nr-1 .. jlo at t - k_j, then j = jlo .. nr-1 at t + k_j
    const int ncirc = G.nr - jlo;                     // circles crossed (each twice)
    int ci = 0;                                       // index into the 2 ncirc circle points
    auto circ_t = [&](int idx) -> double {
        int j = idx < ncirc ? G.nr - 1 - idx : jlo + (idx - ncirc);
        double rj = j * G.r;
        double kj = sqrt((rj * rj - d2) / A);
        return idx < ncirc ? t - kj : t + kj;
    };
    // axial planes kk = 1 .. nz - 1 in the direction of motion
    const bool ax = G.is3d && e2 != 0.0;
    int kk = e2 > 0 ? 1 : G.nz - 1;
    const int dk = e2 > 0 ? 1 : -1;
    auto ax_t = [&](int kq) -> double { return (G.z0 + kq * G.h - S[2]) / e2; };
    auto next_circle = [&](double &tv) -> bool {
        while (ci < 2 * ncirc) {
            double x = circ_t(ci);
            if (x > t0 && x < t1) { tv = x; return true; }
            if (x >= t1) { ci = 2 * ncirc; return false; }
            ++ci;
        }
        return false;
    };
    auto next_axial = [&](double &tv) -> bool {
        if (!ax) return false;
        while (kk >= 1 && kk <= G.nz - 1) {
            double x = ax_t(kk);
            if (x > t0 && x < t1) { tv = x; return true; }
            if (x >= t1) { kk = -1; return false; }
            kk += dk;
        }
        return false;
    };
    int n = 0;
    double prev = t0;
    double tcv = 0, tav = 0;
    bool hc = next_circle(tcv), ha = next_axial(tav);
    for (;;) {
        double tb;
        if (hc && (!ha || tcv <= tav)) {
            tb = tcv;
            ++ci;
            hc = next_circle(tcv);
        } else if (ha) {
            tb = tav;
            kk += dk;
            ha = next_axial(tav);
        } else {
            tb = t1;
        }
        const double ta = prev;
        if ((tb - ta) * L > G.eps) {
            const double tm = 0.5 * (ta + tb);                               // eq. 5
            const double mx = S[0] + tm * e0, my = S[1] + tm * e1, mz = S[2] + tm * e2;
            int ring = (int)floor(sqrt(mx * mx + my * my) / G.r);            // eq. 7
            ring = ring < 0 ? 0 : (ring >= G.nr ? G.nr - 1 : ring);
            int slice = 0;
            if (G.is3d) {
                slice = (int)floor((mz - G.z0) / G.h);                       // eq. 6
                slice = slice < 0 ? 0 : (slice >= G.nz ? G.nz - 1 : slice);
            }
            sink(slice, ring, azimuth(S[0] + ta * e0, S[1] + ta * e1), azimuth(S[0] + tb * e0, S[1] + tb * e1));
            ++n;
        }
        if (tb == t1 && !hc && !ha) break;
        prev = tb;
    }
    return n;
}

// Sectors met in view `view` by a segment of a ring of ng sectors with
// reference azimuths pa, pb (per-view re-binning of Alg. 1): first sector and count,
// the sectors being first, first + 1, ... modulo ng.
USPG_HD inline void rebin_range(int ng, double pa, double pb, double theta, int &first, int &count)
{
    const double dphi = kTwoPiS / ng;                 // eq. 9
    double a = pa + theta, b = pb + theta;            // source angle
    if (a >= kTwoPiS) a -= kTwoPiS;
    if (b >= kTwoPiS) b -= kTwoPiS;
    int Ga = (int)floor(a / dphi), Gb = (int)floor(b / dphi);   // eq. 10
    if (Ga >= ng) Ga = ng - 1;
    if (Gb >= ng) Gb = ng - 1;
    const int lo = Ga < Gb ? Ga : Gb, hi = Ga < Gb ? Gb : Ga;
    if (fabs(a - b) < kPiS) {                         // case 1, eqs. 11-13
        first = lo;
        count = hi - lo + 1;
    } else {                                          // case 2, eqs. 14-16
        first = hi;
        count = ng - hi + lo + 1;
    }
}

// Source angle of view v.
USPG_HD inline double view_angle(int view, double span, int p) { return view * span / p; }

// Whether sector s lies in the circular range (first, count) of a ring of ng.
USPG_HD inline bool in_range(int s, int first, int count, int ng)
{
    int d = s - first;
    if (d < 0) d += ng;
    return d < count;
}

// Record of the mirror image of a view-0 ray (Sec. III.C): across y = 0
// (detector column u <-> U-1-u) the azimuth phi becomes 2 pi - phi; across
// z = 0 (row w <-> V-1-w) slice k becomes nz-1-k.  The order along the ray
// and the partner indices are unchanged.
USPG_HD inline void mirror_record(bool my, bool mz, int nz, uint32_t &sr, double &pa, double &pb)
{
    if (my) {
        pa = pa > 0 ? kTwoPiS - pa : 0.0;
        pb = pb > 0 ? kTwoPiS - pb : 0.0;
    }
    if (mz) sr = pack(nz - 1 - slice_of(sr), ring_of(sr));
}

// Segment sinks: count only, or write records with their partner (the
// earlier record of the same ring and slice, searched only for the ring
// just outside the innermost ring, jlo, back to the start of that ring's
// inbound pass).
struct CountSink {
    USPG_HD void begin(int) {}
    USPG_HD void operator()(int, int, double, double) {}
};

struct FillSink {
    uint32_t *sr;
    double *pa, *pb;
    int32_t *partner;
    int64_t base;
    int n = 0, jlo = 0;
    USPG_HD void begin(int j) { jlo = j; }
    USPG_HD void operator()(int slice, int ring, double a, double b)
    {
        const int64_t at = base + n;
        sr[at] = pack(slice, ring);
        pa[at] = a;
        pb[at] = b;
        int p = -1;
        if (ring == jlo) {
            for (int q = n - 1; q >= 0; --q) {
                const uint32_t o = sr[base + q];
                const int orr = ring_of(o);
                if (orr > jlo) break;
                if (orr == jlo && slice_of(o) == slice) { p = q; break; }
            }
        }
        partner[at] = p;
        ++n;
    }
};

// Sectors of record j of a ray's row (records sr[0..n), partner indices
// relative to the row) in the view of angle theta: the record's run
// (first, count), its partner's run (pf, pc; pc = 0 without a partner), the
// ring's sector count and the paper index of the ring's sector 0 in the
// record's slice.
struct RecordRange {
    int first, count, pf, pc, ng;
    int64_t base;
};

USPG_HD inline RecordRange record_range(const uint32_t *sr, const double *pa, const double *pb,
                                        const int32_t *partner, int64_t j, const int32_t *ng_of,
                                        const int64_t *head, int64_t c2d, double theta)
{
    RecordRange q;
    const int ring = ring_of(sr[j]), slice = slice_of(sr[j]);
    q.ng = ng_of[ring];
    q.pf = 0;
    q.pc = 0;
    rebin_range(q.ng, pa[j], pb[j], theta, q.first, q.count);
    const int32_t pj = partner[j];
    if (pj >= 0) rebin_range(q.ng, pa[pj], pb[pj], theta, q.pf, q.pc);
    q.base = (int64_t)slice * c2d + head[ring];
    return q;
}

// Sector number of entry q of a run, or -1 when the partner's run already
// holds it (the cells a record meets are those its partner does not).
USPG_HD inline int range_sector(const RecordRange &rr, int q)
{
    int s = rr.first + q;
    if (s >= rr.ng) s -= rr.ng;
    return rr.pc && in_range(s, rr.pf, rr.pc, rr.ng) ? -1 : s;
}

// Calls emit(cell) for every cell of entries q0, q0 + 1, ... of a run; returns
// their count.
template <class Emit>
USPG_HD int emit_range(const RecordRange &rr, int q0, Emit &emit)
{
    int m = 0;
    for (int q = q0; q < rr.count; ++q) {
        const int s = range_sector(rr, q);
        if (s < 0) continue;
        emit(rr.base + s);
        ++m;
    }
    return m;
}

// Cells of record j of a ray's row in the view of angle theta: calls
// emit(cell) for every cell the record meets that its partner does not;
// returns their count.
template <class Emit>
USPG_HD int rebin_record(const uint32_t *sr, const double *pa, const double *pb, const int32_t *partner, int64_t j,
                         const int32_t *ng_of, const int64_t *head, int64_t c2d, double theta, Emit &emit)
{
    const RecordRange rr = record_range(sr, pa, pb, partner, j, ng_of, head, c2d, theta);
    return emit_range(rr, 0, emit);
}

// Cells of one ray's re-binned row in a view (theta): calls emit(cell) for
// every distinct cell, record by record; returns the count.
template <class Emit>
USPG_HD int64_t rebin_cells(const uint32_t *sr, const double *pa, const double *pb, const int32_t *partner, int64_t n,
                            const int32_t *ng_of, const int64_t *head, int64_t c2d, double theta, Emit &emit)
{
    int64_t m = 0;
    for (int64_t j = 0; j < n; ++j) m += rebin_record(sr, pa, pb, partner, j, ng_of, head, c2d, theta, emit);
    return m;
}

}  // namespace seg
}  // namespace uspg
