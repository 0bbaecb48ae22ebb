// Coded reference rows of a cone-beam scan (host / device code).
//
// The view-0 rays of one detector column u all lie in the vertical plane
// through the source and that column, so their in-plane walk (ring circles
// and radial planes, Sec. III.B, eqs. 5-16) is the same line for every
// detector row w: the rays differ only in their slope, i.e. in where the
// axial planes cut them and in the factor from ray parameter to length.  A
// coded row therefore stores no (cell, length) pairs.  It holds:
//   * per column: the in-plane path, one record per sector piece with the
//     ray parameter where it starts (FP64, exactly as the walk computes it;
//     a piece ends where the next one starts) and its cell id in slice 0 of
//     the device layout;
//   * per ray: its first piece, its first slice, its chord [t0, t1] (clipped
//     to the slab), its length factor L = |D - S| and e_z, and two bits per
//     entry: whether the entry starts the next piece and whether it starts
//     the next slice.
// Entry e of the row is piece p (first piece + number of piece bits of
// entries 1..e) in slice k (first slice + dk * (j0 + number of slice bits of
// entries 1..e), j0 = 1 when the walk dropped a first sub-piece shorter than
// eps); its length is (min(piece end, plane leaving the slice) - max(piece
// start, plane entering it)) * L, with the chord's ends t0 and t1 standing
// in for the planes before the first and after the last slice: the same
// FP64 operations as the walk, so the rebuilt (id, coefficient) equals the
// stored one bit for bit.  Rows the rule does not reproduce (the
// merged repeat of a line dipping into the next ring inside one sector, a
// piece dropped as shorter than eps in the middle of a row, degenerate
// roundings) are verified against the walk when the codes are built and
// kept as explicit stored rows.
#pragma once

#include "trace_walk.hpp"

#if defined(__clang__)
#pragma clang fp contract(off)
#endif

namespace uspg {
namespace coded {

// Largest number of axial planes a coded row may cross (the kernel keeps the
// plane parameters of a ray in LDS); rows crossing more are explicit.
constexpr int kMaxPlanes = 254;
// Longest coded row (the kernel's register path of 16 chunks of 64
// entries); longer rows are explicit.
constexpr int kMaxCodedEntries = 1024;

// Records the in-plane sector pieces of a column's line (slice 0 ids).
// Consecutive pieces of a line share their end points, so a column keeps one
// boundary array: piece p spans [t[p], t[p + 1]], and the column ends with a
// closing record (its boundary is the last piece's end, its id kNoPiece).
constexpr uint32_t kNoPiece = 0xffffffffu;

struct PieceSink {
    static constexpr bool kPieces = true;
    int64_t base = 0;   // first record of the column
    int n = 0;          // pieces so far
    bool gap = false;   // a piece did not start where the previous one ended
    double last = 0.0;  // end of the last piece
    double *t = nullptr;
    uint32_t *id0 = nullptr;   // null: count only

    USPG_HD void piece(uint32_t id, double ta, double tb)
    {
        if (!(tb > ta)) return;   // empty (a crossing clamped onto the previous one)
        if (n > 0 && ta != last) gap = true;
        if (id0) {
            t[base + n] = ta;
            id0[base + n] = id;
        }
        last = tb;
        ++n;
    }
    // the closing record (call once after the walk, also for no pieces)
    USPG_HD void close()
    {
        if (id0) {
            t[base + n] = n > 0 ? last : 0.0;
            id0[base + n] = kNoPiece;
        }
    }
    USPG_HD void hold() {}
    USPG_HD void arm() {}
    USPG_HD void finish() {}
};

// Walks the in-plane line of detector column u (view 0) into sink; false if
// the line misses the disk.
USPG_HD inline bool walk_column(const walk::TraceGeo &G3, int u, PieceSink &sink)
{
    walk::TraceGeo G = G3;
    G.is3d = 0;   // in-plane: no axial planes, slice 0 ids
    walk::Ray ray;
    if (!walk::setup_ray(G, u, ray)) return false;
    walk::Walker<PieceSink> w(G, ray, sink);
    w.run();
    return true;
}

// Records of a column: its pieces plus the closing record.
USPG_HD inline int column_records(const PieceSink &s) { return s.n + 1; }

// Per-ray header of a coded row (48 bytes).
struct RayCode {
    int32_t n;       // entries (0: the ray misses the cylinder)
    int32_t p0;      // first piece (absolute index into the column records)
    int32_t kj;      // first slice of the walk (bits 0-15), planes crossed J (16-27), j0 (28)
    int32_t word;    // >= 0: first mask word; < 0: explicit row
    double t0, t1;   // chord of the ray (slab-clipped)
    double L;        // |D - S|: length per unit of ray parameter
    double ez;       // z component of D - S
};

// Uniform geometry of the decoding.
struct CodeGeo {
    double z0, h;
    int nz;
    uint32_t Cq, Wc;
};

USPG_HD inline int code_kinit(const RayCode &c) { return c.kj & 0xffff; }
USPG_HD inline int code_planes(const RayCode &c) { return (c.kj >> 16) & 0xfff; }
USPG_HD inline int code_j0(const RayCode &c) { return (c.kj >> 28) & 1; }
USPG_HD inline int code_dk(const RayCode &c) { return c.ez > 0 ? 1 : (c.ez < 0 ? -1 : 0); }

// Parameter of the j-th axial plane (j >= 1) met by a ray that starts in
// slice kinit and moves by dk: the walk's next_plane for slice
// kinit + (j - 1) dk, same operations (+inf past the cylinder's planes).
USPG_HD inline double plane_t(const CodeGeo &Q, int kinit, int dk, int j, double ez)
{
    const int kk = dk > 0 ? kinit + j : kinit - j + 1;
    if (dk == 0 || kk <= 0 || kk >= Q.nz) return INFINITY;
    return (Q.z0 + kk * Q.h - 0.0) / ez;
}

// Bound j (0 .. J + 1) of the slices of a coded ray crossing J planes:
// t0 in front of the first slice, the crossed planes, and after the last
// slice the next plane or t1, whichever comes first.
USPG_HD inline double slice_bound(const CodeGeo &Q, int kinit, int dk, int J, double t0, double t1, double ez, int j)
{
    if (j == 0) return t0;
    double v = plane_t(Q, kinit, dk, j, ez);
    if (j == J + 1) v = v < t1 ? v : t1;
    return v;
}

// Length of an entry: piece [tp, tp1] between slice bounds [be, bl], times L.
USPG_HD inline double entry_length(double tp, double tp1, double be, double bl, double L)
{
    const double lo = tp > be ? tp : be;
    const double hi = tp1 < bl ? tp1 : bl;
    return (hi - lo) * L;
}

// Slice of a device-layout id (view 0).
USPG_HD inline int id_slice(const CodeGeo &Q, uint32_t id) { return (int)((id % Q.Wc) / Q.Cq); }

// Builds the code of one ray from its stored row (row(e, id, a) gives entry
// e of n) and the records of its column ([pb, pe), pe the closing record):
// sets rc (except word) and, when words is not null, writes the
// 2 * ceil(n / 64) mask words: per chunk of 64 entries a word of piece bits
// and a word of slice bits, bit i of chunk k's words belonging to entry
// 64 k + i + 1 (the first entry has none: it starts at p0 and j0).  Returns
// false when the rule does not reproduce the row bit for bit (the ray stays
// explicit).
template <class TC, class Row>
USPG_HD bool code_ray(const CodeGeo &Q, const walk::TraceGeo &G, const walk::Ray &ray, const double *t,
                      const uint32_t *id0, int64_t pb, int64_t pe, const Row &row, int n, bool binary,
                      RayCode &rc, uint64_t *words)
{
    rc.n = n;
    rc.t0 = ray.t0;
    rc.t1 = ray.t1;
    rc.L = ray.L;
    rc.ez = ray.e[2];
    rc.p0 = 0;
    rc.kj = 0;
    if (n == 0) return true;
    if (n > kMaxCodedEntries) return false;
    // first slice of the walk (Walker::init_slices)
    const double zs = ray.S[2] + ray.t0 * ray.e[2];
    int kinit = (int)floor((zs - G.z0) / G.h);
    kinit = kinit < 0 ? 0 : (kinit >= G.nz ? G.nz - 1 : kinit);
    const int dk = ray.e[2] > 0 ? 1 : (ray.e[2] < 0 ? -1 : 0);
    if (kinit >= (1 << 16)) return false;
    uint32_t id;
    TC a;
    // first piece: the first record of the column with the first entry's
    // in-plane cell that reaches past t0
    row(0, id, a);
    const uint32_t c0 = id - (uint32_t)id_slice(Q, id) * Q.Cq;
    int64_t p0 = -1;
    for (int64_t q = pb; q < pe; ++q)
        if (id0[q] == c0 && t[q + 1] > ray.t0) { p0 = q; break; }
    if (p0 < 0 || p0 >= ((int64_t)1 << 31)) return false;
    // pass 1: the (piece, slice) of every entry, checked for steps of 0 or
    // 1; J = planes crossed.  Pass 2: the rebuilt entries against the row.
    int J = 0, j0 = 0;
    for (int pass = 0; pass < 2; ++pass) {
        int jprev = 0;
        int64_t pprev = p0;
        uint64_t pw = 0, kw = 0;
        for (int e = 0; e < n; ++e) {
            row(e, id, a);
            const int k = id_slice(Q, id);
            const uint32_t c = id - (uint32_t)k * Q.Cq;
            const int j = (k - kinit) * dk;
            if (dk == 0 ? k != kinit : j < 0) return false;
            int64_t pc = pprev;
            if (e > 0) {
                if (j - jprev < 0 || j - jprev > 1) return false;
                if (id0[pprev] == c && j == jprev + 1) pc = pprev;               // same piece, next slice
                else if (pprev + 1 < pe && id0[pprev + 1] == c) pc = pprev + 1;   // next piece
                else return false;
            } else {
                // the walk may drop a first sub-piece shorter than eps (a
                // plane right at t0): the first entry is then one plane in
                if (j > 1) return false;
                j0 = j;
            }
            if (pass == 1) {
                const double be = slice_bound(Q, kinit, dk, J, ray.t0, ray.t1, ray.e[2], j);
                const double bl = slice_bound(Q, kinit, dk, J, ray.t0, ray.t1, ray.e[2], j + 1);
                const TC av = binary ? TC(1) : TC(entry_length(t[pc], t[pc + 1], be, bl, ray.L));
                if (!(av == a) || id0[pc] + (uint32_t)k * Q.Cq != id) return false;
                if (e > 0) {
                    const int l = (e - 1) & 63;
                    pw |= (uint64_t)(pc - pprev) << l;
                    kw |= (uint64_t)(j - jprev) << l;
                    if (l == 63 || e == n - 1) {
                        if (words) {
                            words[2 * ((e - 1) >> 6)] = pw;
                            words[2 * ((e - 1) >> 6) + 1] = kw;
                        }
                        pw = kw = 0;
                    }
                }
            }
            pprev = pc;
            jprev = j;
        }
        J = jprev;
        if (J + 1 > kMaxPlanes) return false;
    }
    if (words && n % 64 == 1) {   // the last chunk holds only entry n - 1 = 64 k: its words are empty
        words[2 * ((n - 1) >> 6)] = 0;
        words[2 * ((n - 1) >> 6) + 1] = 0;
    }
    rc.p0 = (int32_t)p0;
    rc.kj = kinit | (J << 16) | (j0 << 28);
    return true;
}

}  // namespace coded
}  // namespace uspg
