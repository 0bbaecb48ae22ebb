// Test-only host build of the library's reference-ray walk
// (paper_2208_12964_amd/csrc/trace_walk.hpp), so the CPU test suite can
// compare its rows with the oracle's without a GPU.  Not part of the library.
#include <cmath>
#include <cstdint>
#include <vector>

#include "../paper_2208_12964_amd/csrc/coded_rows.hpp"
#include "../paper_2208_12964_amd/csrc/trace_walk.hpp"

using namespace uspg::walk;

namespace {

struct State {
    std::vector<int32_t> ng, kq, hq, ring_of;
    std::vector<int64_t> head;
    std::vector<double2> cs;
    TraceGeo G{};
    // coded rows: column records
    std::vector<int64_t> colptr;
    std::vector<double> t;
    std::vector<uint32_t> id0;
    int64_t gaps = 0;
};

State st;

template <class TC>
struct Capture {
    std::vector<uint32_t> ids;
    std::vector<TC> a;
};

}  // namespace

extern "C" {

// Ray of thread tid in the per-ray launches (column_major_ray) for a U x V
// detector.
int64_t hw_column_major(int U, int V, int64_t tid)
{
    TraceGeo G{};
    G.U = U;
    G.V = V;
    return column_major_ray(G, tid, (int64_t)U * V);
}

// Grid and scan of the walk; q = view steps per turn (must divide every ng);
// grp = rings per group of the device layout.
int hw_setup(int nr, int nz, double R, double H, const int32_t *ng, int q, int geom, int is3d, int U,
             int V, double Wu, double Wv, double Dso, double Dsd, int grp)
{
    st = State();
    st.ng.assign(ng, ng + nr);
    st.head.assign(nr + 1, 0);
    st.kq.resize(nr);
    st.hq.assign(nr + 1, 0);
    for (int i = 0; i < nr; ++i) {
        if (ng[i] % q) return -2;
        st.head[i + 1] = st.head[i] + ng[i];
    }
    int64_t cq = wedge_tables(nr, ng, q, grp, st.kq.data(), st.hq.data(), nullptr);
    st.hq[nr] = (int32_t)cq;
    st.ring_of.assign(cq, -1);
    wedge_tables(nr, ng, q, grp, st.kq.data(), st.hq.data(), st.ring_of.data());
    st.cs.resize(st.head[nr]);
    for (int i = 0; i < nr; ++i)
        for (int b = 0; b < ng[i]; ++b) st.cs[st.head[i] + b] = boundary_dir(b, ng[i]);
    TraceGeo &G = st.G;
    G.nr = nr; G.nz = nz; G.is3d = is3d; G.geom = geom;
    G.R = R; G.r = R / nr; G.H = H; G.h = nz > 1 || H > 0 ? H / nz : 0.0; G.z0 = -H / 2;
    G.ng = st.ng.data(); G.head = st.head.data(); G.cs = st.cs.data();
    G.kq = st.kq.data(); G.hq = st.hq.data();
    G.Cq = st.hq[nr]; G.Wc = (int64_t)nz * G.Cq; G.grp = grp;
    G.U = U; G.V = V; G.Wu = Wu; G.Wv = Wv; G.Dso = Dso; G.Dsd = Dsd;
    G.eps = 1e-12 * R;
    return 0;
}

// Row of a ray: counts with the counting sink, then fills; returns the count
// (both passes must agree) or -1 on mismatch, -3 if cap is small.
static int walk_row(Ray &r, uint32_t *ids, double *lens, int cap)
{
    RowSink<false, double> cnt;
    cnt.base = 0; cnt.ids = nullptr; cnt.a = nullptr; cnt.binary = false; cnt.eps = st.G.eps;
    {
        Walker<RowSink<false, double>> w(st.G, r, cnt);
        w.run();
    }
    int n = (int)cnt.count;
    if (n > cap) return -3;
    RowSink<true, double> fill;
    fill.base = 0; fill.ids = ids; fill.a = lens; fill.binary = false; fill.eps = st.G.eps;
    Walker<RowSink<true, double>> w(st.G, r, fill);
    w.run();
    return fill.count == n ? n : -1;
}

// Layout tables: kq, hq (nr entries each) and ring_of_off (Cq entries).
int64_t hw_tables(int32_t *kq, int32_t *hq, int32_t *ring_of)
{
    for (size_t i = 0; i < st.kq.size(); ++i) { kq[i] = st.kq[i]; hq[i] = st.hq[i]; }
    if (ring_of)
        for (size_t o = 0; o < st.ring_of.size(); ++o) ring_of[o] = st.ring_of[o];
    return (int64_t)st.ring_of.size();
}

int hw_trace(int64_t ray, uint32_t *ids, double *lens, int cap)
{
    Ray r;
    if (!setup_ray(st.G, ray, r)) return 0;
    return walk_row(r, ids, lens, cap);
}

// Column records of every detector column (coded rows); returns the total.
int64_t hw_columns()
{
    const int U = st.G.U;
    st.colptr.assign(U + 1, 0);
    st.gaps = 0;
    for (int u = 0; u < U; ++u) {
        uspg::coded::PieceSink cnt;
        uspg::coded::walk_column(st.G, u, cnt);
        st.colptr[u + 1] = st.colptr[u] + uspg::coded::column_records(cnt);
        st.gaps += cnt.gap;
    }
    const int64_t m = st.colptr[U];
    st.t.assign(m, 0.0);
    st.id0.assign(m, 0);
    for (int u = 0; u < U; ++u) {
        uspg::coded::PieceSink fill;
        fill.base = st.colptr[u];
        fill.t = st.t.data();
        fill.id0 = st.id0.data();
        uspg::coded::walk_column(st.G, u, fill);
        fill.close();
    }
    return m;
}

int64_t hw_column_gaps() { return st.gaps; }

// Codes ray `ray` from its FP32 stored row and rebuilds the row from the
// code alone (ids, lens: cap entries).  Returns the row length, -2 when the
// row is left explicit, -1 on a mismatch of the rebuilt row, -3 if cap is
// small.  info[0..3] = p0, kinit, planes crossed, mask words.
int hw_code_ray(int64_t ray, uint32_t *ids, float *lens, int cap, int64_t *info)
{
    using namespace uspg::coded;
    Ray r;
    if (!setup_ray(st.G, ray, r)) return 0;
    RowSink<false, float> cnt;
    cnt.base = 0; cnt.ids = nullptr; cnt.a = nullptr; cnt.binary = false; cnt.eps = st.G.eps;
    { Walker<RowSink<false, float>> w(st.G, r, cnt); w.run(); }
    const int n = (int)cnt.count;
    if (n > cap) return -3;
    std::vector<uint32_t> sid(n);
    std::vector<float> sa(n);
    RowSink<true, float> fill;
    fill.base = 0; fill.ids = sid.data(); fill.a = sa.data(); fill.binary = false; fill.eps = st.G.eps;
    { Walker<RowSink<true, float>> w(st.G, r, fill); w.run(); }
    CodeGeo Q{st.G.z0, st.G.h, st.G.nz, (uint32_t)st.G.Cq, (uint32_t)st.G.Wc};
    const int u = (int)(ray % st.G.U);
    RayCode rc{};
    std::vector<uint64_t> words(2 * ((n + 63) / 64) + 2, 0);
    auto row = [&](int e, uint32_t &id, float &a) { id = sid[e]; a = sa[e]; };
    if (!code_ray<float>(Q, st.G, r, st.t.data(), st.id0.data(), st.colptr[u], st.colptr[u + 1] - 1, row, n,
                         false, rc, words.data()))
        return -2;
    // rebuild from the code only, as the kernel does
    const int dk = code_dk(rc), kinit = code_kinit(rc), J = code_planes(rc);
    std::vector<double> bounds(J + 2);
    for (int j = 0; j <= J + 1; ++j) bounds[j] = slice_bound(Q, kinit, dk, J, rc.t0, rc.t1, rc.ez, j);
    int64_t pacc = rc.p0;
    int jacc = code_j0(rc);
    for (int e = 0; e < n; ++e) {
        if (e > 0) {
            const uint64_t pwd = words[2 * ((e - 1) >> 6)], kwd = words[2 * ((e - 1) >> 6) + 1];
            pacc += (pwd >> ((e - 1) & 63)) & 1;
            jacc += (int)((kwd >> ((e - 1) & 63)) & 1);
        }
        const int64_t p = pacc;
        ids[e] = st.id0[p] + (uint32_t)(kinit + dk * jacc) * Q.Cq;
        lens[e] = (float)entry_length(st.t[p], st.t[p + 1], bounds[jacc], bounds[jacc + 1], rc.L);
        if (ids[e] != sid[e] || !(lens[e] == sa[e])) return -1;
    }
    info[0] = rc.p0; info[1] = kinit; info[2] = J; info[3] = 2 * ((n + 63) / 64);
    return n;
}

// Row of an arbitrary line from S towards D.
int hw_trace_line(const double *S, const double *D, uint32_t *ids, double *lens, int cap)
{
    Ray r;
    if (!setup_line(st.G, S, D, r)) return 0;
    return walk_row(r, ids, lens, cap);
}

}  // extern "C"
