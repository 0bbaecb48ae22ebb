// Test-only host build of the library's reference-ray walk
// (paper_2208_12964_amd/csrc/trace_walk.hpp), so the CPU test suite can
// compare its rows with the oracle's without a GPU.  Not part of the library.
#include <cmath>
#include <cstdint>
#include <vector>

#include "../paper_2208_12964_amd/csrc/trace_walk.hpp"

using namespace uspg::walk;

namespace {

struct State {
    std::vector<int32_t> ng, kq, hq, ring_of;
    std::vector<int64_t> head;
    std::vector<double2> cs;
    TraceGeo G{};
};

State st;

template <class TC>
struct Capture {
    std::vector<uint32_t> ids;
    std::vector<TC> a;
};

}  // namespace

extern "C" {

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

// Row of an arbitrary line from S towards D.
int hw_trace_line(const double *S, const double *D, uint32_t *ids, double *lens, int cap)
{
    Ray r;
    if (!setup_line(st.G, S, D, r)) return 0;
    return walk_row(r, ids, lens, cap);
}

}  // extern "C"
