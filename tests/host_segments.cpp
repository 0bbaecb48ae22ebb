// Test-only host build of the library's segment records and per-view
// re-binning (paper_2208_12964_amd/csrc/segments.hpp), so the CPU test suite
// can compare them with the oracle's without a GPU.  Not part of the library.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <vector>

#include "../paper_2208_12964_amd/csrc/segments.hpp"

using namespace uspg;

namespace {

struct State {
    std::vector<int32_t> ng;
    std::vector<int64_t> head;
    walk::TraceGeo G{};
    double span = 0;
    int p = 1;
};

State st;

}  // namespace

extern "C" {

int hs_setup(int nr, int nz, double R, double H, const int32_t *ng, int geom, int is3d, int U, int V, double Wu,
             double Wv, double Dso, double Dsd, double span, int p)
{
    st = State();
    st.ng.assign(ng, ng + nr);
    st.head.assign(nr + 1, 0);
    for (int i = 0; i < nr; ++i) st.head[i + 1] = st.head[i] + ng[i];
    walk::TraceGeo &G = st.G;
    G.nr = nr; G.nz = nz; G.is3d = is3d; G.geom = geom;
    G.R = R; G.r = R / nr; G.H = H; G.h = nz > 1 || H > 0 ? H / nz : 0.0; G.z0 = -H / 2;
    G.ng = st.ng.data(); G.head = st.head.data();
    G.U = U; G.V = V; G.Wu = Wu; G.Wv = Wv; G.Dso = Dso; G.Dsd = Dsd;
    G.eps = 1e-12 * R;
    st.span = span;
    st.p = p;
    return 0;
}

// Records of one view-0 ray: returns the count (count and fill passes must
// agree, else -1; -3 if cap is small).
int hs_segments(int64_t ray, int32_t *slice, int32_t *ring, double *pa, double *pb, int32_t *partner, int cap)
{
    seg::CountSink cs;
    int n = seg::segments_of_ray(st.G, ray, cs);
    if (n > cap) return -3;
    std::vector<uint32_t> sr(n > 0 ? n : 1);
    seg::FillSink fs{sr.data(), pa, pb, partner, 0};
    int m = seg::segments_of_ray(st.G, ray, fs);
    if (m != n) return -1;
    for (int j = 0; j < n; ++j) {
        slice[j] = seg::slice_of(sr[j]);
        ring[j] = seg::ring_of(sr[j]);
    }
    return n;
}

// Records of ray `ray` obtained as the library's quarter tracing does: the
// quadrant ray's records mirrored (returns the count, or -3 if cap is small).
int hs_segments_mirrored(int64_t ray, int32_t *slice, int32_t *ring, double *pa, double *pb, int32_t *partner,
                         int cap)
{
    const int U = st.G.U, V = st.G.V;
    const int u = (int)(ray % U), w = (int)(ray / U);
    const int uq = u < U - 1 - u ? u : U - 1 - u, wq = w < V - 1 - w ? w : V - 1 - w;
    const bool my = uq != u, mz = wq != w;
    int n = hs_segments((int64_t)wq * U + uq, slice, ring, pa, pb, partner, cap);
    if (n < 0) return n;
    for (int j = 0; j < n; ++j) {
        uint32_t sr = seg::pack(slice[j], ring[j]);
        seg::mirror_record(my, mz, st.G.nz, sr, pa[j], pb[j]);
        slice[j] = seg::slice_of(sr);
        ring[j] = seg::ring_of(sr);
    }
    return n;
}

// Re-binned row (cells ascending) of one ray in one view.
int hs_row(int view, int64_t ray, int64_t *cells, int cap)
{
    seg::CountSink cs;
    int n = seg::segments_of_ray(st.G, ray, cs);
    std::vector<uint32_t> sr(n > 0 ? n : 1);
    std::vector<double> pa(n > 0 ? n : 1), pb(n > 0 ? n : 1);
    std::vector<int32_t> partner(n > 0 ? n : 1);
    seg::FillSink fs{sr.data(), pa.data(), pb.data(), partner.data(), 0};
    seg::segments_of_ray(st.G, ray, fs);
    std::vector<int64_t> out;
    auto emit = [&out](int64_t c) { out.push_back(c); };
    seg::rebin_cells(sr.data(), pa.data(), pb.data(), partner.data(), n, st.ng.data(), st.head.data(),
                     st.head[st.G.nr], seg::view_angle(view, st.span, st.p), emit);
    std::sort(out.begin(), out.end());
    if ((int)out.size() > cap) return -3;
    for (size_t j = 0; j < out.size(); ++j) cells[j] = out[j];
    // distinct cells only
    for (size_t j = 1; j < out.size(); ++j)
        if (out[j] == out[j - 1]) return -2;
    return (int)out.size();
}

}  // extern "C"
