// Many independent reconstructions run together.
//
// Two modes.  LOCKSTEP (the default): launch t performs step t -- one (view,
// colour class) batch -- of every problem at once, each problem with as many
// workgroups as its largest class needs (one ray per wavefront); problems
// that have finished skip out.  Kernel boundaries order the steps, so no
// cross-workgroup synchronisation is needed inside a launch and every
// problem gets the whole machine's worth of parallelism.  PERSISTENT: one
// workgroup owns one problem (a 2D slice or a small volume) for the whole
// solve: it walks sweeps > views > colour classes and, for each class, spreads
// the class's rays over its wavefronts (one ray per wavefront, the same per-ray
// routine as the single-problem kernel), with a workgroup barrier between
// classes.  A problem whose device-layout image fits the workgroup's LDS keeps
// the image there for the whole solve (loaded once, written back once);
// larger ones work on their image in global memory (L2-resident for these
// sizes).  The per-problem pointers travel in the kernel arguments, so a run
// needs no host-to-device copies; the static part of each problem (its
// reference rows and layout constants) is uploaded once when the batch is
// built.  The autotuner times the workgroup size (the number of rays of a
// class in flight per problem) and the LDS choice on scratch copies of the
// images; neither changes the arithmetic, so every setting gives the same
// bits, equal to running the problems one at a time.
#include <algorithm>
#include <cstddef>
#include <vector>

#include "mart_coded.hpp"
#include "mart_row.hpp"
#include "uspg_internal.hpp"

struct uspg_batch {
    int n = 0, dtype = USPG_F32, device = 0;
    std::vector<const uspg_coeffs *> co;
    uspg::DevBuf d_static;
    int mode = 1;                 // 0 persistent, 1 lockstep
    int block = 256;              // threads per workgroup
    int use_lds = 1;              // allow LDS-resident images
    size_t lds_limit = 0;         // bytes of dynamic LDS a workgroup may use
    size_t lds_bytes = 0;         // dynamic LDS of the launch
    int maxc = 16;
    bool any_kept = false;        // some problem runs kept per-view rows
    bool any_coded = false;       // some problem has coded rows
    bool nt = true;               // lockstep coefficient loads with the non-temporal hint
    std::vector<int> lds_mode;    // per problem
    // lockstep
    uspg::DevBuf d_dyn, d_wgbeg;  // per-problem run arguments, workgroup prefix
    std::vector<int> wgbeg;       // n + 1 entries
    void *h_dyn = nullptr;        // pinned staging for d_dyn
    hipEvent_t dyn_copied = nullptr;
    // lockstep groups: problems [grp_first[g], grp_first[g + 1]) run from
    // step grp_step[g] to grp_step[g + 1] (one group unless their working
    // sets outgrow the last-level cache together)
    std::vector<int> grp_first, grp_step;
    // the lockstep launch sequence captured as one graph
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
    int g_steps = -1, g_block = -1, g_nt = -1;
    std::vector<int> g_first, g_step;   // the groups it was captured for
};

namespace uspg {

// The codes of a coefficient set for the batch kernels (mart.hip).
batchk::CodeTab code_tab(const uspg_coeffs *c);

namespace {

using row::mart_row;

constexpr int kMaxBatch = 96;     // problems per launch (kernel-argument space)

struct ProblemStatic {
    const int64_t *rowptr;
    const void *coef;     // Coef<TC> pairs
    int64_t nrays;
    uint32_t Wc, Wtot;
    int U, Ku, Kv, n_views, lds;
    const int64_t *view_start;  // kept per-view rows: first entry of each view; null: shifted reference rows
    batchk::CodeTab K;          // coded rows (K.codes null: none)
};

// Row forms of a lockstep launch: stored shifted rows only, some kept
// per-view rows, or some coded rows (read through the codes; the other
// problems' stored rows as usual).
constexpr int kRowsStored = 0, kRowsKept = 1, kRowsCoded = 2;

// Class rows per band of the ray order for coded problems (as in the
// single-problem coded kernel).
constexpr int kLockstepBand = 8;

// Lockstep groups: bytes of image lines per entry of a class, and the
// per-step budget of a group (of the 256 MB last-level cache).
constexpr double kLineBytesPerEntry = 9.0;
constexpr double kStepCacheBytes = 200e6;

// The codes of a coefficient set and the projections are read-only while
// MART kernels run.  Read through the constant address space, a
// wavefront-uniform ray header, its bit words and its measurement load into
// scalar registers (mart_coded gets the same from restrict-qualified
// arguments; here the pointers come from the problem table): 83 -> 65
// vector registers for the 8-chunk body.
typedef const __attribute__((address_space(4))) uint64_t ConstU64;
typedef const __attribute__((address_space(4))) int32_t ConstI32;
typedef const __attribute__((address_space(4))) double ConstF64;

static_assert(sizeof(coded::RayCode) == 48 && offsetof(coded::RayCode, t0) == 16 &&
                  offsetof(coded::RayCode, ez) == 40,
              "code_of reads the header as four int32 then four doubles");

__device__ __forceinline__ coded::RayCode code_of(const coded::RayCode *codes, int64_t r)
{
    const coded::RayCode *g = codes + r;
    ConstI32 *i = (ConstI32 *)g;
    ConstF64 *d = (ConstF64 *)&g->t0;
    coded::RayCode rc;
    rc.n = i[0];
    rc.p0 = i[1];
    rc.kj = i[2];
    rc.word = i[3];
    rc.t0 = d[0];
    rc.t1 = d[1];
    rc.L = d[2];
    rc.ez = d[3];
    return rc;
}

// Rows of view v: the reference rows with the cell ids shifted by v Wc
// (v < n_views <= q, so v Wc < Wtot), or the view's own kept rows (no
// shift).  Row pointers first, so that an empty row costs nothing more.
// KEPT = false: no problem of the launch has kept rows, and the kernels
// compile without the per-problem test.
template <bool KEPT>
__device__ inline const int64_t *view_rowptr(const ProblemStatic &S, int v)
{
    if constexpr (!KEPT) return S.rowptr;
    return S.view_start ? S.rowptr + (int64_t)v * (S.nrays + 1) : S.rowptr;
}

template <class TC, bool KEPT>
__device__ inline const Coef<TC> *view_coef(const ProblemStatic &S, int v, uint32_t &shift)
{
    const Coef<TC> *base = static_cast<const Coef<TC> *>(S.coef);
    if constexpr (!KEPT) {
        shift = (uint32_t)(((uint64_t)v * S.Wc) % S.Wtot);
        return base;
    }
    shift = S.view_start ? 0u : (uint32_t)v * S.Wc;
    return S.view_start ? base + S.view_start[v] : base;
}

template <class T>
struct ProblemDyn {
    const T *P;
    T *f;                 // device-layout image (caller's work buffer)
    int sweeps;
    int offset;           // lockstep: global step at which the problem starts
    T beta;
};

template <class T>
struct MultiArgs {
    const ProblemStatic *st;
    int first;            // index of the first problem of this launch
    ProblemDyn<T> dyn[kMaxBatch];
};

template <class T, class TC, int MAXC, bool KEPT>
__global__ void mart_multi(MultiArgs<T> A)
{
    extern __shared__ unsigned char smem[];
    T *lds = reinterpret_cast<T *>(smem);
    const ProblemStatic S = A.st[A.first + blockIdx.x];
    const ProblemDyn<T> D = A.dyn[blockIdx.x];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nwaves = blockDim.x >> 6;
    if (S.lds) {
        for (uint32_t i = threadIdx.x; i < S.Wtot; i += blockDim.x) lds[i] = D.f[i];
        __syncthreads();
    }
    const int K = S.Ku * S.Kv;
    for (int sw = 0; sw < D.sweeps; ++sw) {
        for (int v = 0; v < S.n_views; ++v) {
            const int64_t *rp = view_rowptr<KEPT>(S, v);
            uint32_t shift;
            const Coef<TC> *co = view_coef<TC, KEPT>(S, v, shift);
            const T *Pv = D.P + (int64_t)v * S.nrays;
            for (int c = 0; c < K; ++c) {
                const int cu = c % S.Ku, cw = c / S.Ku;
                const int nu = (S.U - cu + S.Ku - 1) / S.Ku;
                const int nw = ((int)(S.nrays / S.U) - cw + S.Kv - 1) / S.Kv;
                const int ncls = nu * nw;
                for (int x = wave; x < ncls; x += nwaves) {
                    const int64_t r = (int64_t)(cw + (x / nu) * S.Kv) * S.U + cu + (x % nu) * S.Ku;
                    const int64_t beg = rp[r];
                    const int n = (int)(rp[r + 1] - beg);
                    if (n == 0) continue;
                    if (S.lds)
                        mart_row<T, TC, MAXC>(lds, shift, S.Wtot, D.beta, co + beg, n, Pv[r], lane);
                    else
                        mart_row<T, TC, MAXC>(D.f, shift, S.Wtot, D.beta, co + beg, n, Pv[r], lane);
                }
                __syncthreads();
            }
        }
    }
    if (S.lds) {
        for (uint32_t i = threadIdx.x; i < S.Wtot; i += blockDim.x) D.f[i] = lds[i];
    }
}

// Step `step` of every problem: workgroup b belongs to the problem whose
// prefix range holds it; its wavefronts take that problem's rays of the
// current (view, class) in order.  (Capping this grid and striding, as the
// single-problem batch kernel does, made it 6-42 % slower.)
template <class T, class TC, int MAXC, int ROWS, bool NT>
__global__ __launch_bounds__(256) void mart_lockstep(const ProblemStatic *st, const ProblemDyn<T> *dyn,
                                                     const int *wgbeg, int n, int step, int wg0)
{
    constexpr bool KEPT = ROWS == kRowsKept;
    // slice bounds of a coded ray, one table per wavefront (at most 4)
    __shared__ double planes[ROWS == kRowsCoded ? 4 : 1][ROWS == kRowsCoded ? coded::kMaxPlanes + 2 : 1];
    // each XCD takes a contiguous run of the virtual workgroups, as in the
    // single-problem kernel; the launch covers the workgroups from wg0 on
    const int b = wg0 + row::xcd_block(blockIdx.x, gridDim.x);
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (wgbeg[mid] <= b) lo = mid;
        else hi = mid - 1;
    }
    const ProblemStatic S = st[lo];
    const ProblemDyn<T> D = dyn[lo];
    const int K = S.Ku * S.Kv;
    const int local = step - D.offset;
    if (local < 0 || local >= D.sweeps * S.n_views * K) return;
    const int c = local % K;
    const int v = (local / K) % S.n_views;
    const int cu = c % S.Ku, cw = c / S.Ku;
    const int nu = (S.U - cu + S.Ku - 1) / S.Ku;
    const int nw = ((int)(S.nrays / S.U) - cw + S.Kv - 1) / S.Kv;
    const int x = __builtin_amdgcn_readfirstlane((b - wgbeg[lo]) * (blockDim.x >> 6) + (threadIdx.x >> 6));
    if (x >= nu * nw) return;
    int64_t r = (int64_t)(cw + (x / nu) * S.Kv) * S.U + cu + (x % nu) * S.Ku;
    if constexpr (ROWS == kRowsCoded) {
        if (S.K.codes) {
            // the coded kernel's band order (bands of kLockstepBand class
            // rows, w fastest), so that rays in flight share their columns'
            // in-plane paths; rays of one class are independent, so the
            // order leaves the bits alone
            const int wb = x / (kLockstepBand * nu);
            const int xl = x - wb * kLockstepBand * nu;
            const int h = nw - wb * kLockstepBand < kLockstepBand ? nw - wb * kLockstepBand : kLockstepBand;
            r = (int64_t)(cw + (wb * kLockstepBand + xl % h) * S.Kv) * S.U + cu + (xl / h) * S.Ku;
            const coded::RayCode rc = code_of(S.K.codes, r);
            if (rc.n == 0) return;
            if (rc.word >= 0) {   // rebuilt from the codes (same entries, same bits)
                const uint32_t shift = (uint32_t)(((uint64_t)v * S.Wc) % S.Wtot);
                const T P = ((const __attribute__((address_space(4))) T *)D.P)[(int64_t)v * S.nrays + r];
                batchk::coded_row_any<T, TC, MAXC>(S.K, (const ConstU64 *)S.K.words, D.f, shift, S.Wtot, D.beta, rc,
                                                   P, threadIdx.x & 63, planes[threadIdx.x >> 6]);
                return;
            }
        }
    }
    const int64_t *rp = view_rowptr<KEPT>(S, v);
    const int64_t beg = rp[r];
    const int len = (int)(rp[r + 1] - beg);
    if (len == 0) return;
    uint32_t shift;
    const Coef<TC> *co = view_coef<TC, KEPT>(S, v, shift);
    mart_row<T, TC, MAXC, NT>(D.f, shift, S.Wtot, D.beta, co + beg, len, D.P[(int64_t)v * S.nrays + r],
                              threadIdx.x & 63);
}

// The step sequence is captured once into a graph (per step count and launch
// shape) and replayed with one graph launch; the run arguments it reads live
// in d_dyn, refreshed before every replay.
template <class T, class TC, int MAXC, int ROWS, bool NT>
int lockstep_typed(uspg_batch *b, int steps, hipStream_t s)
{
    if (!b->gexec || b->g_steps != steps || b->g_block != b->block || b->g_nt != (int)NT ||
        b->g_first != b->grp_first || b->g_step != b->grp_step) {
        if (b->gexec) (void)hipGraphExecDestroy(b->gexec);
        if (b->graph) (void)hipGraphDestroy(b->graph);
        b->gexec = nullptr;
        b->graph = nullptr;
        hipStream_t cs;
        USPG_HIP(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
        int rc = USPG_OK;
        if (hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) != hipSuccess) {
            rc = fail(USPG_E_HIP, "hipStreamBeginCapture failed");
        } else {
            // step t launches the workgroups of its group's problems only
            size_t g = 0;
            for (int t = 0; t < steps; ++t) {
                while (g + 2 < b->grp_step.size() && t >= b->grp_step[g + 1]) ++g;
                const int w0 = b->wgbeg[b->grp_first[g]], w1 = b->wgbeg[b->grp_first[g + 1]];
                hipLaunchKernelGGL((mart_lockstep<T, TC, MAXC, ROWS, NT>), dim3(w1 - w0), dim3(b->block), 0, cs,
                                   b->d_static.as<ProblemStatic>(), b->d_dyn.as<ProblemDyn<T>>(),
                                   b->d_wgbeg.as<int>(), b->n, t, w0);
            }
            if (hipStreamEndCapture(cs, &b->graph) != hipSuccess ||
                hipGraphInstantiate(&b->gexec, b->graph, nullptr, nullptr, 0) != hipSuccess)
                rc = fail(USPG_E_HIP, "capturing the lockstep graph failed");
        }
        (void)hipStreamDestroy(cs);
        if (rc != USPG_OK) return rc;
        b->g_steps = steps;
        b->g_block = b->block;
        b->g_nt = (int)NT;
        b->g_first = b->grp_first;
        b->g_step = b->grp_step;
    }
    USPG_HIP(hipGraphLaunch(b->gexec, s));
    return USPG_OK;
}

template <class T, class TC, int ROWS, bool NT>
int lockstep_chunks(uspg_batch *b, int steps, hipStream_t s)
{
    if (b->maxc <= 2) return lockstep_typed<T, TC, 2, ROWS, NT>(b, steps, s);
    if (b->maxc <= 4) return lockstep_typed<T, TC, 4, ROWS, NT>(b, steps, s);
    if (b->maxc <= 8) return lockstep_typed<T, TC, 8, ROWS, NT>(b, steps, s);
    return lockstep_typed<T, TC, 16, ROWS, NT>(b, steps, s);
}

template <class T, class TC>
int lockstep_maxc(uspg_batch *b, int steps, hipStream_t s)
{
    if (b->any_kept)
        return b->nt ? lockstep_chunks<T, TC, kRowsKept, true>(b, steps, s)
                     : lockstep_chunks<T, TC, kRowsKept, false>(b, steps, s);
    if (b->any_coded)
        return b->nt ? lockstep_chunks<T, TC, kRowsCoded, true>(b, steps, s)
                     : lockstep_chunks<T, TC, kRowsCoded, false>(b, steps, s);
    return b->nt ? lockstep_chunks<T, TC, kRowsStored, true>(b, steps, s)
                 : lockstep_chunks<T, TC, kRowsStored, false>(b, steps, s);
}

template <class T, class TC, int MAXC, bool KEPT>
int launch_typed(const uspg_batch *b, MultiArgs<T> &A, int count, hipStream_t s)
{
    auto k = mart_multi<T, TC, MAXC, KEPT>;
    if (b->lds_bytes > 65536)
        USPG_HIP(hipFuncSetAttribute((const void *)k, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)b->lds_bytes));
    hipLaunchKernelGGL(k, dim3(count), dim3(b->block), b->lds_bytes, s, A);
    USPG_HIP(hipGetLastError());
    return USPG_OK;
}

template <class T, class TC>
int launch_maxc(const uspg_batch *b, MultiArgs<T> &A, int count, hipStream_t s)
{
    if (b->any_kept) {
        if (b->maxc <= 2) return launch_typed<T, TC, 2, true>(b, A, count, s);
        if (b->maxc <= 4) return launch_typed<T, TC, 4, true>(b, A, count, s);
        if (b->maxc <= 8) return launch_typed<T, TC, 8, true>(b, A, count, s);
        return launch_typed<T, TC, 16, true>(b, A, count, s);
    }
    if (b->maxc <= 2) return launch_typed<T, TC, 2, false>(b, A, count, s);
    if (b->maxc <= 4) return launch_typed<T, TC, 4, false>(b, A, count, s);
    if (b->maxc <= 8) return launch_typed<T, TC, 8, false>(b, A, count, s);
    return launch_typed<T, TC, 16, false>(b, A, count, s);
}

// Solve on device-layout images (already permuted into work[i]).
template <class T>
int solve_native(const uspg_batch *b, const void *const *proj, void *const *work, const int32_t *n_sweeps,
                 const double *beta, hipStream_t s)
{
    MultiArgs<T> A;
    A.st = b->d_static.as<ProblemStatic>();
    for (int first = 0; first < b->n; first += kMaxBatch) {
        const int count = std::min(kMaxBatch, b->n - first);
        A.first = first;
        for (int j = 0; j < count; ++j) {
            A.dyn[j].P = static_cast<const T *>(proj[first + j]);
            A.dyn[j].f = static_cast<T *>(work[first + j]);
            A.dyn[j].sweeps = n_sweeps[first + j];
            A.dyn[j].offset = 0;
            A.dyn[j].beta = (T)beta[first + j];
        }
        const bool cf64 = stored_coeff_dtype(b->co[0]) == USPG_F64;
        int rc = cf64 ? launch_maxc<T, double>(b, A, count, s) : launch_maxc<T, float>(b, A, count, s);
        if (rc != USPG_OK) return rc;
    }
    return USPG_OK;
}

template <class T>
int solve_lockstep(uspg_batch *b, const void *const *proj, void *const *work, const int32_t *n_sweeps,
                   const double *beta, hipStream_t s)
{
    // the staging buffer may still feed the previous run's copy
    USPG_HIP(hipEventSynchronize(b->dyn_copied));
    auto *dyn = static_cast<ProblemDyn<T> *>(b->h_dyn);
    // Problems in order, in groups whose image lines touched per step fit
    // the last-level cache together (about 9 bytes per entry of a class:
    // 128-byte lines holding some 14 of its entries); each group starts at
    // the step the previous one ends.  Measured: sixteen 128-ring cone
    // problems in one group ran 2.7x slower per step than eight.
    b->grp_first.assign(1, 0);
    b->grp_step.assign(1, 0);
    double bytes = 0;
    int start = 0, steps = 0;
    for (int i = 0; i < b->n; ++i) {
        const uspg_coeffs *c = b->co[i];
        const double step_bytes = kLineBytesPerEntry * (double)c->nnz / (double)(c->Ku * c->Kv);
        if (i > 0 && bytes > 0 && bytes + step_bytes > kStepCacheBytes) {
            start = steps;
            b->grp_first.push_back(i);
            b->grp_step.push_back(start);
            bytes = 0;
        }
        bytes += step_bytes;
        dyn[i].P = static_cast<const T *>(proj[i]);
        dyn[i].f = static_cast<T *>(work[i]);
        dyn[i].sweeps = n_sweeps[i];
        dyn[i].offset = start;
        dyn[i].beta = (T)beta[i];
        steps = std::max(steps, start + n_sweeps[i] * c->scan.n_views * c->Ku * c->Kv);
    }
    b->grp_first.push_back(b->n);
    b->grp_step.push_back(steps);
    USPG_HIP(hipMemcpyAsync(b->d_dyn.p, dyn, sizeof(ProblemDyn<T>) * b->n, hipMemcpyHostToDevice, s));
    USPG_HIP(hipEventRecord(b->dyn_copied, s));
    const bool cf64 = stored_coeff_dtype(b->co[0]) == USPG_F64;
    return cf64 ? lockstep_maxc<T, double>(b, steps, s) : lockstep_maxc<T, float>(b, steps, s);
}

int solve(uspg_batch *b, const void *const *proj, void *const *work, const int32_t *n_sweeps,
          const double *beta, hipStream_t s)
{
    if (b->mode == 1) {
        if (b->dtype == USPG_F64) return solve_lockstep<double>(b, proj, work, n_sweeps, beta, s);
        return solve_lockstep<float>(b, proj, work, n_sweeps, beta, s);
    }
    if (b->dtype == USPG_F64) return solve_native<double>(b, proj, work, n_sweeps, beta, s);
    return solve_native<float>(b, proj, work, n_sweeps, beta, s);
}

ProblemStatic static_of(const uspg_coeffs *c)
{
    ProblemStatic p;
    const bool kept = kept_rows(c);
    p.rowptr = kept ? c->view_rowptr.as<int64_t>() : c->rowptr.as<int64_t>();
    p.coef = kept ? c->view_coef.p : c->coef.p;
    p.view_start = kept ? c->d_view_start.as<int64_t>() : nullptr;
    p.nrays = c->nrays;
    p.Wc = (uint32_t)c->Wc;
    p.Wtot = (uint32_t)solve_cells(c);
    p.U = c->scan.det_u;
    p.Ku = c->Ku;
    p.Kv = c->Kv;
    p.n_views = c->scan.n_views;
    p.lds = 0;
    p.K = kept ? batchk::CodeTab{} : code_tab(c);
    return p;
}

// Workgroups of 4 wavefronts that cover a problem's largest class.
int lockstep_groups(const uspg_coeffs *c, int waves)
{
    const int64_t nu0 = (c->scan.det_u + c->Ku - 1) / c->Ku, nw0 = (c->scan.det_v + c->Kv - 1) / c->Kv;
    return (int)((nu0 * nw0 + waves - 1) / waves);
}

// Upload the static descriptors for the current LDS setting.
int upload_static(uspg_batch *b)
{
    const size_t tsz = b->dtype == USPG_F64 ? sizeof(double) : sizeof(float);
    std::vector<ProblemStatic> st(b->n);
    b->lds_bytes = 0;
    b->any_kept = false;
    b->any_coded = false;
    b->lds_mode.assign(b->n, 0);
    int maxrow = 0;
    for (int i = 0; i < b->n; ++i) {
        const uspg_coeffs *c = b->co[i];
        ProblemStatic &p = st[i];
        p = static_of(c);
        const size_t need = (size_t)solve_cells(c) * tsz;
        p.lds = b->use_lds && need <= b->lds_limit;
        b->lds_mode[i] = p.lds;
        if (p.lds) b->lds_bytes = std::max(b->lds_bytes, need);
        maxrow = std::max(maxrow, (int)stored_max_row(c));
        b->any_kept = b->any_kept || kept_rows(c);
        b->any_coded = b->any_coded || c->coded;
    }
    b->maxc = (maxrow + 63) / 64;
    // lockstep coefficient loads: non-temporal unless every coefficient set
    // (each counted once) and image of the batch fit the last-level cache
    {
        std::vector<const uspg_coeffs *> sets;
        size_t coef_bytes = 0, image_bytes = 0;
        for (int i = 0; i < b->n; ++i) {
            const uspg_coeffs *c = b->co[i];
            if (std::find(sets.begin(), sets.end(), c) == sets.end()) {
                sets.push_back(c);
                coef_bytes += coef_set_bytes(c);
            }
            image_bytes += (size_t)solve_cells(c) * tsz;
        }
        b->nt = stream_coefs(coef_bytes, image_bytes);
    }
    // lockstep: enough workgroups for each problem's largest class
    const int waves = b->block / 64;
    b->wgbeg.assign(b->n + 1, 0);
    for (int i = 0; i < b->n; ++i) b->wgbeg[i + 1] = b->wgbeg[i] + lockstep_groups(b->co[i], waves);
    if (hipMemcpy(b->d_static.p, st.data(), sizeof(ProblemStatic) * b->n, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(b->d_wgbeg.p, b->wgbeg.data(), sizeof(int) * (b->n + 1), hipMemcpyHostToDevice) != hipSuccess)
        return fail(USPG_E_HIP, "uploading batch descriptors failed");
    return USPG_OK;
}

int check_runs(const uspg_batch *b, const void *const *proj, void *const *image, void *const *work,
               const size_t *work_bytes, const int32_t *n_sweeps, const double *beta)
{
    if (!proj || !image || !work || !work_bytes || !n_sweeps || !beta) return fail(USPG_E_ARG, "null argument");
    for (int i = 0; i < b->n; ++i) {
        if (!proj[i] || !image[i] || !work[i]) return fail(USPG_E_ARG, "null buffer in batch");
        if (n_sweeps[i] < 0 || !(beta[i] > 0)) return fail(USPG_E_ARG, "n_sweeps >= 0 and beta > 0");
        if (work_bytes[i] < uspg_mart_workspace_bytes(b->co[i], b->dtype, 0.0))
            return fail(USPG_E_NOMEM, "work space too small");
    }
    return USPG_OK;
}

}  // namespace
}  // namespace uspg

// Continuous-batching engine: slots hold admitted problems; every step call
// advances all active slots through the lockstep kernel, each from the
// global step at which it was admitted.
struct uspg_engine {
    int max_slots = 0, dtype = USPG_F32, coeff_dtype = USPG_F32, device = 0;
    int64_t gstep = 0;                    // global step of the next launch
    struct Slot {
        bool used = false;
        const uspg_coeffs *c = nullptr;
        const void *proj = nullptr;
        void *image = nullptr, *work = nullptr;
        int sweeps = 0, total = 0, groups = 0;
        bool wide = false;                // its classes alone fill the capped grid
        int64_t offset = 0;
        double beta = 0;
    };
    std::vector<Slot> slots;
    std::vector<int> active;              // slot ids in admission order
    std::vector<int> table;               // the active slots of the lockstep launch
    std::vector<int> wide;                // the active slots launched one by one
    int grid = 0;
    uspg::DevBuf d_static, d_dyn, d_wgbeg;
    void *h_stage = nullptr;              // pinned: static, dyn, wgbeg
    size_t stage_bytes = 0;
    hipEvent_t staged = nullptr;
};

namespace uspg {
namespace {

constexpr int kEngineWaves = 4;

// Problems whose largest class needs at least the single-problem kernel's
// capped grid fill the chip alone: each of their steps is launched with that
// kernel, one problem after another (measured on a 256-ring, 32-view cone:
// two such problems in one lockstep launch took 272 us per step, two
// single-problem launches 224 us).  The others share one lockstep launch.
// Both kernels run the same row update, so the bits do not change.
template <class T>
int engine_upload(uspg_engine *e, hipStream_t s)
{
    USPG_HIP(hipEventSynchronize(e->staged));
    e->table.clear();
    e->wide.clear();
    for (int id : e->active) (e->slots[id].wide ? e->wide : e->table).push_back(id);
    const int n = (int)e->table.size();
    auto *st = static_cast<ProblemStatic *>(e->h_stage);
    auto *dyn = reinterpret_cast<ProblemDyn<T> *>(st + e->max_slots);
    int *wg = reinterpret_cast<int *>(dyn + e->max_slots);
    wg[0] = 0;
    for (int j = 0; j < n; ++j) {
        const uspg_engine::Slot &sl = e->slots[e->table[j]];
        st[j] = static_of(sl.c);
        dyn[j].P = static_cast<const T *>(sl.proj);
        dyn[j].f = static_cast<T *>(sl.work);
        dyn[j].sweeps = sl.sweeps;
        // steps are counted from the engine's current base so int fits
        dyn[j].offset = (int)(sl.offset - e->gstep);
        dyn[j].beta = (T)sl.beta;
        wg[j + 1] = wg[j] + sl.groups;
    }
    e->grid = wg[n];
    if (n > 0) {
        USPG_HIP(hipMemcpyAsync(e->d_static.p, st, sizeof(ProblemStatic) * n, hipMemcpyHostToDevice, s));
        USPG_HIP(hipMemcpyAsync(e->d_dyn.p, dyn, sizeof(ProblemDyn<T>) * n, hipMemcpyHostToDevice, s));
        USPG_HIP(hipMemcpyAsync(e->d_wgbeg.p, wg, sizeof(int) * (n + 1), hipMemcpyHostToDevice, s));
    }
    USPG_HIP(hipEventRecord(e->staged, s));
    return USPG_OK;
}

// Offsets were uploaded relative to the engine's step count at this call,
// so the launches of one call are numbered from 0.  Step t of a problem is
// its step e->gstep + t - offset (view-major, class-minor, as in mart_run).
// Problems are independent, so only each problem's own steps need to stay
// in order: the lockstep steps go first, then the steps of each wide
// problem in one run, which keeps that problem's image in the caches
// (two 256-ring problems alternating step by step took 10 % longer).
template <class T, class TC, int MAXC, int ROWS, bool NT>
int engine_launch(uspg_engine *e, int steps, hipStream_t s)
{
    if (!e->table.empty())
        for (int t = 0; t < steps; ++t)
            hipLaunchKernelGGL((mart_lockstep<T, TC, MAXC, ROWS, NT>), dim3(e->grid), dim3(64 * kEngineWaves), 0, s,
                               e->d_static.as<ProblemStatic>(), e->d_dyn.as<ProblemDyn<T>>(),
                               e->d_wgbeg.as<int>(), (int)e->table.size(), t, 0);
    for (int id : e->wide) {
        const uspg_engine::Slot &sl = e->slots[id];
        const int K = sl.c->Ku * sl.c->Kv;
        for (int t = 0; t < steps; ++t) {
            const int64_t local = e->gstep + t - sl.offset;
            if (local < 0 || local >= sl.total) continue;
            const int cl = (int)(local % K);
            const int v = (int)((local / K) % sl.c->scan.n_views);
            const int rc = batch_step(sl.c, e->dtype, sl.proj, sl.work, sl.beta, v, cl, s);
            if (rc != USPG_OK) return rc;
        }
    }
    USPG_HIP(hipGetLastError());
    return USPG_OK;
}

template <class T, class TC, int ROWS, bool NT>
int engine_chunks(uspg_engine *e, int64_t chunks, int steps, hipStream_t s)
{
    if (chunks <= 2) return engine_launch<T, TC, 2, ROWS, NT>(e, steps, s);
    if (chunks <= 4) return engine_launch<T, TC, 4, ROWS, NT>(e, steps, s);
    if (chunks <= 8) return engine_launch<T, TC, 8, ROWS, NT>(e, steps, s);
    return engine_launch<T, TC, 16, ROWS, NT>(e, steps, s);
}

template <class T, class TC>
int engine_maxc(uspg_engine *e, int steps, hipStream_t s)
{
    int64_t longest = 0;
    bool kept = false, coded_any = false;
    // the lockstep launch reads every table problem's rows and image: the
    // coefficient loads keep the non-temporal hint unless they all fit the
    // last-level cache (each coefficient set counted once)
    std::vector<const uspg_coeffs *> sets;
    size_t coef_bytes = 0, image_bytes = 0;
    for (int id : e->table) {
        const uspg_coeffs *c = e->slots[id].c;
        longest = std::max<int64_t>(longest, stored_max_row(c));
        kept = kept || kept_rows(c);
        coded_any = coded_any || c->coded;
        if (std::find(sets.begin(), sets.end(), c) == sets.end()) {
            sets.push_back(c);
            coef_bytes += coef_set_bytes(c);
        }
        image_bytes += (size_t)solve_cells(c) * sizeof(T);
    }
    const bool nt = stream_coefs(coef_bytes, image_bytes);
    const int64_t chunks = (longest + 63) / 64;
    if (kept)
        return nt ? engine_chunks<T, TC, kRowsKept, true>(e, chunks, steps, s)
                  : engine_chunks<T, TC, kRowsKept, false>(e, chunks, steps, s);
    if (coded_any)
        return nt ? engine_chunks<T, TC, kRowsCoded, true>(e, chunks, steps, s)
                  : engine_chunks<T, TC, kRowsCoded, false>(e, chunks, steps, s);
    return nt ? engine_chunks<T, TC, kRowsStored, true>(e, chunks, steps, s)
              : engine_chunks<T, TC, kRowsStored, false>(e, chunks, steps, s);
}

}  // namespace
}  // namespace uspg

using namespace uspg;

extern "C" {

int uspg_build_batch(int32_t n, const uspg_coeffs *const *coeffs, int32_t dtype, uspg_batch **out)
{
    if (!coeffs || !out || n <= 0) return fail(USPG_E_ARG, "null or empty batch");
    if (dtype != USPG_F32 && dtype != USPG_F64) return fail(USPG_E_ARG, "dtype");
    *out = nullptr;
    int dev = 0;
    USPG_HIP(hipGetDevice(&dev));
    for (int i = 0; i < n; ++i) {
        if (!coeffs[i]) return fail(USPG_E_ARG, "null coefficients in batch");
        if (coeffs[i]->pending) return fail(USPG_E_ARG, "pending coefficients in batch");
        if (coeffs[i]->device != dev) return fail(USPG_E_ARG, "coefficients on another device");
        if (coeffs[i]->segments && !kept_rows(coeffs[i]))
            return fail(USPG_E_ARG, "segment-record coefficients join a batch only with their view rows kept");
        if (stored_coeff_dtype(coeffs[i]) != stored_coeff_dtype(coeffs[0]))
            return fail(USPG_E_ARG, "all problems of a batch must share the coefficient type");
    }
    auto *b = new uspg_batch();
    b->n = n;
    b->dtype = dtype;
    b->device = dev;
    b->co.assign(coeffs, coeffs + n);
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) != hipSuccess) {
        delete b;
        return fail(USPG_E_HIP, "hipGetDeviceProperties failed");
    }
    b->lds_limit = prop.sharedMemPerBlock;
    int rc = b->d_static.alloc(sizeof(ProblemStatic) * n);
    if (rc == USPG_OK) rc = b->d_dyn.alloc(sizeof(ProblemDyn<double>) * n);
    if (rc == USPG_OK) rc = b->d_wgbeg.alloc(sizeof(int) * (n + 1));
    if (rc == USPG_OK && (hipHostMalloc(&b->h_dyn, sizeof(ProblemDyn<double>) * n) != hipSuccess ||
                          hipEventCreateWithFlags(&b->dyn_copied, hipEventDisableTiming) != hipSuccess ||
                          hipEventRecord(b->dyn_copied, nullptr) != hipSuccess))
        rc = fail(USPG_E_HIP, "batch staging allocation failed");
    if (rc == USPG_OK) rc = upload_static(b);
    if (rc != USPG_OK) {
        uspg_free_batch(b);
        return rc;
    }
    *out = b;
    return USPG_OK;
}

int uspg_batch_info(const uspg_batch *b, int32_t *mode, int32_t *block_threads, int32_t *use_lds,
                    int32_t *n_lds, int64_t *lds_bytes)
{
    if (!b) return fail(USPG_E_ARG, "null batch");
    if (mode) *mode = b->mode;
    if (block_threads) *block_threads = b->block;
    if (use_lds) *use_lds = b->use_lds;
    if (n_lds) *n_lds = (int32_t)std::count(b->lds_mode.begin(), b->lds_mode.end(), 1);
    if (lds_bytes) *lds_bytes = (int64_t)b->lds_bytes;
    return USPG_OK;
}

int uspg_batch_set(uspg_batch *b, int32_t mode, int32_t block_threads, int32_t use_lds)
{
    if (!b) return fail(USPG_E_ARG, "null batch");
    if (mode != 0 && mode != 1) return fail(USPG_E_ARG, "mode must be 0 (persistent) or 1 (lockstep)");
    if (block_threads < 64 || block_threads > 1024 || block_threads % 64 ||
        (mode == 1 && block_threads > 256))
        return fail(USPG_E_ARG, "block_threads: multiple of 64 in [64, 1024] (lockstep: <= 256)");
    int rc = check_device(b->device);
    if (rc != USPG_OK) return rc;
    b->mode = mode;
    b->block = block_threads;
    b->use_lds = use_lds ? 1 : 0;
    return upload_static(b);
}

int mart_run_batch(uspg_batch *b, const void *const *proj, void *const *image, void *const *work,
                   const size_t *work_bytes, const int32_t *n_sweeps, const double *beta, void *stream)
{
    if (!b) return fail(USPG_E_ARG, "null batch");
    int rc = check_runs(b, proj, image, work, work_bytes, n_sweeps, beta);
    if (rc == USPG_OK) rc = check_device(b->device);
    if (rc != USPG_OK) return rc;
    hipStream_t s = (hipStream_t)stream;
    for (int i = 0; i < b->n; ++i)
        if ((rc = layout_permute(b->co[i], b->dtype, image[i], work[i], 1, s)) != USPG_OK) return rc;
    if ((rc = solve(b, proj, work, n_sweeps, beta, s)) != USPG_OK) return rc;
    for (int i = 0; i < b->n; ++i)
        if ((rc = layout_permute(b->co[i], b->dtype, work[i], image[i], 0, s)) != USPG_OK) return rc;
    return USPG_OK;
}

int uspg_batch_autotune(uspg_batch *b, const void *const *proj, const void *const *image,
                        void *const *work, const size_t *work_bytes, int32_t probe_sweeps,
                        const double *beta, void *stream, double *best_ms)
{
    if (!b || probe_sweeps <= 0) return fail(USPG_E_ARG, "null batch or probe_sweeps <= 0");
    std::vector<int32_t> sweeps(b->n, probe_sweeps);
    int rc = check_runs(b, proj, (void *const *)image, work, work_bytes, sweeps.data(), beta);
    if (rc == USPG_OK) rc = check_device(b->device);
    if (rc != USPG_OK) return rc;
    hipStream_t s = (hipStream_t)stream;
    // candidates: lockstep with 2 or 4 rays per workgroup; persistent with
    // 256 / 512 / 1024 threads, with and without LDS-resident images
    const int cand[][3] = {{1, 128, 0}, {1, 256, 0}, {0, 256, 1}, {0, 512, 1}, {0, 1024, 1},
                           {0, 512, 0}};
    double best = 1e300;
    int best_mode = b->mode, best_block = b->block, best_lds = b->use_lds;
    hipEvent_t e0, e1;
    USPG_HIP(hipEventCreate(&e0));
    USPG_HIP(hipEventCreate(&e1));
    for (const auto &cd : cand) {
        {
            b->mode = cd[0];
            b->block = cd[1];
            b->use_lds = cd[2];
            if ((rc = upload_static(b)) != USPG_OK) break;
            // fresh scratch copies of the images in the device layout
            for (int i = 0; i < b->n && rc == USPG_OK; ++i)
                rc = layout_permute(b->co[i], b->dtype, image[i], work[i], 1, s);
            if (rc != USPG_OK) break;
            if (hipEventRecord(e0, s) != hipSuccess) { rc = fail(USPG_E_HIP, "event"); break; }
            if ((rc = solve(b, proj, work, sweeps.data(), beta, s)) != USPG_OK) break;
            if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) {
                rc = fail(USPG_E_HIP, "event");
                break;
            }
            float ms = 0.f;
            (void)hipEventElapsedTime(&ms, e0, e1);
            if (ms < best) {
                best = ms;
                best_mode = cd[0];
                best_block = cd[1];
                best_lds = cd[2];
            }
        }
        if (rc != USPG_OK) break;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    b->mode = best_mode;
    b->block = best_block;
    b->use_lds = best_lds;
    int rc2 = upload_static(b);
    if (rc != USPG_OK) return rc;
    if (best_ms) *best_ms = best;
    return rc2;
}

int uspg_engine_create(int32_t max_slots, int32_t dtype, int32_t coeff_dtype, uspg_engine **out)
{
    if (!out || max_slots <= 0) return fail(USPG_E_ARG, "null output or max_slots <= 0");
    if ((dtype != USPG_F32 && dtype != USPG_F64) || (coeff_dtype != USPG_F32 && coeff_dtype != USPG_F64))
        return fail(USPG_E_ARG, "dtype");
    *out = nullptr;
    auto *e = new uspg_engine();
    e->max_slots = max_slots;
    e->dtype = dtype;
    e->coeff_dtype = coeff_dtype;
    e->slots.resize(max_slots);
    int rc = current_device_id(&e->device);
    e->stage_bytes = (sizeof(ProblemStatic) + sizeof(ProblemDyn<double>) + sizeof(int)) * (max_slots + 1);
    if (rc == USPG_OK) rc = e->d_static.alloc(sizeof(ProblemStatic) * max_slots);
    if (rc == USPG_OK) rc = e->d_dyn.alloc(sizeof(ProblemDyn<double>) * max_slots);
    if (rc == USPG_OK) rc = e->d_wgbeg.alloc(sizeof(int) * (max_slots + 1));
    if (rc == USPG_OK && (hipHostMalloc(&e->h_stage, e->stage_bytes) != hipSuccess ||
                          hipEventCreateWithFlags(&e->staged, hipEventDisableTiming) != hipSuccess ||
                          hipEventRecord(e->staged, nullptr) != hipSuccess))
        rc = fail(USPG_E_HIP, "engine staging allocation failed");
    if (rc != USPG_OK) {
        uspg_engine_destroy(e);
        return rc;
    }
    *out = e;
    return USPG_OK;
}

int uspg_engine_admit(uspg_engine *e, const uspg_coeffs *c, const void *proj, void *image, void *work,
                      size_t work_bytes, int32_t n_sweeps, double beta, void *stream, int32_t *slot)
{
    if (!e || !c || !proj || !image || !work) return fail(USPG_E_ARG, "null argument");
    if (n_sweeps <= 0 || !(beta > 0)) return fail(USPG_E_ARG, "n_sweeps > 0 and beta > 0");
    if (c->pending) return fail(USPG_E_ARG, "pending coefficients");
    if (c->segments && !kept_rows(c))
        return fail(USPG_E_ARG, "segment-record coefficients join an engine only with their view rows kept");
    if (stored_coeff_dtype(c) != e->coeff_dtype) return fail(USPG_E_ARG, "coefficient type differs from the engine's");
    if (work_bytes < uspg_mart_workspace_bytes(c, e->dtype, 0.0)) return fail(USPG_E_NOMEM, "work space too small");
    int rc = check_device(e->device);
    if (rc != USPG_OK) return rc;
    int id = -1;
    for (int i = 0; i < e->max_slots; ++i)
        if (!e->slots[i].used) { id = i; break; }
    if (id < 0) return fail(USPG_E_NOMEM, "no free slot");
    if ((rc = layout_permute(c, e->dtype, image, work, 1, (hipStream_t)stream)) != USPG_OK) return rc;
    uspg_engine::Slot &sl = e->slots[id];
    sl.used = true;
    sl.c = c;
    sl.proj = proj;
    sl.image = image;
    sl.work = work;
    sl.sweeps = n_sweeps;
    sl.total = n_sweeps * c->scan.n_views * c->Ku * c->Kv;
    sl.groups = lockstep_groups(c, kEngineWaves);
    sl.wide = sl.groups >= batch_grid_cap();
    sl.offset = e->gstep;
    sl.beta = beta;
    e->active.push_back(id);
    if (slot) *slot = id;
    return USPG_OK;
}

int uspg_engine_step(uspg_engine *e, int32_t n_steps, void *stream, int32_t *finished, int32_t cap,
                     int32_t *n_finished)
{
    if (!e || n_steps <= 0 || !n_finished) return fail(USPG_E_ARG, "null engine/output or n_steps <= 0");
    *n_finished = 0;
    int rc = check_device(e->device);
    if (rc != USPG_OK) return rc;
    if (e->active.empty()) return USPG_OK;
    hipStream_t s = (hipStream_t)stream;
    // step numbers inside a call start at 0: the offsets are re-based and
    // uploaded on every call
    rc = e->dtype == USPG_F64 ? engine_upload<double>(e, s) : engine_upload<float>(e, s);
    if (rc != USPG_OK) return rc;
    const bool cf64 = e->coeff_dtype == USPG_F64;
    if (e->dtype == USPG_F64)
        rc = cf64 ? engine_maxc<double, double>(e, n_steps, s) : engine_maxc<double, float>(e, n_steps, s);
    else
        rc = cf64 ? engine_maxc<float, double>(e, n_steps, s) : engine_maxc<float, float>(e, n_steps, s);
    if (rc != USPG_OK) return rc;
    e->gstep += n_steps;
    std::vector<int> still;
    for (int id : e->active) {
        uspg_engine::Slot &sl = e->slots[id];
        if (e->gstep - sl.offset >= sl.total) {
            if ((rc = layout_permute(sl.c, e->dtype, sl.work, sl.image, 0, s)) != USPG_OK) return rc;
            if (finished && *n_finished < cap) finished[*n_finished] = id;
            ++*n_finished;
            sl = uspg_engine::Slot();
        } else {
            still.push_back(id);
        }
    }
    e->active.swap(still);
    return USPG_OK;
}

int uspg_engine_info(const uspg_engine *e, int32_t *active, int64_t *global_step)
{
    if (!e) return fail(USPG_E_ARG, "null engine");
    if (active) *active = (int32_t)e->active.size();
    if (global_step) *global_step = e->gstep;
    return USPG_OK;
}

void uspg_engine_destroy(uspg_engine *e)
{
    if (!e) return;
    if (e->staged) {
        (void)hipEventSynchronize(e->staged);
        (void)hipEventDestroy(e->staged);
    }
    if (e->h_stage) (void)hipHostFree(e->h_stage);
    e->d_static.release();
    e->d_dyn.release();
    e->d_wgbeg.release();
    delete e;
}

void uspg_free_batch(uspg_batch *b)
{
    if (!b) return;
    if (b->dyn_copied) {
        (void)hipEventSynchronize(b->dyn_copied);
        (void)hipEventDestroy(b->dyn_copied);
    }
    if (b->h_dyn) (void)hipHostFree(b->h_dyn);
    if (b->gexec) (void)hipGraphExecDestroy(b->gexec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->d_static.release();
    b->d_dyn.release();
    b->d_wgbeg.release();
    delete b;
}

}  // extern "C"
