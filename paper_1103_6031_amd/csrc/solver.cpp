// Host side of the MI355X multigrid library: validation, workspace carving, the FAS V-cycle
// schedule (Hahn & Abel 2011, Section 3.2, steps 1-9; Section 3.3 on nested patches), the
// FP64 and mixed-precision drivers, LPT and the C ABI of include/mgic.h.
//
// Level list: L[0] is the finest level (the innermost patch, or the base when there are no
// patches), L[nh-1] the periodic base, L[nh..] its coarsenings down to an odd (or 1-cell) grid.
// Every level l < last has a parent L[l+1] holding its coarse representation at ParentMap::off.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "mg_internal.h"
#include "mgic.h"

namespace mgic {

static thread_local std::string g_err;

static int fail(int code, const std::string& msg) {
    g_err = msg;
    return code;
}

int report_error(int code, const char* msg) { return fail(code, msg); }

// on failure the runtime's last-error state is cleared as well, so that a failed call here is
// not reported again by the caller's next, unrelated HIP call
#define MG_HIP(call)                                                                           \
    do {                                                                                       \
        hipError_t e_ = (call);                                                                \
        if (e_ != hipSuccess) {                                                                \
            (void)hipGetLastError();                                                           \
            return fail(MG_EHIP, std::string(#call) + ": " + hipGetErrorString(e_));           \
        }                                                                                      \
    } while (0)

// ----------------------------------------------------------------------------------------------
// workspace carving (the same code computes sizes when base == nullptr)
// ----------------------------------------------------------------------------------------------
struct Carver {
    char* base;
    size_t off = 0;
    explicit Carver(void* b) : base((char*)b) {}
    template <class T>
    T* take(size_t count) {
        off = (off + 255) & ~(size_t)255;
        T* p = base ? (T*)(base + off) : nullptr;
        off += count * sizeof(T);
        return p;
    }
};

struct Level {
    Dims d{0, 0, 0};
    double h = 0;
    bool periodic = false;  // base or a coarsening of it
    int p = -1;             // hierarchy index (0 = base), -1 for coarsenings
    Lay lay{};              // storage: colour-split rows on even periodic levels, else natural
    ParentMap pm{};         // coarse representation inside L[l+1]
    CovBox child{};         // region of this level covered by L[l-1]
    double* u_user = nullptr;  // caller's array of a hierarchy level (natural rows)
    double *u = nullptr, *f = nullptr, *g = nullptr, *uold = nullptr;   // working arrays (lay)
    double* gpart = nullptr;   // patches: the parent's part of each ghost value, 2 per ghost cell
    float *u32 = nullptr, *f32 = nullptr, *g32 = nullptr, *uold32 = nullptr;
    double* ualt = nullptr;  // second u of the fused mixed-precision outer step (ping-pong)
    float* ealt = nullptr;   // second e of the same
    // second u and f of a coarsening run by the fused tile kernels (written by the pre leg)
    bool fusable = false;
    double *ua = nullptr, *fa = nullptr;
    float *ua32 = nullptr, *fa32 = nullptr;
};

struct Plan {
    std::vector<Level> L;
    int nh = 0;      // hierarchy levels (patches + base)
    int last = 0;    // index of the coarsest level
    int nu1 = 2, nu2 = 2;
    int tail = -1;   // first level of the single-workgroup tail V-cycle (-1: none)
    bool mixed = false;
    double* partials = nullptr;  // kMaxPartials per level segment
    double* scal = nullptr;      // device scalars
};

enum { S_FSUM = 0, S_FNORM = 1, S_RNORM = 2, S_USUM = 3, S_TMP = 4, S_COUNT = 8 };

template <class T> struct B { T *u, *f, *g, *uold, *ua, *fa; };
template <class T> static B<T> bufs(Level& l);
template <> B<double> bufs<double>(Level& l) { return {l.u, l.f, l.g, l.uold, l.ua, l.fa}; }
template <> B<float> bufs<float>(Level& l) { return {l.u32, l.f32, l.g32, l.uold32, l.ua32, l.fa32}; }

static bool odd_ok(int m) { return m == 1 || m == 3 || m == 5 || m == 7; }

static int validate_hier(const mg_hier* H) {
    if (!H) return fail(MG_EINVAL, "hierarchy is NULL");
    if (H->nlev < 1 || H->nlev > MG_MAX_LEVELS) return fail(MG_EINVAL, "nlev out of range");
    const mg_level& b = H->lev[0];
    const int N = b.n[0];
    if (N < 1 || b.n[1] != N || b.n[2] != N) return fail(MG_EINVAL, "base must be cubic n^3, n >= 1");
    int m = N;
    while (m % 2 == 0) m /= 2;
    if (!odd_ok(m)) return fail(MG_EINVAL, "base size must be 2^k * m with m in {1,3,5,7}");
    if (!(b.h > 0) || !std::isfinite(b.h)) return fail(MG_EINVAL, "base spacing must be positive");
    if ((long long)N * N * N >= (1ll << 31)) return fail(MG_EINVAL, "base has 2^31 cells or more");
    for (int p = 1; p < H->nlev; ++p) {
        const mg_level& l = H->lev[p];
        const mg_level& q = H->lev[p - 1];
        if (std::fabs(l.h - 0.5 * q.h) > 1e-12 * q.h) return fail(MG_EINVAL, "patch spacing must be half its parent's");
        for (int a = 0; a < 3; ++a) {
            if (l.n[a] < 4 || l.n[a] % 2) return fail(MG_EINVAL, "patch sizes must be even and >= 4");
            const int lo = l.off[a], hi = l.off[a] + l.n[a] / 2;
            bool ok;
            if (p == 1) ok = lo >= 0 && hi <= q.n[a] && l.n[a] / 2 <= q.n[a] - 2;
            else ok = lo >= 4 && hi <= q.n[a] - 4;
            if (!ok) return fail(MG_EINVAL, "patch " + std::to_string(p) + " not properly nested in its parent");
        }
        if ((long long)l.n[0] * l.n[1] * l.n[2] >= (1ll << 31)) return fail(MG_EINVAL, "patch has 2^31 cells or more");
    }
    return MG_OK;
}

// Build the level list and carve buffers.  u_user / f_user may be null (size query).
static int build_plan(const mg_hier* H, const mg_opts* o, Carver& cv, double* const* u_user, Plan& P,
                      bool fuse = true) {
    int rc = validate_hier(H);
    if (rc) return rc;
    P.nu1 = o ? o->nu1 : 2;
    P.nu2 = o ? o->nu2 : 2;
    P.mixed = o && o->prec == MG_MIXED;
    if (P.nu1 < 0 || P.nu2 < 0 || P.nu1 + P.nu2 > 64) return fail(MG_EINVAL, "nu1/nu2 out of range");
    const int np = H->nlev - 1;
    P.L.clear();
    for (int p = np; p >= 0; --p) {
        Level l;
        const mg_level& m = H->lev[p];
        l.d = Dims{m.n[0], m.n[1], m.n[2]};
        l.h = p == 0 ? m.h : H->lev[0].h / (double)(1 << p);
        l.periodic = p == 0;
        l.p = p;
        P.L.push_back(l);
    }
    P.nh = (int)P.L.size();
    {
        int N = H->lev[0].n[0];
        double h = H->lev[0].h;
        while (N % 2 == 0) {
            N /= 2;
            h *= 2.0;
            Level l;
            l.d = Dims{N, N, N};
            l.h = h;
            l.periodic = true;
            P.L.push_back(l);
        }
    }
    P.last = (int)P.L.size() - 1;
    // colour-split rows wherever a level has even rows (periodic levels above the odd coarsest,
    // and every patch)
    for (auto& L : P.L) L.lay = mklay(L.d, L.d.z % 2 == 0 ? 1 : 0);
    for (int l = 0; l < P.last; ++l) {
        Level& L = P.L[l];
        Level& Q = P.L[l + 1];
        const int* o = L.p >= 1 ? H->lev[L.p].off : nullptr;
        L.pm = ParentMap(Q.lay, o ? o[0] : 0, o ? o[1] : 0, o ? o[2] : 0, Q.periodic ? 1 : 0);
        Q.child.lo[0] = L.pm.off[0]; Q.child.lo[1] = L.pm.off[1]; Q.child.lo[2] = L.pm.off[2];
        Q.child.n[0] = L.d.x / 2; Q.child.n[1] = L.d.y / 2; Q.child.n[2] = L.d.z / 2;
    }
    for (int l = 0; l <= P.last; ++l) {
        Level& L = P.L[l];
        const size_t n = L.d.cells();
        const bool hier = L.p >= 0;
        if (hier) L.u_user = u_user ? u_user[L.p] : nullptr;
        L.u = (hier && !L.lay.split) ? L.u_user : cv.take<double>(n);
        L.f = cv.take<double>(n);
        if (!L.periodic) L.g = cv.take<double>(ghost_cells(L.d));
        if (!L.periodic) L.gpart = cv.take<double>(2 * ghost_cells(L.d));
        if (l < P.last) L.uold = cv.take<double>(n / 8);
        if (P.mixed) {
            L.u32 = cv.take<float>(n);
            L.f32 = cv.take<float>(n);
            if (!L.periodic) L.g32 = cv.take<float>(ghost_cells(L.d));
            if (l < P.last) L.uold32 = cv.take<float>(n / 8);
            if (l == 0 && P.nh == 1 && L.lay.split && n > kTailMaxCells) {
                L.ualt = cv.take<double>(n);
                L.ealt = cv.take<float>(n);
            }
        }
    }
    // coarsenings (below the base: their whole box is the restriction of the finer level) that
    // are power-of-two cubes of 16^3, 32^3 or 64^3 run as two fused tile launches per cycle; their
    // second arrays are reserved whatever nu1 / nu2 are, so that the workspace size depends on
    // the shapes and the precision only
    if (fuse)
        for (int l = 1; l < P.last; ++l) {
            Level& L = P.L[l];
            const int n = L.d.x;
            if (L.p >= 0 || !L.periodic || L.d.y != n || L.d.z != n || !level_fusable(n, 1, 1)) continue;
            L.fusable = true;
            const size_t c = L.d.cells();
            if (P.mixed) {
                L.ua32 = cv.take<float>(c);
                L.fa32 = cv.take<float>(c);
            } else {
                L.ua = cv.take<double>(c);
                L.fa = cv.take<double>(c);
            }
        }
    // the small periodic levels at the bottom, below any fused one, run as one single-workgroup
    // launch (measured: a fused 16^3 level and an 8^3 tail take 28 us per FP32 cycle, a 16^3
    // tail 32 us)
    for (int l = 0; l <= P.last; ++l)
        if (P.L[l].periodic && !P.L[l].fusable && P.L[l].d.cells() <= kTailMaxCells &&
            P.last - l < kTailMaxLevels) {
            P.tail = l;
            break;
        }
    P.partials = cv.take<double>((size_t)kMaxPartials * (P.nh + 1));
    P.scal = cv.take<double>(S_COUNT);
    return MG_OK;
}

// ----------------------------------------------------------------------------------------------
// optional timing of the finest-level smoother launches (HIP events on the launch stream)
// ----------------------------------------------------------------------------------------------
// set for the duration of an allocation-free call: no timing events, and residual readbacks go
// to host stack memory instead of the pinned buffer below
static thread_local bool g_noalloc = false;

struct KProf {
    bool on = false;
    long long period = 1, count = 0;   // time the launches with count % period == 0
    std::vector<hipEvent_t> pool;
    struct Rec { hipEvent_t a, b; double bytes; };
    std::vector<Rec> recs;
    hipEvent_t get() {
        if (!pool.empty()) { hipEvent_t e = pool.back(); pool.pop_back(); return e; }
        hipEvent_t e = nullptr;
        if (hipEventCreate(&e) != hipSuccess) e = nullptr;
        return e;
    }
};
static thread_local KProf g_kprof;

// start / stop events for one timed launch (both null when timing is off)
struct KEvents {
    hipEvent_t a = nullptr, b = nullptr;
    KEvents(bool time_it) {
        if (!time_it || !g_kprof.on || g_noalloc) return;
        if (g_kprof.count++ % g_kprof.period) return;
        a = g_kprof.get();
        b = g_kprof.get();
        if (!a || !b) a = b = nullptr;
    }
    void done(double bytes) {
        if (a) g_kprof.recs.push_back({a, b, bytes});
    }
};

static double* pinned_scratch() {
    static thread_local double* p = nullptr;
    if (!p) {
        if (hipHostMalloc((void**)&p, 64 * sizeof(double), hipHostMallocDefault) != hipSuccess) p = nullptr;
    }
    return p;
}

// MG_EINVAL (with the reason) when st is being captured into a graph: for entry points whose
// work includes host readbacks, uploads or waits
static int refuse_capture(hipStream_t st, const char* what) {
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    MG_HIP(hipStreamIsCapturing(st, &cap));
    if (cap != hipStreamCaptureStatusNone) return fail(MG_EINVAL, std::string(what) + " cannot run under stream capture");
    return MG_OK;
}

// ---- graphs ------------------------------------------------------------------------------------
// Instantiated graphs live until the thread ends; they are deliberately not destroyed at exit,
// when the HIP runtime may already be gone.
struct GraphCache {
    struct Entry {
        hipGraphExec_t ex = nullptr;
        unsigned long long last = 0;   // tick of the last replay
    };
    std::map<std::string, Entry> exec;
    std::map<std::string, int> seen;   // uses of keys not captured yet
    unsigned long long tick = 0;
    hipStream_t cap = nullptr;  // capture stream (capture is illegal on the null stream)
};
// instantiated graphs kept per thread; beyond this the least recently replayed one is dropped
// (dropping them all at once made a workload re-capture its whole working set after other
// workloads had filled the cache)
constexpr size_t kMaxGraphs = 256;
static thread_local GraphCache g_graphs;

// kernel attributes that must be set before any capture
static int graph_setup() {
    static thread_local bool done = false;
    if (done) return MG_OK;
    MG_HIP(tail_kernel_setup());
    MG_HIP(batch_kernel_setup());
    done = true;
    return MG_OK;
}

// runs `body` on st, or replays its graph, captured under `key` at the capture_at-th use of the
// key (1: the first), so that launch sequences run once are never captured
template <class F>
static int run_graph(bool use_graph, const std::string& key, hipStream_t st, F body, int capture_at = 1) {
    if (!use_graph) {
        body(st);
        MG_HIP(hipGetLastError());
        return MG_OK;
    }
    auto it = g_graphs.exec.find(key);
    if (it == g_graphs.exec.end()) {
        if (capture_at > 1 && ++g_graphs.seen[key] < capture_at) {
            body(st);
            MG_HIP(hipGetLastError());
            return MG_OK;
        }
        g_graphs.seen.erase(key);
        if (int rc = graph_setup()) return rc;
        if (!g_graphs.cap) MG_HIP(hipStreamCreateWithFlags(&g_graphs.cap, hipStreamNonBlocking));
        if (g_graphs.exec.size() >= kMaxGraphs) {
            auto old = g_graphs.exec.begin();
            for (auto e = g_graphs.exec.begin(); e != g_graphs.exec.end(); ++e)
                if (e->second.last < old->second.last) old = e;
            (void)hipGraphExecDestroy(old->second.ex);
            g_graphs.exec.erase(old);
        }
        if (g_graphs.seen.size() >= 4096) g_graphs.seen.clear();
        MG_HIP(hipStreamBeginCapture(g_graphs.cap, hipStreamCaptureModeThreadLocal));
        body(g_graphs.cap);
        hipGraph_t g = nullptr;
        MG_HIP(hipStreamEndCapture(g_graphs.cap, &g));
        hipGraphExec_t ex = nullptr;
        const hipError_t e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        MG_HIP(e);
        it = g_graphs.exec.emplace(key, GraphCache::Entry{ex, 0}).first;
    }
    it->second.last = ++g_graphs.tick;
    MG_HIP(hipGraphLaunch(it->second.ex, st));
    return MG_OK;
}

// ----------------------------------------------------------------------------------------------
// V-cycle schedule
// ----------------------------------------------------------------------------------------------
// mode 1: compute the parent's part of the ghosts and keep it; mode 2: reuse the part kept by the
// last mode-1 fill of this level in the same precision, with the parent unchanged since
template <class T>
static void ghosts(Plan& P, int l, hipStream_t st, int mode = 0) {
    Level& L = P.L[l];
    B<T> b = bufs<T>(L), pb = bufs<T>(P.L[l + 1]);
    launch_ghost_fill<T>(pb.u, b.u, b.g, L.lay, L.pm, 1, st, L.gpart, mode);
}

// returns whether a patch's ghosts were filled (then the parent's part of them is kept)
template <class T>
static bool smooth(Plan& P, int l, int sweeps, hipStream_t st, bool skip_first_red = false,
                   const T* corr_pu = nullptr) {
    Level& L = P.L[l];
    B<T> b = bufs<T>(L);
    const bool timed = l == 0;
    const double half_bytes = 0.5 * (double)L.d.cells() * 3.0 * sizeof(T);  // 3 words per update
    bool filled = false;
    for (int s = 0; s < sweeps; ++s)
        for (int c = 0; c < 2; ++c) {
            if (skip_first_red && s == 0 && c == 0) continue;  // already done by the fused outer step
            if (corr_pu && s == 0 && c == 0) {   // step 8 folded into the first red half-sweep (untimed)
                launch_rbgs_vec_corr<T>(b.u, b.f, L.lay, L.h, corr_pu, b.uold, st);
                continue;
            }
            // only the patch changes during the pass: the parent's part is formed once
            if (!L.periodic) ghosts<T>(P, l, st, filled ? 2 : 1);
            filled = !L.periodic;
            KEvents ev(timed);
            if (L.periodic && rbgs_vec_ok(L.lay, sizeof(T)))
                launch_rbgs_vec<T>(b.u, b.f, L.lay, L.h, c, st, ev.a, ev.b);
            else
                launch_rbgs_half<T>(b.u, b.f, L.periodic ? nullptr : b.g, L.lay, L.h, c, st, ev.a, ev.b);
            ev.done(half_bytes);
        }
    return filled;
}

// level l runs as the two fused tile launches (its arrays for them are reserved and the sweep
// counts fit the kernels' halos)
template <class T>
static bool fused(Plan& P, int l) {
    Level& L = P.L[l];
    return L.fusable && bufs<T>(L).ua && level_fusable(L.d.x, P.nu1, P.nu2);
}

// a periodic colour-split power-of-two cube with a colour-split parent: its transfers take the
// power-of-two kernels
static bool p2lev(const Level& L) {
    const Lay& A = L.lay;
    return L.periodic && A.pow2 && A.split && A.d.x == A.d.y && A.d.y == A.d.z && A.d.x >= 4 &&
           L.pm.off[0] == 0 && L.pm.off[1] == 0 && L.pm.off[2] == 0;
}

template <class T>
static void vcycle(Plan& P, int l, hipStream_t st, bool skip_first_red = false) {
    Level& L = P.L[l];
    B<T> b = bufs<T>(L);
    if (l == P.tail) {  // this level and all below: one launch
        TailPlan<T> tp{};
        tp.n = P.last - l + 1;
        tp.nu1 = P.nu1;
        tp.nu2 = P.nu2;
        tp.fas0 = l > 0 && fused<T>(P, l - 1);   // a fused parent leaves step 6 to this level
        for (int k = 0; k < tp.n; ++k) {
            B<T> c = bufs<T>(P.L[l + k]);
            tp.lev[k] = TailLevel<T>{c.u, c.f, P.L[l + k].lay, P.L[l + k].h, 0, 0, 0};
        }
        tail_assign_lds(tp);
        launch_tail<T>(tp, st);
        return;
    }
    if (l == P.last) {  // step 1
        launch_coarsest<T>(b.u, b.f, L.d.x, L.h, st);
        return;
    }
    Level& Q = P.L[l + 1];
    B<T> q = bufs<T>(Q);
    if (fused<T>(P, l)) {
        // step 6 of the parent and steps 2-5 in one launch, step 7, steps 8-9 in one launch
        launch_level_pre<T>(b.u, b.f, b.ua, b.fa, q.u, q.f, b.uold, L.d.x, L.h, P.nu1, st);
        vcycle<T>(P, l + 1, st);
        launch_level_post<T>(b.ua, b.fa, q.u, b.uold, b.u, L.d.x, L.h, P.nu2, st);
        return;
    }
    const bool filled = smooth<T>(P, l, P.nu1, st, skip_first_red);  // step 2
    if (!L.periodic) ghosts<T>(P, l, st, filled ? 2 : 0);
    // steps 3-5, then step 6 on the covered region of the parent (a fused parent does its own)
    const bool p2 = p2lev(L);
    if (p2) launch_resid_restrict_p2<T>(b.u, b.f, L.d.x, L.h, q.u, q.f, b.uold, st);
    else launch_resid_restrict<T>(b.u, b.f, L.periodic ? nullptr : b.g, L.lay, L.h, q.u, q.f, b.uold, L.pm, st);
    if (!fused<T>(P, l + 1)) {
        if (p2 && Q.lay.pow2 && Q.lay.split && rbgs_vec_ok(Q.lay, sizeof(T))) launch_fas_vec<T>(q.u, q.f, Q.d.x, Q.h, st);
        else if (p2 && Q.lay.pow2 && Q.lay.split) launch_fas_rhs_p2<T>(q.u, q.f, Q.d.x, Q.h, st);
        else launch_fas_rhs<T>(q.u, q.f, L.pm, Dims{L.d.x / 2, L.d.y / 2, L.d.z / 2}, Q.h, st);
    }
    vcycle<T>(P, l + 1, st);                         // step 7
    // black cells only where nothing reads the red ones before the red half-sweep rewrites them:
    // a patch's ghost fill reads both colours of its first two layers
    // step 8: on power-of-two levels the black correction is applied by the first red half-sweep
    // of step 9, as it reads the black cells
    // (measured: FP64 at 256^3 and above is faster as two passes)
    const bool fold = p2 && P.nu2 > 0 && rbgs_vec_ok(L.lay, sizeof(T)) &&
                      (sizeof(T) == 4 || L.d.cells() < ((size_t)1 << 24));
    if (fold) {
        smooth<T>(P, l, P.nu2, st, false, q.u);      // steps 8-9
        return;
    }
    if (p2 && P.nu2 > 0) launch_prolong_black_p2<T>(b.u, L.d.x, q.u, b.uold, st);  // step 8
    else launch_prolong<T>(b.u, L.lay, q.u, b.uold, L.pm, P.nu2 > 0 && L.periodic, st);
    smooth<T>(P, l, P.nu2, st);                      // step 9
}

static long long updates_per_cycle(const Plan& P) {
    long long s = 0;
    for (int l = 0; l < P.last; ++l) s += (long long)(P.nu1 + P.nu2) * (long long)P.L[l].d.cells();
    return s;
}

// covered cells of every hierarchy level := mean of their children, finest first
template <class T>
static void restrict_up(Plan& P, T* const* v, hipStream_t st) {
    for (int l = 0; l + 1 < P.nh; ++l) launch_restrict_cov<T>(v[l], P.L[l].lay, v[l + 1], P.L[l].pm, st);
}

// sum over the base of v (after restrict_up) -> scal[slot]
static void base_sum(Plan& P, const double* vbase, int slot, hipStream_t st) {
    int np = 0;
    CovBox none{};
    launch_sum(vbase, P.L[P.nh - 1].lay, none, 0, P.partials, &np, st);
    SegList s{};
    s.n = 1; s.off[0] = 0; s.cnt[0] = np; s.w[0] = 1.0;
    launch_finalize(P.partials, s, P.scal + slot, st);
}

// composite sum of v^2 * vol over uncovered cells -> scal[slot]
static void composite_sq(Plan& P, double* const* v, int slot, hipStream_t st) {
    SegList s{};
    s.n = P.nh;
    for (int l = 0; l < P.nh; ++l) {
        int np = 0;
        CovBox cb = l > 0 ? P.L[l].child : CovBox{};
        launch_sum(v[l], P.L[l].lay, cb, 1, P.partials + (size_t)l * kMaxPartials, &np, st);
        s.off[l] = l * kMaxPartials;
        s.cnt[l] = np;
        s.w[l] = P.L[l].h * P.L[l].h * P.L[l].h;
    }
    launch_finalize(P.partials, s, P.scal + slot, st);
}

// composite FP64 residual of the current u (covered coarse cells restricted first);
// r written as R to rout[l] if given (natural rows if rout_natural, else the level's layout);
// sum r^2 vol -> scal[S_RNORM]
template <class R>
static void composite_residual(Plan& P, R* const* rout, bool rout_natural, hipStream_t st) {
    std::vector<double*> u(P.nh);
    for (int l = 0; l < P.nh; ++l) u[l] = P.L[l].u;
    restrict_up<double>(P, u.data(), st);
    SegList s{};
    s.n = P.nh;
    for (int l = 0; l < P.nh; ++l) {
        Level& L = P.L[l];
        if (!L.periodic) ghosts<double>(P, l, st);
        int np = 0;
        CovBox cb = l > 0 ? L.child : CovBox{};
        const Lay LR = rout_natural ? mklay(L.d, 0) : L.lay;
        launch_residual<double, R>(L.u, L.f, L.periodic ? nullptr : L.g, L.lay, L.h, cb, rout ? rout[l] : nullptr,
                                   LR, P.partials + (size_t)l * kMaxPartials, &np, st);
        s.off[l] = l * kMaxPartials;
        s.cnt[l] = np;
        s.w[l] = L.h * L.h * L.h;
    }
    launch_finalize(P.partials, s, P.scal + S_RNORM, st);
}

// f working copies: copy, restrict bottom-up, subtract the composite mean (unless fix_mean is
// false: the caller's f is taken as it is); |f|^2 -> scal[S_FNORM]
static int prepare_f(Plan& P, const double* const* f_user, hipStream_t st, bool fix_mean = true) {
    if (fix_mean && P.nh == 1 && P.L[0].lay.split) {
        // one periodic level: copy-in with the sum, then mean removal with the sum of squares
        // (the same partial sums, so the same bits, as the separate passes below)
        Level& L = P.L[0];
        if (!f_user[0]) return fail(MG_EINVAL, "f pointer is NULL");
        int np = 0;
        launch_relayout_sum(f_user[0], L.f, L.lay, P.partials, &np, st);
        SegList s{};
        s.n = 1; s.off[0] = 0; s.cnt[0] = np; s.w[0] = 1.0;
        launch_finalize(P.partials, s, P.scal + S_FSUM, st);
        launch_submean_sumsq(L.f, L.lay, P.scal + S_FSUM, 1.0 / (double)L.d.cells(), P.partials, &np, st);
        s.cnt[0] = np;
        s.w[0] = L.h * L.h * L.h;
        launch_finalize(P.partials, s, P.scal + S_FNORM, st);
        return MG_OK;
    }
    for (int l = 0; l < P.nh; ++l) {
        if (!f_user[P.L[l].p]) return fail(MG_EINVAL, "f pointer is NULL");
        launch_relayout<double, double>(f_user[P.L[l].p], mklay(P.L[l].d, 0), P.L[l].f, P.L[l].lay, st);
    }
    std::vector<double*> f(P.nh);
    for (int l = 0; l < P.nh; ++l) f[l] = P.L[l].f;
    restrict_up<double>(P, f.data(), st);
    if (fix_mean) {
        const Level& base = P.L[P.nh - 1];
        base_sum(P, base.f, S_FSUM, st);
        const double inv = 1.0 / (double)base.d.cells();
        for (int l = 0; l < P.nh; ++l) launch_sub_mean<double>(P.L[l].f, P.L[l].d.cells(), P.scal + S_FSUM, inv, st);
    }
    composite_sq(P, f.data(), S_FNORM, st);
    return MG_OK;
}

// covered cells of u := the mean of their children; then (fix_mean) the composite mean removed
static void gauge_u(Plan& P, hipStream_t st, bool fix_mean = true) {
    std::vector<double*> u(P.nh);
    for (int l = 0; l < P.nh; ++l) u[l] = P.L[l].u;
    restrict_up<double>(P, u.data(), st);
    if (!fix_mean) return;
    const Level& base = P.L[P.nh - 1];
    base_sum(P, base.u, S_USUM, st);
    const double inv = 1.0 / (double)base.d.cells();
    for (int l = 0; l < P.nh; ++l) launch_sub_mean<double>(P.L[l].u, P.L[l].d.cells(), P.scal + S_USUM, inv, st);
}

static int read_scalars(Plan& P, int first, int count, double* out, hipStream_t st) {
    if (g_noalloc) {   // pageable destination: the copy is complete once the stream has drained
        double tmp[S_COUNT];
        if (count > S_COUNT) return fail(MG_EINVAL, "internal: scalar readback too long");
        MG_HIP(hipMemcpyAsync(tmp, P.scal + first, count * sizeof(double), hipMemcpyDeviceToHost, st));
        MG_HIP(hipStreamSynchronize(st));
        for (int i = 0; i < count; ++i) out[i] = tmp[i];
        return MG_OK;
    }
    double* pin = pinned_scratch();
    if (!pin) return fail(MG_EHIP, "pinned host buffer unavailable");
    MG_HIP(hipMemcpyAsync(pin, P.scal + first, count * sizeof(double), hipMemcpyDeviceToHost, st));
    MG_HIP(hipStreamSynchronize(st));
    for (int i = 0; i < count; ++i) out[i] = pin[i];
    return MG_OK;
}

// FP32 inner cycles for the next FP64 correction of the mixed-precision solve.  opt > 0 fixes the
// count.  Otherwise (the default) it is chosen from the residuals: each inner cycle contracts the
// error roughly tenfold, so kInnerMax cycles (about 1e-4) stay well above FP32 round-off and up
// to that many run per correction; once two corrections have been measured, the observed
// contraction per cycle, rho, predicts how many cycles bring rel below tol, and no more than that
// many run.  The rule reads only the residual history, so a batched solve makes the same choices
// as a solo one.  (Measured at 256^3: a cap of 4 keeps the cycle count of a cap of 3 with one
// outer step fewer per solve.)
constexpr int kInnerMax = 4;
static int inner_count(int opt, bool fixed, double rel, double prev_rel, int prev_n, double tol) {
    if (opt > 0) return opt;
    if (fixed || prev_n <= 0 || !(prev_rel > 0) || !(rel > 0) || !std::isfinite(rel) || !(tol > 0)) return kInnerMax;
    const double rho = std::pow(rel / prev_rel, 1.0 / prev_n);
    if (!(rho > 0) || rho >= 0.5) return kInnerMax;
    const double m = std::ceil(std::log(tol / rel) / std::log(rho));
    return (int)std::min<double>(kInnerMax, std::max(1.0, m));
}

// graph key of a solve's plan: every kernel argument of its cycles and outer steps follows from
// the workspace address, the shapes, spacings and sweep counts (and the caller's u where a level
// is solved in place); the steps that read f or write u add those pointers
static std::string plan_key(const Plan& P, const void* ws) {
    std::string k = "solo|" + std::to_string((uintptr_t)ws) + "|" + std::to_string(P.nu1) + "," +
                    std::to_string(P.nu2) + "," + std::to_string((int)P.mixed) + "," + std::to_string(P.tail);
    for (const Level& L : P.L) {
        uint64_t hb;
        std::memcpy(&hb, &L.h, sizeof(hb));
        k += "|" + std::to_string(L.d.x) + "," + std::to_string(L.d.y) + "," + std::to_string(L.d.z) + "," +
             std::to_string(L.pm.off[0]) + "," + std::to_string(L.pm.off[1]) + "," + std::to_string(L.pm.off[2]) +
             "," + std::to_string(hb) + "," + std::to_string((int)L.fusable);
        if (L.u && L.u == L.u_user) k += "," + std::to_string((uintptr_t)L.u_user);
    }
    return k;
}

static std::string user_key(const mg_hier* H, const double* const* f, double* const* u) {
    std::string k;
    for (int p = 0; p < H->nlev; ++p) k += "|" + std::to_string((uintptr_t)f[p]) + "," + std::to_string((uintptr_t)u[p]);
    return k;
}

// the tuned inner-cycle count for this problem shape (0: none recorded; defined with the tuner)
static int tuned_inner(const mg_hier* H, const mg_opts* o);

static int solve(const mg_hier* H, const double* const* f, double* const* u, const mg_opts* o, mg_stats* stats,
                 void* ws, size_t ws_bytes, hipStream_t st) {
    if (!o) return fail(MG_EINVAL, "options are NULL");
    if (!f || !u) return fail(MG_EINVAL, "f/u pointer arrays are NULL");
    if (o->max_cycles < 0) return fail(MG_EINVAL, "max_cycles < 0");
    if (o->prec != MG_FP64 && o->prec != MG_MIXED) return fail(MG_EINVAL, "unknown precision");
    if (o->inner < 0 || o->inner > 16) return fail(MG_EINVAL, "inner cycles out of range (0..16)");
    if (int v = validate_hier(H)) return v;
    for (int p = 0; p < H->nlev; ++p)
        if (!u[p] || !f[p]) return fail(MG_EINVAL, "level pointer is NULL");
    mg_opts tuned;
    if (o->prec == MG_MIXED && o->inner == 0) {   // a count the tuner recorded for this shape
        const int k = tuned_inner(H, o);
        if (k > 0) {
            tuned = *o;
            tuned.inner = k;
            o = &tuned;
        }
    }
    Plan P;
    Carver size_cv(nullptr);
    int rc = build_plan(H, o, size_cv, u, P);
    if (rc) return rc;
    if (!ws || ws_bytes < size_cv.off) return fail(MG_EINVAL, "workspace too small: need " + std::to_string(size_cv.off));
    if (((uintptr_t)ws) & 255) return fail(MG_EINVAL, "workspace must be 256-byte aligned");
    Carver cv(ws);
    build_plan(H, o, cv, u, P);
    (void)hipGetLastError();

    const bool fixed = (o->flags & MG_FIXED_CYCLES) != 0;
    const bool guess = (o->flags & MG_USE_INITIAL_GUESS) != 0;
    const bool fix_mean = (o->flags & MG_NO_MEAN_FIX) == 0;
    const std::string mtag = fix_mean ? "" : "|nomean";
    // A caller capturing the stream into a graph gets the launches themselves: no graphs of our
    // own, no host readback, no wait at the end.  Only a fixed number of cycles can run so.
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    MG_HIP(hipStreamIsCapturing(st, &cap));
    const bool capturing = cap != hipStreamCaptureStatusNone;
    if (capturing && !fixed)
        return fail(MG_EINVAL, "under stream capture only MG_FIXED_CYCLES solves run (a converging solve reads its residual back)");
    // Launch sequences that repeat (a cycle, an outer step) are replayed as HIP graphs, captured
    // the second time a sequence is met for this workspace and plan; not with kernel timing (its
    // events are recorded by the dispatches) nor in the allocation-free call.
    const bool use_graph = (o->flags & MG_NO_GRAPH) == 0 && !g_noalloc && !g_kprof.on && !capturing;
    const std::string gkey = use_graph ? plan_key(P, ws) : std::string();
    const std::string ukey = use_graph ? user_key(H, f, u) : std::string();
    double* pin = nullptr;   // the readback buffer (a fixed-cycle solve reads nothing back)
    if (!g_noalloc && !fixed && !(pin = pinned_scratch())) return fail(MG_EHIP, "pinned host buffer unavailable");
    // one step of the solve: `launches`, then (count > 0) the copy of scal[first .. first + count)
    // to the host and a wait for the stream
    auto step = [&](const std::string& var, auto&& launches, int first, int count, double* out) -> int {
        if (!use_graph) {
            launches(st);
            MG_HIP(hipGetLastError());
            return count ? read_scalars(P, first, count, out, st) : MG_OK;
        }
        // the key names the copy too: a step captured without it (fixed cycles) must never be
        // replayed where the host reads its result
        const std::string key = gkey + var + "|c" + std::to_string(first) + "," + std::to_string(count);
        const int rcg = run_graph(true, key, st, [&](hipStream_t s) {
            launches(s);
            if (count) (void)hipMemcpyAsync(pin, P.scal + first, count * sizeof(double), hipMemcpyDeviceToHost, s);
        }, 2);
        if (rcg) return rcg;
        if (count) {
            MG_HIP(hipStreamSynchronize(st));
            for (int i = 0; i < count; ++i) out[i] = pin[i];
        }
        return MG_OK;
    };

    // a zero start of the fused mixed-precision path needs no fill: its first outer step takes
    // u as zero without reading it and writes the zero iterate itself
    const bool zero_start = !guess && P.mixed && P.L[0].ualt;
    double fs[2] = {0, 0};
    // without the mean fix only |f|^2 is read back (the mean removed is reported as 0)
    rc = step(std::string("|prep") + (guess ? "g" : "z") + mtag + ukey, [&](hipStream_t s) {
        prepare_f(P, f, s, fix_mean);
        for (int l = 0; l < P.nh; ++l) {
            Level& L = P.L[l];
            if (zero_start) continue;
            if (!guess) launch_fill<double>(L.u, L.d.cells(), 0.0, s);
            else if (L.u != L.u_user) launch_relayout<double, double>(L.u_user, mklay(L.d, 0), L.u, L.lay, s);
        }
    }, fix_mean ? S_FSUM : S_FNORM, fixed ? 0 : (fix_mean ? 2 : 1), fix_mean ? fs : fs + 1);
    if (rc) return rc;

    mg_stats S;
    std::memset(&S, 0, sizeof(S));
    for (double& v : S.res_hist) v = NAN;
    double check_prev = NAN;   // relative residual at the previous FP64 correction
    int last_inner = 0;        // inner cycles run since it
    double fnorm2 = 0;
    if (!fixed) {
        S.f_mean_removed = fs[0] / (double)P.L[P.nh - 1].d.cells();
        fnorm2 = fs[1];
        if (!std::isfinite(fnorm2) || !std::isfinite(fs[0])) {
            S.rel_res = NAN;
            if (stats) *stats = S;
            return fail(MG_EDIVERGED, "right-hand side contains NaN or Inf");
        }
    }
    const long long upc = updates_per_cycle(P);
    double rel = NAN, prev = INFINITY;
    int grow = 0, status = MG_ENOCONV, cycles = 0;
    auto check = [&](double r2) -> int {
        rel = fnorm2 > 0 ? std::sqrt(r2 / fnorm2) : 0.0;
        if (cycles >= 1 && cycles <= 64) S.res_hist[cycles - 1] = rel;
        if (!std::isfinite(rel)) return MG_EDIVERGED;
        grow = rel > prev ? grow + 1 : 0;
        prev = rel;
        if (grow >= 3) return MG_EDIVERGED;
        return rel <= o->tol ? MG_OK : 1;
    };
    auto ptag = [](const void* q) { return std::to_string((uintptr_t)q); };

    if (!P.mixed) {
        if (guess && !fixed) {
            double r2;
            rc = step("|g64", [&](hipStream_t s) { composite_residual<double>(P, nullptr, false, s); }, S_RNORM, 1, &r2);
            if (rc) return rc;
            const int c = check(r2);
            if (c == MG_OK) status = MG_OK;
            else if (c == MG_EDIVERGED) status = MG_EDIVERGED;   // NaN/Inf in the initial guess
        }
        while (status == MG_ENOCONV && cycles < o->max_cycles) {
            double r2 = 0;
            rc = step(fixed ? "|c64f" : "|c64", [&](hipStream_t s) {
                vcycle<double>(P, 0, s);
                if (!fixed) composite_residual<double>(P, nullptr, false, s);
            }, S_RNORM, fixed ? 0 : 1, &r2);
            if (rc) return rc;
            ++cycles;
            S.cell_updates += upc;
            if (fixed) continue;
            const int c = check(r2);
            if (c == MG_OK) status = MG_OK;
            else if (c == MG_EDIVERGED) { status = MG_EDIVERGED; break; }
        }
    } else if (P.L[0].ualt) {
        // single periodic level: the correction update, the FP64 residual, the FP32 right-hand
        // side and the first red half-sweep of the next inner cycle are one kernel
        Level& L = P.L[0];
        bool pending = false;
        bool u_zero = zero_start;   // the iterate is +0 and not stored (a zero start, before its first correction)
        for (;;) {
            double r2 = 0;
            rc = step("|o" + std::to_string((int)u_zero) + std::to_string((int)pending) + ptag(L.u) + ptag(L.u32),
                      [&](hipStream_t s) {
                          int np = 0;
                          launch_outer_split(u_zero ? nullptr : L.u, pending ? L.u32 : nullptr, L.f, L.ualt, L.f32,
                                             L.ealt, L.lay, L.h, P.partials, &np, s);
                          SegList sg{};
                          sg.n = 1; sg.off[0] = 0; sg.cnt[0] = np; sg.w[0] = L.h * L.h * L.h;
                          launch_finalize(P.partials, sg, P.scal + S_RNORM, s);
                      }, S_RNORM, fixed ? 0 : 1, &r2);
            if (rc) return rc;
            if (pending) u_zero = false;   // this step stored u = 0 + e
            std::swap(L.u, L.ualt);
            std::swap(L.u32, L.ealt);
            if (!fixed) {
                int c = check(r2);
                if (c == MG_OK) { status = MG_OK; break; }
                if (c == MG_EDIVERGED) { status = MG_EDIVERGED; break; }
            }
            if (cycles >= o->max_cycles) break;
            const int nin = inner_count(o->inner, fixed, rel, check_prev, last_inner, o->tol);
            check_prev = rel;
            last_inner = 0;
            for (int k = 0; k < nin && cycles < o->max_cycles; ++k) {
                rc = step("|i" + std::to_string((int)(k == 0)) + ptag(L.u32),
                          [&](hipStream_t s) { vcycle<float>(P, 0, s, /*skip_first_red=*/k == 0); }, 0, 0, nullptr);
                if (rc) return rc;
                ++cycles;
                ++last_inner;
                S.cell_updates += upc;
            }
            pending = true;
        }
        if (u_zero) launch_fill<double>(L.u, L.d.cells(), 0.0, st);   // stopped before any correction
    } else {
        std::vector<float*> rhs(P.nh);
        for (int l = 0; l < P.nh; ++l) rhs[l] = P.L[l].f32;
        bool pending = false;   // FP32 corrections not yet added to u
        for (;;) {
            double r2 = 0;
            rc = step(pending ? "|r1" : "|r0", [&](hipStream_t s) {
                if (pending)
                    for (int l = 0; l < P.nh; ++l) launch_add_f32_to_f64(P.L[l].u, P.L[l].u32, P.L[l].d.cells(), s);
                composite_residual<float>(P, rhs.data(), false, s);
            }, S_RNORM, fixed ? 0 : 1, &r2);
            if (rc) return rc;
            pending = false;
            if (!fixed) {
                int c = check(r2);
                if (c == MG_OK) { status = MG_OK; break; }
                if (c == MG_EDIVERGED) { status = MG_EDIVERGED; break; }
            }
            if (cycles >= o->max_cycles) break;
            const int nin = inner_count(o->inner, fixed, rel, check_prev, last_inner, o->tol);
            check_prev = rel;
            last_inner = 0;
            for (int k = 0; k < nin && cycles < o->max_cycles; ++k) {
                rc = step(k == 0 ? "|j1" : "|j0", [&](hipStream_t s) {
                    if (k == 0)
                        for (int l = 0; l < P.nh; ++l) launch_fill<float>(P.L[l].u32, P.L[l].d.cells(), 0.0f, s);
                    vcycle<float>(P, 0, s);
                }, 0, 0, nullptr);
                if (rc) return rc;
                ++cycles;
                ++last_inner;
                S.cell_updates += upc;
            }
            pending = true;
        }
        if (pending)
            for (int l = 0; l < P.nh; ++l) launch_add_f32_to_f64(P.L[l].u, P.L[l].u32, P.L[l].d.cells(), st);
    }
    rc = step("|fin" + ptag(P.L[0].u) + mtag + ukey, [&](hipStream_t s) {   // P.L[0].u: where the fused path ended
        if (fix_mean && P.nh == 1 && P.L[0].u != P.L[0].u_user) {
            // one periodic level: its sum, then the copy back with the mean removed
            Level& L = P.L[0];
            base_sum(P, L.u, S_USUM, s);
            launch_relayout_sub(L.u, L.lay, L.u_user, mklay(L.d, 0), P.scal + S_USUM, 1.0 / (double)L.d.cells(), s);
        } else {
            gauge_u(P, s, fix_mean);
            for (int l = 0; l < P.nh; ++l) {
                Level& L = P.L[l];
                if (L.u != L.u_user) launch_relayout<double, double>(L.u, L.lay, L.u_user, mklay(L.d, 0), s);
            }
        }
    }, 0, 0, nullptr);
    if (rc) return rc;
    MG_HIP(hipGetLastError());
    if (fixed) {
        if (!capturing) MG_HIP(hipStreamSynchronize(st));  // surface asynchronous faults at the API boundary
        status = MG_OK;
    }
    S.cycles = cycles;
    S.rel_res = rel;
    if (stats) *stats = S;
    if (status == MG_ENOCONV) return fail(MG_ENOCONV, "not converged after " + std::to_string(cycles) + " cycles");
    if (status == MG_EDIVERGED) return fail(MG_EDIVERGED, "residual diverged (NaN/Inf or growth)");
    return MG_OK;
}

// ----------------------------------------------------------------------------------------------
// allocation-free solve: the workspace is a static device array, one copy per GPU
// ----------------------------------------------------------------------------------------------
static __device__ __align__(256) unsigned char scratch[MG_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void* g_scratch_ptr[kMaxDevices] = {};

// device address of the current device's copy of `scratch`, looked up once per device with that
// device current (host code never passes the symbol itself: on the host it is only a stand-in)
static int scratch_address(void** out) {
    int dev = -1;
    MG_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(MG_EINVAL, "device index out of range for the scratch table");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        MG_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p || ((uintptr_t)p & 255)) return fail(MG_EHIP, "scratch array has no aligned device address");
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return MG_OK;
}

struct NoAllocScope {
    NoAllocScope() { g_noalloc = true; }
    ~NoAllocScope() { g_noalloc = false; }
};

static int solve_noalloc(const mg_hier* H, const double* const* f, double* const* u, const mg_opts* o,
                         mg_stats* stats, hipStream_t st) {
    if (!o) return fail(MG_EINVAL, "options are NULL");
    if (int v = validate_hier(H)) return v;
    Plan P;
    Carver size_cv(nullptr);
    if (int rc = build_plan(H, o, size_cv, nullptr, P)) return rc;
    if (size_cv.off > (size_t)MG_SCRATCH_BYTES)
        return fail(MG_EINVAL, "problem needs " + std::to_string(size_cv.off) + " workspace bytes, above the " +
                                   std::to_string((size_t)MG_SCRATCH_BYTES) + " of the static scratch array");
    void* ws = nullptr;
    if (int rc = scratch_address(&ws)) return rc;
    NoAllocScope scope;
    return solve(H, f, u, o, stats, ws, (size_t)MG_SCRATCH_BYTES, st);
}

static mg_hier single_level(int n, double h) {
    mg_hier H;
    std::memset(&H, 0, sizeof(H));
    H.nlev = 1;
    H.lev[0].n[0] = H.lev[0].n[1] = H.lev[0].n[2] = n;
    H.lev[0].h = h;
    return H;
}

// ----------------------------------------------------------------------------------------------
// LPT
// ----------------------------------------------------------------------------------------------
struct LptPlan {
    std::vector<double*> phi;  // restricted copies (P > 0) or the user's arrays
    double* padded = nullptr;  // one padded level (three, 'padstride' apart, for the LLA density)
    size_t padstride = 0;
    double* psi = nullptr;     // tau scratch: 3 gradient fields
    double* partials = nullptr;
    double* scal = nullptr;
};

// what: 1 displacements, 2 tau (and displacements), 3 LLA density (three displacement components
// per level are copied and padded instead of one potential)
static size_t lpt_carve(const mg_hier* H, int what, Carver& cv, LptPlan& lp) {
    // patch padding for either gradient order: 3 for the displacements (sixth order; 2 for the
    // fourth), 6 for tau (4), 2 for the LLA density
    const int R = what == 2 ? 6 : (what == 1 ? 3 : 2), nc = what == 3 ? 3 : 1;
    size_t maxpad = 0;
    lp.phi.assign((size_t)nc * H->nlev, nullptr);
    if (H->nlev > 1)
        for (int p = 0; p < H->nlev; ++p) {
            const mg_level& l = H->lev[p];
            for (int c = 0; c < nc; ++c) lp.phi[(size_t)c * H->nlev + p] = cv.take<double>((size_t)l.n[0] * l.n[1] * l.n[2]);
            if (p > 0) {
                size_t s = (size_t)(l.n[0] + 2 * R) * (l.n[1] + 2 * R) * (l.n[2] + 2 * R);
                if (s > maxpad) maxpad = s;
            }
        }
    if (maxpad) lp.padded = cv.take<double>(nc * maxpad);
    lp.padstride = maxpad;
    if (what == 2) {
        size_t m = (size_t)H->lev[0].n[0] * H->lev[0].n[1] * H->lev[0].n[2];
        for (int p = 1; p < H->nlev; ++p) {
            const mg_level& l = H->lev[p];
            const size_t s = (size_t)(l.n[0] + 6) * (l.n[1] + 6) * (l.n[2] + 6);
            if (s > m) m = s;
        }
        lp.psi = cv.take<double>(3 * m);
    }
    lp.partials = cv.take<double>(kMaxPartials);
    lp.scal = cv.take<double>(S_COUNT);
    return cv.off;
}

static ParentMap parent_of(const mg_hier* H, int p) {
    const mg_level& q = H->lev[p - 1];
    const int* o = H->lev[p].off;
    return ParentMap(Lay(Dims{q.n[0], q.n[1], q.n[2]}, 0), o[0], o[1], o[2], p == 1 ? 1 : 0);
}

static Dims dims_of(const mg_hier* H, int p) { return Dims{H->lev[p].n[0], H->lev[p].n[1], H->lev[p].n[2]}; }
static double h_of(const mg_hier* H, int p) { return H->lev[0].h / (double)(1 << p); }

static int lpt_common(const mg_hier* H, int what, const double* const* phi, void* ws, size_t ws_bytes,
                      hipStream_t st, LptPlan& lp, int order = 4) {
    int rc = validate_hier(H);
    if (rc) return rc;
    if (order != 4 && order != 6) return fail(MG_EINVAL, "grad_order must be 4 or 6");
    // the periodic stencils wrap an offset of up to order / 2 cells once
    if (H->lev[0].n[0] < 2) return fail(MG_EINVAL, "LPT needs a base of at least 2^3 cells");
    if (order == 6 && H->lev[0].n[0] < 3) return fail(MG_EINVAL, "the sixth-order gradient needs a base of at least 3^3 cells");
    if (!phi) return fail(MG_EINVAL, "phi is NULL");
    for (int p = 0; p < H->nlev; ++p)
        if (!phi[p]) return fail(MG_EINVAL, "phi level pointer is NULL");
    Carver sz(nullptr);
    LptPlan tmp;
    const size_t need = lpt_carve(H, what, sz, tmp);
    if (!ws || ws_bytes < need) return fail(MG_EINVAL, "workspace too small: need " + std::to_string(need));
    if (((uintptr_t)ws) & 255) return fail(MG_EINVAL, "workspace must be 256-byte aligned");
    Carver cv(ws);
    lpt_carve(H, what, cv, lp);
    (void)hipGetLastError();
    if (H->nlev == 1) {
        lp.phi[0] = const_cast<double*>(phi[0]);
        return MG_OK;
    }
    for (int p = 0; p < H->nlev; ++p)
        MG_HIP(hipMemcpyAsync(lp.phi[p], phi[p], dims_of(H, p).cells() * sizeof(double), hipMemcpyDeviceToDevice, st));
    for (int p = H->nlev - 1; p >= 1; --p)
        launch_restrict_cov<double>(lp.phi[p], mklay(dims_of(H, p), 0), lp.phi[p - 1], parent_of(H, p), st);
    return MG_OK;
}

// ----------------------------------------------------------------------------------------------
// batched periodic solves
//
// Every instance keeps its own plan and workspace slice, exactly as a solo mg_solve_level would
// carve it.  The V-cycles of all instances run together: depth d of the schedule is level d of
// every instance whose single-workgroup tail starts below d, so one launch per step and depth
// covers them all; the tails of all instances are one launch of one workgroup each.  Each
// instance sees the same operations in the same order as its solo solve, and every batched
// kernel gives a block the same cells (and reduction striding) it has in a solo launch, so the
// results are bit-identical to mg_solve_level.  The fixed launch sequences are captured once as
// HIP graphs per workspace and batch shape and replayed for every cycle; a device flag per
// instance retires converged instances without changing the graphs.
// ----------------------------------------------------------------------------------------------

struct BLaunch {
    int off = 0, n = 0;      // segments [off, off + n) of the table
    unsigned grid = 0;       // blocks (sum of the segments' nblk)
    int block = kBlock, V = 1;
};

struct SmoothShape {
    int block = kBlock, V = 1;
};

enum { F_FSUM = 0, F_FNORM = 1, F_RNORM = 2, F_USUM = 3, F_COUNT = 4 };

struct BatchPlan {
    std::vector<int> ids;        // caller's index of each batched instance
    std::vector<Plan> P;
    int D = 0;                   // depths of grid levels (above every instance's tail)
    bool mixed = false;
    // static tables: [0] float, [1] double; float tables by parity of the finest correction buffer
    std::vector<BSeg> segs;
    std::vector<BLaunch> sm[2][2], rr[2][2], fas[2][2], pr[2][2];
    BLaunch outer[2], resid;
    std::vector<TailPlan<float>> tpf;
    std::vector<TailPlan<double>> tpd;
    unsigned lds_f = 0, lds_d = 0;
    std::vector<BFin> fins;      // F_COUNT tables of n entries
    // device side (in the workspace)
    BSeg* segs_dev = nullptr;
    size_t segs_cap = 0;         // table capacity (segments)
    TailPlan<float>* tpf_dev = nullptr;
    TailPlan<double>* tpd_dev = nullptr;
    BFin* fins_dev = nullptr;
    int* active_dev = nullptr;
    double* bscal = nullptr;     // n * S_COUNT scalars
    // ping-pong buffers of the finest level: A = the plan's u / u32, B = ualt / ealt
    std::vector<double*> Au, Bu;
    std::vector<float*> Ae, Be;
};

// blocks of batched half-sweep, FAS and black-prolongation segments (the kernels' own work
// decomposition decides them)
unsigned rbgs_split_blocks(const Lay& L, int block, int V);
unsigned fas_blocks(const Lay& C, const ParentMap& pm, int elem);
unsigned prolong_black_blocks(const Lay& L, const ParentMap& pm, int elem);

static bool batchable(int n) { return n % 2 == 0 && (size_t)n * n * n > kTailMaxCells; }

static BLaunch add_launch(std::vector<BSeg>& tab, std::vector<BSeg> segs, int block = kBlock, int V = 1) {
    BLaunch L;
    L.off = (int)tab.size();
    L.n = (int)segs.size();
    L.block = block;
    L.V = V;
    unsigned b = 0;
    for (auto& s : segs) {
        s.blk0 = b;
        b += s.nblk;
        tab.push_back(s);
    }
    L.grid = b;
    return L;
}

static unsigned cdiv(size_t a, size_t b) { return (unsigned)((a + b - 1) / b); }
static unsigned red_blocks(size_t cells) { return (unsigned)grid_for(cells, kBlock * kRedV, kMaxPartials); }

static BSeg seg0(int inst, unsigned nblk) {
    BSeg s{};
    s.inst = inst;
    s.nblk = nblk;
    s.L = Lay(Dims{1, 1, 1}, 0);
    s.C = Lay(Dims{1, 1, 1}, 0);
    return s;
}

template <class T> static T* ubuf(Level& L);
template <> double* ubuf<double>(Level& L) { return L.u; }
template <> float* ubuf<float>(Level& L) { return L.u32; }

// the V-cycle tables of precision T (ti = 0 float, 1 double); fine_u replaces level 0's u
template <class T>
static void vcycle_tables(BatchPlan& B, int ti, int par, const std::vector<T*>& fine_u,
                          const std::vector<SmoothShape>& shape) {
    auto& tab = B.segs;
    const int n = (int)B.P.size();
    B.sm[ti][par].assign(B.D, BLaunch{});
    B.rr[ti][par].assign(B.D, BLaunch{});
    B.fas[ti][par].assign(B.D, BLaunch{});
    B.pr[ti][par].assign(B.D, BLaunch{});
    for (int d = 0; d < B.D; ++d) {
        std::vector<BSeg> sm, rr, fa, pr;
        const SmoothShape sh = shape[d];
        for (int i = 0; i < n; ++i) {
            Plan& P = B.P[i];
            if (d >= P.tail) continue;
            Level& L = P.L[d];
            Level& Q = P.L[d + 1];
            ::mgic::B<T> b = bufs<T>(L), q = bufs<T>(Q);
            T* u = d == 0 ? fine_u[i] : b.u;
            const size_t cells = L.d.cells();
            const Lay C(Dims{L.d.x / 2, L.d.y / 2, L.d.z / 2}, 0);
            BSeg s = seg0(i, rbgs_split_blocks(L.lay, sh.block, sh.V));
            s.L = L.lay;
            s.h = L.h;
            s.a[0] = u;
            s.a[1] = b.f;
            sm.push_back(s);
            s = seg0(i, cdiv(C.d.cells(), kBlock));
            s.L = L.lay;
            s.C = C;
            s.pm = L.pm;
            s.h = L.h;
            s.a[0] = u; s.a[1] = b.f; s.a[2] = q.u; s.a[3] = q.f; s.a[4] = b.uold;
            rr.push_back(s);
            s = seg0(i, fas_blocks(C, L.pm, (int)sizeof(T)));
            s.C = C;
            s.pm = L.pm;
            s.h = Q.h;
            s.a[0] = q.u; s.a[1] = q.f;
            fa.push_back(s);
            s = seg0(i, B.P[i].nu2 > 0 ? prolong_black_blocks(L.lay, L.pm, (int)sizeof(T)) : cdiv(cells, kBlock));
            s.L = L.lay;
            s.pm = L.pm;
            s.a[0] = u; s.a[1] = q.u; s.a[2] = b.uold;
            pr.push_back(s);
        }
        B.sm[ti][par][d] = add_launch(tab, sm, sh.block, sh.V);
        B.rr[ti][par][d] = add_launch(tab, rr);
        B.fas[ti][par][d] = add_launch(tab, fa);
        B.pr[ti][par][d] = add_launch(tab, pr);
    }
}

template <class T>
static std::vector<TailPlan<T>> tail_plans(BatchPlan& B, unsigned& lds) {
    std::vector<TailPlan<T>> v;
    lds = 0;
    for (int i = 0; i < (int)B.P.size(); ++i) {
        Plan& P = B.P[i];
        TailPlan<T> tp{};
        tp.n = P.last - P.tail + 1;
        tp.nu1 = P.nu1;
        tp.nu2 = P.nu2;
        tp.inst = i;
        for (int k = 0; k < tp.n; ++k) {
            ::mgic::B<T> c = bufs<T>(P.L[P.tail + k]);
            tp.lev[k] = TailLevel<T>{c.u, c.f, P.L[P.tail + k].lay, P.L[P.tail + k].h, 0, 0, 0};
        }
        lds = std::max(lds, tail_assign_lds(tp));
        v.push_back(tp);
    }
    return v;
}

// size of the batch region after the instance slices (segment capacity for the static tables
// plus the per-call ones)
static size_t batch_segs_cap(const BatchPlan& B) {
    return (size_t)(12 * B.D + 12) * B.P.size() + 16;
}

// build plans (cv == null: sizes only); returns bytes of the whole workspace or 0 on error
static size_t batch_layout(int ninst, const int* n, const double* h, const mg_opts* o, char* ws, BatchPlan& B,
                           std::vector<size_t>& slice, std::vector<size_t>& slice_bytes) {
    size_t off = 0;
    slice.assign(ninst, 0);
    slice_bytes.assign(ninst, 0);
    B.ids.clear();
    B.P.clear();
    B.mixed = o && o->prec == MG_MIXED;
    for (int i = 0; i < ninst; ++i) {
        mg_hier H = single_level(n[i], h ? h[i] : 1.0);
        Plan P;
        Carver cv(nullptr);
        // batched instances run the one-step kernels (no fused levels); the others are solo solves
        if (build_plan(&H, o, cv, nullptr, P, !batchable(n[i]))) return 0;
        slice[i] = off;
        slice_bytes[i] = (cv.off + 255) & ~(size_t)255;
        off += slice_bytes[i];
        if (batchable(n[i])) {
            Plan Q;
            Carver c2(ws ? ws + slice[i] : nullptr);
            build_plan(&H, o, c2, nullptr, Q, false);
            B.ids.push_back(i);
            B.P.push_back(Q);
        }
    }
    B.D = 0;
    for (auto& P : B.P) B.D = std::max(B.D, P.tail);
    B.segs_cap = batch_segs_cap(B);
    const size_t ni = B.P.size();
    Carver cv(ws ? ws + off : nullptr);
    B.segs_dev = cv.take<BSeg>(B.segs_cap);
    B.tpf_dev = cv.take<TailPlan<float>>(ni);
    B.tpd_dev = cv.take<TailPlan<double>>(ni);
    B.fins_dev = cv.take<BFin>(F_COUNT * ni);
    B.active_dev = cv.take<int>(ni + 1);
    B.bscal = cv.take<double>((ni + 1) * S_COUNT);
    return off + cv.off;
}

// ---- autotuning of the batched smoother: block size and cells per thread, per depth ----------
static std::mutex g_tune_mu;
static std::map<std::string, std::vector<SmoothShape>> g_tune;

static std::string batch_key(const BatchPlan& B, int ti) {
    std::string k = std::to_string(ti) + ":" + std::to_string(B.P.empty() ? 0 : B.P[0].nu1) + ":";
    for (auto& P : B.P) k += std::to_string(P.L[0].d.x) + ",";
    return k;
}

static const SmoothShape kShapes[] = {{256, 1}, {256, 2}, {256, 4}, {128, 2}, {128, 4}, {512, 1}, {512, 2}};
constexpr int kNumShapes = (int)(sizeof(kShapes) / sizeof(kShapes[0]));
static int g_force_shape = -1;        // >= 0: every depth takes kShapes[g_force_shape], no timing
static std::string g_tune_path;       // JSON file the tuned shapes persist in ("" = none)
// tuned FP32 inner-cycle counts of mixed-precision solo solves, per problem shape (0: the rule)
static std::map<std::string, int> g_inner;

// shape of a solo solve for the inner-cycle table: the levels (sizes, offsets), the sweeps and the
// decade of the tolerance; spacings do not change the iteration's contraction
static std::string inner_key(const mg_hier* H, const mg_opts* o) {
    std::string k = "inner:" + std::to_string(o->nu1) + "," + std::to_string(o->nu2) + ":" +
                    std::to_string((int)std::lround(std::log10(o->tol > 0 ? o->tol : 1.0))) + ":";
    for (int p = 0; p < H->nlev; ++p) {
        const mg_level& l = H->lev[p];
        k += std::to_string(l.n[0]) + "," + std::to_string(l.n[1]) + "," + std::to_string(l.n[2]);
        if (p) k += "@" + std::to_string(l.off[0]) + "," + std::to_string(l.off[1]) + "," + std::to_string(l.off[2]);
        k += ";";
    }
    return k;
}

static thread_local bool g_tuning_inner = false;   // set while the tuner times the candidates

static int tuned_inner(const mg_hier* H, const mg_opts* o) {
    if (g_tuning_inner) return 0;
    std::lock_guard<std::mutex> g(g_tune_mu);
    auto it = g_inner.find(inner_key(H, o));
    return it == g_inner.end() ? 0 : it->second;
}

// The tuning cache file: {"format": "mgic-tuning-2", "entries": [{"key": "...", "shapes":
// [[block, cells per thread], ...]}, ..., {"key": "inner:...", "inner": k}, ...]}: the batched
// smoother's shapes per batch shape and precision, and the inner-cycle count per solo problem shape.
// Files of the earlier format "mgic-batch-smoother-tuning-1" (shapes only) are read as well.
static bool parse_tune_file(const std::string& text, std::map<std::string, std::vector<SmoothShape>>& out,
                            std::map<std::string, int>& inner) {
    if (text.find("\"mgic-batch-smoother-tuning-1\"") == std::string::npos &&
        text.find("\"mgic-tuning-2\"") == std::string::npos)
        return false;
    size_t pos = 0;
    while ((pos = text.find("\"key\"", pos)) != std::string::npos) {
        size_t q0 = text.find('"', text.find(':', pos) + 1);
        if (q0 == std::string::npos) return false;
        size_t q1 = text.find('"', q0 + 1);
        if (q1 == std::string::npos) return false;
        const std::string key = text.substr(q0 + 1, q1 - q0 - 1);
        const size_t next = text.find("\"key\"", q1);
        const size_t ai = text.find("\"inner\"", q1);
        if (ai != std::string::npos && ai < next) {
            int k = -1;
            if (std::sscanf(text.c_str() + text.find(':', ai) + 1, " %d", &k) != 1 || k < 0 || k > 16) return false;
            inner[key] = k;
            pos = ai;
            continue;
        }
        size_t a = text.find("\"shapes\"", q1);
        if (a == std::string::npos || a > next) return false;
        a = text.find('[', a);
        const size_t end = text.find("]]", a);
        if (a == std::string::npos || end == std::string::npos) return false;
        std::vector<SmoothShape> v;
        size_t i = a + 1;
        while (i < end) {
            const size_t b = text.find('[', i);
            if (b == std::string::npos || b > end) break;
            int blk = 0, cpt = 0;
            if (std::sscanf(text.c_str() + b, "[%d ,%d", &blk, &cpt) != 2 &&
                std::sscanf(text.c_str() + b, "[%d, %d", &blk, &cpt) != 2)
                return false;
            bool known = false;
            for (const SmoothShape& sh : kShapes) known = known || (sh.block == blk && sh.V == cpt);
            if (!known) return false;
            v.push_back(SmoothShape{blk, cpt});
            i = text.find(']', b) + 1;
        }
        out[key] = v;
        pos = end;
    }
    return true;
}

static void save_tune_file() {   // under g_tune_mu
    if (g_tune_path.empty()) return;
    std::string t = "{\"format\": \"mgic-tuning-2\", \"entries\": [";
    bool first = true;
    for (auto& kv : g_tune) {
        t += first ? "\n" : ",\n";
        first = false;
        t += "  {\"key\": \"" + kv.first + "\", \"shapes\": [";
        for (size_t i = 0; i < kv.second.size(); ++i)
            t += (i ? ", [" : "[") + std::to_string(kv.second[i].block) + ", " + std::to_string(kv.second[i].V) + "]";
        t += "]}";
    }
    for (auto& kv : g_inner) {
        t += first ? "\n" : ",\n";
        first = false;
        t += "  {\"key\": \"" + kv.first + "\", \"inner\": " + std::to_string(kv.second) + "}";
    }
    t += "\n]}\n";
    const std::string tmp = g_tune_path + ".tmp";
    if (FILE* fh = std::fopen(tmp.c_str(), "w")) {
        const bool ok = std::fwrite(t.data(), 1, t.size(), fh) == t.size();
        std::fclose(fh);
        if (ok) std::rename(tmp.c_str(), g_tune_path.c_str());
    }
}

template <class T>
static int tune_smoother(BatchPlan& B, int ti, hipStream_t st, std::vector<SmoothShape>& out) {
    const std::string key = batch_key(B, ti);
    {
        std::lock_guard<std::mutex> g(g_tune_mu);
        if (g_force_shape >= 0) {
            out.assign(B.D, kShapes[g_force_shape]);
            return MG_OK;
        }
        auto it = g_tune.find(key);
        if (it != g_tune.end() && (int)it->second.size() == B.D) {
            out = it->second;
            return MG_OK;
        }
    }
    out.assign(B.D, SmoothShape{});
    const int n = (int)B.P.size();
    std::vector<int> ones(n + 1, 1);
    MG_HIP(hipMemcpyAsync(B.active_dev, ones.data(), ones.size() * sizeof(int), hipMemcpyHostToDevice, st));
    hipEvent_t e0, e1;
    MG_HIP(hipEventCreate(&e0));
    MG_HIP(hipEventCreate(&e1));
    for (int d = 0; d < B.D; ++d) {
        float best = 1e30f;
        for (const SmoothShape& sh : kShapes) {
            std::vector<BSeg> tab, segs;
            for (int i = 0; i < n; ++i) {
                Plan& P = B.P[i];
                if (d >= P.tail) continue;
                Level& L = P.L[d];
                BSeg s = seg0(i, rbgs_split_blocks(L.lay, sh.block, sh.V));
                s.L = L.lay;
                s.h = L.h;
                s.a[0] = ubuf<T>(L);
                s.a[1] = bufs<T>(L).f;
                segs.push_back(s);
            }
            BLaunch la = add_launch(tab, segs, sh.block, sh.V);
            MG_HIP(hipMemcpyAsync(B.segs_dev, tab.data(), tab.size() * sizeof(BSeg), hipMemcpyHostToDevice, st));
            for (int r = 0; r < 2; ++r)
                launch_b_rbgs<T>(B.segs_dev, la.n, la.grid, la.block, la.V, B.active_dev, r & 1, st);
            MG_HIP(hipEventRecord(e0, st));
            const int reps = 6;
            for (int r = 0; r < reps; ++r)
                launch_b_rbgs<T>(B.segs_dev, la.n, la.grid, la.block, la.V, B.active_dev, r & 1, st);
            MG_HIP(hipEventRecord(e1, st));
            MG_HIP(hipEventSynchronize(e1));
            float ms = 0.f;
            MG_HIP(hipEventElapsedTime(&ms, e0, e1));
            if (ms < best) {
                best = ms;
                out[d] = sh;
            }
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    MG_HIP(hipGetLastError());
    std::lock_guard<std::mutex> g(g_tune_mu);
    g_tune[key] = out;
    save_tune_file();
    return MG_OK;
}

// pinned host mirror of the batch scalars and flags; reallocation drops the cached graphs that
// copy into it
static thread_local double* g_bpin = nullptr;
static thread_local size_t g_bpin_n = 0;
static double* batch_pinned(size_t n) {
    if (n <= g_bpin_n) return g_bpin;
    for (auto& kv : g_graphs.exec) (void)hipGraphExecDestroy(kv.second.ex);
    g_graphs.exec.clear();
    if (g_bpin) (void)hipHostFree(g_bpin);
    g_bpin = nullptr;
    g_bpin_n = 0;
    size_t cap = 1024;
    while (cap < n) cap *= 2;
    if (hipHostMalloc((void**)&g_bpin, cap * sizeof(double), hipHostMallocDefault) != hipSuccess) return nullptr;
    g_bpin_n = cap;
    return g_bpin;
}

// one batched V-cycle of precision T (ti: 0 float, 1 double) with the tables of parity par
template <class T>
static void b_vcycle(BatchPlan& B, int ti, int par, bool skip_first_red, hipStream_t st) {
    const int* act = B.active_dev;
    BSeg* sd = B.segs_dev;
    for (int d = 0; d < B.D; ++d) {
        const BLaunch& sm = B.sm[ti][par][d];
        for (int s = 0; s < B.P[0].nu1; ++s)
            for (int c = 0; c < 2; ++c) {
                if (skip_first_red && d == 0 && s == 0 && c == 0) continue;
                if (sm.n) launch_b_rbgs<T>(sd + sm.off, sm.n, sm.grid, sm.block, sm.V, act, c, st);
            }
        const BLaunch& rr = B.rr[ti][par][d];
        if (rr.n) launch_b_resid_restrict<T>(sd + rr.off, rr.n, rr.grid, act, st);
        const BLaunch& fa = B.fas[ti][par][d];
        if (fa.n) launch_b_fas<T>(sd + fa.off, fa.n, fa.grid, act, st);
    }
    if (ti == 0) launch_b_tail<float>(B.tpf_dev, (int)B.P.size(), B.lds_f, act, st);
    else launch_b_tail<double>(B.tpd_dev, (int)B.P.size(), B.lds_d, act, st);
    for (int d = B.D - 1; d >= 0; --d) {
        const BLaunch& pr = B.pr[ti][par][d];
        if (pr.n) launch_b_prolong<T>(sd + pr.off, pr.n, pr.grid, act, B.P[0].nu2 > 0, st);
        const BLaunch& sm = B.sm[ti][par][d];
        for (int s = 0; s < B.P[0].nu2; ++s)
            for (int c = 0; c < 2; ++c)
                if (sm.n) launch_b_rbgs<T>(sd + sm.off, sm.n, sm.grid, sm.block, sm.V, act, c, st);
    }
}

struct InstState {
    int cycles = 0, status = 1 /* running */, grow = 0, par = 0;
    double rel = NAN, prev = INFINITY, fnorm2 = 0;
    double check_prev = NAN;   // mixed: relative residual at the previous FP64 correction
    int last_inner = 0;        // mixed: inner cycles run since it
    bool active = true;
    bool early = false;   // stopped before the first cycle (non-finite source): u is not written
};

// codes (optional, ninst entries): each instance's own result (MG_OK / MG_ENOCONV / MG_EDIVERGED),
// filled when the call returns one of those
static int solve_batch(int ninst, const int* n, const double* h, const double* const* f, double* const* u,
                       const mg_opts* o, mg_stats* stats, void* ws, size_t ws_bytes, hipStream_t st,
                       int* codes = nullptr) {
    if (ninst < 1 || !n || !h || !f || !u || !o) return fail(MG_EINVAL, "NULL argument");
    if (o->max_cycles < 0) return fail(MG_EINVAL, "max_cycles < 0");
    if (o->prec != MG_FP64 && o->prec != MG_MIXED) return fail(MG_EINVAL, "unknown precision");
    if (o->inner < 0 || o->inner > 16) return fail(MG_EINVAL, "inner cycles out of range (0..16)");
    if (o->flags & MG_NO_MEAN_FIX) return fail(MG_EINVAL, "the batched solve always removes the mean (MG_NO_MEAN_FIX)");
    for (int i = 0; i < ninst; ++i)
        if (!f[i] || !u[i]) return fail(MG_EINVAL, "instance pointer is NULL");
    BatchPlan B;
    std::vector<size_t> slice, sbytes;
    const size_t need = batch_layout(ninst, n, h, o, nullptr, B, slice, sbytes);
    if (!need) return MG_EINVAL;   // build_plan reported the reason
    if (!ws || ws_bytes < need) return fail(MG_EINVAL, "workspace too small: need " + std::to_string(need));
    if (((uintptr_t)ws) & 255) return fail(MG_EINVAL, "workspace must be 256-byte aligned");
    if (int rc = refuse_capture(st, "the batched solve (it uploads tables and reads flags back)")) return rc;
    batch_layout(ninst, n, h, o, (char*)ws, B, slice, sbytes);
    (void)hipGetLastError();
    int worst = MG_OK;
    // instances outside the batched schedule (tiny or odd grids) are solved on their own
    std::vector<char> in_batch(ninst, 0);
    for (int i : B.ids) in_batch[i] = 1;
    for (int i = 0; i < ninst; ++i) {
        if (in_batch[i]) continue;
        mg_hier H = single_level(n[i], h[i]);
        const double* fp[1] = {f[i]};
        double* up[1] = {u[i]};
        const int rc = solve(&H, fp, up, o, stats ? stats + i : nullptr, (char*)ws + slice[i], sbytes[i], st);
        if (rc == MG_EINVAL || rc == MG_EHIP) return rc;
        if (rc && !worst) worst = rc;
        if (codes) codes[i] = rc;
    }
    const int ni = (int)B.P.size();
    if (!ni) return worst;
    const bool fixed = (o->flags & MG_FIXED_CYCLES) != 0;
    const bool guess = (o->flags & MG_USE_INITIAL_GUESS) != 0;
    const bool use_graph = (o->flags & MG_NO_GRAPH) == 0;
    B.mixed = o->prec == MG_MIXED;
    MG_HIP(batch_kernel_setup());   // function attributes must be set outside any graph capture
    for (int i = 0; i < ni; ++i) {
        Level& L = B.P[i].L[0];
        B.Au.push_back(L.u);
        B.Bu.push_back(L.ualt);
        B.Ae.push_back(L.u32);
        B.Be.push_back(L.ealt);
    }
    // autotuned smoother shapes (timed on the workspace before anything in it matters)
    std::vector<SmoothShape> shf, shd;
    int rc;
    if (B.mixed) {
        if ((rc = tune_smoother<float>(B, 0, st, shf))) return rc;
    } else {
        if ((rc = tune_smoother<double>(B, 1, st, shd))) return rc;
    }
    // static tables
    B.segs.clear();
    if (B.mixed) {
        vcycle_tables<float>(B, 0, 0, B.Be, shf);   // after an even outer step e lives in B
        vcycle_tables<float>(B, 0, 1, B.Ae, shf);
        B.tpf = tail_plans<float>(B, B.lds_f);
        if (B.lds_f > kTailLdsBound) return fail(MG_EINVAL, "internal: tail LDS above its bound");
        for (int par = 0; par < 2; ++par) {
            std::vector<BSeg> v;
            for (int i = 0; i < ni; ++i) {
                Level& L = B.P[i].L[0];
                BSeg s = seg0(i, red_blocks(L.d.cells()));
                s.L = L.lay;
                s.h = L.h;
                s.part = B.P[i].partials;
                s.a[0] = par ? B.Bu[i] : B.Au[i];
                s.a[1] = par ? B.Be[i] : B.Ae[i];
                s.a[2] = L.f;
                s.a[3] = par ? B.Au[i] : B.Bu[i];
                s.a[4] = L.f32;
                s.a[5] = par ? B.Ae[i] : B.Be[i];
                v.push_back(s);
            }
            B.outer[par] = add_launch(B.segs, v);
        }
    } else {
        std::vector<double*> fu(ni);
        for (int i = 0; i < ni; ++i) fu[i] = B.Au[i];
        vcycle_tables<double>(B, 1, 0, fu, shd);
        B.tpd = tail_plans<double>(B, B.lds_d);
        if (B.lds_d > kTailLdsBound) return fail(MG_EINVAL, "internal: tail LDS above its bound");
        std::vector<BSeg> v;
        for (int i = 0; i < ni; ++i) {
            Level& L = B.P[i].L[0];
            BSeg s = seg0(i, red_blocks(L.d.cells()));
            s.L = L.lay;
            s.h = L.h;
            s.part = B.P[i].partials;
            s.a[0] = L.u;
            s.a[1] = L.f;
            v.push_back(s);
        }
        B.resid = add_launch(B.segs, v);
    }
    B.fins.assign((size_t)F_COUNT * ni, BFin{});
    for (int i = 0; i < ni; ++i) {
        Level& L = B.P[i].L[0];
        const double h3 = L.h * L.h * L.h;
        const int cnt = (int)red_blocks(L.d.cells());
        double* sc = B.bscal + (size_t)i * S_COUNT;
        B.fins[F_FSUM * ni + i] = BFin{B.P[i].partials, cnt, 1.0, sc + S_FSUM};
        B.fins[F_FNORM * ni + i] = BFin{B.P[i].partials, cnt, h3, sc + S_FNORM};
        B.fins[F_RNORM * ni + i] = BFin{B.P[i].partials, cnt, h3, sc + S_RNORM};
        B.fins[F_USUM * ni + i] = BFin{B.P[i].partials, cnt, 1.0, sc + S_USUM};
    }
    // per-call tables: input and output conversions, initial guess, gauge (user pointers)
    std::vector<BSeg> fin_rel, sub_f, uinit;
    for (int i = 0; i < ni; ++i) {
        Level& L = B.P[i].L[0];
        const int id = B.ids[i];
        const size_t cells = L.d.cells();
        BSeg s = seg0(i, red_blocks(cells));      // copy-in with the sum (as the solo solve)
        s.L = L.lay;
        s.part = B.P[i].partials;
        s.a[0] = (void*)f[id];
        s.a[1] = L.f;
        fin_rel.push_back(s);
        s = seg0(i, red_blocks(cells));           // mean removal with the sum of squares
        s.L = L.lay;
        s.h = 1.0 / (double)cells;
        s.part = B.P[i].partials;
        s.a[0] = L.f;
        s.a[1] = B.bscal + (size_t)i * S_COUNT + S_FSUM;
        sub_f.push_back(s);
        if (guess) {
            s = seg0(i, (unsigned)grid_for(cells, kBlock, 8192));
            s.L = Lay(L.d, 0);
            s.C = L.lay;
            s.a[0] = u[id];
            s.a[1] = B.Au[i];
        } else {
            s = seg0(i, (unsigned)grid_for(cells, kBlock, 4096));
            s.L = L.lay;
            s.a[0] = B.Au[i];
        }
        uinit.push_back(s);
    }
    const BLaunch la_frel = add_launch(B.segs, fin_rel);
    const BLaunch la_subf = add_launch(B.segs, sub_f);
    const BLaunch la_uinit = add_launch(B.segs, uinit);
    const size_t out_off = B.segs.size();   // output tables are filled in at the end
    if (out_off + 3 * (size_t)ni > B.segs_cap) return fail(MG_EINVAL, "internal: batch table overflow");

    double* pin = batch_pinned((size_t)(ni + 1) * S_COUNT + ni + 1);
    if (!pin) return fail(MG_EHIP, "pinned host buffer unavailable");
    int* pflags = (int*)(pin + (size_t)(ni + 1) * S_COUNT);
    MG_HIP(hipMemcpyAsync(B.segs_dev, B.segs.data(), B.segs.size() * sizeof(BSeg), hipMemcpyHostToDevice, st));
    if (!B.tpf.empty())
        MG_HIP(hipMemcpyAsync(B.tpf_dev, B.tpf.data(), B.tpf.size() * sizeof(TailPlan<float>), hipMemcpyHostToDevice, st));
    if (!B.tpd.empty())
        MG_HIP(hipMemcpyAsync(B.tpd_dev, B.tpd.data(), B.tpd.size() * sizeof(TailPlan<double>), hipMemcpyHostToDevice, st));
    MG_HIP(hipMemcpyAsync(B.fins_dev, B.fins.data(), B.fins.size() * sizeof(BFin), hipMemcpyHostToDevice, st));
    std::vector<InstState> S(ni);
    std::vector<int> sent(ni, -1);
    // device flags follow S[i].active; the pinned source is rewritten only after the stream has
    // drained, since an earlier upload may still be reading it
    auto upload_flags = [&]() -> int {
        bool same = true;
        for (int i = 0; i < ni; ++i) same = same && sent[i] == (S[i].active ? 1 : 0);
        if (same) return MG_OK;
        MG_HIP(hipStreamSynchronize(st));
        for (int i = 0; i < ni; ++i) pflags[i] = sent[i] = S[i].active ? 1 : 0;
        MG_HIP(hipMemcpyAsync(B.active_dev, pflags, ni * sizeof(int), hipMemcpyHostToDevice, st));
        return MG_OK;
    };
    if ((rc = upload_flags())) return rc;
    BSeg* sd = B.segs_dev;
    const int* act = B.active_dev;
    const size_t nscal = (size_t)ni * S_COUNT;

    // source preparation (a1): working copy, mean, mean removal, norm
    launch_b_relayout_sum(sd + la_frel.off, la_frel.n, la_frel.grid, act, st);
    launch_b_finalize(B.fins_dev + F_FSUM * ni, ni, act, st);
    launch_b_submean_sumsq(sd + la_subf.off, la_subf.n, la_subf.grid, act, st);
    launch_b_finalize(B.fins_dev + F_FNORM * ni, ni, act, st);
    // a zero start of the mixed path needs no fill (its first outer step takes u as zero)
    if (guess) launch_b_relayout(sd + la_uinit.off, la_uinit.n, la_uinit.grid, act, st);
    else if (!B.mixed) launch_b_zero<double>(sd + la_uinit.off, la_uinit.n, la_uinit.grid, act, st);
    MG_HIP(hipMemcpyAsync(pin, B.bscal, nscal * sizeof(double), hipMemcpyDeviceToHost, st));
    MG_HIP(hipStreamSynchronize(st));
    std::vector<mg_stats> out(ni);
    for (int i = 0; i < ni; ++i) {
        std::memset(&out[i], 0, sizeof(mg_stats));
        for (double& v : out[i].res_hist) v = NAN;
        const double fsum = pin[(size_t)i * S_COUNT + S_FSUM], fn2 = pin[(size_t)i * S_COUNT + S_FNORM];
        out[i].f_mean_removed = fixed ? 0.0 : fsum / (double)B.P[i].L[0].d.cells();
        S[i].fnorm2 = fn2;
        if (!fixed && (!std::isfinite(fn2) || !std::isfinite(fsum))) {
            S[i].status = MG_EDIVERGED;
            S[i].active = false;
            S[i].early = true;
        }
    }
    if ((rc = upload_flags())) return rc;

    auto check = [&](int i, double r2) -> int {
        InstState& s = S[i];
        s.rel = s.fnorm2 > 0 ? std::sqrt(r2 / s.fnorm2) : 0.0;
        if (s.cycles >= 1 && s.cycles <= 64) out[i].res_hist[s.cycles - 1] = s.rel;
        if (!std::isfinite(s.rel)) return MG_EDIVERGED;
        s.grow = s.rel > s.prev ? s.grow + 1 : 0;
        s.prev = s.rel;
        if (s.grow >= 3) return MG_EDIVERGED;
        return s.rel <= o->tol ? MG_OK : 1;
    };
    auto any_active = [&]() {
        for (auto& s : S)
            if (s.active) return true;
        return false;
    };
    // residual readback and convergence decisions of the active instances
    auto decide = [&](int par) {
        for (int i = 0; i < ni; ++i) {
            if (!S[i].active) continue;
            S[i].par = par;
            if (!fixed) {
                const int c = check(i, pin[(size_t)i * S_COUNT + S_RNORM]);
                if (c != 1) {
                    S[i].status = c;
                    S[i].active = false;
                    continue;
                }
            }
            if (S[i].cycles >= o->max_cycles) {
                S[i].status = fixed ? MG_OK : MG_ENOCONV;
                S[i].active = false;
            }
        }
    };
    std::string shape_tag;
    for (const SmoothShape& sh : B.mixed ? shf : shd) shape_tag += std::to_string(sh.block) + "x" + std::to_string(sh.V) + ",";
    const std::string wkey = std::to_string((uintptr_t)ws) + "|" + batch_key(B, B.mixed ? 0 : 1) + "|" + shape_tag + "|" +
                             std::to_string(o->nu2) + "|" +
                             std::to_string(B.segs.size()) + "|" + (fixed ? "f" : "c");
    if (B.mixed) {
        bool first = true;
        int par = 0;
        while (any_active()) {
            const std::string k = wkey + (first ? (guess ? "|outer0g" : "|outer0z") : (par ? "|outer1" : "|outer2"));
            rc = run_graph(use_graph, k, st, [&](hipStream_t s) {
                const BLaunch& ol = B.outer[par];
                launch_b_outer(sd + ol.off, ol.n, ol.grid, act, first ? 0 : 1, (first && !guess) ? 1 : 0, s);
                launch_b_finalize(B.fins_dev + F_RNORM * ni, ni, act, s);
                (void)hipMemcpyAsync(pin, B.bscal, nscal * sizeof(double), hipMemcpyDeviceToHost, s);
            });
            if (rc) return rc;
            if (!fixed) MG_HIP(hipStreamSynchronize(st));
            decide(par);
            if (!any_active()) break;
            // inner cycles per instance by the same rule as a solo solve; the k-th cycle of the
            // round runs on the instances that asked for more than k (one graph per cycle)
            std::vector<int> nin(ni, 0);
            std::vector<char> solving(ni, 0);
            int rounds = 0;
            for (int i = 0; i < ni; ++i) {
                solving[i] = S[i].active;
                if (!S[i].active) continue;
                nin[i] = std::min(inner_count(o->inner, fixed, S[i].rel, S[i].check_prev, S[i].last_inner, o->tol),
                                  o->max_cycles - S[i].cycles);
                S[i].check_prev = S[i].rel;
                S[i].last_inner = nin[i];
                rounds = std::max(rounds, nin[i]);
            }
            for (int k = 0; k < rounds; ++k) {
                for (int i = 0; i < ni; ++i) S[i].active = solving[i] && k < nin[i];
                if ((rc = upload_flags())) return rc;
                rc = run_graph(use_graph, wkey + "|vc" + std::to_string(par) + (k == 0 ? "f" : "n"), st,
                               [&](hipStream_t s) { b_vcycle<float>(B, 0, par, k == 0, s); });
                if (rc) return rc;
                for (int i = 0; i < ni; ++i)
                    if (S[i].active) {
                        ++S[i].cycles;
                        out[i].cell_updates += updates_per_cycle(B.P[i]);
                    }
            }
            for (int i = 0; i < ni; ++i) S[i].active = solving[i];
            if ((rc = upload_flags())) return rc;
            first = false;
            par ^= 1;
        }
    } else {
        if (guess && !fixed) {
            launch_b_residual(sd + B.resid.off, B.resid.n, B.resid.grid, act, st);
            launch_b_finalize(B.fins_dev + F_RNORM * ni, ni, act, st);
            MG_HIP(hipMemcpyAsync(pin, B.bscal, nscal * sizeof(double), hipMemcpyDeviceToHost, st));
            MG_HIP(hipStreamSynchronize(st));
            for (int i = 0; i < ni; ++i) {
                if (!S[i].active) continue;
                const int c = check(i, pin[(size_t)i * S_COUNT + S_RNORM]);
                if (c != 1) {   // converged already, or NaN/Inf in the initial guess
                    S[i].status = c;
                    S[i].active = false;
                }
            }
            if ((rc = upload_flags())) return rc;
        }
        for (int i = 0; i < ni; ++i)
            if (S[i].active && S[i].cycles >= o->max_cycles) {
                S[i].status = fixed ? MG_OK : MG_ENOCONV;
                S[i].active = false;
            }
        if ((rc = upload_flags())) return rc;
        while (any_active()) {
            rc = run_graph(use_graph, wkey + "|cycle64", st, [&](hipStream_t s) {
                b_vcycle<double>(B, 1, 0, false, s);
                if (!fixed) {
                    launch_b_residual(sd + B.resid.off, B.resid.n, B.resid.grid, act, s);
                    launch_b_finalize(B.fins_dev + F_RNORM * ni, ni, act, s);
                    (void)hipMemcpyAsync(pin, B.bscal, nscal * sizeof(double), hipMemcpyDeviceToHost, s);
                }
            });
            if (rc) return rc;
            if (!fixed) MG_HIP(hipStreamSynchronize(st));
            for (int i = 0; i < ni; ++i)
                if (S[i].active) {
                    ++S[i].cycles;
                    out[i].cell_updates += updates_per_cycle(B.P[i]);
                }
            decide(0);
            if ((rc = upload_flags())) return rc;
        }
    }
    // gauge (zero mean) and conversion back, for every instance that reached the loop
    std::vector<BSeg> osum, orel;
    for (int i = 0; i < ni; ++i) {
        S[i].active = !S[i].early;
        Level& L = B.P[i].L[0];
        double* uf = !B.mixed ? L.u : (S[i].par ? B.Au[i] : B.Bu[i]);
        const size_t cells = L.d.cells();
        BSeg s = seg0(i, red_blocks(cells));
        s.L = L.lay;
        s.part = B.P[i].partials;
        s.a[0] = uf;
        osum.push_back(s);
        s = seg0(i, (unsigned)grid_for(cells, kBlock, 8192));   // copy back with the mean removed
        s.L = L.lay;
        s.C = Lay(L.d, 0);
        s.h = 1.0 / (double)cells;
        s.a[0] = uf;
        s.a[1] = u[B.ids[i]];
        s.a[2] = B.bscal + (size_t)i * S_COUNT + S_USUM;
        orel.push_back(s);
    }
    std::vector<BSeg> tail_tab(B.segs.begin(), B.segs.begin() + out_off);
    const BLaunch la_osum = add_launch(tail_tab, osum);
    const BLaunch la_orel = add_launch(tail_tab, orel);
    MG_HIP(hipMemcpyAsync(sd + out_off, tail_tab.data() + out_off, (tail_tab.size() - out_off) * sizeof(BSeg),
                          hipMemcpyHostToDevice, st));
    if ((rc = upload_flags())) return rc;
    launch_b_sum(sd + la_osum.off, la_osum.n, la_osum.grid, act, 0, st);
    launch_b_finalize(B.fins_dev + F_USUM * ni, ni, act, st);
    launch_b_relayout_sub(sd + la_orel.off, la_orel.n, la_orel.grid, act, st);
    MG_HIP(hipGetLastError());
    MG_HIP(hipStreamSynchronize(st));
    for (int i = 0; i < ni; ++i) {
        out[i].cycles = S[i].cycles;
        out[i].rel_res = S[i].rel;
        if (stats) stats[B.ids[i]] = out[i];
    }
    // the first failure in instance order decides the return code
    std::vector<int> code(ninst, MG_OK);
    for (int i = 0; i < ni; ++i) code[B.ids[i]] = S[i].status;
    if (codes)
        for (int i = 0; i < ninst; ++i)
            if (in_batch[i]) codes[i] = code[i];
    for (int i = 0; i < ninst; ++i)
        if (in_batch[i] && code[i] != MG_OK && !worst) worst = code[i];
    if (worst == MG_ENOCONV) return fail(MG_ENOCONV, "an instance did not converge within max_cycles");
    if (worst == MG_EDIVERGED) return fail(MG_EDIVERGED, "an instance diverged (NaN/Inf or growth)");
    return worst;
}

// the batched periodic solves with each instance's own result code (for the hierarchy batch)
int solve_batch_codes(int ninst, const int* n, const double* h, const double* const* f, double* const* u,
                      const mg_opts* o, mg_stats* stats, int* codes, void* ws, size_t ws_bytes, hipStream_t st) {
    return solve_batch(ninst, n, h, f, u, o, stats, ws, ws_bytes, st, codes);
}

static size_t batch_bytes(int ninst, const int* n, const mg_opts* o) {
    if (ninst < 1 || !n) return 0;
    BatchPlan B;
    std::vector<double> h(ninst, 1.0);
    std::vector<size_t> slice, sbytes;
    mg_opts oo{};
    if (o) oo = *o;
    return batch_layout(ninst, n, h.data(), o ? &oo : nullptr, nullptr, B, slice, sbytes);
}

}  // namespace mgic

// ==============================================================================================
// C ABI
// ==============================================================================================
using namespace mgic;

// ----------------------------------------------------------------------------------------------
// periodic FAS with the order-2/4/6 Laplacians of Table 1 (Section 3.2): n = 2^lg, FP64
// ----------------------------------------------------------------------------------------------
struct HoPlan {
    int lg = 0, order = 2, nlev = 0;     // levels l = 0..nlev-1 have 2^(lg-l) cells per axis
    double h = 1.0;
    double* u[12]{};      // level 0: the caller's array
    double* f[12]{};      // level 0: f minus its mean; coarser levels: the FAS right-hand side
    double* uold[12]{};   // the restricted iterate before the coarse solve (levels >= 1)
    double* tmp[12]{};    // the other buffer of the out-of-place half-sweeps (levels with 2^3+ cells)
    float* e32[12]{};     // mixed precision: the FP32 correction and its V-cycle arrays, every level
    float* f32[12]{};     // (level 0: the FP64 residual rounded to FP32)
    float* uold32[12]{};
    float* tmp32[12]{};
    double* part = nullptr;
    double* scal = nullptr;   // [0] sum f, [1] sum (f - mean)^2, [2] sum r^2, [3] sum u, [4] unused
};

template <class T> struct HoArr { T* const* u; T* const* f; T* const* uold; T* const* tmp; };
static HoArr<double> ho_arr(const HoPlan& P, double) { return {P.u, P.f, P.uold, P.tmp}; }
static HoArr<float> ho_arr(const HoPlan& P, float) { return {P.e32, P.f32, P.uold32, P.tmp32}; }

static int ho_plan(int n, double h, int order, Carver& cv, double* u, HoPlan& P) {
    const int lg = log2_exact(n);
    if (lg < 1 || lg > 10) return fail(MG_EINVAL, "higher-order solve: n must be a power of two in 2..1024");
    if (order != 2 && order != 4 && order != 6) return fail(MG_EINVAL, "order must be 2, 4 or 6");
    if (!(h > 0) || !std::isfinite(h)) return fail(MG_EINVAL, "h must be positive and finite");
    P.lg = lg;
    P.order = order;
    P.h = h;
    P.nlev = lg + 1;
    for (int l = 0; l < P.nlev; ++l) {
        const size_t cells = (size_t)1 << (3 * (lg - l));
        P.u[l] = l == 0 ? u : cv.take<double>(cells);
        P.f[l] = cv.take<double>(cells);
        if (l > 0) P.uold[l] = cv.take<double>(cells);
        if (l < lg) P.tmp[l] = cv.take<double>(cells);
    }
    for (int l = 0; l < P.nlev; ++l) {   // the FP32 arrays are reserved whatever the precision
        const size_t cells = (size_t)1 << (3 * (lg - l));
        P.e32[l] = cv.take<float>(cells);
        P.f32[l] = cv.take<float>(cells);
        if (l > 0) P.uold32[l] = cv.take<float>(cells);
        if (l < lg) P.tmp32[l] = cv.take<float>(cells);
    }
    P.part = cv.take<double>(kHoParts);
    P.scal = cv.take<double>(8);
    return MG_OK;
}

static int ho_read(const double* dev, int count, double* out, hipStream_t st) {
    double* pin = pinned_scratch();
    if (!pin) return fail(MG_EHIP, "pinned host buffer unavailable");
    MG_HIP(hipMemcpyAsync(pin, dev, count * sizeof(double), hipMemcpyDeviceToHost, st));
    MG_HIP(hipStreamSynchronize(st));
    for (int i = 0; i < count; ++i) out[i] = pin[i];
    return MG_OK;
}

template <class T>
static void ho_smooth(HoPlan& P, const HoArr<T>& A, int l, int sweeps, hipStream_t st) {
    const int lg = P.lg - l;
    const double h = std::ldexp(P.h, l);
    const double half_bytes = 3.0 * sizeof(T) * (double)((size_t)1 << (3 * lg));   // in, f read; out written
    for (int s = 0; s < sweeps; ++s)
        for (int c = 0; c < 2; ++c) {
            KEvents ev(l == 0);
            const T* in = c == 0 ? A.u[l] : A.tmp[l];
            T* out = c == 0 ? A.tmp[l] : A.u[l];
            launch_ho_half<T>(in, out, A.f[l], lg, h, P.order, c, st, ev.a, ev.b);
            ev.done(half_bytes);
        }
}

template <class T>
static void ho_vcycle(HoPlan& P, int nu1, int nu2, hipStream_t st) {
    const HoArr<T> A = ho_arr(P, T(0));
    const int L = P.nlev - 1;   // the single-cell level
    for (int l = 0; l < L; ++l) {
        ho_smooth<T>(P, A, l, nu1, st);
        const int lgc = P.lg - l - 1;
        launch_ho_resid_restrict<T>(A.u[l], A.f[l], A.u[l + 1], A.uold[l + 1], A.f[l + 1], lgc, std::ldexp(P.h, l),
                                    P.order, st);
        launch_ho_fas<T>(A.u[l + 1], A.f[l + 1], lgc, std::ldexp(P.h, l + 1), P.order, st);
    }
    launch_ho_fill<T>(A.u[L], 0, T(0), st);   // one cell: u = 0
    for (int l = L - 1; l >= 0; --l) {
        launch_ho_prolong<T>(A.u[l], A.u[l + 1], A.uold[l + 1], P.lg - l, st);
        ho_smooth<T>(P, A, l, nu2, st);
    }
}

extern "C" {

size_t mg_ho_workspace_bytes(int n, int order) {
    HoPlan P;
    Carver cv(nullptr);
    if (ho_plan(n, 1.0, order, cv, nullptr, P)) return 0;
    return cv.off;
}

int mg_solve_level_ho(int n, double h, int order, const double* f, double* u, const mg_opts* o, mg_stats* stats,
                      void* ws, size_t ws_bytes, void* stream) {
    hipStream_t st = (hipStream_t)stream;
    if (!o) return fail(MG_EINVAL, "options are NULL");
    if (!f || !u) return fail(MG_EINVAL, "f or u is NULL");
    if (o->max_cycles < 0) return fail(MG_EINVAL, "max_cycles < 0");
    if (o->prec != MG_FP64 && o->prec != MG_MIXED) return fail(MG_EINVAL, "unknown precision");
    if (o->inner < 0 || o->inner > 16) return fail(MG_EINVAL, "inner cycles out of range (0..16)");
    if (o->nu1 < 0 || o->nu2 < 0 || o->nu1 + o->nu2 > 64) return fail(MG_EINVAL, "nu1/nu2 out of range");
    if (o->flags & ~(MG_USE_INITIAL_GUESS | MG_FIXED_CYCLES)) return fail(MG_EINVAL, "unknown flags");
    // the finest level iterates in the caller's u, which the kernels access as 16-byte pairs
    if ((uintptr_t)u & 15) return fail(MG_EINVAL, "u must be 16-byte aligned");
    HoPlan P;
    Carver size_cv(nullptr);
    int rc = ho_plan(n, h, order, size_cv, u, P);
    if (rc) return rc;
    if (!ws || ws_bytes < size_cv.off) return fail(MG_EINVAL, "workspace too small: need " + std::to_string(size_cv.off));
    if (((uintptr_t)ws) & 255) return fail(MG_EINVAL, "workspace must be 256-byte aligned");
    if ((rc = refuse_capture(st, "the higher-order solve"))) return rc;
    Carver cv(ws);
    ho_plan(n, h, order, cv, u, P);
    (void)hipGetLastError();

    const bool fixed = (o->flags & MG_FIXED_CYCLES) != 0;
    const bool guess = (o->flags & MG_USE_INITIAL_GUESS) != 0;
    const int lg = P.lg;
    const double cells = (double)((size_t)1 << (3 * lg));
    mg_stats S;
    std::memset(&S, 0, sizeof(S));
    for (double& v : S.res_hist) v = NAN;
    launch_ho_sum(f, lg, P.part, P.scal + 0, st);                          // composite mean of f ...
    launch_ho_sub(f, P.scal + 0, P.f[0], lg, P.part, P.scal + 1, st);      // ... removed, and |f|^2
    if (!guess) launch_ho_fill<double>(P.u[0], lg, 0.0, st);
    double fnorm2 = 0.0;
    if (!fixed) {
        double fs[2];
        if ((rc = ho_read(P.scal, 2, fs, st))) return rc;
        S.f_mean_removed = fs[0] / cells;
        fnorm2 = fs[1];
        if (!std::isfinite(fs[0]) || !std::isfinite(fs[1])) {
            S.rel_res = NAN;
            if (stats) *stats = S;
            return fail(MG_EDIVERGED, "right-hand side contains NaN or Inf");
        }
    }
    long long upc = 0;
    for (int l = 0; l < lg; ++l) upc += (long long)(o->nu1 + o->nu2) << (3 * (lg - l));
    double rel = NAN, prev = INFINITY;
    int grow = 0, status = MG_ENOCONV, cycles = 0;
    const bool mixed = o->prec == MG_MIXED;
    auto check = [&]() -> int {
        double r2;
        if (mixed) launch_ho_resid32(P.u[0], P.f[0], P.f32[0], lg, h, order, P.part, P.scal + 2, st);
        else launch_ho_rnorm(P.u[0], P.f[0], lg, h, order, P.part, P.scal + 2, st);
        if (int e = ho_read(P.scal + 2, 1, &r2, st)) return e;
        rel = fnorm2 > 0 ? std::sqrt(r2 / fnorm2) : 0.0;
        if (cycles >= 1 && cycles <= 64) S.res_hist[cycles - 1] = rel;
        if (!std::isfinite(rel)) return MG_EDIVERGED;
        grow = rel > prev ? grow + 1 : 0;
        prev = rel;
        if (grow >= 3) return MG_EDIVERGED;
        return rel <= o->tol ? MG_OK : 1;
    };
    if (!mixed) {
        if (guess && !fixed) {
            const int c = check();
            if (c == MG_OK) status = MG_OK;
            else if (c == MG_EHIP) return c;
            else if (c == MG_EDIVERGED) status = MG_EDIVERGED;   // a NaN or Inf guess
        }
        while (status == MG_ENOCONV && cycles < o->max_cycles) {
            ho_vcycle<double>(P, o->nu1, o->nu2, st);
            ++cycles;
            S.cell_updates += upc;
            if (fixed) continue;
            const int c = check();
            if (c == MG_OK) status = MG_OK;
            else if (c == MG_EHIP) return c;
            else if (c == MG_EDIVERGED) { status = MG_EDIVERGED; break; }
        }
    } else {
        // defect correction: the FP64 residual (rounded to FP32) is the right-hand side of `inner`
        // FP32 V-cycles from e = 0, and u += e; the stopping test is on the FP64 residual.  By
        // default 3 per correction: at 256^3 that measured faster than the 7-point path's rule
        // chosen from the contraction (7.8 against 9.4 ms at order 4, 13.2 against 12.9 at order 6).
        const int inner = o->inner > 0 ? o->inner : 3;
        for (;;) {
            if (fixed) {
                if (cycles >= o->max_cycles) break;
                launch_ho_resid32(P.u[0], P.f[0], P.f32[0], lg, h, order, P.part, P.scal + 2, st);
            } else {
                const int c = check();
                if (c == MG_OK) { status = MG_OK; break; }
                if (c == MG_EHIP) return c;
                if (c == MG_EDIVERGED) { status = MG_EDIVERGED; break; }
                if (cycles >= o->max_cycles) break;
            }
            launch_ho_fill<float>(P.e32[0], lg, 0.0f, st);
            const int k = std::min(inner, o->max_cycles - cycles);
            for (int i = 0; i < k; ++i) {
                ho_vcycle<float>(P, o->nu1, o->nu2, st);
                ++cycles;
                S.cell_updates += upc;
            }
            launch_ho_add32(P.u[0], P.e32[0], lg, st);
        }
    }
    if (fixed) status = MG_OK;
    launch_ho_sum(P.u[0], lg, P.part, P.scal + 3, st);                     // zero-mean gauge of u
    launch_ho_sub(P.u[0], P.scal + 3, P.u[0], lg, P.part, P.scal + 4, st);
    MG_HIP(hipGetLastError());
    S.cycles = cycles;
    S.rel_res = fixed ? NAN : rel;
    if (stats) *stats = S;
    if (status == MG_ENOCONV) return fail(MG_ENOCONV, "no convergence within max_cycles");
    if (status == MG_EDIVERGED) return fail(MG_EDIVERGED, "residual diverged");
    return MG_OK;
}

}  // extern "C"

// ----------------------------------------------------------------------------------------------
// higher-order Laplacians on nested patches (Section 3.3 with Tables 1 and 2), FP64: patches in
// natural order with R = order / 2 ghost layers per face; the base and its coarsenings run the
// periodic higher-order V-cycle above
// ----------------------------------------------------------------------------------------------
struct HozLevel {
    HozPatch P{};
    double *u = nullptr, *f = nullptr, *tmp = nullptr, *g = nullptr, *uold = nullptr;
    double* gpart = nullptr;   // the parent's part of the ghosts, kept between the fills of a pass
    int cov_lo[3] = {0, 0, 0}, cov_n[3] = {0, 0, 0};   // box covered by the next patch (n = 0: none)
};

struct HozPlan {
    int order = 4, R = 2, np = 0, N0 = 0;
    double h0 = 1.0;
    double* ubase = nullptr;
    HoPlan base;                      // base.u[0] = ubase, base.f[0] = the base right-hand side
    std::vector<HozLevel> pat;        // pat[p - 1] = patch p
    int base_cov_lo[3] = {0, 0, 0}, base_cov_n[3] = {0, 0, 0};
    HozW W{};
    double* part = nullptr;           // kHozParts per level (at least kHoParts)
    double* scal = nullptr;           // [0] sum f, [1] |f|^2, [2] |r|^2, [3] sum u
};

static std::vector<double> lagrange_w(const std::vector<double>& nodes, double x) {
    std::vector<double> w;
    for (size_t i = 0; i < nodes.size(); ++i) {
        double num = 1.0, den = 1.0;
        for (size_t j = 0; j < nodes.size(); ++j)
            if (j != i) {
                num *= x - nodes[j];
                den *= nodes[i] - nodes[j];
            }
        w.push_back(num / den);
    }
    return w;
}

static HozW hoz_weights(int order) {
    const int R = order / 2;
    HozW W{};
    std::vector<double> par;
    for (int k = -R; k <= R; ++k) par.push_back(k);
    for (int side = 0; side < 2; ++side) {
        const std::vector<double> w = lagrange_w(par, side ? 0.25 : -0.25);
        for (size_t i = 0; i < w.size(); ++i) W.par[side][i] = w[i];
    }
    std::vector<double> nodes;
    for (int k = 0; k < R; ++k) nodes.push_back(-(2.0 * k + 1.0));
    for (int i = 0; i <= R; ++i) nodes.push_back(i + 0.5);
    for (int gl = 0; gl < R; ++gl) {
        const std::vector<double> w = lagrange_w(nodes, -(gl + 0.5));
        for (size_t i = 0; i < w.size(); ++i) W.nor[gl][i] = w[i];
    }
    // Table 2: flux operators of order 1, 3, 5 over the 2R cells around a face, outside first
    static const int F1[2] = {-1, 1}, F3[4] = {-1, 15, -15, 1}, F5[6] = {2, -25, 245, -245, 25, -2};
    const int* F = R == 1 ? F1 : (R == 2 ? F3 : F5);
    const double den = R == 1 ? 1.0 : (R == 2 ? 12.0 : 180.0);
    W.S = 0.0;
    for (int m = 0; m < 2 * R; ++m) {
        W.F[m] = F[m] / den;
        if (m < R) W.S += W.F[m];
    }
    return W;
}

static int hoz_plan(const mg_hier* H, int order, Carver& cv, HozPlan& Z) {
    if (int v = validate_hier(H)) return v;
    if (order != 2 && order != 4 && order != 6) return fail(MG_EINVAL, "order must be 2, 4 or 6");
    const int R = order / 2;
    Z.order = order;
    Z.R = R;
    Z.np = H->nlev - 1;
    Z.N0 = H->lev[0].n[0];
    Z.h0 = H->lev[0].h;
    if (log2_exact(Z.N0) < 1 || Z.N0 > 1024) return fail(MG_EINVAL, "higher-order hierarchy: base n must be a power of two in 2..1024");
    for (int p = 1; p <= Z.np; ++p)
        for (int a = 0; a < 3; ++a) {
            if (H->lev[p].n[a] < 2 * R) return fail(MG_EINVAL, "higher-order hierarchy: patch sizes must be >= order");
            if (p == 1 && Z.N0 - H->lev[1].n[a] / 2 < R)
                return fail(MG_EINVAL, "higher-order hierarchy: the base must leave >= order/2 cells uncovered per axis");
        }
    const size_t nb = (size_t)Z.N0 * Z.N0 * Z.N0;
    Z.ubase = cv.take<double>(nb);
    if (int rc = ho_plan(Z.N0, Z.h0, order, cv, Z.ubase, Z.base)) return rc;
    Z.pat.assign(Z.np, HozLevel{});
    for (int p = 1; p <= Z.np; ++p) {
        HozLevel& L = Z.pat[p - 1];
        for (int a = 0; a < 3; ++a) {
            L.P.n[a] = H->lev[p].n[a];
            L.P.off[a] = H->lev[p].off[a];
            L.P.pn[a] = H->lev[p - 1].n[a];
        }
        L.P.pper = p == 1;
        L.P.h = Z.h0 / (double)(1 << p);
        const size_t c = (size_t)L.P.n[0] * L.P.n[1] * L.P.n[2];
        L.u = cv.take<double>(c);
        L.f = cv.take<double>(c);
        L.tmp = cv.take<double>(c);
        L.g = cv.take<double>(hoz_face_off(L.P.n, R, 6));
        L.gpart = cv.take<double>(2 * (size_t)R * hoz_face_off(L.P.n, 1, 6));
        L.uold = cv.take<double>(c / 8);
    }
    for (int p = 1; p <= Z.np; ++p) {   // the box of level p - 1 covered by patch p
        int* lo = p == 1 ? Z.base_cov_lo : Z.pat[p - 2].cov_lo;
        int* cn = p == 1 ? Z.base_cov_n : Z.pat[p - 2].cov_n;
        for (int a = 0; a < 3; ++a) {
            lo[a] = H->lev[p].off[a];
            cn[a] = H->lev[p].n[a] / 2;
        }
    }
    Z.W = hoz_weights(order);
    // partial sums: kHozParts per level for the composite sums, kHoParts for the base sums
    Z.part = cv.take<double>(std::max((size_t)kHozParts * (Z.np + 1), (size_t)kHoParts));
    Z.scal = cv.take<double>(8);
    return MG_OK;
}

static double* hoz_pu(HozPlan& Z, int p) { return p == 1 ? Z.base.u[0] : Z.pat[p - 2].u; }
static double* hoz_pf(HozPlan& Z, int p) { return p == 1 ? Z.base.f[0] : Z.pat[p - 2].f; }

// covered cells of every level := the mean of their children, finest first (u or f arrays)
static void hoz_restrict_up(HozPlan& Z, bool of_f, hipStream_t st) {
    for (int p = Z.np; p >= 1; --p) {
        HozLevel& L = Z.pat[p - 1];
        launch_hoz_restrict(of_f ? L.f : L.u, L.P, of_f ? hoz_pf(Z, p) : hoz_pu(Z, p), st);
    }
}

// composite sum of squares (mode 0: v = f; mode 1: the residual) over the uncovered cells of every
// level, volume-weighted, into scal[slot]; kept: every patch's parent part of its ghosts is still
// the one its last smoothing pass kept (right after a V-cycle with post-smoothing)
static void hoz_composite_sq(HozPlan& Z, int mode, int slot, hipStream_t st, bool kept = false) {
    SegList sg{};
    sg.n = Z.np + 1;
    const int nb3[3] = {Z.N0, Z.N0, Z.N0};
    for (int p = 0; p <= Z.np; ++p) {
        double* part = Z.part + (size_t)p * kHozParts;
        if (p == 0) {
            launch_hoz_psum(mode == 0 ? 0 : 2, mode == 0 ? Z.base.f[0] : Z.base.u[0], Z.base.f[0], nullptr, nb3,
                            Z.base_cov_lo, Z.base_cov_n, Z.h0, Z.order, part, st);
        } else {
            HozLevel& L = Z.pat[p - 1];
            if (mode == 1) launch_hoz_ghost(hoz_pu(Z, p), L.u, L.g, L.P, Z.W, Z.order, 1, st, L.gpart, kept ? 2 : 0);
            launch_hoz_psum(mode == 0 ? 0 : 1, mode == 0 ? L.f : L.u, L.f, L.g, L.P.n, L.cov_lo, L.cov_n, L.P.h,
                            Z.order, part, st);
        }
        const double h = p == 0 ? Z.h0 : Z.pat[p - 1].P.h;
        sg.off[p] = p * kHozParts;
        sg.cnt[p] = kHozParts;
        sg.w[p] = h * h * h;
    }
    launch_finalize(Z.part, sg, Z.scal + slot, st);
}

// only the patch changes during a smoothing pass: the parent's part of its ghosts is formed by
// the pass's first fill (or taken as kept: first = 2) and reused by the later ones
static void hoz_smooth(HozPlan& Z, int p, int sweeps, hipStream_t st, int first = 1) {
    HozLevel& L = Z.pat[p - 1];
    for (int s = 0; s < sweeps; ++s)
        for (int c = 0; c < 2; ++c) {
            const double* in = c == 0 ? L.u : L.tmp;
            double* out = c == 0 ? L.tmp : L.u;
            launch_hoz_ghost(hoz_pu(Z, p), in, L.g, L.P, Z.W, Z.order, 1, st, L.gpart, s + c == 0 ? first : 2);
            launch_hoz_half(in, out, L.f, L.g, L.P, Z.order, c, st);
        }
}

// kept: every patch's parent part is still the one kept by its post-smoothing in the previous
// V-cycle (a patch's parent changes only between its pre- and post-smoothing: by the parent's own
// smoothing and correction; restrictions write covered parent cells, which no ghost reads)
static void hoz_vcycle(HozPlan& Z, int p, int nu1, int nu2, hipStream_t st, bool kept = false) {
    if (p == 0) {
        ho_vcycle<double>(Z.base, nu1, nu2, st);
        return;
    }
    HozLevel& L = Z.pat[p - 1];
    hoz_smooth(Z, p, nu1, st, kept ? 2 : 1);                                       // step 2
    launch_hoz_ghost(hoz_pu(Z, p), L.u, L.g, L.P, Z.W, Z.order, 1, st, L.gpart, nu1 > 0 || kept ? 2 : 0);
    launch_hoz_resid_restrict(L.u, L.f, L.g, L.P, Z.order, hoz_pu(Z, p), hoz_pf(Z, p), L.uold, st);   // 3-5
    const int* lo = p == 1 ? Z.base_cov_lo : Z.pat[p - 2].cov_lo;
    const int* cn = p == 1 ? Z.base_cov_n : Z.pat[p - 2].cov_n;
    const int nb3[3] = {Z.N0, Z.N0, Z.N0};
    launch_hoz_fas(hoz_pu(Z, p), hoz_pf(Z, p), p == 1 ? nb3 : Z.pat[p - 2].P.n, p == 1, lo, cn, 2.0 * L.P.h, Z.order,
                   st);                                                            // step 6
    hoz_vcycle(Z, p - 1, nu1, nu2, st, kept);                                      // step 7
    launch_hoz_prolong(L.u, L.P, hoz_pu(Z, p), L.uold, st);                        // step 8
    hoz_smooth(Z, p, nu2, st);                                                     // step 9
}

static int hoz_read(const double* dev, int count, double* out, hipStream_t st) { return ho_read(dev, count, out, st); }

extern "C" {

size_t mg_ho_hierarchy_workspace_bytes(const mg_hier* hier, int order) {
    HozPlan Z;
    Carver cv(nullptr);
    if (hoz_plan(hier, order, cv, Z)) return 0;
    return cv.off;
}

int mg_solve_hierarchy_ho(const mg_hier* hier, int order, const double* const* f, double* const* u,
                          const mg_opts* o, mg_stats* stats, void* ws, size_t ws_bytes, void* stream) {
    hipStream_t st = (hipStream_t)stream;
    if (!o) return fail(MG_EINVAL, "options are NULL");
    if (!f || !u) return fail(MG_EINVAL, "f/u pointer arrays are NULL");
    if (o->max_cycles < 0) return fail(MG_EINVAL, "max_cycles < 0");
    if (o->prec != MG_FP64) return fail(MG_EINVAL, "the higher-order hierarchy solve is FP64 only");
    if (o->nu1 < 0 || o->nu2 < 0 || o->nu1 + o->nu2 > 64) return fail(MG_EINVAL, "nu1/nu2 out of range");
    if (o->flags & ~(MG_USE_INITIAL_GUESS | MG_FIXED_CYCLES | MG_NO_GRAPH)) return fail(MG_EINVAL, "unknown flags");
    HozPlan Z;
    Carver size_cv(nullptr);
    int rc = hoz_plan(hier, order, size_cv, Z);
    if (rc) return rc;
    for (int p = 0; p < hier->nlev; ++p)
        if (!f[p] || !u[p]) return fail(MG_EINVAL, "level pointer is NULL");
    if (!ws || ws_bytes < size_cv.off) return fail(MG_EINVAL, "workspace too small: need " + std::to_string(size_cv.off));
    if (((uintptr_t)ws) & 255) return fail(MG_EINVAL, "workspace must be 256-byte aligned");
    if ((rc = refuse_capture(st, "the higher-order hierarchy solve"))) return rc;
    Carver cv(ws);
    hoz_plan(hier, order, cv, Z);
    (void)hipGetLastError();
    const bool fixed = (o->flags & MG_FIXED_CYCLES) != 0;
    const bool guess = (o->flags & MG_USE_INITIAL_GUESS) != 0;
    const size_t nbase = (size_t)Z.N0 * Z.N0 * Z.N0;
    auto cells = [&](int p) {
        return p == 0 ? nbase : (size_t)Z.pat[p - 1].P.n[0] * Z.pat[p - 1].P.n[1] * Z.pat[p - 1].P.n[2];
    };
    auto uarr = [&](int p) { return p == 0 ? Z.base.u[0] : Z.pat[p - 1].u; };
    auto farr = [&](int p) { return p == 0 ? Z.base.f[0] : Z.pat[p - 1].f; };
    // source preparation: working copies, covered cells from their children, composite mean removed
    for (int p = 0; p <= Z.np; ++p)
        MG_HIP(hipMemcpyAsync(farr(p), f[p], cells(p) * sizeof(double), hipMemcpyDeviceToDevice, st));
    hoz_restrict_up(Z, true, st);
    launch_ho_sum(Z.base.f[0], Z.base.lg, Z.part, Z.scal + 0, st);
    for (int p = 0; p <= Z.np; ++p) launch_sub_mean<double>(farr(p), cells(p), Z.scal + 0, 1.0 / (double)nbase, st);
    hoz_composite_sq(Z, 0, 1, st);
    for (int p = 0; p <= Z.np; ++p) {
        if (guess) MG_HIP(hipMemcpyAsync(uarr(p), u[p], cells(p) * sizeof(double), hipMemcpyDeviceToDevice, st));
        else launch_fill<double>(uarr(p), cells(p), 0.0, st);
    }
    mg_stats S;
    std::memset(&S, 0, sizeof(S));
    for (double& v : S.res_hist) v = NAN;
    double fnorm2 = 0.0;
    if (!fixed) {
        double fs[2];
        if ((rc = hoz_read(Z.scal, 2, fs, st))) return rc;
        S.f_mean_removed = fs[0] / (double)nbase;
        fnorm2 = fs[1];
        if (!std::isfinite(fs[0]) || !std::isfinite(fs[1])) {
            S.rel_res = NAN;
            if (stats) *stats = S;
            return fail(MG_EDIVERGED, "right-hand side contains NaN or Inf");
        }
    }
    long long upc = 0;
    for (int l = 0; l < Z.base.lg; ++l) upc += (long long)(o->nu1 + o->nu2) << (3 * (Z.base.lg - l));
    for (int p = 1; p <= Z.np; ++p) upc += (long long)(o->nu1 + o->nu2) * (long long)cells(p);
    double rel = NAN, prev = INFINITY;
    int grow = 0, status = MG_ENOCONV, cycles = 0;
    bool kept = false;   // the parent parts kept by the last V-cycle's post-smoothing are current
    auto check = [&]() -> int {
        hoz_restrict_up(Z, false, st);
        hoz_composite_sq(Z, 1, 2, st, kept);
        double r2;
        if (int e = hoz_read(Z.scal + 2, 1, &r2, st)) return e;
        rel = fnorm2 > 0 ? std::sqrt(r2 / fnorm2) : 0.0;
        if (cycles >= 1 && cycles <= 64) S.res_hist[cycles - 1] = rel;
        if (!std::isfinite(rel)) return MG_EDIVERGED;
        grow = rel > prev ? grow + 1 : 0;
        prev = rel;
        if (grow >= 3) return MG_EDIVERGED;
        return rel <= o->tol ? MG_OK : 1;
    };
    if (guess && !fixed) {
        const int c = check();
        if (c == MG_EHIP) return c;
        if (c == MG_OK || c == MG_EDIVERGED) status = c;
    }
    while (status == MG_ENOCONV && cycles < o->max_cycles) {
        hoz_vcycle(Z, Z.np, o->nu1, o->nu2, st, kept);
        kept = o->nu2 > 0;
        ++cycles;
        S.cell_updates += upc;
        if (fixed) continue;
        const int c = check();
        if (c == MG_EHIP) return c;
        if (c == MG_OK || c == MG_EDIVERGED) status = c;
    }
    if (fixed) status = MG_OK;
    // gauge: covered cells from their children, composite (= base) mean removed, copy back
    hoz_restrict_up(Z, false, st);
    launch_ho_sum(Z.base.u[0], Z.base.lg, Z.part, Z.scal + 3, st);
    for (int p = 0; p <= Z.np; ++p) {
        launch_sub_mean<double>(uarr(p), cells(p), Z.scal + 3, 1.0 / (double)nbase, st);
        MG_HIP(hipMemcpyAsync(u[p], uarr(p), cells(p) * sizeof(double), hipMemcpyDeviceToDevice, st));
    }
    MG_HIP(hipGetLastError());
    if (fixed) MG_HIP(hipStreamSynchronize(st));
    S.cycles = cycles;
    S.rel_res = fixed ? NAN : rel;
    if (stats) *stats = S;
    if (status == MG_ENOCONV) return fail(MG_ENOCONV, "no convergence within max_cycles");
    if (status == MG_EDIVERGED) return fail(MG_EDIVERGED, "residual diverged");
    return MG_OK;
}

int mg_ghost_fill_ho(const mg_hier* hier, int order, int p, const double* const* u, double* ghosts, int flux_match,
                     void* stream) {
    HozPlan Z;
    Carver cv(nullptr);
    if (int rc = hoz_plan(hier, order, cv, Z)) return rc;
    if (p < 1 || p >= hier->nlev) return fail(MG_EINVAL, "p must name a patch");
    if (!u || !u[p] || !u[p - 1] || !ghosts) return fail(MG_EINVAL, "NULL argument");
    launch_hoz_ghost(u[p - 1], u[p], ghosts, Z.pat[p - 1].P, Z.W, order, flux_match ? 1 : 0, (hipStream_t)stream);
    MG_HIP(hipGetLastError());
    return MG_OK;
}

}  // extern "C"

extern "C" {

const char* mg_last_error(void) { return g_err.c_str(); }

int mg_batch_tune_candidates(void) { return kNumShapes; }

int mg_batch_force_shape(int index) {
    if (index < -1 || index >= kNumShapes) return fail(MG_EINVAL, "shape index out of range");
    std::lock_guard<std::mutex> g(g_tune_mu);
    g_force_shape = index;
    return MG_OK;
}

int mg_tune_cache(const char* path) {
    std::lock_guard<std::mutex> g(g_tune_mu);
    if (!path || !*path) {
        g_tune_path.clear();
        return 0;
    }
    std::map<std::string, std::vector<SmoothShape>> loaded;
    std::map<std::string, int> loaded_inner;
    if (FILE* fh = std::fopen(path, "r")) {
        std::string text;
        char buf[4096];
        size_t k;
        while ((k = std::fread(buf, 1, sizeof(buf), fh)) > 0) text.append(buf, k);
        std::fclose(fh);
        if (!parse_tune_file(text, loaded, loaded_inner))
            return fail(MG_EINVAL, std::string("not a tuning cache file: ") + path);
    }
    for (auto& kv : loaded) g_tune[kv.first] = kv.second;
    for (auto& kv : loaded_inner) g_inner[kv.first] = kv.second;
    g_tune_path = path;
    if (!g_tune.empty() || !g_inner.empty()) save_tune_file();   // the file holds every entry the process knows
    return (int)(loaded.size() + loaded_inner.size());
}

int mg_tune_inner(const mg_hier* hier, const double* const* f, double* const* u, const mg_opts* opts, int* best,
                  double* ms, void* workspace, size_t workspace_bytes, void* stream) {
    if (!opts || !best) return fail(MG_EINVAL, "NULL argument");
    if (opts->prec != MG_MIXED) return fail(MG_EINVAL, "inner cycles are tuned for mixed-precision solves");
    if (int v = validate_hier(hier)) return v;
    hipStream_t st = (hipStream_t)stream;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    MG_HIP(hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        (void)hipGetLastError();
        return fail(MG_EHIP, "hipEventCreate failed");
    }
    int best_k = -1, last_rc = MG_OK;
    double best_ms = 0.0;
    std::string last_err;
    g_tuning_inner = true;
    for (int k = 0; k <= kInnerMax; ++k) {   // 0: the contraction rule
        mg_opts o = *opts;
        o.inner = k;
        o.flags &= ~MG_USE_INITIAL_GUESS;
        double t = -1.0;
        int rc = MG_OK;
        for (int rep = 0; rep < 3 && rc == MG_OK; ++rep) {   // the first call captures the graphs
            mg_stats sdummy;
            (void)hipEventRecord(e0, st);
            rc = solve(hier, f, u, &o, &sdummy, workspace, workspace_bytes, st);
            (void)hipEventRecord(e1, st);
            (void)hipEventSynchronize(e1);
            float m = 0.f;
            if (rc == MG_OK && rep && hipEventElapsedTime(&m, e0, e1) == hipSuccess && (t < 0 || m < t)) t = m;
        }
        if (ms) ms[k] = rc == MG_OK ? t : -1.0;
        if (rc == MG_OK && t >= 0 && (best_k < 0 || t < best_ms)) {
            best_k = k;
            best_ms = t;
        } else if (rc != MG_OK) {
            last_rc = rc;
            last_err = g_err;
        }
    }
    g_tuning_inner = false;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    (void)hipGetLastError();
    if (best_k < 0) return fail(last_rc ? last_rc : MG_EHIP, "no inner-cycle count solved the problem: " + last_err);
    *best = best_k;
    std::lock_guard<std::mutex> g(g_tune_mu);
    g_inner[inner_key(hier, opts)] = best_k;
    save_tune_file();
    return MG_OK;
}

int mg_kprof_enable(int period) {
    if (period < 0) return fail(MG_EINVAL, "kernel timing period < 0");
    g_kprof.on = period != 0;
    g_kprof.period = period > 0 ? period : 1;
    g_kprof.count = 0;
    return MG_OK;
}

int mg_kprof_read(double* ms_total, long long* launches, double* bytes_total) {
    double ms = 0.0, by = 0.0;
    long long n = 0;
    for (auto& r : g_kprof.recs) {
        float t = 0.f;
        MG_HIP(hipEventSynchronize(r.b));
        MG_HIP(hipEventElapsedTime(&t, r.a, r.b));
        ms += t;
        by += r.bytes;
        ++n;
        g_kprof.pool.push_back(r.a);
        g_kprof.pool.push_back(r.b);
    }
    g_kprof.recs.clear();
    if (ms_total) *ms_total = ms;
    if (launches) *launches = n;
    if (bytes_total) *bytes_total = by;
    return MG_OK;
}

size_t mg_workspace_bytes(const mg_hier* hier, const mg_opts* opts) {
    Plan P;
    Carver cv(nullptr);
    if (build_plan(hier, opts, cv, nullptr, P)) return 0;
    return cv.off;
}

int mg_solve_level(int n, double h, const double* f, double* u, const mg_opts* opts, mg_stats* stats,
                   void* workspace, size_t workspace_bytes, void* stream) {
    mg_hier H = single_level(n, h);
    const double* fp[1] = {f};
    double* up[1] = {u};
    return solve(&H, fp, up, opts, stats, workspace, workspace_bytes, (hipStream_t)stream);
}

int mg_solve_hierarchy(const mg_hier* hier, const double* const* f, double* const* u, const mg_opts* opts,
                       mg_stats* stats, void* workspace, size_t workspace_bytes, void* stream) {
    return solve(hier, f, u, opts, stats, workspace, workspace_bytes, (hipStream_t)stream);
}

int mg_solve_hierarchy_noalloc(const mg_hier* hier, const double* const* f, double* const* u, const mg_opts* opts,
                               mg_stats* stats, void* stream) {
    return solve_noalloc(hier, f, u, opts, stats, (hipStream_t)stream);
}

int mg_residual_hierarchy(const mg_hier* hier, const double* const* f, double* const* u, double* const* r,
                          double* rel, void* workspace, size_t workspace_bytes, void* stream) {
    hipStream_t st = (hipStream_t)stream;
    if (!hier || !f || !u || !r) return fail(MG_EINVAL, "NULL argument");
    for (int p = 0; p < hier->nlev; ++p)
        if (!f[p] || !u[p] || !r[p]) return fail(MG_EINVAL, "level pointer is NULL");
    mg_opts o{};
    o.nu1 = o.nu2 = 2;
    Plan P;
    Carver sz(nullptr);
    int rc = build_plan(hier, &o, sz, u, P);
    if (rc) return rc;
    if (!workspace || workspace_bytes < sz.off) return fail(MG_EINVAL, "workspace too small");
    Carver cv(workspace);
    build_plan(hier, &o, cv, u, P);
    (void)hipGetLastError();
    if ((rc = prepare_f(P, f, st))) return rc;
    for (int l = 0; l < P.nh; ++l) {
        Level& L = P.L[l];
        if (L.u != L.u_user) launch_relayout<double, double>(L.u_user, mklay(L.d, 0), L.u, L.lay, st);
    }
    std::vector<double*> rr(P.nh);
    for (int l = 0; l < P.nh; ++l) rr[l] = r[P.L[l].p];
    composite_residual<double>(P, rr.data(), true, st);
    for (int l = 0; l < P.nh; ++l) {
        Level& L = P.L[l];
        if (L.u != L.u_user) launch_relayout<double, double>(L.u, L.lay, L.u_user, mklay(L.d, 0), st);
    }
    MG_HIP(hipGetLastError());
    if (rel) {
        double v[3];
        if ((rc = read_scalars(P, S_FSUM, 3, v, st))) return rc;
        *rel = v[1] > 0 ? std::sqrt(v[2] / v[1]) : 0.0;
    }
    return MG_OK;
}

size_t lpt_workspace_bytes(const mg_hier* hier, int what) {
    if (validate_hier(hier) || what < 1 || what > 3) return 0;
    Carver cv(nullptr);
    LptPlan lp;
    return lpt_carve(hier, what, cv, lp);
}

int lpt_displacements(const mg_hier* hier, const double* const* phi, double* const* out, int grad_order,
                      double scale, void* workspace, size_t workspace_bytes, void* stream) {
    hipStream_t st = (hipStream_t)stream;
    if (!out) return fail(MG_EINVAL, "out is NULL");
    LptPlan lp;
    int rc = lpt_common(hier, 1, phi, workspace, workspace_bytes, st, lp, grad_order);
    if (rc) return rc;
    const int rg = grad_order / 2;
    for (int p = 0; p < hier->nlev; ++p) {
        if (!out[3 * p] || !out[3 * p + 1] || !out[3 * p + 2]) return fail(MG_EINVAL, "output pointer is NULL");
        const Dims d = dims_of(hier, p);
        const double h = h_of(hier, p);
        if (p == 0) {
            launch_grad4(lp.phi[0], 0, d, h, scale, out[0], out[1], out[2], st, grad_order);
        } else {
            launch_wide_ghost(lp.phi[p - 1], lp.phi[p], lp.padded, d, parent_of(hier, p), rg, st);
            launch_grad4(lp.padded, rg, d, h, scale, out[3 * p], out[3 * p + 1], out[3 * p + 2], st, grad_order);
        }
    }
    MG_HIP(hipGetLastError());
    return MG_OK;
}

}  // extern "C"

namespace mgic {
// tau on every level (composite mean removed); on the base from base_grad (s G4 phi, post =
// 1 / s^2) when given, else from phi
static int tau_levels(const mg_hier* hier, LptPlan& lp, double* const* tau, double* const* base_grad, double post,
                      hipStream_t st, int order) {
    for (int p = 0; p < hier->nlev; ++p) {
        if (!tau[p]) return fail(MG_EINVAL, "tau level pointer is NULL");
        const Dims d = dims_of(hier, p);
        const double h = h_of(hier, p);
        if (p == 0 && base_grad) {
            launch_tau_from_grad(base_grad[0], base_grad[1], base_grad[2], d, h, post, tau[0], st, order);
        } else if (p == 0) {
            launch_tau(lp.phi[0], 0, d, h, tau[0], lp.psi, st, order);
        } else {   // ghosts of width `order`: D = G o G reaches order / 2 twice
            launch_wide_ghost(lp.phi[p - 1], lp.phi[p], lp.padded, d, parent_of(hier, p), order, st);
            launch_tau(lp.padded, order, d, h, tau[p], lp.psi, st, order);
        }
    }
    // composite mean: covered cells := mean of children, then subtract the base mean everywhere
    for (int p = hier->nlev - 1; p >= 1; --p)
        launch_restrict_cov<double>(tau[p], mklay(dims_of(hier, p), 0), tau[p - 1], parent_of(hier, p), st);
    int np = 0;
    CovBox none{};
    launch_sum(tau[0], mklay(dims_of(hier, 0), 0), none, 0, lp.partials, &np, st);
    SegList s{};
    s.n = 1; s.off[0] = 0; s.cnt[0] = np; s.w[0] = 1.0;
    launch_finalize(lp.partials, s, lp.scal, st);
    const double inv = 1.0 / (double)dims_of(hier, 0).cells();
    for (int p = 0; p < hier->nlev; ++p) launch_sub_mean<double>(tau[p], dims_of(hier, p).cells(), lp.scal, inv, st);
    MG_HIP(hipGetLastError());
    return MG_OK;
}
}  // namespace mgic

extern "C" {

int lpt2_source(const mg_hier* hier, const double* const* phi, double* const* tau, int grad_order, void* workspace,
                size_t workspace_bytes, void* stream) {
    hipStream_t st = (hipStream_t)stream;
    if (!tau) return fail(MG_EINVAL, "tau is NULL");
    LptPlan lp;
    int rc = lpt_common(hier, 2, phi, workspace, workspace_bytes, st, lp, grad_order);
    if (rc) return rc;
    return tau_levels(hier, lp, tau, nullptr, 1.0, st, grad_order);
}

int lpt_displacements_and_source(const mg_hier* hier, const double* const* phi, double* const* out, int grad_order,
                                 double scale, double* const* tau, void* workspace, size_t workspace_bytes,
                                 void* stream) {
    hipStream_t st = (hipStream_t)stream;
    if (!out || !tau) return fail(MG_EINVAL, "out or tau is NULL");
    if (!(scale != 0.0) || !std::isfinite(scale)) return fail(MG_EINVAL, "scale must be finite and non-zero");
    LptPlan lp;
    int rc = lpt_common(hier, 2, phi, workspace, workspace_bytes, st, lp, grad_order);
    if (rc) return rc;
    const int rg = grad_order / 2;
    for (int p = 0; p < hier->nlev; ++p) {
        if (!out[3 * p] || !out[3 * p + 1] || !out[3 * p + 2]) return fail(MG_EINVAL, "output pointer is NULL");
        const Dims d = dims_of(hier, p);
        const double h = h_of(hier, p);
        if (p == 0) {
            launch_grad4(lp.phi[0], 0, d, h, scale, out[0], out[1], out[2], st, grad_order);
        } else {
            launch_wide_ghost(lp.phi[p - 1], lp.phi[p], lp.padded, d, parent_of(hier, p), rg, st);
            launch_grad4(lp.padded, rg, d, h, scale, out[3 * p], out[3 * p + 1], out[3 * p + 2], st, grad_order);
        }
    }
    return tau_levels(hier, lp, tau, out, 1.0 / (scale * scale), st, grad_order);
}

int lpt_lla_density(const mg_hier* hier, const double* const* disp, const double* const* disp2,
                    double* const* delta, void* workspace, size_t workspace_bytes, void* stream) {
    hipStream_t st = (hipStream_t)stream;
    int rc = validate_hier(hier);
    if (rc) return rc;
    if (hier->lev[0].n[0] < 2) return fail(MG_EINVAL, "LPT needs a base of at least 2^3 cells");
    if (!disp || !delta) return fail(MG_EINVAL, "disp or delta is NULL");
    const int nl = hier->nlev;
    for (int k = 0; k < 3 * nl; ++k)
        if (!disp[k] || (disp2 && !disp2[k])) return fail(MG_EINVAL, "displacement pointer is NULL");
    for (int p = 0; p < nl; ++p)
        if (!delta[p]) return fail(MG_EINVAL, "delta level pointer is NULL");
    Carver sz(nullptr);
    LptPlan lp;
    const size_t need = lpt_carve(hier, 3, sz, lp);
    if (!workspace || workspace_bytes < need) return fail(MG_EINVAL, "workspace too small: need " + std::to_string(need));
    if (((uintptr_t)workspace) & 255) return fail(MG_EINVAL, "workspace must be 256-byte aligned");
    Carver cv(workspace);
    lpt_carve(hier, 3, cv, lp);
    (void)hipGetLastError();
    if (nl == 1) {
        const double* a[3] = {disp[0], disp[1], disp[2]};
        const double* b[3] = {disp2 ? disp2[0] : nullptr, disp2 ? disp2[1] : nullptr, disp2 ? disp2[2] : nullptr};
        launch_lla(a, disp2 ? b : nullptr, 0, dims_of(hier, 0), h_of(hier, 0), delta[0], st);
    } else {
        // working copies of L (= disp + disp2), covered cells restricted from the finer level
        auto comp = [&](int c, int p) { return lp.phi[(size_t)c * nl + p]; };
        for (int p = 0; p < nl; ++p)
            for (int c = 0; c < 3; ++c) {
                const size_t n = dims_of(hier, p).cells();
                if (disp2) launch_add2(disp[3 * p + c], disp2[3 * p + c], comp(c, p), n, st);
                else MG_HIP(hipMemcpyAsync(comp(c, p), disp[3 * p + c], n * sizeof(double), hipMemcpyDeviceToDevice, st));
            }
        for (int p = nl - 1; p >= 1; --p)
            for (int c = 0; c < 3; ++c)
                launch_restrict_cov<double>(comp(c, p), mklay(dims_of(hier, p), 0), comp(c, p - 1), parent_of(hier, p), st);
        for (int p = 0; p < nl; ++p) {
            const Dims d = dims_of(hier, p);
            if (p == 0) {
                const double* a[3] = {comp(0, 0), comp(1, 0), comp(2, 0)};
                launch_lla(a, nullptr, 0, d, h_of(hier, 0), delta[0], st);
            } else {
                const double* a[3];
                for (int c = 0; c < 3; ++c) {
                    double* pad = lp.padded + (size_t)c * lp.padstride;
                    launch_wide_ghost(comp(c, p - 1), comp(c, p), pad, d, parent_of(hier, p), 2, st);
                    a[c] = pad;
                }
                launch_lla(a, nullptr, 2, d, h_of(hier, p), delta[p], st);
            }
        }
    }
    // renormalisation: covered cells := mean of their children, then the base mean (the composite
    // volume mean) is subtracted everywhere
    for (int p = nl - 1; p >= 1; --p)
        launch_restrict_cov<double>(delta[p], mklay(dims_of(hier, p), 0), delta[p - 1], parent_of(hier, p), st);
    int np = 0;
    CovBox none{};
    launch_sum(delta[0], mklay(dims_of(hier, 0), 0), none, 0, lp.partials, &np, st);
    SegList s{};
    s.n = 1; s.off[0] = 0; s.cnt[0] = np; s.w[0] = 1.0;
    launch_finalize(lp.partials, s, lp.scal, st);
    const double inv = 1.0 / (double)dims_of(hier, 0).cells();
    for (int p = 0; p < nl; ++p) launch_sub_mean<double>(delta[p], dims_of(hier, p).cells(), lp.scal, inv, st);
    MG_HIP(hipGetLastError());
    return MG_OK;
}

size_t mg_batch_workspace_bytes(int ninst, const int* n, const mg_opts* opts) {
    return batch_bytes(ninst, n, opts);
}

int mg_solve_batch(int ninst, const int* n, const double* h, const double* const* f, double* const* u,
                   const mg_opts* opts, mg_stats* stats, void* workspace, size_t workspace_bytes, void* stream) {
    return solve_batch(ninst, n, h, f, u, opts, stats, workspace, workspace_bytes, (hipStream_t)stream);
}

int mg_smooth_level(int n, double h, const double* f, double* u, int half_sweeps, int prec, void* workspace,
                    size_t workspace_bytes, void* stream) {
    hipStream_t st = (hipStream_t)stream;
    if (!f || !u || half_sweeps < 0) return fail(MG_EINVAL, "bad argument");
    if (n < 2 || n % 2) return fail(MG_EINVAL, "smoothing needs an even periodic grid");
    mg_hier H = single_level(n, h);
    mg_opts o{};
    o.nu1 = o.nu2 = 2;
    o.prec = prec;
    Plan P;
    Carver sz(nullptr);
    double* up[1] = {u};
    int rc = build_plan(&H, &o, sz, up, P);
    if (rc) return rc;
    if (!workspace || workspace_bytes < sz.off) return fail(MG_EINVAL, "workspace too small");
    Carver cv(workspace);
    build_plan(&H, &o, cv, up, P);
    (void)hipGetLastError();
    Level& L = P.L[0];
    const Lay nat(L.d, 0);
    if (prec == MG_FP64) {
        launch_relayout<double, double>(f, nat, L.f, L.lay, st);
        launch_relayout<double, double>(u, nat, L.u, L.lay, st);
        smooth<double>(P, 0, half_sweeps / 2, st);
        if (half_sweeps & 1) launch_rbgs_half<double>(L.u, L.f, nullptr, L.lay, L.h, 0, st);
        launch_relayout<double, double>(L.u, L.lay, u, nat, st);
    } else {
        launch_relayout<double, float>(f, nat, L.f32, L.lay, st);
        launch_relayout<double, float>(u, nat, L.u32, L.lay, st);
        smooth<float>(P, 0, half_sweeps / 2, st);
        if (half_sweeps & 1) launch_rbgs_half<float>(L.u32, L.f32, nullptr, L.lay, L.h, 0, st);
        launch_relayout<float, double>(L.u32, L.lay, u, nat, st);
    }
    MG_HIP(hipGetLastError());
    return MG_OK;
}

int mg_ghost_fill(const mg_hier* hier, int p, const double* const* u, double* ghosts, int flux_match, void* stream) {
    int rc = validate_hier(hier);
    if (rc) return rc;
    if (p < 1 || p >= hier->nlev) return fail(MG_EINVAL, "p must name a patch");
    if (!u || !u[p] || !u[p - 1] || !ghosts) return fail(MG_EINVAL, "NULL argument");
    (void)hipGetLastError();
    launch_ghost_fill<double>(u[p - 1], u[p], ghosts, Lay(dims_of(hier, p), 0), parent_of(hier, p), flux_match,
                              (hipStream_t)stream);
    MG_HIP(hipGetLastError());
    return MG_OK;
}

}  // extern "C"
