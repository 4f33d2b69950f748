// Batched solves of independent hierarchies (a periodic base with nested patches each).
//
// Single-level instances go to the batched periodic schedule (shared launches per V-cycle step
// and level depth, replayed from graphs).  Instances with patches are each the solo solve of
// Sections 3.2-3.3: their patch levels are sequences of short launches (a 128^3 patch half-sweep
// and its ghost fill take a few microseconds each, bound by launch and memory latency), so the
// batch runs several of them at once, one per lane: a library worker thread with its own stream
// of default priority.  Kernels of different instances then overlap on the device.  Every
// instance runs the same kernels with the same arguments as its solo solve, so its bits, cycles
// and residual history are those of mg_solve_hierarchy.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <condition_variable>
#include <functional>
#include <map>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "mgic.h"

namespace mgic {

int report_error(int code, const char* msg);
int solve_batch_codes(int ninst, const int* n, const double* h, const double* const* f, double* const* u,
                      const mg_opts* o, mg_stats* stats, int* codes, void* ws, size_t ws_bytes, hipStream_t st);

namespace {

// Concurrent hierarchy solves.  With the caller's stream, three lanes fill the four hardware
// queues a process gets by default.  Measured on eight zoom hierarchies (128^3 base, three
// 128^3 patches, mixed): 2 lanes 28.7 ms, 3 lanes 25.7 ms, 4 lanes 29.9 ms, 6 lanes 25.7 ms,
// against 45.3 ms one after another.
constexpr int kLanes = 3;

size_t up256(size_t b) { return (b + 255) & ~(size_t)255; }

// Worker threads, created on first use and kept for the life of the process (their thread-local
// graph caches and pinned buffers are reused by later batches).  start() hands every lane the
// same job; wait() returns once all of them have finished it.
class Lanes {
  public:
    void start(int lanes, std::function<void(int)> job) {
        std::lock_guard<std::mutex> lk(mu_);
        while ((int)threads_ < lanes) {
            const int w = threads_++;
            std::thread([this, w] { loop(w); }).detach();
        }
        job_ = std::move(job);
        want_ = lanes;
        busy_ = lanes;
        ++gen_;
        go_.notify_all();
    }
    void wait() {
        std::unique_lock<std::mutex> lk(mu_);
        idle_.wait(lk, [&] { return busy_ == 0; });
        job_ = nullptr;
    }

  private:
    void loop(int w) {
        unsigned long long seen = 0;
        std::unique_lock<std::mutex> lk(mu_);
        for (;;) {
            go_.wait(lk, [&] { return gen_ != seen; });
            seen = gen_;
            if (w >= want_) continue;
            std::function<void(int)> job = job_;
            lk.unlock();
            job(w);
            lk.lock();
            if (--busy_ == 0) idle_.notify_all();
        }
    }
    std::mutex mu_;
    std::condition_variable go_, idle_;
    std::function<void(int)> job_;
    unsigned long long gen_ = 0;
    int threads_ = 0, want_ = 0, busy_ = 0;
};

// per device: one stream and one completion event per lane, and the batch's start event
struct DevRes {
    hipStream_t s[kLanes] = {};
    hipEvent_t done[kLanes] = {};
    hipEvent_t start = nullptr;
    bool ready = false;
};

std::mutex g_call_mu;                 // one hierarchy batch at a time uses the lanes
Lanes* g_lanes = nullptr;             // never destroyed: the threads outlive static destructors
std::map<int, DevRes> g_dev;

int dev_res(int dev, DevRes*& out) {
    DevRes& R = g_dev[dev];
    if (!R.ready) {
        for (int k = 0; k < kLanes; ++k) {
            if (!R.s[k] && hipStreamCreateWithFlags(&R.s[k], hipStreamNonBlocking) != hipSuccess)
                return report_error(MG_EHIP, "stream creation failed");
            if (!R.done[k] && hipEventCreateWithFlags(&R.done[k], hipEventDisableTiming) != hipSuccess)
                return report_error(MG_EHIP, "event creation failed");
        }
        if (!R.start && hipEventCreateWithFlags(&R.start, hipEventDisableTiming) != hipSuccess)
            return report_error(MG_EHIP, "event creation failed");
        R.ready = true;
    }
    out = &R;
    return MG_OK;
}

struct Layout {
    std::vector<int> single, multi;   // instance ids: batched single levels / solo solves on the lanes
    std::vector<int> n;               // single-level sizes, in `single` order
    size_t batch_bytes = 0;
    std::vector<size_t> off, bytes;   // per instance with patches (index into multi)
    size_t total = 0;
};

int check_opts(const mg_opts* o) {
    if (!o) return report_error(MG_EINVAL, "options are NULL");
    if (o->max_cycles < 0) return report_error(MG_EINVAL, "max_cycles < 0");
    if (o->prec != MG_FP64 && o->prec != MG_MIXED) return report_error(MG_EINVAL, "unknown precision");
    if (o->inner < 0 || o->inner > 16) return report_error(MG_EINVAL, "inner cycles out of range (0..16)");
    return MG_OK;
}

// sizes of every part; 0 (with the reason recorded) when an instance is invalid
size_t layout(int ninst, const mg_hier* const* hier, const mg_opts* o, Layout& L) {
    if (ninst < 1 || !hier) {
        report_error(MG_EINVAL, "no instances");
        return 0;
    }
    if (check_opts(o)) return 0;
    for (int i = 0; i < ninst; ++i) {
        if (!hier[i]) {
            report_error(MG_EINVAL, ("instance " + std::to_string(i) + ": hierarchy is NULL").c_str());
            return 0;
        }
        // without the mean fix every instance is a solo solve (the batched schedule always
        // removes the mean)
        if (hier[i]->nlev == 1 && !(o->flags & MG_NO_MEAN_FIX)) {
            L.single.push_back(i);
            L.n.push_back(hier[i]->lev[0].n[0]);
        } else {
            L.multi.push_back(i);
        }
    }
    size_t off = 0;
    if (!L.single.empty()) {
        // a single-level description must be a valid hierarchy too (cubic base, positive h)
        for (int i : L.single)
            if (mg_workspace_bytes(hier[i], o) == 0) return 0;
        L.batch_bytes = mg_batch_workspace_bytes((int)L.single.size(), L.n.data(), o);
        if (!L.batch_bytes) return 0;
        off = up256(L.batch_bytes);
    }
    for (int i : L.multi) {
        const size_t b = mg_workspace_bytes(hier[i], o);
        if (!b) {
            const std::string why = mg_last_error();
            report_error(MG_EINVAL, ("instance " + std::to_string(i) + ": " + why).c_str());
            return 0;
        }
        L.off.push_back(off);
        L.bytes.push_back(b);
        off += up256(b);
    }
    L.total = off;
    return off;
}

}  // namespace

size_t batch_hier_bytes(int ninst, const mg_hier* const* hier, const mg_opts* o) {
    Layout L;
    return layout(ninst, hier, o, L);
}

int solve_batch_hier(int ninst, const mg_hier* const* hier, const double* const* const* f, double* const* const* u,
                     const mg_opts* o, mg_stats* stats, void* ws, size_t ws_bytes, hipStream_t st) {
    if (!f || !u) return report_error(MG_EINVAL, "f/u pointer arrays are NULL");
    Layout L;
    const size_t need = layout(ninst, hier, o, L);
    if (!need) return MG_EINVAL;
    for (int i = 0; i < ninst; ++i) {
        if (!f[i] || !u[i]) return report_error(MG_EINVAL, ("instance " + std::to_string(i) + ": NULL level array").c_str());
        for (int p = 0; p < hier[i]->nlev; ++p)
            if (!f[i][p] || !u[i][p])
                return report_error(MG_EINVAL, ("instance " + std::to_string(i) + ": level pointer is NULL").c_str());
    }
    if (!ws || ws_bytes < need)
        return report_error(MG_EINVAL, ("workspace too small: need " + std::to_string(need)).c_str());
    if (((uintptr_t)ws) & 255) return report_error(MG_EINVAL, "workspace must be 256-byte aligned");
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(st, &cap) != hipSuccess) return report_error(MG_EHIP, "stream query failed");
    if (cap != hipStreamCaptureStatusNone)
        return report_error(MG_EINVAL, "the hierarchy batch cannot run under stream capture (its lanes wait on the host)");

    std::vector<int> code(ninst, MG_OK);
    std::vector<mg_stats> S(ninst);
    std::vector<std::string> msg(ninst);
    int hard = MG_OK;   // MG_EINVAL / MG_EHIP from any part
    std::string hard_msg;

    std::unique_lock<std::mutex> call(g_call_mu);
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return report_error(MG_EHIP, "no current device");
    DevRes* R = nullptr;
    const int lanes = std::min<int>(kLanes, (int)L.multi.size());
    if (lanes > 0) {
        if (int rc = dev_res(dev, R)) return rc;
        if (!g_lanes) g_lanes = new Lanes();
        // the lanes start after everything already queued on the caller's stream
        if (hipEventRecord(R->start, st) != hipSuccess) return report_error(MG_EHIP, "event record failed");
    }
    // largest instances first, taken by whichever lane is free
    std::vector<int> order(L.multi.size());
    for (size_t k = 0; k < order.size(); ++k) order[k] = (int)k;
    auto cells = [&](int k) {
        const mg_hier* H = hier[L.multi[k]];
        double c = 0;
        for (int p = 0; p < H->nlev; ++p) c += (double)H->lev[p].n[0] * H->lev[p].n[1] * H->lev[p].n[2];
        return c;
    };
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return cells(a) > cells(b); });
    std::atomic<int> next{0};
    std::vector<hipError_t> lane_err(kLanes, hipSuccess);
    if (lanes > 0) {
        g_lanes->start(lanes, [&](int lane) {
            hipError_t e = hipSetDevice(dev);
            const hipStream_t s = R->s[lane];
            if (e == hipSuccess) e = hipStreamWaitEvent(s, R->start, 0);
            if (e != hipSuccess) {
                lane_err[lane] = e;
                return;
            }
            for (;;) {
                const int k = next.fetch_add(1);
                if (k >= (int)order.size()) break;
                const int slot = order[k];
                const int i = L.multi[slot];
                code[i] = mg_solve_hierarchy(hier[i], f[i], u[i], o, &S[i], (char*)ws + L.off[slot], L.bytes[slot], s);
                if (code[i] != MG_OK) msg[i] = mg_last_error();
            }
            lane_err[lane] = hipEventRecord(R->done[lane], s);
        });
    }
    // meanwhile the single-level instances, batched, on the caller's stream
    if (!L.single.empty()) {
        const int k = (int)L.single.size();
        std::vector<double> h(k);
        std::vector<const double*> fp(k);
        std::vector<double*> up(k);
        std::vector<int> c(k, MG_OK);
        std::vector<mg_stats> sb(k);
        for (int j = 0; j < k; ++j) {
            const int i = L.single[j];
            h[j] = hier[i]->lev[0].h;
            fp[j] = f[i][0];
            up[j] = u[i][0];
        }
        const int rc = solve_batch_codes(k, L.n.data(), h.data(), fp.data(), up.data(), o, sb.data(), c.data(), ws,
                                         L.batch_bytes, st);
        if (rc == MG_EINVAL || rc == MG_EHIP) {
            hard = rc;
            hard_msg = mg_last_error();
        } else {
            for (int j = 0; j < k; ++j) {
                code[L.single[j]] = c[j];
                S[L.single[j]] = sb[j];
            }
        }
    }
    if (lanes > 0) {
        g_lanes->wait();
        for (int k = 0; k < lanes; ++k) {
            if (lane_err[k] != hipSuccess && !hard) {
                hard = MG_EHIP;
                hard_msg = std::string("lane setup failed: ") + hipGetErrorString(lane_err[k]);
            }
            // later work on the caller's stream follows every lane's solves
            if (lane_err[k] == hipSuccess && hipStreamWaitEvent(st, R->done[k], 0) != hipSuccess && !hard) {
                hard = MG_EHIP;
                hard_msg = "stream join failed";
            }
        }
    }
    call.unlock();
    if (stats)
        for (int i = 0; i < ninst; ++i) stats[i] = S[i];
    for (int i = 0; i < ninst && !hard; ++i)
        if (code[i] == MG_EINVAL || code[i] == MG_EHIP) {
            hard = code[i];
            hard_msg = "instance " + std::to_string(i) + ": " + msg[i];
        }
    if (hard) return report_error(hard, hard_msg.c_str());
    for (int i = 0; i < ninst; ++i)
        if (code[i] != MG_OK) {
            const std::string m = "instance " + std::to_string(i) +
                                  (code[i] == MG_EDIVERGED ? " diverged (NaN/Inf or growth)"
                                                           : " did not converge within max_cycles");
            return report_error(code[i], m.c_str());
        }
    return MG_OK;
}

}  // namespace mgic

extern "C" {

size_t mg_batch_hier_workspace_bytes(int ninst, const mg_hier* const* hier, const mg_opts* opts) {
    return mgic::batch_hier_bytes(ninst, hier, opts);
}

int mg_solve_batch_hier(int ninst, const mg_hier* const* hier, const double* const* const* f, double* const* const* u,
                        const mg_opts* opts, mg_stats* stats, void* workspace, size_t workspace_bytes, void* stream) {
    return mgic::solve_batch_hier(ninst, hier, f, u, opts, stats, workspace, workspace_bytes, (hipStream_t)stream);
}

}  // extern "C"
