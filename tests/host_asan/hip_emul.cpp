// Host-only emulation of the HIP runtime calls and of the kernel launchers that
// the library's host code (engine.hip) makes, for running that code under the
// address and undefined-behaviour sanitizers on a machine without a GPU.
//
// Device memory is plain heap memory (so the sanitizer sees every access of
// it), copies are memcpy, and a launcher "runs" a launch group by reading every
// descriptor of its table and touching the first and last element of every
// buffer the descriptor names.  A descriptor must also agree with its group
// (shape, mask kind, route, rank tier), so a table that was overwritten by
// another step before a group read it is reported.
//
// Work on the stream passed to emul_set_slow_stream() is deferred: its launches
// (and anything queued behind them) run only when the stream, or an event
// recorded on it, is synchronised, while a copy issued on that stream when
// nothing is pending runs at once.  This is the order in which a copy engine
// finishes a small upload before slow kernels ahead of nothing; it lets a test
// catch a descriptor table that a call on another stream rewrites while a
// launch on this stream has yet to read it.  Every other stream runs at once.
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <functional>
#include <map>
#include <set>
#include <vector>

#include "common.hpp"
#include "kernels.hpp"

namespace {

struct Op {
    std::function<void()> run;
    long long id;          // > 0 for an event record: the event's record number
};

hipStream_t g_slow = nullptr;
std::deque<Op> g_queue;               // deferred work of the slow stream
long long g_next_record = 1;
std::map<hipEvent_t, long long> g_event_pending;   // event -> record number not yet run
int g_errors = 0;
long long g_groups_run = 0;

struct Capture {
    std::vector<std::function<void()>> ops;
};
std::map<hipStream_t, Capture*> g_capturing;
std::set<void*> g_live;               // live emulated allocations

void report(const char* what) {
    ++g_errors;
    std::fprintf(stderr, "emul: %s\n", what);
}

void flush_until(long long id) {
    while (!g_queue.empty()) {
        Op op = g_queue.front();
        g_queue.pop_front();
        if (op.run) op.run();
        if (op.id > 0) {
            for (auto it = g_event_pending.begin(); it != g_event_pending.end();) {
                if (it->second == op.id) it = g_event_pending.erase(it);
                else ++it;
            }
            if (op.id == id) return;
        }
    }
}

void flush_all() { flush_until(-1); }

// Issues f on stream st: recorded into a capture, deferred on the slow stream,
// else run at once.
void issue(hipStream_t st, std::function<void()> f, bool is_copy) {
    auto cap = g_capturing.find(st);
    if (cap != g_capturing.end()) {
        cap->second->ops.push_back(std::move(f));
        return;
    }
    if (st == g_slow && g_slow != nullptr && (!is_copy || !g_queue.empty())) {
        g_queue.push_back(Op{std::move(f), 0});
        return;
    }
    f();
}

template <class T>
void touch(const T* p, size_t n) {
    if (!p || n == 0) return;
    volatile char sink = 0;
    sink ^= reinterpret_cast<const volatile char*>(p)[0];
    sink ^= reinterpret_cast<const volatile char*>(p + n)[-1];
    (void)sink;
}

int tier(int r) { return r <= 8 ? 8 : r <= 16 ? 16 : r <= 32 ? 32 : r <= 64 ? 64 : 128; }
int acc_tier(int r) { return r <= 32 ? 2 : r <= 64 ? 4 : 8; }

// Which launcher a group reaches (the invariants a launch relies on differ).
enum Phase { P_STATS, P_SOLVE, P_FRAME, P_UPDATE, P_OUT, P_SAMPLE };

// What a kernel of the launch reads of one descriptor, and the launch-wide
// arguments it relies on: the grid covers the descriptor's shape, rank and
// rows; kernels instantiated per transform length see only that shape;
// kernels instantiated per rank tier see only that tier.
void check_frame(const tsl::Batch& b, const tsl::FrameArgs& a, Phase ph) {
    ++g_groups_run;
    if (a.n1 > b.n1 || a.n2 > b.n2) report("descriptor larger than its launch");
    if (a.r < 1 || a.r > b.r_max) report("descriptor rank above its launch's");
    if (a.mode == tsl::MODE_LINES && a.n_rows > b.rows_max) report("descriptor rows above the launch's capacity");
    const bool frame_route = a.mode == tsl::MODE_POINTS || !a.kspace;
    switch (ph) {
        case P_STATS:
            if (a.mode != b.mode) report("statistics launch mixes mask kinds");
            if (a.mode == tsl::MODE_LINES && b.table && acc_tier(a.r) != acc_tier(b.r_max))
                report("statistics launch mixes accumulator tiers");
            break;
        case P_SOLVE:
            if (b.table && tier(a.r) != tier(b.r_max)) report("solve launch mixes rank tiers");
            break;
        case P_FRAME:
            if (a.n1 != b.n1 || a.n2 != b.n2) report("frame-route launch mixes shapes");
            if (!frame_route) report("k-space frame in a frame-route launch");
            break;
        case P_UPDATE:
            if (a.n1 != b.n1 || a.n2 != b.n2) report("update launch mixes shapes");
            if (a.kspace != (b.kspace ? 1 : 0)) report("update launch mixes routes");
            break;
        case P_OUT:
            if ((a.r <= 32) != (b.r_max <= 32)) report("output launch mixes single- and multi-pass ranks");
            if (a.X_out && !b.want_x) report("output frame without output tiles");
            if (a.K_next > 0 && !b.want_sample) report("row draw without a draw block");
            break;
        case P_SAMPLE:
            break;
    }
    const size_t n1 = size_t(a.n1), n2 = size_t(a.n2), r = size_t(a.r);
    touch(a.A, n1 * r); touch(a.B, n2 * r); touch(a.Ahat, n1 * r); touch(a.Bhat, n2 * r);
    touch(a.dev, 1); touch(a.gamma64, r); touch(a.gamma32, r);
    touch(a.frame, n1 * n2); touch(a.Wb, n2 * r); touch(a.GA, n1 * r);
    touch(a.zm, size_t(tsl::n_sparts(a.n1)) * tsl::n_jparts(a.n2) * tsl::kSRows * r);
    touch(a.zw, size_t(tsl::n_sparts(a.n1)) * n2 * r);
    touch(a.bcopy, n2 * r);
    touch(a.acopy, n1 * r);
    touch(a.part, size_t(tsl::n_parts(a.n1, a.n2)) * tsl::slot_size(a.r));
    touch(a.hpart, size_t(tsl::n_hparts(a.n1, a.n2)) * r);
    touch(a.wq, size_t(tsl::cdiv(a.r, 16)) * n1);
    if (a.mode == tsl::MODE_LINES) {
        touch(a.rows, size_t(a.n_rows));
        touch(a.y, (a.y_full ? n1 : size_t(a.n_rows)) * n2);
    } else {
        touch(a.mask, n1 * n2);
        touch(a.y, n1 * n2);
    }
    touch(a.X_out, n1 * n2); touch(a.A_out, n1 * r); touch(a.B_out, n2 * r); touch(a.gamma_out, r);
    if (a.K_next > 0) { touch(a.rows_next, size_t(a.K_next)); touch(a.n_next, 1); }
    if (a.info_out) touch(a.info_out, 4);
}

hipError_t run_group(const tsl::Batch& b0, hipStream_t st, Phase ph) {
    tsl::Batch b = b0;
    tsl::FrameArgs one{};
    if (b.one) one = *b.one;          // a by-value descriptor is copied at launch, as a kernel argument is
    issue(st, [b, one, ph]() {
        if (b.one) { check_frame(b, one, ph); return; }
        for (int i = 0; i < b.count; ++i) check_frame(b, b.table[i], ph);
    }, false);
    return hipSuccess;
}

}  // namespace

// ------------------------------------------------------------ test controls
extern "C" void emul_set_slow_stream(void* st) { g_slow = reinterpret_cast<hipStream_t>(st); }
extern "C" int emul_errors() { return g_errors; }
extern "C" long long emul_groups_run() { return g_groups_run; }
extern "C" size_t emul_live_allocations() { return g_live.size(); }
extern "C" void emul_flush() { flush_all(); }

// ------------------------------------------------------------ launchers
namespace tsl {
hipError_t launch_synth_rowfft(const Batch& b, hipStream_t st) { return b.mode == MODE_POINTS || !b.kspace ? run_group(b, st, P_FRAME) : hipSuccess; }
hipError_t launch_row_inv_grad(const Batch& b, hipStream_t st) { return b.mode == MODE_POINTS || !b.kspace ? run_group(b, st, P_FRAME) : hipSuccess; }
hipError_t launch_col_resid(const Batch& b, hipStream_t st) { return b.mode == MODE_POINTS || !b.kspace ? run_group(b, st, P_FRAME) : hipSuccess; }
hipError_t launch_update_a(const Batch& b, hipStream_t st) { return run_group(b, st, P_UPDATE); }
hipError_t launch_update_b(const Batch& b, hipStream_t st) { return run_group(b, st, P_UPDATE); }
hipError_t launch_stats(const Batch& b, hipStream_t st) { return run_group(b, st, P_STATS); }
hipError_t launch_solve(const Batch& b, hipStream_t st) { return run_group(b, st, P_SOLVE); }
hipError_t launch_synth_out(const Batch& b, hipStream_t st) { return run_group(b, st, P_OUT); }
hipError_t launch_sample(const Batch& b, hipStream_t st) { return run_group(b, st, P_SAMPLE); }
hipError_t launch_coil_gain(const CoilArgs& a, hipStream_t st) {
    issue(st, [a]() { touch(a.H, size_t(a.C) * a.n1 * a.n2); touch(a.gain, 1); }, false);
    return hipSuccess;
}
hipError_t launch_coil_step(const CoilArgs& a, hipStream_t st) {
    issue(st, [a]() {
        const size_t P = size_t(a.n1) * a.n2, r = size_t(a.r);
        touch(a.A, a.n1 * r); touch(a.B, a.n2 * r); touch(a.Ahat, a.n1 * r); touch(a.Bhat, a.n2 * r);
        touch(a.dev, 1); touch(a.gamma64, r); touch(a.gamma32, r);
        touch(a.H, size_t(a.C) * P); touch(a.P, r * P); touch(a.Q, size_t(a.C) * P); touch(a.theta, P);
        touch(a.GA, a.n1 * r); touch(a.GB, a.n2 * r);
        touch(a.gslot, size_t(a.C) * a.n1 * r * r); touch(a.hslot, size_t(a.C) * a.n1 * r); touch(a.gain, 1);
        if (a.n_rows > 0) { touch(a.rows, size_t(a.n_rows)); touch(a.y, size_t(a.C) * a.n_rows * a.n2); }
        if (a.A_out) touch(a.A_out, a.n1 * r);
        if (a.B_out) touch(a.B_out, a.n2 * r);
        if (a.gamma_out) touch(a.gamma_out, r);
    }, false);
    return hipSuccess;
}
hipError_t launch_sample_points(const FrameArgs& a, int K, unsigned char* mask, int* n_out, int* draws,
                                hipStream_t st) {
    issue(st, [a, K, mask, n_out, draws]() {
        touch(a.Ahat, size_t(a.n1) * a.r); touch(a.Bhat, size_t(a.n2) * a.r); touch(a.dev, 1);
        touch(mask, size_t(a.n1) * a.n2); touch(n_out, 1);
        if (draws) touch(draws, size_t(K));
    }, false);
    return hipSuccess;
}
hipError_t launch_rowfft(int n1, int n2, int batch, const float2* in, float2* out, bool, hipStream_t st) {
    issue(st, [=]() { touch(in, size_t(batch) * n1 * n2); touch(out, size_t(batch) * n1 * n2); }, false);
    return hipSuccess;
}
hipError_t launch_colfft(int n1, int n2, int batch, const float2* in, float2* out, bool inv, hipStream_t st) {
    return launch_rowfft(n1, n2, batch, in, out, inv, st);
}
hipError_t launch_factor_fft(int n, int r, const float2* in, float2* out, bool, hipStream_t st) {
    issue(st, [=]() { touch(in, size_t(n) * r); touch(out, size_t(n) * r); }, false);
    return hipSuccess;
}
void init_kernel_attributes() {}
bool size_supported(int n) {
    switch (n) {
#define TSL_X(N) case N: return true;
        TSL_FOR_EACH_N(TSL_X)
#undef TSL_X
        default: return false;
    }
}
}  // namespace tsl

// ------------------------------------------------------------ runtime calls
extern "C" {

hipError_t hipMalloc(void** p, size_t n) {
    *p = std::malloc(n ? n : 1);
    g_live.insert(*p);
    return *p ? hipSuccess : hipErrorOutOfMemory;
}
hipError_t hipFree(void* p) {
    flush_all();                      // freeing device memory waits for the device
    if (p && !g_live.erase(p)) report("hipFree of an unknown pointer");
    std::free(p);
    return hipSuccess;
}
hipError_t hipHostMalloc(void** p, size_t n, unsigned int) { return hipMalloc(p, n); }
hipError_t hipHostFree(void* p) { return hipFree(p); }
hipError_t hipMemcpy(void* d, const void* s, size_t n, hipMemcpyKind) {
    flush_all();
    std::memcpy(d, s, n);
    return hipSuccess;
}
hipError_t hipMemcpyAsync(void* d, const void* s, size_t n, hipMemcpyKind, hipStream_t st) {
    issue(st, [=]() { std::memcpy(d, s, n); }, true);
    return hipSuccess;
}
hipError_t hipMemsetAsync(void* d, int v, size_t n, hipStream_t st) {
    issue(st, [=]() { std::memset(d, v, n); }, true);
    return hipSuccess;
}
hipError_t hipEventCreate(hipEvent_t* e) {
    *e = reinterpret_cast<hipEvent_t>(new int(0));
    return hipSuccess;
}
hipError_t hipEventCreateWithFlags(hipEvent_t* e, unsigned) { return hipEventCreate(e); }
hipError_t hipEventDestroy(hipEvent_t e) {
    g_event_pending.erase(e);
    delete reinterpret_cast<int*>(e);
    return hipSuccess;
}
hipError_t hipEventRecord(hipEvent_t e, hipStream_t st) {
    if (st == g_slow && g_slow != nullptr && !g_queue.empty()) {
        const long long id = g_next_record++;
        g_event_pending[e] = id;
        g_queue.push_back(Op{nullptr, id});
    } else {
        g_event_pending.erase(e);
    }
    return hipSuccess;
}
hipError_t hipEventSynchronize(hipEvent_t e) {
    auto it = g_event_pending.find(e);
    if (it != g_event_pending.end()) flush_until(it->second);
    return hipSuccess;
}
hipError_t hipEventElapsedTime(float* ms, hipEvent_t, hipEvent_t) {
    *ms = 0.0f;
    return hipSuccess;
}
hipError_t hipGetDevice(int* d) { *d = 0; return hipSuccess; }
hipError_t hipSetDevice(int) { return hipSuccess; }
const char* hipGetErrorString(hipError_t) { return "emulated HIP error"; }
hipError_t hipStreamCreateWithFlags(hipStream_t* s, unsigned) {
    *s = reinterpret_cast<hipStream_t>(new int(0));
    return hipSuccess;
}
hipError_t hipStreamDestroy(hipStream_t s) {
    delete reinterpret_cast<int*>(s);
    return hipSuccess;
}
hipError_t hipStreamSynchronize(hipStream_t) {
    flush_all();
    return hipSuccess;
}
hipError_t hipStreamBeginCapture(hipStream_t st, hipStreamCaptureMode) {
    if (g_capturing.count(st)) return hipErrorIllegalState;
    g_capturing[st] = new Capture();
    return hipSuccess;
}
hipError_t hipStreamEndCapture(hipStream_t st, hipGraph_t* g) {
    auto it = g_capturing.find(st);
    if (it == g_capturing.end()) return hipErrorIllegalState;
    *g = reinterpret_cast<hipGraph_t>(it->second);
    g_capturing.erase(it);
    return hipSuccess;
}
hipError_t hipGraphInstantiate(hipGraphExec_t* x, hipGraph_t g, hipGraphNode_t*, char*, size_t) {
    *x = reinterpret_cast<hipGraphExec_t>(new Capture(*reinterpret_cast<Capture*>(g)));
    return hipSuccess;
}
hipError_t hipGraphDestroy(hipGraph_t g) {
    delete reinterpret_cast<Capture*>(g);
    return hipSuccess;
}
hipError_t hipGraphExecDestroy(hipGraphExec_t x) {
    delete reinterpret_cast<Capture*>(x);
    return hipSuccess;
}
hipError_t hipGraphLaunch(hipGraphExec_t x, hipStream_t st) {
    for (const auto& f : reinterpret_cast<Capture*>(x)->ops) issue(st, f, false);
    return hipSuccess;
}

}  // extern "C"
