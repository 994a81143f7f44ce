// Host side of the library: sequence state and workspace, argument checks,
// the launch sequence of one step, batched steps replayed from HIP graphs, the
// admission pool and state checkpoints.  Exposed through the C ABI in tsl.h.
#include <algorithm>
#include <cmath>
#include <cstddef>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "engine.hpp"

namespace tsl {
namespace eng {

thread_local std::string g_err;

int fail(int code, const std::string& msg) {
    g_err = msg;
    return code;
}

int hip_fail(hipError_t e, const char* what) {
    g_err = std::string(what) + ": " + hipGetErrorString(e);
    return TSL_EDEVICE;
}

namespace {
size_t align256(size_t x) { return (x + 255) & ~size_t(255); }
}  // namespace

Layout layout_for(int n1, int n2, int r, int C) {
    Layout L{};
    size_t o = 0;
    auto take = [&](size_t bytes) { size_t at = o; o = align256(o + bytes); return at; };
    L.A = take(size_t(n1) * r * sizeof(float2));
    L.B = take(size_t(n2) * r * sizeof(float2));
    L.Ahat = take(size_t(n1) * r * sizeof(float2));
    L.Bhat = take(size_t(n2) * r * sizeof(float2));
    L.dev = take(sizeof(tsl::SeqDev));
    L.g64 = take(size_t(r) * sizeof(double2));
    L.g32 = take(size_t(r) * sizeof(float2));
    L.frame = take(size_t(n1) * n2 * sizeof(float2));
    L.Wb = take(size_t(n2) * r * sizeof(float2));
    L.GA = take(size_t(n1) * r * sizeof(float2));
    L.zm = take(size_t(tsl::n_sparts(n1)) * tsl::n_jparts(n2) * tsl::kSRows * r * sizeof(float2));
    L.zw = take(size_t(tsl::n_sparts(n1)) * n2 * r * sizeof(float2));
    L.bcopy = take(size_t(n2) * r * sizeof(float2));
    L.acopy = take(size_t(n1) * r * sizeof(float2));
    L.part = take(size_t(tsl::n_parts(n1, n2)) * tsl::slot_size(r) * sizeof(double2));
    L.hpart = take(size_t(tsl::n_hparts(n1, n2)) * r * sizeof(double2));
    L.wq = take(size_t(tsl::cdiv(r, 16)) * n1 * sizeof(double));
    if (C > 0) {
        const size_t P = size_t(n1) * n2;
        L.H = take(size_t(C) * P * sizeof(float2));
        L.P = take(size_t(r) * P * sizeof(float2));
        L.Q = take(size_t(C) * P * sizeof(float2));
        L.gslot = take(size_t(C) * n1 * r * r * sizeof(double2));
        L.hslot = take(size_t(C) * n1 * r * sizeof(double2));
        L.gain = take(sizeof(double));
    }
    L.total = o;
    return L;
}

// -------------------------------------------------------------- frame descriptors
tsl::FrameArgs frame_args(const tsl_seq* s, const tsl_frame& fr) {
    tsl::FrameArgs a{};
    a.n1 = s->n1; a.n2 = s->n2; a.r = s->r;
    a.mode = fr.mask ? tsl::MODE_POINTS : tsl::MODE_LINES;
    a.kspace = (!fr.mask && s->opts.line_route == TSL_ROUTE_KSPACE) ? 1 : 0;
    a.lambda = s->lambda; a.mu_const = s->opts.mu; a.step_mode = s->opts.step_mode;
    a.synth_bf16 = s->opts.synth_bf16;
    a.n_rows = fr.mask ? 0 : fr.n_rows;
    a.A = s->at<float2>(s->lay.A); a.B = s->at<float2>(s->lay.B);
    a.Ahat = s->at<float2>(s->lay.Ahat); a.Bhat = s->at<float2>(s->lay.Bhat);
    a.dev = s->at<tsl::SeqDev>(s->lay.dev);
    a.gamma64 = s->at<double2>(s->lay.g64); a.gamma32 = s->at<float2>(s->lay.g32);
    a.frame = s->at<float2>(s->lay.frame); a.Wb = s->at<float2>(s->lay.Wb); a.GA = s->at<float2>(s->lay.GA);
    a.zm = s->at<float2>(s->lay.zm);
    a.zw = s->at<float2>(s->lay.zw);
    a.bcopy = s->at<float2>(s->lay.bcopy);
    a.acopy = s->at<float2>(s->lay.acopy);
    a.part = s->at<double2>(s->lay.part); a.hpart = s->at<double2>(s->lay.hpart);
    a.rows = fr.rows; a.n_rows_dev = fr.mask ? nullptr : fr.n_rows_dev; a.y_full = fr.y_full ? 1 : 0;
    a.mask = fr.mask; a.y = reinterpret_cast<const float2*>(fr.y);
    a.X_out = reinterpret_cast<float2*>(fr.X_out); a.A_out = reinterpret_cast<float2*>(fr.A_out);
    a.B_out = reinterpret_cast<float2*>(fr.B_out); a.gamma_out = reinterpret_cast<float2*>(fr.gamma_out);
    a.K_next = fr.K_next > 0 ? fr.K_next : 0;
    a.rows_next = fr.rows_next; a.n_next = fr.n_next;
    a.draws_next = nullptr; a.prefix_next = nullptr;
    a.seed = s->opts.seed; a.sid = s->opts.stream_id;
    a.info_out = fr.info_out;
    a.wq = s->at<double>(s->lay.wq);
    return a;
}

namespace {
hipError_t launch_updates(const tsl::Batch& b, hipStream_t st) {
    hipError_t e = tsl::launch_update_a(b, st);
    return e != hipSuccess ? e : tsl::launch_update_b(b, st);
}

// The phases of one step (Algorithm 3 with one coil; Algorithm 4's draw of the
// next rows runs inside the output launch, beside the output tiles).  A group
// runs the three frame-route phases, or none of them on the k-space route,
// whose residual contractions the statistics and update launches take over;
// the launchers of phases a group does not run return at once.
using PhaseFn = hipError_t (*)(const tsl::Batch&, hipStream_t);
struct Phase {
    PhaseFn fn;
    const char* name;
};
const Phase kPhases[TSL_N_PHASES] = {
    {tsl::launch_stats, "partial Grams"},                  // a2
    {tsl::launch_solve, "ridge solve + step size"},        // a3, a8
    {tsl::launch_synth_rowfft, "synthesis + row pass"},    // a4, a5 (rows)
    {tsl::launch_col_resid, "column pass + residual"},     // a5 (columns), a6, a7 (columns)
    {tsl::launch_row_inv_grad, "row inverse + A grad"},    // a7 (rows), a9
    {launch_updates, "factor updates + F_l A, F_r B"},     // a9, a1 (one launch when n1 == n2); k-space: a6, a7
    {tsl::launch_synth_out, "output synthesis + row draw"},  // a10; a11 in one more block per frame
};

}  // namespace

int run_groups(const tsl::Batch* groups, int n_groups, hipStream_t st, hipEvent_t* ev) {
    for (int p = 0; p < TSL_N_PHASES; ++p) {
        if (ev) TSL_HIP(hipEventRecord(ev[p], st));
        for (int g = 0; g < n_groups; ++g) {
            hipError_t e = kPhases[p].fn(groups[g], st);
            if (e != hipSuccess) return hip_fail(e, kPhases[p].name);
        }
    }
    if (ev) TSL_HIP(hipEventRecord(ev[TSL_N_PHASES], st));
    return TSL_OK;
}

int check_frame(const tsl_seq* s, const tsl_frame& fr) {
    if (s->C > 0) return fail(TSL_EINVAL, "a several-coil sequence takes its frames through tsl_push_coils");
    if (fr.mask) {
        if (fr.rows) return fail(TSL_EINVAL, "a frame has both rows and a mask");
        if (!fr.y) return fail(TSL_EINVAL, "null y");
    } else if (fr.n_rows_dev) {
        if (!fr.rows || !fr.y) return fail(TSL_EINVAL, "a device row count needs rows and y");
    } else {
        if (fr.n_rows < 0 || fr.n_rows > s->n1) return fail(TSL_EINVAL, "n_rows must be in [0, n1]");
        if (fr.n_rows > 0 && (!fr.rows || !fr.y)) return fail(TSL_EINVAL, "null rows or y");
    }
    if (fr.K_next < 0) return fail(TSL_EINVAL, "K_next must be >= 0");
    if (fr.K_next > 0 && (!fr.rows_next || !fr.n_next)) return fail(TSL_EINVAL, "null rows_next or n_next");
    return TSL_OK;
}

int rank_tier(int r) {
    return r <= 8 ? 8 : r <= 16 ? 16 : r <= 32 ? 32 : r <= 64 ? 64 : TSL_MAX_R;
}

FrameFacts frame_facts(const tsl_seq* s, const tsl_frame& fr) {
    FrameFacts x{};
    x.n1 = s->n1; x.n2 = s->n2; x.r = s->r;
    x.mode = fr.mask ? MODE_POINTS : MODE_LINES;
    x.kspace = (!fr.mask && s->opts.line_route == TSL_ROUTE_KSPACE) ? 1 : 0;
    x.cap = fr.mask ? s->n1 : std::min(std::max(fr.n_rows, 0), s->n1);
    x.want_x = fr.X_out != nullptr;
    x.want_sample = fr.K_next > 0;
    x.synth = s->opts.synth_bf16;
    return x;
}

namespace {

// Rank tier of the statistics and k-space residual kernels (accumulator tiles).
int acc_tier(int r) { return r <= 32 ? 2 : r <= 64 ? 4 : 8; }
bool on_frame_route(const FrameFacts& a) { return a.mode == MODE_POINTS || !a.kspace; }

// The phases in launch order (see kPhases) and the table order each reads.
bool phase_reads_b(int p) { return p == 2 || p == 3 || p == 4 || p == 5; }

// True if frames a and b (adjacent in the phase's table order) share one launch
// of phase p: the same kernel instantiation and launch-wide arguments.
bool same_launch(int p, const FrameFacts& a, const FrameFacts& b) {
    switch (p) {
        case 0: return a.mode == b.mode && (a.mode == MODE_POINTS || acc_tier(a.r) == acc_tier(b.r));
        case 1: return rank_tier(a.r) == rank_tier(b.r);
        case 2: case 3: case 4:
            return on_frame_route(a) == on_frame_route(b) && (!on_frame_route(a) || (a.n1 == b.n1 && a.n2 == b.n2));
        case 5: return a.n1 == b.n1 && a.n2 == b.n2 && a.kspace == b.kspace;
        default: return (a.r <= 32) == (b.r <= 32) && a.synth == b.synth;
    }
}

template <class Less> void stable_order(int n, int* order, Less less) {
    for (int i = 0; i < n; ++i) order[i] = i;
    if (n <= 256) {                          // insertion sort: no heap use (the allocation-free path)
        for (int i = 1; i < n; ++i) {
            const int v = order[i];
            int p = i;
            while (p > 0 && less(v, order[p - 1])) { order[p] = order[p - 1]; --p; }
            order[p] = v;
        }
    } else {
        std::stable_sort(order, order + n, less);
    }
}

}  // namespace

bool table_orders(const FrameFacts* f, int n, int* order_a, int* order_b) {
    auto key_a = [&](int i) { return std::make_tuple(rank_tier(f[i].r), f[i].mode, f[i].kspace, f[i].n1, f[i].n2); };
    auto key_b = [&](int i) { return std::make_tuple(f[i].n1, f[i].n2, f[i].mode, f[i].kspace, rank_tier(f[i].r)); };
    stable_order(n, order_a, [&](int a, int b) { return key_a(a) < key_a(b); });
    stable_order(n, order_b, [&](int a, int b) { return key_b(a) < key_b(b); });
    for (int i = 0; i < n; ++i)
        if (order_a[i] != order_b[i]) return false;
    return true;
}

int launch_phases(const FrameFacts* fa, const FrameArgs* ta, const FrameFacts* fb, const FrameArgs* tb, int n,
                  hipStream_t st, hipEvent_t* ev) {
    for (int p = 0; p < TSL_N_PHASES; ++p) {
        if (ev) TSL_HIP(hipEventRecord(ev[p], st));
        const bool useb = phase_reads_b(p);
        const FrameFacts* f = useb ? fb : fa;
        const FrameArgs* t = useb ? tb : ta;
        for (int i = 0; i < n;) {
            int j = i + 1;
            while (j < n && same_launch(p, f[i], f[j])) ++j;
            Batch b{};
            b.one = nullptr;
            b.table = t + i;
            b.count = j - i;
            b.mode = f[i].mode;
            b.kspace = f[i].kspace != 0;
            b.synth = f[i].synth;
            b.out_tile = OUT_128x64;
            for (int q = i; q < j; ++q) {
                b.n1 = std::max(b.n1, f[q].n1);
                b.n2 = std::max(b.n2, f[q].n2);
                b.r_max = std::max(b.r_max, f[q].r);
                b.rows_max = std::max(b.rows_max, f[q].cap);
                b.want_x = b.want_x || f[q].want_x;
                b.want_sample = b.want_sample || f[q].want_sample;
            }
            if (p == TSL_N_PHASES - 1 && b.synth == 0) b.out_tile = output_tile(b.n1, b.n2, b.r_max <= 32, b.count);
            hipError_t e = kPhases[p].fn(b, st);
            if (e != hipSuccess) return hip_fail(e, kPhases[p].name);
            i = j;
        }
    }
    if (ev) TSL_HIP(hipEventRecord(ev[TSL_N_PHASES], st));
    return TSL_OK;
}

// -------------------------------------------------------------- output-tile tuner
namespace {

std::mutex g_tune_mu;
std::map<std::tuple<int, int, int, int>, int> g_tune;   // (n1, n2, one pass, count bucket) -> OUT_*
bool g_tune_loaded = false;

int count_bucket(int count) {
    int b = 1;
    while (b < count) b *= 2;
    return b;
}

const char* tune_cache_path() { return std::getenv("TSL_TUNE_CACHE"); }

// Records "n1 n2 one bucket tile" per line.
void load_tune_cache_locked() {
    if (g_tune_loaded) return;
    g_tune_loaded = true;
    const char* path = tune_cache_path();
    if (!path || !*path) return;
    if (FILE* fh = std::fopen(path, "r")) {
        int a, b, c, d, e;
        while (std::fscanf(fh, "%d %d %d %d %d", &a, &b, &c, &d, &e) == 5)
            if (e >= 0 && e < OUT_TILES) g_tune[std::make_tuple(a, b, c, d)] = e;
        std::fclose(fh);
    }
}

}  // namespace

int output_tile(int n1, int n2, bool one_pass, int count) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    load_tune_cache_locked();
    auto it = g_tune.find(std::make_tuple(n1, n2, one_pass ? 1 : 0, count_bucket(count)));
    return it == g_tune.end() ? int(OUT_128x64) : it->second;
}

void set_output_tile(int n1, int n2, bool one_pass, int count, int tile) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    load_tune_cache_locked();
    g_tune[std::make_tuple(n1, n2, one_pass ? 1 : 0, count_bucket(count))] = tile;
}

int tune_output_runs(const FrameFacts* fa, const FrameArgs* host, int n) {
    const char* off = std::getenv("TSL_TUNE");
    if (off && off[0] == '0') return TSL_OK;
    constexpr int P7 = TSL_N_PHASES - 1;
    for (int i = 0; i < n;) {
        int j = i + 1;
        while (j < n && same_launch(P7, fa[i], fa[j])) ++j;
        int n1 = 0, n2 = 0, r_max = 0, rows_max = 0;
        bool any_x = false;
        for (int q = i; q < j; ++q) {
            n1 = std::max(n1, fa[q].n1); n2 = std::max(n2, fa[q].n2); r_max = std::max(r_max, fa[q].r);
            rows_max = std::max(rows_max, fa[q].cap);
            any_x = any_x || fa[q].want_x;
        }
        const auto key = std::make_tuple(n1, n2, r_max <= 32 ? 1 : 0, count_bucket(j - i));
        bool known;
        {
            std::lock_guard<std::mutex> lk(g_tune_mu);
            load_tune_cache_locked();
            known = g_tune.count(key) > 0;
        }
        if (known || !any_x || fa[i].synth != 0) { i = j; continue; }
        // scratch copies of the run's descriptors: X and the drawn rows into
        // scratch buffers, and a status word that lets the output tiles run
        const int m = j - i;
        std::vector<FrameArgs> tmp(host + i, host + j);
        size_t kall = 0;
        for (const FrameArgs& fa_ : tmp) kall += size_t(fa_.K_next > 0 ? fa_.K_next : 0) + 1;
        int* rs = nullptr;
        float2* xs = nullptr;
        FrameArgs* table = nullptr;
        SeqDev* sd = nullptr;
        hipStream_t ts = nullptr;
        hipEvent_t e0 = nullptr, e1 = nullptr;
        auto cleanup = [&]() {
            if (ts) hipStreamSynchronize(ts);
            if (xs) hipFree(xs);
            if (rs) hipFree(rs);
            if (table) hipFree(table);
            if (sd) hipFree(sd);
            if (e0) hipEventDestroy(e0);
            if (e1) hipEventDestroy(e1);
            if (ts) hipStreamDestroy(ts);
        };
        hipError_t e = hipMalloc(&xs, size_t(m) * n1 * n2 * sizeof(float2));
        if (e == hipSuccess) e = hipMalloc(&rs, kall * sizeof(int));
        if (e == hipSuccess) e = hipMalloc(&table, size_t(m) * sizeof(FrameArgs));
        if (e == hipSuccess) e = hipMalloc(&sd, sizeof(SeqDev));
        if (e == hipSuccess) e = hipStreamCreateWithFlags(&ts, hipStreamNonBlocking);
        if (e == hipSuccess) e = hipEventCreate(&e0);
        if (e == hipSuccess) e = hipEventCreate(&e1);
        if (e != hipSuccess) { cleanup(); return hip_fail(e, "output tuner"); }
        SeqDev ok{};
        ok.frame_ok = 1;
        bool any_draw = false;
        size_t ko = 0;
        for (int q = 0; q < m; ++q) {
            tmp[q].X_out = xs + size_t(q) * n1 * n2;
            if (tmp[q].K_next > 0) {
                any_draw = true;
                tmp[q].rows_next = rs + ko;
                ko += size_t(tmp[q].K_next);
                tmp[q].n_next = rs + ko;
                ko += 1;
            }
            tmp[q].draws_next = nullptr;
            tmp[q].prefix_next = nullptr;
            tmp[q].info_out = nullptr;
            tmp[q].dev = sd;
        }
        e = hipMemcpy(table, tmp.data(), size_t(m) * sizeof(FrameArgs), hipMemcpyHostToDevice);
        if (e == hipSuccess) e = hipMemcpy(sd, &ok, sizeof(ok), hipMemcpyHostToDevice);
        Batch b{};
        b.table = table; b.count = m; b.n1 = n1; b.n2 = n2; b.r_max = r_max; b.rows_max = rows_max;
        b.mode = fa[i].mode;
        b.want_x = true; b.want_sample = any_draw; b.synth = 0;
        // three rounds over the tiles (interleaved, so drift hits all alike),
        // each tile's best round kept
        float tile_ms[OUT_TILES];
        for (float& x : tile_ms) x = 1e30f;
        for (int round = 0; round < 3 && e == hipSuccess; ++round)
            for (int v = 0; v < OUT_TILES && e == hipSuccess; ++v) {
                b.out_tile = v;
                e = launch_synth_out(b, ts);                 // warm-up
                if (e == hipSuccess) e = hipEventRecord(e0, ts);
                constexpr int kReps = 5;
                for (int k = 0; k < kReps && e == hipSuccess; ++k) e = launch_synth_out(b, ts);
                if (e == hipSuccess) e = hipEventRecord(e1, ts);
                if (e == hipSuccess) e = hipEventSynchronize(e1);
                float ms = 0.f;
                if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
                if (e == hipSuccess) tile_ms[v] = std::min(tile_ms[v], ms);
            }
        int best = OUT_128x64;
        for (int v = 0; v < OUT_TILES; ++v)
            if (tile_ms[v] < tile_ms[best]) best = v;
        cleanup();
        if (e != hipSuccess) return hip_fail(e, "output tuner");
        {
            std::lock_guard<std::mutex> lk(g_tune_mu);
            g_tune[key] = best;
            const char* path = tune_cache_path();
            if (path && *path)
                if (FILE* fh = std::fopen(path, "a")) {
                    std::fprintf(fh, "%d %d %d %d %d\n", std::get<0>(key), std::get<1>(key), std::get<2>(key),
                                 std::get<3>(key), best);
                    std::fclose(fh);
                }
        }
        i = j;
    }
    return TSL_OK;
}

}  // namespace eng
}  // namespace tsl

using namespace tsl::eng;

namespace {

std::mutex g_graph_mu;

int run_groups(const std::vector<tsl::Batch>& groups, hipStream_t st, hipEvent_t* ev = nullptr) {
    return tsl::eng::run_groups(groups.data(), int(groups.size()), st, ev);
}

int check_seq(const tsl_seq* s) {
    if (!s) return fail(TSL_EINVAL, "null sequence handle");
    return TSL_OK;
}

int set_dev(const tsl_seq* s) {
    TSL_HIP(hipSetDevice(s->device));
    return TSL_OK;
}

// -------------------------------------------------------------- batched step state
struct Composition {
    std::vector<const tsl_seq*> seqs;     // in the order of the call
    std::vector<int> wants;               // per frame: bit0 X, bit4 points, bit5 row draw, bit6 frame route
    std::vector<int> caps;                // per frame: row capacity (sizes the statistics grid)
    std::vector<int> order_a, order_b;    // frame indices in table orders A and B (table_orders)
    std::vector<tsl::eng::FrameFacts> fa, fb;   // the facts in those orders
    bool same = true;                     // order B == order A: the table holds n entries, else 2n
    int entries() const { return int(seqs.size()) * (same ? 1 : 2); }
    bool operator==(const Composition& o) const {
        return seqs == o.seqs && wants == o.wants && caps == o.caps;
    }
};

// One slot of the descriptor ring: pinned host staging, the device table the
// kernels of a step read, the event recorded after that step's launches, and
// the graph captured over this slot's table.  A slot is reused only after the
// host has waited for its event, so neither its staging buffer nor its device
// table is rewritten while a step that reads them may still run, whatever
// stream either step was issued on.  The wait also bounds how far the host runs
// ahead of the GPU (kRing steps); a deeper queue has been seen to stall the
// host for milliseconds while the runtime drains it.
struct Slot {
    tsl::FrameArgs* host = nullptr;       // pinned staging
    tsl::FrameArgs* table = nullptr;      // device table
    size_t cap = 0;                       // entries of both
    hipEvent_t done = nullptr;            // recorded after the last step that used the slot
    Composition comp;                     // composition of `exec`
    hipGraphExec_t exec = nullptr;
};

struct BatchEngine {
    int device = -1;
    hipStream_t cap = nullptr;            // capture stream (never executes work)
    static constexpr int kRing = 3;
    Slot slot[kRing];
    int ring_pos = 0;
    Composition last;                     // composition of the previous call
};

BatchEngine g_batch;

}  // namespace

// A step fixed at creation: its descriptors live in device memory of its own,
// and its launches are either issued directly or replayed from a graph of its own.
struct tsl_batch {
    int device = -1;
    bool dead = false;                    // one of its sequences was closed
    bool launched = false;
    std::vector<tsl_seq*> seqs;
    Composition comp;                     // the frames' order and launch facts over `table`
    tsl::FrameArgs* table = nullptr;
    hipGraphExec_t exec = nullptr;
    hipStream_t last = nullptr;
    ~tsl_batch() {
        if (exec) hipGraphExecDestroy(exec);
        if (table) hipFree(table);
    }
};

namespace {

std::vector<tsl_batch*> g_live_batches;   // guarded by g_graph_mu

void drop_graph(Slot& sl) {
    if (sl.exec) hipGraphExecDestroy(sl.exec);
    sl.exec = nullptr;
    sl.comp = Composition{};
}

void drop_graphs(BatchEngine& be) {
    for (Slot& sl : be.slot) drop_graph(sl);
}

// Takes the next ring slot for a step of n frames: waits (host) for the last
// step that used it, then grows its buffers if needed.  Returns its index.
int take_slot(BatchEngine& be, size_t n, int* slot_out) {
    int dev = 0;
    TSL_HIP(hipGetDevice(&dev));
    if (be.device != dev) {
        // buffers of another device: wait for their last use, then release them
        for (Slot& sl : be.slot) {
            if (sl.done) hipEventSynchronize(sl.done);
            drop_graph(sl);
            if (sl.table) hipFree(sl.table);
            if (sl.host) hipHostFree(sl.host);
            if (sl.done) hipEventDestroy(sl.done);
            sl = Slot{};
        }
        if (be.cap) hipStreamDestroy(be.cap);
        be.cap = nullptr;
        be.device = dev;
        be.last = Composition{};
        TSL_HIP(hipStreamCreateWithFlags(&be.cap, hipStreamNonBlocking));
    }
    const int k = be.ring_pos;
    Slot& sl = be.slot[k];
    if (!sl.done) TSL_HIP(hipEventCreateWithFlags(&sl.done, hipEventDisableTiming));
    TSL_HIP(hipEventSynchronize(sl.done));
    if (sl.cap < n) {
        drop_graph(sl);
        if (sl.table) hipFree(sl.table);
        if (sl.host) hipHostFree(sl.host);
        sl.table = nullptr;
        sl.host = nullptr;
        sl.cap = 0;
        const size_t cap = n < 64 ? 64 : n;
        TSL_HIP(hipMalloc(&sl.table, cap * sizeof(tsl::FrameArgs)));
        TSL_HIP(hipHostMalloc(&sl.host, cap * sizeof(tsl::FrameArgs), hipHostMallocDefault));
        sl.cap = cap;
    }
    be.ring_pos = (k + 1) % BatchEngine::kRing;
    *slot_out = k;
    return TSL_OK;
}

// Validates a batch and orders its frames (table_orders).
int compose(tsl_seq* const* seqs, int n, const tsl_frame* frames, Composition& c) {
    c.seqs.resize(n);
    c.wants.resize(n);
    c.caps.resize(n);
    std::vector<tsl::eng::FrameFacts> facts(n);
    for (int i = 0; i < n; ++i) {
        const tsl_seq* s = seqs[i];
        if (!s) return fail(TSL_EINVAL, "null sequence in batch");
        for (int j = 0; j < i; ++j)
            if (seqs[j] == s) return fail(TSL_EINVAL, "a sequence appears twice in one batch");
        int rc = check_frame(s, frames[i]);
        if (rc != TSL_OK) return rc;
        c.seqs[i] = s;
        c.wants[i] = (frames[i].X_out ? 1 : 0) | (frames[i].mask ? 16 : 0) | (frames[i].K_next > 0 ? 32 : 0) |
                     (!frames[i].mask && s->opts.line_route == TSL_ROUTE_FRAME ? 64 : 0);
        facts[i] = frame_facts(s, frames[i]);
        c.caps[i] = facts[i].cap;
    }
    c.order_a.resize(n);
    c.order_b.resize(n);
    c.same = table_orders(facts.data(), n, c.order_a.data(), c.order_b.data());
    c.fa.resize(n);
    c.fb.resize(n);
    for (int p = 0; p < n; ++p) {
        c.fa[p] = facts[c.order_a[p]];
        c.fb[p] = facts[c.order_b[p]];
    }
    return TSL_OK;
}

// The launches of a composed batch whose table starts at `table`.
int run_composition(const Composition& c, const tsl::FrameArgs* table, hipStream_t st, hipEvent_t* ev = nullptr) {
    const int n = int(c.seqs.size());
    return launch_phases(c.fa.data(), table, c.fb.data(), c.same ? table : table + n, n, st, ev);
}

// Host descriptors of a composed batch: order A, then (if it differs) order B.
void fill_descriptors(const Composition& c, tsl_seq* const* seqs, const tsl_frame* frames, tsl::FrameArgs* out) {
    const int n = int(c.seqs.size());
    for (int p = 0; p < n; ++p) out[p] = frame_args(seqs[c.order_a[p]], frames[c.order_a[p]]);
    if (!c.same)
        for (int p = 0; p < n; ++p) out[n + p] = frame_args(seqs[c.order_b[p]], frames[c.order_b[p]]);
}

// Writes the descriptors of a composed batch into the slot's pinned staging
// buffer and copies them to the slot's device table on `st`.
int stage_table(Slot& sl, const Composition& c, tsl_seq* const* seqs, const tsl_frame* frames, hipStream_t st) {
    const size_t m = size_t(c.entries());
    if (m > sl.cap) return fail(TSL_EINVAL, "internal: descriptor slot too small");
    for (const tsl_seq* q : c.seqs) const_cast<tsl_seq*>(q)->last = st;
    fill_descriptors(c, seqs, frames, sl.host);
    TSL_HIP(hipMemcpyAsync(sl.table, sl.host, m * sizeof(tsl::FrameArgs), hipMemcpyHostToDevice, st));
    return TSL_OK;
}

}  // namespace

// ====================================================================== C ABI
extern "C" {

void tsl_opts_default(tsl_opts* o) {
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->step_mode = TSL_STEP_MM;
    o->mu = 0.0;
    o->allow_lambda0 = 0;
    o->line_route = TSL_ROUTE_KSPACE;
    o->synth_bf16 = TSL_SYNTH_FP32;
}

int tsl_size_supported(int n) { return tsl::size_supported(n) ? 1 : 0; }

static int validate_shape(int n1, int n2, int r) {
    if (!tsl::size_supported(n1) || !tsl::size_supported(n2))
        return fail(TSL_EUNSUPPORTED, "n1 and n2 must be supported transform lengths (see tsl_size_supported)");
    if (r < 1 || r > TSL_MAX_R) return fail(TSL_EINVAL, "r must be in [1, TSL_MAX_R]");
    return TSL_OK;
}

int tsl_footprint(int n1, int n2, int r, size_t* bytes) {
    int rc = validate_shape(n1, n2, r);
    if (rc != TSL_OK) return rc;
    if (!bytes) return fail(TSL_EINVAL, "null bytes");
    *bytes = layout_for(n1, n2, r).total;
    return TSL_OK;
}

const char* tsl_last_error(void) { return g_err.c_str(); }

// The checks tsl_open applies to lambda and the options (also applied to a
// checkpoint's values by tsl_set_state).
static int validate_params(double lambda, const tsl_opts& o) {
    if (!std::isfinite(lambda) || lambda < 0.0) return fail(TSL_EINVAL, "lambda must be finite and >= 0");
    if (lambda == 0.0 && !o.allow_lambda0) return fail(TSL_EINVAL, "lambda == 0 needs allow_lambda0");
    if (o.step_mode != TSL_STEP_MM && o.step_mode != TSL_STEP_CONST) return fail(TSL_EINVAL, "bad step_mode");
    if (o.line_route != TSL_ROUTE_KSPACE && o.line_route != TSL_ROUTE_FRAME) return fail(TSL_EINVAL, "bad line_route");
    if (o.synth_bf16 != TSL_SYNTH_FP32 && o.synth_bf16 != TSL_SYNTH_BF16 && o.synth_bf16 != TSL_SYNTH_BF16X3)
        return fail(TSL_EINVAL, "bad synth_bf16");
    if (o.step_mode == TSL_STEP_CONST && !(o.mu > 0.0 && std::isfinite(o.mu)))
        return fail(TSL_EINVAL, "constant step needs a finite mu > 0");
    return TSL_OK;
}

static int open_impl(tsl_pool* pool, tsl_seq** out, int n1, int n2, int r, double lambda, const tsl_opts* opts,
                     const tsl_c32* A0, const tsl_c32* B0, void* stream, int C = 0, const tsl_c32* H = nullptr) {
    if (!out) return fail(TSL_EINVAL, "null output handle");
    *out = nullptr;
    int rc = validate_shape(n1, n2, r);
    if (rc != TSL_OK) return rc;
    tsl_opts o;
    tsl_opts_default(&o);
    if (opts) o = *opts;
    if ((rc = validate_params(lambda, o)) != TSL_OK) return rc;
    if (!A0 || !B0) return fail(TSL_EINVAL, "null A0 or B0");
    if (C > 0 && !H) return fail(TSL_EINVAL, "null coil maps");
    Layout L = layout_for(n1, n2, r, C);
    tsl::init_kernel_attributes();
    if (pool) {
        std::lock_guard<std::mutex> lk(pool->mu);
        if (pool->used + L.total > pool->budget) return fail(TSL_EBUSY, "pool budget exhausted");
        pool->used += L.total;
    }
    auto release = [&]() {
        if (pool) {
            std::lock_guard<std::mutex> lk(pool->mu);
            pool->used -= L.total;
        }
    };
    tsl_seq* s = new tsl_seq();
    s->n1 = n1; s->n2 = n2; s->r = r; s->lambda = lambda; s->opts = o; s->lay = L; s->bytes = L.total;
    s->C = C;
    s->pool = pool;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    s->last = st;
    hipError_t e = hipGetDevice(&s->device);
    if (e == hipSuccess) e = hipMalloc(&s->arena, L.total);
    if (e != hipSuccess) {
        delete s;
        release();
        return e == hipErrorOutOfMemory ? fail(TSL_ENOMEM, "device allocation failed")
                                        : hip_fail(e, "hipMalloc");
    }
    auto bail = [&](hipError_t err, const char* what) {
        hipFree(s->arena);
        delete s;
        release();
        return hip_fail(err, what);
    };
    if ((e = hipMemsetAsync(s->arena, 0, L.total, st)) != hipSuccess) return bail(e, "memset");
    if ((e = hipMemcpyAsync(s->at<void>(L.A), A0, size_t(n1) * r * sizeof(float2), hipMemcpyDeviceToDevice, st)) !=
        hipSuccess)
        return bail(e, "copy A0");
    if ((e = hipMemcpyAsync(s->at<void>(L.B), B0, size_t(n2) * r * sizeof(float2), hipMemcpyDeviceToDevice, st)) !=
        hipSuccess)
        return bail(e, "copy B0");
    if ((e = tsl::launch_factor_fft(n1, r, s->at<float2>(L.A), s->at<float2>(L.Ahat), false, st)) != hipSuccess)
        return bail(e, "F_l A0");
    if ((e = tsl::launch_factor_fft(n2, r, s->at<float2>(L.B), s->at<float2>(L.Bhat), false, st)) != hipSuccess)
        return bail(e, "F_r B0");
    if (C > 0) {
        if ((e = hipMemcpyAsync(s->at<void>(L.H), H, size_t(C) * n1 * n2 * sizeof(float2), hipMemcpyDeviceToDevice,
                                st)) != hipSuccess)
            return bail(e, "copy coil maps");
        tsl::CoilArgs ca{};
        ca.n1 = n1; ca.n2 = n2; ca.C = C;
        ca.H = s->at<float2>(L.H);
        ca.gain = s->at<double>(L.gain);
        if ((e = tsl::launch_coil_gain(ca, st)) != hipSuccess) return bail(e, "coil gain");
    }
    *out = s;
    return TSL_OK;
}

int tsl_open_coils(tsl_seq** out, int n1, int n2, int r, int C, double lambda, const tsl_opts* opts,
                   const tsl_c32* A0, const tsl_c32* B0, const tsl_c32* H, void* stream) {
    if (C < 1 || C > TSL_MAX_COILS) return fail(TSL_EINVAL, "C must be in [1, TSL_MAX_COILS]");
    if (r > TSL_MAX_COIL_R) return fail(TSL_EINVAL, "a several-coil sequence takes r <= TSL_MAX_COIL_R");
    return open_impl(nullptr, out, n1, n2, r, lambda, opts, A0, B0, stream, C, H);
}

int tsl_push_coils(tsl_seq* s, int n_rows, const int32_t* rows, const tsl_c32* y, tsl_c32* X_out, tsl_c32* A_out,
                   tsl_c32* B_out, tsl_c32* gamma_out, void* stream) {
    if (!s) return fail(TSL_EINVAL, "null sequence handle");
    if (s->C <= 0) return fail(TSL_EINVAL, "tsl_push_coils needs a sequence opened with tsl_open_coils");
    if (n_rows < 0 || n_rows > s->n1) return fail(TSL_EINVAL, "n_rows must be in [0, n1]");
    if (n_rows > 0 && (!rows || !y)) return fail(TSL_EINVAL, "null rows or y");
    TSL_HIP(hipSetDevice(s->device));
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    s->last = st;
    const Layout& L = s->lay;
    tsl::CoilArgs a{};
    a.n1 = s->n1; a.n2 = s->n2; a.r = s->r; a.C = s->C; a.n_rows = n_rows; a.step_mode = s->opts.step_mode;
    a.lambda = s->lambda; a.mu_const = s->opts.mu;
    a.A = s->at<float2>(L.A); a.B = s->at<float2>(L.B); a.Ahat = s->at<float2>(L.Ahat); a.Bhat = s->at<float2>(L.Bhat);
    a.dev = s->at<tsl::SeqDev>(L.dev);
    a.gamma64 = s->at<double2>(L.g64); a.gamma32 = s->at<float2>(L.g32);
    a.H = s->at<float2>(L.H); a.P = s->at<float2>(L.P); a.Q = s->at<float2>(L.Q);
    a.theta = s->at<float2>(L.frame); a.GA = s->at<float2>(L.GA); a.GB = s->at<float2>(L.Wb);
    a.gslot = s->at<double2>(L.gslot); a.hslot = s->at<double2>(L.hslot); a.gain = s->at<double>(L.gain);
    a.rows = rows; a.y = reinterpret_cast<const float2*>(y);
    a.A_out = reinterpret_cast<float2*>(A_out); a.B_out = reinterpret_cast<float2*>(B_out);
    a.gamma_out = reinterpret_cast<float2*>(gamma_out);
    hipError_t e = tsl::launch_coil_step(a, st);
    if (e != hipSuccess) return hip_fail(e, "several-coil step");
    if (X_out) {
        // X_t = A[t] diag(gamma_t) B[t]^T, the output launch of the single-coil step
        tsl::FrameArgs fa{};
        fa.n1 = s->n1; fa.n2 = s->n2; fa.r = s->r; fa.mode = tsl::MODE_LINES;
        fa.A = a.A; fa.B = a.B; fa.Ahat = a.Ahat; fa.Bhat = a.Bhat; fa.dev = a.dev;
        fa.gamma64 = a.gamma64; fa.gamma32 = a.gamma32;
        fa.X_out = reinterpret_cast<float2*>(X_out);
        tsl::Batch b{};
        b.one = &fa;
        b.count = 1;
        b.n1 = s->n1; b.n2 = s->n2; b.r_max = s->r; b.mode = tsl::MODE_LINES;
        b.want_x = true;
        b.synth = s->opts.synth_bf16;
        e = tsl::launch_synth_out(b, st);
        if (e != hipSuccess) return hip_fail(e, "several-coil output");
    }
    return TSL_OK;
}

int tsl_open(tsl_seq** out, int n1, int n2, int r, double lambda, const tsl_opts* opts, const tsl_c32* A0,
             const tsl_c32* B0, void* stream) {
    return open_impl(nullptr, out, n1, n2, r, lambda, opts, A0, B0, stream);
}

int tsl_open_in_pool(tsl_pool* p, tsl_seq** out, int n1, int n2, int r, double lambda, const tsl_opts* opts,
                     const tsl_c32* A0, const tsl_c32* B0, void* stream) {
    if (!p) return fail(TSL_EINVAL, "null pool");
    return open_impl(p, out, n1, n2, r, lambda, opts, A0, B0, stream);
}

int tsl_close(tsl_seq* s) {
    if (!s) return TSL_OK;
    {
        std::lock_guard<std::mutex> lk(g_graph_mu);
        for (Slot& sl : g_batch.slot)
            for (const tsl_seq* q : sl.comp.seqs)
                if (q == s) { drop_graph(sl); break; }
        for (const tsl_seq* q : g_batch.last.seqs)
            if (q == s) { g_batch.last = Composition{}; break; }
        for (tsl_batch* b : g_live_batches)
            for (const tsl_seq* q : b->seqs)
                if (q == s) b->dead = true;
    }
    hipSetDevice(s->device);
    hipError_t e = hipStreamSynchronize(s->last);
    hipFree(s->arena);
    if (s->pool) {
        std::lock_guard<std::mutex> lk(s->pool->mu);
        s->pool->used -= s->bytes;
    }
    delete s;
    if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
    return TSL_OK;
}

int tsl_push_frame(tsl_seq* s, const tsl_frame* frame, void* stream) {
    int rc = check_seq(s);
    if (rc != TSL_OK) return rc;
    if (!frame) return fail(TSL_EINVAL, "null frame");
    if ((rc = check_frame(s, *frame)) != TSL_OK) return rc;
    if ((rc = set_dev(s)) != TSL_OK) return rc;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    s->last = st;
    tsl::FrameArgs a = frame_args(s, *frame);
    tsl::Batch b{};
    b.one = &a;
    b.table = nullptr;
    b.count = 1;
    b.n1 = s->n1; b.n2 = s->n2; b.r_max = s->r; b.mode = a.mode; b.kspace = a.kspace != 0;
    b.rows_max = frame->mask ? s->n1 : std::min(std::max(frame->n_rows, 0), s->n1);
    b.want_x = frame->X_out != nullptr;
    b.want_sample = a.K_next > 0;
    b.synth = s->opts.synth_bf16;
    return run_groups({b}, st);
}

int tsl_epochs(tsl_seq* s, int T, const tsl_frame* frames, int E, const int32_t* order, void* stream) {
    int rc = check_seq(s);
    if (rc != TSL_OK) return rc;
    if (T <= 0 || E <= 0 || !frames || !order) return fail(TSL_EINVAL, "bad epoch arguments");
    for (int k = 0; k < T; ++k) {
        if ((rc = check_frame(s, frames[k])) != TSL_OK) return rc;
        if (frames[k].K_next != 0) return fail(TSL_EINVAL, "frames of a stored scan draw no rows (K_next must be 0)");
    }
    std::vector<int> seen(static_cast<size_t>(T), -1);
    for (int e = 0; e < E; ++e)
        for (int k = 0; k < T; ++k) {
            const int v = order[size_t(e) * T + k];
            if (v < 0 || v >= T || seen[size_t(v)] == e) return fail(TSL_EINVAL, "each pass must be a permutation of 0..T-1");
            seen[size_t(v)] = e;
        }
    if ((rc = set_dev(s)) != TSL_OK) return rc;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    s->last = st;
    std::vector<tsl::FrameArgs> args(static_cast<size_t>(T));
    for (int k = 0; k < T; ++k) args[size_t(k)] = frame_args(s, frames[k]);
    for (int e = 0; e < E; ++e)
        for (int k = 0; k < T; ++k) {
            const int v = order[size_t(e) * T + k];
            const tsl_frame& fr = frames[v];
            tsl::Batch b{};
            b.one = &args[size_t(v)];
            b.count = 1;
            b.n1 = s->n1; b.n2 = s->n2; b.r_max = s->r; b.mode = args[size_t(v)].mode;
            b.kspace = args[size_t(v)].kspace != 0;
            b.rows_max = fr.mask ? s->n1 : std::min(std::max(fr.n_rows, 0), s->n1);
            b.want_x = fr.X_out != nullptr;
            b.want_sample = false;
            b.synth = s->opts.synth_bf16;
            if ((rc = run_groups(&b, 1, st)) != TSL_OK) return rc;
        }
    return TSL_OK;
}

int tsl_push_lines(tsl_seq* s, int n_rows, const int32_t* rows, const tsl_c32* y, tsl_c32* X_out, tsl_c32* A_out,
                   tsl_c32* B_out, tsl_c32* gamma_out, void* stream) {
    tsl_frame f{};
    f.n_rows = n_rows; f.rows = rows; f.y = y;
    f.X_out = X_out; f.A_out = A_out; f.B_out = B_out; f.gamma_out = gamma_out;
    return tsl_push_frame(s, &f, stream);
}

int tsl_push_points(tsl_seq* s, const uint8_t* mask, const tsl_c32* y, tsl_c32* X_out, tsl_c32* A_out,
                    tsl_c32* B_out, tsl_c32* gamma_out, void* stream) {
    if (!mask) return fail(TSL_EINVAL, "null mask");
    tsl_frame f{};
    f.mask = mask; f.y = y;
    f.X_out = X_out; f.A_out = A_out; f.B_out = B_out; f.gamma_out = gamma_out;
    return tsl_push_frame(s, &f, stream);
}

int tsl_sample_lines(tsl_seq* s, int K, int32_t* rows_out, int32_t* n_out, int32_t* draws_out, double* prefix_out,
                     void* stream) {
    int rc = check_seq(s);
    if (rc != TSL_OK) return rc;
    if (K < 1) return fail(TSL_EINVAL, "K must be >= 1");
    if (!rows_out || !n_out) return fail(TSL_EINVAL, "null rows_out or n_out");
    if ((rc = set_dev(s)) != TSL_OK) return rc;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    s->last = st;
    tsl_frame fr{};
    tsl::FrameArgs a = frame_args(s, fr);
    a.K_next = K; a.rows_next = rows_out; a.n_next = n_out; a.draws_next = draws_out; a.prefix_next = prefix_out;
    tsl::Batch b{};
    b.one = &a;
    b.count = 1;
    b.n1 = s->n1; b.n2 = s->n2; b.r_max = s->r; b.mode = a.mode; b.kspace = a.kspace != 0;
    b.want_sample = true;
    hipError_t e = tsl::launch_sample(b, st);
    if (e != hipSuccess) return hip_fail(e, "sample");
    return TSL_OK;
}

int tsl_sample_points(tsl_seq* s, int K, uint8_t* mask_out, int32_t* n_out, int32_t* draws_out, void* stream) {
    int rc = check_seq(s);
    if (rc != TSL_OK) return rc;
    if (K < 1) return fail(TSL_EINVAL, "K must be >= 1");
    if (!mask_out || !n_out) return fail(TSL_EINVAL, "null mask_out or n_out");
    if ((rc = set_dev(s)) != TSL_OK) return rc;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    s->last = st;
    tsl_frame fr{};
    const tsl::FrameArgs a = frame_args(s, fr);
    hipError_t e = tsl::launch_sample_points(a, K, mask_out, n_out, draws_out, st);
    if (e != hipSuccess) return hip_fail(e, "sample points");
    return TSL_OK;
}

int tsl_step_many(tsl_seq* const* seqs, int n, const tsl_frame* frames, void* stream) {
    if (n < 0 || (n > 0 && (!seqs || !frames))) return fail(TSL_EINVAL, "bad batch arguments");
    if (n == 0) return TSL_OK;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    Composition c;
    int rc = compose(seqs, n, frames, c);
    if (rc != TSL_OK) return rc;
    std::lock_guard<std::mutex> lk(g_graph_mu);
    BatchEngine& be = g_batch;
    int k = 0;
    if ((rc = take_slot(be, size_t(c.entries()), &k)) != TSL_OK) return rc;
    Slot& sl = be.slot[k];
    if ((rc = stage_table(sl, c, seqs, frames, st)) != TSL_OK) return rc;
    const bool cached = sl.exec && sl.comp == c;
    const bool repeat = be.last == c;
    be.last = c;
    if (!cached && !repeat) {
        // A composition seen for the first time runs as plain launches; one that
        // repeats (the steady state of a fixed batch) is captured over this
        // slot's table and replayed whenever the slot comes round again.
        rc = run_composition(c, sl.table, st);
        hipError_t er = hipEventRecord(sl.done, st);
        if (rc != TSL_OK) return rc;
        if (er != hipSuccess) return hip_fail(er, "hipEventRecord");
        return TSL_OK;
    }
    if (!cached) {
        drop_graph(sl);
        hipGraph_t graph = nullptr;
        hipError_t eb = hipStreamBeginCapture(be.cap, hipStreamCaptureModeThreadLocal);
        int lrc = eb == hipSuccess ? run_composition(c, sl.table, be.cap) : TSL_OK;
        hipError_t ec = eb == hipSuccess ? hipStreamEndCapture(be.cap, &graph) : eb;
        hipError_t ei = hipSuccess;
        if (lrc == TSL_OK && ec == hipSuccess) ei = hipGraphInstantiate(&sl.exec, graph, nullptr, nullptr, 0);
        if (graph) hipGraphDestroy(graph);
        if (lrc != TSL_OK || ec != hipSuccess || ei != hipSuccess) {
            sl.exec = nullptr;
            // the staged table is in flight on `st`: keep the slot's wait honest
            hipEventRecord(sl.done, st);
            if (lrc != TSL_OK) return lrc;
            return hip_fail(ec != hipSuccess ? ec : ei, ec != hipSuccess ? "stream capture" : "hipGraphInstantiate");
        }
        sl.comp = c;
    }
    hipError_t el = hipGraphLaunch(sl.exec, st);
    hipError_t er = hipEventRecord(sl.done, st);
    if (el != hipSuccess) return hip_fail(el, "hipGraphLaunch");
    if (er != hipSuccess) return hip_fail(er, "hipEventRecord");
    return TSL_OK;
}

int tsl_step_many_timed(tsl_seq* const* seqs, int n, const tsl_frame* frames, double* phase_ms, void* stream) {
    if (n < 0 || (n > 0 && (!seqs || !frames)) || !phase_ms) return fail(TSL_EINVAL, "bad batch arguments");
    if (n == 0) return TSL_OK;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    Composition c;
    int rc = compose(seqs, n, frames, c);
    if (rc != TSL_OK) return rc;
    std::lock_guard<std::mutex> lk(g_graph_mu);
    BatchEngine& be = g_batch;
    int k = 0;
    if ((rc = take_slot(be, size_t(c.entries()), &k)) != TSL_OK) return rc;
    Slot& sl = be.slot[k];
    if ((rc = stage_table(sl, c, seqs, frames, st)) != TSL_OK) return rc;
    hipEvent_t ev[TSL_N_PHASES + 1] = {};
    for (auto& e : ev) {
        hipError_t ee = hipEventCreate(&e);
        if (ee != hipSuccess) {
            for (auto& x : ev) if (x) hipEventDestroy(x);
            hipEventRecord(sl.done, st);
            return hip_fail(ee, "hipEventCreate");
        }
    }
    rc = run_composition(c, sl.table, st, ev);
    hipError_t er = hipEventRecord(sl.done, st);
    if (rc == TSL_OK && er != hipSuccess) rc = hip_fail(er, "hipEventRecord");
    if (rc == TSL_OK) {
        hipError_t e = hipEventSynchronize(ev[TSL_N_PHASES]);
        for (int p = 0; p < TSL_N_PHASES && e == hipSuccess; ++p) {
            float ms = 0.f;
            e = hipEventElapsedTime(&ms, ev[p], ev[p + 1]);
            phase_ms[p] += ms;
        }
        if (e != hipSuccess) rc = hip_fail(e, "phase events");
    }
    for (auto& e : ev) hipEventDestroy(e);
    return rc;
}

int tsl_batch_create(tsl_seq* const* seqs, int n, const tsl_frame* frames, int flags, tsl_batch** out) {
    if (!out) return fail(TSL_EINVAL, "null batch handle pointer");
    *out = nullptr;
    if (n <= 0 || !seqs || !frames) return fail(TSL_EINVAL, "bad batch arguments");
    if (flags & ~TSL_BATCH_GRAPH) return fail(TSL_EINVAL, "unknown batch flags");
    Composition c;
    int rc = compose(seqs, n, frames, c);
    if (rc != TSL_OK) return rc;
    int dev = 0;
    TSL_HIP(hipGetDevice(&dev));
    for (int i = 0; i < n; ++i)
        if (seqs[i]->device != dev) return fail(TSL_EINVAL, "a sequence of the batch is not on the current device");
    std::unique_ptr<tsl_batch> b(new tsl_batch);
    b->device = dev;
    b->seqs.assign(seqs, seqs + n);
    const size_t m = size_t(c.entries());
    std::vector<tsl::FrameArgs> host(m);
    fill_descriptors(c, seqs, frames, host.data());
    if ((rc = tsl::eng::tune_output_runs(c.fa.data(), host.data(), n)) != TSL_OK) return rc;
    TSL_HIP(hipMalloc(&b->table, m * sizeof(tsl::FrameArgs)));
    TSL_HIP(hipMemcpy(b->table, host.data(), m * sizeof(tsl::FrameArgs), hipMemcpyHostToDevice));
    b->comp = c;
    if (flags & TSL_BATCH_GRAPH) {
        hipStream_t cap = nullptr;
        TSL_HIP(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
        hipGraph_t graph = nullptr;
        hipError_t eb = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
        int lrc = eb == hipSuccess ? run_composition(b->comp, b->table, cap) : TSL_OK;
        hipError_t ec = eb == hipSuccess ? hipStreamEndCapture(cap, &graph) : eb;
        hipStreamDestroy(cap);
        if (lrc != TSL_OK || ec != hipSuccess) {
            if (graph) hipGraphDestroy(graph);
            return lrc != TSL_OK ? lrc : hip_fail(ec, "stream capture");
        }
        hipError_t ei = hipGraphInstantiate(&b->exec, graph, nullptr, nullptr, 0);
        hipGraphDestroy(graph);
        if (ei != hipSuccess) {
            b->exec = nullptr;
            return hip_fail(ei, "hipGraphInstantiate");
        }
    }
    std::lock_guard<std::mutex> lk(g_graph_mu);
    g_live_batches.push_back(b.get());
    *out = b.release();
    return TSL_OK;
}

int tsl_batch_launch(tsl_batch* b, void* stream) {
    if (!b) return fail(TSL_EINVAL, "null batch");
    if (b->dead) return fail(TSL_EINVAL, "a sequence of the batch has been closed");
    int dev = 0;
    TSL_HIP(hipGetDevice(&dev));
    if (dev != b->device) return fail(TSL_EINVAL, "batch launched on another device than its own");
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    for (tsl_seq* s : b->seqs) s->last = st;
    b->last = st;
    b->launched = true;
    if (b->exec) {
        TSL_HIP(hipGraphLaunch(b->exec, st));
        return TSL_OK;
    }
    return run_composition(b->comp, b->table, st);
}

int tsl_batch_destroy(tsl_batch* b) {
    if (!b) return TSL_OK;
    {
        std::lock_guard<std::mutex> lk(g_graph_mu);
        g_live_batches.erase(std::remove(g_live_batches.begin(), g_live_batches.end(), b), g_live_batches.end());
    }
    hipSetDevice(b->device);
    hipError_t e = b->launched ? hipStreamSynchronize(b->last) : hipSuccess;
    delete b;
    if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
    return TSL_OK;
}

int tsl_status(tsl_seq* s, int clear) {
    int rc = check_seq(s);
    if (rc != TSL_OK) return rc;
    if ((rc = set_dev(s)) != TSL_OK) return rc;
    TSL_HIP(hipStreamSynchronize(s->last));
    tsl::SeqDev d{};
    TSL_HIP(hipMemcpy(&d, s->at<void>(s->lay.dev), sizeof(d), hipMemcpyDeviceToHost));
    if (clear && d.status != 0) {
        int zero = 0;
        TSL_HIP(hipMemcpy(s->at<char>(s->lay.dev) + offsetof(tsl::SeqDev, status), &zero, sizeof(int),
                          hipMemcpyHostToDevice));
    }
    return d.status;
}

int tsl_get_factors(tsl_seq* s, tsl_c32* A, tsl_c32* B, tsl_c32* Ahat, tsl_c32* Bhat, void* stream) {
    int rc = check_seq(s);
    if (rc != TSL_OK) return rc;
    if ((rc = set_dev(s)) != TSL_OK) return rc;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    s->last = st;
    const size_t a = size_t(s->n1) * s->r * sizeof(float2), b = size_t(s->n2) * s->r * sizeof(float2);
    if (A) TSL_HIP(hipMemcpyAsync(A, s->at<void>(s->lay.A), a, hipMemcpyDeviceToDevice, st));
    if (B) TSL_HIP(hipMemcpyAsync(B, s->at<void>(s->lay.B), b, hipMemcpyDeviceToDevice, st));
    if (Ahat) TSL_HIP(hipMemcpyAsync(Ahat, s->at<void>(s->lay.Ahat), a, hipMemcpyDeviceToDevice, st));
    if (Bhat) TSL_HIP(hipMemcpyAsync(Bhat, s->at<void>(s->lay.Bhat), b, hipMemcpyDeviceToDevice, st));
    return TSL_OK;
}

namespace {
struct BlobHeader {
    char magic[8];
    int version, n1, n2, r;
    double lambda;
    tsl_opts opts;
    double abar;
    long long t;
};
}  // namespace

int tsl_get_state(tsl_seq* s, void* host_blob, size_t* nbytes) {
    int rc = check_seq(s);
    if (rc != TSL_OK) return rc;
    if (!nbytes) return fail(TSL_EINVAL, "null nbytes");
    const size_t a = size_t(s->n1) * s->r * sizeof(float2), b = size_t(s->n2) * s->r * sizeof(float2);
    const size_t need = sizeof(BlobHeader) + 2 * a + 2 * b;
    if (!host_blob) {
        *nbytes = need;
        return TSL_OK;
    }
    if (*nbytes < need) return fail(TSL_EINVAL, "blob too small");
    if ((rc = set_dev(s)) != TSL_OK) return rc;
    TSL_HIP(hipStreamSynchronize(s->last));
    tsl::SeqDev d{};
    TSL_HIP(hipMemcpy(&d, s->at<void>(s->lay.dev), sizeof(d), hipMemcpyDeviceToHost));
    BlobHeader h{};
    std::memcpy(h.magic, "TSLSTAT", 8);
    h.version = 2; h.n1 = s->n1; h.n2 = s->n2; h.r = s->r; h.lambda = s->lambda; h.opts = s->opts;
    h.abar = d.abar; h.t = d.t;
    char* p = static_cast<char*>(host_blob);
    std::memcpy(p, &h, sizeof(h));
    p += sizeof(h);
    TSL_HIP(hipMemcpy(p, s->at<void>(s->lay.A), a, hipMemcpyDeviceToHost)); p += a;
    TSL_HIP(hipMemcpy(p, s->at<void>(s->lay.B), b, hipMemcpyDeviceToHost)); p += b;
    TSL_HIP(hipMemcpy(p, s->at<void>(s->lay.Ahat), a, hipMemcpyDeviceToHost)); p += a;
    TSL_HIP(hipMemcpy(p, s->at<void>(s->lay.Bhat), b, hipMemcpyDeviceToHost));
    *nbytes = need;
    return TSL_OK;
}

int tsl_set_state(tsl_seq* s, const void* host_blob, size_t nbytes) {
    int rc = check_seq(s);
    if (rc != TSL_OK) return rc;
    if (!host_blob || nbytes < sizeof(BlobHeader)) return fail(TSL_EINVAL, "bad blob");
    BlobHeader h{};
    std::memcpy(&h, host_blob, sizeof(h));
    const size_t a = size_t(s->n1) * s->r * sizeof(float2), b = size_t(s->n2) * s->r * sizeof(float2);
    if (std::memcmp(h.magic, "TSLSTAT", 8) != 0 || h.version != 2 || h.n1 != s->n1 || h.n2 != s->n2 ||
        h.r != s->r || nbytes < sizeof(BlobHeader) + 2 * a + 2 * b)
        return fail(TSL_EINVAL, "blob does not match this sequence");
    if ((rc = validate_params(h.lambda, h.opts)) != TSL_OK) return rc;
    if (!std::isfinite(h.abar) || h.abar < 0.0 || h.t < 0) return fail(TSL_EINVAL, "blob holds an invalid alpha_bar or t");
    if ((rc = set_dev(s)) != TSL_OK) return rc;
    TSL_HIP(hipStreamSynchronize(s->last));
    const char* p = static_cast<const char*>(host_blob) + sizeof(h);
    TSL_HIP(hipMemcpy(s->at<void>(s->lay.A), p, a, hipMemcpyHostToDevice)); p += a;
    TSL_HIP(hipMemcpy(s->at<void>(s->lay.B), p, b, hipMemcpyHostToDevice)); p += b;
    TSL_HIP(hipMemcpy(s->at<void>(s->lay.Ahat), p, a, hipMemcpyHostToDevice)); p += a;
    TSL_HIP(hipMemcpy(s->at<void>(s->lay.Bhat), p, b, hipMemcpyHostToDevice));
    tsl::SeqDev d{};
    d.abar = h.abar;
    d.t = h.t;
    TSL_HIP(hipMemcpy(s->at<void>(s->lay.dev), &d, sizeof(d), hipMemcpyHostToDevice));
    const bool changed = h.lambda != s->lambda || std::memcmp(&h.opts, &s->opts, sizeof(tsl_opts)) != 0;
    s->lambda = h.lambda;
    s->opts = h.opts;
    if (changed) {
        // a prepared batch holds descriptors (lambda, step, route, sampler key)
        // taken at its creation: one that holds this sequence is no longer valid
        std::lock_guard<std::mutex> lk(g_graph_mu);
        for (tsl_batch* bt : g_live_batches)
            for (const tsl_seq* q : bt->seqs)
                if (q == s) bt->dead = true;
    }
    return TSL_OK;
}

int tsl_set_output_tile(int n1, int n2, int r, int count, int tile) {
    if (n1 < 1 || n2 < 1 || r < 1 || count < 1 || tile < 0 || tile >= tsl::OUT_TILES)
        return fail(TSL_EINVAL, "bad output-tile setting");
    tsl::eng::set_output_tile(n1, n2, r <= 32, count, tile);
    return TSL_OK;
}

int tsl_output_tile(int n1, int n2, int r, int count) {
    if (n1 < 1 || n2 < 1 || r < 1 || count < 1) return fail(TSL_EINVAL, "bad output-tile query");
    return tsl::eng::output_tile(n1, n2, r <= 32, count);
}

int tsl_shape(const tsl_seq* s, int* n1, int* n2, int* r) {
    if (!s) return fail(TSL_EINVAL, "null sequence handle");
    if (n1) *n1 = s->n1;
    if (n2) *n2 = s->n2;
    if (r) *r = s->r;
    return TSL_OK;
}

int tsl_fft2(int n1, int n2, int batch, const tsl_c32* in, tsl_c32* out, int inverse, void* stream) {
    if (!tsl::size_supported(n1) || !tsl::size_supported(n2)) return fail(TSL_EUNSUPPORTED, "unsupported length");
    if (batch < 0 || (batch > 0 && (!in || !out))) return fail(TSL_EINVAL, "bad fft2 arguments");
    if (batch == 0) return TSL_OK;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    const float2* src = reinterpret_cast<const float2*>(in);
    float2* dst = reinterpret_cast<float2*>(out);
    hipError_t e = tsl::launch_rowfft(n1, n2, batch, src, dst, inverse != 0, st);
    if (e != hipSuccess) return hip_fail(e, "row pass");
    e = tsl::launch_colfft(n1, n2, batch, dst, dst, inverse != 0, st);
    if (e != hipSuccess) return hip_fail(e, "column pass");
    return TSL_OK;
}

int tsl_pool_create(tsl_pool** out, size_t budget_bytes) {
    if (!out) return fail(TSL_EINVAL, "null pool output");
    *out = new tsl_pool();
    (*out)->budget = budget_bytes;
    return TSL_OK;
}

int tsl_pool_destroy(tsl_pool* p) {
    if (!p) return TSL_OK;
    if (p->used != 0) return fail(TSL_EBUSY, "pool still has open sequences");
    delete p;
    return TSL_OK;
}

int tsl_pool_used(const tsl_pool* p, size_t* used, size_t* budget) {
    if (!p) return fail(TSL_EINVAL, "null pool");
    if (used) *used = p->used;
    if (budget) *budget = p->budget;
    return TSL_OK;
}

}  // extern "C"
