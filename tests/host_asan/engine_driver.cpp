// Drives the library's host code (engine.hip, built for the host only) through
// the sequences of calls that the serving loop, the prepared batches and the
// checkpoints make, on top of the emulated runtime of hip_emul.cpp, under the
// address and undefined-behaviour sanitizers.  Exit status 0 = no finding.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <random>
#include <vector>

#include <hip/hip_runtime_api.h>

#include "tsl.h"

extern "C" void emul_set_slow_stream(void* st);
extern "C" int emul_errors();
extern "C" long long emul_groups_run();
extern "C" void emul_flush();

namespace {

int g_fail = 0;

#define EXPECT(cond)                                                          \
    do {                                                                      \
        if (!(cond)) {                                                        \
            std::fprintf(stderr, "FAILED line %d: %s (%s)\n", __LINE__, #cond, \
                         tsl_last_error());                                   \
            ++g_fail;                                                         \
        }                                                                     \
    } while (0)

void* dalloc(size_t n) {
    void* p = nullptr;
    if (hipMalloc(&p, n) != hipSuccess) std::abort();
    std::memset(p, 0, n);
    return p;
}

// A sequence with the caller-owned buffers of one frame of it.
struct Seq {
    tsl_seq* s = nullptr;
    int n1 = 0, n2 = 0, r = 0;
    int32_t* rows = nullptr;     // [n1]
    int32_t* cnt = nullptr;      // [1]
    int32_t* rows_next = nullptr;
    int32_t* n_next = nullptr;
    tsl_c32* y = nullptr;        // [n1][n2]
    uint8_t* mask = nullptr;     // [n1][n2]
    tsl_c32* X = nullptr;
    tsl_c32 *A = nullptr, *B = nullptr, *g = nullptr;
    std::vector<void*> bufs;

    int open(tsl_pool* pool, int n1_, int n2_, int r_, int route, void* st) {
        n1 = n1_; n2 = n2_; r = r_;
        auto take = [&](size_t n) { void* p = dalloc(n); bufs.push_back(p); return p; };
        rows = static_cast<int32_t*>(take(sizeof(int32_t) * n1));
        for (int i = 0; i < n1; ++i) rows[i] = i;
        cnt = static_cast<int32_t*>(take(sizeof(int32_t)));
        rows_next = static_cast<int32_t*>(take(sizeof(int32_t) * n1));
        n_next = static_cast<int32_t*>(take(sizeof(int32_t)));
        y = static_cast<tsl_c32*>(take(sizeof(tsl_c32) * n1 * n2));
        mask = static_cast<uint8_t*>(take(size_t(n1) * n2));
        X = static_cast<tsl_c32*>(take(sizeof(tsl_c32) * n1 * n2));
        A = static_cast<tsl_c32*>(take(sizeof(tsl_c32) * n1 * r));
        B = static_cast<tsl_c32*>(take(sizeof(tsl_c32) * n2 * r));
        g = static_cast<tsl_c32*>(take(sizeof(tsl_c32) * r));
        tsl_opts o;
        tsl_opts_default(&o);
        o.line_route = route;
        o.stream_id = uint64_t(n1) * 1000 + r;
        const int rc = pool ? tsl_open_in_pool(pool, &s, n1, n2, r, 0.05, &o, A, B, st)
                            : tsl_open(&s, n1, n2, r, 0.05, &o, A, B, st);
        if (rc != TSL_OK) free_bufs();
        return rc;
    }
    tsl_frame frame(int kind, int nrows) const {
        tsl_frame f{};
        if (kind == 1) {
            f.mask = mask; f.y = y;
        } else {
            f.n_rows = nrows; f.rows = rows; f.y = y; f.y_full = 1;
            if (kind == 2) { f.n_rows_dev = cnt; f.K_next = n1 / 8 > 0 ? n1 / 8 : 1; f.rows_next = rows_next; f.n_next = n_next; }
        }
        f.X_out = X; f.A_out = A; f.B_out = B; f.gamma_out = g;
        return f;
    }
    void free_bufs() {
        for (void* p : bufs) hipFree(p);
        bufs.clear();
    }
    void close() {
        if (s) EXPECT(tsl_close(s) == TSL_OK);
        s = nullptr;
        free_bufs();
    }
};

struct Shape { int n1, n2, r, route; };
const Shape kShapes[] = {{128, 128, 16, 0}, {128, 128, 64, 0}, {192, 160, 32, 0}, {256, 256, 32, 0},
                         {64, 64, 8, 1},    {256, 256, 64, 1},  {120, 200, 5, 0},  {384, 384, 48, 0}};

// Two streams, one of them slow: a call on the fast stream must never rewrite
// the descriptors that a call on the slow stream has yet to read.
void two_streams() {
    hipStream_t slow = nullptr, fast = nullptr;
    hipStreamCreateWithFlags(&slow, 0);
    hipStreamCreateWithFlags(&fast, 0);
    emul_set_slow_stream(slow);
    std::vector<Seq> a(3), b(2);
    for (Seq& q : a) EXPECT(q.open(nullptr, 128, 128, 16, 0, slow) == TSL_OK);
    for (Seq& q : b) EXPECT(q.open(nullptr, 256, 256, 64, 0, fast) == TSL_OK);
    emul_flush();                           // the opens are done; the slow stream starts idle
    const int before = emul_errors();
    for (int it = 0; it < 12; ++it) {
        std::vector<tsl_seq*> sa, sb;
        std::vector<tsl_frame> fa, fb;
        for (Seq& q : a) { sa.push_back(q.s); fa.push_back(q.frame(0, 16)); }
        for (Seq& q : b) { sb.push_back(q.s); fb.push_back(q.frame(it % 2 ? 2 : 0, 32)); }
        EXPECT(tsl_step_many(sa.data(), int(sa.size()), fa.data(), slow) == TSL_OK);
        EXPECT(tsl_step_many(sb.data(), int(sb.size()), fb.data(), fast) == TSL_OK);
    }
    emul_flush();
    if (emul_errors() != before) std::fprintf(stderr, "two streams: %d findings\n", emul_errors() - before);
    for (Seq& q : a) q.close();
    for (Seq& q : b) q.close();
    emul_set_slow_stream(nullptr);
    hipStreamDestroy(slow);
    hipStreamDestroy(fast);
}

// The serving loop's pattern: admission against a pool budget, batches whose
// composition changes from call to call and sometimes repeats (graph capture
// and replay), scans closed and new ones opened between steps.
void serving(unsigned seed) {
    std::mt19937 rng(seed);
    hipStream_t st = nullptr;
    hipStreamCreateWithFlags(&st, 0);
    emul_set_slow_stream(st);
    size_t one = 0;
    EXPECT(tsl_footprint(256, 256, 32, &one) == TSL_OK);
    tsl_pool* pool = nullptr;
    EXPECT(tsl_pool_create(&pool, one * 9) == TSL_OK);
    std::vector<Seq> live;
    int busy = 0;
    for (int step = 0; step < 160; ++step) {
        // admissions
        for (int k = 0; k < 3; ++k) {
            const Shape& sh = kShapes[rng() % 8];
            Seq q;
            const int rc = q.open(pool, sh.n1, sh.n2, sh.r, sh.route, st);
            if (rc == TSL_EBUSY) { ++busy; break; }
            EXPECT(rc == TSL_OK);
            if (rc == TSL_OK) live.push_back(q);
        }
        if (live.empty()) continue;
        // the batch: all live scans, or (every other step) the same prefix again
        const int n = (step % 5 == 1 || step % 5 == 2) ? int(live.size()) : 1 + int(rng() % live.size());
        std::vector<tsl_seq*> seqs;
        std::vector<tsl_frame> frames;
        for (int i = 0; i < n; ++i) {
            seqs.push_back(live[i].s);
            const int kind = live[i].n1 == 64 ? 1 : int(rng() % 3 == 0 ? 2 : 0);
            frames.push_back(live[i].frame(kind == 1 ? 1 : kind, int(rng() % (live[i].n1 + 1))));
        }
        if (step % 17 == 3) {
            double ms[TSL_N_PHASES] = {};
            EXPECT(tsl_step_many_timed(seqs.data(), n, frames.data(), ms, st) == TSL_OK);
        } else {
            EXPECT(tsl_step_many(seqs.data(), n, frames.data(), st) == TSL_OK);
        }
        // retire some scans
        if (step % 4 == 3 && !live.empty()) {
            const size_t k = rng() % live.size();
            EXPECT(tsl_status(live[k].s, 0) == TSL_OK);
            live[k].close();
            live.erase(live.begin() + long(k));
        }
    }
    EXPECT(busy > 0);                       // the budget was really exercised
    for (Seq& q : live) q.close();
    size_t used = 1, budget = 0;
    EXPECT(tsl_pool_used(pool, &used, &budget) == TSL_OK);
    EXPECT(used == 0);
    EXPECT(tsl_pool_destroy(pool) == TSL_OK);
    emul_set_slow_stream(nullptr);
    hipStreamDestroy(st);
}

// Prepared batches, checkpoints and argument errors.
void prepared_and_state() {
    hipStream_t st = nullptr;
    hipStreamCreateWithFlags(&st, 0);
    std::vector<Seq> qs(4);
    for (int i = 0; i < 4; ++i) EXPECT(qs[i].open(nullptr, kShapes[i].n1, kShapes[i].n2, kShapes[i].r, 0, st) == TSL_OK);
    std::vector<tsl_seq*> seqs;
    std::vector<tsl_frame> frames;
    for (Seq& q : qs) { seqs.push_back(q.s); frames.push_back(q.frame(2, q.n1 / 4)); }
    for (int flags = 0; flags <= TSL_BATCH_GRAPH; ++flags) {
        tsl_batch* bt = nullptr;
        EXPECT(tsl_batch_create(seqs.data(), 4, frames.data(), flags, &bt) == TSL_OK);
        for (int k = 0; k < 5; ++k) EXPECT(tsl_batch_launch(bt, st) == TSL_OK);
        // a checkpoint with other options invalidates the batch
        size_t nb = 0;
        EXPECT(tsl_get_state(qs[1].s, nullptr, &nb) == TSL_OK);
        std::vector<unsigned char> blob(nb);
        EXPECT(tsl_get_state(qs[1].s, blob.data(), &nb) == TSL_OK);
        EXPECT(tsl_set_state(qs[1].s, blob.data(), nb) == TSL_OK);      // same options: still valid
        EXPECT(tsl_batch_launch(bt, st) == TSL_OK);
        std::vector<unsigned char> bad = blob;
        double nan = std::nan("");
        std::memcpy(bad.data() + 8 + 4 * sizeof(int), &nan, sizeof(double));   // lambda of the header
        EXPECT(tsl_set_state(qs[1].s, bad.data(), nb) == TSL_EINVAL);
        bad = blob;
        bad[0] = 'X';
        EXPECT(tsl_set_state(qs[1].s, bad.data(), nb) == TSL_EINVAL);
        EXPECT(tsl_set_state(qs[1].s, blob.data(), nb - 1) == TSL_EINVAL);
        bad = blob;
        const double lam2 = 0.5;
        std::memcpy(bad.data() + 8 + 4 * sizeof(int), &lam2, sizeof(double));
        EXPECT(tsl_set_state(qs[1].s, bad.data(), nb) == TSL_OK);
        EXPECT(tsl_batch_launch(bt, st) == TSL_EINVAL);
        EXPECT(tsl_batch_destroy(bt) == TSL_OK);
        EXPECT(tsl_set_state(qs[1].s, blob.data(), nb) == TSL_OK);
    }
    // closing a sequence invalidates a batch that holds it
    tsl_batch* bt = nullptr;
    EXPECT(tsl_batch_create(seqs.data(), 4, frames.data(), 0, &bt) == TSL_OK);
    // argument errors return before anything is enqueued
    tsl_seq* dup[2] = {qs[0].s, qs[0].s};
    tsl_frame f2[2] = {frames[0], frames[0]};
    EXPECT(tsl_step_many(dup, 2, f2, st) == TSL_EINVAL);
    tsl_frame badf = qs[0].frame(0, qs[0].n1 + 1);
    EXPECT(tsl_step_many(&seqs[0], 1, &badf, st) == TSL_EINVAL);
    EXPECT(tsl_push_frame(qs[0].s, &badf, st) == TSL_EINVAL);
    tsl_frame ok = qs[0].frame(0, 3);
    EXPECT(tsl_push_frame(qs[0].s, &ok, st) == TSL_OK);
    tsl_frame pts = qs[0].frame(1, 0);
    EXPECT(tsl_push_frame(qs[0].s, &pts, st) == TSL_OK);
    EXPECT(tsl_sample_lines(qs[0].s, 9, qs[0].rows_next, qs[0].n_next, nullptr, nullptr, st) == TSL_OK);
    EXPECT(tsl_fft2(qs[0].n1, qs[0].n2, 1, qs[0].y, qs[0].X, 0, st) == TSL_OK);
    EXPECT(tsl_get_factors(qs[0].s, qs[0].A, qs[0].B, nullptr, nullptr, st) == TSL_OK);
    qs[2].close();
    EXPECT(tsl_batch_launch(bt, st) == TSL_EINVAL);
    EXPECT(tsl_batch_destroy(bt) == TSL_OK);
    for (Seq& q : qs) q.close();
    hipStreamDestroy(st);
}

}  // namespace

int main() {
    two_streams();
    for (unsigned seed = 1; seed <= 4; ++seed) serving(seed);
    prepared_and_state();
    emul_flush();
    const int e = emul_errors();
    std::printf("engine host checks: %lld descriptor reads, %d emulation findings, %d failed expectations\n",
                emul_groups_run(), e, g_fail);
    return (e == 0 && g_fail == 0) ? 0 : 1;
}
