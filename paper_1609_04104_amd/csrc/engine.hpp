// Internals of the host engine shared by its source files: a sequence's state
// and workspace layout, error reporting, frame descriptors and the launch of a
// step's phases over launch groups.
#pragma once

#include <cstddef>
#include <mutex>
#include <string>

#include "kernels.hpp"
#include "tsl.h"

// Byte offsets of a sequence's arrays inside its one device arena.
struct Layout {
    size_t A, B, Ahat, Bhat, dev, g64, g32, frame, Wb, GA, zm, zw, bcopy, acopy, part, hpart, wq;
    // several coils (0 for a single-coil sequence)
    size_t H, P, Q, gslot, hslot, gain;
    size_t total;
};

struct tsl_pool {
    std::mutex mu;
    size_t budget = 0, used = 0;
};

struct tsl_seq {
    int n1 = 0, n2 = 0, r = 0, device = 0;
    int C = 0;                            // coils (tsl_open_coils), 0 for a single-coil sequence
    double lambda = 0;
    tsl_opts opts{};
    char* arena = nullptr;
    size_t bytes = 0;
    Layout lay{};
    hipStream_t last = nullptr;
    tsl_pool* pool = nullptr;
    template <class T> T* at(size_t off) const { return reinterpret_cast<T*>(arena + off); }
};

namespace tsl {
namespace eng {

// Records the message for tsl_last_error and returns `code`.
int fail(int code, const std::string& msg);
// Records a HIP failure and returns TSL_EDEVICE.
int hip_fail(hipError_t e, const char* what);

#define TSL_HIP(call)                                                   \
    do {                                                                \
        hipError_t e_ = (call);                                         \
        if (e_ != hipSuccess) return ::tsl::eng::hip_fail(e_, #call);   \
    } while (0)

Layout layout_for(int n1, int n2, int r, int C = 0);

// The descriptor of frame `fr` of sequence `s` (plain host pointers).
FrameArgs frame_args(const tsl_seq* s, const tsl_frame& fr);

// Synchronous checks of one frame's arguments (TSL_OK or TSL_EINVAL).
int check_frame(const tsl_seq* s, const tsl_frame& fr);

// The kernels are instantiated for rank tiers (a register-resident solve up to
// 8, 16 and 32, wider accumulators up to 64 and 128); a launch group takes the
// tier of its largest rank, so frames are grouped by tier as well as by shape
// and a rank-16 frame never runs the kernels sized for rank 64.
int rank_tier(int r);

// Launches every phase for every group, phase by phase; with `ev` non-null,
// records ev[p] before phase p and ev[TSL_N_PHASES] after the last.
int run_groups(const Batch* groups, int n_groups, hipStream_t st, hipEvent_t* ev = nullptr);

// What the launch plan of a batched step needs to know of one frame.
struct FrameFacts {
    int n1, n2, r, mode, kspace, cap, want_x, want_sample, synth;
};
FrameFacts frame_facts(const tsl_seq* s, const tsl_frame& fr);

// A batched step keeps its descriptors in two orders.  Order A sorts by (rank
// tier, mask kind, route, shape): the phases whose kernels are instantiated per
// rank tier and take any shape (statistics, solve, k-space residual, output)
// launch once per run of adjacent frames with the same instantiation.  Order B
// sorts by (shape, mask kind, route, rank tier) for the phases instantiated per
// transform length (the frame-route passes and the factor updates).  Both are
// stable (call order kept among equal keys); facts, order_a and order_b hold n
// entries.  Returns true when the two orders coincide (one table serves both).
bool table_orders(const FrameFacts* facts, int n, int* order_a, int* order_b);

// Launches every phase of a batched step whose descriptors sit in table ta
// (order A, facts fa) and tb (order B, facts fb), phase by phase, one launch
// per maximal run of adjacent frames that share the phase's kernel
// instantiation (the grid covers the largest frame of the run; the kernels
// leave the blocks a smaller frame does not need).  `ev` as in run_groups.
int launch_phases(const FrameFacts* fa, const FrameArgs* ta, const FrameFacts* fb, const FrameArgs* tb, int n,
                  hipStream_t st, hipEvent_t* ev = nullptr);

// Output-tile tuner: the block tile of the output synthesis for a launch of
// `count` frames of at most n1 x n2 (one pass of ranks or several): the
// measured fastest (tune_output_runs, or a TSL_TUNE_CACHE record), else the
// default 128 x 64.
int output_tile(int n1, int n2, bool one_pass, int count);
void set_output_tile(int n1, int n2, bool one_pass, int count, int tile);
// Times every output tile on the output launches of a batch whose descriptors
// (order A) are `host` (facts fa) and records the fastest for each launch not
// yet known; nothing the caller owns is written (the timed launches write
// their frames and drawn rows to scratch).  Off when TSL_TUNE=0.
int tune_output_runs(const FrameFacts* fa, const FrameArgs* host, int n);

}  // namespace eng
}  // namespace tsl
