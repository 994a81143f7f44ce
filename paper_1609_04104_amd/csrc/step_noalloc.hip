// The allocation-free batched step (tsl_step_many_noalloc): the same launch
// groups and kernels as tsl_step_many, with the frame descriptors kept in one
// fixed device array per GPU instead of device memory the library allocates,
// and no graph.  Made for callers that cannot allocate (code under HIP graph
// capture, tight serving loops, harnesses that forbid hipMalloc).
#include <algorithm>
#include <cstring>
#include <mutex>

#include "engine.hpp"

using namespace tsl::eng;

namespace {

constexpr int kStaticFrames = TSL_STATIC_MAX_FRAMES;

// The descriptor array (two orders of up to kStaticFrames descriptors, see
// table_orders).  Each GPU the library runs on holds its own copy until
// the process ends.  Host code never names it in a kernel argument or a copy:
// its device address comes from hipGetSymbolAddress, looked up once per device
// with that device current (device_scratch).
static __device__ __align__(256) unsigned char scratch[2 * kStaticFrames * sizeof(tsl::FrameArgs)];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
tsl::FrameArgs* g_scratch_ptr[kMaxDevices] = {};

// The current device's copy of `scratch` (looked up on the first call there).
int device_scratch(int dev, tsl::FrameArgs** out) {
    if (dev < 0 || dev >= kMaxDevices) return fail(TSL_EINVAL, "device index beyond the supported range");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        TSL_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
        if (!ptr) return fail(TSL_EDEVICE, "no device address for the descriptor array");
        g_scratch_ptr[dev] = static_cast<tsl::FrameArgs*>(ptr);
    }
    *out = g_scratch_ptr[dev];
    return TSL_OK;
}

// Descriptors travel to the array as kernel arguments (no host staging buffer
// whose reuse would need a wait), kPutFrames per launch; thread i stores the
// chunk's 32-bit word i.
constexpr int kPutFrames = 3584 / int(sizeof(tsl::FrameArgs));
static_assert(kPutFrames >= 1, "a descriptor is larger than one upload");
static_assert(sizeof(tsl::FrameArgs) % 4 == 0, "descriptors are copied in 32-bit words");
struct PutChunk {
    tsl::FrameArgs f[kPutFrames];
};
constexpr int kPutWords = int(sizeof(PutChunk) / 4);
static_assert(kPutWords <= 1024, "one thread per word of a chunk");

__global__ void __launch_bounds__(1024) k_put_descriptors(PutChunk c, unsigned* __restrict__ dst, int n_words) {
    const int i = int(threadIdx.x);
    if (i < n_words) {
        unsigned w;
        __builtin_memcpy(&w, reinterpret_cast<const unsigned char*>(&c) + 4 * i, 4);
        dst[i] = w;
    }
}

// The step's frame facts and table orders without heap use (table_orders
// sorts n <= 256 frames by insertion).
struct StaticComposition {
    int n = 0;
    bool same = true;
    int order_a[kStaticFrames], order_b[kStaticFrames];
    tsl::eng::FrameFacts facts[kStaticFrames], fa[kStaticFrames], fb[kStaticFrames];
};

int compose_static(tsl_seq* const* seqs, int n, const tsl_frame* frames, int dev, StaticComposition& c) {
    for (int i = 0; i < n; ++i) {
        const tsl_seq* s = seqs[i];
        if (!s) return fail(TSL_EINVAL, "null sequence in batch");
        for (int j = 0; j < i; ++j)
            if (seqs[j] == s) return fail(TSL_EINVAL, "a sequence appears twice in one batch");
        if (s->device != dev) return fail(TSL_EINVAL, "a sequence of the batch is not on the current device");
        int rc = check_frame(s, frames[i]);
        if (rc != TSL_OK) return rc;
        c.facts[i] = frame_facts(s, frames[i]);
    }
    c.n = n;
    c.same = table_orders(c.facts, n, c.order_a, c.order_b);
    for (int p = 0; p < n; ++p) {
        c.fa[p] = c.facts[c.order_a[p]];
        c.fb[p] = c.facts[c.order_b[p]];
    }
    return TSL_OK;
}

}  // namespace

extern "C" int tsl_step_many_noalloc(tsl_seq* const* seqs, int n, const tsl_frame* frames, void* stream) {
    if (n < 0 || (n > 0 && (!seqs || !frames))) return fail(TSL_EINVAL, "bad batch arguments");
    if (n > kStaticFrames)
        return fail(TSL_EINVAL, "tsl_step_many_noalloc takes at most TSL_STATIC_MAX_FRAMES (256) frames per call");
    if (n == 0) return TSL_OK;
    int dev = 0;
    TSL_HIP(hipGetDevice(&dev));
    StaticComposition c;          // about 30 KiB of stack: no heap use on this path
    int rc = compose_static(seqs, n, frames, dev, c);
    if (rc != TSL_OK) return rc;
    tsl::FrameArgs* table = nullptr;
    if ((rc = device_scratch(dev, &table)) != TSL_OK) return rc;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    for (int i = 0; i < n; ++i) seqs[i]->last = st;
    // order A at [0, n), order B (if it differs) at [n, 2n)
    const int m = c.same ? n : 2 * n;
    for (int p0 = 0; p0 < m; p0 += kPutFrames) {
        const int cnt = std::min(kPutFrames, m - p0);
        PutChunk chunk;
        std::memset(&chunk, 0, sizeof(chunk));
        for (int q = 0; q < cnt; ++q) {
            const int p = p0 + q;
            const int i = p < n ? c.order_a[p] : c.order_b[p - n];
            chunk.f[q] = frame_args(seqs[i], frames[i]);
        }
        const int words = cnt * int(sizeof(tsl::FrameArgs) / 4);
        k_put_descriptors<<<1, kPutWords, 0, st>>>(chunk, reinterpret_cast<unsigned*>(table + p0), words);
        TSL_HIP(hipGetLastError());
    }
    return launch_phases(c.fa, table, c.fb, c.same ? table : table + n, n, st);
}
