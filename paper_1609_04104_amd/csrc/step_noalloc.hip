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

// The descriptor array.  Each GPU the library runs on holds its own copy until
// the process ends.  Host code never names it in a kernel argument or a copy:
// its device address comes from hipGetSymbolAddress, looked up once per device
// with that device current (device_scratch).
static __device__ __align__(256) unsigned char scratch[kStaticFrames * sizeof(tsl::FrameArgs)];

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

// tsl_step_many's grouping without heap use: launch groups by (n1, n2, mask
// kind and route, rank tier) in ascending key order, call order kept inside a
// group.
struct StaticComposition {
    int n = 0, n_groups = 0;
    int order[kStaticFrames];
    int group_start[kStaticFrames];
    tsl::Batch groups[kStaticFrames];
};

int compose_static(tsl_seq* const* seqs, int n, const tsl_frame* frames, int dev, StaticComposition& c) {
    int key[kStaticFrames][4];
    int cap[kStaticFrames];
    for (int i = 0; i < n; ++i) {
        const tsl_seq* s = seqs[i];
        if (!s) return fail(TSL_EINVAL, "null sequence in batch");
        for (int j = 0; j < i; ++j)
            if (seqs[j] == s) return fail(TSL_EINVAL, "a sequence appears twice in one batch");
        if (s->device != dev) return fail(TSL_EINVAL, "a sequence of the batch is not on the current device");
        int rc = check_frame(s, frames[i]);
        if (rc != TSL_OK) return rc;
        const int kind = frames[i].mask ? 1 : (s->opts.line_route == TSL_ROUTE_FRAME ? 2 : 0);
        key[i][0] = s->n1; key[i][1] = s->n2; key[i][2] = kind; key[i][3] = rank_tier(s->r);
        cap[i] = frames[i].mask ? s->n1 : std::min(std::max(frames[i].n_rows, 0), s->n1);
    }
    auto less = [&](int a, int b) {
        for (int q = 0; q < 4; ++q)
            if (key[a][q] != key[b][q]) return key[a][q] < key[b][q];
        return false;
    };
    for (int i = 0; i < n; ++i) {          // stable insertion sort of the frame indices by key
        int p = i;
        while (p > 0 && less(i, c.order[p - 1])) {
            c.order[p] = c.order[p - 1];
            --p;
        }
        c.order[p] = i;
    }
    c.n = n;
    c.n_groups = 0;
    for (int p = 0; p < n; ++p) {
        const int i = c.order[p];
        if (p == 0 || less(c.order[p - 1], i)) {
            tsl::Batch b{};
            b.n1 = key[i][0]; b.n2 = key[i][1];
            b.mode = key[i][2] == 1 ? tsl::MODE_POINTS : tsl::MODE_LINES;
            b.kspace = key[i][2] == 0;
            c.group_start[c.n_groups] = p;
            c.groups[c.n_groups++] = b;
        }
        tsl::Batch& b = c.groups[c.n_groups - 1];
        b.count += 1;
        b.r_max = std::max(b.r_max, seqs[i]->r);
        b.rows_max = std::max(b.rows_max, cap[i]);
        b.want_x = b.want_x || frames[i].X_out != nullptr;
        b.want_sample = b.want_sample || frames[i].K_next > 0;
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
    StaticComposition c;          // about 14 KiB of stack: no heap use on this path
    int rc = compose_static(seqs, n, frames, dev, c);
    if (rc != TSL_OK) return rc;
    tsl::FrameArgs* table = nullptr;
    if ((rc = device_scratch(dev, &table)) != TSL_OK) return rc;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    for (int p0 = 0; p0 < n; p0 += kPutFrames) {
        const int m = std::min(kPutFrames, n - p0);
        PutChunk chunk;
        std::memset(&chunk, 0, sizeof(chunk));
        for (int q = 0; q < m; ++q) {
            const int i = c.order[p0 + q];
            seqs[i]->last = st;
            chunk.f[q] = frame_args(seqs[i], frames[i]);
        }
        const int words = m * int(sizeof(tsl::FrameArgs) / 4);
        k_put_descriptors<<<1, kPutWords, 0, st>>>(chunk, reinterpret_cast<unsigned*>(table + p0), words);
        TSL_HIP(hipGetLastError());
    }
    for (int g = 0; g < c.n_groups; ++g) c.groups[g].table = table + c.group_start[g];
    return run_groups(c.groups, c.n_groups, st);
}
