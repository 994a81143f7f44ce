// Per-sequence device state, per-frame launch descriptors and the status word.
#pragma once

#include "common.hpp"

namespace tsl {

// Device status codes (same values as the TSL_* codes of the C ABI).
enum : int { ST_OK = 0, ST_EINVAL = -1, ST_ENOTPD = -4, ST_ENONFINITE = -5 };

// Scalars resident on the device for one sequence.
struct SeqDev {
    double abar;        // alpha_bar of the last committed frame
    long long t;        // frames committed
    int status;         // sticky: 0 or a negative ST_* code
    int frame_ok;       // the current frame's solve succeeded
    // written by the solve kernel, read by the later kernels of the same frame
    double mu, shrink, alpha, abar_new;
    long long t_new;
    double kappa_proxy; // max / min pivot D_k of G = L D L^H (squared diagonal ratio of the Cholesky factor)
};

enum : int { MODE_LINES = 0, MODE_POINTS = 1 };

// Slots of the Gram statistics, each the entries on and above the diagonal of
// an r x r Hermitian matrix packed by rows (slot_size(r) entries, entry (i, j),
// i <= j, at upk(i, j, r)): first the partials
// of (F_l A)^H F_l A over kGRows rows of F_l A each, then those of
// (F_r B)^H F_r B, then the partials of the sampled part (kSRows sampled rows
// per slot for line masks, kPRows mask rows per slot for point masks).  The
// right-hand side partials are [sampled slot][readout chunk of kJCH samples]
// for line masks and [sampled slot] for point masks.
constexpr int kGRows = 64;      // rows of F_l A or F_r B per factor-Gram partial
constexpr int kSRows = 32;      // sampled rows per (Gram, rhs) partial, line masks
constexpr int kPRows = 32;      // mask rows per (Gram, rhs) partial, point masks
constexpr int kJCH = 32;        // readout samples per right-hand-side partial, line masks
constexpr int kKQ = 16;         // sampled rows per block of the k-space residual (partials of E^T conj(Ahat_S))
constexpr int kKCols = 128;     // readout samples per block of the k-space residual (partials of E conj(Bhat))

__host__ __device__ constexpr inline int cdiv(int a, int b) { return (a + b - 1) / b; }
__host__ __device__ constexpr inline int slot_size(int r) { return r * (r + 1) / 2; }
__host__ __device__ constexpr inline int upk(int i, int j, int r) { return i * r - i * (i - 1) / 2 + (j - i); }
__host__ __device__ inline int n_gparts(int n) { return cdiv(n, kGRows); }
__host__ __device__ inline int n_sparts(int n1) { return cdiv(n1, kPRows); }   // >= cdiv(n1, kSRows)
__host__ __device__ inline int n_jparts(int n2) { return cdiv(n2, kJCH); }
__host__ __device__ inline int n_parts(int n1, int n2) { return n_gparts(n1) + n_gparts(n2) + n_sparts(n1); }
__host__ __device__ inline int n_hparts(int n1, int n2) { return n_sparts(n1) * n_jparts(n2); }
__host__ __device__ inline int n_qparts(int n1) { return cdiv(n1, kKQ); }
__host__ __device__ inline int n_cparts(int n2) { return cdiv(n2, kKCols); }

// Pointer types of a frame descriptor.  The host fills descriptors with plain
// pointers; device code reads the same bits as pointers into the global address
// space (every one addresses device global memory), which lets the compiler use
// global rather than flat memory instructions (flat loads also count against the
// LDS wait counter, which serialises LDS traffic behind them).
template <class T> using HostPtr = T*;
#ifdef __HIP_DEVICE_COMPILE__
template <class T> using GlobalPtr = __attribute__((address_space(1))) T*;
#else
template <class T> using GlobalPtr = T*;
#endif

// Everything the kernels of one frame of one sequence read or write.
template <template <class> class P>
struct FrameArgsT {
    int n1, n2, r, mode;
    int kspace;           // line mask on the k-space route (the update forms the gradients from zm, zw, the copies and the Grams)
    double lambda, mu_const;
    int step_mode, n_rows;
    int synth_bf16;       // SYN_FP32, SYN_BF16 or SYN_BF16X3 (mfma.hpp): operands of the syntheses
    // resident state
    P<float2> A, B, Ahat, Bhat;
    P<SeqDev> dev;
    P<double2> gamma64;
    P<float2> gamma32;
    // workspace
    P<float2> frame;      // [n1][n2]: row-transformed synthesis, then the column-back-projected residual
    P<float2> Wb;         // [n2][r]: Z^T conj(A), Z the column-back-projected residual (= E^T conj(Ahat_S))
    P<float2> GA;         // [n1][r]: Theta conj(B) (frame route)
    // k-space route, written by the statistics launch for the update (which overwrites Ahat, Bhat):
    P<float2> zm;         // [n_sparts(n1)][n_jparts(n2)][kSRows][r]: Y_S conj(Bhat) per chunk of sampled
                          // rows and of readout samples (rows of a chunk in list order)
    P<float2> zw;         // [n_sparts(n1)][n2][r]: Y_S^T conj(Ahat_S) per chunk of sampled rows
    P<float2> bcopy;      // [n2][r]: Bhat of frame t - 1
    P<float2> acopy;      // [n1][r]: the sampled rows of Ahat of frame t - 1, in list order
    P<double2> part;      // [n_parts][r][r] partial Grams
    P<double2> hpart;     // [n_hparts][r] partial right-hand sides
    // inputs of the frame
    P<const int> rows;
    P<const int> n_rows_dev;   // device row count (lines), or null to use n_rows
    int y_full;                // lines: y is [n1][n2] and row k is read at y + k*n2
    P<const unsigned char> mask;
    P<const float2> y;
    // outputs (may be null)
    P<float2> X_out, A_out, B_out, gamma_out;
    // draw of the next frame's rows (K_next == 0: none)
    int K_next;
    P<int> rows_next;
    P<int> n_next;
    P<int> draws_next;         // [K_next] rows of the individual trials, or null
    P<double> prefix_next;     // [n1] weight prefix, or null
    unsigned long long seed, sid;
    P<double> info_out;        // [4]: alpha_t, alpha_bar_t, mu_t, max/min pivot of G_t, or null
    P<double> wq;              // [cdiv(r, 16)][n1]: the draw's row-weight block sums of the current F_l A,
                               // written by the A update (valid when this frame's update committed)
};
using FrameArgs = FrameArgsT<HostPtr>;
using DevFrame = FrameArgsT<GlobalPtr>;
static_assert(sizeof(FrameArgs) == sizeof(DevFrame), "host and device descriptors share one layout");

__device__ __forceinline__ DevFrame dev_frame(const FrameArgs& a) {
    DevFrame d;
    __builtin_memcpy(&d, &a, sizeof(d));
    return d;
}

// Row capacity of a line-mask frame: n_rows (the length of the row list), at
// most n1.  With a device row count, n_rows is the capacity of the list.
__device__ __forceinline__ int frame_rows_cap(const DevFrame& f) {
    return f.n_rows < 0 ? 0 : (f.n_rows > f.n1 ? f.n1 : f.n_rows);
}
// Row count of a line-mask frame, clamped to [0, capacity] so that no kernel
// reads outside the row list; the sampled-row statistics kernel latches
// ST_EINVAL when a device count was out of range.
__device__ __forceinline__ int frame_rows(const DevFrame& f) {
    const int cap = frame_rows_cap(f);
    if (!f.n_rows_dev) return cap;
    const int n = *f.n_rows_dev;
    return n < 0 ? 0 : (n > cap ? cap : n);
}

// A masked load that puts the mask into the address: a lane whose operand is
// masked off reads a zero constant instead.  No select on the loaded value
// follows (such a select has to wait for the load where it is written, and the
// compiler may turn it into a branch around the load), so the wait moves to the
// value's first real use and a batch of these loads goes out back to back.
__device__ __align__(16) const float g_zero_f4[4] = {0.f, 0.f, 0.f, 0.f};
template <class T> __device__ __forceinline__ T load_or_zero(bool ok, GlobalPtr<const T> p) {
    static_assert(sizeof(T) <= 16, "the zero constant holds 16 bytes");
    const GlobalPtr<const T> z = (GlobalPtr<const T>)(const void*)g_zero_f4;
    GlobalPtr<const T> a = ok ? p : z;
    // an empty statement that claims to change the address (it holds no
    // instruction): the compiler cannot split the load back into two loads
    // under branches
    asm("" : "+v"(a));
    return *a;
}

// A store past the cache, for values that only a later launch reads: the end of
// this launch then has fewer dirty lines to write back before the next starts.
__device__ __forceinline__ void store_nt(GlobalPtr<float2> p, float2 v) {
    typedef float nt2 __attribute__((ext_vector_type(2)));
    __builtin_nontemporal_store(nt2{v.x, v.y}, reinterpret_cast<GlobalPtr<nt2>>(p));
}

// Samples of row `row`, listed at position q of the row set (lines).
__device__ __forceinline__ GlobalPtr<const float2> line_samples(const DevFrame& f, int q, int row) {
    return f.y + size_t(f.y_full ? row : q) * f.n2;
}

// Where a kernel finds its descriptor: one by value (single-sequence push) or
// an entry of a device table (batched step).
// bx() is the block's index inside its frame; live() is false for the padding
// blocks of a table launch (they return at once).
struct OneFrame {
    FrameArgs a;
    __device__ __forceinline__ DevFrame get() const { return dev_frame(a); }
    __device__ __forceinline__ int bx() const { return int(blockIdx.x); }
    __device__ __forceinline__ bool live() const { return true; }
};

// The hardware deals consecutive workgroup ids round-robin to the kXcds XCDs,
// each with its own L2.  A table launch therefore numbers its blocks so that
// all X blocks of one frame share an XCD: a group of kXcds frames takes
// kXcds * X consecutive ids and frame kXcds * G + j gets the ids with residue j.
// A frame's factors are then fetched into one L2 once instead of into all of them.
constexpr int kXcds = 8;
struct FrameTable {
    const FrameArgs* __restrict__ t;
    int X, count;
    __device__ __forceinline__ int y() const {
        const int L = int(blockIdx.x), span = kXcds * X;
        return kXcds * (L / span) + (L % span) % kXcds;
    }
    __device__ __forceinline__ int bx() const { return (int(blockIdx.x) % (kXcds * X)) / kXcds; }
    __device__ __forceinline__ bool live() const { return y() < count; }
    __device__ __forceinline__ DevFrame get() const { return dev_frame(t[y()]); }
};

// Latch an error code if none is latched yet (first error wins).
__device__ __forceinline__ void latch(SeqDev* d, int code) {
    atomicCAS(&d->status, 0, code);
}

// A block-uniform read of the frame's go/no-go flags: thread 0 reads, the
// block agrees through LDS, so every thread takes the same branch.
__device__ __forceinline__ bool block_frame_ok(const SeqDev* d, bool need_solve) {
    __shared__ int s_go;
    if (threadIdx.x == 0) {
        int st = __hip_atomic_load(&d->status, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        int ok = need_solve ? d->frame_ok : 1;
        s_go = (st == 0 && ok) ? 1 : 0;
    }
    __syncthreads();
    int go = s_go;
    __syncthreads();
    return go != 0;
}

__device__ __forceinline__ bool finite2(float2 v) {
    return isfinite(v.x) && isfinite(v.y);
}

// Block-cooperative copy of n elements, element e = load(e) stored by store(e, v):
// each thread issues U independent loads before it stores any of them, so U
// memory latencies overlap instead of following one another.
template <int U, class T, class Load, class Store>
__device__ __forceinline__ void stage_copy(int n, Load load, Store store) {
    for (int e0 = threadIdx.x; e0 < n; e0 += int(blockDim.x) * U) {
        T v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int e = e0 + u * int(blockDim.x);
            if (e < n) v[u] = load(e);
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int e = e0 + u * int(blockDim.x);
            if (e < n) store(e, v[u]);
        }
    }
}

}  // namespace tsl
