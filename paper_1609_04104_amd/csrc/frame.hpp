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
    double kappa_proxy; // max pivot^2 / min pivot^2 of the Cholesky factor
};

enum : int { MODE_LINES = 0, MODE_POINTS = 1 };

// Slots of the Gram statistics: [0] = (F_l A)^H F_l A, [1] = (F_r B)^H F_r B (one
// block each, all rows), then the partials of the sampled part: kSRows sampled
// rows per slot for line masks, kPRows mask rows per slot for point masks.
constexpr int kSRows = 32;      // sampled rows per (Gram, rhs) partial, line masks
constexpr int kPRows = 32;      // mask rows per (Gram, rhs) partial, point masks

__host__ __device__ inline int cdiv(int a, int b) { return (a + b - 1) / b; }
__host__ __device__ inline int n_sparts(int n1) { return cdiv(n1, kPRows); }   // >= cdiv(n1, kSRows)
__host__ __device__ inline int n_parts(int n1, int n2) { return 2 + n_sparts(n1); }

// Everything the kernels of one frame of one sequence read or write.
struct FrameArgs {
    int n1, n2, r, mode;
    double lambda, mu_const;
    int step_mode, n_rows;
    // resident state
    float2 *A, *B, *Ahat, *Bhat;
    SeqDev* dev;
    double2* gamma64;
    float2* gamma32;
    // workspace
    float2* frame;      // [n1][n2]: row-transformed synthesis, then the column-back-projected residual
    float2* Wb;         // [n2][r]: Z^T conj(A), Z the column-back-projected residual
    float2* GA;         // [n1][r]: Theta conj(B)
    double2* part;      // [n_parts][r][r] partial Grams
    double2* hpart;     // [n_sparts][r] partial right-hand sides
    // inputs of the frame
    const int* rows;
    const int* n_rows_dev;   // device row count (lines), or null to use n_rows
    int y_full;              // lines: y is [n1][n2] and row k is read at y + k*n2
    const unsigned char* mask;
    const float2* y;
    // outputs (may be null)
    float2 *X_out, *A_out, *B_out, *gamma_out;
    // draw of the next frame's rows (K_next == 0: none)
    int K_next;
    int* rows_next;
    int* n_next;
    int* draws_next;         // [K_next] rows of the individual trials, or null
    double* prefix_next;     // [n1] weight prefix, or null
    unsigned long long seed, sid;
};

// Row capacity of a line-mask frame: n_rows (the length of the row list), at
// most n1.  With a device row count, n_rows is the capacity of the list.
__device__ __forceinline__ int frame_rows_cap(const FrameArgs& f) {
    return f.n_rows < 0 ? 0 : (f.n_rows > f.n1 ? f.n1 : f.n_rows);
}
// Row count of a line-mask frame, clamped to [0, capacity] so that no kernel
// reads outside the row list; the sampled-row statistics kernel latches
// ST_EINVAL when a device count was out of range.
__device__ __forceinline__ int frame_rows(const FrameArgs& f) {
    const int cap = frame_rows_cap(f);
    if (!f.n_rows_dev) return cap;
    const int n = *f.n_rows_dev;
    return n < 0 ? 0 : (n > cap ? cap : n);
}

// Samples of row `row`, listed at position q of the row set (lines).
__device__ __forceinline__ const float2* line_samples(const FrameArgs& f, int q, int row) {
    return f.y + size_t(f.y_full ? row : q) * f.n2;
}

// Where a kernel finds its descriptor: one by value (single-sequence push) or
// entry blockIdx.y of a device table (batched step).
struct OneFrame {
    FrameArgs a;
    __device__ __forceinline__ const FrameArgs& get() const { return a; }
};
struct FrameTable {
    const FrameArgs* t;
    __device__ __forceinline__ const FrameArgs& get() const { return t[blockIdx.y]; }
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
