// Informative line sampling (Algorithm 4 on rows, with the row score of
// Sec. VI-C) for one frame, run by one block of at least kSampleThreads threads.
// Used by the standalone draw kernel and by the extra block per frame of the
// B-update launch, which runs beside the B update (the draw reads F_l A of
// the new A only).
//
// Row weight w_i = N2 ||abar_i||^2 + R where abar_i is row i of F_l A with
// every column of nonzero norm normalised (a zero column is left out); K
// trials with replacement, trial k taking u_k = (first Philox4x64-10 word at
// counter (t+1, k, 0, 0), key (seed, stream id)) >> 11, times 2^-53, and
// drawing the first row whose inclusive weight prefix exceeds u_k W (W the
// computed total, the last row if none).  Every sum runs in index order in
// FP64 without fused multiply-adds, so the rows drawn match any IEEE
// implementation of the same order bit for bit.
#pragma once

#include "frame.hpp"
#include "tsl.h"

namespace tsl {

constexpr int kSampleThreads = 256;   // threads that work on a draw (a bigger block idles the rest)
constexpr int kUPre = 256;            // uniforms computed beside the prefix sum
constexpr int kChunk = 2048;          // factor entries per staged chunk of rows (16 KiB)
constexpr int kChunkLoads = kChunk / kSampleThreads;   // loads per thread that cover one chunk
constexpr int kBatch = 8;             // LDS loads a sequential sum keeps one batch ahead
constexpr int kResident = 2;          // chunks of F_l A held in registers at a time
constexpr int kPB = 16;               // prefix values one thread holds per batch
struct alignas(16) SampleLds {
    double pref[kMaxN + kPB];         // weights, then their inclusive prefix (padded: the prefix
                                      // reads and writes up to kPB values past n1, never used)
    double c[TSL_MAX_R];              // column energies
    double u[kUPre];                  // u_k for k < kUPre
    double buf[kChunk];               // a chunk of energies E_ir
    int mark[kMaxN];
    int wcount[kMaxN / 64];
};

// Philox4x64-10 (Salmon et al., SC'11): ten rounds of two 64 x 64 -> 128-bit
// products with the published multipliers and Weyl key increments.
__device__ __forceinline__ void philox4x64_10(uint64_t (&x)[4], uint64_t k0, uint64_t k1) {
    constexpr uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
    constexpr uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
#pragma unroll
    for (int round = 0; round < 10; ++round) {
        const uint64_t lo0 = M0 * x[0], hi0 = __umul64hi(M0, x[0]);
        const uint64_t lo1 = M1 * x[2], hi1 = __umul64hi(M1, x[2]);
        const uint64_t y0 = hi1 ^ x[1] ^ k0, y2 = hi0 ^ x[3] ^ k1;
        x[0] = y0;
        x[1] = lo1;
        x[2] = y2;
        x[3] = lo0;
        k0 += W0;
        k1 += W1;
    }
}

__device__ __forceinline__ double uniform_trial(uint64_t t, int k, uint64_t seed, uint64_t sid) {
    uint64_t x[4] = {t, uint64_t(k), 0ull, 0ull};
    philox4x64_10(x, seed, sid);
    return double(x[0] >> 11) * 0x1.0p-53;
}

// Squared magnitude in FP64 (both products exact, one rounding in the sum).
__device__ __forceinline__ double energy(float2 a) {
#pragma clang fp contract(off)
    const double ax = a.x, ay = a.y;
    return ax * ax + ay * ay;
}

// acc += buf[i R + r] for i = 0, 1, ..., nb - 1 in order (one or two columns
// per lane), with the LDS loads of the next batch of rows in flight while the
// current one is added; two register sets alternate, so no copies are needed.
template <bool TWO>
__device__ __forceinline__ void column_chain(const double* buf, int R, int r0, int r1, int nb, double& acc0,
                                             double& acc1) {
#pragma clang fp contract(off)
    constexpr int B = TWO ? kBatch / 2 : kBatch;      // rows per register set (nb is a multiple of kBatch)
    double a0[B], a1[B], b0[B], b1[B];
    auto load = [&](double (&x0)[B], double (&x1)[B], int i0) {
#pragma unroll
        for (int w = 0; w < B; ++w) {
            x0[w] = buf[(i0 + w) * R + r0];
            if constexpr (TWO) x1[w] = buf[(i0 + w) * R + r1];
        }
    };
    auto add = [&](const double (&x0)[B], const double (&x1)[B]) {
#pragma unroll
        for (int w = 0; w < B; ++w) {
            acc0 = acc0 + x0[w];
            if constexpr (TWO) acc1 = acc1 + x1[w];
        }
    };
    load(a0, a1, 0);
    for (int il = 0; il < nb; il += 2 * B) {
        const bool more = il + B < nb;
        if (more) load(b0, b1, il + B);
        add(a0, a1);
        if (more) {
            if (il + 2 * B < nb) load(a0, a1, il + 2 * B);
            add(b0, b1);
        }
    }
}

__device__ __forceinline__ void draw_rows(const DevFrame& f, SampleLds& L) {
#pragma clang fp contract(off)
    const int K = f.K_next;
    if (K <= 0) return;
    const int n1 = f.n1, n2 = f.n2, R = f.r, tid = threadIdx.x, nt = blockDim.x;
    const bool worker = tid < kSampleThreads;        // whole wavefronts
    GlobalPtr<const float2> Ah = f.Ahat;
    const uint64_t t_next = uint64_t(f.dev->t + 1);

    // For the column energies, rows of F_l A come in chunks of ck rows (a
    // multiple of kBatch, ck R <= kChunk), kResident chunks at a time held in
    // registers across the block: coalesced loads at indices clamped into the
    // factor, zero past the end.
    const int ck = min((kChunk / R) / kBatch * kBatch, cdiv(n1, kBatch) * kBatch);
    const int span = kResident * ck;                 // rows held at a time
    float2 a[kResident][kChunkLoads];
    auto load_span = [&](int I0) {
        sfor<kResident>([&](auto sc) {
            constexpr int sub = decltype(sc)::value;
            const int i0 = I0 + sub * ck;
            const int ne = max(min(ck, n1 - i0), 0) * R;
#pragma unroll
            for (int u = 0; u < kChunkLoads; ++u) {
                const int e = tid + u * kSampleThreads;
                const float2 v = Ah[min(size_t(i0) * R + e, size_t(n1) * R - 1)];
                a[sub][u] = e < ne ? v : float2{0.f, 0.f};
            }
        });
    };

    // 1. Column energies c_r = sum_i E_ir in row order: the block writes a
    //    chunk's energies E_ir = |Ahat_ir|^2 (FP64) to LDS, then wavefront 0
    //    adds them up, lane l owning columns l and l + 64.  Rows past n1 are
    //    zero, and adding +0 leaves a nonnegative sum unchanged.
    {
        const int r0 = min(tid, R - 1), r1 = min(tid + 64, R - 1);
        const bool two = R > 64;
        double acc0 = 0.0, acc1 = 0.0;
        for (int I0 = 0; I0 < n1; I0 += span) {
            if (worker) load_span(I0);
            sfor<kResident>([&](auto sc) {
                constexpr int sub = decltype(sc)::value;
                const int i0 = I0 + sub * ck;
                if (i0 < n1) {
                    if (worker) {
#pragma unroll
                        for (int u = 0; u < kChunkLoads; ++u) L.buf[tid + u * kSampleThreads] = energy(a[sub][u]);
                    }
                    __syncthreads();
                    if (tid < 64) {
                        const int nb = cdiv(min(ck, n1 - i0), kBatch) * kBatch;   // rows past n1 are zero
                        if (two) column_chain<true>(L.buf, R, r0, r1, nb, acc0, acc1);
                        else column_chain<false>(L.buf, R, r0, r1, nb, acc0, acc1);
                    }
                    __syncthreads();
                }
            });
        }
        if (tid < 64 && tid < R) L.c[tid] = acc0;
        if (tid < 64 && tid + 64 < R) L.c[tid + 64] = acc1;
    }
    for (int i = tid; i < n1; i += nt) L.mark[i] = 0;
    __syncthreads();

    // 2. w_i = N2 q_i + R with q_i = sum_r E_ir / c_r in column order, one thread
    //    per row: the thread reads its row of F_l A (just read above, so mostly
    //    from cache) eight entries at a time and adds its terms in order (a
    //    zero column's term is 0, which leaves q unchanged).
    for (int i = tid; i < n1; i += nt) {
        const size_t row0 = size_t(i) * R;
        double q = 0.0;
        for (int r0 = 0; r0 < R; r0 += 8) {
            float2 v[8];
#pragma unroll
            for (int w = 0; w < 8; ++w) v[w] = Ah[row0 + min(r0 + w, R - 1)];
#pragma unroll
            for (int w = 0; w < 8; ++w) {
                const double c = L.c[min(r0 + w, R - 1)];
                const double t = energy(v[w]) / (c > 0.0 ? c : 1.0);
                q = q + ((r0 + w < R && c > 0.0) ? t : 0.0);
            }
        }
        double w = double(n2) * q;
        w = w + double(R);
        L.pref[i] = w;
    }
    __syncthreads();

    // 3. Inclusive prefix in row order (one thread, loads a batch ahead; the
    //    padded tail is read and written but never used); meanwhile the other
    //    wavefronts draw the first kUPre uniforms.
    if (tid >= 64) {
        const int kp = min(K, kUPre);
        for (int k = tid - 64; k < kp; k += nt - 64) L.u[k] = uniform_trial(t_next, k, f.seed, f.sid);
    }
    if (tid == 0) {
        double2* p2 = reinterpret_cast<double2*>(L.pref);
        constexpr int kH = kPB / 2;
        double run = 0.0;
        for (int h0 = 0; h0 < cdiv(n1, 2); h0 += kH) {
            double2 v[kH];
#pragma unroll
            for (int w = 0; w < kH; ++w) v[w] = p2[h0 + w];
#pragma unroll
            for (int w = 0; w < kH; ++w) {
                run = run + v[w].x;
                v[w].x = run;
                run = run + v[w].y;
                v[w].y = run;
            }
#pragma unroll
            for (int w = 0; w < kH; ++w) p2[h0 + w] = v[w];
        }
    }
    __syncthreads();

    // 4. Trials: first row whose prefix exceeds u_k W.
    const double W = L.pref[n1 - 1];
    for (int k = tid; k < K; k += nt) {
        const double u = k < kUPre ? L.u[k] : uniform_trial(t_next, k, f.seed, f.sid);
        const double target = u * W;
        int lo = 0, hi = n1;
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (target < L.pref[mid]) hi = mid; else lo = mid + 1;
        }
        const int idx = lo < n1 ? lo : n1 - 1;
        if (f.draws_next) f.draws_next[k] = idx;
        L.mark[idx] = 1;
    }
    __syncthreads();

    // 5. The distinct rows in ascending order: per 64-row word a ballot, its
    //    population count gives the word's offset, the lane's rank inside the
    //    word its position (integers, so the result is exact).
    const int nw = cdiv(n1, 64), lane = tid % 64;
    for (int wd = tid / 64; wd < nw; wd += nt / 64) {
        const int i = wd * 64 + lane;
        const unsigned long long m = __ballot(i < n1 && L.mark[i]);
        if (lane == 0) L.wcount[wd] = __popcll(m);
    }
    __syncthreads();
    for (int wd = tid / 64; wd < nw; wd += nt / 64) {
        const int i = wd * 64 + lane;
        const bool on = i < n1 && L.mark[i];
        const unsigned long long m = __ballot(on);
        int base = 0;
        for (int v = 0; v < wd; ++v) base += L.wcount[v];
        if (on) f.rows_next[base + __popcll(m & ((1ull << lane) - 1ull))] = i;
    }
    if (tid == 0) {
        int total = 0;
        for (int v = 0; v < nw; ++v) total += L.wcount[v];
        f.n_next[0] = total;
    }
    if (f.prefix_next)
        for (int i = tid; i < n1; i += nt) f.prefix_next[i] = L.pref[i];
}

}  // namespace tsl
