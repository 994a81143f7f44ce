// Informative line sampling (Algorithm 4 on rows, with the row score of
// Sec. VI-C) for one frame, run by one block of NT threads.  Used by the
// standalone draw kernel and by the first block of each frame of the output
// launch, which runs beside the output tiles (the draw reads F_l A of the new
// A only).
//
// Row weight w_i = N2 ||abar_i||^2 + R where abar_i is row i of F_l A with
// every column of nonzero norm normalised (a zero column is left out); K
// trials with replacement, trial k taking u_k = (first Philox4x64-10 word at
// counter (t+1, k, 0, 0), key (seed, stream id)) >> 11, times 2^-53, and
// drawing the first row whose inclusive weight prefix exceeds u_k W (W the
// computed total, the last row if none).  The paper fixes no order for these
// sums; every one of them runs in FP64 without fused multiply-adds as
// sequential sums over consecutive blocks of kSumBlock terms (each from 0),
// then the block sums in block order (from 0), and the prefix is the matching
// blocked scan, so the rows drawn match any IEEE implementation of the same
// order bit for bit while no dependent chain is longer than about
// 2 sqrt(terms).
#pragma once

#include "frame.hpp"
#include "tsl.h"

namespace tsl {

constexpr int kSampleThreads = 256;   // block size of the standalone draw kernel
constexpr int kUPre = 256;            // uniforms computed beside the prefix sum
constexpr int kSumBlock = 16;         // terms per block of the blocked sums
constexpr int kMaxBlk = kMaxN / kSumBlock;
static_assert(TSL_MAX_R % kSumBlock == 0, "column blocks tile the widest rank");
struct alignas(16) SampleLds {
    double pref[kMaxN];               // weights, then their inclusive prefix
    double c[TSL_MAX_R];              // column energies
    double u[kUPre];                  // u_k for k < kUPre
    double part[kMaxBlk * TSL_MAX_R]; // block sums: [row block][column], then [row][column block]
    double tot[kMaxBlk];              // the prefix's block totals, then the blocks before each
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

// Steps 1-2 of a draw for a factor F ([n][R], complex64): column energies
// c_r = sum over rows of E_ir = |F_ir|^2 (FP64) -- thread (b, r) adds rows
// [kSumBlock b, kSumBlock (b + 1)) of column r with all of its loads in flight
// (coalesced over r, indices clamped into the factor, rows past n adding +0,
// which leaves a nonnegative sum unchanged), the block sums meet in LDS and
// thread r adds them in block order -- then, for every row i and column block
// k, the sum of the terms E_ir / c_r of that block (a zero column's term is 0)
// into part[i * ncb + k]; the caller adds a row's block sums in block order.
// Ends with the block synchronised.
template <int NT>
__device__ __forceinline__ void row_weight_blocks(GlobalPtr<const float2> Fm, int n, int R, double* c_lds,
                                                  double* part) {
#pragma clang fp contract(off)
    const int tid = threadIdx.x;
    const int nblk = cdiv(n, kSumBlock), ncb = cdiv(R, kSumBlock);
    const size_t last = size_t(n) * R - 1;
    for (int p0 = 0; p0 < nblk * R; p0 += NT) {
        const int p = p0 + tid, b = p / R, r = p % R;
        float2 v[kSumBlock];
#pragma unroll
        for (int j = 0; j < kSumBlock; ++j) v[j] = Fm[min(size_t(b * kSumBlock + j) * R + r, last)];
        double pt = 0.0;
#pragma unroll
        for (int j = 0; j < kSumBlock; ++j) {
            const double e = energy(v[j]);
            pt = pt + (b * kSumBlock + j < n ? e : 0.0);
        }
        if (p < nblk * R) part[p] = pt;
    }
    __syncthreads();
    if (tid < R) {
        double cr = 0.0;
        for (int b = 0; b < nblk; ++b) cr = cr + part[b * R + tid];
        c_lds[tid] = cr;
    }
    __syncthreads();
    for (int p0 = 0; p0 < n * ncb; p0 += NT) {
        const int p = p0 + tid, i = min(p / ncb, n - 1), k = p % ncb;
        const size_t row0 = size_t(i) * R;
        float2 v[kSumBlock];
#pragma unroll
        for (int j = 0; j < kSumBlock; ++j) v[j] = Fm[row0 + min(k * kSumBlock + j, R - 1)];
        double pt = 0.0;
#pragma unroll
        for (int j = 0; j < kSumBlock; ++j) {
            const int r = k * kSumBlock + j;
            const double cc = c_lds[min(r, R - 1)];
            const double t = energy(v[j]) / (cc > 0.0 ? cc : 1.0);
            pt = pt + ((r < R && cc > 0.0) ? t : 0.0);
        }
        if (p < n * ncb) part[p] = pt;
    }
    __syncthreads();
}

// With parts_ready, the A update of this frame has left every row's block sums
// over the column blocks (wq[k][i], the terms E_ir / c_r of column block k in
// the order of step 2 below) and steps 1-2 reduce to adding them in block order;
// otherwise (the standalone draw, a frame that was not committed) they are
// formed here from F_l A.  Both give the same weights bit for bit.
template <int NT>
__device__ __forceinline__ void draw_rows(const DevFrame& f, SampleLds& L, bool parts_ready = false) {
#pragma clang fp contract(off)
    static_assert(NT % 64 == 0 && NT >= TSL_MAX_R && NT >= kMaxBlk, "block shape");
    const int K = f.K_next;
    if (K <= 0) return;
    const int n1 = f.n1, n2 = f.n2, R = f.r, tid = threadIdx.x;
    GlobalPtr<const float2> Ah = f.Ahat;
    const uint64_t t_next = uint64_t(f.dev->t + 1);
    const int nblk = cdiv(n1, kSumBlock), ncb = cdiv(R, kSumBlock);
    if (parts_ready) {
        for (int i = tid; i < n1; i += NT) {
            double part[TSL_MAX_R / kSumBlock];
#pragma unroll
            for (int k = 0; k < TSL_MAX_R / kSumBlock; ++k)
                if (k < ncb) part[k] = f.wq[size_t(k) * n1 + i];
            double q = 0.0;
#pragma unroll
            for (int k = 0; k < TSL_MAX_R / kSumBlock; ++k)
                if (k < ncb) q = q + part[k];
            double w = double(n2) * q;
            w = w + double(R);
            L.pref[i] = w;
            L.mark[i] = 0;
        }
        __syncthreads();
    } else {

    row_weight_blocks<NT>(Ah, n1, R, L.c, L.part);
    for (int i = tid; i < n1; i += NT) L.mark[i] = 0;
    __syncthreads();
    for (int i = tid; i < n1; i += NT) {
        double q = 0.0;
        for (int k = 0; k < ncb; ++k) q = q + L.part[i * ncb + k];
        double w = double(n2) * q;
        w = w + double(R);
        L.pref[i] = w;
    }
    __syncthreads();
    }

    // 3. Inclusive prefix, blocked: thread b scans its block of rows in order
    //    and keeps the block total, thread 0 adds the totals in block order
    //    (the sum of the blocks before each), and every row adds its block's
    //    offset; meanwhile the other wavefronts draw the first kUPre uniforms.
    if (tid >= 64) {
        const int kp = min(K, kUPre);
        for (int k = tid - 64; k < kp; k += NT - 64) L.u[k] = uniform_trial(t_next, k, f.seed, f.sid);
    }
    if (tid < nblk) {
        const int i0 = tid * kSumBlock, ni = min(kSumBlock, n1 - i0);
        double run = 0.0;
        for (int j = 0; j < ni; ++j) {
            run = run + L.pref[i0 + j];
            L.pref[i0 + j] = run;
        }
        L.tot[tid] = run;
    }
    __syncthreads();
    if (tid == 0) {
        double before = 0.0;
        for (int b = 0; b < nblk; ++b) {
            const double t = L.tot[b];
            L.tot[b] = before;
            before = before + t;
        }
    }
    __syncthreads();
    for (int i = tid; i < n1; i += NT) L.pref[i] = L.tot[i / kSumBlock] + L.pref[i];
    __syncthreads();

    // 4. Trials: first row whose prefix exceeds u_k W.
    const double W = L.pref[n1 - 1];
    for (int k = tid; k < K; k += NT) {
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
    for (int wd = tid / 64; wd < nw; wd += NT / 64) {
        const int i = wd * 64 + lane;
        const unsigned long long m = __ballot(i < n1 && L.mark[i]);
        if (lane == 0) L.wcount[wd] = __popcll(m);
    }
    __syncthreads();
    for (int wd = tid / 64; wd < nw; wd += NT / 64) {
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
        for (int i = tid; i < n1; i += NT) f.prefix_next[i] = L.pref[i];
}

// ---------------------------------------------------------------- points (eq. 13)
// Algorithm 4 on entries.  With a_i = ||abar_i||^2 over the rows of the
// column-normalised F_l A and b_j = ||bbar_j||^2 over those of F_r B (each
// summing to R), eq. 13 is the mixture s(i, j) = N2/(N1+N2) (a_i/R)(1/N2) +
// N1/(N1+N2) (1/N1)(b_j/R).  Trial k for frame t takes the first three Philox
// words at counter (t, k, 1, 0), u_m = (w_m >> 11) 2^-53: component A if
// u0 (N1 + N2) < N2, the weighted index the first whose inclusive blocked
// prefix exceeds u1 W (clamped to the last), the other floor(u2 N) (clamped to
// N - 1).  The distinct points are marked in an LDS bitmap; the mask is written
// from it and their count is its population count.
constexpr int kPointThreads = 512;
struct alignas(16) PointLds {
    double pa[kMaxN], pb[kMaxN];      // row weights of F_l A and F_r B, then their inclusive prefixes
    double c[TSL_MAX_R];
    double part[kMaxBlk * TSL_MAX_R];
    double tot[2][kMaxBlk];
    unsigned bits[kMaxN * kMaxN / 32];
    int cnt[kPointThreads / 64];
};

template <int NT>
__device__ __forceinline__ void blocked_scan(double* w, int n, double* tot) {
#pragma clang fp contract(off)
    const int tid = threadIdx.x, nblk = cdiv(n, kSumBlock);
    if (tid < nblk) {
        const int i0 = tid * kSumBlock, ni = min(kSumBlock, n - i0);
        double run = 0.0;
        for (int j = 0; j < ni; ++j) {
            run = run + w[i0 + j];
            w[i0 + j] = run;
        }
        tot[tid] = run;
    }
    __syncthreads();
    if (tid == 0) {
        double before = 0.0;
        for (int b = 0; b < nblk; ++b) {
            const double t = tot[b];
            tot[b] = before;
            before = before + t;
        }
    }
    __syncthreads();
    for (int i = tid; i < n; i += NT) w[i] = tot[i / kSumBlock] + w[i];
    __syncthreads();
}

__device__ __forceinline__ int first_above(const double* pref, int n, double target) {
    int lo = 0, hi = n;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (target < pref[mid]) hi = mid; else lo = mid + 1;
    }
    return lo < n ? lo : n - 1;
}

template <int NT>
__device__ __forceinline__ void draw_points(const DevFrame& f, int K, unsigned char* __restrict__ mask,
                                            int* __restrict__ n_out, int* __restrict__ draws, PointLds& L) {
#pragma clang fp contract(off)
    const int n1 = f.n1, n2 = f.n2, R = f.r, tid = threadIdx.x;
    const int ncb = cdiv(R, kSumBlock), nbits = n1 * n2, nwords = cdiv(nbits, 32);
    const uint64_t t_next = uint64_t(f.dev->t + 1);
    for (int w = tid; w < nwords; w += NT) L.bits[w] = 0u;
    GlobalPtr<const float2> facs[2] = {f.Ahat, f.Bhat};
    double* outs[2] = {L.pa, L.pb};
    const int ns[2] = {n1, n2};
    for (int which = 0; which < 2; ++which) {
        row_weight_blocks<NT>(facs[which], ns[which], R, L.c, L.part);
        for (int i = tid; i < ns[which]; i += NT) {
            double q = 0.0;
            for (int k = 0; k < ncb; ++k) q = q + L.part[i * ncb + k];
            outs[which][i] = q;
        }
        __syncthreads();
        blocked_scan<NT>(outs[which], ns[which], L.tot[which]);
    }
    const double Wa = L.pa[n1 - 1], Wb = L.pb[n2 - 1];
    for (int k = tid; k < K; k += NT) {
        uint64_t x[4] = {t_next, uint64_t(k), 1ull, 0ull};
        philox4x64_10(x, f.seed, f.sid);
        const double u0 = double(x[0] >> 11) * 0x1.0p-53, u1 = double(x[1] >> 11) * 0x1.0p-53;
        const double u2 = double(x[2] >> 11) * 0x1.0p-53;
        int i, j;
        if (u0 * double(n1 + n2) < double(n2)) {
            i = first_above(L.pa, n1, u1 * Wa);
            j = min(int(floor(u2 * double(n2))), n2 - 1);
        } else {
            j = first_above(L.pb, n2, u1 * Wb);
            i = min(int(floor(u2 * double(n1))), n1 - 1);
        }
        const int e = i * n2 + j;
        if (draws) draws[k] = e;
        atomicOr(&L.bits[e >> 5], 1u << (e & 31));
    }
    __syncthreads();
    int mine = 0;
    for (int e = tid; e < nbits; e += NT) {
        const unsigned on = (L.bits[e >> 5] >> (e & 31)) & 1u;
        mask[e] = static_cast<unsigned char>(on);
        mine += int(on);
    }
    for (int m = 32; m > 0; m >>= 1) mine += __shfl_xor(mine, m, 64);
    if (tid % 64 == 0) L.cnt[tid / 64] = mine;
    __syncthreads();
    if (tid == 0) {
        int total = 0;
        for (int w = 0; w < NT / 64; ++w) total += L.cnt[w];
        n_out[0] = total;
    }
}

}  // namespace tsl
