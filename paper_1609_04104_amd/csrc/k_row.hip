// Row-direction kernels (transform length n2, rows contiguous in memory).
//
//  k_synth_rowfft  synthesis of X- = A diag(gamma_t) B^T (eq. 2 slice; Algorithm 3
//                  forms F(a_r b_r^T)) fused with the forward row pass of the 2-D
//                  transform F(X) = F_l X F_r (Sec. IV): the frame is written
//                  once, already transformed along its rows.
//  k_row_inv_grad  inverse row pass of Theta = F^{-1}(Xi) (Sec. IV-B) fused with
//                  the gradient contraction Theta conj(B) of Algorithm 3's A
//                  update; Theta never leaves the chip.
//  k_rowfft        plain row pass of the standalone 2-D transform.
#include "fft_engine.hpp"
#include "kernels.hpp"

namespace tsl {
namespace {

constexpr int kRC = 8;   // rank columns staged per pass

template <int N> struct RowShape {
    static constexpr int P = Plan<N>::P, Q = Plan<N>::Q, T = Plan<N>::T;
    static constexpr int ROWS = (256 / T) > 0 ? 256 / T : 1;   // rows per block
    static constexpr int THREADS = ROWS * T;
    // LDS exchange: row rl, entry (b, a) at rl*RSTR + b*pitch + a.
    static constexpr int PITCH_NK = (Q % 2) ? Q : Q + 1;        // b = k1 < P, a = n2 < Q
    static constexpr int PITCH_KN = (P % 2) ? P : P + 1;        // b = m1 < Q, a = k1 < P
    static constexpr int RSTR = (P * PITCH_NK > Q * PITCH_KN) ? P * PITCH_NK : Q * PITCH_KN;
    static constexpr int XSIZE = ROWS * RSTR;
};

// Natural-layout thread (s = n2 < Q) -> k-layout thread (s = k1 < P) through LDS.
template <int N, int T>
__device__ __forceinline__ void row_swap_nk(float2 (&v)[T], float2* s_x, int rl, int s) {
    using S = RowShape<N>;
    if (s < S::Q) {
        sfor<S::P>([&](auto k) {
            constexpr int k1 = decltype(k)::value;
            s_x[rl * S::RSTR + k1 * S::PITCH_NK + s] = v[k1];
        });
    }
    __syncthreads();
    if (s < S::P) {
        sfor<S::Q>([&](auto n) {
            constexpr int n2 = decltype(n)::value;
            v[n2] = s_x[rl * S::RSTR + s * S::PITCH_NK + n2];
        });
    }
}

// ---------------------------------------------------------------- K1
template <int N2, class Src>
__global__ void __launch_bounds__(256) k_synth_rowfft(Src src) {
    using S = RowShape<N2>;
    constexpr int P = S::P, Q = S::Q, T = S::T, ROWS = S::ROWS;
    __shared__ float2 s_tw[N2];
    __shared__ float2 s_B[kRC * N2];        // [c][j] = B[j][r0 + c]
    __shared__ float2 s_ag[ROWS * kRC];     // [row][c] = A[i][r0 + c] gamma[r0 + c]
    __shared__ float2 s_x[S::XSIZE];

    const DevFrame f = src.get();
    if (!block_frame_ok(f.dev, true)) return;
    const int n1 = f.n1, R = f.r;
    const int tid = threadIdx.x, s = tid % T, rl = tid / T;
    const int i = blockIdx.x * ROWS + rl;
    load_tw<N2>(s_tw);

    float2 v[T];
    sfor<T>([&](auto k) { v[decltype(k)::value] = float2{0.f, 0.f}; });
    for (int r0 = 0; r0 < R; r0 += kRC) {
        __syncthreads();
        stage_copy<8, float2>(
            kRC * N2,
            [&](int e) {
                const int j = e / kRC, c = e % kRC;
                return (r0 + c < R) ? f.B[j * R + r0 + c] : float2{0.f, 0.f};
            },
            [&](int e, float2 v) { s_B[(e % kRC) * N2 + e / kRC] = v; });
        for (int e = tid; e < ROWS * kRC; e += blockDim.x) {
            const int rr = e / kRC, c = e % kRC, ii = blockIdx.x * ROWS + rr;
            s_ag[e] = (r0 + c < R && ii < n1) ? cmul(f.A[ii * R + r0 + c], f.gamma32[r0 + c])
                                               : float2{0.f, 0.f};
        }
        __syncthreads();
        if (s < Q) {
#pragma unroll
            for (int c = 0; c < kRC; ++c) {
                const float2 a = s_ag[rl * kRC + c];
                sfor<P>([&](auto q) {
                    constexpr int n1c = decltype(q)::value;
                    cfma(v[n1c], a, s_B[c * N2 + Q * n1c + s]);
                });
            }
        }
    }
    if (s < Q) dft_twiddle<N2, P, false>(v, s, s_tw);
    row_swap_nk<N2>(v, s_x, rl, s);
    if (s < P) {
        dft_only<Q, false>(v);
        if (i < n1) {
            float2* out = f.frame + size_t(i) * N2;
            sfor<Q>([&](auto k) {
                constexpr int k2 = decltype(k)::value;
                out[s + P * k2] = cscale(v[k2], InvSqrt<N2>::value);
            });
        }
    }
}

// ---------------------------------------------------------------- K3
template <int N2, class Src>
__global__ void __launch_bounds__(256) k_row_inv_grad(Src src) {
    using S = RowShape<N2>;
    constexpr int P = S::P, Q = S::Q, T = S::T, ROWS = S::ROWS;
    __shared__ float2 s_tw[N2];
    __shared__ float2 s_B[kRC * N2];              // [c][j] = B[j][r0 + c]
    __shared__ float2 s_x[S::XSIZE];
    __shared__ float2 s_red[ROWS * P * kRC];      // [row][s][c] partial sums
    __shared__ int s_bad;

    const DevFrame f = src.get();
    if (!block_frame_ok(f.dev, true)) return;
    const int n1 = f.n1, R = f.r;
    const int tid = threadIdx.x, s = tid % T, rl = tid / T;
    const int i = blockIdx.x * ROWS + rl;
    if (tid == 0) s_bad = 0;
    load_tw<N2>(s_tw);

    float2 v[T];
    sfor<T>([&](auto k) { v[decltype(k)::value] = float2{0.f, 0.f}; });
    if (s < Q && i < n1) {
        const float2* in = f.frame + size_t(i) * N2;
        sfor<P>([&](auto q) { v[decltype(q)::value] = in[Q * decltype(q)::value + s]; });
    }
    __syncthreads();   // twiddles visible
    if (s < Q) dft_twiddle<N2, P, true>(v, s, s_tw);
    row_swap_nk<N2>(v, s_x, rl, s);
    if (s < P) {
        dft_only<Q, true>(v);
        sfor<Q>([&](auto k) { v[decltype(k)::value] = cscale(v[decltype(k)::value], InvSqrt<N2>::value); });
    }
    // v[k2] = Theta[i][s + P*k2] for threads s < P.
    bool bad = false;
    for (int r0 = 0; r0 < R; r0 += kRC) {
        __syncthreads();
        stage_copy<8, float2>(
            kRC * N2,
            [&](int e) {
                const int j = e / kRC, c = e % kRC;
                return (r0 + c < R) ? f.B[j * R + r0 + c] : float2{0.f, 0.f};
            },
            [&](int e, float2 v) { s_B[(e % kRC) * N2 + e / kRC] = v; });
        __syncthreads();
        if (s < P) {
#pragma unroll
            for (int c = 0; c < kRC; ++c) {
                float2 acc{0.f, 0.f};
                sfor<Q>([&](auto k) {
                    constexpr int k2 = decltype(k)::value;
                    const float2 b = s_B[c * N2 + s + P * k2];
                    acc = cadd(acc, cmulc(v[k2], b));
                });
                s_red[(rl * P + s) * kRC + c] = acc;
            }
        }
        __syncthreads();
        for (int e = tid; e < ROWS * kRC; e += blockDim.x) {
            const int rr = e / kRC, c = e % kRC, ii = blockIdx.x * ROWS + rr;
            if (ii < n1 && r0 + c < R) {
                float2 g{0.f, 0.f};
                for (int q = 0; q < P; ++q) g = cadd(g, s_red[(rr * P + q) * kRC + c]);
                bad |= !finite2(g);
                f.GA[size_t(ii) * R + r0 + c] = g;
            }
        }
    }
    if (bad) s_bad = 1;
    __syncthreads();
    if (tid == 0 && s_bad) latch(f.dev, ST_ENONFINITE);
}

// ---------------------------------------------------------------- standalone row pass
template <int N2, bool INV>
__global__ void __launch_bounds__(256) k_rowfft(const float2* in, float2* out, int nrows) {
    using S = RowShape<N2>;
    constexpr int P = S::P, Q = S::Q, T = S::T, ROWS = S::ROWS;
    __shared__ float2 s_tw[N2];
    __shared__ float2 s_x[S::XSIZE];
    const int tid = threadIdx.x, s = tid % T, rl = tid / T;
    const size_t i = size_t(blockIdx.x) * ROWS + rl;
    load_tw<N2>(s_tw);
    float2 v[T];
    sfor<T>([&](auto k) { v[decltype(k)::value] = float2{0.f, 0.f}; });
    if (s < Q && i < size_t(nrows)) {
        const float2* src = in + i * N2;
        sfor<P>([&](auto q) { v[decltype(q)::value] = src[Q * decltype(q)::value + s]; });
    }
    __syncthreads();
    if (s < Q) dft_twiddle<N2, P, INV>(v, s, s_tw);
    row_swap_nk<N2>(v, s_x, rl, s);
    if (s < P) {
        dft_only<Q, INV>(v);
        if (i < size_t(nrows)) {
            float2* dst = out + i * N2;
            sfor<Q>([&](auto k) {
                constexpr int k2 = decltype(k)::value;
                dst[s + P * k2] = cscale(v[k2], InvSqrt<N2>::value);
            });
        }
    }
}

template <int N2> hipError_t launch_k1_n(const Batch& b, hipStream_t st) {
    using S = RowShape<N2>;
    dim3 grid(cdiv(b.n1, S::ROWS), b.table ? b.count : 1);
    if (b.table) k_synth_rowfft<N2, FrameTable><<<grid, S::THREADS, 0, st>>>(FrameTable{b.table});
    else k_synth_rowfft<N2, OneFrame><<<grid, S::THREADS, 0, st>>>(OneFrame{*b.one});
    return hipGetLastError();
}
template <int N2> hipError_t launch_k3_n(const Batch& b, hipStream_t st) {
    using S = RowShape<N2>;
    dim3 grid(cdiv(b.n1, S::ROWS), b.table ? b.count : 1);
    if (b.table) k_row_inv_grad<N2, FrameTable><<<grid, S::THREADS, 0, st>>>(FrameTable{b.table});
    else k_row_inv_grad<N2, OneFrame><<<grid, S::THREADS, 0, st>>>(OneFrame{*b.one});
    return hipGetLastError();
}
template <int N2> hipError_t launch_rowfft_n(int nrows, const float2* in, float2* out, bool inv, hipStream_t st) {
    using S = RowShape<N2>;
    dim3 grid(cdiv(nrows, S::ROWS));
    if (inv) k_rowfft<N2, true><<<grid, S::THREADS, 0, st>>>(in, out, nrows);
    else k_rowfft<N2, false><<<grid, S::THREADS, 0, st>>>(in, out, nrows);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_synth_rowfft(const Batch& b, hipStream_t st) {
    switch (b.n2) {
#define TSL_X(N) case N: return launch_k1_n<N>(b, st);
        TSL_FOR_EACH_N(TSL_X)
#undef TSL_X
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_row_inv_grad(const Batch& b, hipStream_t st) {
    switch (b.n2) {
#define TSL_X(N) case N: return launch_k3_n<N>(b, st);
        TSL_FOR_EACH_N(TSL_X)
#undef TSL_X
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_rowfft(int n1, int n2, int batch, const float2* in, float2* out, bool inv, hipStream_t st) {
    const int nrows = n1 * batch;
    switch (n2) {
#define TSL_X(N) case N: return launch_rowfft_n<N>(nrows, in, out, inv, st);
        TSL_FOR_EACH_N(TSL_X)
#undef TSL_X
        default: return hipErrorInvalidValue;
    }
}

}  // namespace tsl
