// Column-direction kernels (transform along the row index of a row-major array).
//
// A block owns kTW adjacent columns and all N rows of them, so a column
// transform needs no transpose: every global access is a kTW-wide contiguous
// row segment, and the two exchanges of the transform go through LDS.
//
//  k_col_resid   forward column pass of F(X-) (Sec. IV), the masked residual
//                Xi = M .* (Y - F(X-)) of Algorithm 3 (e = y - <phi, gamma>), the
//                inverse column pass of Theta = F^{-1}(Xi) (Sec. IV-B), and
//                W = Z^T conj(A) with Z the column-inverted residual.  Since
//                Theta = Z F_r^H and F_r is symmetric, Theta^T conj(A) =
//                F_r^H W, so the B gradient needs only a length-n2 inverse
//                transform of the n2 x R matrix W (done in k_update_b).
//  k_update_a    A <- (1 - lambda mu/t) A + mu Theta conj(B) conj(diag gamma)
//                (Algorithm 3, S2) and the k-space factor F_l A of the new A.
//  k_update_b    Theta^T conj(A) = F_r^H W, then the B update and F_r B.
//  k_colfft      plain column pass of the standalone 2-D transform.
//  k_factor_fft  column transform of an [n][r] factor (start-up transforms).
#include "fft_engine.hpp"
#include "kernels.hpp"

namespace tsl {
namespace {

constexpr int kTW = 16;   // columns per block (128-byte row segments)
constexpr int kRW = 8;    // rank columns per pass of Z^T conj(A)

template <int N> struct ColShape {
    static constexpr int P = Plan<N>::P, Q = Plan<N>::Q, T = Plan<N>::T;
    static constexpr int THREADS = kTW * T;
    static constexpr int PITCH_NK = odd_pitch(Q, kTW);   // entry (k1, n2, c) at k1*PITCH_NK + n2*kTW + c
    static constexpr int PITCH_KN = odd_pitch(P, kTW);   // entry (m1, k1, c) at m1*PITCH_KN + k1*kTW + c
    static constexpr int XSIZE = (P * PITCH_NK > Q * PITCH_KN) ? P * PITCH_NK : Q * PITCH_KN;
};

// natural layout (thread s = n2 < Q) -> k-layout (thread s = k1 < P)
template <int N, int T>
__device__ __forceinline__ void col_swap_nk(float2 (&v)[T], float2* s_x, int c, int s) {
    using S = ColShape<N>;
    __syncthreads();
    if (s < S::Q) {
        sfor<S::P>([&](auto k) {
            constexpr int k1 = decltype(k)::value;
            s_x[k1 * S::PITCH_NK + s * kTW + c] = v[k1];
        });
    }
    __syncthreads();
    if (s < S::P) {
        sfor<S::Q>([&](auto n) {
            constexpr int n2 = decltype(n)::value;
            v[n2] = s_x[s * S::PITCH_NK + n2 * kTW + c];
        });
    }
}

// k-layout (thread s = k1 < P) -> natural layout (thread s = m1 < Q)
template <int N, int T>
__device__ __forceinline__ void col_swap_kn(float2 (&v)[T], float2* s_x, int c, int s) {
    using S = ColShape<N>;
    __syncthreads();
    if (s < S::P) {
        sfor<S::Q>([&](auto m) {
            constexpr int m1 = decltype(m)::value;
            s_x[m1 * S::PITCH_KN + s * kTW + c] = v[m1];
        });
    }
    __syncthreads();
    if (s < S::Q) {
        sfor<S::P>([&](auto k) {
            constexpr int k1 = decltype(k)::value;
            v[k1] = s_x[s * S::PITCH_KN + k1 * kTW + c];
        });
    }
}

template <int T> __device__ __forceinline__ void zero(float2 (&v)[T]) {
    sfor<T>([&](auto k) { v[decltype(k)::value] = float2{0.f, 0.f}; });
}

constexpr int cmax(int a, int b) { return a > b ? a : b; }

// ---------------------------------------------------------------- K2
template <int N1, class Src>
__global__ void __launch_bounds__(512) k_col_resid(Src src) {
    using S = ColShape<N1>;
    constexpr int P = S::P, Q = S::Q, T = S::T;
    constexpr int AW = N1 * kRW;            // A chunk [i][cc]
    constexpr int RW = Q * kTW * kRW;       // partials [s][c][cc]
    __shared__ float2 s_tw[N1];
    __shared__ int s_map[N1];
    __shared__ float2 s_u[cmax(S::XSIZE, AW + RW)];
    __shared__ int s_bad;

    const DevFrame f = src.get();
    if (!block_frame_ok(f.dev, true)) return;
    const int n2 = f.n2, R = f.r;
    const int tid = threadIdx.x, c = tid % kTW, s = tid / kTW;
    const int col = blockIdx.x * kTW + c;
    const bool cv = col < n2;
    load_tw<N1>(s_tw);
    if (tid == 0) s_bad = 0;
    if (f.mode == MODE_LINES) {
        for (int k = tid; k < N1; k += blockDim.x) s_map[k] = -1;
        __syncthreads();
        const int nr = frame_rows(f);
        for (int q = tid; q < nr; q += blockDim.x) {
            const int k = f.rows[q];
            if (k >= 0 && k < N1) s_map[k] = q;
        }
    }
    __syncthreads();

    float2 v[T];
    zero(v);
    if (s < Q && cv) {
        sfor<P>([&](auto q) {
            constexpr int n1c = decltype(q)::value;
            v[n1c] = f.frame[size_t(Q * n1c + s) * n2 + col];
        });
    }
    if (s < Q) dft_twiddle<N1, P, false>(v, s, s_tw);
    col_swap_nk<N1>(v, s_u, c, s);
    if (s < P) {
        dft_only<Q, false>(v);
        const bool lines = f.mode == MODE_LINES;
        sfor<Q>([&](auto kk) {
            constexpr int k2 = decltype(kk)::value;
            const int k = s + P * k2;
            const float2 K = cscale(v[k2], InvSqrt<N1>::value);
            float2 e{0.f, 0.f};
            if (cv) {
                if (lines) {
                    const int q = s_map[k];
                    if (q >= 0) e = csub(line_samples(f, q, k)[col], K);
                } else if (f.mask[size_t(k) * n2 + col]) {
                    e = csub(f.y[size_t(k) * n2 + col], K);
                }
            }
            v[k2] = e;
        });
        dft_twiddle<N1, Q, true>(v, s, s_tw);
    }
    col_swap_kn<N1>(v, s_u, c, s);
    if (s < Q) {
        dft_only<P, true>(v);
        sfor<P>([&](auto m) {
            constexpr int m2 = decltype(m)::value;
            v[m2] = cscale(v[m2], InvSqrt<N1>::value);
            if (cv) f.frame[size_t(s + Q * m2) * n2 + col] = v[m2];
        });
    }
    // v[m2] = Z[s + Q*m2][col] for threads s < Q.  W[col][r] = sum_i Z[i][col] conj(A[i][r]).
    float2* s_A = s_u;
    float2* s_r = s_u + AW;
    bool bad = false;
    for (int r0 = 0; r0 < R; r0 += kRW) {
        __syncthreads();
        stage_copy<8, float2>(
            N1 * kRW,
            [&](int e) {
                const int ii = e / kRW, cc = e % kRW;
                return (r0 + cc < R) ? f.A[size_t(ii) * R + r0 + cc] : float2{0.f, 0.f};
            },
            [&](int e, float2 v) { s_A[e] = v; });
        __syncthreads();
        if (s < Q) {
#pragma unroll
            for (int cc = 0; cc < kRW; ++cc) {
                float2 acc{0.f, 0.f};
                sfor<P>([&](auto m) {
                    constexpr int m2 = decltype(m)::value;
                    acc = cadd(acc, cmulc(v[m2], s_A[(s + Q * m2) * kRW + cc]));
                });
                s_r[(s * kTW + c) * kRW + cc] = acc;
            }
        }
        __syncthreads();
        for (int e = tid; e < kTW * kRW; e += blockDim.x) {
            const int c2 = e / kRW, cc = e % kRW, colw = blockIdx.x * kTW + c2;
            if (colw < n2 && r0 + cc < R) {
                float2 w{0.f, 0.f};
                for (int q = 0; q < Q; ++q) w = cadd(w, s_r[(q * kTW + c2) * kRW + cc]);
                bad |= !finite2(w);
                f.Wb[size_t(colw) * R + r0 + cc] = w;
            }
        }
    }
    if (bad) s_bad = 1;
    __syncthreads();
    if (tid == 0 && s_bad) latch(f.dev, ST_ENONFINITE);
}

// ---------------------------------------------------------------- K4 (A)
template <int N1, class Src>
__global__ void __launch_bounds__(512) k_update_a(Src src) {
    using S = ColShape<N1>;
    constexpr int P = S::P, Q = S::Q, T = S::T;
    __shared__ float2 s_tw[N1];
    __shared__ float2 s_x[S::XSIZE];
    const DevFrame f = src.get();
    if (!block_frame_ok(f.dev, true)) return;
    const int R = f.r;
    if (int(blockIdx.x) * kTW >= R) return;
    SeqDev* d = f.dev;
    const double mu = d->mu, sh = d->shrink;
    const int tid = threadIdx.x, c = tid % kTW, s = tid / kTW;
    const int r = blockIdx.x * kTW + c;
    const bool rv = r < R;
    const double2 g = rv ? f.gamma64[r] : double2{0.0, 0.0};
    load_tw<N1>(s_tw);
    if (blockIdx.x == 0 && tid == 0) {
        d->abar = d->abar_new;
        d->t = d->t_new;
    }
    float2 v[T];
    zero(v);
    if (s < Q && rv) {
        sfor<P>([&](auto q) {
            constexpr int n1c = decltype(q)::value;
            const size_t at = size_t(Q * n1c + s) * R + r;
            const float2 a = f.A[at], ga = f.GA[at];
            // ga * conj(gamma) in double
            const double gr = double(ga.x) * g.x + double(ga.y) * g.y;
            const double gi = double(ga.y) * g.x - double(ga.x) * g.y;
            const float2 an{float(sh * a.x + mu * gr), float(sh * a.y + mu * gi)};
            f.A[at] = an;
            if (f.A_out) f.A_out[at] = an;
            v[n1c] = an;
        });
    }
    __syncthreads();
    if (s < Q) dft_twiddle<N1, P, false>(v, s, s_tw);
    col_swap_nk<N1>(v, s_x, c, s);
    if (s < P) {
        dft_only<Q, false>(v);
        if (rv) {
            sfor<Q>([&](auto k) {
                constexpr int k2 = decltype(k)::value;
                f.Ahat[size_t(s + P * k2) * R + r] = cscale(v[k2], InvSqrt<N1>::value);
            });
        }
    }
}

// ---------------------------------------------------------------- K4 (B)
template <int N2, class Src>
__global__ void __launch_bounds__(512) k_update_b(Src src) {
    using S = ColShape<N2>;
    constexpr int P = S::P, Q = S::Q, T = S::T;
    __shared__ float2 s_tw[N2];
    __shared__ float2 s_x[S::XSIZE];
    const DevFrame f = src.get();
    if (!block_frame_ok(f.dev, true)) return;
    const int R = f.r;
    if (int(blockIdx.x) * kTW >= R) return;
    const SeqDev* d = f.dev;
    const double mu = d->mu, sh = d->shrink;
    const int tid = threadIdx.x, c = tid % kTW, s = tid / kTW;
    const int r = blockIdx.x * kTW + c;
    const bool rv = r < R;
    const double2 g = rv ? f.gamma64[r] : double2{0.0, 0.0};
    load_tw<N2>(s_tw);
    float2 v[T];
    zero(v);
    if (s < Q && rv) {
        sfor<P>([&](auto q) {
            constexpr int n1c = decltype(q)::value;
            v[n1c] = f.Wb[size_t(Q * n1c + s) * R + r];
        });
    }
    __syncthreads();
    // Theta^T conj(A) = F_r^H W: inverse transform along the row index of W.
    if (s < Q) dft_twiddle<N2, P, true>(v, s, s_tw);
    col_swap_nk<N2>(v, s_x, c, s);
    if (s < P) {
        dft_only<Q, true>(v);
        sfor<Q>([&](auto k) {
            constexpr int k2 = decltype(k)::value;
            const float2 gb = cscale(v[k2], InvSqrt<N2>::value);
            float2 bn{0.f, 0.f};
            if (rv) {
                const size_t at = size_t(s + P * k2) * R + r;
                const float2 b = f.B[at];
                const double gr = double(gb.x) * g.x + double(gb.y) * g.y;
                const double gi = double(gb.y) * g.x - double(gb.x) * g.y;
                bn = float2{float(sh * b.x + mu * gr), float(sh * b.y + mu * gi)};
                f.B[at] = bn;
                if (f.B_out) f.B_out[at] = bn;
            }
            v[k2] = bn;
        });
        // F_r B of the new B, starting from this k-layout.
        dft_twiddle<N2, Q, false>(v, s, s_tw);
    }
    col_swap_kn<N2>(v, s_x, c, s);
    if (s < Q) {
        dft_only<P, false>(v);
        if (rv) {
            sfor<P>([&](auto m) {
                constexpr int m2 = decltype(m)::value;
                f.Bhat[size_t(s + Q * m2) * R + r] = cscale(v[m2], InvSqrt<N2>::value);
            });
        }
    }
}

// ---------------------------------------------------------------- standalone column pass
// Column transform of `batch` arrays [N1][ld] (columns 0..ncols-1), natural order.
template <int N1, bool INV>
__global__ void __launch_bounds__(512) k_colfft(const float2* in, float2* out, int ncols, int ld,
                                                 size_t batch_stride) {
    using S = ColShape<N1>;
    constexpr int P = S::P, Q = S::Q, T = S::T;
    __shared__ float2 s_tw[N1];
    __shared__ float2 s_x[S::XSIZE];
    const int tid = threadIdx.x, c = tid % kTW, s = tid / kTW;
    const int col = blockIdx.x * kTW + c;
    const bool cv = col < ncols;
    const float2* src = in + blockIdx.y * batch_stride;
    float2* dst = out + blockIdx.y * batch_stride;
    load_tw<N1>(s_tw);
    float2 v[T];
    zero(v);
    if (s < Q && cv) {
        sfor<P>([&](auto q) {
            constexpr int n1c = decltype(q)::value;
            v[n1c] = src[size_t(Q * n1c + s) * ld + col];
        });
    }
    __syncthreads();
    if (s < Q) dft_twiddle<N1, P, INV>(v, s, s_tw);
    col_swap_nk<N1>(v, s_x, c, s);
    if (s < P) {
        dft_only<Q, INV>(v);
        if (cv) {
            sfor<Q>([&](auto k) {
                constexpr int k2 = decltype(k)::value;
                dst[size_t(s + P * k2) * ld + col] = cscale(v[k2], InvSqrt<N1>::value);
            });
        }
    }
}

template <int N1> hipError_t launch_k2_n(const Batch& b, hipStream_t st) {
    using S = ColShape<N1>;
    dim3 grid(cdiv(b.n2, kTW), b.table ? b.count : 1);
    if (b.table) k_col_resid<N1, FrameTable><<<grid, S::THREADS, 0, st>>>(FrameTable{b.table});
    else k_col_resid<N1, OneFrame><<<grid, S::THREADS, 0, st>>>(OneFrame{*b.one});
    return hipGetLastError();
}
template <int N1> hipError_t launch_k4a_n(const Batch& b, hipStream_t st) {
    using S = ColShape<N1>;
    dim3 grid(cdiv(b.r_max, kTW), b.table ? b.count : 1);
    if (b.table) k_update_a<N1, FrameTable><<<grid, S::THREADS, 0, st>>>(FrameTable{b.table});
    else k_update_a<N1, OneFrame><<<grid, S::THREADS, 0, st>>>(OneFrame{*b.one});
    return hipGetLastError();
}
template <int N2> hipError_t launch_k4b_n(const Batch& b, hipStream_t st) {
    using S = ColShape<N2>;
    dim3 grid(cdiv(b.r_max, kTW), b.table ? b.count : 1);
    if (b.table) k_update_b<N2, FrameTable><<<grid, S::THREADS, 0, st>>>(FrameTable{b.table});
    else k_update_b<N2, OneFrame><<<grid, S::THREADS, 0, st>>>(OneFrame{*b.one});
    return hipGetLastError();
}
template <int N1>
hipError_t launch_colfft_n(int ncols, int ld, int batch, size_t bstride, const float2* in, float2* out, bool inv,
                           hipStream_t st) {
    using S = ColShape<N1>;
    dim3 grid(cdiv(ncols, kTW), batch);
    if (inv) k_colfft<N1, true><<<grid, S::THREADS, 0, st>>>(in, out, ncols, ld, bstride);
    else k_colfft<N1, false><<<grid, S::THREADS, 0, st>>>(in, out, ncols, ld, bstride);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_col_resid(const Batch& b, hipStream_t st) {
    switch (b.n1) {
#define TSL_X(N) case N: return launch_k2_n<N>(b, st);
        TSL_FOR_EACH_N(TSL_X)
#undef TSL_X
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_update_a(const Batch& b, hipStream_t st) {
    switch (b.n1) {
#define TSL_X(N) case N: return launch_k4a_n<N>(b, st);
        TSL_FOR_EACH_N(TSL_X)
#undef TSL_X
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_update_b(const Batch& b, hipStream_t st) {
    switch (b.n2) {
#define TSL_X(N) case N: return launch_k4b_n<N>(b, st);
        TSL_FOR_EACH_N(TSL_X)
#undef TSL_X
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_colfft(int n1, int n2, int batch, const float2* in, float2* out, bool inv, hipStream_t st) {
    switch (n1) {
#define TSL_X(N) case N: return launch_colfft_n<N>(n2, n2, batch, size_t(n1) * n2, in, out, inv, st);
        TSL_FOR_EACH_N(TSL_X)
#undef TSL_X
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_factor_fft(int n, int r, const float2* in, float2* out, bool inv, hipStream_t st) {
    switch (n) {
#define TSL_X(N) case N: return launch_colfft_n<N>(r, r, 1, 0, in, out, inv, st);
        TSL_FOR_EACH_N(TSL_X)
#undef TSL_X
        default: return hipErrorInvalidValue;
    }
}

bool size_supported(int n) {
    switch (n) {
#define TSL_X(N) case N: return true;
        TSL_FOR_EACH_N(TSL_X)
#undef TSL_X
        default: return false;
    }
}

int plan_threads(int n) {
    switch (n) {
#define TSL_X(N) case N: return Plan<N>::T;
        TSL_FOR_EACH_N(TSL_X)
#undef TSL_X
        default: return 0;
    }
}

}  // namespace tsl
