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
#include <atomic>

#include "fft_engine.hpp"
#include "kernels.hpp"
#include "mfma.hpp"
#include "sampler.hpp"

namespace tsl {
namespace {

constexpr int kTW = 16;   // columns per block (128-byte row segments)
constexpr int kWNT = 2;   // 16-rank MFMA tiles per pass of Z^T conj(A)

template <int N> struct ColShape {
    static constexpr int P = Plan<N>::P, Q = Plan<N>::Q, T = Plan<N>::T;
    static constexpr int THREADS = kTW * T;
    static constexpr int THREADS64 = (THREADS + 63) / 64 * 64;   // whole wavefronts (matrix-core passes)
    // k-space factor updates whose grid fits the device in one round: at least
    // eight wavefronts (the ones past the transform's rows take part in the
    // gradient terms only, which halves their dependent load groups)
    static constexpr int KS_THREADS = THREADS64 < 512 ? 512 : THREADS64;
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
__global__ void __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(ColShape<N1>::THREADS64 <= 256 ? 4 : 1)))
k_col_resid(Src src) {
    using S = ColShape<N1>;
    constexpr int P = S::P, Q = S::Q, T = S::T;
    constexpr int kWaves = S::THREADS64 / 64;
    constexpr int WNT = P > 16 ? 1 : kWNT;         // rank tiles per pass (register budget)
    constexpr int SW = kWaves * kTW * WNT * 16;    // per-wavefront partials of W
    __shared__ float2 s_tw[N1];
    __shared__ int s_map[N1];
    __shared__ float2 s_u[cmax(S::XSIZE, SW)];
    __shared__ int s_bad;

    if (!src.live()) return;
    const DevFrame f = src.get();
    const int n2 = f.n2, R = f.r;
    const int tid = threadIdx.x, c = tid % kTW, s = tid / kTW;
    const int col = src.bx() * kTW + c;
    const bool cv = col < n2;
    const bool lines = f.mode == MODE_LINES;
    // Loads that depend on nothing but the descriptor go out before the status
    // check (they read inside the frame's own buffers either way): the block's
    // columns of the row-transformed frame, the sampled-row count and indices.
    float2 v[T];
    zero(v);
    if (s < Q && cv) {
        sfor<P>([&](auto q) {
            constexpr int n1c = decltype(q)::value;
            v[n1c] = f.frame[size_t(Q * n1c + s) * n2 + col];
        });
    }
    const int cap = lines ? frame_rows_cap(f) : 0;
    const int nd = (lines && f.n_rows_dev) ? *f.n_rows_dev : cap;
    const int my_row = tid < cap ? f.rows[tid] : -1;
    for (int k = tid; k < N1; k += blockDim.x) s_map[k] = -1;
    if (tid == 0) s_bad = 0;
    load_tw<N1>(s_tw);
    if (!block_frame_ok(f.dev, true)) return;   // its barriers also order s_map's reset
    if (lines) {
        const int nr = nd < 0 ? 0 : (nd > cap ? cap : nd);
        if (tid < nr && my_row >= 0 && my_row < N1) s_map[my_row] = tid;
        for (int q = tid + int(blockDim.x); q < nr; q += blockDim.x) {
            const int k = f.rows[q];
            if (k >= 0 && k < N1) s_map[k] = q;
        }
    }
    __syncthreads();
    // The samples this thread's residual entries need (k = s + P k2 after the
    // forward transform), loaded now so that they arrive during the transform.
    // Masked lanes read a zero constant instead (the mask is in the address):
    // no select waits for these loads here, so they stay in flight through
    // the forward transform.
    float2 ys[Q];
    unsigned on = 0;                               // bit k2: entry k2 is sampled
    if (!lines) {
        // the mask bytes first: the bits below wait for them, not for the samples
        const bool ok = s < P && cv;
        unsigned char mk[Q];
        sfor<Q>([&](auto kk) {
            constexpr int k2 = decltype(kk)::value;
            mk[k2] = load_or_zero<unsigned char>(ok, f.mask + size_t(s + P * k2) * n2 + col);
        });
        sfor<Q>([&](auto kk) {
            constexpr int k2 = decltype(kk)::value;
            ys[k2] = load_or_zero<float2>(ok, f.y + size_t(s + P * k2) * n2 + col);
        });
        sfor<Q>([&](auto kk) {
            constexpr int k2 = decltype(kk)::value;
            if (mk[k2]) on |= 1u << k2;
        });
    } else {
        sfor<Q>([&](auto kk) {
            constexpr int k2 = decltype(kk)::value;
            const int k = s + P * k2;
            const int q = (s < P && cv) ? s_map[k] : -1;
            const bool ok = q >= 0;
            if (ok) on |= 1u << k2;
            ys[k2] = load_or_zero<float2>(ok, line_samples(f, ok ? q : 0, k) + col);
        });
    }
    if (s < Q) dft_twiddle<N1, P, false>(v, s, s_tw);
    col_swap_nk<N1>(v, s_u, c, s);
    if (s < P) {
        dft_only<Q, false>(v);
        sfor<Q>([&](auto kk) {
            constexpr int k2 = decltype(kk)::value;
            const float2 K = cscale(v[k2], InvSqrt<N1>::value);
            v[k2] = (on >> k2) & 1u ? csub(ys[k2], K) : float2{0.f, 0.f};
        });
        dft_twiddle<N1, Q, true>(v, s, s_tw);
    }
    // The factor values of the W contraction below, one 16-rank tile at a time:
    // few registers, so that four blocks share a compute unit and one block's
    // loads wait while the others compute.
    const int lane = tid % 64, wave = __builtin_amdgcn_readfirstlane(tid / 64), n = lane % 16;
    float2 av0[P];
    // masked lanes read the zero constant, as for the samples above
    auto load_a = [&](int t, float2 (&av)[P]) {
        sfor<P>([&](auto mc) {
            constexpr int m2 = decltype(mc)::value;
            const int i = s + Q * m2, r = 16 * t + n;
            av[m2] = load_or_zero<float2>(s < Q && r < R, f.A + size_t(i) * R + r);
        });
    };
    col_swap_kn<N1>(v, s_u, c, s);
    if (s < Q) {
        dft_only<P, true>(v);
        sfor<P>([&](auto m) {
            constexpr int m2 = decltype(m)::value;
            v[m2] = cscale(v[m2], InvSqrt<N1>::value);
            if (cv) f.frame[size_t(s + Q * m2) * n2 + col] = v[m2];
        });
    }
    // v[m2] = Z[s + Q*m2][col] for threads s < Q.  W[col][r] = sum_i Z[i][col] conj(A[i][r])
    // on the matrix cores: M = the block's kTW columns (lane % 16), N = 16 ranks
    // per tile, and the K index runs over rows, each lane feeding its own rows.
    // Gauss's three-multiplication form with the conjugate's sign on the factor:
    // P1 = sum Zr Ar, P2 = sum Zi (-Ai), P3 = sum (Zr + Zi)(Ar - Ai), so that
    // Re W = P1 - P2 and Im W = P3 - P1 - P2: three 16x16x4 steps per four rows
    // and rank tile.  A pass takes WNT rank tiles; the wavefronts' partial sums
    // over their rows meet in LDS and are added in wavefront order.
    load_a(0, av0);
    static_assert(kTW == 16, "one MFMA row per column of the tile");
    float2* s_w = s_u;                                   // [wave][c][WNT * 16]
    bool bad = false;
    const int ntr = cdiv(R, 16);                         // rank tiles
    for (int n0 = 0; n0 < R; n0 += WNT * 16) {
        f32x4 p1[WNT], p2[WNT], p3[WNT];
#pragma unroll
        for (int u = 0; u < WNT; ++u) p1[u] = p2[u] = p3[u] = f32x4{0.f, 0.f, 0.f, 0.f};
        auto products = [&](int u, const float2 (&av)[P]) {
            sfor<P>([&](auto mc) {
                constexpr int m2 = decltype(mc)::value;
                const float2 z = (s < Q) ? v[m2] : float2{0.f, 0.f};
                const float2 a = av[m2];
                p1[u] = mfma_16x16x4(z.x, a.x, p1[u]);
                p2[u] = mfma_16x16x4(z.y, -a.y, p2[u]);
                p3[u] = mfma_16x16x4(z.x + z.y, a.x - a.y, p3[u]);
            });
        };
        // tiles t0 = n0 / 16 and t0 + 1, one register set reused
        const int t0 = n0 / 16;
        products(0, av0);
        if constexpr (WNT > 1) {
            if (t0 + 1 < ntr) {
                load_a(t0 + 1, av0);
                products(1, av0);
            }
        }
        if (t0 + WNT < ntr) load_a(t0 + WNT, av0);      // the next pass's first tile
        __syncthreads();
#pragma unroll
        for (int u = 0; u < WNT; ++u)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int cc = 4 * (lane / 16) + e;                // column of the tile
                s_w[(wave * kTW + cc) * (WNT * 16) + 16 * u + n] =
                    float2{p1[u][e] - p2[u][e], p3[u][e] - p1[u][e] - p2[u][e]};
            }
        __syncthreads();
        for (int e = tid; e < kTW * WNT * 16; e += blockDim.x) {
            const int c2 = e / (WNT * 16), rr = e % (WNT * 16), colw = src.bx() * kTW + c2;
            if (colw < n2 && n0 + rr < R) {
                float2 w = s_w[c2 * (WNT * 16) + rr];
                for (int q = 1; q < kWaves; ++q) w = cadd(w, s_w[(q * kTW + c2) * (WNT * 16) + rr]);
                bad |= !finite2(w);
                f.Wb[size_t(colw) * R + n0 + rr] = w;
            }
        }
    }
    if (bad) s_bad = 1;
    __syncthreads();
    if (tid == 0 && s_bad) latch(f.dev, ST_ENONFINITE);
}

// ---------------------------------------------------------------- sampler weights of the new F_l A
// The A update block for ranks [kTW bx, kTW bx + kTW) (one column block of the
// sampler's blocked sums, kTW == kSumBlock) also forms, from the complex64
// values of the new F_l A it wrote (their energies E_ir in s_e[i][c]), the
// column energies c_r and every row's block sum over its columns of E_ir / c_r
// in the sampler's order (sampler.hpp), into wq[bx][i]; the draw of the same
// step then only adds the block sums of each row.
static_assert(kTW == kSumBlock, "an update block owns one column block of the sampler's sums");
constexpr int kWeightParts = (kMaxN / kSumBlock + 1) * kTW;   // block sums, then the column energies
template <int N1>
__device__ __forceinline__ void row_weight_parts(const DevFrame& f, int bx, const double* s_e, double* s_cp) {
#pragma clang fp contract(off)
    constexpr int nblk = (N1 + kSumBlock - 1) / kSumBlock;
    const int tid = threadIdx.x, R = f.r;
    for (int p = tid; p < nblk * kTW; p += blockDim.x) {      // thread (b, c): rows of block b, column c
        const int b = p / kTW, c = p % kTW;
        double part = 0.0;
#pragma unroll
        for (int j = 0; j < kSumBlock; ++j) {
            const int i = b * kSumBlock + j;
            part = part + (i < N1 ? s_e[min(i, N1 - 1) * kTW + c] : 0.0);
        }
        s_cp[p] = part;
    }
    __syncthreads();
    double* s_c = s_cp + nblk * kTW;
    if (tid < kTW) {
        double cr = 0.0;
        for (int b = 0; b < nblk; ++b) cr = cr + s_cp[b * kTW + tid];
        s_c[tid] = cr;
    }
    __syncthreads();
    for (int i = tid; i < N1; i += blockDim.x) {
        double part = 0.0;
#pragma unroll
        for (int c = 0; c < kTW; ++c) {
            const int r = bx * kTW + c;
            const double cc = s_c[c];
            const double t = s_e[i * kTW + c] / (cc > 0.0 ? cc : 1.0);
            part = part + ((r < R && cc > 0.0) ? t : 0.0);
        }
        f.wq[size_t(bx) * N1 + i] = part;
    }
}

// ---------------------------------------------------------------- k-space gradients
// On the k-space route (line masks) the residual E = Y_S - Ahat_S diag(gamma) Bhat^T
// of Algorithm 3 on the samples is not formed.  Its two contractions with the
// factors split into a data term and a model term,
//     M = E conj(Bhat)     = Y_S conj(Bhat)     + Ahat_S T_B,  T_B[s][r] = -gamma_s G_B[r][s],
//     W = E^T conj(Ahat_S) = Y_S^T conj(Ahat_S) + Bhat T_AS,   T_AS[s][r] = -gamma_s G_AS[r][s],
// with G_B = Bhat^H Bhat and G_AS = Ahat_S^H Ahat_S the Grams that the statistics
// launch already sums for the solve (sum_j Bhat_js conj(Bhat_jr) = G_B[r][s]).
// The statistics launch leaves the data terms (partials per chunk) and copies
// of Bhat and of the sampled rows of Ahat of frame t - 1 (this launch
// overwrites both); the update block of ranks [r0, r0 + kTW) adds the partials
// of its columns and the model term, K = R, on the matrix cores.

// Entry (r, s) of a Hermitian Gram summed over `ns` partial slots in slot order
// (a slot holds the entries on and above the diagonal, packed by rows); eight slots'
// loads go out before their adds (indices clamped, values past ns selected away).
__device__ __forceinline__ double2 gram_entry(GlobalPtr<const double2> slots, int ns, int R, int r, int s) {
    const bool up = r <= s;
    const size_t at = size_t(up ? upk(r, s, R) : upk(s, r, R));
    double2 acc{0.0, 0.0};
    for (int k0 = 0; k0 < ns; k0 += 8) {
        double2 v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const double2 x = slots[size_t(k0 + u < ns ? k0 + u : k0) * slot_size(R) + at];
            v[u] = k0 + u < ns ? x : double2{0.0, 0.0};
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            acc.x += v[u].x;
            acc.y += v[u].y;
        }
    }
    return up ? acc : double2{acc.x, -acc.y};
}

// s_T[s][c] = -gamma_s G[r0 + c][s] (FP64 product, stored as complex64; 0 past
// the rank): the model term's factor with its sign.
__device__ __forceinline__ void fill_model_t(const DevFrame& f, GlobalPtr<const double2> slots, int ns, int r0,
                                             float2* s_T) {
    const int R = f.r;
    for (int e = threadIdx.x; e < R * kTW; e += blockDim.x) {
        const int sr = e / kTW, r = r0 + e % kTW;
        float2 t{0.f, 0.f};
        if (r < R) {
            const double2 gm = gram_entry(slots, ns, R, r, sr);
            const double2 gs = f.gamma64[sr];
            t = float2{float(-(gs.x * gm.x - gs.y * gm.y)), float(-(gs.x * gm.y + gs.y * gm.x))};
        }
        s_T[e] = t;
    }
}

// store(e, sum over k < np of at(e, k)) for every e < n (thread-strided), the
// sums in part order in FP64; E elements per thread and C parts at a time have
// their loads in flight together (indices clamped, values past the ends
// selected away).
template <int E, int C, class At, class Store>
__device__ __forceinline__ void sum_fill(int n, int np, At at, Store store) {
    const int nt = int(blockDim.x);
    for (int e0 = int(threadIdx.x); e0 < n; e0 += E * nt) {
        double2 acc[E];
#pragma unroll
        for (int u = 0; u < E; ++u) acc[u] = double2{0.0, 0.0};
        for (int k0 = 0; k0 < np; k0 += C) {
            float2 v[E][C];
#pragma unroll
            for (int u = 0; u < E; ++u)
#pragma unroll
                for (int w = 0; w < C; ++w) {
                    const int e = e0 + u * nt, k = k0 + w;
                    const float2 x = at(min(e, n - 1), min(k, np - 1));
                    v[u][w] = (e < n && k < np) ? x : float2{0.f, 0.f};
                }
#pragma unroll
            for (int u = 0; u < E; ++u)
#pragma unroll
                for (int w = 0; w < C; ++w) {
                    acc[u].x += v[u][w].x;
                    acc[u].y += v[u][w].y;
                }
        }
#pragma unroll
        for (int u = 0; u < E; ++u) {
            const int e = e0 + u * nt;
            if (e < n) store(e, float2{float(acc[u].x), float(acc[u].y)});
        }
    }
}

// s_out[row_of(q)][c] += sum_{s < R} X[q][s] s_T[s][c] for q < nrows, c < kTW
// (X: [nrows][R] complex64) on the FP32 matrix cores in Gauss's three-product
// form (M = 16 rows, N = kTW ranks, K = four ranks per step).  A wavefront takes
// kMI row tiles per round; the K loop is the outer one, so that one group of
// kMC steps' operand loads serves all of them, and the next group's loads go
// out before the current group's products (few tiles: one tile and long
// groups; many tiles: several tiles and short groups, for the registers).
// Every thread of the block calls it.
template <int kMI, int kMC, class RowOf>
__device__ __forceinline__ void model_add(GlobalPtr<const float2> X, int nrows, int R, const float2* s_T,
                                          float2* s_out, RowOf row_of) {
    static_assert(kTW == 16, "one matrix-core column tile of ranks per block");
    const int lane = threadIdx.x % 64, wave = __builtin_amdgcn_readfirstlane(threadIdx.x / 64);
    const int nw = int(blockDim.x) / 64, m = lane % 16, g = lane / 16;
    const int ntile = cdiv(nrows, 16), nst = cdiv(R, 4);
    for (int base = wave; base < ntile; base += kMI * nw) {
        f32x4 p1[kMI], p2[kMI], p3[kMI];
#pragma unroll
        for (int u = 0; u < kMI; ++u) p1[u] = p2[u] = p3[u] = f32x4{0.f, 0.f, 0.f, 0.f};
        float2 xa0[kMI][kMC], tb0[kMC], xa1[kMI][kMC], tb1[kMC];
        auto load = [&](int st0, float2 (&xa)[kMI][kMC], float2 (&tb)[kMC]) {
#pragma unroll
            for (int v = 0; v < kMC; ++v) {
                const int k = 4 * (st0 + v) + g, kc = min(k, R - 1);
                const bool ok = st0 + v < nst && k < R;
                const float2 t0 = s_T[kc * kTW + m];
                tb[v] = ok ? t0 : float2{0.f, 0.f};
#pragma unroll
                for (int u = 0; u < kMI; ++u) {
                    const int q = 16 * (base + nw * u) + m;
                    const float2 x = X[size_t(min(q, nrows - 1)) * R + kc];
                    xa[u][v] = (ok && q < nrows) ? x : float2{0.f, 0.f};
                }
            }
        };
        auto products = [&](const float2 (&xa)[kMI][kMC], const float2 (&tb)[kMC]) {
#pragma unroll
            for (int v = 0; v < kMC; ++v)
#pragma unroll
                for (int u = 0; u < kMI; ++u) {
                    const float2 x = xa[u][v], y = tb[v];
                    p1[u] = mfma_16x16x4(x.x, y.x, p1[u]);
                    p2[u] = mfma_16x16x4(x.y, y.y, p2[u]);
                    p3[u] = mfma_16x16x4(x.x + x.y, y.x + y.y, p3[u]);
                }
        };
        load(0, xa0, tb0);
        for (int st0 = 0; st0 < nst; st0 += 2 * kMC) {
            if (st0 + kMC < nst) load(st0 + kMC, xa1, tb1);
            products(xa0, tb0);
            if (st0 + kMC >= nst) break;
            if (st0 + 2 * kMC < nst) load(st0 + 2 * kMC, xa0, tb0);
            products(xa1, tb1);
        }
        // D[4 g + i][m] of tile base + nw u: row 16 tile + 4 g + i, column m
#pragma unroll
        for (int u = 0; u < kMI; ++u)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int q = 16 * (base + nw * u) + 4 * g + i;
                if (q < nrows) {
                    float2& o = s_out[row_of(q) * kTW + m];
                    o = float2{o.x + (p1[u][i] - p2[u][i]), o.y + (p3[u][i] - p1[u][i] - p2[u][i])};
                }
            }
    }
}

// Sampled-row count of a k-space frame (clamped as the statistics launch clamps it).
__device__ __forceinline__ int kspace_rows(const DevFrame& f) { return frame_rows(f); }

// Dynamic LDS of a k-space update block: s_T [R][kTW], s_rows [n1].
__host__ __device__ constexpr size_t grad_lds(int R, int n1) { return size_t(R) * kTW * 8 + size_t(n1) * 4; }

// ---------------------------------------------------------------- K4 (A)
// Block bx of the A update of one frame (ranks [kTW bx, kTW bx + kTW)); s_tw
// holds N1 twiddles, s_x the exchange area of ColShape<N1>.
template <int N1>
__device__ __forceinline__ void update_a_body(const DevFrame& f, int bx, float2* s_tw, float2* s_x, double* s_cp,
                                              float2* s_dyn) {
    using S = ColShape<N1>;
    static_assert(S::XSIZE >= N1 * kTW, "the exchange area holds the energies of the block's columns");
    constexpr int P = S::P, Q = S::Q, T = S::T;
    const int R = f.r;
    if (bx * kTW >= R) return;
    const int tid = threadIdx.x, c = tid % kTW, s = tid / kTW;
    const int r = bx * kTW + c;
    const bool rv = r < R;
    // Loads that need only the descriptor go out before the status check (inside
    // the frame's own buffers): twiddles, gamma, and on the frame route A and GA
    // (both in row order; the k-space route loads A later).
    load_tw<N1>(s_tw);
    const double2 g = rv ? f.gamma64[r] : double2{0.0, 0.0};
    float2 v[T], apre[T];
    zero(v);
    zero(apre);
    if (!f.kspace && s < Q && rv) {
        sfor<P>([&](auto q) {
            constexpr int n1c = decltype(q)::value;
            const size_t at = size_t(Q * n1c + s) * R + r;
            apre[n1c] = f.A[at];
            v[n1c] = f.GA[at];
        });
    }
    if (!block_frame_ok(f.dev, true)) return;
    SeqDev* d = f.dev;
    const double mu = d->mu, sh = d->shrink;
    if (bx == 0 && tid == 0) {
        d->abar = d->abar_new;
        d->t = d->t_new;
    }
    if (f.kspace) {
        // Theta conj(B) = F_l^H M with M = E conj(Bhat) on the sampled rows and
        // zero elsewhere (above), built in s_x as [N1][kTW] with row i of the
        // frame at i kTW: the data term's partials over the readout chunks, then
        // the model term added.
        const int nS = kspace_rows(f), r0 = bx * kTW, nJ = n_jparts(f.n2);
        float2* s_T = s_dyn;
        int* s_rows = reinterpret_cast<int*>(s_T + R * kTW);
        for (int e = tid; e < N1 * kTW; e += blockDim.x) s_x[e] = float2{0.f, 0.f};
        for (int q = tid; q < nS; q += blockDim.x) s_rows[q] = f.rows[q];
        fill_model_t(f, f.part + size_t(n_gparts(N1)) * slot_size(R), n_gparts(f.n2), r0, s_T);
        __syncthreads();
        GlobalPtr<const float2> Zm = f.zm;
        sum_fill<2, 8>(
            nS * kTW, nJ,
            [&](int e, int j) {
                const int q = e / kTW, rr = min(r0 + e % kTW, R - 1);
                return float2(Zm[((size_t(q / kSRows) * nJ + j) * kSRows + q % kSRows) * R + rr]);
            },
            [&](int e, float2 z) { s_x[s_rows[e / kTW] * kTW + e % kTW] = r0 + e % kTW < R ? z : float2{0.f, 0.f}; });
        __syncthreads();
        model_add<1, 8>(f.acopy, nS, R, s_T, s_x, [&](int q) { return s_rows[q]; });
        // A at the update's layout after the transform (loaded here, where the
        // model term no longer holds registers; it arrives during the transform)
        if (s < P && rv)
            sfor<Q>([&](auto k) {
                constexpr int k2 = decltype(k)::value;
                apre[k2] = f.A[size_t(s + P * k2) * R + r];
            });
        __syncthreads();
        if (s < Q && rv)
            sfor<P>([&](auto qc) {
                constexpr int n1c = decltype(qc)::value;
                v[n1c] = s_x[(Q * n1c + s) * kTW + c];
            });
        // then the update in the transform's output layout and F_l A of the
        // new A, as in the B update
        __syncthreads();
        if (s < Q) dft_twiddle<N1, P, true>(v, s, s_tw);
        col_swap_nk<N1>(v, s_x, c, s);
        if (s < P) {
            dft_only<Q, true>(v);
            sfor<Q>([&](auto k) {
                constexpr int k2 = decltype(k)::value;
                const float2 ga = cscale(v[k2], InvSqrt<N1>::value);
                float2 an{0.f, 0.f};
                if (rv) {
                    const size_t at = size_t(s + P * k2) * R + r;
                    const float2 a = apre[k2];
                    const double gr = double(ga.x) * g.x + double(ga.y) * g.y;
                    const double gi = double(ga.y) * g.x - double(ga.x) * g.y;
                    an = float2{float(sh * a.x + mu * gr), float(sh * a.y + mu * gi)};
                    f.A[at] = an;
                    if (f.A_out) f.A_out[at] = an;
                }
                v[k2] = an;
            });
            dft_twiddle<N1, Q, false>(v, s, s_tw);
        }
        col_swap_kn<N1>(v, s_x, c, s);
        if (s < Q) {
            dft_only<P, false>(v);
            sfor<P>([&](auto m) {
                constexpr int m2 = decltype(m)::value;
                v[m2] = cscale(v[m2], InvSqrt<N1>::value);
                if (rv) store_nt(f.Ahat + size_t(s + Q * m2) * R + r, v[m2]);   // read by the next step
            });
        }
        __syncthreads();                      // s_x is free: it takes the energies
        double* s_e = reinterpret_cast<double*>(s_x);
        if (s < Q)
            sfor<P>([&](auto m) {
                constexpr int m2 = decltype(m)::value;
                s_e[(s + Q * m2) * kTW + c] = rv ? energy(v[m2]) : 0.0;
            });
        __syncthreads();
        row_weight_parts<N1>(f, bx, s_e, s_cp);
        return;
    }
    if (s < Q && rv) {
        sfor<P>([&](auto q) {
            constexpr int n1c = decltype(q)::value;
            const size_t at = size_t(Q * n1c + s) * R + r;
            const float2 a = apre[n1c], ga = v[n1c];
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
        sfor<Q>([&](auto k) {
            constexpr int k2 = decltype(k)::value;
            v[k2] = cscale(v[k2], InvSqrt<N1>::value);
            if (rv) store_nt(f.Ahat + size_t(s + P * k2) * R + r, v[k2]);   // read by the next step
        });
    }
    __syncthreads();                          // s_x is free: it takes the energies
    double* s_e = reinterpret_cast<double*>(s_x);
    if (s < P)
        sfor<Q>([&](auto k) {
            constexpr int k2 = decltype(k)::value;
            s_e[(s + P * k2) * kTW + c] = rv ? energy(v[k2]) : 0.0;
        });
    __syncthreads();
    row_weight_parts<N1>(f, bx, s_e, s_cp);
}

// Dynamic LDS of the update launches: the k-space gradients' areas (grad_lds).
template <int N1, class Src>
__global__ void __launch_bounds__(512) k_update_a(Src src) {
    extern __shared__ float2 s_dyn[];
    __shared__ float2 s_tw[N1];
    __shared__ float2 s_x[ColShape<N1>::XSIZE];
    __shared__ double s_cp[kWeightParts];
    if (!src.live()) return;
    update_a_body<N1>(src.get(), src.bx(), s_tw, s_x, s_cp, s_dyn);
}

// ---------------------------------------------------------------- K4 (B)
// Block bx of the B update of one frame, as the A update above.
template <int N2>
__device__ __forceinline__ void update_b_body(const DevFrame& f, int bx, float2* s_tw, float2* s_x, float2* s_dyn) {
    using S = ColShape<N2>;
    static_assert(S::XSIZE >= N2 * kTW, "the exchange area holds the block's columns of W");
    constexpr int P = S::P, Q = S::Q, T = S::T;
    const int R = f.r;
    if (bx * kTW >= R) return;
    const int tid = threadIdx.x, c = tid % kTW, s = tid / kTW;
    const int r = bx * kTW + c;
    const bool rv = r < R;
    // Loads that need only the descriptor go out before the status check (inside
    // the frame's own buffers): twiddles, gamma, and on the frame route W and B
    // at the update's layout (the k-space route loads B later).
    load_tw<N2>(s_tw);
    const double2 g = rv ? f.gamma64[r] : double2{0.0, 0.0};
    float2 v[T];
    zero(v);
    if (!f.kspace && s < Q && rv) {
        sfor<P>([&](auto q) {
            constexpr int n1c = decltype(q)::value;
            v[n1c] = f.Wb[size_t(Q * n1c + s) * R + r];
        });
    }
    float2 bpre[Q];
    auto load_bpre = [&]() {
        sfor<Q>([&](auto k) {
            constexpr int k2 = decltype(k)::value;
            bpre[k2] = (s < P && rv) ? float2(f.B[size_t(s + P * k2) * R + r]) : float2{0.f, 0.f};
        });
    };
    if (!f.kspace) load_bpre();
    if (!block_frame_ok(f.dev, true)) return;
    const SeqDev* d = f.dev;
    const double mu = d->mu, sh = d->shrink;
    if (f.kspace) {
        // W = E^T conj(Ahat_S) (above), built in s_x as [N2][kTW]: the data
        // term's partials over the chunks of sampled rows, then the model term
        const int nsc = cdiv(kspace_rows(f), kSRows), r0 = bx * kTW;
        float2* s_T = s_dyn;
        const int gAB = n_gparts(f.n1) + n_gparts(N2);
        GlobalPtr<const float2> Zw = f.zw;
        auto zw_at = [&](int e, int k) { return float2(Zw[(size_t(k) * N2 + e / kTW) * R + min(r0 + e % kTW, R - 1)]); };
        auto zw_put = [&](int e, float2 z) { s_x[e] = r0 + e % kTW < R ? z : float2{0.f, 0.f}; };
        if (nsc == 1) {
            // one chunk of sampled rows: a copy, all of a thread's loads in flight together
            constexpr int E = cdiv(N2 * kTW, S::THREADS64);   // covers the smallest launch
            float2 zv[E];
#pragma unroll
            for (int u = 0; u < E; ++u) zv[u] = zw_at(min(tid + u * int(blockDim.x), N2 * kTW - 1), 0);
#pragma unroll
            for (int u = 0; u < E; ++u)
                if (tid + u * int(blockDim.x) < N2 * kTW) zw_put(tid + u * int(blockDim.x), zv[u]);
        } else {
            sum_fill<8, 1>(N2 * kTW, nsc, zw_at, zw_put);
        }
        fill_model_t(f, f.part + size_t(gAB) * slot_size(R), nsc, r0, s_T);
        __syncthreads();
        model_add<2, 4>(f.bcopy, N2, R, s_T, s_x, [](int j) { return j; });
        load_bpre();                          // B at the update's layout, arriving during the transform
        __syncthreads();
        if (s < Q && rv)
            sfor<P>([&](auto q) {
                constexpr int n1c = decltype(q)::value;
                v[n1c] = s_x[(Q * n1c + s) * kTW + c];
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
                const float2 b = bpre[k2];
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
                store_nt(f.Bhat + size_t(s + Q * m2) * R + r, cscale(v[m2], InvSqrt<N2>::value));   // read by the next step
            });
        }
    }
}

template <int N2, class Src>
__global__ void __launch_bounds__(512) k_update_b(Src src) {
    extern __shared__ float2 s_dyn[];
    __shared__ float2 s_tw[N2];
    __shared__ float2 s_x[ColShape<N2>::XSIZE];
    if (!src.live()) return;
    update_b_body<N2>(src.get(), src.bx(), s_tw, s_x, s_dyn);
}

// Both updates in one launch for square frames (they are independent: each
// uses the factors of frame t - 1): blocks [0, ga) update A, the rest B.
template <int N, class Src>
__global__ void __launch_bounds__(512) k_update_ab(Src src, int ga) {
    extern __shared__ float2 s_dyn[];
    __shared__ float2 s_tw[N];
    __shared__ float2 s_x[ColShape<N>::XSIZE];
    __shared__ double s_cp[kWeightParts];
    if (!src.live()) return;
    const DevFrame f = src.get();
    if (src.bx() < ga) update_a_body<N>(f, src.bx(), s_tw, s_x, s_cp, s_dyn);
    else update_b_body<N>(f, src.bx() - ga, s_tw, s_x, s_dyn);
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
    const int gx = cdiv(b.n2, kTW);
    const dim3 grid = frame_grid(b, gx);
    if (b.table) k_col_resid<N1, FrameTable><<<grid, S::THREADS64, 0, st>>>(FrameTable{b.table, gx, b.count});
    else k_col_resid<N1, OneFrame><<<grid, S::THREADS64, 0, st>>>(OneFrame{*b.one});
    return hipGetLastError();
}
// The update launches take whole wavefronts (the k-space gradients run on the
// matrix cores; on the k-space route at least eight of them, ColShape::KS_THREADS)
// and, on the k-space route, the gradient areas in dynamic LDS.
inline size_t update_lds(const Batch& b) { return b.kspace ? grad_lds(b.r_max, b.n1) : 0; }
// compute units of the current device (looked up once per device)
inline int device_cus() {
    static std::atomic<int> cus[16];
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 16) return 0;
    int v = cus[dev].load(std::memory_order_relaxed);
    if (v == 0) {
        if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
        cus[dev].store(v, std::memory_order_relaxed);
    }
    return v;
}
// More wavefronts per block only while the launch is one round of blocks (the
// step is then latency-bound); a larger launch keeps the smaller blocks, of
// which more share a compute unit.
template <int N> inline int update_threads(const Batch& b, const dim3& grid) {
    return b.kspace && int(grid.x) <= device_cus() ? ColShape<N>::KS_THREADS : ColShape<N>::THREADS64;
}
template <int N1> hipError_t launch_k4a_n(const Batch& b, hipStream_t st) {
    const int ga = cdiv(b.r_max, kTW);
    const size_t lds = update_lds(b);
    if (b.n1 == b.n2) {                       // both updates in one launch
        const int gx = 2 * ga;
        const dim3 grid = frame_grid(b, gx);
        const int nt = update_threads<N1>(b, grid);
        if (b.table) k_update_ab<N1, FrameTable><<<grid, nt, lds, st>>>(FrameTable{b.table, gx, b.count}, ga);
        else k_update_ab<N1, OneFrame><<<grid, nt, lds, st>>>(OneFrame{*b.one}, ga);
        return hipGetLastError();
    }
    const dim3 grid = frame_grid(b, ga);
    const int nt = update_threads<N1>(b, grid);
    if (b.table) k_update_a<N1, FrameTable><<<grid, nt, lds, st>>>(FrameTable{b.table, ga, b.count});
    else k_update_a<N1, OneFrame><<<grid, nt, lds, st>>>(OneFrame{*b.one});
    return hipGetLastError();
}
template <int N2> hipError_t launch_k4b_n(const Batch& b, hipStream_t st) {
    const int gb = cdiv(b.r_max, kTW);
    const dim3 grid = frame_grid(b, gb);
    const int nt = update_threads<N2>(b, grid);
    const size_t lds = update_lds(b);
    if (b.table) k_update_b<N2, FrameTable><<<grid, nt, lds, st>>>(FrameTable{b.table, gb, b.count});
    else k_update_b<N2, OneFrame><<<grid, nt, lds, st>>>(OneFrame{*b.one});
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
    if (b.kspace) return hipSuccess;   // frame route only
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
    if (b.n1 == b.n2) return hipSuccess;      // launched with the A update
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
