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
#include "mfma.hpp"

namespace tsl {
namespace {


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

// ---------------------------------------------------------------- matrix-core tiles
// A block of 256 threads (four wavefronts) covers ROWS frame rows.  The frame's
// complex contractions run on 16x16x4 FP32 MFMAs with the complex product split
// into real ones over a K index (rank or column, re/im).  MT x NT tiles of 16 x 16.
constexpr int kRowBlock = 256;
constexpr int kRowWaves = kRowBlock / 64;
template <int N> struct RowTiles {
    static constexpr int ROWS = RowShape<N>::ROWS;
    static constexpr int PITCH = N + 2;                 // natural [row][col] tile pitch: conflict-free 16-row reads
    static constexpr int MT = (ROWS + 15) / 16;
    static constexpr int NT = (N + 15) / 16;
    static constexpr int TPW = (MT * NT + kRowWaves - 1) / kRowWaves;   // synthesis tiles per wavefront
};
constexpr int cmax2(int a, int b) { return a > b ? a : b; }

// ---------------------------------------------------------------- K1
// X-[i][j] = sum_r AG[i][r] B[j][r] (AG = A diag(gamma)): with K = (r, re/im),
// P_re = [Re AG, -Im AG], P_im = [Im AG, Re AG] and Q = [Re B; Im B],
// Re X = P_re Q and Im X = P_im Q.  kSynRC ranks of B (all n2 rows) and of AG
// (the block's rows) are staged in LDS per pass with coalesced loads; the
// operands of the 16x16x4 steps are read from there.  The tiles land in LDS as
// [row][col] and the row transform reads its natural-layout inputs from there.
constexpr int kSynRC = 8;                  // ranks staged per pass (BF16 steps)
constexpr int kSynBP = kSynRC + 1;         // LDS pitch (float2) of a staged row
// ranks staged per pass of the FP32 steps: 16 (8 past 256 columns, so that the
// staging area stays within a quarter of the compute unit's LDS)
template <int N2> constexpr int syn_rc32() { return N2 <= 256 ? 16 : 8; }
template <int N2, class Src>
__global__ void __launch_bounds__(kRowBlock) __attribute__((amdgpu_waves_per_eu(4))) k_synth_rowfft(Src src) {
    using S = RowShape<N2>;
    using RT = RowTiles<N2>;
    constexpr int P = S::P, Q = S::Q, T = S::T, ROWS = S::ROWS, PITCH = RT::PITCH;
    constexpr int SB = N2 * kSynBP, SA = RT::MT * 16 * kSynBP;      // staged B rows, staged AG rows (BF16)
    constexpr int SB32 = N2 * (syn_rc32<N2>() + 1), SA32 = RT::MT * 16 * (syn_rc32<N2>() + 1);   // FP32 passes
    __shared__ float2 s_tw[N2];
    __shared__ float2 s_x[cmax2(cmax2(S::XSIZE, ROWS * PITCH), cmax2(SB + SA, SB32 + SA32))];

    if (!src.live()) return;
    const DevFrame f = src.get();
    if (!block_frame_ok(f.dev, true)) return;
    const int n1 = f.n1, R = f.r;
    const int tid = threadIdx.x, s = tid % T, rl = tid / T;
    const int i = src.bx() * ROWS + rl;
    const bool live = rl < ROWS && i < n1;
    // the wavefront index in a scalar register, so that tile loops branch uniformly
    // and the matrix-core steps never run under a partial exec mask
    const int lane = tid % 64, wave = __builtin_amdgcn_readfirstlane(tid / 64), m = lane % 16, g = lane / 16;
    const int i0 = src.bx() * ROWS;
    load_tw<N2>(s_tw);

    {
        float2* s_b = s_x;                  // [j][c] = B[j][r0 + c] (BF16 passes)
        float2* s_ag = s_x + SB;            // [row][c] = A[i0 + row][r0 + c] gamma[r0 + c] (BF16 passes)
        f32x4 accr[RT::TPW], acci[RT::TPW];
#pragma unroll
        for (int u = 0; u < RT::TPW; ++u) accr[u] = acci[u] = f32x4{0.f, 0.f, 0.f, 0.f};
        const int bf = __builtin_amdgcn_readfirstlane(f.synth_bf16);   // uniform: scalar branch
        static_assert(kSynRC == 8, "a BF16 step covers the 16 K entries of one pass");
        if (bf == SYN_FP32) {
            // RC ranks of B (all n2 rows) and of AG (the block's rows) are
            // staged in LDS per pass: consecutive lanes load consecutive ranks
            // of a row, so that the loads of RC lanes share one row segment (in
            // the matrix-core layout, neighbouring lanes read different rows
            // and every lane costs the L1 a tag lookup of its own; that lookup
            // rate, not the latency, bounded the direct loads).  The other
            // blocks on the compute unit cover a pass's load latency.
            // Lane (m, g) of tile (mt, nt) feeds
            // AG[16 mt + m][r] and B[16 nt + m][r], r = r0 + 4 q + g, to the
            // K step q, in Gauss's three-multiplication form:
            // P1 = sum Re AG Re B, P2 = sum Im AG Im B,
            // P3 = sum (Re AG + Im AG)(Re B + Im B), Re X = P1 - P2 and
            // Im X = P3 - P1 - P2.
            constexpr int RC = syn_rc32<N2>(), BP = RC + 1;
            constexpr int NB = cdiv(N2 * RC, kRowBlock), NA = cdiv(RT::MT * 16 * RC, kRowBlock);
            float2* s_b32 = s_x;                                     // [j][c] = B[j][r0 + c]
            float2* s_ag32 = s_x + N2 * BP;                          // [row][c] = AG[i0 + row][r0 + c]
            f32x4 p3[RT::TPW];
#pragma unroll
            for (int u = 0; u < RT::TPW; ++u) p3[u] = f32x4{0.f, 0.f, 0.f, 0.f};
            float2 rb[NB < 4 ? NB : 4], ra[NA], rg[NA];
            // B in groups of at most eight loads per thread (the registers that
            // hold a group stay few), then AG
            constexpr int GB = NB < 4 ? NB : 4;
            auto fetch_b = [&](int r0, int k0) {
#pragma unroll
                for (int k = 0; k < GB; ++k) {
                    const int e = tid + (k0 + k) * kRowBlock, j = e / RC, c = e % RC;
                    rb[k] = load_or_zero<float2>(k0 + k < NB && j < N2 && r0 + c < R, f.B + size_t(j) * R + r0 + c);
                }
            };
            auto stage_b = [&](int k0) {
#pragma unroll
                for (int k = 0; k < GB; ++k) {
                    const int e = tid + (k0 + k) * kRowBlock;
                    if (k0 + k < NB && e < N2 * RC) s_b32[(e / RC) * BP + e % RC] = rb[k];
                }
            };
            auto fetch = [&](int r0) {                               // AG: global -> registers
#pragma unroll
                for (int k = 0; k < NA; ++k) {
                    const int e = tid + k * kRowBlock, row = e / RC, c = e % RC;
                    const bool ok = row < ROWS && i0 + row < n1 && r0 + c < R;
                    ra[k] = load_or_zero<float2>(ok, f.A + size_t(i0 + row) * R + r0 + c);
                    rg[k] = load_or_zero<float2>(ok, f.gamma32 + r0 + c);
                }
            };
            auto stage = [&]() {                                     // AG: registers -> LDS
#pragma unroll
                for (int k = 0; k < NA; ++k) {
                    const int e = tid + k * kRowBlock;
                    if (e < RT::MT * 16 * RC) s_ag32[(e / RC) * BP + e % RC] = cmul(ra[k], rg[k]);
                }
            };
            auto steps = [&]() {
#pragma unroll
                for (int q = 0; q < RC / 4; ++q)
#pragma unroll
                    for (int u = 0; u < RT::TPW; ++u) {
                        const int tile = wave + kRowWaves * u;
                        if (tile >= RT::MT * RT::NT) break;
                        const int mt = tile / RT::NT, nt = tile % RT::NT, j = 16 * nt + m;
                        const float2 x = s_ag32[(16 * mt + m) * BP + 4 * q + g];
                        const float2 yb = s_b32[(j < N2 ? j : N2 - 1) * BP + 4 * q + g];   // clamped, then masked
                        const float2 y = j < N2 ? yb : float2{0.f, 0.f};
                        accr[u] = mfma_16x16x4(x.x, y.x, accr[u]);
                        acci[u] = mfma_16x16x4(x.y, y.y, acci[u]);
                        p3[u] = mfma_16x16x4(x.x + x.y, y.x + y.y, p3[u]);
                    }
            };
            for (int r0 = 0; r0 < R; r0 += RC) {
                fetch(r0);
                fetch_b(r0, 0);
                __syncthreads();                                     // the previous pass's steps are done
                stage();
                stage_b(0);
                for (int k0 = GB; k0 < NB; k0 += GB) {
                    fetch_b(r0, k0);
                    stage_b(k0);
                }
                __syncthreads();
                steps();
            }
#pragma unroll
            for (int u = 0; u < RT::TPW; ++u)
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const float q1 = accr[u][e], q2 = acci[u][e];
                    accr[u][e] = q1 - q2;
                    acci[u][e] = p3[u][e] - q1 - q2;
                }
        } else {
            for (int r0 = 0; r0 < R; r0 += kSynRC) {
                const int nr = min(kSynRC, R - r0);
                __syncthreads();
                stage_copy<8, float2>(
                    N2 * kSynRC,
                    [&](int e) {
                        const int j = e / kSynRC, c = e % kSynRC;
                        return c < nr ? float2(f.B[size_t(j) * R + r0 + c]) : float2{0.f, 0.f};
                    },
                    [&](int e, float2 v) { s_b[(e / kSynRC) * kSynBP + e % kSynRC] = v; });
                for (int e = tid; e < RT::MT * 16 * kSynRC; e += blockDim.x) {
                    const int row = e / kSynRC, c = e % kSynRC, ia = i0 + row;
                    s_ag[row * kSynBP + c] = (c < nr && row < ROWS && ia < n1)
                                                 ? cmul(float2(f.A[size_t(ia) * R + r0 + c]), float2(f.gamma32[r0 + c]))
                                                 : float2{0.f, 0.f};
                }
                __syncthreads();
                // one 16x16x16 BF16 step per pass: lane (m, g) supplies K entries
                // 4 g + e, e < 4, i.e. rank 2 g + e / 2, real part if e is even
#pragma unroll
                for (int u = 0; u < RT::TPW; ++u) {
                    const int tile = wave + kRowWaves * u;
                    if (tile >= RT::MT * RT::NT) break;
                    const int mt = tile / RT::NT, nt = tile % RT::NT, j = 16 * nt + m;
                    bf16x4 pr_h, pi_h, q_h, pr_l, pi_l, q_l;
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        const int c = 2 * g + e / 2;
                        const bool re = (e & 1) == 0;
                        const float2 a = s_ag[(16 * mt + m) * kSynBP + c];
                        const float2 b = s_b[(j < N2 ? j : N2 - 1) * kSynBP + c];
                        const float pr = re ? a.x : -a.y, pi = re ? a.y : a.x;
                        const float q = j < N2 ? (re ? b.x : b.y) : 0.f;
                        if (bf == SYN_BF16X3) {
                            const BfPair sr = split_bf16(pr), si = split_bf16(pi), sq = split_bf16(q);
                            pr_h[e] = sr.hi;
                            pr_l[e] = sr.lo;
                            pi_h[e] = si.hi;
                            pi_l[e] = si.lo;
                            q_h[e] = sq.hi;
                            q_l[e] = sq.lo;
                        } else {
                            pr_h[e] = static_cast<__bf16>(pr);
                            pi_h[e] = static_cast<__bf16>(pi);
                            q_h[e] = static_cast<__bf16>(q);
                        }
                    }
                    accr[u] = mfma_16x16x16_bf16(pr_h, q_h, accr[u]);
                    acci[u] = mfma_16x16x16_bf16(pi_h, q_h, acci[u]);
                    if (bf == SYN_BF16X3) {
                        accr[u] = mfma_16x16x16_bf16(pr_h, q_l, accr[u]);
                        acci[u] = mfma_16x16x16_bf16(pi_h, q_l, acci[u]);
                        accr[u] = mfma_16x16x16_bf16(pr_l, q_h, accr[u]);
                        acci[u] = mfma_16x16x16_bf16(pi_l, q_h, acci[u]);
                    }
                }
            }
        }
        __syncthreads();                    // staging area becomes the output tile
#pragma unroll
        for (int u = 0; u < RT::TPW; ++u) {
            const int tile = wave + kRowWaves * u;
            if (tile >= RT::MT * RT::NT) break;
            const int mt = tile / RT::NT, nt = tile % RT::NT, j = 16 * nt + m;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int row = 16 * mt + 4 * g + e;
                if (row < ROWS && j < N2) s_x[row * PITCH + j] = float2{accr[u][e], acci[u][e]};
            }
        }
    }
    __syncthreads();
    float2 v[T];
    sfor<T>([&](auto k) { v[decltype(k)::value] = float2{0.f, 0.f}; });
    if (s < Q && rl < ROWS)
        sfor<P>([&](auto q) {
            constexpr int n1c = decltype(q)::value;
            v[n1c] = s_x[rl * PITCH + Q * n1c + s];
        });
    __syncthreads();   // the row exchange below reuses s_x
    if (s < Q) dft_twiddle<N2, P, false>(v, s, s_tw);
    row_swap_nk<N2>(v, s_x, rl < ROWS ? rl : 0, rl < ROWS ? s : T);
    if (s < P && live) {
        dft_only<Q, false>(v);
        float2* out = f.frame + size_t(i) * N2;
        sfor<Q>([&](auto k) {
            constexpr int k2 = decltype(k)::value;
            out[s + P * k2] = cscale(v[k2], InvSqrt<N2>::value);
        });
    }
}

// ---------------------------------------------------------------- K3
// G_A[i][r] = sum_j Theta[i][j] conj(B[j][r]): with K = (j, re/im),
// P_re = [Re Th, Im Th], P_im = [Im Th, -Re Th] and Q = [Re B; Im B],
// Re G_A = P_re Q and Im G_A = P_im Q.  Theta sits in LDS as [row][col]; the
// wavefronts split the M tiles and, when there are fewer than four of them, the
// K range, and partial sums over K ranges are added in a fixed order.
constexpr int kGNT = 2;   // 16-rank tiles per pass
template <int N2, class Src>
__global__ void __launch_bounds__(kRowBlock) __attribute__((amdgpu_waves_per_eu(RowTiles<N2>::MT == 1 ? 4 : 3)))
k_row_inv_grad(Src src) {
    using S = RowShape<N2>;
    using RT = RowTiles<N2>;
    constexpr int P = S::P, Q = S::Q, T = S::T, ROWS = S::ROWS, PITCH = RT::PITCH, MT = RT::MT;
    constexpr int MW = MT < kRowWaves ? MT : kRowWaves;      // wavefronts across M tiles
    constexpr int KS = kRowWaves / MW;                        // ... and across K ranges
    constexpr int MPW = (MT + MW - 1) / MW;                   // M tiles per wavefront
    constexpr int KSTEPS = (N2 + 1) / 2;                      // two columns per 16x16x4 step
    constexpr int KPW = (KSTEPS + KS - 1) / KS;
    // Partial sums: [ks][row][rank] over four K ranges with several M tiles;
    // with one M tile the wavefronts take (rank tile, K half) and one half's
    // 16 x 16 tiles pass through LDS.  With one M tile the partials share the
    // twiddles' array (the transform is over before the contraction starts),
    // which keeps a block within a quarter of the compute unit's LDS.
    constexpr int SP = MT == 1 ? kGNT * 16 * 16 : KS * MT * 16 * kGNT * 16;
    constexpr int AUX = MT == 1 ? cmax2(N2, SP) : N2 + SP;
    __shared__ float2 s_aux[AUX];
    __shared__ float2 s_x[cmax2(S::XSIZE, ROWS * PITCH)];
    __shared__ int s_bad;
    float2* s_tw = s_aux;
    float2* s_p = MT == 1 ? s_aux : s_aux + N2;

    if (!src.live()) return;
    const DevFrame f = src.get();
    if (!block_frame_ok(f.dev, true)) return;
    const int n1 = f.n1, R = f.r;
    const int tid = threadIdx.x, s = tid % T, rl = tid / T;
    const int i = src.bx() * ROWS + rl;
    const bool live = rl < ROWS && i < n1;
    if (tid == 0) s_bad = 0;
    load_tw<N2>(s_tw);

    float2 v[T];
    sfor<T>([&](auto k) { v[decltype(k)::value] = float2{0.f, 0.f}; });
    if (s < Q && live) {
        const float2* in = f.frame + size_t(i) * N2;
        sfor<P>([&](auto q) { v[decltype(q)::value] = in[Q * decltype(q)::value + s]; });
    }
    __syncthreads();   // twiddles visible
    if (s < Q) dft_twiddle<N2, P, true>(v, s, s_tw);
    row_swap_nk<N2>(v, s_x, rl < ROWS ? rl : 0, rl < ROWS ? s : T);
    if (s < P) {
        dft_only<Q, true>(v);
        sfor<Q>([&](auto k) { v[decltype(k)::value] = cscale(v[decltype(k)::value], InvSqrt<N2>::value); });
    }
    __syncthreads();   // every thread is done with the exchange area
    // v[k2] = Theta[i][s + P*k2] for threads s < P: natural tile into LDS (zero rows past n1)
    if (s < P && rl < ROWS)
        sfor<Q>([&](auto k) {
            constexpr int k2 = decltype(k)::value;
            s_x[rl * PITCH + s + P * k2] = live ? v[k2] : float2{0.f, 0.f};
        });
    __syncthreads();

    const int lane = tid % 64, wave = tid / 64, m = lane % 16, g = lane / 16;
    const int mw = wave % MW, ks = wave / MW;
    const bool im = g & 1;
    bool bad = false;
    if constexpr (MT == 1) {
        // Wavefront (rank tile rs of the pass, K half kh); lane (m, g) feeds
        // Theta[m][j] and B[j][r], j = 4 t + g, to the K step t.  Gauss's
        // three-multiplication form with the conjugate's sign on B:
        // P1 = sum Re Th Re B, P2 = sum Im Th (-Im B),
        // P3 = sum (Re Th + Im Th)(Re B - Im B), so that Re G_A = P1 - P2 and
        // Im G_A = P3 - P1 - P2: three 16x16x4 steps per four columns.
        static_assert(kGNT == 2 && kRowWaves == 4, "two rank tiles by two K halves");
        const int rs = __builtin_amdgcn_readfirstlane(wave % 2), kh = __builtin_amdgcn_readfirstlane(wave / 2);
        constexpr int KS4 = (N2 + 3) / 4, KH = (KS4 + 1) / 2, KB = 8;   // K steps, per half, per load group
        const int t0 = kh * KH, t1 = min(KS4, t0 + KH);
        for (int n0 = 0; n0 < R; n0 += kGNT * 16) {
            f32x4 p1 = {0.f, 0.f, 0.f, 0.f}, p2 = p1, p3 = p1;
            const int r = n0 + 16 * rs + m;
            for (int tb = t0; tb < t1; tb += KB) {
                float2 bv[KB];
#pragma unroll
                for (int k = 0; k < KB; ++k) {
                    const int j = 4 * (tb + k) + g;
                    bv[k] = load_or_zero<float2>(tb + k < t1 && j < N2 && r < R, f.B + size_t(j) * R + r);
                }
#pragma unroll
                for (int k = 0; k < KB; ++k) {
                    const int j = 4 * (tb + k) + g;
                    const float2 th = (tb + k < t1 && m < ROWS && j < N2) ? s_x[m * PITCH + j] : float2{0.f, 0.f};
                    const float2 b = bv[k];
                    p1 = mfma_16x16x4(th.x, b.x, p1);
                    p2 = mfma_16x16x4(th.y, -b.y, p2);
                    p3 = mfma_16x16x4(th.x + th.y, b.x - b.y, p3);
                }
            }
            // D[4 g + e][m] = (row 4 g + e, rank r): the second half's tiles go
            // through LDS and are added to the first half's, in that order
            if (kh == 1)
#pragma unroll
                for (int e = 0; e < 4; ++e)
                    s_p[(rs * 16 + 4 * g + e) * 16 + m] = float2{p1[e] - p2[e], p3[e] - p1[e] - p2[e]};
            __syncthreads();
            if (kh == 0)
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int row = 4 * g + e, ii = src.bx() * ROWS + row;
                    const float2 q = s_p[(rs * 16 + row) * 16 + m];
                    const float2 gsum{(p1[e] - p2[e]) + q.x, (p3[e] - p1[e] - p2[e]) + q.y};
                    if (row < ROWS && ii < n1 && r < R) {
                        bad |= !finite2(gsum);
                        f.GA[size_t(ii) * R + r] = gsum;
                    }
                }
            __syncthreads();
        }
    } else
    for (int n0 = 0; n0 < R; n0 += kGNT * 16) {
        f32x4 accr[MPW][kGNT], acci[MPW][kGNT];
#pragma unroll
        for (int a = 0; a < MPW; ++a)
#pragma unroll
            for (int u = 0; u < kGNT; ++u) accr[a][u] = acci[a][u] = f32x4{0.f, 0.f, 0.f, 0.f};
        if (ks < KS) {
            constexpr int KB = 8;                         // steps whose B operands load together
            const int t0 = ks * KPW, t1 = min(KSTEPS, t0 + KPW);
            for (int tb = t0; tb < t1; tb += KB) {
                float bv[KB][kGNT];
#pragma unroll
                for (int k = 0; k < KB; ++k) {
                    const int j = 2 * (tb + k) + g / 2;
#pragma unroll
                    for (int u = 0; u < kGNT; ++u) {
                        const int r = n0 + 16 * u + m;
                        const bool ok = tb + k < t1 && j < N2 && r < R;
                        const float2 b = ok ? float2(f.B[size_t(j) * R + r]) : float2{0.f, 0.f};
                        bv[k][u] = im ? b.y : b.x;
                    }
                }
#pragma unroll
                for (int k = 0; k < KB; ++k) {
                    const int j = 2 * (tb + k) + g / 2;
#pragma unroll
                    for (int a = 0; a < MPW; ++a) {
                        const int mt = mw + MW * a;
                        const int row = 16 * mt + m;
                        const float2 th = (tb + k < t1 && mt < MT && row < ROWS && j < N2) ? s_x[row * PITCH + j]
                                                                                            : float2{0.f, 0.f};
                        const float pr = im ? th.y : th.x, pi = im ? -th.x : th.y;
#pragma unroll
                        for (int u = 0; u < kGNT; ++u) {
                            accr[a][u] = mfma_16x16x4(pr, bv[k][u], accr[a][u]);
                            acci[a][u] = mfma_16x16x4(pi, bv[k][u], acci[a][u]);
                        }
                    }
                }
            }
        }
        // partial sums: D[4 g + e][m] = (row 16 mt + 4 g + e, rank n0 + 16 u + m)
        if (ks < KS)
#pragma unroll
            for (int a = 0; a < MPW; ++a) {
                const int mt = mw + MW * a;
                if (mt >= MT) continue;
#pragma unroll
                for (int u = 0; u < kGNT; ++u)
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        const int row = 16 * mt + 4 * g + e;
                        s_p[(ks * MT * 16 + row) * (kGNT * 16) + 16 * u + m] = float2{accr[a][u][e], acci[a][u][e]};
                    }
            }
        __syncthreads();
        for (int e = tid; e < ROWS * kGNT * 16; e += blockDim.x) {
            const int row = e / (kGNT * 16), rr = e % (kGNT * 16), ii = src.bx() * ROWS + row;
            if (ii < n1 && n0 + rr < R) {
                float2 gsum = s_p[row * (kGNT * 16) + rr];
                for (int q = 1; q < KS; ++q) gsum = cadd(gsum, s_p[(q * MT * 16 + row) * (kGNT * 16) + rr]);
                bad |= !finite2(gsum);
                f.GA[size_t(ii) * R + n0 + rr] = gsum;
            }
        }
        __syncthreads();
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
    const int gx = cdiv(b.n1, S::ROWS);
    const dim3 grid = frame_grid(b, gx);
    if (b.table) k_synth_rowfft<N2, FrameTable><<<grid, kRowBlock, 0, st>>>(FrameTable{b.table, gx, b.count});
    else k_synth_rowfft<N2, OneFrame><<<grid, kRowBlock, 0, st>>>(OneFrame{*b.one});
    return hipGetLastError();
}
template <int N2> hipError_t launch_k3_n(const Batch& b, hipStream_t st) {
    using S = RowShape<N2>;
    const int gx = cdiv(b.n1, S::ROWS);
    const dim3 grid = frame_grid(b, gx);
    if (b.table) k_row_inv_grad<N2, FrameTable><<<grid, kRowBlock, 0, st>>>(FrameTable{b.table, gx, b.count});
    else k_row_inv_grad<N2, OneFrame><<<grid, kRowBlock, 0, st>>>(OneFrame{*b.one});
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
    if (b.kspace) return hipSuccess;   // frame route only
    switch (b.n2) {
#define TSL_X(N) case N: return launch_k1_n<N>(b, st);
        TSL_FOR_EACH_N(TSL_X)
#undef TSL_X
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_row_inv_grad(const Batch& b, hipStream_t st) {
    if (b.kspace) return hipSuccess;   // frame route only
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
