// k-space route of a line-mask step (Sec. IV-B with one coil).
//
// With the separable transform F(X) = F_l X F_r^T and the k-space factors
// Ahat = F_l A, Bhat = F_r B, the prediction at the sampled rows S is
// K_S = Ahat_S diag(gamma) Bhat^T, so the residual of Algorithm 3 on the
// samples is E = Y_S - Ahat_S diag(gamma) Bhat^T (|S| x n2).  The inverse
// transform of the zero-filled residual, Theta = F_l^H Xi conj(F_r), is the sum
// over samples of e_l times the conjugate sampling matrix, so its contractions
// with the factors reduce to the samples:
//     Theta conj(B)    = F_l^H (rows S: E conj(Bhat), zero elsewhere),
//     Theta^T conj(A)  = F_r^H (E^T conj(Ahat_S)).
// k_kres forms E, M = E conj(Bhat) (scattered to the rows of S in GA, the other
// rows zeroed) and W = E^T conj(Ahat_S) per chunk of sampled rows (in wpart);
// the A update applies F_l^H to GA (k_update_a), the B update adds the W
// partials in chunk order and applies F_r^H (k_update_b).
//
// A block (eight wavefronts) owns kKQ sampled rows and kKCols readout samples of
// one frame and runs over them in chunks of up to 128 columns (fewer at large
// ranks, so that the chunk of Bhat fits in LDS), wavefront w taking columns
// [16 w, 16 w + 16) of a chunk.  Its M covers its samples only: the block of
// samples p writes it to slab p (GA for p = 0, mpart for p >= 1) at the sampled
// rows, every slab holds 0 on the other rows, and the A update adds the slabs
// in order.  Per chunk, on FP32 matrix cores with the complex products split
// over K = (index, re/im) as in the synthesis:
//   E tile [q][j]  = y - sum_r (Ahat_S gamma)[q][r] Bhat[j][r]   (K = ranks)
//   M     [q][r] += sum_j E[q][j] conj(Bhat[j][r])               (K = the wavefront's columns)
//   W tile [j][r]  = sum_q E[q][j] conj(Ahat_S[q][r])            (K = the block's rows)
// A wavefront's E tile goes through its own LDS area (one wavefront's LDS
// accesses complete in order).  At the end the wavefronts' M sums are added
// in wavefront order.
#include <algorithm>

#include "kernels.hpp"
#include "mfma.hpp"
#include "tsl.h"

namespace tsl {
namespace {

constexpr int kKT = 512;            // threads per block (eight wavefronts)
constexpr int kKW = kKT / 64;       // wavefronts; wavefront w takes columns [16 w, 16 w + 16) of a chunk
constexpr int kEP = 17;             // LDS pitch of a wavefront's E tile (float2)
constexpr size_t kBBudget = 48 * 1024;   // LDS for the Bhat chunk
static_assert(kKQ == 16, "one matrix-core row tile of sampled rows per block");
static_assert(kKCols == 16 * kKW, "a block's samples are one chunk of all its wavefronts' tiles");

// Columns per chunk: all eight wavefronts' tiles, fewer when the Bhat chunk
// [cols][R + 1] would not fit the budget (large ranks).
inline __host__ __device__ int kres_cols(int R) {
    const int fit = int(kBBudget / (size_t(R + 1) * sizeof(float2))) / 16 * 16;
    return fit < 16 * kKW ? fit : 16 * kKW;
}
constexpr int kYL = kKQ * 16 * kKW / kKT;                   // sample loads per thread

// Dynamic LDS: s_b [cols][R + 1] (Bhat chunk; at the end the wavefronts' M
// sums [kKW][16][R]), s_a [16][R + 1] (Ahat rows), s_e [kKW][16][kEP] (E tiles).
size_t kres_lds(int R) {
    return (size_t(kres_cols(R)) * (R + 1) + size_t(kKQ) * (R + 1) + size_t(kKW) * 16 * kEP) * sizeof(float2);
}

template <int RT, class Src>
__global__ void __launch_bounds__(kKT) k_kres(Src src, int nblk) {
    extern __shared__ float2 s_dyn[];
    __shared__ float2 s_g[TSL_MAX_R];
    __shared__ int s_row[kKQ];
    __shared__ unsigned char s_on[kMaxN];
    __shared__ int s_bad;
    if (!src.live()) return;
    const DevFrame f = src.get();
    const int n1 = f.n1, n2 = f.n2, R = f.r, tid = threadIdx.x, RP = R + 1;
    const int JC = kres_cols(R);
    float2* s_b = s_dyn;
    float2* s_a = s_b + JC * RP;
    float2* s_e = s_a + kKQ * RP;
    const int lane = tid % 64, wave = __builtin_amdgcn_readfirstlane(tid / 64);
    const int m = lane % 16, g4 = lane / 16;
    const int ncp = n_cparts(n2), bx = src.bx(), qc = bx / ncp, cp = bx % ncp, q0 = qc * kKQ;
    const int c0 = cp * kKCols, c1 = min(n2, c0 + kKCols);   // the block's samples
    // Loads that need nothing but the descriptor go out before the status check
    // (all inside the frame's own buffers): the row count, the row list, gamma
    // and the first round of the first chunk of Bhat.
    const int cap = frame_rows_cap(f);
    const int nd = f.n_rows_dev ? *f.n_rows_dev : cap;
    const int row_mine = (tid < kKQ && q0 + tid < cap) ? f.rows[q0 + tid] : -1;
    const int row_list = tid < cap ? f.rows[tid] : -1;
    const float2 gam = tid < R ? float2(f.gamma32[tid]) : float2{0.f, 0.f};
    // (staging loads read at indices clamped into range and select the values
    // past it away, so that they go out back to back with no branch between)
    float2 b0[4];
    const int nb0 = min(JC, c1 - c0) * R;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const int e = tid + u * kKT;
        const float2 v = f.Bhat[size_t(c0) * R + min(e, nb0 - 1)];
        b0[u] = e < nb0 ? v : float2{0.f, 0.f};
    }
    for (int i = tid; i < n1; i += kKT) s_on[i] = 0;
    if (tid == 0) s_bad = 0;
    if (!block_frame_ok(f.dev, true)) return;        // its barriers also order the resets above
    const int S = nd < 0 ? 0 : (nd > cap ? cap : nd);
    const int nq = max(0, min(kKQ, S - q0));
    if (tid < R) s_g[tid] = gam;
    for (int r = tid + kKT; r < R; r += kKT) s_g[r] = f.gamma32[r];
    if (tid < kKQ) s_row[tid] = (tid < nq && row_mine >= 0 && row_mine < n1) ? row_mine : -1;
    if (tid < S && row_list >= 0 && row_list < n1) s_on[row_list] = 1;
    for (int q = tid + kKT; q < S; q += kKT) {
        const int row = f.rows[q];
        if (row >= 0 && row < n1) s_on[row] = 1;
    }
    __syncthreads();
    // Ahat rows of the block
    for (int e = tid; e < kKQ * R; e += kKT) {
        const int q = e / R, c = e % R, row = s_row[q];
        const float2 v = f.Ahat[size_t(max(row, 0)) * R + c];
        s_a[q * RP + c] = row >= 0 ? v : float2{0.f, 0.f};
    }
    // rows that this block zeroes in every slab: the unsampled rows i with i mod nblk = bx
    const int nown = bx < n1 ? cdiv(n1 - bx, nblk) : 0;
    for (int e = tid; e < nown * R; e += kKT) {
        const int i = bx + (e / R) * nblk;
        if (!s_on[i]) {
            f.GA[size_t(i) * R + e % R] = float2{0.f, 0.f};
            for (int p = 1; p < ncp; ++p) f.mpart[(size_t(p) * n1 + i) * R + e % R] = float2{0.f, 0.f};
        }
    }
    if (nq == 0) return;                             // uniform

    bool bad = false;
    f32x4 mr[RT], mi[RT];
#pragma unroll
    for (int t = 0; t < RT; ++t) mr[t] = mi[t] = f32x4{0.f, 0.f, 0.f, 0.f};
    float2* s_ew = s_e + wave * 16 * kEP;            // this wavefront's E tile [q][j]
    for (int j0 = c0; j0 < c1; j0 += JC) {
        const int njc = min(JC, c1 - j0), nbc = njc * R;   // columns and Bhat entries of the chunk
        __syncthreads();                             // the previous chunk's reads of s_b are done
        {   // the samples and the chunk of Bhat, four loads per thread in flight per round
            float2 yv[kYL];
#pragma unroll
            for (int u = 0; u < kYL; ++u) {
                const int e = tid + u * kKT, q = e / (16 * kKW), j = e % (16 * kKW), row = s_row[q];
                // a row that is not live reads the block's first row (q0 < S here)
                const float2 v = line_samples(f, q0 + (row >= 0 ? q : 0), max(row, 0))[j0 + min(j, njc - 1)];
                yv[u] = (row >= 0 && j < njc) ? v : float2{0.f, 0.f};
            }
            for (int e0 = 0; e0 < JC * R; e0 += 4 * kKT) {
                float2 bv[4];
                if (j0 == c0 && e0 == 0) {
#pragma unroll
                    for (int u = 0; u < 4; ++u) bv[u] = b0[u];
                } else {
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        const int e = e0 + tid + u * kKT;
                        const float2 v = f.Bhat[size_t(j0) * R + min(e, nbc - 1)];
                        bv[u] = e < nbc ? v : float2{0.f, 0.f};
                    }
                }
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const int e = e0 + tid + u * kKT;
                    if (e < JC * R) s_b[(e / R) * RP + e % R] = bv[u];
                }
            }
            // samples, to the wavefront that owns their columns
#pragma unroll
            for (int u = 0; u < kYL; ++u) {
                const int e = tid + u * kKT, q = e / (16 * kKW), j = e % (16 * kKW);
                s_e[(j / 16) * 16 * kEP + q * kEP + j % 16] = yv[u];
            }
        }
        __syncthreads();
        const int jt0 = j0 + 16 * wave;              // first column of this wavefront's tile
        if (16 * wave < JC && jt0 < c1) {            // uniform
            // E tile: prediction on the matrix cores in Gauss's three-product form
            // (lane K entry g4 takes rank 4 k + g4: P1 = sum ag.x b.x, P2 = sum
            // ag.y b.y, P3 = sum (ag.x + ag.y)(b.x + b.y), Re = P1 - P2,
            // Im = P3 - P1 - P2), then y - prediction
            f32x4 p1{0.f, 0.f, 0.f, 0.f}, p2{0.f, 0.f, 0.f, 0.f}, p3{0.f, 0.f, 0.f, 0.f};
#pragma unroll 2
            for (int k = 0; k < cdiv(R, 4); ++k) {
                const int c = min(4 * k + g4, R - 1);
                const bool cv = 4 * k + g4 < R;
                const float2 a = s_a[m * RP + c], gm = s_g[c];
                const float2 ag = cv ? cmul(a, gm) : float2{0.f, 0.f};
                const float2 b = s_b[(16 * wave + m) * RP + c];
                p1 = mfma_16x16x4(ag.x, b.x, p1);
                p2 = mfma_16x16x4(ag.y, b.y, p2);
                p3 = mfma_16x16x4(ag.x + ag.y, b.x + b.y, p3);
            }
            f32x4 er, ei;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                er[i] = p1[i] - p2[i];
                ei[i] = p3[i] - p1[i] - p2[i];
            }
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int q = 4 * g4 + i, j = m;
                const float2 yq = s_ew[q * kEP + j];
                const bool live = q < nq && jt0 + j < c1;
                const float2 e = live ? float2{yq.x - er[i], yq.y - ei[i]} : float2{0.f, 0.f};
                bad |= live && !finite2(yq);
                s_ew[q * kEP + j] = e;
            }
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            // M += E conj(Bhat) over the tile's columns; W tile = E^T conj(Ahat_S);
            // up to rank 32 both in the three-product form with the conjugate's
            // sign on the factor (lane K entry g4 takes tile column or sample 4 k + g4)
#pragma unroll
            for (int t = 0; t < RT; ++t) {
                if (16 * t >= R) break;              // uniform
                const int rc = min(16 * t + m, R - 1);
                const bool rv = 16 * t + m < R;
                f32x4 wr, wi;
                if constexpr (RT <= 2) {
                    f32x4 m1{0.f, 0.f, 0.f, 0.f}, m2{0.f, 0.f, 0.f, 0.f};
                    f32x4 w1{0.f, 0.f, 0.f, 0.f}, w2{0.f, 0.f, 0.f, 0.f}, w3{0.f, 0.f, 0.f, 0.f};
#pragma unroll 2
                    for (int k = 0; k < 4; ++k) {
                        const int kk = 4 * k + g4;
                        const float2 em = s_ew[m * kEP + kk];         // E[q = m][j = kk]
                        const float2 et = s_ew[kk * kEP + m];         // E[q = kk][j = m]
                        const float2 bl = s_b[(16 * wave + kk) * RP + rc];
                        const float2 al = s_a[kk * RP + rc];
                        const float2 b = rv ? float2{bl.x, -bl.y} : float2{0.f, 0.f};   // conj(Bhat)
                        const float2 a = rv ? float2{al.x, -al.y} : float2{0.f, 0.f};   // conj(Ahat)
                        m1 = mfma_16x16x4(em.x, b.x, m1);
                        m2 = mfma_16x16x4(em.y, b.y, m2);
                        mi[t] = mfma_16x16x4(em.x + em.y, b.x + b.y, mi[t]);
                        w1 = mfma_16x16x4(et.x, a.x, w1);
                        w2 = mfma_16x16x4(et.y, a.y, w2);
                        w3 = mfma_16x16x4(et.x + et.y, a.x + a.y, w3);
                    }
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        mr[t][i] += m1[i] - m2[i];
                        mi[t][i] -= m1[i] + m2[i];
                        wr[i] = w1[i] - w2[i];
                        wi[i] = w3[i] - w1[i] - w2[i];
                    }
                } else {
                    // wider ranks keep the four-product form, which needs fewer
                    // registers (two blocks per compute unit)
                    const bool pim = g4 & 1;             // which part this lane's K entry takes
                    wr = wi = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll 2
                    for (int k = 0; k < 8; ++k) {
                        const int kk = 2 * k + g4 / 2;
                        const float2 em = s_ew[m * kEP + kk];     // E[q = m][j = kk]
                        const float2 et = s_ew[kk * kEP + m];     // E[q = kk][j = m]
                        const float2 b = s_b[(16 * wave + kk) * RP + rc];
                        const float2 a = s_a[kk * RP + rc];
                        const float bq = rv ? (pim ? b.y : b.x) : 0.f;
                        const float aq = rv ? (pim ? a.y : a.x) : 0.f;
                        mr[t] = mfma_16x16x4(pim ? em.y : em.x, bq, mr[t]);   // Re: er br + ei bi
                        mi[t] = mfma_16x16x4(pim ? -em.x : em.y, bq, mi[t]);  // Im: ei br - er bi
                        wr = mfma_16x16x4(pim ? et.y : et.x, aq, wr);
                        wi = mfma_16x16x4(pim ? -et.x : et.y, aq, wi);
                    }
                }
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int j = jt0 + 4 * g4 + i, r = 16 * t + m;
                    if (j < n2 && r < R) {
                        const float2 w{wr[i], wi[i]};
                        bad |= !finite2(w);
                        f.wpart[(size_t(qc) * n2 + j) * R + r] = w;
                    }
                }
            }
        }
    }
    // the wavefronts' M sums meet in LDS (over the Bhat chunk) and are added in order
    const int nw = min(kKW, cdiv(min(JC, c1 - c0), 16));   // wavefronts that took columns
    __syncthreads();
    float2* s_m = s_b;                               // [wave][q][r]
    if (wave < nw) {
#pragma unroll
        for (int t = 0; t < RT; ++t) {
            if (16 * t >= R) break;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int q = 4 * g4 + i, r = 16 * t + m;
                if (r < R) s_m[(wave * kKQ + q) * R + r] = float2{mr[t][i], mi[t][i]};
            }
        }
    }
    __syncthreads();
    const GlobalPtr<float2> slab = cp == 0 ? f.GA : f.mpart + size_t(cp) * n1 * R;
    for (int e = tid; e < nq * R; e += kKT) {
        const int q = e / R, r = e % R, row = s_row[q];
        float2 acc = s_m[q * R + r];
        for (int w = 1; w < nw; ++w) acc = cadd(acc, s_m[(w * kKQ + q) * R + r]);
        bad |= !finite2(acc);
        if (row >= 0) slab[size_t(row) * R + r] = acc;
    }
    if (bad) s_bad = 1;
    __syncthreads();
    if (tid == 0 && s_bad) latch(f.dev, ST_ENONFINITE);
}

}  // namespace

void kres_attributes() {
    const int ms = int(kres_lds(TSL_MAX_R));
    auto set = [&](const void* k) { hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, ms); };
    set(reinterpret_cast<const void*>(&k_kres<2, FrameTable>));
    set(reinterpret_cast<const void*>(&k_kres<2, OneFrame>));
    set(reinterpret_cast<const void*>(&k_kres<4, FrameTable>));
    set(reinterpret_cast<const void*>(&k_kres<4, OneFrame>));
    set(reinterpret_cast<const void*>(&k_kres<8, FrameTable>));
    set(reinterpret_cast<const void*>(&k_kres<8, OneFrame>));
}

template <int RT> void launch_kres_rt(const Batch& b, hipStream_t st) {
    const int gx = std::max(1, n_qparts(b.rows_max)) * n_cparts(b.n2);
    const dim3 grid = frame_grid(b, gx);
    const size_t lds = kres_lds(b.r_max);
    if (b.table) k_kres<RT, FrameTable><<<grid, kKT, lds, st>>>(FrameTable{b.table, gx, b.count}, gx);
    else k_kres<RT, OneFrame><<<grid, kKT, lds, st>>>(OneFrame{*b.one}, gx);
}

hipError_t launch_kres(const Batch& b, hipStream_t st) {
    if (!b.kspace) return hipSuccess;             // k-space route only
    if (b.r_max <= 32) launch_kres_rt<2>(b, st);
    else if (b.r_max <= 64) launch_kres_rt<4>(b, st);
    else launch_kres_rt<8>(b, st);
    return hipGetLastError();
}

}  // namespace tsl
