// Kernels that are not templated on a transform length.
//
//  k_stats      FP64 partial statistics of S1 (Sec. III-A) for one frame.  With a
//               line mask S the regression matrix of Algorithm 3 (one coil) is
//               [Phi]_{(i,j),r} = (F_l a_r)_i (F_r b_r)_j, so its Gram is the
//               Hadamard product (Ahat_S^H Ahat_S) .* (Bhat^H Bhat) and
//               Phi^H y = sum_{i in S} conj(Ahat_i) .* (y_i conj(Bhat)); with a
//               point mask both are summed entry by entry.  Partials cover row
//               chunks and are reduced in a fixed order by the solve.  On the
//               k-space route the same launch also leaves the data terms of the
//               residual's two gradient contractions, Y_S conj(Bhat) and
//               Y_S^T conj(Ahat_S) (partials per chunk, from the operands it has
//               staged anyway), and copies of Bhat and of the sampled rows of
//               Ahat for the update (k_col.hip), which overwrites both.
//  k_solve      G = Phi^H Phi + lambda I, Cholesky, gamma_t = G^{-1} Phi^H y (the
//               closed form of the ridge problem), the step size alpha_t of the
//               majorizer (Sec. III-A; Gershgorin bound of diag(g)^H A^H A diag(g)
//               and of the B analogue, plus lambda/t), alpha_bar_t and mu_t (eq. 6).
//  k_synth_out  X_t = A[t] diag(gamma_t) B[t]^T (Sec. IV-A).
//  k_sample     Algorithm 4 on rows with the score of Sec. VI-C (sampler.hpp).
#include "fft_engine.hpp"
#include "kernels.hpp"
#include "mfma.hpp"
#include "sampler.hpp"
#include "tsl.h"

#include <mutex>

namespace tsl {
namespace {

__device__ __forceinline__ void dacc_cj(double2& acc, float2 a, float2 b) {   // acc += conj(a) b
    const double ar = a.x, ai = a.y, br = b.x, bi = b.y;
    acc.x += ar * br + ai * bi;
    acc.y += ar * bi - ai * br;
}
__device__ __forceinline__ double2 dcmul(double2 a, double2 b) {
    return double2{a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
__device__ __forceinline__ double2 dcmulc(double2 a, double2 b) {   // a conj(b)
    return double2{a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y};
}
__device__ __forceinline__ double dabs(double2 a) { return sqrt(a.x * a.x + a.y * a.y); }

// Cholesky pivot of a positive d: ip = 1/sqrt(d) from the hardware estimate and
// two Newton steps y <- y + (y/2)(1 - d y^2) (each roughly doubles the correct
// bits), and p = d ip = sqrt(d).  Eight dependent operations instead of a
// square root followed by a division, on the solve's serial path.
__device__ __forceinline__ void pivot(double d, double& p, double& ip) {
    double y = __builtin_amdgcn_rsq(d);
#pragma unroll
    for (int it = 0; it < 2; ++it) {
        const double e = fma(-d * y, y, 1.0);
        y = fma(0.5 * y, e, y);
    }
    ip = y;
    p = d * y;
}

// ---------------------------------------------------------------- Gram statistics
// Blocks of kSB threads.  A Gram is accumulated from rows staged in LDS as FP64
// (products of FP32 values are exact there).  Every block writes its own
// partial slot and the solve sums the slots in slot order, so the result does
// not depend on block scheduling.
constexpr int kSB = 256;
static_assert(kJCH >= kSRows, "the rhs products reuse the readout-chunk staging area");

// Upper entries (r <= s) of sum_q conj(x_qr) x_qs over the nq rows of s_x ([nq][R],
// complex64 or complex128, widened when read) on FP64 matrix cores, three
// 16x16x4 steps per four rows (below); the wavefronts take the 16 x 16 tiles on
// and above the diagonal.
__device__ __forceinline__ double2 widen(float2 v) { return double2{v.x, v.y}; }
__device__ __forceinline__ double2 widen(double2 v) { return v; }
template <class T>
__device__ void gram_staged(const T* s_x, int nq, int R, double2* out) {
    // wavefront index in a scalar register: uniform tile loops, full exec masks
    // around the matrix-core steps; operands are read at clamped indices and
    // masked.  Gauss's three-multiplication form over K = four rows per step:
    // with a = conj(x_r), b = x_s, P1 = sum ar br, P2 = sum ai bi,
    // P3 = sum (ar + ai)(br + bi), Re = P1 - P2 and Im = P3 - P1 - P2.
    const int lane = threadIdx.x % 64, wave = __builtin_amdgcn_readfirstlane(threadIdx.x / 64), nw = blockDim.x / 64;
    const int m = lane % 16, g = lane / 16;
    const int TM = (R + 15) / 16, ntiles = TM * (TM + 1) / 2;
    for (int tile = wave; tile < ntiles; tile += nw) {
        int mi = 0, t = tile;
        while (t >= TM - mi) { t -= TM - mi; ++mi; }
        const int ni = mi + t;
        const int ra = 16 * mi + m, sb = 16 * ni + m;
        f64x4 p1 = {0.0, 0.0, 0.0, 0.0}, p2 = {0.0, 0.0, 0.0, 0.0}, p3 = {0.0, 0.0, 0.0, 0.0};
        for (int q0 = 0; q0 < nq; q0 += 4) {
            const int q = q0 + g, qc = min(q, nq - 1);
            const double2 xa0 = widen(s_x[qc * R + min(ra, R - 1)]), xb0 = widen(s_x[qc * R + min(sb, R - 1)]);
            const double2 xa = (q < nq && ra < R) ? xa0 : double2{0.0, 0.0};
            const double2 xb = (q < nq && sb < R) ? xb0 : double2{0.0, 0.0};
            p1 = mfma_16x16x4_f64(xa.x, xb.x, p1);
            p2 = mfma_16x16x4_f64(-xa.y, xb.y, p2);
            p3 = mfma_16x16x4_f64(xa.x - xa.y, xb.x + xb.y, p3);
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int rr = 16 * mi + 4 * i + g, ss = 16 * ni + m;
            if (rr < R && ss < R && rr <= ss) out[upk(rr, ss, R)] = double2{p1[i] - p2[i], p3[i] - p1[i] - p2[i]};
        }
    }
}

// Factor-Gram block b: rows [kGRows b, kGRows (b+1)) of F_l A for b < n_gparts(n1),
// else the corresponding rows of F_r B; the partial goes to slot b.
// With check, the frame's status is read after the first round of loads is in
// flight (the loads stay inside the factor either way).
__device__ void factor_gram_block(const DevFrame& f, int b, float2* s_x, bool check) {
    const int gA = n_gparts(f.n1), R = f.r;
    const bool isA = b < gA;
    const int n = isA ? f.n1 : f.n2, q0 = (isA ? b : b - gA) * kGRows, nq = min(kGRows, n - q0);
    GlobalPtr<const float2> X = (isA ? f.Ahat : f.Bhat) + size_t(q0) * R;
    constexpr int kFL = 8;
    const int ne = nq * R;
    for (int e0 = 0; e0 < ne; e0 += kFL * kSB) {
        float2 v[kFL];
#pragma unroll
        for (int u = 0; u < kFL; ++u)     // clamped index: no branch between the loads
            v[u] = float2(X[min(e0 + int(threadIdx.x) + u * kSB, ne - 1)]);
        if (e0 == 0 && check && !block_frame_ok(f.dev, false)) return;   // uniform
        const bool keep = !isA && f.kspace;      // the k-space update reads Bhat of frame t - 1 from the copy
#pragma unroll
        for (int u = 0; u < kFL; ++u) {
            const int e = e0 + int(threadIdx.x) + u * kSB;
            if (e < ne) {
                s_x[e] = v[u];
                if (keep) store_nt(f.bcopy + size_t(q0) * R + e, v[u]);
            }
        }
    }
    __syncthreads();
    gram_staged(s_x, nq, R, f.part + size_t(b) * slot_size(R));
}

// Line masks, one launch for all of S1's statistics.  Blocks [0, gAB) are the
// factor-Gram partials (gAB = n_gparts(n1) + n_gparts(n2)); block gAB + k nJ + c
// gAB + k (k < nsg, the launch's chunks of kSRows sampled rows) validates the
// rows [kSRows k, kSRows (k+1)) of the row list and writes the Gram of those rows
// of F_l A to slot gAB + k; block gAB + nsg + k nJ + c writes the right-hand-side
// partial h_r = sum_q conj(Ahat_{row_q, r}) sum_j y_qj conj(Bhat_jr) over the same
// rows and readout samples [kJCH c, kJCH (c+1)) (Phi^H y restricted to the
// block's samples) to hpart[k nJ + c].  (A block doing both kept the launch
// waiting on its Gram.)
// RT: rank tiles of 16 the readout products are sized for (R <= 16 RT).
template <int RT, class Src>
__global__ void __launch_bounds__(kSB) k_lstats(Src src, int nsg) {
    extern __shared__ double2 s_dyn[];
    __shared__ int s_err;
    __shared__ int s_row[kSRows];
    if (!src.live()) return;
    const DevFrame f = src.get();
    const int n1 = f.n1, n2 = f.n2, R = f.r, tid = threadIdx.x;
    const int gAB = n_gparts(n1) + n_gparts(n2);
    if (src.bx() < gAB) {
        factor_gram_block(f, src.bx(), reinterpret_cast<float2*>(s_dyn), true);
        return;
    }
    const int nJ = n_jparts(n2);
    const bool gram_role = src.bx() < gAB + nsg;    // the Gram of one chunk of sampled rows
    const int k = gram_role ? src.bx() - gAB : (src.bx() - gAB - nsg) / nJ;
    const int c = gram_role ? 0 : (src.bx() - gAB - nsg) % nJ;
    const int q0 = k * kSRows;
    const int j0 = c * kJCH, nj = gram_role ? 0 : min(kJCH, n2 - j0);
    // Loads that need nothing but the descriptor go out before the status check
    // (inside the frame's own buffers): the row count, the block's row indices
    // (and each next one, for the ascending check) and the first round of the
    // readout chunk of F_r B.
    const int cap = frame_rows_cap(f);
    const int nd = f.n_rows_dev ? *f.n_rows_dev : cap;
    const int row_raw = (tid < kSRows && q0 + tid < cap) ? f.rows[q0 + tid] : -1;
    const int next_raw = (gram_role && tid < kSRows && q0 + tid + 1 < cap) ? f.rows[q0 + tid + 1] : -1;
    // Every staging load reads a valid address (indices clamped into range) and
    // only the LDS store is predicated, so the loads of a round go out back to
    // back; kLU loads per thread per round.
    constexpr int kLU = 4;
    const int nb = nj * R;
    float2 bv[kLU];
    auto load_b = [&](int e0) {
#pragma unroll
        for (int u = 0; u < kLU; ++u) bv[u] = float2(f.Bhat[size_t(j0) * R + min(e0 + tid + u * kSB, nb - 1)]);
    };
    if (!gram_role) load_b(0);
    if (tid == 0) s_err = 0;
    if (!block_frame_ok(f.dev, false)) return;      // its barriers also order s_err's reset
    const int n_rows = nd < 0 ? 0 : (nd > cap ? cap : nd);
    if (k == 0 && gram_role && tid == 0 && f.n_rows_dev && (nd < 0 || nd > cap)) latch(f.dev, ST_EINVAL);
    if (q0 >= n_rows) return;
    const int nq = min(n_rows, q0 + kSRows) - q0;
    float2* s_x = reinterpret_cast<float2*>(s_dyn);   // [kSRows][R]  sampled rows of F_l A (complex64)
    // the readout chunk of F_r B and the samples stay complex64 in LDS (widened
    // when read), which keeps a block at 32 KiB at R = 32
    float2* s_b = s_x + kSRows * R;                               // [kJCH][R]
    float2* s_y = s_b + kJCH * R;                                 // [kSRows][kJCH]
    for (int e0 = 0; e0 < nb;) {
#pragma unroll
        for (int u = 0; u < kLU; ++u) {
            const int e = e0 + tid + u * kSB;
            if (e < nb) s_b[e] = bv[u];
        }
        e0 += kLU * kSB;
        if (e0 >= nb) break;
        load_b(e0);
    }
    // Then the sampled rows of F_l A and their samples, once the row indices
    // are in LDS.
    const int nx = nq * R, ny = gram_role ? 0 : nq * kJCH;
    if (tid < nq) {                           // rows inside [0, n1), strictly ascending
        const int q = q0 + tid, row = row_raw;
        bool ok = row >= 0 && row < n1;
        if (gram_role) {
            if (q + 1 < n_rows) ok = ok && next_raw > row;
            if (!ok) atomicCAS(&s_err, 0, ST_EINVAL);
        }
        s_row[tid] = (row >= 0 && row < n1) ? row : -1;
    }
    __syncthreads();
    bool fin = true;
    for (int e0 = 0; e0 < max(nx, ny); e0 += kLU * kSB) {
        float2 xv[kLU], yv[kLU];
        int xr[kLU], yr[kLU];
#pragma unroll
        for (int u = 0; u < kLU; ++u) {
            const int ex = min(e0 + tid + u * kSB, nx - 1);
            xr[u] = s_row[ex / R];
            xv[u] = float2(f.Ahat[size_t(max(xr[u], 0)) * R + ex % R]);
            if (!gram_role) {                 // uniform; the Gram role stages no samples (ny = 0)
                const int ey = min(e0 + tid + u * kSB, ny - 1);
                const int q = ey / kJCH, jj = min(ey % kJCH, nj - 1);
                yr[u] = s_row[q];
                yv[u] = float2(line_samples(f, q0 + q, max(yr[u], 0))[j0 + jj]);
            }
        }
#pragma unroll
        for (int u = 0; u < kLU; ++u) {
            const int e = e0 + tid + u * kSB;
            if (e < nx) {
                const float2 x = xr[u] >= 0 ? xv[u] : float2{0.f, 0.f};
                s_x[e] = x;
                if (gram_role && f.kspace) store_nt(f.acopy + size_t(q0) * R + e, x);   // Ahat_S of frame t - 1
            }
            if (e < ny) {
                const bool live = yr[u] >= 0 && e % kJCH < nj;
                const float2 y = live ? yv[u] : float2{0.f, 0.f};
                fin = fin && finite2(y);
                s_y[e] = y;
            }
        }
    }
    __syncthreads();
    if (gram_role) {
        gram_staged(s_x, nq, R, f.part + size_t(gAB + k) * slot_size(R));
    } else {
    // z[q][r] = sum_j y_qj conj(Bhat_jr) over the chunk on FP64 matrix cores
    // (M = the sampled rows, N = ranks, K = four samples per step) in Gauss's
    // three-multiplication form: P1 = sum yr br, P2 = sum yi (-bi),
    // P3 = sum (yr + yi)(br - bi), Re z = P1 - P2, Im z = P3 - P1 - P2.
    const int lane = tid % 64, wave = __builtin_amdgcn_readfirstlane(tid / 64), m = lane % 16, g = lane / 16;
    const int TMq = (nq + 15) / 16, TMr = (R + 15) / 16, nzt = TMq * TMr;
    constexpr int kZT = ((kSRows + 15) / 16 * RT + kSB / 64 - 1) / (kSB / 64);
    f64x4 zp1[kZT], zp2[kZT], zp3[kZT];
#pragma unroll
    for (int u = 0; u < kZT; ++u) zp1[u] = zp2[u] = zp3[u] = f64x4{0.0, 0.0, 0.0, 0.0};
    for (int j0 = 0; j0 < nj; j0 += 4) {
        const int j = j0 + g;
#pragma unroll
        for (int u = 0; u < kZT; ++u) {
            const int tile = wave + (kSB / 64) * u;
            if (tile >= nzt) break;
            const int q = 16 * (tile / TMr) + m, r = 16 * (tile % TMr) + m, jc = min(j, nj - 1);
            const float2 yf = s_y[min(q, nq - 1) * kJCH + jc], bf = s_b[jc * R + min(r, R - 1)];
            const double2 yv0{yf.x, yf.y}, bv0{bf.x, bf.y};
            const double2 yv = (q < nq && j < nj) ? yv0 : double2{0.0, 0.0};
            const double2 bv = (r < R && j < nj) ? bv0 : double2{0.0, 0.0};
            zp1[u] = mfma_16x16x4_f64(yv.x, bv.x, zp1[u]);
            zp2[u] = mfma_16x16x4_f64(yv.y, -bv.y, zp2[u]);
            zp3[u] = mfma_16x16x4_f64(yv.x + yv.y, bv.x - bv.y, zp3[u]);
        }
    }
    if (f.kspace) {
        // k-space route: zw[j][r] = sum_q y_qj conj(Ahat_{row_q, r}) over the
        // block's rows and samples, the chunk's share of Y_S^T conj(Ahat_S), on
        // the FP32 matrix cores (M = samples, N = ranks, K = four rows per step;
        // three-product form with the conjugate's sign on the factor)
        const int TMj = (nj + 15) / 16, nwt = TMj * TMr;
        for (int tile = wave; tile < nwt; tile += kSB / 64) {
            const int tj = tile / TMr, tr = tile % TMr, jj = 16 * tj + m, rr = 16 * tr + m;
            f32x4 w1{0.f, 0.f, 0.f, 0.f}, w2{0.f, 0.f, 0.f, 0.f}, w3{0.f, 0.f, 0.f, 0.f};
            for (int q4 = 0; q4 < nq; q4 += 4) {
                const int q = q4 + g, qc = min(q, nq - 1);
                const float2 yf = s_y[qc * kJCH + min(jj, kJCH - 1)], af = s_x[qc * R + min(rr, R - 1)];
                const bool yok = q < nq && jj < nj, aok = q < nq && rr < R;
                const float yr = yok ? yf.x : 0.f, yi = yok ? yf.y : 0.f;
                const float ar = aok ? af.x : 0.f, ai = aok ? -af.y : 0.f;
                w1 = mfma_16x16x4(yr, ar, w1);
                w2 = mfma_16x16x4(yi, ai, w2);
                w3 = mfma_16x16x4(yr + yi, ar + ai, w3);
            }
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int j = 16 * tj + 4 * g + i, r = 16 * tr + m;
                if (j < nj && r < R) store_nt(f.zw + (size_t(k) * n2 + j0 + j) * R + r, float2{w1[i] - w2[i], w3[i] - w1[i] - w2[i]});
            }
        }
    }
    __syncthreads();                          // s_b and s_y are reused for the products below
    double2* s_p = reinterpret_cast<double2*>(s_b);   // [nq][R]: z[q][r] conj(Ahat_{row_q, r})
#pragma unroll
    for (int u = 0; u < kZT; ++u) {
        const int tile = wave + (kSB / 64) * u;
        if (tile >= nzt) break;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int q = 16 * (tile / TMr) + 4 * i + g, r = 16 * (tile % TMr) + m;
            const double2 z{zp1[u][i] - zp2[u][i], zp3[u][i] - zp1[u][i] - zp2[u][i]};
            if (q < nq && r < R) {
                s_p[q * R + r] = dcmulc(z, widen(s_x[q * R + r]));
                if (f.kspace) store_nt(f.zm + ((size_t(k) * nJ + c) * kSRows + q) * R + r, float2{float(z.x), float(z.y)});
            }
        }
    }
    __syncthreads();
    if (tid < R) {
        double2 h{0.0, 0.0};
        for (int q = 0; q < nq; ++q) { h.x += s_p[q * R + tid].x; h.y += s_p[q * R + tid].y; }
        f.hpart[size_t(k * nJ + c) * R + tid] = h;
    }
    }
    if (!fin) atomicCAS(&s_err, 0, ST_ENONFINITE);
    __syncthreads();
    if (tid == 0 && s_err) latch(f.dev, s_err);
}

// a factor-Gram block, or a sampled block: rows of F_l A (FP64), then the
// complex64 chunk of F_r B and samples, later overlaid by the FP64 products
// (Factor rows and sampled rows are staged as complex64 and widened when read:
// at R = 32 a block then takes 24 KiB, so six share a compute unit and a full
// batch of statistics blocks goes out in one round.)
size_t lstats_lds(int R) {
    const size_t gram = size_t(kGRows) * R * sizeof(float2);
    const size_t staged = size_t(kJCH * R + kSRows * kJCH) * sizeof(float2);
    const size_t prod = size_t(kSRows) * R * sizeof(double2);
    const size_t samp = size_t(kSRows) * R * sizeof(float2) + (staged > prod ? staged : prod);
    return gram > samp ? gram : samp;
}

constexpr int kPW = 32;        // sampled entries staged per window of a point-mask Gram
constexpr int kMaxAcc = 8;     // Gram entries one thread accumulates per pass (point masks)
constexpr int kPStage = kPW > kGRows ? kPW : kGRows;   // staged rows: a point window or a factor-Gram chunk

// Point masks.  Blocks [0, gAB) are the factor-Gram partials as above; block
// gAB + k forms explicit Phi^H Phi and Phi^H y over mask rows [kPRows k, kPRows (k+1))
// into slot gAB + k and hpart[k].
template <class Src>
__global__ void __launch_bounds__(kSB) k_pstats(Src src) {
    extern __shared__ double2 s_dyn[];            // kPStage * R
    __shared__ double2 s_yw[kPW];
    __shared__ int s_err;
    if (!src.live()) return;
    const DevFrame f = src.get();
    if (!block_frame_ok(f.dev, false)) return;
    const int n1 = f.n1, n2 = f.n2, R = f.r, tid = threadIdx.x;
    const int gAB = n_gparts(n1) + n_gparts(n2);
    if (src.bx() < gAB) {
        factor_gram_block(f, src.bx(), reinterpret_cast<float2*>(s_dyn), false);
        return;
    }
    const int k = src.bx() - gAB;
    double2* out = f.part + size_t(gAB + k) * slot_size(R);
    if (tid == 0) s_err = 0;
    __syncthreads();
    // The sampled entries of rows [i0, i1) taken in windows of kPW candidates;
    // each window stages phi_{(i,j),r} = Ahat_ir Bhat_jr (zero where not sampled)
    // and accumulates Phi^H Phi (r <= s) and Phi^H y.
    const int i0 = k * kPRows;
    if (i0 >= n1) return;
    const int ncand = (min(n1, i0 + kPRows) - i0) * n2;
    double2* s_phi = s_dyn;                       // [kPW][R]
    const int RR = R * R;
    const int npass = cdiv(cdiv(RR, kSB), kMaxAcc);
    bool fin = true;
    for (int pass = 0; pass < npass; ++pass) {
        double2 acc[kMaxAcc];
#pragma unroll
        for (int u = 0; u < kMaxAcc; ++u) acc[u] = double2{0.0, 0.0};
        double2 hacc{0.0, 0.0};
        for (int w0 = 0; w0 < ncand; w0 += kPW) {
            __syncthreads();
            for (int e = tid; e < kPW * R; e += blockDim.x) {
                const int w = e / R, r = e % R, cidx = w0 + w;
                double2 phi{0.0, 0.0};
                if (cidx < ncand) {
                    const int i = i0 + cidx / n2, j = cidx % n2;
                    if (f.mask[size_t(i) * n2 + j]) {
                        const float2 a = f.Ahat[size_t(i) * R + r], b = f.Bhat[size_t(j) * R + r];
                        phi = double2{double(a.x) * b.x - double(a.y) * b.y, double(a.x) * b.y + double(a.y) * b.x};
                    }
                }
                s_phi[e] = phi;
            }
            for (int w = tid; w < kPW; w += blockDim.x) {
                const int cidx = w0 + w;
                double2 yy{0.0, 0.0};
                if (cidx < ncand) {
                    const int i = i0 + cidx / n2, j = cidx % n2;
                    if (f.mask[size_t(i) * n2 + j]) {
                        const float2 v = f.y[size_t(i) * n2 + j];
                        fin = fin && finite2(v);
                        yy = double2{v.x, v.y};
                    }
                }
                s_yw[w] = yy;
            }
            __syncthreads();
#pragma unroll
            for (int u = 0; u < kMaxAcc; ++u) {
                const int e = tid + (pass * kMaxAcc + u) * kSB;
                if (e < RR) {
                    const int r = e / R, s2 = e % R;
                    if (r <= s2) {
                        for (int w = 0; w < kPW; ++w) {
                            const double2 pr = s_phi[w * R + r], ps = s_phi[w * R + s2];
                            acc[u].x += pr.x * ps.x + pr.y * ps.y;
                            acc[u].y += pr.x * ps.y - pr.y * ps.x;
                        }
                    }
                }
            }
            if (pass == 0) {
                for (int r = tid; r < R; r += blockDim.x) {
                    for (int w = 0; w < kPW; ++w) {
                        const double2 pr = s_phi[w * R + r], yy = s_yw[w];
                        hacc.x += pr.x * yy.x + pr.y * yy.y;
                        hacc.y += pr.x * yy.y - pr.y * yy.x;
                    }
                }
            }
        }
#pragma unroll
        for (int u = 0; u < kMaxAcc; ++u) {
            const int e = tid + (pass * kMaxAcc + u) * kSB;
            if (e < RR && (e / R) <= (e % R)) out[upk(e / R, e % R, R)] = acc[u];
        }
        if (pass == 0 && tid < R) f.hpart[size_t(k) * R + tid] = hacc;
    }
    if (!fin) atomicCAS(&s_err, 0, ST_ENONFINITE);
    __syncthreads();
    if (tid == 0 && s_err) latch(f.dev, s_err);
}

// Sums of slot ranges of the statistics for U entries per thread: out[u] =
// sum over slots s < n (in slot order) of base[s * stride + up[u]]; loads are
// issued kSlotPF slots at a time for all U entries together.
constexpr int kSlotPF = 8;
template <int U>
__device__ __forceinline__ void slot_sums(const double2* base, size_t stride, int n, const size_t (&up)[U],
                                          const bool (&ok)[U], double2 (&out)[U]) {
#pragma unroll
    for (int u = 0; u < U; ++u) out[u] = double2{0.0, 0.0};
    for (int k0 = 0; k0 < n; k0 += kSlotPF) {
        double2 w[U][kSlotPF];
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
            for (int q = 0; q < kSlotPF; ++q)
                w[u][q] = (ok[u] && k0 + q < n) ? base[size_t(k0 + q) * stride + up[u]] : double2{0.0, 0.0};
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
            for (int q = 0; q < kSlotPF; ++q) { out[u].x += w[u][q].x; out[u].y += w[u][q].y; }
    }
}

// Right-hand side h = Phi^H y of thread r's entry: the sum of its partials in order.
__device__ __forceinline__ double2 rhs_sum(const DevFrame& f, int r, int nh) {
    size_t up[1] = {size_t(r)};
    bool ok[1] = {true};
    double2 out[1];
    slot_sums<1>(f.hpart, size_t(f.r), nh, up, ok, out);
    return out[0];
}

// ---------------------------------------------------------------- solve
__device__ __forceinline__ int pk(int i, int j) { return i * (i + 1) / 2 + j; }   // j <= i

// General R: one block per sequence, G packed in LDS, row-parallel right-looking
// Cholesky with block barriers between the steps.
constexpr int kSolveThreads = 256;
constexpr int kSolveU = 4;   // entries of G a thread gathers per pass

template <class Src>
__global__ void __launch_bounds__(kSolveThreads) k_solve(Src src) {
    extern __shared__ double2 s_dyn[];
    __shared__ int s_fail;
    __shared__ double s_piv_lo, s_piv_hi;
    __shared__ double s_wbest[kSolveThreads / 64];
    if (!src.live()) return;
    const DevFrame f = src.get();
    SeqDev* d = f.dev;
    if (!block_frame_ok(d, false)) {
        if (threadIdx.x == 0) d->frame_ok = 0;
        return;
    }
    const int R = f.r, n1 = f.n1, tid = threadIdx.x;
    const bool lines = f.mode == MODE_LINES;
    const int ns = lines ? cdiv(frame_rows(f), kSRows) : cdiv(n1, kPRows);
    const int gA = n_gparts(n1), gB = n_gparts(f.n2), gAB = gA + gB;
    const int nh = ns * (lines ? n_jparts(f.n2) : 1);
    const size_t RR = size_t(slot_size(R));   // entries per slot
    const double2* pa = f.part;               // slots of (F_l A)^H F_l A
    const double2* pb = f.part + gA * RR;     // slots of (F_r B)^H F_r B
    const double2* ps = f.part + gAB * RR;    // slots of the sampled part
    double2* L = s_dyn;                       // packed lower triangle of G, then of its factor
    double2* h = s_dyn + R * (R + 1) / 2;     // right-hand side, then gamma
    const double lam = f.lambda;

    // G = Phi^H Phi + lambda I from the statistics (slot entry (j, i), j <= i,
    // holds G_ji = conj(G_ij)): the sampled part summed over its slots, then
    // (lines) times the B Gram entrywise.
    const int npairs = R * (R + 1) / 2;
    for (int e0 = 0; e0 < npairs; e0 += kSolveThreads * kSolveU) {
        size_t up[kSolveU];
        bool ok[kSolveU];
        int ii[kSolveU], jj[kSolveU];
#pragma unroll
        for (int u = 0; u < kSolveU; ++u) {
            const int e = e0 + tid + kSolveThreads * u;
            int i = int((sqrt(8.0 * e + 1.0) - 1.0) * 0.5);
            while (i * (i + 1) / 2 > e) --i;
            while ((i + 1) * (i + 2) / 2 <= e) ++i;
            ok[u] = e < npairs;
            ii[u] = i;
            jj[u] = e - i * (i + 1) / 2;
            up[u] = ok[u] ? size_t(upk(jj[u], i, R)) : 0;
        }
        double2 g[kSolveU], gb[kSolveU];
        slot_sums<kSolveU>(ps, RR, ns, up, ok, g);
        if (lines) slot_sums<kSolveU>(pb, RR, gB, up, ok, gb);
#pragma unroll
        for (int u = 0; u < kSolveU; ++u) {
            if (!ok[u]) continue;
            double2 v = lines ? dcmul(g[u], gb[u]) : g[u];
            v.y = -v.y;
            if (ii[u] == jj[u]) v = double2{v.x + lam, 0.0};
            L[pk(ii[u], jj[u])] = v;
        }
    }
    for (int r = tid; r < R; r += kSolveThreads) h[r] = rhs_sum(f, r, nh);
    if (tid == 0) { s_fail = 0; s_piv_lo = 1e308; s_piv_hi = 0.0; }
    __syncthreads();

    // Cholesky G = L L^H, right-looking: at step k every lane i > k scales its
    // entry of column k by 1/L_kk and then updates its own row of the trailing
    // triangle (row i is contiguous in the packed layout).  s_inv keeps 1/L_kk.
    double* s_inv = reinterpret_cast<double*>(h + R);
    for (int k = 0; k < R; ++k) {
        const double dd = L[pk(k, k)].x;                 // same value in every lane
        if (!(dd > 0.0) || !isfinite(dd)) {
            if (tid == 0) s_fail = ST_ENOTPD;
            break;
        }
        double p, ip;
        pivot(dd, p, ip);
        __syncthreads();
        if (tid == 0) {
            L[pk(k, k)] = double2{p, 0.0};
            s_inv[k] = ip;
            s_piv_lo = fmin(s_piv_lo, p);
            s_piv_hi = fmax(s_piv_hi, p);
        }
        for (int i = k + 1 + tid; i < R; i += kSolveThreads) {
            const double2 v = L[pk(i, k)];
            L[pk(i, k)] = double2{v.x * ip, v.y * ip};
        }
        __syncthreads();
        for (int i = k + 1 + tid; i < R; i += kSolveThreads) {
            double2* Li = L + pk(i, 0);
            const double2 lik = Li[k];
            int j = k + 1;
            for (; j + 4 <= i + 1; j += 4) {
                double2 c[4], o[4];
#pragma unroll
                for (int w = 0; w < 4; ++w) { c[w] = L[pk(j + w, k)]; o[w] = Li[j + w]; }
#pragma unroll
                for (int w = 0; w < 4; ++w) {
                    const double2 t = dcmulc(lik, c[w]);      // L_ik conj(L_jk)
                    Li[j + w] = double2{o[w].x - t.x, o[w].y - t.y};
                }
            }
            for (; j <= i; ++j) {
                const double2 t = dcmulc(lik, L[pk(j, k)]);
                Li[j].x -= t.x;
                Li[j].y -= t.y;
            }
        }
        __syncthreads();
    }
    __syncthreads();
    if (!s_fail) {
        for (int k = 0; k < R; ++k) {         // L z = h
            const double2 zk{h[k].x * s_inv[k], h[k].y * s_inv[k]};
            __syncthreads();
            if (tid == 0) h[k] = zk;
            for (int i = k + 1 + tid; i < R; i += kSolveThreads) {
                const double2 t = dcmul(L[pk(i, k)], zk);
                h[i].x -= t.x;
                h[i].y -= t.y;
            }
            __syncthreads();
        }
        for (int k = R - 1; k >= 0; --k) {    // L^H gamma = z
            const double2 gk{h[k].x * s_inv[k], h[k].y * s_inv[k]};
            __syncthreads();
            if (tid == 0) h[k] = gk;
            for (int i = tid; i < k; i += kSolveThreads) {
                const double2 t = dcmulc(gk, L[pk(k, i)]);   // conj(L_ki) gamma_k
                h[i].x -= t.x;
                h[i].y -= t.y;
            }
            __syncthreads();
        }
        for (int r = tid; r < R; r += kSolveThreads)
            if (!isfinite(h[r].x) || !isfinite(h[r].y)) s_fail = ST_ENONFINITE;
    }
    __syncthreads();
    if (s_fail) {
        if (tid == 0) {
            latch(d, s_fail);
            d->frame_ok = 0;
        }
        return;
    }
    // Gershgorin row sums of diag(g)^H M diag(g), M = A^H A and B^H B (each
    // summed over its slots); the factor's LDS (R(R+1) doubles >= R*R) holds the
    // |entries| of one M at a time.
    double* mag = reinterpret_cast<double*>(s_dyn);
    double* s_ag = s_inv + R;                 // |gamma_r|
    for (int r = tid; r < R; r += kSolveThreads) s_ag[r] = dabs(h[r]);
    __syncthreads();
    double best = 0.0;
    for (int which = 0; which < 2; ++which) {
        const double2* pm = which ? pb : pa;
        const int nm = which ? gB : gA;
        __syncthreads();
        for (int e0 = 0; e0 < R * R; e0 += kSolveThreads * kSolveU) {
            size_t up[kSolveU];
            bool ok[kSolveU];
#pragma unroll
            for (int u = 0; u < kSolveU; ++u) {
                const int e = e0 + tid + kSolveThreads * u;
                const int r = e / R, c = e % R;
                ok[u] = e < R * R;
                up[u] = !ok[u] ? 0 : size_t(r <= c ? upk(r, c, R) : upk(c, r, R));
            }
            double2 v[kSolveU];
            slot_sums<kSolveU>(pm, RR, nm, up, ok, v);
#pragma unroll
            for (int u = 0; u < kSolveU; ++u) {
                const int e = e0 + tid + kSolveThreads * u;
                if (ok[u]) mag[e] = s_ag[e / R] * dabs(v[u]) * s_ag[e % R];
            }
        }
        __syncthreads();
        for (int r = tid; r < R; r += kSolveThreads) {
            const double* mr = mag + r * R;
            double row = 0.0;
            int c = 0;
            for (; c + 8 <= R; c += 8) {
                double v[8];
#pragma unroll
                for (int w = 0; w < 8; ++w) v[w] = mr[c + w];
#pragma unroll
                for (int w = 0; w < 8; ++w) row += v[w];
            }
            for (; c < R; ++c) row += mr[c];
            best = fmax(best, row);
        }
    }
    __syncthreads();
    for (int m = 32; m > 0; m >>= 1) best = fmax(best, __shfl_xor(best, m, 64));
    if (tid % 64 == 0) s_wbest[tid / 64] = best;
    __syncthreads();
    if (tid == 0)
        for (int w = 0; w < kSolveThreads / 64; ++w) best = fmax(best, s_wbest[w]);
    for (int r = tid; r < R; r += kSolveThreads) {
        f.gamma64[r] = h[r];
        const float2 g32{float(h[r].x), float(h[r].y)};
        f.gamma32[r] = g32;
        if (f.gamma_out) f.gamma_out[r] = g32;
    }
    if (tid == 0) {
        const long long tn = d->t + 1;
        const double alpha = lam / double(tn) + best;
        const double abar = d->abar + alpha;
        const double mu = f.step_mode == TSL_STEP_MM ? 1.0 / abar : f.mu_const;
        d->t_new = tn;
        d->alpha = alpha;
        d->abar_new = abar;
        d->mu = mu;
        d->shrink = 1.0 - lam * mu / double(tn);
        d->kappa_proxy = (s_piv_hi / s_piv_lo) * (s_piv_hi / s_piv_lo);
        d->frame_ok = 1;
        if (f.info_out) {
            f.info_out[0] = alpha;
            f.info_out[1] = abar;
            f.info_out[2] = mu;
            f.info_out[3] = d->kappa_proxy;
        }
    }
}

// ---------------------------------------------------------------- register solve (R <= 64)
// A block of kRegBlk threads per sequence.  The whole block first gathers G, h
// and the magnitudes of the two factor Grams into LDS with all of its loads in
// flight at once (issued before the frame's status is known, over the row
// capacity of the descriptor; the device row count only selects which sampled
// slots are added).  Wavefront 0 then factors G = L D L^H (unit lower L) with
// lane i keeping row i in registers and runs the forward substitution L z = h
// inside the same sweep; gamma = L^{-H} D^{-1} z follows with the columns of L
// read back through LDS.  Rows R..RB-1 are padded with the identity and a zero
// right-hand side, which leaves gamma unchanged.  The Gershgorin sums of the
// step size use the whole block.
__device__ __forceinline__ double readlane_d(double v, int lane) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane(int(b), lane);
    const int hi = __builtin_amdgcn_readlane(int(b >> 32), lane);
    return __longlong_as_double((static_cast<long long>(hi) << 32) | static_cast<unsigned int>(lo));
}
__device__ __forceinline__ double2 readlane_d2(double2 v, int lane) {
    return double2{readlane_d(v.x, lane), readlane_d(v.y, lane)};
}
// 1 / d for d > 0: the hardware estimate (relative error near 2^-23) refined by
// one Newton step, which squares the error (near 2^-46): far below what the
// FP32 products of gamma resolve, and two dependent operations shorter on the
// solve's serial path than a second step.
__device__ __forceinline__ double recip(double d) {
    const double y = __builtin_amdgcn_rcp(d);
    return fma(y, fma(-d, y, 1.0), y);
}

constexpr int kRegBlk = 256;
// partial slots of each statistic loaded per round (fewer at RB = 64, where a
// thread gathers nine upper entries)
template <int RB> constexpr int gather_pf() { return RB <= 32 ? 4 : 1; }

template <int RB, class Src>
__global__ void __launch_bounds__(kRegBlk) k_solve_reg(Src src) {
    static_assert(RB <= 64 && kRegBlk % RB == 0 && (kRegBlk / RB) <= 64, "row groups must sit inside a wavefront");
    constexpr int TPR = kRegBlk / RB;                       // threads per row in the Gershgorin sums
    // Row pitch of the LDS matrices: one element more than a row, so that a
    // column read or written across lanes (row i in lane i) spreads over the
    // banks instead of landing every lane on the same ones.
    constexpr int GP = RB + 1;
    __shared__ double2 s_g[RB * GP];       // G row-major, then L below the diagonal
    __shared__ double s_m[2][RB * GP];     // |(F_l A)^H F_l A|, |(F_r B)^H F_r B|
    __shared__ double2 s_h[RB];            // gamma
    __shared__ double2 s_hp[kRegBlk];      // the first kRegBlk right-hand-side partial entries
    __shared__ double2 s_c[2][RB];         // column k of the partly reduced G during step k (two buffers)
    __shared__ double s_ik[2];             // 1 / D_k (two buffers; four-wavefront sweep)
    __shared__ double s_dk[RB];            // the pivots D_k (four-wavefront sweep)
    __shared__ double s_ag[RB];            // |gamma|
    __shared__ double s_best[kRegBlk / 64];
    __shared__ double s_kappa;
    __shared__ int s_fail;
    if (!src.live()) return;
    const DevFrame f = src.get();
    SeqDev* d = f.dev;
    const int R = f.r, tid = threadIdx.x, lane = tid % 64, wave = tid / 64;
    const bool lines = f.mode == MODE_LINES;
    // slot counts over the capacity (loads) and over the rows of this frame (sums)
    const int ns_cap = lines ? cdiv(frame_rows_cap(f), kSRows) : cdiv(f.n1, kPRows);
    const int ns = lines ? cdiv(frame_rows(f), kSRows) : ns_cap;
    const int gA = n_gparts(f.n1), gB = n_gparts(f.n2), gAB = gA + gB;
    const int hper = lines ? n_jparts(f.n2) : 1;
    const int nh_cap = ns_cap * hper, nh = ns * hper;
    const size_t RR = size_t(slot_size(R));   // entries per slot
    const double2* pa = f.part;               // slots of (F_l A)^H F_l A
    const double2* pb = f.part + gA * RR;     // slots of (F_r B)^H F_r B
    const double2* ps = f.part + gAB * RR;    // slots of the sampled part
    const double lam = f.lambda;
    // the step size's inputs (unchanged until this frame commits), read now so
    // that the epilogue does not wait for them
    const long long t_prev = d->t;
    const double abar_prev = d->abar;

    // Gather.  A slot holds the upper triangle packed by rows: entry (r, c),
    // r <= c, is G_rc at upk(r, c, R).  Each thread takes upper entries (in the
    // same packed order, so a wavefront's loads are contiguous) and writes both
    // (i, j) and its conjugate mirror (j, i).
    constexpr int NU = RB * (RB + 1) / 2;
    constexpr int U = (NU + kRegBlk - 1) / kRegBlk;   // upper entries per thread
    size_t up[U];
    bool ok[U];
    int ui[U], uj[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
        int e = tid + u * kRegBlk, i = 0;
        if (e < NU)
            while (e >= RB - i) { e -= RB - i; ++i; }
        ui[u] = i;
        uj[u] = i + e;
        ok[u] = tid + u * kRegBlk < NU && uj[u] < R;
        up[u] = ok[u] ? size_t(upk(ui[u], uj[u], R)) : 0;
    }
    // one right-hand-side partial entry per thread (entry q R + r is slot q of
    // h_r) and the first kGatherPF slots of all three statistics are in flight
    // before the status check
    // (every load reads a valid address -- slot indices are clamped into the
    // statistic's range -- and a select drops what lies past the count, so that
    // the loads are issued back to back with no branch between them)
    const double2 hpe0 = f.hpart[min(tid, max(nh_cap * R - 1, 0))];
    const double2 hpe = tid < nh_cap * R ? hpe0 : double2{0.0, 0.0};
    double2 g[U], ma[U], mb[U];
#pragma unroll
    for (int u = 0; u < U; ++u) g[u] = ma[u] = mb[u] = double2{0.0, 0.0};
    const int nmax = max(gA, max(gB, ns_cap));
    constexpr int kGatherPF = gather_pf<RB>();
    double2 wa[U][kGatherPF], wb[U][kGatherPF], ws[U][kGatherPF];
    auto load_round = [&](int k0) {
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
            for (int q = 0; q < kGatherPF; ++q) {
                const int k = k0 + q;
                const double2 va = pa[size_t(min(k, gA - 1)) * RR + up[u]];
                const double2 vb = pb[size_t(min(k, gB - 1)) * RR + up[u]];
                const double2 vs = ps[size_t(min(k, max(ns_cap - 1, 0))) * RR + up[u]];
                wa[u][q] = (ok[u] && k < gA) ? va : double2{0.0, 0.0};
                wb[u][q] = (ok[u] && k < gB) ? vb : double2{0.0, 0.0};
                ws[u][q] = (ok[u] && k < ns_cap) ? vs : double2{0.0, 0.0};
            }
    };
    auto add_round = [&](int k0) {
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
            for (int q = 0; q < kGatherPF; ++q) {
                ma[u].x += wa[u][q].x; ma[u].y += wa[u][q].y;
                mb[u].x += wb[u][q].x; mb[u].y += wb[u][q].y;
                if (k0 + q < ns) { g[u].x += ws[u][q].x; g[u].y += ws[u][q].y; }
            }
    };
    load_round(0);
    if (!block_frame_ok(d, false)) {
        if (tid == 0) d->frame_ok = 0;
        return;
    }
    s_hp[tid] = hpe;
    add_round(0);
    for (int k0 = kGatherPF; k0 < nmax; k0 += kGatherPF) {
        load_round(k0);
        add_round(k0);
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
        if (tid + u * kRegBlk >= NU) continue;
        const int i = ui[u], j = uj[u];
        double2 v{0.0, 0.0};
        if (ok[u]) {
            v = lines ? dcmul(g[u], mb[u]) : g[u];
            if (i == j) v = double2{v.x + lam, 0.0};
        } else if (i == j) {
            v = double2{1.0, 0.0};                    // identity padding
        }
        const double am = dabs(ma[u]), bm = dabs(mb[u]);
        s_g[i * GP + j] = v;
        s_m[0][i * GP + j] = am;
        s_m[1][i * GP + j] = bm;
        if (i != j) {
            s_g[j * GP + i] = double2{v.x, -v.y};
            s_m[0][j * GP + i] = am;
            s_m[1][j * GP + i] = bm;
        }
    }
    __syncthreads();

    double2 hv{0.0, 0.0};
    double dinv = 0.0;                            // 1 / D_ii of the lane's row (wavefront 0)
    // h_i = sum of its slots in slot order (wavefront 0, both halves)
    auto gather_h = [&](int i) {
        if (i < R)
            for (int q = 0; q < nh; ++q) {
                const int e = q * R + i;
                const double2 v = e < kRegBlk ? s_hp[e] : f.hpart[e];
                hv.x += v.x;
                hv.y += v.y;
            }
    };
    if constexpr (RB >= 32) {
        // Right-looking L D L^H shared by the four wavefronts, one barrier per
        // step.  Thread t holds row i = t % RB of the columns j = NG m + g,
        // g = t / RB (NG = 8 column groups of four columns at RB = 32: lane l of
        // wavefront w in group 2 w + l / 32; NG = 4 groups of sixteen columns at
        // RB = 64: wavefront w is group w).  Step k reads the unscaled column
        // c = G[:, k] and 1/D_k from LDS and applies G_ij -= c_i conj(c_j) / D_k
        // to its columns; the lane group that holds column k+1 reduces it first
        // and puts it and its pivot's reciprocal in the other LDS buffers for
        // the next step.  Wavefront 0 also keeps L
        // (into s_g), 1/D and the forward substitution L z = h.  Entries above
        // the diagonal and of finished columns receive updates too (never
        // read).  No branches on the pivots: one that is not positive and
        // finite is replaced by 1 in its reciprocal, and the check after the
        // sweep rejects the frame.
        constexpr int NG = kRegBlk / RB, CPL = RB / NG;   // column groups in the block, columns per lane
        const int i = tid % RB, g = tid / RB;
        double2 gr[CPL];
        sfor<CPL>([&](auto mc) {
            constexpr int m = decltype(mc)::value;
            gr[m] = s_g[i * GP + NG * m + g];
        });
        if (wave == 0) gather_h(i);
        // the thread that holds a pivot records it and its reciprocal (of 1 in
        // place of a pivot that is not positive and finite); the checks on the
        // recorded pivots run once after the sweep
        auto put_pivot = [&](int k, double dn) {
            s_dk[k] = dn;
            s_ik[k % 2] = recip((dn > 0.0 && isfinite(dn)) ? dn : 1.0);
        };
        if (g == 0) s_c[0][i] = gr[0];
        if (g == 0 && i == 0) put_pivot(0, gr[0].x);
        __syncthreads();
        sfor<RB>([&](auto kc) {
            constexpr int k = decltype(kc)::value;
            const double ik = s_ik[k % 2];
            const double2 ci = s_c[k % 2][i];                   // G_ik
            const double2 li{ci.x * ik, ci.y * ik};             // L_ik
            if (wave == 0) {
                if (i == k) dinv = ik;
                if (lane < RB && i > k) s_g[i * GP + k] = li;
                const double2 zk = readlane_d2(hv, k);          // z_k
                if (i > k) {
                    hv.x = fma(-li.x, zk.x, fma(li.y, zk.y, hv.x));
                    hv.y = fma(-li.x, zk.y, fma(-li.y, zk.x, hv.y));
                }
            }
            // G_ij -= L_ik conj(c_j)
            auto upd = [&](double2& v, double2 cj) {
                v = double2{fma(-li.x, cj.x, fma(-li.y, cj.y, v.x)), fma(-li.y, cj.x, fma(li.x, cj.y, v.y))};
            };
            if constexpr (k + 1 < RB) {
                constexpr int k1 = k + 1, g1 = k1 % NG, m1 = k1 / NG;
                const bool own = g == g1;                        // this lane group holds column k+1
                if (own) {
                    upd(gr[m1], s_c[k % 2][k1]);
                    s_c[k1 % 2][i] = gr[m1];
                    if (i == k1) put_pivot(k1, gr[m1].x);
                }
                sfor<CPL>([&](auto mc) {
                    constexpr int m = decltype(mc)::value;
                    if constexpr (NG * m + NG - 1 > k)
                        if (m != m1 || !own) upd(gr[m], s_c[k % 2][NG * m + g]);
                });
                __syncthreads();
            }
        });
        if (wave == 0) {
            // pivot checks and the conditioning figure over the recorded pivots
            bool bad = false;
            double lo = 1e308, hi = 0.0;
            for (int k = lane; k < RB; k += 64) {
                const double dk = s_dk[k];
                bad = bad || !(dk > 0.0) || !isfinite(dk);
                if (k < R) { lo = fmin(lo, dk); hi = fmax(hi, dk); }
            }
#pragma unroll
            for (int m = 32; m > 0; m >>= 1) {
                lo = fmin(lo, __shfl_xor(lo, m, 64));
                hi = fmax(hi, __shfl_xor(hi, m, 64));
            }
            const bool any_bad = __any(bad);
            if (lane == 0) {
                s_fail = any_bad ? ST_ENOTPD : 0;
                s_kappa = hi / lo;
            }
        }
    } else {
    // Wavefront 0: right-looking L D L^H, one column ahead.  Lane l holds row
    // i = l % RB of the columns j = NG m + l / RB (NG = 64 / RB column groups,
    // so all 64 lanes work).  Step k reads the unscaled column c = G[:, k]
    // from LDS and applies G_ij -= c_i conj(c_j) / D_k; the column k+1 is
    // reduced first, so its pivot's reciprocal and its copy into LDS run
    // beside the rest of the update.  Entries above the diagonal and of
    // finished columns receive updates too (never read).  A wavefront's LDS
    // accesses complete in order, so the fences only keep the compiler from
    // moving them.  The sweep has no branches: a pivot that is not positive and
    // finite sets `fail` (the same in every lane) and is replaced by 1 so that
    // the remaining steps stay finite; the frame is then rejected.
    constexpr int NG = 64 / RB, CPL = RB / NG;    // column groups, columns per lane
    double2 gr[CPL];
    if (wave == 0) {
        const int i = lane % RB, h = lane / RB;
        sfor<CPL>([&](auto mc) {
            constexpr int m = decltype(mc)::value;
            gr[m] = s_g[i * GP + NG * m + h];
        });
        gather_h(i);
        if (h == 0) s_c[0][i] = gr[0];
        double dk = readlane_d(gr[0].x, 0);
        bool fail = !(dk > 0.0) || !isfinite(dk);
        double ik = recip(fail ? 1.0 : dk);
        double d_lo = 1e308, d_hi = 0.0;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        sfor<RB>([&](auto kc) {
            constexpr int k = decltype(kc)::value;
            if (k < R) { d_lo = fmin(d_lo, dk); d_hi = fmax(d_hi, dk); }
            if (i == k) dinv = ik;
            const double2 ci = s_c[k % 2][i];                   // G_ik
            const double2 li{ci.x * ik, ci.y * ik};             // L_ik
            if (h == 0 && i > k) s_g[i * GP + k] = li;
            const double2 zk = readlane_d2(hv, k);              // z_k
            if (i > k) {
                hv.x = fma(-li.x, zk.x, fma(li.y, zk.y, hv.x));
                hv.y = fma(-li.x, zk.y, fma(-li.y, zk.x, hv.y));
            }
            // G_ij -= L_ik conj(c_j)
            auto upd = [&](double2& v, double2 cj) {
                v = double2{fma(-li.x, cj.x, fma(-li.y, cj.y, v.x)), fma(-li.y, cj.x, fma(li.x, cj.y, v.y))};
            };
            if constexpr (k + 1 < RB) {
                constexpr int k1 = k + 1, ko1 = k1 % NG, km1 = k1 / NG;
                upd(gr[km1], s_c[k % 2][NG * km1 + h]);
                if (h == ko1) s_c[k1 % 2][i] = gr[km1];
                const double dn = readlane_d(gr[km1].x, k1 + ko1 * RB);
                const bool fn = !(dn > 0.0) || !isfinite(dn);
                const double in = recip(fn ? 1.0 : dn);
                sfor<CPL>([&](auto mc) {
                    constexpr int m = decltype(mc)::value;
                    if constexpr (m != km1 && NG * m + NG - 1 > k) upd(gr[m], s_c[k % 2][NG * m + h]);
                });
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
                dk = dn;
                ik = in;
                fail = fail || fn;
            }
        });
        if (lane == 0) {
            s_fail = fail ? ST_ENOTPD : 0;
            s_kappa = d_hi / d_lo;
        }
    }
    }
    __syncthreads();
    if (wave == 0 && !s_fail) {
        // y = D^{-1} z, then L^H gamma = y from the last row up, the columns of
        // L read back from LDS kBS rows at a time (lcol[k] = L_{k, lane})
        constexpr int kBS = RB < 32 ? RB : 32;
        hv = double2{hv.x * dinv, hv.y * dinv};
        sfor<RB / kBS>([&](auto bc) {
            constexpr int k0 = RB - kBS * (decltype(bc)::value + 1);
            double2 lcol[kBS];
            sfor<kBS>([&](auto kc) {
                constexpr int k = decltype(kc)::value;
                lcol[k] = lane < RB ? s_g[(k0 + k) * GP + lane] : double2{0.0, 0.0};
            });
            sfor<kBS>([&](auto kc) {
                constexpr int kk = kBS - 1 - decltype(kc)::value, k = k0 + kk;
                const double2 gk = readlane_d2(hv, k);
                if (lane < k) {
                    hv.x = fma(-lcol[kk].x, gk.x, fma(-lcol[kk].y, gk.y, hv.x));   // - conj(L_{k,lane}) gamma_k
                    hv.y = fma(-lcol[kk].x, gk.y, fma(lcol[kk].y, gk.x, hv.y));
                }
            });
        });
        const bool live = lane < R;
        const bool nonfinite = __any(live && (!isfinite(hv.x) || !isfinite(hv.y)));
        if (live) {
            s_h[lane] = hv;
            s_ag[lane] = dabs(hv);
        }
        if (lane == 0 && nonfinite) s_fail = ST_ENONFINITE;
    }
    __syncthreads();
    if (s_fail) {
        if (tid == 0) {
            latch(d, s_fail);
            d->frame_ok = 0;
        }
        return;
    }
    // Gershgorin row sums of diag(g)^H M diag(g) for M = A^H A and B^H B:
    // TPR consecutive threads share a row, then the block takes the maximum.
    {
        const int r = tid / TPR, p = tid % TPR;
        double ra = 0.0, rb = 0.0;
        if (r < R)
            for (int c = p; c < R; c += TPR) {
                ra += s_m[0][r * GP + c] * s_ag[c];
                rb += s_m[1][r * GP + c] * s_ag[c];
            }
#pragma unroll
        for (int m = 1; m < TPR; m <<= 1) {
            ra += __shfl_xor(ra, m, 64);
            rb += __shfl_xor(rb, m, 64);
        }
        double best = r < R ? fmax(ra, rb) * s_ag[r] : 0.0;
#pragma unroll
        for (int m = 32; m > 0; m >>= 1) best = fmax(best, __shfl_xor(best, m, 64));
        if (lane == 0) s_best[wave] = best;
    }
    __syncthreads();
    if (tid < R) {
        const double2 gv = s_h[tid];
        f.gamma64[tid] = gv;
        const float2 g32{float(gv.x), float(gv.y)};
        f.gamma32[tid] = g32;
        if (f.gamma_out) f.gamma_out[tid] = g32;
    }
    if (tid == 0) {
        double best = 0.0;
#pragma unroll
        for (int w = 0; w < kRegBlk / 64; ++w) best = fmax(best, s_best[w]);
        const long long tn = t_prev + 1;
        const double alpha = lam / double(tn) + best;
        const double abar = abar_prev + alpha;
        const double mu = f.step_mode == TSL_STEP_MM ? 1.0 / abar : f.mu_const;
        d->t_new = tn;
        d->alpha = alpha;
        d->abar_new = abar;
        d->mu = mu;
        d->shrink = 1.0 - lam * mu / double(tn);
        d->kappa_proxy = s_kappa;
        d->frame_ok = 1;
        if (f.info_out) {
            f.info_out[0] = alpha;
            f.info_out[1] = abar;
            f.info_out[2] = mu;
            f.info_out[3] = s_kappa;
        }
    }
}

// ---------------------------------------------------------------- output synthesis
// X_t = A diag(gamma) B^T on the matrix cores in Gauss's three-multiplication
// form: with AG = A diag(gamma), P1 = sum_r Re AG Re B, P2 = sum_r Im AG Im B and
// P3 = sum_r (Re AG + Im AG)(Re B + Im B), Re X = P1 - P2 and
// Im X = P3 - P1 - P2; a 32x32x2 FP32 MFMA step takes two ranks (K over ranks),
// so a rank pair costs three steps instead of four.  A block owns a 128 x 64 tile of
// X (eight 32 x 32 wavefront tiles); the rows of AG and of B it needs are
// staged in LDS with coalesced loads, kOutRC ranks at a time.
// The block tile (TM x TN of X, one wavefront per 32 x 32 sub-tile) is a
// launch choice (OutTile): 128 x 64 by default, 64 x 64 or 128 x 128 where the
// tuner measured them faster; every output entry is computed the same way in
// each, so the choice changes no result.
constexpr int kOutRC = 32;                   // ranks staged per pass
constexpr int kOutPitch = kOutRC + 1;        // LDS row pitch (float2): conflict-free column reads

// With ds = 1, block 0 of each frame draws the frame's next rows (Algorithm 4,
// which needs only F_l A of the new A) beside the output tiles; the two roles
// share one LDS area.
template <int TM, int TN> struct OutShape {
    static constexpr int THREADS = (TM / 32) * (TN / 32) * 64;
    static constexpr size_t LDS = size_t(TM + TN) * kOutPitch * sizeof(float2);
    static constexpr size_t RAW = LDS > sizeof(SampleLds) ? LDS : sizeof(SampleLds);
};
// Block order of a table launch of the output synthesis: first the output
// tiles of every frame (X per frame, numbered as in FrameTable so that a
// frame's tiles share an XCD), then the draw blocks (ds per frame, frame y's at
// a position with the residue of its tiles).  The tiles carry the matrix-core
// work; dealt out first, they spread evenly over the compute units (two per
// unit in a launch of 64 frames of 256 x 256), and the light draw blocks fill
// in after them instead of stacking a third tile block on some units.
struct OutTable {
    const FrameArgs* __restrict__ t;
    int X, count, ds;
    __device__ __forceinline__ int tile_blocks() const { return (count + kXcds - 1) / kXcds * kXcds * X; }
    __device__ __forceinline__ int y() const {
        const int L = int(blockIdx.x), T = tile_blocks();
        if (L >= T) return (L - T) / ds;
        const int span = kXcds * X;
        return kXcds * (L / span) + (L % span) % kXcds;
    }
    __device__ __forceinline__ int bx() const {
        const int L = int(blockIdx.x), T = tile_blocks();
        if (L >= T) return (L - T) % ds;
        return ds + (L % (kXcds * X)) / kXcds;
    }
    __device__ __forceinline__ bool live() const { return y() < count; }
    __device__ __forceinline__ DevFrame get() const { return dev_frame(t[y()]); }
};

// ONE: every rank fits one pass (R <= kOutRC), so no staging load is in
// flight beside the accumulators and the kernel needs fewer registers.
// BF: SYN_FP32 (FP32 steps, two ranks each), SYN_BF16 or SYN_BF16X3 (BF16
// steps, sixteen ranks each: lane half h takes ranks c0 + 8h + j, j < 8).
template <bool ONE, int BF, int TM, int TN, class Src>
__global__ void __launch_bounds__((TM / 32) * (TN / 32) * 64) k_synth_out(Src src, int ds) {
    constexpr int kOutTM = TM, kOutTN = TN, kOutThreads = OutShape<TM, TN>::THREADS;
    __shared__ __align__(16) unsigned char s_raw[OutShape<TM, TN>::RAW];
    if (!src.live()) return;
    const DevFrame f = src.get();
    if (src.bx() < ds) {
        // a committed frame's A update left the row-weight block sums
        const bool ready = block_frame_ok(f.dev, true);
        draw_rows<kOutThreads>(f, *reinterpret_cast<SampleLds*>(s_raw), ready);
        return;
    }
    float2* s_ag = reinterpret_cast<float2*>(s_raw);   // [row][c] = A[i0 + row][r0 + c] gamma[r0 + c]
    float2* s_b = s_ag + kOutTM * kOutPitch;           // [row][c] = B[j0 + row][r0 + c]
    if (f.X_out == nullptr) return;
    const int n1 = f.n1, n2 = f.n2, R = f.r, tid = threadIdx.x, tile = src.bx() - ds;
    const int lane = tid % 64, w = tid / 64;
    const int tiles_x = cdiv(n2, kOutTN);
    const int bi = (tile / tiles_x) * kOutTM, bj = (tile % tiles_x) * kOutTN;
    if (bi >= n1) return;                   // a launch sized for a larger frame of the run
    const int wi = 32 * (w / (TN / 32)), wj = 32 * (w % (TN / 32));    // wavefront tile inside the block tile
    const int m = lane % 32, h = lane / 32;
    // A, gamma and B of a rank pass, all loads in flight together; the first
    // pass goes out before the status check (it reads the frame's own factors)
    constexpr int kLA = kOutTM * kOutRC / kOutThreads, kLB = kOutTN * kOutRC / kOutThreads;
    static_assert(kOutThreads % kOutRC == 0, "a thread stages one rank column");
    float2 la[kLA], lg, lb[kLB];
    // (indices clamped into range and the values past it selected away, so the
    // loads go out back to back)
    // (32-bit byte offsets from the frame's factor bases: one register per load address)
    const GlobalPtr<const char> Ab = reinterpret_cast<GlobalPtr<const char>>(f.A);
    const GlobalPtr<const char> Bb = reinterpret_cast<GlobalPtr<const char>>(f.B);
    auto load_pass = [&](int r0) {
        const int nr = min(kOutRC, R - r0), c = tid % kOutRC, cc = r0 + min(c, nr - 1);   // the thread's rank
        const float2 g = f.gamma32[cc];
        lg = c < nr ? g : float2{0.f, 0.f};
#pragma unroll
        for (int u = 0; u < kLA; ++u) {
            const int e = tid + u * kOutThreads, row = e / kOutRC, i = bi + row;
            const unsigned off = unsigned(min(i, n1 - 1) * R + cc) * 8u;
            const float2 a = *reinterpret_cast<GlobalPtr<const float2>>(Ab + off);
            la[u] = (i < n1 && c < nr) ? a : float2{0.f, 0.f};
        }
#pragma unroll
        for (int u = 0; u < kLB; ++u) {
            const int e = tid + u * kOutThreads, row = e / kOutRC, c = e % kOutRC, j = bj + row;
            const unsigned off = unsigned(min(j, n2 - 1) * R + r0 + min(c, nr - 1)) * 8u;
            const float2 b = *reinterpret_cast<GlobalPtr<const float2>>(Bb + off);
            lb[u] = (j < n2 && c < nr) ? b : float2{0.f, 0.f};
        }
    };
    load_pass(0);
    if (!block_frame_ok(f.dev, true)) return;
    f32x16 p1 = {}, p2 = {}, p3 = {};        // sum ar br, sum ai bi, sum (ar + ai)(br + bi)
    for (int r0 = 0; r0 < (ONE ? 1 : R); r0 += kOutRC) {
        const int nr = min(kOutRC, R - r0);
        if (!ONE) {
            __syncthreads();
            if (r0 > 0) load_pass(r0);
        }
#pragma unroll
        for (int u = 0; u < kLA; ++u) {
            const int e = tid + u * kOutThreads;
            s_ag[(e / kOutRC) * kOutPitch + e % kOutRC] = cmul(la[u], lg);
        }
#pragma unroll
        for (int u = 0; u < kLB; ++u) {
            const int e = tid + u * kOutThreads;
            s_b[(e / kOutRC) * kOutPitch + e % kOutRC] = lb[u];
        }
        __syncthreads();
        const float2* pa = s_ag + (wi + m) * kOutPitch;
        const float2* pb = s_b + (wj + m) * kOutPitch;
        // three real products per complex one: Re = P1 - P2, Im = P3 - P1 - P2
        if constexpr (BF == SYN_FP32) {
            // two ranks per step (K = 2: lane half h takes rank c0 + h)
            for (int c0 = 0; c0 < nr; c0 += 2) {
                const int c = min(c0 + h, nr - 1);
                const bool cv = c0 + h < nr;
                const float2 ag0 = pa[c], bb0 = pb[c];
                const float2 ag = cv ? ag0 : float2{0.f, 0.f}, bb = cv ? bb0 : float2{0.f, 0.f};
                p1 = mfma_32x32x2(ag.x, bb.x, p1);
                p2 = mfma_32x32x2(ag.y, bb.y, p2);
                p3 = mfma_32x32x2(ag.x + ag.y, bb.x + bb.y, p3);
            }
        } else {
            for (int c0 = 0; c0 < nr; c0 += 16) {
                bf16x8 ah[3], bh[3], al[3], bl[3];     // [re, im, re + im] of AG and of B
#pragma unroll
                for (int j = 0; j < 8; ++j) {
                    const int c = c0 + 8 * h + j;
                    const bool cv = c < nr;
                    const float2 ag0 = pa[min(c, nr - 1)], bb0 = pb[min(c, nr - 1)];
                    const float2 ag = cv ? ag0 : float2{0.f, 0.f}, bb = cv ? bb0 : float2{0.f, 0.f};
                    const float av[3] = {ag.x, ag.y, ag.x + ag.y}, bv[3] = {bb.x, bb.y, bb.x + bb.y};
#pragma unroll
                    for (int q = 0; q < 3; ++q) {
                        if constexpr (BF == SYN_BF16X3) {
                            const BfPair sa = split_bf16(av[q]), sb = split_bf16(bv[q]);
                            ah[q][j] = sa.hi;
                            al[q][j] = sa.lo;
                            bh[q][j] = sb.hi;
                            bl[q][j] = sb.lo;
                        } else {
                            ah[q][j] = static_cast<__bf16>(av[q]);
                            bh[q][j] = static_cast<__bf16>(bv[q]);
                        }
                    }
                }
                p1 = mfma_32x32x16_bf16(ah[0], bh[0], p1);
                p2 = mfma_32x32x16_bf16(ah[1], bh[1], p2);
                p3 = mfma_32x32x16_bf16(ah[2], bh[2], p3);
                if constexpr (BF == SYN_BF16X3) {
                    p1 = mfma_32x32x16_bf16(ah[0], bl[0], p1);
                    p2 = mfma_32x32x16_bf16(ah[1], bl[1], p2);
                    p3 = mfma_32x32x16_bf16(ah[2], bl[2], p3);
                    p1 = mfma_32x32x16_bf16(al[0], bh[0], p1);
                    p2 = mfma_32x32x16_bf16(al[1], bh[1], p2);
                    p3 = mfma_32x32x16_bf16(al[2], bh[2], p3);
                }
            }
        }
    }
    const int i0 = bi + wi, j = bj + wj + m;
    if (i0 >= n1 || j >= n2) return;
#pragma unroll
    for (int v = 0; v < 16; ++v) {
        const int row = i0 + mfma32_row(v, lane);
        // X_t is the caller's: no later kernel of the step reads it, so it is
        // stored past the cache (the end of the launch then has less to write back)
        if (row < n1)
            __builtin_nontemporal_store(f32x2{p1[v] - p2[v], p3[v] - p1[v] - p2[v]},
                                        reinterpret_cast<GlobalPtr<f32x2>>(f.X_out + size_t(row) * n2 + j));
    }
}

// ---------------------------------------------------------------- sampler
// The draw on its own (tsl_sample_lines); a step draws inside the output launch.
template <class Src>
__global__ void __launch_bounds__(kSampleThreads) k_sample(Src src) {
    __shared__ SampleLds s_l;
    if (!src.live()) return;
    draw_rows<kSampleThreads>(src.get(), s_l);
}

// The point draw (tsl_sample_points), one block.
__global__ void __launch_bounds__(kPointThreads) k_sample_points(OneFrame src, int K, unsigned char* mask, int* n_out,
                                                                 int* draws) {
    __shared__ PointLds s_l;
    const DevFrame f = src.get();
    draw_points<kPointThreads>(f, K, mask, n_out, draws, s_l);
}

// packed factor, right-hand side / gamma, then 1/L_kk and |gamma_r| (R doubles each)
size_t solve_lds(int R) { return size_t(R * (R + 1) / 2 + R) * sizeof(double2) + 2 * size_t(R) * sizeof(double); }

}  // namespace

void init_kernel_attributes() {
    static std::once_flag once;
    std::call_once(once, [] {
        const int ms = int(size_t(kPStage) * TSL_MAX_R * sizeof(double2));
        hipFuncSetAttribute(reinterpret_cast<const void*>(&k_pstats<FrameTable>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, ms);
        hipFuncSetAttribute(reinterpret_cast<const void*>(&k_pstats<OneFrame>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, ms);
        const int ml = int(lstats_lds(TSL_MAX_R));
        for (const void* k : {reinterpret_cast<const void*>(&k_lstats<2, FrameTable>),
                              reinterpret_cast<const void*>(&k_lstats<2, OneFrame>),
                              reinterpret_cast<const void*>(&k_lstats<4, FrameTable>),
                              reinterpret_cast<const void*>(&k_lstats<4, OneFrame>),
                              reinterpret_cast<const void*>(&k_lstats<8, FrameTable>),
                              reinterpret_cast<const void*>(&k_lstats<8, OneFrame>)})
            hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, ml);
        const int mv = int(solve_lds(TSL_MAX_R));
        hipFuncSetAttribute(reinterpret_cast<const void*>(&k_solve<FrameTable>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, mv);
        hipFuncSetAttribute(reinterpret_cast<const void*>(&k_solve<OneFrame>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, mv);
    });
}

hipError_t launch_stats(const Batch& b, hipStream_t st) {
    const int gAB = n_gparts(b.n1) + n_gparts(b.n2);
    if (b.mode == MODE_LINES) {
        const int nsg = cdiv(b.rows_max > 0 ? b.rows_max : 1, kSRows);   // chunks of sampled rows
        const int gx = gAB + nsg * (1 + n_jparts(b.n2));
        const dim3 grid = frame_grid(b, gx);
        const size_t lds = lstats_lds(b.r_max);
        auto go = [&](auto rt) {
            constexpr int RT = decltype(rt)::value;
            if (b.table) k_lstats<RT, FrameTable><<<grid, kSB, lds, st>>>(FrameTable{b.table, gx, b.count}, nsg);
            else k_lstats<RT, OneFrame><<<grid, kSB, lds, st>>>(OneFrame{*b.one}, nsg);
        };
        if (b.r_max <= 32) go(std::integral_constant<int, 2>{});
        else if (b.r_max <= 64) go(std::integral_constant<int, 4>{});
        else go(std::integral_constant<int, 8>{});
    } else {
        const size_t lds = size_t(kPStage) * b.r_max * sizeof(double2);
        const int gx = gAB + n_sparts(b.n1);
        const dim3 grid = frame_grid(b, gx);
        if (b.table) k_pstats<FrameTable><<<grid, kSB, lds, st>>>(FrameTable{b.table, gx, b.count});
        else k_pstats<OneFrame><<<grid, kSB, lds, st>>>(OneFrame{*b.one});
    }
    return hipGetLastError();
}

template <int RB> void launch_solve_reg(const Batch& b, hipStream_t st) {
    const int gx = 1;
    const dim3 grid = frame_grid(b, gx);
    if (b.table) k_solve_reg<RB, FrameTable><<<grid, kRegBlk, 0, st>>>(FrameTable{b.table, gx, b.count});
    else k_solve_reg<RB, OneFrame><<<grid, kRegBlk, 0, st>>>(OneFrame{*b.one});
}

hipError_t launch_solve(const Batch& b, hipStream_t st) {
    if (b.r_max <= 8) { launch_solve_reg<8>(b, st); return hipGetLastError(); }
    if (b.r_max <= 16) { launch_solve_reg<16>(b, st); return hipGetLastError(); }
    if (b.r_max <= 32) { launch_solve_reg<32>(b, st); return hipGetLastError(); }
    if (b.r_max <= 64) { launch_solve_reg<64>(b, st); return hipGetLastError(); }
    const int gx = 1;
    const dim3 grid = frame_grid(b, gx);
    const size_t lds = solve_lds(b.r_max);
    if (b.table) k_solve<FrameTable><<<grid, kSolveThreads, lds, st>>>(FrameTable{b.table, gx, b.count});
    else k_solve<OneFrame><<<grid, kSolveThreads, lds, st>>>(OneFrame{*b.one});
    return hipGetLastError();
}

hipError_t launch_synth_out(const Batch& b, hipStream_t st) {
    const int ds = b.want_sample ? 1 : 0;
    auto go = [&](auto one, auto bf, auto tm, auto tn) {
        constexpr bool ONE = decltype(one)::value;
        constexpr int BF = decltype(bf)::value, TM = decltype(tm)::value, TN = decltype(tn)::value;
        constexpr int NT = OutShape<TM, TN>::THREADS;
        const int gx = ds + (b.want_x ? cdiv(b.n1, TM) * cdiv(b.n2, TN) : 0);
        if (gx == 0) return;
        const dim3 grid = frame_grid(b, gx);
        if (b.table)
            k_synth_out<ONE, BF, TM, TN, OutTable><<<grid, NT, 0, st>>>(OutTable{b.table, gx - ds, b.count, ds}, ds);
        else k_synth_out<ONE, BF, TM, TN, OneFrame><<<grid, NT, 0, st>>>(OneFrame{*b.one}, ds);
    };
    using I128 = std::integral_constant<int, 128>;
    using I64 = std::integral_constant<int, 64>;
    auto with_bf = [&](auto one) {
        if (b.synth == SYN_BF16) go(one, std::integral_constant<int, SYN_BF16>{}, I128{}, I64{});
        else if (b.synth == SYN_BF16X3) go(one, std::integral_constant<int, SYN_BF16X3>{}, I128{}, I64{});
        else if (b.out_tile == OUT_64x64) go(one, std::integral_constant<int, SYN_FP32>{}, I64{}, I64{});
        else if (b.out_tile == OUT_128x128) go(one, std::integral_constant<int, SYN_FP32>{}, I128{}, I128{});
        else go(one, std::integral_constant<int, SYN_FP32>{}, I128{}, I64{});
    };
    if (b.r_max <= kOutRC) with_bf(std::true_type{});
    else with_bf(std::false_type{});
    return hipGetLastError();
}

hipError_t launch_sample_points(const FrameArgs& a, int K, unsigned char* mask, int* n_out, int* draws,
                                hipStream_t st) {
    k_sample_points<<<1, kPointThreads, 0, st>>>(OneFrame{a}, K, mask, n_out, draws);
    return hipGetLastError();
}

hipError_t launch_sample(const Batch& b, hipStream_t st) {
    if (!b.want_sample) return hipSuccess;
    const int gx = 1;
    const dim3 grid = frame_grid(b, gx);
    if (b.table) k_sample<FrameTable><<<grid, kSampleThreads, 0, st>>>(FrameTable{b.table, gx, b.count});
    else k_sample<OneFrame><<<grid, kSampleThreads, 0, st>>>(OneFrame{*b.one});
    return hipGetLastError();
}

}  // namespace tsl
