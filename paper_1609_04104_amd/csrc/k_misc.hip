// Kernels that are not templated on a transform length.
//
//  k_stats      FP64 partial statistics of S1 (Sec. III-A) for one frame.  With a
//               line mask S the regression matrix of Algorithm 3 (one coil) is
//               [Phi]_{(i,j),r} = (F_l a_r)_i (F_r b_r)_j, so its Gram is the
//               Hadamard product (Ahat_S^H Ahat_S) .* (Bhat^H Bhat) and
//               Phi^H y = sum_{i in S} conj(Ahat_i) .* (y_i conj(Bhat)); with a
//               point mask both are summed entry by entry.  Partials cover row
//               chunks and are reduced in a fixed order by k_solve.
//  k_solve      G = Phi^H Phi + lambda I, Cholesky, gamma_t = G^{-1} Phi^H y (the
//               closed form of the ridge problem), the step size alpha_t of the
//               majorizer (Sec. III-A; Gershgorin bound of diag(g)^H A^H A diag(g)
//               and of the B analogue, plus lambda/t), alpha_bar_t and mu_t (eq. 6).
//  k_synth_out  X_t = A[t] diag(gamma_t) B[t]^T (Sec. IV-A).
//  k_sample     Algorithm 4 on rows with the score of Sec. VI-C.
#include "fft_engine.hpp"
#include "kernels.hpp"
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

// out[r][s] = sum_q conj(X_{row(q), r}) X_{row(q), s} over q < nq (nq <= kGramRows),
// for r <= s only; the nq rows are staged once in s_rows (nq * R values).
template <class RowOf>
__device__ void gram_upper(const float2* X, int R, int nq, RowOf row_of, double2* out, float2* s_rows) {
    const int tid = threadIdx.x;
    __syncthreads();
    for (int e = tid; e < nq * R; e += blockDim.x) {
        const int q = e / R, r = e % R;
        const int row = row_of(q);
        s_rows[e] = row >= 0 ? X[size_t(row) * R + r] : float2{0.f, 0.f};
    }
    __syncthreads();
    for (int e = tid; e < R * R; e += blockDim.x) {
        const int r = e / R, s = e % R;
        if (r > s) continue;
        double2 acc{0.0, 0.0};
        for (int q = 0; q < nq; ++q) dacc_cj(acc, s_rows[q * R + r], s_rows[q * R + s]);
        out[e] = acc;
    }
}

template <class Src>
__global__ void __launch_bounds__(256) k_stats(Src src) {
    extern __shared__ float2 s_rows[];            // [kGramRows][R]
    __shared__ double2 s_h[kSRows * TSL_MAX_R];
    __shared__ int s_err;
    const FrameArgs& f = src.get();
    if (!block_frame_ok(f.dev, false)) return;
    const int n1 = f.n1, n2 = f.n2, R = f.r, tid = threadIdx.x;
    const int na = n_gram_a(n1), nb = n_gram_b(n2);
    const int item = blockIdx.x;
    double2* out = f.part + size_t(item) * R * R;
    if (item < na + nb) {
        const bool isa = item < na;
        const float2* X = isa ? f.Ahat : f.Bhat;
        const int n = isa ? n1 : n2;
        const int i0 = (isa ? item : item - na) * kGramRows;
        const int nq = min(n, i0 + kGramRows) - i0;
        gram_upper(X, R, nq, [&](int q) { return i0 + q; }, out, s_rows);
        return;
    }
    const int k = item - na - nb;
    if (tid == 0) s_err = 0;
    __syncthreads();
    if (f.mode == MODE_LINES) {
        const int n_rows = frame_rows(f);
        if (k == 0 && tid == 0 && f.n_rows_dev) {
            const int nd = *f.n_rows_dev;
            if (nd < 0 || nd > n1) latch(f.dev, ST_EINVAL);
        }
        const int q0 = k * kSRows;
        if (q0 >= n_rows) return;
        const int nq = min(n_rows, q0 + kSRows) - q0;
        // validate this chunk's rows: inside [0, n1), strictly ascending
        if (tid < nq) {
            const int q = q0 + tid, row = f.rows[q];
            bool ok = row >= 0 && row < n1;
            if (q + 1 < n_rows) ok = ok && f.rows[q + 1] > row;
            if (!ok) atomicCAS(&s_err, 0, ST_EINVAL);
        }
        auto row_of = [&](int q) {
            const int row = f.rows[q0 + q];
            return (row >= 0 && row < n1) ? row : -1;
        };
        gram_upper(f.Ahat, R, nq, row_of, out, s_rows);
        // z_q[r] = sum_j conj(Bhat_jr) y_qj, then h[r] = sum_q conj(Ahat_{row_q, r}) z_q[r]
        for (int e = tid; e < nq * R; e += blockDim.x) {
            const int q = e / R, r = e % R;
            const int row = row_of(q);
            double2 z{0.0, 0.0};
            bool fin = true;
            if (row >= 0) {
                const float2* yq = line_samples(f, q0 + q, row);
                for (int j = 0; j < n2; ++j) {
                    const float2 yy = yq[j];
                    fin = fin && finite2(yy);
                    dacc_cj(z, f.Bhat[size_t(j) * R + r], yy);
                }
            }
            if (!fin) atomicCAS(&s_err, 0, ST_ENONFINITE);
            const float2 a = row >= 0 ? f.Ahat[size_t(row) * R + r] : float2{0.f, 0.f};
            s_h[q * R + r] = dcmulc(z, double2{a.x, a.y});
        }
        __syncthreads();
        for (int r = tid; r < R; r += blockDim.x) {
            double2 h{0.0, 0.0};
            for (int q = 0; q < nq; ++q) { h.x += s_h[q * R + r].x; h.y += s_h[q * R + r].y; }
            f.hpart[size_t(k) * R + r] = h;
        }
    } else {
        const int i0 = k * kPRows;
        if (i0 >= n1) return;
        const int i1 = min(n1, i0 + kPRows);
        // G[r][s] += sum over sampled (i, j) of conj(Ahat_ir Bhat_jr) Ahat_is Bhat_js, r <= s
        const int RR = R * R;
        for (int e = tid; e < RR; e += blockDim.x) {
            const int r = e / R, s = e % R;
            if (r > s) continue;
            double2 acc{0.0, 0.0};
            for (int i = i0; i < i1; ++i) {
                const float2 ar = f.Ahat[size_t(i) * R + r], as = f.Ahat[size_t(i) * R + s];
                double2 m{0.0, 0.0};   // sum_j conj(Bhat_jr) Bhat_js over the sampled j of row i
                const unsigned char* mrow = f.mask + size_t(i) * n2;
                for (int j = 0; j < n2; ++j)
                    if (mrow[j]) dacc_cj(m, f.Bhat[size_t(j) * R + r], f.Bhat[size_t(j) * R + s]);
                double2 aa{0.0, 0.0};
                dacc_cj(aa, ar, as);
                const double2 p = dcmul(aa, m);
                acc.x += p.x;
                acc.y += p.y;
            }
            out[e] = acc;
        }
        for (int r = tid; r < R; r += blockDim.x) {
            double2 h{0.0, 0.0};
            bool fin = true;
            for (int i = i0; i < i1; ++i) {
                const unsigned char* mrow = f.mask + size_t(i) * n2;
                double2 z{0.0, 0.0};
                for (int j = 0; j < n2; ++j) {
                    if (!mrow[j]) continue;
                    const float2 yy = f.y[size_t(i) * n2 + j];
                    fin = fin && finite2(yy);
                    dacc_cj(z, f.Bhat[size_t(j) * R + r], yy);
                }
                const float2 a = f.Ahat[size_t(i) * R + r];
                const double2 c = dcmulc(z, double2{a.x, a.y});
                h.x += c.x;
                h.y += c.y;
            }
            if (!fin) atomicCAS(&s_err, 0, ST_ENONFINITE);
            f.hpart[size_t(k) * R + r] = h;
        }
    }
    __syncthreads();
    if (tid == 0 && s_err) latch(f.dev, s_err);
}

// ---------------------------------------------------------------- solve
__device__ __forceinline__ int pk(int i, int j) { return i * (i + 1) / 2 + j; }   // j <= i

template <class Src>
__global__ void __launch_bounds__(256) k_solve(Src src) {
    extern __shared__ double2 s_dyn[];
    __shared__ double s_red[kBlock];
    __shared__ int s_fail;
    __shared__ double s_piv_lo, s_piv_hi;
    const FrameArgs& f = src.get();
    SeqDev* d = f.dev;
    if (!block_frame_ok(d, false)) {
        if (threadIdx.x == 0) d->frame_ok = 0;
        return;
    }
    const int R = f.r, n1 = f.n1, n2 = f.n2, tid = threadIdx.x;
    const int na = n_gram_a(n1), nb = n_gram_b(n2);
    const bool lines = f.mode == MODE_LINES;
    const int ns = lines ? cdiv(frame_rows(f), kSRows) : cdiv(n1, kPRows);
    const size_t RR = size_t(R) * R;
    const double2* pa = f.part;
    const double2* pb = f.part + na * RR;
    const double2* ps = f.part + (na + nb) * RR;
    double2* L = s_dyn;
    double2* h = s_dyn + R * (R + 1) / 2;
    const double lam = f.lambda;

    // G (lower triangle, packed); stored partials hold the upper entries (j, i), j <= i.
    for (int e = tid; e < R * R; e += blockDim.x) {
        const int i = e / R, j = e % R;
        if (j > i) continue;
        const size_t up = size_t(j) * R + i;
        double2 g{0.0, 0.0};
        if (lines) {
            double2 gs{0.0, 0.0}, gb{0.0, 0.0};
            for (int k = 0; k < ns; ++k) { gs.x += ps[k * RR + up].x; gs.y += ps[k * RR + up].y; }
            for (int k = 0; k < nb; ++k) { gb.x += pb[k * RR + up].x; gb.y += pb[k * RR + up].y; }
            g = dcmul(gs, gb);
        } else {
            for (int k = 0; k < ns; ++k) { g.x += ps[k * RR + up].x; g.y += ps[k * RR + up].y; }
        }
        g.y = -g.y;                      // G_ij = conj(G_ji)
        if (i == j) g = double2{g.x + lam, 0.0};
        L[pk(i, j)] = g;
    }
    for (int r = tid; r < R; r += blockDim.x) {
        double2 hv{0.0, 0.0};
        for (int k = 0; k < ns; ++k) { hv.x += f.hpart[size_t(k) * R + r].x; hv.y += f.hpart[size_t(k) * R + r].y; }
        h[r] = hv;
    }
    if (tid == 0) { s_fail = 0; s_piv_lo = 1e308; s_piv_hi = 0.0; }
    __syncthreads();

    // Cholesky G = L L^H, left-looking by columns.
    for (int j = 0; j < R; ++j) {
        if (tid == 0) {
            double dd = L[pk(j, j)].x;
            for (int k = 0; k < j; ++k) { const double2 l = L[pk(j, k)]; dd -= l.x * l.x + l.y * l.y; }
            if (!(dd > 0.0) || !isfinite(dd)) {
                s_fail = ST_ENOTPD;
            } else {
                const double p = sqrt(dd);
                L[pk(j, j)] = double2{p, 0.0};
                s_piv_lo = fmin(s_piv_lo, p);
                s_piv_hi = fmax(s_piv_hi, p);
            }
        }
        __syncthreads();
        if (s_fail) break;
        const double p = L[pk(j, j)].x;
        for (int i = j + 1 + tid; i < R; i += blockDim.x) {
            double2 acc = L[pk(i, j)];
            for (int k = 0; k < j; ++k) {
                const double2 t = dcmulc(L[pk(i, k)], L[pk(j, k)]);
                acc.x -= t.x;
                acc.y -= t.y;
            }
            L[pk(i, j)] = double2{acc.x / p, acc.y / p};
        }
        __syncthreads();
    }
    if (!s_fail) {
        // L z = h
        for (int k = 0; k < R; ++k) {
            if (tid == 0) { const double p = L[pk(k, k)].x; h[k] = double2{h[k].x / p, h[k].y / p}; }
            __syncthreads();
            const double2 zk = h[k];
            for (int i = k + 1 + tid; i < R; i += blockDim.x) {
                const double2 t = dcmul(L[pk(i, k)], zk);
                h[i].x -= t.x;
                h[i].y -= t.y;
            }
            __syncthreads();
        }
        // L^H gamma = z
        for (int k = R - 1; k >= 0; --k) {
            if (tid == 0) { const double p = L[pk(k, k)].x; h[k] = double2{h[k].x / p, h[k].y / p}; }
            __syncthreads();
            const double2 gk = h[k];
            for (int i = tid; i < k; i += blockDim.x) {
                const double2 l = L[pk(k, i)];
                const double2 t = dcmulc(gk, l);   // conj(L_ki) gamma_k
                h[i].x -= t.x;
                h[i].y -= t.y;
            }
            __syncthreads();
        }
        for (int r = tid; r < R; r += blockDim.x)
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
    // Gershgorin row sums of diag(g)^H M diag(g) for M = A^H A and B^H B.
    double best = 0.0;
    for (int r = tid; r < R; r += blockDim.x) {
        const double gr = dabs(h[r]);
        double ra = 0.0, rb = 0.0;
        for (int s = 0; s < R; ++s) {
            const size_t up = r <= s ? size_t(r) * R + s : size_t(s) * R + r;
            double2 ga{0.0, 0.0}, gb{0.0, 0.0};
            for (int k = 0; k < na; ++k) { ga.x += pa[k * RR + up].x; ga.y += pa[k * RR + up].y; }
            for (int k = 0; k < nb; ++k) { gb.x += pb[k * RR + up].x; gb.y += pb[k * RR + up].y; }
            const double gs = dabs(h[s]);
            ra += gr * dabs(ga) * gs;
            rb += gr * dabs(gb) * gs;
        }
        best = fmax(best, fmax(ra, rb));
    }
    s_red[tid] = best;
    __syncthreads();
    for (int w = kBlock / 2; w > 0; w >>= 1) {
        if (tid < w) s_red[tid] = fmax(s_red[tid], s_red[tid + w]);
        __syncthreads();
    }
    for (int r = tid; r < R; r += blockDim.x) {
        f.gamma64[r] = h[r];
        const float2 g32{float(h[r].x), float(h[r].y)};
        f.gamma32[r] = g32;
        if (f.gamma_out) f.gamma_out[r] = g32;
    }
    if (tid == 0) {
        const long long tn = d->t + 1;
        const double alpha = lam / double(tn) + s_red[0];
        const double abar = d->abar + alpha;
        const double mu = f.step_mode == TSL_STEP_MM ? 1.0 / abar : f.mu_const;
        d->t_new = tn;
        d->alpha = alpha;
        d->abar_new = abar;
        d->mu = mu;
        d->shrink = 1.0 - lam * mu / double(tn);
        d->kappa_proxy = (s_piv_hi / s_piv_lo) * (s_piv_hi / s_piv_lo);
        d->frame_ok = 1;
    }
}

// ---------------------------------------------------------------- output synthesis
constexpr int kOutRows = 32, kOutCols = 64, kOutRC = 8;

template <class Src>
__global__ void __launch_bounds__(256) k_synth_out(Src src) {
    __shared__ float2 s_a[kOutRows * kOutRC];    // [row][c] = A[i][r0+c] gamma[r0+c]
    __shared__ float2 s_b[kOutRC * kOutCols];    // [c][col] = B[j][r0+c]
    const FrameArgs& f = src.get();
    if (f.X_out == nullptr) return;
    if (!block_frame_ok(f.dev, true)) return;
    const int n1 = f.n1, n2 = f.n2, R = f.r, tid = threadIdx.x;
    const int tiles_x = cdiv(n2, kOutCols);
    const int tx = blockIdx.x % tiles_x, ty = blockIdx.x / tiles_x;
    const int i0 = ty * kOutRows, j0 = tx * kOutCols;
    if (i0 >= n1) return;
    const int lx = tid % kOutCols, ly = tid / kOutCols;   // ly < 4: rows ly*8 .. ly*8+7
    float2 acc[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) acc[u] = float2{0.f, 0.f};
    for (int r0 = 0; r0 < R; r0 += kOutRC) {
        __syncthreads();
        {
            const int rr = tid / kOutRC, c = tid % kOutRC, i = i0 + rr;
            s_a[tid] = (i < n1 && r0 + c < R) ? cmul(f.A[size_t(i) * R + r0 + c], f.gamma32[r0 + c])
                                              : float2{0.f, 0.f};
        }
        for (int e = tid; e < kOutRC * kOutCols; e += blockDim.x) {
            const int col = e / kOutRC, c = e % kOutRC, j = j0 + col;
            s_b[c * kOutCols + col] = (j < n2 && r0 + c < R) ? f.B[size_t(j) * R + r0 + c] : float2{0.f, 0.f};
        }
        __syncthreads();
#pragma unroll
        for (int c = 0; c < kOutRC; ++c) {
            const float2 b = s_b[c * kOutCols + lx];
#pragma unroll
            for (int u = 0; u < 8; ++u) cfma(acc[u], s_a[(ly * 8 + u) * kOutRC + c], b);
        }
    }
    const int j = j0 + lx;
    if (j < n2) {
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int i = i0 + ly * 8 + u;
            if (i < n1) f.X_out[size_t(i) * n2 + j] = acc[u];
        }
    }
}

// ---------------------------------------------------------------- sampler
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

template <class Src>
__global__ void __launch_bounds__(256) k_sample(Src src) {
#pragma clang fp contract(off)
    extern __shared__ double s_pref[];           // [n1] weights, then their prefix
    __shared__ double s_c[TSL_MAX_R];
    __shared__ int s_mark[kMaxN];
    const FrameArgs& f = src.get();
    const int K = f.K_next;
    if (K <= 0) return;
    const int n1 = f.n1, n2 = f.n2, R = f.r, tid = threadIdx.x;
    // column energies ||ahat_r||^2, sequential in i
    for (int r = tid; r < R; r += blockDim.x) {
        double acc = 0.0;
        for (int i = 0; i < n1; ++i) {
            const float2 a = f.Ahat[size_t(i) * R + r];
            const double ax = a.x, ay = a.y;
            const double e = ax * ax + ay * ay;
            acc = acc + e;
        }
        s_c[r] = acc;
    }
    __syncthreads();
    // w_i = N2 ||abar_i||^2 + R, sequential in r
    for (int i = tid; i < n1; i += blockDim.x) {
        double q = 0.0;
        for (int r = 0; r < R; ++r) {
            const double c = s_c[r];
            if (c > 0.0) {
                const float2 a = f.Ahat[size_t(i) * R + r];
                const double ax = a.x, ay = a.y;
                const double e = ax * ax + ay * ay;
                q = q + e / c;
            }
        }
        double w = double(n2) * q;
        w = w + double(R);
        s_pref[i] = w;
        s_mark[i] = 0;
    }
    __syncthreads();
    if (tid == 0) {
        double acc = 0.0;
        for (int i = 0; i < n1; ++i) {
            acc = acc + s_pref[i];
            s_pref[i] = acc;
        }
    }
    __syncthreads();
    const double W = s_pref[n1 - 1];
    const uint64_t t_next = uint64_t(f.dev->t + 1);
    for (int k = tid; k < K; k += blockDim.x) {
        uint64_t x[4] = {t_next, uint64_t(k), 0ull, 0ull};
        philox4x64_10(x, f.seed, f.sid);
        const double u = double(x[0] >> 11) * 0x1.0p-53;
        const double target = u * W;
        int lo = 0, hi = n1;               // first i with target < prefix[i]
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (target < s_pref[mid]) hi = mid; else lo = mid + 1;
        }
        const int idx = lo < n1 ? lo : n1 - 1;
        if (f.draws_next) f.draws_next[k] = idx;
        s_mark[idx] = 1;
    }
    __syncthreads();
    if (tid == 0) {
        int cnt = 0;
        for (int i = 0; i < n1; ++i)
            if (s_mark[i]) f.rows_next[cnt++] = i;
        f.n_next[0] = cnt;
    }
    if (f.prefix_next)
        for (int i = tid; i < n1; i += blockDim.x) f.prefix_next[i] = s_pref[i];
}

size_t solve_lds(int R) { return size_t(R * (R + 1) / 2 + R) * sizeof(double2); }

}  // namespace

void init_kernel_attributes() {
    static std::once_flag once;
    std::call_once(once, [] {
        const int ms = int(size_t(kGramRows) * TSL_MAX_R * sizeof(float2));
        hipFuncSetAttribute(reinterpret_cast<const void*>(&k_stats<FrameTable>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, ms);
        hipFuncSetAttribute(reinterpret_cast<const void*>(&k_stats<OneFrame>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, ms);
        const int mv = int(solve_lds(TSL_MAX_R));
        hipFuncSetAttribute(reinterpret_cast<const void*>(&k_solve<FrameTable>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, mv);
        hipFuncSetAttribute(reinterpret_cast<const void*>(&k_solve<OneFrame>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, mv);
    });
}

hipError_t launch_stats(const Batch& b, hipStream_t st) {
    dim3 grid(n_parts(b.n1, b.n2), b.table ? b.count : 1);
    const size_t lds = size_t(kGramRows) * b.r_max * sizeof(float2);
    if (b.table) k_stats<FrameTable><<<grid, kBlock, lds, st>>>(FrameTable{b.table});
    else k_stats<OneFrame><<<grid, kBlock, lds, st>>>(OneFrame{*b.one});
    return hipGetLastError();
}

hipError_t launch_solve(const Batch& b, hipStream_t st) {
    dim3 grid(1, b.table ? b.count : 1);
    const size_t lds = solve_lds(b.r_max);
    if (b.table) k_solve<FrameTable><<<grid, kBlock, lds, st>>>(FrameTable{b.table});
    else k_solve<OneFrame><<<grid, kBlock, lds, st>>>(OneFrame{*b.one});
    return hipGetLastError();
}

hipError_t launch_synth_out(const Batch& b, hipStream_t st) {
    if (!b.want_x) return hipSuccess;
    dim3 grid(cdiv(b.n1, kOutRows) * cdiv(b.n2, kOutCols), b.table ? b.count : 1);
    if (b.table) k_synth_out<FrameTable><<<grid, kBlock, 0, st>>>(FrameTable{b.table});
    else k_synth_out<OneFrame><<<grid, kBlock, 0, st>>>(OneFrame{*b.one});
    return hipGetLastError();
}

hipError_t launch_sample(const Batch& b, hipStream_t st) {
    if (!b.want_sample) return hipSuccess;
    dim3 grid(1, b.table ? b.count : 1);
    const size_t lds = size_t(b.n1) * sizeof(double);
    if (b.table) k_sample<FrameTable><<<grid, kBlock, lds, st>>>(FrameTable{b.table});
    else k_sample<OneFrame><<<grid, kBlock, lds, st>>>(OneFrame{*b.one});
    return hipGetLastError();
}

}  // namespace tsl
