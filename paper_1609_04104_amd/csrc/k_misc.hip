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

// ---------------------------------------------------------------- Gram statistics
// Blocks of kGThreads threads in kGGroups row groups: every group owns the same
// upper-triangle entries (kGE per thread per pass) and takes every kGGroups-th
// staged row; the groups' partial sums are added in group order at the end.
// Rows are staged once per pass as FP64 (s_x, kGStage complex entries).
constexpr int kGThreads = 1024;
constexpr int kGGroups = 4;
constexpr int kGTh = kGThreads / kGGroups;
constexpr int kGStage = 4096;
constexpr int kGE = 4;
constexpr int kGRed = (kGGroups - 1) * kGTh * kGE;   // complex entries of s_red

__device__ __forceinline__ double2 dconj_mul(double2 a, double2 b) {   // conj(a) b
    return double2{a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x};
}

template <class RowOf>
__device__ void gram_upper(const float2* X, int R, int nq, RowOf row_of, double2* out, double2* s_x,
                           double2* s_red) {
    const int tid = threadIdx.x, g = tid / kGTh, t = tid % kGTh;
    const int npairs = R * (R + 1) / 2;
    const int npass = cdiv(npairs, kGTh * kGE);
    const int stage_rows = max(1, kGStage / R);
    for (int pass = 0; pass < npass; ++pass) {
        int er[kGE], es[kGE];
        double2 acc[kGE];
#pragma unroll
        for (int u = 0; u < kGE; ++u) {
            int e = t + (pass * kGE + u) * kGTh, r = 0;
            if (e < npairs) {
                while (e >= R - r) { e -= R - r; ++r; }
                er[u] = r;
                es[u] = r + e;
            } else {
                er[u] = 0;
                es[u] = -1;
            }
            acc[u] = double2{0.0, 0.0};
        }
        for (int q0 = 0; q0 < nq; q0 += stage_rows) {
            const int ns = min(stage_rows, nq - q0);
            __syncthreads();
            stage_copy<8, float2>(
                ns * R,
                [&](int e) {
                    const int row = row_of(q0 + e / R);
                    return row >= 0 ? X[size_t(row) * R + e % R] : float2{0.f, 0.f};
                },
                [&](int e, float2 v) { s_x[e] = double2{v.x, v.y}; });
            __syncthreads();
            for (int q = g; q < ns; q += kGGroups) {
                const double2* xq = s_x + q * R;
                double2 a[kGE], b[kGE];
#pragma unroll
                for (int u = 0; u < kGE; ++u) {
                    a[u] = xq[er[u]];
                    b[u] = xq[es[u] < 0 ? 0 : es[u]];
                }
#pragma unroll
                for (int u = 0; u < kGE; ++u) {
                    const double2 p = dconj_mul(a[u], b[u]);
                    acc[u].x += p.x;
                    acc[u].y += p.y;
                }
            }
        }
        __syncthreads();
        if (g > 0) {
#pragma unroll
            for (int u = 0; u < kGE; ++u) s_red[((g - 1) * kGTh + t) * kGE + u] = acc[u];
        }
        __syncthreads();
        if (g == 0) {
#pragma unroll
            for (int u = 0; u < kGE; ++u) {
                if (es[u] < 0) continue;
                double2 v = acc[u];
                for (int gg = 1; gg < kGGroups; ++gg) {
                    const double2 w = s_red[((gg - 1) * kGTh + t) * kGE + u];
                    v.x += w.x;
                    v.y += w.y;
                }
                out[size_t(er[u]) * R + es[u]] = v;
            }
        }
    }
}

// (F_l A)^H F_l A (block 0) and (F_r B)^H F_r B (block 1), upper entries.
template <class Src>
__global__ void __launch_bounds__(kGThreads) k_gram2(Src src) {
    __shared__ double2 s_x[kGStage];
    __shared__ double2 s_red[kGRed];
    const FrameArgs& f = src.get();
    if (!block_frame_ok(f.dev, false)) return;
    const int R = f.r;
    double2* out = f.part + size_t(blockIdx.x) * R * R;
    const float2* X = blockIdx.x == 0 ? f.Ahat : f.Bhat;
    gram_upper(X, R, blockIdx.x == 0 ? f.n1 : f.n2, [](int q) { return q; }, out, s_x, s_red);
}

constexpr int kJC = 32;          // readout samples staged per pass of the right-hand side
static_assert(kSRows * kJC <= kGThreads, "one staged sample per thread");
constexpr int kZ = (kSRows * TSL_MAX_R + kGThreads - 1) / kGThreads;

// Line masks: Gram of the sampled rows of F_l A and the right-hand side
// Phi^H y over sampled rows [kSRows k, kSRows (k+1)); also checks the rows.
// Blocks 0 and 1 compute the Grams of F_l A and F_r B (as k_gram2); blocks
// 2.. are the sampled-row blocks, so one launch covers all of S1's statistics.
template <class Src>
__global__ void __launch_bounds__(kGThreads) k_lstats(Src src) {
    __shared__ double2 s_x[kGStage];
    __shared__ double2 s_red[kGRed];
    __shared__ int s_err;
    const FrameArgs& f = src.get();
    if (!block_frame_ok(f.dev, false)) return;
    const int n1 = f.n1, n2 = f.n2, R = f.r, tid = threadIdx.x;
    if (blockIdx.x < 2) {
        const float2* X = blockIdx.x == 0 ? f.Ahat : f.Bhat;
        gram_upper(X, R, blockIdx.x == 0 ? n1 : n2, [](int q) { return q; },
                   f.part + size_t(blockIdx.x) * R * R, s_x, s_red);
        return;
    }
    const int k = blockIdx.x - 2;
    double2* out = f.part + size_t(2 + k) * R * R;
    if (tid == 0) s_err = 0;
    __syncthreads();
    const int n_rows = frame_rows(f);
    if (k == 0 && tid == 0 && f.n_rows_dev) {
        const int nd = *f.n_rows_dev;
        if (nd < 0 || nd > frame_rows_cap(f)) latch(f.dev, ST_EINVAL);
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
    gram_upper(f.Ahat, R, nq, row_of, out, s_x, s_red);
    // Z[q][r] = sum_j y_qj conj(Bhat_jr): Bhat staged in s_x ([kJC][R]), the
    // samples in s_red ([nq][kJC]), kJC readout samples per pass.
    double2 z[kZ];
#pragma unroll
    for (int u = 0; u < kZ; ++u) z[u] = double2{0.0, 0.0};
    bool fin = true;
    // register prefetch of the next chunk: kPB Bhat values and one sample per thread
    constexpr int kPB = (kJC * TSL_MAX_R + kGThreads - 1) / kGThreads;
    float2 pb[kPB], py = float2{0.f, 0.f};
    auto fetch = [&](int j0) {
        const int nj = min(kJC, n2 - j0);
#pragma unroll
        for (int u = 0; u < kPB; ++u) {
            const int e = tid + u * kGThreads;
            pb[u] = e < nj * R ? f.Bhat[size_t(j0) * R + e] : float2{0.f, 0.f};
        }
        py = float2{0.f, 0.f};
        if (tid < nq * kJC) {
            const int q = tid / kJC, jj = tid % kJC, row = row_of(q);
            if (row >= 0 && jj < nj) {
                py = line_samples(f, q0 + q, row)[j0 + jj];
                fin = fin && finite2(py);
            }
        }
    };
    fetch(0);
    for (int j0 = 0; j0 < n2; j0 += kJC) {
        const int nj = min(kJC, n2 - j0);
        __syncthreads();
#pragma unroll
        for (int u = 0; u < kPB; ++u) {
            const int e = tid + u * kGThreads;
            if (e < nj * R) s_x[e] = double2{pb[u].x, pb[u].y};
        }
        if (tid < nq * kJC) s_red[tid] = double2{py.x, py.y};
        __syncthreads();
        if (j0 + kJC < n2) fetch(j0 + kJC);
#pragma unroll
        for (int u = 0; u < kZ; ++u) {
            const int e = tid + u * kGThreads;
            if (e < nq * R) {
                const int q = e / R, r = e % R;
                const double2* yq = s_red + q * kJC;
                int jj = 0;
                for (; jj + 4 <= nj; jj += 4) {
                    double2 b[4], yv[4];
#pragma unroll
                    for (int w = 0; w < 4; ++w) { b[w] = s_x[(jj + w) * R + r]; yv[w] = yq[jj + w]; }
#pragma unroll
                    for (int w = 0; w < 4; ++w) {
                        const double2 p = dconj_mul(b[w], yv[w]);
                        z[u].x += p.x;
                        z[u].y += p.y;
                    }
                }
                for (; jj < nj; ++jj) {
                    const double2 p = dconj_mul(s_x[jj * R + r], yq[jj]);
                    z[u].x += p.x;
                    z[u].y += p.y;
                }
            }
        }
    }
    if (!fin) atomicCAS(&s_err, 0, ST_ENONFINITE);
    // h = sum_q conj(Ahat_{row_q}) .* Z[q], summed over q in ascending order
    __syncthreads();
#pragma unroll
    for (int u = 0; u < kZ; ++u) {
        const int e = tid + u * kGThreads;
        if (e < nq * R) {
            const int row = row_of(e / R);
            const float2 a = row >= 0 ? f.Ahat[size_t(row) * R + e % R] : float2{0.f, 0.f};
            s_x[e] = dcmulc(z[u], double2{a.x, a.y});
        }
    }
    __syncthreads();
    if (tid < R) {
        double2 h{0.0, 0.0};
        for (int q = 0; q < nq; ++q) { h.x += s_x[q * R + tid].x; h.y += s_x[q * R + tid].y; }
        f.hpart[size_t(k) * R + tid] = h;
    }
    __syncthreads();
    if (tid == 0 && s_err) latch(f.dev, s_err);
}

constexpr int kPW = 32;        // sampled entries staged per window of a point-mask Gram
constexpr int kMaxAcc = 8;     // Gram entries one thread accumulates per pass (point masks)

// Point masks: explicit Phi^H Phi and Phi^H y over mask rows [kPRows k, kPRows (k+1)).
template <class Src>
__global__ void __launch_bounds__(256) k_pstats(Src src) {
    extern __shared__ float2 s_rows[];            // kPW * R double2s
    __shared__ double2 s_yw[kPW];
    __shared__ int s_err;
    const FrameArgs& f = src.get();
    if (!block_frame_ok(f.dev, false)) return;
    const int n1 = f.n1, n2 = f.n2, R = f.r, tid = threadIdx.x;
    const int k = blockIdx.x;
    double2* out = f.part + size_t(2 + k) * R * R;
    if (tid == 0) s_err = 0;
    __syncthreads();
    // Point mask: the sampled entries of rows [i0, i1) taken in windows of kPW
    // candidates; each window stages phi_{(i,j),r} = Ahat_ir Bhat_jr (zero where
    // not sampled) and accumulates Phi^H Phi (r <= s) and Phi^H y.
    const int i0 = k * kPRows;
    if (i0 >= n1) return;
    const int ncand = (min(n1, i0 + kPRows) - i0) * n2;
    double2* s_phi = reinterpret_cast<double2*>(s_rows);   // [kPW][R]
    const int RR = R * R;
    const int npass = cdiv(cdiv(RR, kBlock), kMaxAcc);
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
                const int e = tid + (pass * kMaxAcc + u) * kBlock;
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
            const int e = tid + (pass * kMaxAcc + u) * kBlock;
            if (e < RR && (e / R) <= (e % R)) out[e] = acc[u];
        }
        if (pass == 0 && tid < R) f.hpart[size_t(k) * R + tid] = hacc;
    }
    if (!fin) atomicCAS(&s_err, 0, ST_ENONFINITE);
    __syncthreads();
    if (tid == 0 && s_err) latch(f.dev, s_err);
}

// ---------------------------------------------------------------- solve
__device__ __forceinline__ int pk(int i, int j) { return i * (i + 1) / 2 + j; }   // j <= i

// One wavefront per sequence: every barrier below is a single-wave barrier.
constexpr int kSolveThreads = 64;
constexpr int kPF = 16;      // independent global loads a lane issues before using them

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int m = 32; m > 0; m >>= 1) v += __shfl_xor(v, m, 64);
    return v;
}

template <class Src>
__global__ void __launch_bounds__(kSolveThreads) k_solve(Src src) {
    extern __shared__ double2 s_dyn[];
    __shared__ int s_fail;
    __shared__ double s_piv_lo, s_piv_hi;
    const FrameArgs& f = src.get();
    SeqDev* d = f.dev;
    if (!block_frame_ok(d, false)) {
        if (threadIdx.x == 0) d->frame_ok = 0;
        return;
    }
    const int R = f.r, n1 = f.n1, tid = threadIdx.x;
    const bool lines = f.mode == MODE_LINES;
    const int ns = lines ? cdiv(frame_rows(f), kSRows) : cdiv(n1, kPRows);
    const size_t RR = size_t(R) * R;
    const double2* pa = f.part;               // (F_l A)^H F_l A
    const double2* pb = f.part + RR;          // (F_r B)^H F_r B
    const double2* ps = f.part + 2 * RR;      // partials of the sampled part
    double2* L = s_dyn;                       // packed lower triangle of G, then of its factor
    double2* h = s_dyn + R * (R + 1) / 2;     // right-hand side, then gamma
    const double lam = f.lambda;

    // G = Phi^H Phi + lambda I from the statistics (stored upper entries (j, i), j <= i):
    // the sampled part summed over its partials in slot order, then (lines) times
    // the B Gram entrywise.  Each lane issues kPF independent loads before using them.
    const int npairs = R * (R + 1) / 2;
    for (int e0 = 0; e0 < npairs; e0 += kSolveThreads * kPF) {
        double2 g[kPF], gb[kPF];
        int ii[kPF], jj[kPF];
#pragma unroll
        for (int u = 0; u < kPF; ++u) {
            const int e = e0 + tid + kSolveThreads * u;
            int i = int((sqrt(8.0 * e + 1.0) - 1.0) * 0.5);
            while (i * (i + 1) / 2 > e) --i;
            while ((i + 1) * (i + 2) / 2 <= e) ++i;
            ii[u] = e < npairs ? i : -1;
            jj[u] = e - i * (i + 1) / 2;
            const size_t up = size_t(jj[u]) * R + i;
            g[u] = (e < npairs && ns > 0) ? ps[up] : double2{0.0, 0.0};
            gb[u] = (e < npairs && lines) ? pb[up] : double2{0.0, 0.0};
        }
        for (int k = 1; k < ns; ++k) {
#pragma unroll
            for (int u = 0; u < kPF; ++u) {
                if (ii[u] < 0) continue;
                const double2 v = ps[k * RR + size_t(jj[u]) * R + ii[u]];
                g[u].x += v.x;
                g[u].y += v.y;
            }
        }
#pragma unroll
        for (int u = 0; u < kPF; ++u) {
            if (ii[u] < 0) continue;
            double2 v = lines ? dcmul(g[u], gb[u]) : g[u];
            v.y = -v.y;                          // G_ij = conj(G_ji)
            if (ii[u] == jj[u]) v = double2{v.x + lam, 0.0};
            L[pk(ii[u], jj[u])] = v;
        }
    }
    for (int r = tid; r < R; r += kSolveThreads) {
        double2 hv{0.0, 0.0};
        for (int k = 0; k < ns; ++k) {
            const double2 v = f.hpart[size_t(k) * R + r];
            hv.x += v.x;
            hv.y += v.y;
        }
        h[r] = hv;
    }
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
        const double p = sqrt(dd), ip = 1.0 / p;
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
    // Gershgorin row sums of diag(g)^H M diag(g), M = A^H A and B^H B; the
    // factor's LDS (R(R+1) doubles >= R*R) holds the |entries| of one M at a time.
    double* mag = reinterpret_cast<double*>(s_dyn);
    double* s_ag = s_inv + R;                 // |gamma_r|
    for (int r = tid; r < R; r += kSolveThreads) s_ag[r] = dabs(h[r]);
    __syncthreads();
    double best = 0.0;
    for (int which = 0; which < 2; ++which) {
        const double2* pm = which ? pb : pa;
        __syncthreads();
        for (int e0 = 0; e0 < R * R; e0 += kSolveThreads * kPF) {
            double2 v[kPF];
#pragma unroll
            for (int u = 0; u < kPF; ++u) {
                const int e = e0 + tid + kSolveThreads * u;
                const int r = e / R, c = e % R;
                const size_t up = r <= c ? size_t(r) * R + c : size_t(c) * R + r;
                v[u] = e < R * R ? pm[up] : double2{0.0, 0.0};
            }
#pragma unroll
            for (int u = 0; u < kPF; ++u) {
                const int e = e0 + tid + kSolveThreads * u;
                if (e < R * R) mag[e] = s_ag[e / R] * dabs(v[u]) * s_ag[e % R];
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
    }
}

// ---------------------------------------------------------------- register solve (R <= 32)
// One wavefront, no barriers: lane i keeps row i of G (then of its Cholesky
// factor L) in registers, and column k is broadcast lane to lane with
// readlane at step k.  Rows R..RB-1 are padded with the identity (and a zero
// right-hand side), which leaves gamma unchanged.
__device__ __forceinline__ double readlane_d(double v, int lane) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane(int(b), lane);
    const int hi = __builtin_amdgcn_readlane(int(b >> 32), lane);
    return __longlong_as_double((static_cast<long long>(hi) << 32) | static_cast<unsigned int>(lo));
}
__device__ __forceinline__ double2 readlane_d2(double2 v, int lane) {
    return double2{readlane_d(v.x, lane), readlane_d(v.y, lane)};
}

template <int RB, class Src>
__global__ void __launch_bounds__(kSolveThreads) k_solve_reg(Src src) {
    __shared__ double2 s_l[RB * RB];              // L, row-major, for the back substitution
    const FrameArgs& f = src.get();
    SeqDev* d = f.dev;
    if (!block_frame_ok(d, false)) {
        if (threadIdx.x == 0) d->frame_ok = 0;
        return;
    }
    const int R = f.r, lane = threadIdx.x;
    const bool lines = f.mode == MODE_LINES;
    const int ns = lines ? cdiv(frame_rows(f), kSRows) : cdiv(f.n1, kPRows);
    const size_t RR = size_t(R) * R;
    const double2* pa = f.part;               // (F_l A)^H F_l A
    const double2* pb = f.part + RR;          // (F_r B)^H F_r B
    const double2* ps = f.part + 2 * RR;      // partials of the sampled part
    const double lam = f.lambda;
    const bool live = lane < R;

    // row i = lane of G = Phi^H Phi + lambda I; stored upper entries (j, i) give G_ij = conj(.)
    double2 g[RB];
    sfor<RB>([&](auto jc) {
        constexpr int j = decltype(jc)::value;
        double2 v{0.0, 0.0};
        if (live && j <= lane) {
            const size_t up = size_t(j) * R + lane;
            for (int k = 0; k < ns; ++k) { const double2 w = ps[k * RR + up]; v.x += w.x; v.y += w.y; }
            if (lines) v = dcmul(v, pb[up]);
            v.y = -v.y;
            if (j == lane) v = double2{v.x + lam, 0.0};
        } else if (!live && j == lane) {
            v = double2{1.0, 0.0};
        }
        g[j] = v;
    });
    double2 hv{0.0, 0.0};
    if (live)
        for (int k = 0; k < ns; ++k) { const double2 w = f.hpart[size_t(k) * R + lane]; hv.x += w.x; hv.y += w.y; }

    // right-looking Cholesky (dkk is the same in every lane, so `fail` is uniform)
    bool fail = false;
    double piv_lo = 1e308, piv_hi = 0.0;
    sfor<RB>([&](auto kc) {
        constexpr int k = decltype(kc)::value;
        if (fail) return;
        const double dkk = readlane_d(g[k].x, k);
        if (!(dkk > 0.0) || !isfinite(dkk)) { fail = true; return; }
        const double p = sqrt(dkk), ip = 1.0 / p;
        if (k < R) { piv_lo = fmin(piv_lo, p); piv_hi = fmax(piv_hi, p); }
        if (lane == k) g[k] = double2{p, 0.0};
        else if (lane > k) g[k] = double2{g[k].x * ip, g[k].y * ip};
        sfor<RB>([&](auto jc) {
            constexpr int j = decltype(jc)::value;
            if constexpr (j > k) {
                const double2 ljk = readlane_d2(g[k], j);
                if (lane >= j) {
                    const double2 t = dcmulc(g[k], ljk);      // L_ik conj(L_jk)
                    g[j].x -= t.x;
                    g[j].y -= t.y;
                }
            }
        });
    });
    if (!fail) {
        // L z = h
        sfor<RB>([&](auto kc) {
            constexpr int k = decltype(kc)::value;
            const double ip = 1.0 / readlane_d(g[k].x, k);
            const double2 hk = readlane_d2(hv, k);
            const double2 zk{hk.x * ip, hk.y * ip};
            if (lane == k) hv = zk;
            else if (lane > k) {
                const double2 t = dcmul(g[k], zk);
                hv.x -= t.x;
                hv.y -= t.y;
            }
        });
        // L^H gamma = z, with column `lane` of L read back from LDS
        sfor<RB>([&](auto jc) {
            constexpr int j = decltype(jc)::value;
            if (lane < RB) s_l[lane * RB + j] = (j <= lane) ? g[j] : double2{0.0, 0.0};
        });
        __syncthreads();
        double2 lcol[RB];
        sfor<RB>([&](auto kc) {
            constexpr int k = decltype(kc)::value;
            lcol[k] = (lane < RB) ? s_l[k * RB + lane] : double2{0.0, 0.0};   // L_{k, lane}
        });
        sfor<RB>([&](auto kc) {
            constexpr int k = RB - 1 - decltype(kc)::value;
            const double ip = 1.0 / readlane_d(g[k].x, k);
            const double2 zk = readlane_d2(hv, k);
            const double2 gk{zk.x * ip, zk.y * ip};
            if (lane == k) hv = gk;
            else if (lane < k) {
                const double2 t = dcmulc(gk, lcol[k]);    // conj(L_{k,lane}) gamma_k
                hv.x -= t.x;
                hv.y -= t.y;
            }
        });
    }
    const bool nonfinite = __any(live && !fail && (!isfinite(hv.x) || !isfinite(hv.y)));
    if (fail || nonfinite) {
        if (lane == 0) {
            latch(d, fail ? ST_ENOTPD : ST_ENONFINITE);
            d->frame_ok = 0;
        }
        return;
    }
    // |gamma_s| for every s, then the Gershgorin row sums of diag(g)^H M diag(g)
    const double ga = live ? dabs(hv) : 0.0;
    double gab[RB];
    sfor<RB>([&](auto sc) { gab[decltype(sc)::value] = readlane_d(ga, decltype(sc)::value); });
    double best = 0.0;
    for (int which = 0; which < 2; ++which) {
        const double2* pm = which ? pb : pa;
        double row = 0.0;
        sfor<RB>([&](auto sc) {
            constexpr int c = decltype(sc)::value;
            if (live && c < R) {
                const size_t up = lane <= c ? size_t(lane) * R + c : size_t(c) * R + lane;
                row += dabs(pm[up]) * gab[c];
            }
        });
        best = fmax(best, row * ga);
    }
    sfor<RB>([&](auto sc) { best = fmax(best, readlane_d(best, decltype(sc)::value)); });
    if (live) {
        f.gamma64[lane] = hv;
        const float2 g32{float(hv.x), float(hv.y)};
        f.gamma32[lane] = g32;
        if (f.gamma_out) f.gamma_out[lane] = g32;
    }
    if (lane == 0) {
        const long long tn = d->t + 1;
        const double alpha = lam / double(tn) + best;
        const double abar = d->abar + alpha;
        const double mu = f.step_mode == TSL_STEP_MM ? 1.0 / abar : f.mu_const;
        d->t_new = tn;
        d->alpha = alpha;
        d->abar_new = abar;
        d->mu = mu;
        d->shrink = 1.0 - lam * mu / double(tn);
        d->kappa_proxy = (piv_hi / piv_lo) * (piv_hi / piv_lo);
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
            const float2 av = (i < n1 && r0 + c < R) ? f.A[size_t(i) * R + r0 + c] : float2{0.f, 0.f};
            const float2 gv = (r0 + c < R) ? f.gamma32[r0 + c] : float2{0.f, 0.f};
            stage_copy<2, float2>(
                kOutRC * kOutCols,
                [&](int e) {
                    const int col = e / kOutRC, cc = e % kOutRC, j = j0 + col;
                    return (j < n2 && r0 + cc < R) ? f.B[size_t(j) * R + r0 + cc] : float2{0.f, 0.f};
                },
                [&](int e, float2 v) { s_b[(e % kOutRC) * kOutCols + e / kOutRC] = v; });
            s_a[tid] = cmul(av, gv);
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

constexpr int kSampleStage = 8192;   // factor entries staged per pass (64 KiB)

template <class Src>
__global__ void __launch_bounds__(256) k_sample(Src src) {
#pragma clang fp contract(off)
    extern __shared__ float2 s_a[];              // staged rows of F_l A (kSampleStage entries)
    __shared__ double s_pref[kMaxN];             // weights, then their inclusive prefix
    __shared__ double s_c[TSL_MAX_R];
    __shared__ int s_mark[kMaxN];
    const FrameArgs& f = src.get();
    const int K = f.K_next;
    if (K <= 0) return;
    const int n1 = f.n1, n2 = f.n2, R = f.r, tid = threadIdx.x;
    const int chunk = kSampleStage / R;          // rows per staged pass
    // pass 1: column energies ||ahat_r||^2, each summed in row order
    double acc = 0.0;
    for (int i0 = 0; i0 < n1; i0 += chunk) {
        const int ni = min(chunk, n1 - i0);
        __syncthreads();
        stage_copy<8, float2>(ni * R, [&](int e) { return f.Ahat[size_t(i0) * R + e]; },
                              [&](int e, float2 v) { s_a[e] = v; });
        __syncthreads();
        if (tid < R) {
            int i = 0;
            for (; i + 8 <= ni; i += 8) {          // loads batched; additions still in row order
                float2 a[8];
#pragma unroll
                for (int w = 0; w < 8; ++w) a[w] = s_a[(i + w) * R + tid];
#pragma unroll
                for (int w = 0; w < 8; ++w) {
                    const double ax = a[w].x, ay = a[w].y;
                    const double e = ax * ax + ay * ay;
                    acc = acc + e;
                }
            }
            for (; i < ni; ++i) {
                const float2 a = s_a[i * R + tid];
                const double ax = a.x, ay = a.y;
                const double e = ax * ax + ay * ay;
                acc = acc + e;
            }
        }
    }
    if (tid < R) s_c[tid] = acc;
    // pass 2: w_i = N2 ||abar_i||^2 + R, each summed in column order (the staged
    // rows are still in LDS when the whole factor fits in one pass)
    for (int i0 = 0; i0 < n1; i0 += chunk) {
        const int ni = min(chunk, n1 - i0);
        __syncthreads();
        if (chunk < n1)
            stage_copy<8, float2>(ni * R, [&](int e) { return f.Ahat[size_t(i0) * R + e]; },
                                  [&](int e, float2 v) { s_a[e] = v; });
        __syncthreads();
        for (int il = tid; il < ni; il += blockDim.x) {
            const int i = i0 + il;
            double q = 0.0;
            for (int r = 0; r < R; ++r) {
                const double c = s_c[r];
                if (c > 0.0) {
                    const float2 a = s_a[il * R + r];
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
    }
    __syncthreads();
    if (tid == 0) {                        // sequential in i, loads batched by 8
        double run = 0.0;
        int i = 0;
        for (; i + 8 <= n1; i += 8) {
            double v[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) v[u] = s_pref[i + u];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                run = run + v[u];
                v[u] = run;
            }
#pragma unroll
            for (int u = 0; u < 8; ++u) s_pref[i + u] = v[u];
        }
        for (; i < n1; ++i) {
            run = run + s_pref[i];
            s_pref[i] = run;
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
    // ascending distinct rows: thread tid owns rows [2 tid, 2 tid + 2); exclusive
    // scan of the per-thread counts (integers, so any order is exact)
    const int i0 = 2 * tid;
    const int m0 = (i0 < n1) ? s_mark[i0] : 0, m1 = (i0 + 1 < n1) ? s_mark[i0 + 1] : 0;
    __shared__ int s_scan[kBlock];
    s_scan[tid] = m0 + m1;
    __syncthreads();
    for (int off = 1; off < kBlock; off <<= 1) {
        const int v = tid >= off ? s_scan[tid - off] : 0;
        __syncthreads();
        s_scan[tid] += v;
        __syncthreads();
    }
    const int base = s_scan[tid] - (m0 + m1);
    if (m0) f.rows_next[base] = i0;
    if (m1) f.rows_next[base + m0] = i0 + 1;
    if (tid == kBlock - 1) f.n_next[0] = s_scan[tid];
    if (f.prefix_next)
        for (int i = tid; i < n1; i += blockDim.x) f.prefix_next[i] = s_pref[i];
}

// packed factor, right-hand side / gamma, then 1/L_kk and |gamma_r| (R doubles each)
size_t solve_lds(int R) { return size_t(R * (R + 1) / 2 + R) * sizeof(double2) + 2 * size_t(R) * sizeof(double); }

}  // namespace

void init_kernel_attributes() {
    static std::once_flag once;
    std::call_once(once, [] {
        const int ms = int(size_t(kPW) * TSL_MAX_R * sizeof(double2));
        hipFuncSetAttribute(reinterpret_cast<const void*>(&k_pstats<FrameTable>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, ms);
        hipFuncSetAttribute(reinterpret_cast<const void*>(&k_pstats<OneFrame>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, ms);
        const int mr = int(size_t(kSampleStage) * sizeof(float2));
        hipFuncSetAttribute(reinterpret_cast<const void*>(&k_sample<FrameTable>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, mr);
        hipFuncSetAttribute(reinterpret_cast<const void*>(&k_sample<OneFrame>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, mr);
        const int mv = int(solve_lds(TSL_MAX_R));
        hipFuncSetAttribute(reinterpret_cast<const void*>(&k_solve<FrameTable>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, mv);
        hipFuncSetAttribute(reinterpret_cast<const void*>(&k_solve<OneFrame>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, mv);
    });
}

hipError_t launch_stats(const Batch& b, hipStream_t st) {
    const unsigned ny = b.table ? b.count : 1;
    if (b.mode == MODE_LINES) {
        dim3 grid(2 + cdiv(b.rows_max > 0 ? b.rows_max : 1, kSRows), ny);
        if (b.table) k_lstats<FrameTable><<<grid, kGThreads, 0, st>>>(FrameTable{b.table});
        else k_lstats<OneFrame><<<grid, kGThreads, 0, st>>>(OneFrame{*b.one});
    } else {
        if (b.table) k_gram2<FrameTable><<<dim3(2, ny), kGThreads, 0, st>>>(FrameTable{b.table});
        else k_gram2<OneFrame><<<dim3(2, ny), kGThreads, 0, st>>>(OneFrame{*b.one});
        const size_t lds = size_t(kPW) * b.r_max * sizeof(double2);
        dim3 grid(cdiv(b.n1, kPRows), ny);
        if (b.table) k_pstats<FrameTable><<<grid, kBlock, lds, st>>>(FrameTable{b.table});
        else k_pstats<OneFrame><<<grid, kBlock, lds, st>>>(OneFrame{*b.one});
    }
    return hipGetLastError();
}

template <int RB> void launch_solve_reg(const Batch& b, hipStream_t st) {
    dim3 grid(1, b.table ? b.count : 1);
    if (b.table) k_solve_reg<RB, FrameTable><<<grid, kSolveThreads, 0, st>>>(FrameTable{b.table});
    else k_solve_reg<RB, OneFrame><<<grid, kSolveThreads, 0, st>>>(OneFrame{*b.one});
}

hipError_t launch_solve(const Batch& b, hipStream_t st) {
    if (b.r_max <= 8) { launch_solve_reg<8>(b, st); return hipGetLastError(); }
    if (b.r_max <= 16) { launch_solve_reg<16>(b, st); return hipGetLastError(); }
    if (b.r_max <= 32) { launch_solve_reg<32>(b, st); return hipGetLastError(); }
    dim3 grid(1, b.table ? b.count : 1);
    const size_t lds = solve_lds(b.r_max);
    if (b.table) k_solve<FrameTable><<<grid, kSolveThreads, lds, st>>>(FrameTable{b.table});
    else k_solve<OneFrame><<<grid, kSolveThreads, lds, st>>>(OneFrame{*b.one});
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
    const size_t lds = size_t(kSampleStage) * sizeof(float2);
    if (b.table) k_sample<FrameTable><<<grid, kBlock, lds, st>>>(FrameTable{b.table});
    else k_sample<OneFrame><<<grid, kBlock, lds, st>>>(OneFrame{*b.one});
    return hipGetLastError();
}

}  // namespace tsl
