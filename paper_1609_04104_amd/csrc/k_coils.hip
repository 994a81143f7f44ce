// Algorithm 3 with C coils (Sec. IV-B, tomographic parallel MRI), line masks.
//
// The regression matrix of coil c no longer factors into a Hadamard product
// (the sensitivity map H_c couples rows and columns), so S1 forms its columns
// explicitly: for each coil the R images H_c .* (a_r b_r^T) go through the 2-D
// transform, and the sampled rows of the results give that coil's part of
// Phi^H Phi and Phi^H y in FP64.  S2 evaluates the residual through the
// synthesis (Phi gamma = F(H_c .* A diag(gamma) B^T) at the samples, by
// linearity): per coil, H_c .* X- is transformed, the sampled rows are replaced
// by y_c minus the prediction and the rest zeroed (Xi_c), the inverse transform
// gives F^{-1}(Xi_c), and Theta = sum_c conj(H_c) .* F^{-1}(Xi_c).  Then
// G_A = Theta conj(B), G_B = Theta^T conj(A) and the updates of Algorithm 3.
// Every kernel here handles one frame of one sequence.
#include <algorithm>
#include <cstdint>

#include "fft_engine.hpp"
#include "kernels.hpp"
#include "tsl.h"

namespace tsl {
namespace {

constexpr int kCB = 256;          // threads per block
constexpr int kCW = 32;           // samples staged per window of the Gram kernel

__device__ __forceinline__ double2 dz() { return double2{0.0, 0.0}; }

// P[r][p][q] = H_c[p][q] A[p][r] B[q][r] for r < R (the images whose
// transforms are the columns of coil c's regression matrix).
__global__ void __launch_bounds__(kCB) k_mc_rank_images(CoilArgs a, int c) {
    const size_t P = size_t(a.n1) * a.n2, total = P * a.r;
    for (size_t e = size_t(blockIdx.x) * kCB + threadIdx.x; e < total; e += size_t(gridDim.x) * kCB) {
        const int r = int(e / P);
        const size_t pq = e % P;
        const int p = int(pq / a.n2), q = int(pq % a.n2);
        const float2 h = a.H[size_t(c) * P + pq];
        const float2 ab = cmul(a.A[size_t(p) * a.r + r], a.B[size_t(q) * a.r + r]);
        a.P[e] = cmul(h, ab);
    }
}

// Block q: the sampled row i = rows[q].  Upper entries (r <= s) of
// sum_j conj(Phi_{c,r}[i, j]) Phi_{c,s}[i, j] into gslot[c][q] and
// sum_j conj(Phi_{c,r}[i, j]) y_c[q][j] into hslot[c][q], in FP64 (products
// of complex64 values widened exactly).  Coil 0's blocks also check the row
// list (range, strictly ascending); every block checks its samples.
__global__ void __launch_bounds__(kCB) k_mc_gram(CoilArgs a, int c) {
    __shared__ double2 s_phi[kCW][TSL_MAX_COIL_R];
    __shared__ double2 s_y[kCW];
    __shared__ int s_err;
    const int q = blockIdx.x, tid = threadIdx.x, R = a.r, n2 = a.n2;
    if (tid == 0) s_err = 0;
    __syncthreads();
    const int row = a.rows[q];
    if (tid == 0) {
        bool ok = row >= 0 && row < a.n1;
        if (q + 1 < a.n_rows) ok = ok && a.rows[q + 1] > row;
        if (c == 0 && !ok) s_err = ST_EINVAL;
    }
    __syncthreads();
    const bool row_ok = row >= 0 && row < a.n1;
    const size_t P = size_t(a.n1) * n2;
    const float2* yq = a.y + (size_t(c) * a.n_rows + q) * n2;
    constexpr int kAcc = (TSL_MAX_COIL_R * (TSL_MAX_COIL_R + 1) / 2 + kCB - 1) / kCB;   // upper entries per thread
    double2 acc[kAcc], hacc = dz();
#pragma unroll
    for (int u = 0; u < kAcc; ++u) acc[u] = dz();
    int ur[kAcc], us[kAcc];
#pragma unroll
    for (int u = 0; u < kAcc; ++u) {          // upper entry e -> (r, s), r <= s, packed by rows
        int e = tid + u * kCB, r = 0;
        const int NU = R * (R + 1) / 2;
        if (e >= NU) { ur[u] = -1; us[u] = -1; continue; }
        while (e >= R - r) { e -= R - r; ++r; }
        ur[u] = r;
        us[u] = r + e;
    }
    bool fin = true;
    for (int j0 = 0; j0 < n2; j0 += kCW) {
        __syncthreads();
        for (int e = tid; e < kCW * R; e += kCB) {
            const int w = e / R, r = e % R, j = j0 + w;
            double2 v = dz();
            if (j < n2 && row_ok) {
                const float2 f = a.P[size_t(r) * P + size_t(row) * n2 + j];
                v = double2{f.x, f.y};
            }
            s_phi[w][r] = v;
        }
        for (int w = tid; w < kCW; w += kCB) {
            const int j = j0 + w;
            double2 v = dz();
            if (j < n2) {
                const float2 f = yq[j];
                fin = fin && isfinite(f.x) && isfinite(f.y);
                v = double2{f.x, f.y};
            }
            s_y[w] = v;
        }
        __syncthreads();
#pragma unroll
        for (int u = 0; u < kAcc; ++u) {
            if (ur[u] < 0) continue;
            const int r = ur[u], s = us[u];
            for (int w = 0; w < kCW; ++w) {
                const double2 pr = s_phi[w][r], ps = s_phi[w][s];
                acc[u].x += pr.x * ps.x + pr.y * ps.y;
                acc[u].y += pr.x * ps.y - pr.y * ps.x;
            }
        }
        if (tid < R)
            for (int w = 0; w < kCW; ++w) {
                const double2 pr = s_phi[w][tid], yy = s_y[w];
                hacc.x += pr.x * yy.x + pr.y * yy.y;
                hacc.y += pr.x * yy.y - pr.y * yy.x;
            }
    }
    const size_t slot = size_t(c) * a.n1 + q;
#pragma unroll
    for (int u = 0; u < kAcc; ++u)
        if (ur[u] >= 0) a.gslot[slot * R * R + size_t(ur[u]) * R + us[u]] = acc[u];
    if (tid < R) a.hslot[slot * R + tid] = hacc;
    if (!fin) atomicCAS(&s_err, 0, ST_ENONFINITE);
    __syncthreads();
    if (tid == 0 && s_err) latch(a.dev, s_err);
}

// S1 and the step size, one block: G = sum of the slots (coil by coil, row by
// row, in order) + lambda I, h likewise; Cholesky G = L L^H in LDS (right
// looking, a barrier per step; a pivot that is not positive and finite
// rejects the frame), gamma = L^{-H} L^{-1} h; alpha_t = lambda/t + g max over
// the two factors of the Gershgorin bound of diag(gamma)^H M diag(gamma),
// M = A^H A or B^H B (FP64), g = max over pixels of sum_c |H_c|^2.
__global__ void __launch_bounds__(kCB) k_mc_solve(CoilArgs a) {
    __shared__ double2 s_g[TSL_MAX_COIL_R * TSL_MAX_COIL_R];
    __shared__ double2 s_h[TSL_MAX_COIL_R];
    __shared__ double s_ag[TSL_MAX_COIL_R];
    __shared__ double s_best[kCB / 64];
    __shared__ int s_fail;
    SeqDev* d = a.dev;
    const int R = a.r, tid = threadIdx.x;
    if (!block_frame_ok(d, false)) {
        if (tid == 0) d->frame_ok = 0;
        return;
    }
    const int ns = a.C * a.n_rows;              // slots, coil-major
    for (int e = tid; e < R * R; e += kCB) {
        const int r = e / R, s = e % R;
        double2 v = dz();
        if (r <= s)
            for (int k = 0; k < ns; ++k) {
                const int c = k / a.n_rows, q = k % a.n_rows;
                const double2 w = a.gslot[(size_t(c) * a.n1 + q) * R * R + e];
                v.x += w.x;
                v.y += w.y;
            }
        if (r == s) v = double2{v.x + a.lambda, 0.0};
        if (r <= s) {
            s_g[r * R + s] = v;
            s_g[s * R + r] = double2{v.x, -v.y};
        }
    }
    if (tid < R) {
        double2 v = dz();
        for (int k = 0; k < ns; ++k) {
            const int c = k / a.n_rows, q = k % a.n_rows;
            const double2 w = a.hslot[(size_t(c) * a.n1 + q) * R + tid];
            v.x += w.x;
            v.y += w.y;
        }
        s_h[tid] = v;
    }
    if (tid == 0) s_fail = 0;
    __syncthreads();
    // G = L L^H, L kept in the lower triangle
    for (int k = 0; k < R; ++k) {
        if (tid == 0) {
            const double dk = s_g[k * R + k].x;
            if (!(dk > 0.0) || !isfinite(dk)) s_fail = ST_ENOTPD;
            s_g[k * R + k] = double2{sqrt(dk > 0.0 && isfinite(dk) ? dk : 1.0), 0.0};
        }
        __syncthreads();
        const double lkk = s_g[k * R + k].x;
        for (int i = k + 1 + tid; i < R; i += kCB) {
            const double2 v = s_g[i * R + k];
            s_g[i * R + k] = double2{v.x / lkk, v.y / lkk};
        }
        __syncthreads();
        const int m = R - k - 1;
        for (int e = tid; e < m * m; e += kCB) {
            const int i = k + 1 + e / m, j = k + 1 + e % m;
            if (j > i) continue;
            const double2 li = s_g[i * R + k], lj = s_g[j * R + k];   // G_ij -= L_ik conj(L_jk)
            double2 v = s_g[i * R + j];
            v.x -= li.x * lj.x + li.y * lj.y;
            v.y -= li.y * lj.x - li.x * lj.y;
            s_g[i * R + j] = v;
        }
        __syncthreads();
    }
    if (s_fail) {
        if (tid == 0) {
            latch(d, s_fail);
            d->frame_ok = 0;
        }
        return;
    }
    if (tid == 0) {
        for (int i = 0; i < R; ++i) {           // L z = h
            double2 v = s_h[i];
            for (int k = 0; k < i; ++k) {
                const double2 l = s_g[i * R + k], z = s_h[k];
                v.x -= l.x * z.x - l.y * z.y;
                v.y -= l.x * z.y + l.y * z.x;
            }
            const double lii = s_g[i * R + i].x;
            s_h[i] = double2{v.x / lii, v.y / lii};
        }
        for (int i = R - 1; i >= 0; --i) {      // L^H gamma = z
            double2 v = s_h[i];
            for (int k = i + 1; k < R; ++k) {
                const double2 l = s_g[k * R + i], g = s_h[k];   // conj(L_ki) gamma_k
                v.x -= l.x * g.x + l.y * g.y;
                v.y -= l.x * g.y - l.y * g.x;
            }
            const double lii = s_g[i * R + i].x;
            s_h[i] = double2{v.x / lii, v.y / lii};
        }
        bool bad = false;
        for (int i = 0; i < R; ++i) bad = bad || !isfinite(s_h[i].x) || !isfinite(s_h[i].y);
        if (bad) s_fail = ST_ENONFINITE;
    }
    __syncthreads();
    if (s_fail) {
        if (tid == 0) {
            latch(d, s_fail);
            d->frame_ok = 0;
        }
        return;
    }
    if (tid < R) {
        const double2 g = s_h[tid];
        s_ag[tid] = sqrt(g.x * g.x + g.y * g.y);
        a.gamma64[tid] = g;
        const float2 g32{float(g.x), float(g.y)};
        a.gamma32[tid] = g32;
        if (a.gamma_out) a.gamma_out[tid] = g32;
    }
    __syncthreads();
    // Gershgorin row sums of diag(g)^H M diag(g): thread (which, r) forms row r of M
    double best = 0.0;
    for (int e = tid; e < 2 * R; e += kCB) {
        const int which = e / R, r = e % R;
        const int n = which ? a.n2 : a.n1;
        const float2* F = which ? a.B : a.A;
        double row = 0.0;
        for (int s = 0; s < R; ++s) {
            double2 m = dz();
            for (int p = 0; p < n; ++p) {
                const float2 x = F[size_t(p) * R + r], y = F[size_t(p) * R + s];
                m.x += double(x.x) * y.x + double(x.y) * y.y;
                m.y += double(x.x) * y.y - double(x.y) * y.x;
            }
            row += s_ag[s] * sqrt(m.x * m.x + m.y * m.y);
        }
        best = fmax(best, row * s_ag[r]);
    }
    for (int m = 32; m > 0; m >>= 1) best = fmax(best, __shfl_xor(best, m, 64));
    if (tid % 64 == 0) s_best[tid / 64] = best;
    __syncthreads();
    if (tid == 0) {
        for (int w = 0; w < kCB / 64; ++w) best = fmax(best, s_best[w]);
        const long long tn = d->t + 1;
        const double alpha = a.lambda / double(tn) + a.gain[0] * best;
        const double abar = d->abar + alpha;
        const double mu = a.step_mode == TSL_STEP_MM ? 1.0 / abar : a.mu_const;
        d->t_new = tn;
        d->alpha = alpha;
        d->abar_new = abar;
        d->mu = mu;
        d->shrink = 1.0 - a.lambda * mu / double(tn);
        d->frame_ok = 1;
    }
}

// Q[c] = H_c .* (A diag(gamma) B^T) for every coil (X- of the frame, then its
// coil-weighted copies).
__global__ void __launch_bounds__(kCB) k_mc_coil_images(CoilArgs a) {
    if (!block_frame_ok(a.dev, true)) return;
    const size_t P = size_t(a.n1) * a.n2;
    for (size_t pq = size_t(blockIdx.x) * kCB + threadIdx.x; pq < P; pq += size_t(gridDim.x) * kCB) {
        const int p = int(pq / a.n2), q = int(pq % a.n2);
        float2 x{0.f, 0.f};
        for (int r = 0; r < a.r; ++r)
            x = cadd(x, cmul(cmul(a.A[size_t(p) * a.r + r], a.gamma32[r]), a.B[size_t(q) * a.r + r]));
        for (int c = 0; c < a.C; ++c) a.Q[size_t(c) * P + pq] = cmul(a.H[size_t(c) * P + pq], x);
    }
}

// Xi_c: the sampled rows become y_c minus the transformed prediction, the
// other rows zero.  Block (c, i) per row of each coil.
__global__ void __launch_bounds__(kCB) k_mc_resid(CoilArgs a) {
    if (!block_frame_ok(a.dev, true)) return;
    const int c = blockIdx.x / a.n1, i = blockIdx.x % a.n1;
    int lo = 0, hi = a.n_rows;                  // position of row i in the ascending row list
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (a.rows[mid] < i) lo = mid + 1; else hi = mid;
    }
    const int q = (lo < a.n_rows && a.rows[lo] == i) ? lo : -1;
    const size_t base = (size_t(c) * a.n1 + i) * a.n2;
    for (int j = threadIdx.x; j < a.n2; j += kCB) {
        float2 v{0.f, 0.f};
        if (q >= 0) {
            const float2 y = a.y[(size_t(c) * a.n_rows + q) * a.n2 + j];
            const float2 k = a.Q[base + j];
            v = float2{y.x - k.x, y.y - k.y};
        }
        a.Q[base + j] = v;
    }
}

// Theta = sum_c conj(H_c) .* F^{-1}(Xi_c), coils added in order.
__global__ void __launch_bounds__(kCB) k_mc_theta(CoilArgs a) {
    if (!block_frame_ok(a.dev, true)) return;
    const size_t P = size_t(a.n1) * a.n2;
    for (size_t pq = size_t(blockIdx.x) * kCB + threadIdx.x; pq < P; pq += size_t(gridDim.x) * kCB) {
        float2 t{0.f, 0.f};
        for (int c = 0; c < a.C; ++c) t = cadd(t, cmulc(a.Q[size_t(c) * P + pq], a.H[size_t(c) * P + pq]));
        a.theta[pq] = t;
    }
}

// G_A[i][r] = sum_j Theta[i][j] conj(B[j][r]) (threads [0, n1 R)) and
// G_B[j][r] = sum_i Theta[i][j] conj(A[i][r]) (threads [n1 R, (n1 + n2) R)),
// FP64 sums.
__global__ void __launch_bounds__(kCB) k_mc_grad(CoilArgs a) {
    if (!block_frame_ok(a.dev, true)) return;
    const int R = a.r, n1 = a.n1, n2 = a.n2;
    const int e = blockIdx.x * kCB + threadIdx.x;
    if (e < n1 * R) {
        const int i = e / R, r = e % R;
        double2 s = dz();
        for (int j = 0; j < n2; ++j) {
            const float2 t = a.theta[size_t(i) * n2 + j], b = a.B[size_t(j) * R + r];
            s.x += double(t.x) * b.x + double(t.y) * b.y;
            s.y += double(t.y) * b.x - double(t.x) * b.y;
        }
        a.GA[size_t(i) * R + r] = float2{float(s.x), float(s.y)};
    } else if (e < (n1 + n2) * R) {
        const int j = (e - n1 * R) / R, r = (e - n1 * R) % R;
        double2 s = dz();
        for (int i = 0; i < n1; ++i) {
            const float2 t = a.theta[size_t(i) * n2 + j], x = a.A[size_t(i) * R + r];
            s.x += double(t.x) * x.x + double(t.y) * x.y;
            s.y += double(t.y) * x.x - double(t.x) * x.y;
        }
        a.GB[size_t(j) * R + r] = float2{float(s.x), float(s.y)};
    }
}

// A <- shrink A + mu G_A conj(gamma), B likewise (both from the factors at
// t-1: the gradients were formed from them); commits alpha_bar and t.
__global__ void __launch_bounds__(kCB) k_mc_update(CoilArgs a) {
    if (!block_frame_ok(a.dev, true)) return;
    SeqDev* d = a.dev;
    const double mu = d->mu, sh = d->shrink;
    const int R = a.r, na = a.n1 * R, nb = a.n2 * R;
    const int e = blockIdx.x * kCB + threadIdx.x;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        d->abar = d->abar_new;
        d->t = d->t_new;
    }
    if (e >= na + nb) return;
    const bool isA = e < na;
    const int k = isA ? e : e - na, r = k % R;
    const double2 g = a.gamma64[r];
    const float2 x = isA ? float2(a.A[k]) : float2(a.B[k]);
    const float2 v = isA ? float2(a.GA[k]) : float2(a.GB[k]);
    const double gr = double(v.x) * g.x + double(v.y) * g.y;     // v conj(gamma_r)
    const double gi = double(v.y) * g.x - double(v.x) * g.y;
    const float2 xn{float(sh * x.x + mu * gr), float(sh * x.y + mu * gi)};
    if (isA) {
        a.A[k] = xn;
        if (a.A_out) a.A_out[k] = xn;
    } else {
        a.B[k] = xn;
        if (a.B_out) a.B_out[k] = xn;
    }
}

// max over pixels of sum_c |H_c|^2, one block.
__global__ void __launch_bounds__(kCB) k_mc_gain(CoilArgs a) {
    __shared__ double s_m[kCB / 64];
    const size_t P = size_t(a.n1) * a.n2;
    double m = 0.0;
    for (size_t pq = threadIdx.x; pq < P; pq += kCB) {
        double s = 0.0;
        for (int c = 0; c < a.C; ++c) {
            const float2 h = a.H[size_t(c) * P + pq];
            s += double(h.x) * h.x + double(h.y) * h.y;
        }
        m = fmax(m, s);
    }
    for (int k = 32; k > 0; k >>= 1) m = fmax(m, __shfl_xor(m, k, 64));
    if (threadIdx.x % 64 == 0) s_m[threadIdx.x / 64] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 0; w < kCB / 64; ++w) m = fmax(m, s_m[w]);
        a.gain[0] = m;
    }
}

unsigned grid_for(size_t n) { return unsigned(std::min<size_t>((n + kCB - 1) / kCB, 8192)); }

}  // namespace

hipError_t launch_coil_gain(const CoilArgs& a, hipStream_t st) {
    k_mc_gain<<<1, kCB, 0, st>>>(a);
    return hipGetLastError();
}

hipError_t launch_coil_step(const CoilArgs& a, hipStream_t st) {
    const size_t P = size_t(a.n1) * a.n2;
    hipError_t e = hipSuccess;
    if (a.n_rows > 0) {
        for (int c = 0; c < a.C && e == hipSuccess; ++c) {
            k_mc_rank_images<<<grid_for(P * a.r), kCB, 0, st>>>(a, c);
            e = hipGetLastError();
            if (e == hipSuccess) e = launch_rowfft(a.n1, a.n2, a.r, a.P, a.P, false, st);
            if (e == hipSuccess) e = launch_colfft(a.n1, a.n2, a.r, a.P, a.P, false, st);
            if (e == hipSuccess) {
                k_mc_gram<<<a.n_rows, kCB, 0, st>>>(a, c);
                e = hipGetLastError();
            }
        }
    }
    if (e != hipSuccess) return e;
    k_mc_solve<<<1, kCB, 0, st>>>(a);
    k_mc_coil_images<<<grid_for(P), kCB, 0, st>>>(a);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if ((e = launch_rowfft(a.n1, a.n2, a.C, a.Q, a.Q, false, st)) != hipSuccess) return e;
    if ((e = launch_colfft(a.n1, a.n2, a.C, a.Q, a.Q, false, st)) != hipSuccess) return e;
    k_mc_resid<<<unsigned(a.C * a.n1), kCB, 0, st>>>(a);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if ((e = launch_rowfft(a.n1, a.n2, a.C, a.Q, a.Q, true, st)) != hipSuccess) return e;
    if ((e = launch_colfft(a.n1, a.n2, a.C, a.Q, a.Q, true, st)) != hipSuccess) return e;
    k_mc_theta<<<grid_for(P), kCB, 0, st>>>(a);
    k_mc_grad<<<grid_for(size_t(a.n1 + a.n2) * a.r), kCB, 0, st>>>(a);
    k_mc_update<<<grid_for(size_t(a.n1 + a.n2) * a.r), kCB, 0, st>>>(a);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if ((e = launch_factor_fft(a.n1, a.r, a.A, a.Ahat, false, st)) != hipSuccess) return e;
    return launch_factor_fft(a.n2, a.r, a.B, a.Bhat, false, st);
}

}  // namespace tsl
