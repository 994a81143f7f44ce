// Building blocks of the LDS-staged, transpose-free 1-D transforms.
//
// A length-N transform (N = P * Q, see Plan<N>) is spread over T = max(P, Q)
// threads.  With input index n = Q*n1 + n2 and output index k = k1 + P*k2:
//   pass 1  thread n2 (< Q) holds x[Q*n1 + n2], n1 < P; DFT_P over n1, then
//           multiplies entry k1 by w_N^(n2*k1);
//   swap    entry (k1, n2) moves through LDS from thread n2 to thread k1;
//   pass 2  thread k1 (< P) holds the Q entries (k1, n2); DFT_Q over n2 gives
//           X[k1 + P*k2], k2 < Q.
// The inverse of such a "k-layout" (thread k1 holding index k1 + P*k2) runs
// the same three steps with the roles of P and Q swapped and lands back in
// the natural layout (thread m1 < Q holding index m1 + Q*m2, m2 < P), so a
// forward-modify-inverse chain needs no reordering.  Every load and store of
// a thread group touches consecutive addresses.
#pragma once

#include "common.hpp"

namespace tsl {

// Twiddle tables w_N^e = exp(-2 pi i e / N), e < N, built at compile time.
template <int N> struct TwTable {
    float x[N];
    float y[N];
};
template <int N> constexpr TwTable<N> make_tw() {
    TwTable<N> t{};
    for (int e = 0; e < N; ++e) {
        t.x[e] = float(cx_cos2pi(e, N));
        t.y[e] = float(-cx_sin2pi(e, N));
    }
    return t;
}
template <int N> __device__ constexpr TwTable<N> g_tw = make_tw<N>();

// Cooperative copy of the length-N twiddle table into LDS.
template <int N> __device__ __forceinline__ void load_tw(float2* s_tw) {
    for (int e = threadIdx.x; e < N; e += blockDim.x) s_tw[e] = float2{g_tw<N>.x[e], g_tw<N>.y[e]};
}

template <bool INV> __device__ __forceinline__ float2 tw_at(const float2* s_tw, int e) {
    float2 w = s_tw[e];
    return INV ? float2{w.x, -w.y} : w;
}

// DFT of length D on v[0..D), then entry k multiplied by w_N^(idx*k).
template <int N, int D, bool INV, int T>
__device__ __forceinline__ void dft_twiddle(float2 (&v)[T], int idx, const float2* s_tw) {
    float2 a[D];
    sfor<D>([&](auto i) { a[decltype(i)::value] = v[decltype(i)::value]; });
    Dft<D, INV>::run(a);
    sfor<D>([&](auto kc) {
        constexpr int k = decltype(kc)::value;
        v[k] = (k == 0) ? a[k] : cmul(a[k], tw_at<INV>(s_tw, idx * k));
    });
}

// DFT of length D on v[0..D).
template <int D, bool INV, int T> __device__ __forceinline__ void dft_only(float2 (&v)[T]) {
    float2 a[D];
    sfor<D>([&](auto i) { a[decltype(i)::value] = v[decltype(i)::value]; });
    Dft<D, INV>::run(a);
    sfor<D>([&](auto i) { v[decltype(i)::value] = a[decltype(i)::value]; });
}

// Odd multiple of `unit` not below n*unit: an LDS pitch that spreads the
// lanes of a wave over both halves of the bank space.
__host__ __device__ constexpr int odd_pitch(int n, int unit) { return ((n % 2) ? n : n + 1) * unit; }

}  // namespace tsl
