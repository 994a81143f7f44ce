// Shared device helpers: complex arithmetic, compile-time twiddles, unrolled
// loops and the in-register DFT codelets every transform in the library uses.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>
#include <utility>

#define TSL_HD __host__ __device__ __forceinline__

namespace tsl {

// ----------------------------------------------------------------- complex
TSL_HD float2 c2(float x, float y) { return float2{x, y}; }
TSL_HD float2 cadd(float2 a, float2 b) { return float2{a.x + b.x, a.y + b.y}; }
TSL_HD float2 csub(float2 a, float2 b) { return float2{a.x - b.x, a.y - b.y}; }
TSL_HD float2 cmul(float2 a, float2 b) { return float2{a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x}; }
// a * conj(b)
TSL_HD float2 cmulc(float2 a, float2 b) { return float2{a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y}; }
TSL_HD float2 cscale(float2 a, float s) { return float2{a.x * s, a.y * s}; }
TSL_HD float2 cconj(float2 a) { return float2{a.x, -a.y}; }
// multiply by -i (forward) or +i (inverse)
template <bool INV> TSL_HD float2 cmul_mi(float2 a) {
    return INV ? float2{-a.y, a.x} : float2{a.y, -a.x};
}
// acc += a * b
TSL_HD void cfma(float2& acc, float2 a, float2 b) {
    acc.x += a.x * b.x - a.y * b.y;
    acc.y += a.x * b.y + a.y * b.x;
}

// ----------------------------------------------------------------- compile-time trig
constexpr double kPi = 3.14159265358979323846264338327950288;

constexpr double cx_cos_series(double x) {
    double x2 = x * x, term = 1.0, sum = 1.0;
    for (int k = 1; k < 16; ++k) {
        term *= -x2 / double((2 * k - 1) * (2 * k));
        sum += term;
    }
    return sum;
}
constexpr double cx_sin_series(double x) {
    double x2 = x * x, term = x, sum = x;
    for (int k = 1; k < 16; ++k) {
        term *= -x2 / double((2 * k) * (2 * k + 1));
        sum += term;
    }
    return sum;
}
// cos / sin of 2 pi num / den, reduced exactly to the first octant.
constexpr double cx_cos2pi(long num, long den) {
    long n = num % den;
    if (n < 0) n += den;
    long q = (4 * n) / den, rem = 4 * n - q * den;   // angle = pi/2 (q + rem/den)
    double s = 0, c = 0;
    if (2 * rem > den) {
        double y = (kPi / 2) * double(den - rem) / double(den);
        s = cx_cos_series(y); c = cx_sin_series(y);
    } else {
        double x = (kPi / 2) * double(rem) / double(den);
        s = cx_sin_series(x); c = cx_cos_series(x);
    }
    switch (q & 3) {
        case 0: return c;
        case 1: return -s;
        case 2: return -c;
        default: return s;
    }
}
constexpr double cx_sin2pi(long num, long den) { return cx_cos2pi(num * 4 - den, 4 * den); }

// sqrt by Newton iteration (for compile-time scale factors).
constexpr double cx_sqrt(double a) {
    double x = a > 1.0 ? a : 1.0;
    for (int i = 0; i < 64; ++i) x = 0.5 * (x + a / x);
    return x;
}
template <int N> struct InvSqrt {
    static constexpr float value = float(1.0 / cx_sqrt(double(N)));
};

// w_N^e = exp(-+ 2 pi i e / N) as float (sign by INV), evaluated at compile time.
template <int N, int E, bool INV> struct Tw {
    static constexpr float re = float(cx_cos2pi(E, N));
    static constexpr float im = INV ? float(cx_sin2pi(E, N)) : float(-cx_sin2pi(E, N));
};

// ----------------------------------------------------------------- unrolled loops
template <typename F, int... Is>
TSL_HD void sfor_impl(F&& f, std::integer_sequence<int, Is...>) {
    (f(std::integral_constant<int, Is>{}), ...);
}
template <int N, typename F> TSL_HD void sfor(F&& f) {
    sfor_impl(f, std::make_integer_sequence<int, N>{});
}

// ----------------------------------------------------------------- DFT codelets
// In-register DFT of length M on v[0..M), natural order in and out, unscaled.
// Forward kernel exp(-2 pi i k n / M), inverse exp(+...).  Composite lengths use
// one Cooley-Tukey split M = P*Q with input index Q*n1 + n2 and output index
// k1 + P*k2, recursively.
constexpr int codelet_radix(int m) {
    return (m % 4 == 0 && m != 8) ? 4 : (m % 2 == 0) ? 2 : (m % 3 == 0) ? 3 : (m % 5 == 0) ? 5 : m;
}

template <int M, bool INV> struct Dft;

template <bool INV> struct Dft<1, INV> {
    template <typename A> static TSL_HD void run(A&) {}
};
template <bool INV> struct Dft<2, INV> {
    template <typename A> static TSL_HD void run(A& v) {
        float2 a = v[0], b = v[1];
        v[0] = cadd(a, b);
        v[1] = csub(a, b);
    }
};
template <bool INV> struct Dft<3, INV> {
    template <typename A> static TSL_HD void run(A& v) {
        constexpr float h = 0.866025403784438646763723170752936183f;  // sqrt(3)/2
        float2 a = v[0], b = v[1], c = v[2];
        float2 t1 = cadd(b, c);
        float2 t2 = csub(a, cscale(t1, 0.5f));
        float2 d = cscale(csub(b, c), h);
        float2 md = cmul_mi<INV>(d);            // -i d (forward), +i d (inverse)
        v[0] = cadd(a, t1);
        v[1] = cadd(t2, md);
        v[2] = csub(t2, md);
    }
};
template <bool INV> struct Dft<4, INV> {
    template <typename A> static TSL_HD void run(A& v) {
        float2 a = v[0], b = v[1], c = v[2], d = v[3];
        float2 s0 = cadd(a, c), s1 = csub(a, c), s2 = cadd(b, d), s3 = cmul_mi<INV>(csub(b, d));
        v[0] = cadd(s0, s2);
        v[1] = cadd(s1, s3);
        v[2] = csub(s0, s2);
        v[3] = csub(s1, s3);
    }
};
template <bool INV> struct Dft<5, INV> {
    template <typename A> static TSL_HD void run(A& v) {
        constexpr float c1 = float(cx_cos2pi(1, 5)), c2v = float(cx_cos2pi(2, 5));
        constexpr float s1 = float(cx_sin2pi(1, 5)), s2 = float(cx_sin2pi(2, 5));
        float2 a0 = v[0];
        float2 t1 = cadd(v[1], v[4]), t2 = cadd(v[2], v[3]);
        float2 t3 = csub(v[1], v[4]), t4 = csub(v[2], v[3]);
        float2 r1 = cadd(a0, cadd(cscale(t1, c1), cscale(t2, c2v)));
        float2 r2 = cadd(a0, cadd(cscale(t1, c2v), cscale(t2, c1)));
        float2 i1 = cmul_mi<INV>(cadd(cscale(t3, s1), cscale(t4, s2)));   // -i (s1 t3 + s2 t4)
        float2 i2 = cmul_mi<INV>(csub(cscale(t3, s2), cscale(t4, s1)));   // -i (s2 t3 - s1 t4)
        v[0] = cadd(a0, cadd(t1, t2));
        v[1] = cadd(r1, i1);
        v[4] = csub(r1, i1);
        v[2] = cadd(r2, i2);
        v[3] = csub(r2, i2);
    }
};

template <int M, bool INV> struct Dft {
    static constexpr int P = codelet_radix(M);
    static constexpr int Q = M / P;
    static_assert(P * Q == M && P > 1 && Q > 1, "length must be a product of 2, 3, 5");
    template <typename A> static TSL_HD void run(A& v) {
        float2 tmp[M];
        sfor<Q>([&](auto n2c) {
            constexpr int n2 = decltype(n2c)::value;
            float2 a[P];
            sfor<P>([&](auto n1c) { a[decltype(n1c)::value] = v[Q * decltype(n1c)::value + n2]; });
            Dft<P, INV>::run(a);
            sfor<P>([&](auto k1c) {
                constexpr int k1 = decltype(k1c)::value;
                constexpr float wr = Tw<M, (n2 * k1) % M, INV>::re;
                constexpr float wi = Tw<M, (n2 * k1) % M, INV>::im;
                tmp[k1 * Q + n2] = (n2 * k1 == 0) ? a[k1] : cmul(a[k1], float2{wr, wi});
            });
        });
        sfor<P>([&](auto k1c) {
            constexpr int k1 = decltype(k1c)::value;
            float2 b[Q];
            sfor<Q>([&](auto n2c) { b[decltype(n2c)::value] = tmp[k1 * Q + decltype(n2c)::value]; });
            Dft<Q, INV>::run(b);
            sfor<Q>([&](auto k2c) { v[k1 + P * decltype(k2c)::value] = b[decltype(k2c)::value]; });
        });
    }
};

// ----------------------------------------------------------------- transform plans
// Two-pass decomposition N = P * Q of a length-N transform across threads:
// pass 1 runs DFT_P on every n2 < Q (input index Q*n1 + n2), pass 2 runs DFT_Q
// on every k1 < P (output index k1 + P*k2).  T threads cover one transform.
template <int N> struct Plan;
#define TSL_PLAN(N_, P_, Q_)                                         \
    template <> struct Plan<N_> {                                    \
        static constexpr int P = P_, Q = Q_;                         \
        static constexpr int T = (P_ > Q_) ? P_ : Q_;                \
        static_assert(P_ * Q_ == N_, "plan");                        \
    };
TSL_PLAN(8, 4, 2)
TSL_PLAN(16, 4, 4)
TSL_PLAN(24, 6, 4)
TSL_PLAN(32, 8, 4)
TSL_PLAN(40, 8, 5)
TSL_PLAN(48, 8, 6)
TSL_PLAN(64, 8, 8)
TSL_PLAN(80, 10, 8)
TSL_PLAN(96, 12, 8)
TSL_PLAN(100, 10, 10)
TSL_PLAN(120, 12, 10)
TSL_PLAN(128, 16, 8)
TSL_PLAN(144, 12, 12)
TSL_PLAN(160, 16, 10)
TSL_PLAN(192, 16, 12)
TSL_PLAN(200, 20, 10)
TSL_PLAN(240, 16, 15)
TSL_PLAN(256, 16, 16)
TSL_PLAN(288, 18, 16)
TSL_PLAN(320, 20, 16)
TSL_PLAN(384, 24, 16)
TSL_PLAN(400, 20, 20)
TSL_PLAN(480, 24, 20)
TSL_PLAN(512, 32, 16)
#undef TSL_PLAN

// X-macro over the supported lengths (keep in sync with the plans above).
#define TSL_FOR_EACH_N(X) \
    X(8) X(16) X(24) X(32) X(40) X(48) X(64) X(80) X(96) X(100) X(120) X(128) X(144) \
    X(160) X(192) X(200) X(240) X(256) X(288) X(320) X(384) X(400) X(480) X(512)

constexpr int kMaxN = 512;

}  // namespace tsl
