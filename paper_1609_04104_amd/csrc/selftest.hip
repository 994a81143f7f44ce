// Host-side check of the in-register DFT codelets (no device use).
#include <cmath>

#include "common.hpp"
#include "tsl.h"

namespace {

template <int M, bool INV> double check_one() {
    float2 v[M];
    double ref[2 * M];
    double xr[M], xi[M];
    for (int n = 0; n < M; ++n) {
        xr[n] = std::sin(0.7 * n + 0.3) + 0.25 * n / M;
        xi[n] = std::cos(1.3 * n * n + 0.1) - 0.5;
        v[n] = float2{float(xr[n]), float(xi[n])};
    }
    const double sg = INV ? 1.0 : -1.0;
    for (int k = 0; k < M; ++k) {
        double sr = 0, si = 0;
        for (int n = 0; n < M; ++n) {
            double a = sg * 2.0 * tsl::kPi * double((long(k) * n) % M) / M;
            double c = std::cos(a), s = std::sin(a);
            double fr = double(float(xr[n])), fi = double(float(xi[n]));
            sr += fr * c - fi * s;
            si += fr * s + fi * c;
        }
        ref[2 * k] = sr;
        ref[2 * k + 1] = si;
    }
    tsl::Dft<M, INV>::run(v);
    double num = 0, den = 0;
    for (int k = 0; k < M; ++k) {
        double dr = v[k].x - ref[2 * k], di = v[k].y - ref[2 * k + 1];
        num += dr * dr + di * di;
        den += ref[2 * k] * ref[2 * k] + ref[2 * k + 1] * ref[2 * k + 1];
    }
    return std::sqrt(num / den);
}

template <int M> double check_both() {
    double a = check_one<M, false>(), b = check_one<M, true>();
    return a > b ? a : b;
}

}  // namespace

extern "C" double tsl_selftest_codelets(void) {
    double worst = 0;
    auto upd = [&](double e) { if (!(e <= worst)) worst = e; };
    upd(check_both<2>()); upd(check_both<3>()); upd(check_both<4>()); upd(check_both<5>());
    upd(check_both<6>()); upd(check_both<8>()); upd(check_both<9>()); upd(check_both<10>());
    upd(check_both<12>()); upd(check_both<15>()); upd(check_both<16>()); upd(check_both<18>());
    upd(check_both<20>()); upd(check_both<24>()); upd(check_both<25>()); upd(check_both<32>());
    return worst;
}
