// Checks the register-resident DCT-II / DCT-III of the spectral kernel, the
// same source compiled for the host, against the O(L^2) definition in long
// double: c_k = a_k sum_l x_l cos(pi (2l + 1) k / (2L)).
#include <cmath>
#include <cstdio>
#include <random>

#include "muffin_device.hpp"

template <typename T, int L>
static double check(std::mt19937_64& rng, bool inverse) {
    std::normal_distribution<double> nd;
    double worst = 0.0;
    for (int trial = 0; trial < 20; ++trial) {
        T v[L];
        long double x[L];
        for (int l = 0; l < L; ++l) { x[l] = (long double)(T)nd(rng); v[l] = (T)x[l]; }
        if (inverse) muffin::dct3_ortho<T, L>(v); else muffin::dct2_ortho<T, L>(v);
        const long double pi = 3.141592653589793238462643383279502884L;
        long double nrm = 0, err = 0;
        for (int k = 0; k < L; ++k) {
            long double ref = 0;
            for (int l = 0; l < L; ++l) {
                if (!inverse) {
                    long double a = k == 0 ? sqrtl(1.0L / L) : sqrtl(2.0L / L);
                    ref += a * cosl(pi * (2 * l + 1) * k / (2.0L * L)) * x[l];
                } else {
                    long double a = l == 0 ? sqrtl(1.0L / L) : sqrtl(2.0L / L);
                    ref += a * cosl(pi * (2 * k + 1) * l / (2.0L * L)) * x[l];
                }
            }
            nrm += ref * ref;
            err += (ref - v[k]) * (ref - v[k]);
        }
        double r = (double)sqrtl(err / nrm);
        if (r > worst) worst = r;
    }
    return worst;
}

template <int L>
static int run(std::mt19937_64& rng) {
    int bad = 0;
    const double e64f = check<double, L>(rng, false), e64i = check<double, L>(rng, true);
    const double e32f = check<float, L>(rng, false), e32i = check<float, L>(rng, true);
    std::printf("L=%3d  f64 dct2 %.2e dct3 %.2e   f32 dct2 %.2e dct3 %.2e\n", L, e64f, e64i, e32f, e32i);
    if (e64f > 1e-14 || e64i > 1e-14) ++bad;
    if (e32f > 2e-6 || e32i > 2e-6) ++bad;
    return bad;
}

int main() {
    std::mt19937_64 rng(1234);
    int bad = run<1>(rng) + run<2>(rng) + run<4>(rng) + run<8>(rng) + run<16>(rng) + run<32>(rng) + run<64>(rng);
    if (!bad) std::printf("ALL OK\n");
    return bad ? 1 : 0;
}
