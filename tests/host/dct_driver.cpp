// Checks the register-resident transforms of the spectral kernels, the same
// source compiled for the host, against their O(L^2) definitions in long
// double:
//   DCT-II  c_k = a_k sum_l x_l cos(pi (2l + 1) k / (2L)), a_0 = sqrt(1/L), a_k = sqrt(2/L)
//   DCT-III its transpose (the inverse)
//   DCT-IV  y_k = sqrt(2/L) sum_l x_l cos(pi (2l + 1)(2k + 1) / (4L))
// and the 2N-band form of the DCT-II (256 and 128 bands): a butterfly of the
// two halves (u_n = (x_n + x_{2N-1-n}) / sqrt 2, w_n = (x_n - x_{2N-1-n}) /
// sqrt 2) then DCT-II(u) for the even and DCT-IV(w) for the odd
// coefficients, and back, in the kernels' order of operations.
#include <cmath>
#include <cstdio>
#include <random>

#include "muffin_device.hpp"

enum Kind { DCT2 = 0, DCT3 = 1, DCT4 = 2 };

static long double basis(int kind, int L, int k, int l) {
    const long double pi = 3.141592653589793238462643383279502884L;
    if (kind == DCT2) return (k == 0 ? sqrtl(1.0L / L) : sqrtl(2.0L / L)) * cosl(pi * (2 * l + 1) * k / (2.0L * L));
    if (kind == DCT3) return (l == 0 ? sqrtl(1.0L / L) : sqrtl(2.0L / L)) * cosl(pi * (2 * k + 1) * l / (2.0L * L));
    return sqrtl(2.0L / L) * cosl(pi * (2 * l + 1) * (2 * k + 1) / (4.0L * L));
}

template <typename T, int L>
static double check(std::mt19937_64& rng, int kind) {
    std::normal_distribution<double> nd;
    double worst = 0.0;
    for (int trial = 0; trial < 20; ++trial) {
        T v[L];
        long double x[L];
        for (int l = 0; l < L; ++l) { x[l] = (long double)(T)nd(rng); v[l] = (T)x[l]; }
        if (kind == DCT2) muffin::dct2_ortho<T, L>(v);
        else if (kind == DCT3) muffin::dct3_ortho<T, L>(v);
        else muffin::dct4_ortho<T, L>(v);
        long double nrm = 0, err = 0;
        for (int k = 0; k < L; ++k) {
            long double ref = 0;
            for (int l = 0; l < L; ++l) ref += basis(kind, L, k, l) * x[l];
            nrm += ref * ref;
            err += (ref - v[k]) * (ref - v[k]);
        }
        const double r = (double)sqrtl(err / nrm);
        if (r > worst) worst = r;
    }
    return worst;
}

// The 2N-band DCT-II and its inverse through the two halves, as the kernels
// do it at 256 bands (N = 128) and 128 bands (N = 64); the exchange between
// their two waves is a plain copy here.
template <typename T, int N>
static void split2n(T (&lo)[N], T (&hi)[N], bool inverse) {
    const T rs = T(0.70710678118654752440084436210484903928);
    T a[N], b[N];
    for (int i = 0; i < N; ++i) { a[i] = lo[i]; b[i] = hi[i]; }
    if (!inverse) {
        // lo: bands 0..N-1, hi: bands N..2N-1
        for (int n = 0; n < N; ++n) lo[n] = (a[n] + b[N - 1 - n]) * rs;      // u
        for (int j = 0; j < N; ++j) hi[j] = (a[j] - b[N - 1 - j]) * rs;      // w
        muffin::dct2_ortho<T, N>(lo);                                       // c_{2k}
        muffin::dct4_ortho<T, N>(hi);                                       // c_{2k+1}
    } else {
        muffin::dct3_ortho<T, N>(a);                                        // u
        muffin::dct4_ortho<T, N>(b);                                        // w
        for (int n = 0; n < N; ++n) lo[n] = (a[n] + b[n]) * rs;            // x_n
        for (int n = 0; n < N; ++n) hi[N - 1 - n] = (a[n] - b[n]) * rs;    // x_{2N-1-n}
    }
}

template <typename T, int N>
static double check_split(std::mt19937_64& rng, bool inverse) {
    constexpr int L = 2 * N;
    std::normal_distribution<double> nd;
    double worst = 0.0;
    for (int trial = 0; trial < 10; ++trial) {
        T lo[N], hi[N];
        long double x[L];
        for (int l = 0; l < L; ++l) x[l] = (long double)(T)nd(rng);
        if (!inverse) {
            for (int i = 0; i < N; ++i) { lo[i] = (T)x[i]; hi[i] = (T)x[N + i]; }
        } else {
            // coefficient c_{2k} in lo[k], c_{2k+1} in hi[k]
            for (int k = 0; k < N; ++k) { lo[k] = (T)x[2 * k]; hi[k] = (T)x[2 * k + 1]; }
        }
        split2n<T, N>(lo, hi, inverse);
        long double nrm = 0, err = 0;
        for (int k = 0; k < L; ++k) {
            long double ref = 0;
            for (int l = 0; l < L; ++l) ref += basis(inverse ? DCT3 : DCT2, L, k, l) * x[l];
            const long double got = inverse ? (k < N ? lo[k] : hi[k - N]) : (k % 2 == 0 ? lo[k / 2] : hi[k / 2]);
            nrm += ref * ref;
            err += (ref - got) * (ref - got);
        }
        const double r = (double)sqrtl(err / nrm);
        if (r > worst) worst = r;
    }
    return worst;
}

// The kernels' exchange of the forward and inverse butterflies (two rounds
// of N/2 registers through LDS, slots by round_reg / slot_of) with the two
// waves' LDS rows as host arrays: it must give the plain butterflies of
// split2n bit for bit.
template <typename T, int N>
static bool exchange_matches(std::mt19937_64& rng) {
    using muffin::round_reg;
    using muffin::slot_of;
    const T rs = T(0.70710678118654752440084436210484903928);
    std::normal_distribution<double> nd;
    for (int inverse = 0; inverse < 2; ++inverse) {
        T v0[N], v1[N], lo[N], hi[N];
        for (int i = 0; i < N; ++i) { v0[i] = lo[i] = (T)nd(rng); v1[i] = hi[i] = (T)nd(rng); }
        for (int q = 0; q < 2; ++q) {
            T x0[N / 2], x1[N / 2];
            for (int i = 0; i < N / 2; ++i) { x0[i] = v0[round_reg<N>(q, i)]; x1[i] = v1[round_reg<N>(q, i)]; }
            for (int i = 0; i < N / 2; ++i) {
                const int n = round_reg<N>(q, i);
                v0[n] = (v0[n] + x1[inverse ? slot_of<N>(n) : slot_of<N>(N - 1 - n)]) * rs;
            }
            for (int i = 0; i < N / 4; ++i) {
                const int j = q == 0 ? i : N / 4 + i;
                const T a = v1[j], b = v1[N - 1 - j];
                if (!inverse) {
                    v1[j] = (x0[slot_of<N>(j)] - b) * rs;
                    v1[N - 1 - j] = (x0[slot_of<N>(N - 1 - j)] - a) * rs;
                } else {
                    v1[N - 1 - j] = (x0[slot_of<N>(j)] - a) * rs;
                    v1[j] = (x0[slot_of<N>(N - 1 - j)] - b) * rs;
                }
            }
        }
        // the plain butterflies on the same values
        T a[N], b[N];
        for (int i = 0; i < N; ++i) { a[i] = lo[i]; b[i] = hi[i]; }
        for (int n = 0; n < N; ++n) {
            if (!inverse) { lo[n] = (a[n] + b[N - 1 - n]) * rs; hi[n] = (a[n] - b[N - 1 - n]) * rs; }
            else { lo[n] = (a[n] + b[n]) * rs; hi[N - 1 - n] = (a[n] - b[n]) * rs; }
        }
        for (int i = 0; i < N; ++i)
            if (v0[i] != lo[i] || v1[i] != hi[i]) return false;
    }
    return true;
}

template <int L>
static int run(std::mt19937_64& rng) {
    int bad = 0;
    double e[2][3];
    for (int kind = 0; kind < 3; ++kind) {
        e[0][kind] = check<double, L>(rng, kind);
        e[1][kind] = check<float, L>(rng, kind);
    }
    std::printf("L=%3d  f64 dct2 %.2e dct3 %.2e dct4 %.2e   f32 dct2 %.2e dct3 %.2e dct4 %.2e\n", L, e[0][0],
                e[0][1], e[0][2], e[1][0], e[1][1], e[1][2]);
    for (int kind = 0; kind < 3; ++kind) {
        if (e[0][kind] > 1e-14) ++bad;
        if (e[1][kind] > 2e-6) ++bad;
    }
    return bad;
}

int main() {
    std::mt19937_64 rng(1234);
    int bad = run<1>(rng) + run<2>(rng) + run<4>(rng) + run<8>(rng) + run<16>(rng) + run<32>(rng) + run<64>(rng) +
              run<128>(rng);
    const double s64f = check_split<double, 128>(rng, false), s64i = check_split<double, 128>(rng, true);
    const double s32f = check_split<float, 128>(rng, false), s32i = check_split<float, 128>(rng, true);
    std::printf("L=256 (two halves)  f64 dct2 %.2e dct3 %.2e   f32 dct2 %.2e dct3 %.2e\n", s64f, s64i, s32f, s32i);
    if (s64f > 1e-14 || s64i > 1e-14) ++bad;
    if (s32f > 2e-6 || s32i > 2e-6) ++bad;
    const double h64f = check_split<double, 64>(rng, false), h64i = check_split<double, 64>(rng, true);
    const double h32f = check_split<float, 64>(rng, false), h32i = check_split<float, 64>(rng, true);
    std::printf("L=128 (two halves)  f64 dct2 %.2e dct3 %.2e   f32 dct2 %.2e dct3 %.2e\n", h64f, h64i, h32f, h32i);
    if (h64f > 1e-14 || h64i > 1e-14) ++bad;
    if (h32f > 2e-6 || h32i > 2e-6) ++bad;
    const bool ex = exchange_matches<float, 128>(rng) && exchange_matches<double, 128>(rng) &&
                    exchange_matches<float, 64>(rng) && exchange_matches<double, 64>(rng);
    std::printf("two-wave exchange (N = 128, 64): %s\n", ex ? "bitwise the plain butterflies" : "MISMATCH");
    if (!ex) ++bad;
    if (!bad) std::printf("ALL OK\n");
    return bad ? 1 : 0;
}
