// Wavelet bases of the spatial dictionary W_s (Section 4: the Dirac basis
// and the orthonormal Daubechies bases Db1-Db8): the scaling filters,
// derived on the host in FP64, and the per-pass driver of the DWT kernels
// (muffin_wavelet.hip).
#include <hip/hip_runtime.h>

#include <cmath>
#include <complex>

#include "muffin.h"
#include "muffin_ctx.hpp"
#include "muffin_kernels.hpp"
#include "muffin_layout.hpp"

namespace muffin {

using cd = std::complex<double>;

// Daubechies' construction: |m0(w)|^2 = cos(w/2)^(2p) Q(sin(w/2)^2),
// Q(y) = sum_{k<p} C(p-1+k, k) y^k.  The roots y_i of Q (Durand-Kerner
// iteration) map to root pairs z, 1/z of z^2 - (2 - 4 y_i) z + 1; the filter
// polynomial is (1 + z)^p prod (z - z_i) over the roots with |z_i| > 1, and
// h_k (k < 2p) its z^k coefficients scaled to sum sqrt(2).
int daubechies_filter(int p, double* h) {
    if (p < 1 || p > 8) return MUFFIN_EINVAL;
    double q[8];                                 // Q's coefficients, ascending
    for (int k = 0; k < p; ++k) {
        double c = 1.0;                          // C(p-1+k, k)
        for (int i = 1; i <= k; ++i) c = c * double(p - 1 + i) / double(i);
        q[k] = c;
    }
    const int deg = p - 1;
    cd roots[8];
    if (deg > 0) {
        auto Q = [&](cd y) {                     // monic Q / q[deg], Horner
            cd v = 1.0;
            for (int k = deg - 1; k >= 0; --k) v = v * y + q[k] / q[deg];
            return v;
        };
        for (int i = 0; i < deg; ++i) roots[i] = std::pow(cd(0.4, 0.9), double(i));
        for (int it = 0; it < 500; ++it) {
            double moved = 0.0;
            for (int i = 0; i < deg; ++i) {
                cd den = 1.0;
                for (int j = 0; j < deg; ++j)
                    if (j != i) den *= roots[i] - roots[j];
                const cd step = Q(roots[i]) / den;
                roots[i] -= step;
                moved = std::fmax(moved, std::abs(step) / std::fmax(1.0, std::abs(roots[i])));
            }
            if (moved < 1e-16) break;
        }
    }
    cd poly[16] = {};
    int n = 1;
    poly[0] = 1.0;
    auto mul_linear = [&](cd c0, cd c1) {        // poly *= c0 + c1 z
        for (int k = n; k >= 0; --k) poly[k] = (k < n ? poly[k] * c0 : cd(0.0)) + (k > 0 ? poly[k - 1] * c1 : cd(0.0));
        ++n;
    };
    for (int i = 0; i < p; ++i) mul_linear(1.0, 1.0);
    for (int i = 0; i < deg; ++i) {
        const cd b = 2.0 - 4.0 * roots[i];
        const cd disc = std::sqrt(b * b - 4.0);
        const cd z1 = 0.5 * (b + disc), z2 = 0.5 * (b - disc);
        const cd zr = std::abs(z1) > 1.0 ? z1 : z2;
        mul_linear(-zr, 1.0);
    }
    double sum = 0.0;
    for (int k = 0; k < 2 * p; ++k) sum += poly[k].real();
    for (int k = 0; k < 2 * p; ++k) h[k] = poly[k].real() * (std::sqrt(2.0) / sum);
    return MUFFIN_OK;
}

int dict_setup(muffin_ctx* c) {
    for (int b = 0; b < c->lay.n_w; ++b) {
        const int p = c->params.spatial[b + 1];
        c->wK[b] = 2 * p;
        if (int rc = daubechies_filter(p, c->wh[b])) {
            set_error("Daubechies filter Db%d", p);
            return rc;
        }
    }
    return MUFFIN_OK;
}

// steps III and VI of every wavelet basis from X (z_b updated) and their
// terms of B_rest (added to it); with update = false only the B_rest terms
// of the stored z_b
static int dict_run(muffin_ctx* c, bool update) {
    const muffin_shape& s = c->shape;
    const int J = c->lay.levels;
    const double tau = c->params.mu_s / c->params.rho_T;
    const long vb = long(s.ny) * s.nx;
    for (int b = 0; b < c->lay.n_w; ++b) {
        char* z = P(c, c->lay.wz[b]);
        const double* h = c->wh[b];
        const int K = c->wK[b];
        if (update) {
            for (int j = 0; j < J; ++j) {
                const int sy = s.ny >> j, sx = s.nx >> j;
                const void* in = j == 0 ? (const void*)P(c, c->lay.x) : (const void*)P(c, c->lay.wtmp[j]);
                void* ll = j + 1 < J ? (void*)P(c, c->lay.wtmp[j + 1]) : nullptr;
                HIP_TRY(launch_dwt_fwd(s.dtype, K, h, in, j == 0 ? s.nx : sx, j == 0 ? vb : long(sy) * sx, z,
                                       s.nx, vb, ll, sy, sx, s.L, tau, c->stream));
            }
        }
        for (int j = J - 1; j >= 0; --j) {
            const int sy = s.ny >> j, sx = s.nx >> j;
            const void* ll = j + 1 < J ? (const void*)P(c, c->lay.wtmp[j + 1]) : nullptr;
            if (j == 0)
                HIP_TRY(launch_dwt_inv(s.dtype, K, h, ll, z, s.nx, vb, P(c, c->lay.brest), s.nx, vb, sy, sx, s.L,
                                       tau, c->params.rho_T, true, c->stream));
            else
                HIP_TRY(launch_dwt_inv(s.dtype, K, h, ll, z, s.nx, vb, P(c, c->lay.wtmp[j]), sx, long(sy) * sx,
                                       sy, sx, s.L, tau, 1.0, false, c->stream));
        }
    }
    return MUFFIN_OK;
}

int dict_pass(muffin_ctx* c) { return dict_run(c, true); }
int dict_brest(muffin_ctx* c) { return dict_run(c, false); }

// keep T_b, Gamma_T,b of every wavelet basis under new parameters (as the
// re-encoding of z_T): z_b <- soft(z_b, tau) + ratio clip(z_b, tau)
int dict_reencode(muffin_ctx* c, double ratio, double tau) {
    for (int b = 0; b < c->lay.n_w; ++b)
        HIP_TRY(launch_reencode(c->shape.dtype, nullptr, P(c, c->lay.wz[b]), nullptr, nullptr, voxels(c->shape),
                                1.0, ratio, tau, 0.0, c->stream));
    return MUFFIN_OK;
}

}  // namespace muffin

extern "C" int muffin_wavelet_filter(int p, double* h) {
    if (!h || p < MUFFIN_DB1 || p > MUFFIN_DB8) {
        muffin::set_error("muffin_wavelet_filter: p = %d outside [1, 8] or h NULL", p);
        return MUFFIN_EINVAL;
    }
    return muffin::daubechies_filter(p, h);
}
