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
    if (c->lay.n_w == 0) return MUFFIN_OK;
    double tab[kMaxWavelets * 32] = {};
    for (int b = 0; b < c->lay.n_w; ++b) {
        const int p = c->params.spatial[b + 1];
        c->wK[b] = 2 * p;
        if (int rc = daubechies_filter(p, c->wh[b])) {
            set_error("Daubechies filter Db%d", p);
            return rc;
        }
        const int K = c->wK[b];
        for (int k = 0; k < K; ++k) {
            tab[32 * b + k] = c->wh[b][k];
            tab[32 * b + 16 + k] = (k & 1) ? -c->wh[b][K - 1 - k] : c->wh[b][K - 1 - k];
        }
    }
    // the device filter table of the all-bases launches, in the iteration's precision
    if (c->shape.dtype == MUFFIN_F64) {
        HIP_TRY(hipMemcpy(P(c, c->lay.wfilt), tab, sizeof(tab), hipMemcpyHostToDevice));
    } else {
        float t32[kMaxWavelets * 32];
        for (int i = 0; i < kMaxWavelets * 32; ++i) t32[i] = float(tab[i]);
        HIP_TRY(hipMemcpy(P(c, c->lay.wfilt), t32, sizeof(t32), hipMemcpyHostToDevice));
    }
    return MUFFIN_OK;
}

namespace {

// consecutive bases' cubes and scratch images lie at fixed strides (elements)
struct DictGeom {
    long zstride = 0;
    long tstride[kMaxDwtLevels] = {};
};

int dict_geom(muffin_ctx* c, DictGeom& G) {
    const int J = c->lay.levels, nw = c->lay.n_w;
    const size_t es = elem_size(c->shape);
    auto stride = [&](size_t off0, size_t off1) { return nw > 1 ? long((off1 - off0) / es) : 0L; };
    G.zstride = stride(c->lay.wz[0], c->lay.wz[nw > 1 ? 1 : 0]);
    for (int j = 1; j < J; ++j) G.tstride[j] = stride(c->lay.wtmp[0][j], c->lay.wtmp[nw > 1 ? 1 : 0][j]);
    for (int b = 1; b < nw; ++b) {
        bool ok = c->lay.wz[b] - c->lay.wz[0] == size_t(b) * size_t(G.zstride) * es;
        for (int j = 1; j < J; ++j)
            ok = ok && c->lay.wtmp[b][j] - c->lay.wtmp[0][j] == size_t(b) * size_t(G.tstride[j]) * es;
        if (!ok) {
            set_error("wavelet workspace regions are not evenly spaced");
            return MUFFIN_EDEVICE;
        }
    }
    return MUFFIN_OK;
}

// the launch descriptor of bases b0 .. b0 + n - 1 (coefficients in z_b)
DwtLevel dict_level(muffin_ctx* c, const DictGeom& G, int b0, int n) {
    const muffin_shape& s = c->shape;
    DwtLevel A{};
    A.ftab = P(c, c->lay.wfilt) + size_t(b0) * 32 * elem_size(s);
    for (int b = 0; b < n; ++b) A.kpack |= unsigned(c->wK[b0 + b] / 2) << (4 * b);
    A.n = n;
    A.L = s.L;
    A.ld = s.nx;
    A.z0 = P(c, c->lay.wz[b0]);
    A.zstride = G.zstride;
    A.z_bs = long(s.ny) * s.nx;
    A.tau = c->params.mu_s / c->params.rho_T;
    A.rho_T = c->params.rho_T;
    return A;
}

// Analysis of the image cube `in` ([L][ny][nx]) by bases b0 .. b0 + A.n - 1,
// level by level (LL through the scratch images); in modes 1 and 2 the
// work-group sums go to wpart from block *pos on (advanced).
int dict_analysis(muffin_ctx* c, const DictGeom& G, DwtLevel A, int b0, const void* in, long* pos) {
    const muffin_shape& s = c->shape;
    const int J = c->lay.levels;
    const int nq = A.mode == 1 ? 3 : (A.mode == 3 ? GRAD_NQ : 1);
    for (int j = 0; j < J; ++j) {
        A.sy = s.ny >> j;
        A.sx = s.nx >> j;
        A.in0 = j == 0 ? in : (const void*)P(c, c->lay.wtmp[b0][j]);
        A.in_bstride = j == 0 ? 0 : G.tstride[j];
        A.in_ld = j == 0 ? s.nx : A.sx;
        A.in_bs = j == 0 ? long(s.ny) * s.nx : long(A.sy) * A.sx;
        A.ll0 = j + 1 < J ? (void*)P(c, c->lay.wtmp[b0][j + 1]) : nullptr;
        A.llstride = j + 1 < J ? G.tstride[j + 1] : 0;
        if (A.mode != 0) {
            // the finest level runs every basis in one work-group per tile and band
            const long nb = dwt_tiles(A.sy, A.sx) * s.L * (j == 0 ? 1 : A.n);
            if (*pos + nb > c->lay.wblocks) {
                set_error("wavelet report sums: %ld work-groups beyond %ld", *pos + nb, c->lay.wblocks);
                return MUFFIN_EDEVICE;
            }
            A.partials = (double*)P(c, c->lay.wpart) + *pos * nq;
            *pos += nb;
        }
        HIP_TRY(launch_dwt_fwd_all(s.dtype, A, c->stream, j == 0));
    }
    return MUFFIN_OK;
}

// Synthesis by bases b0 .. b0 + A.n - 1 of their coefficient cubes (A.z0,
// stride A.zstride, coefficient function A.mode): out += scale * sum_b
// W_b^T f(z_b), the finest level of every basis summed in one launch.
int dict_synthesis(muffin_ctx* c, const DictGeom& G, DwtLevel A, int b0, void* out, double scale) {
    const muffin_shape& s = c->shape;
    const int J = c->lay.levels;
    for (int j = J - 1; j >= 1; --j) {
        A.sy = s.ny >> j;
        A.sx = s.nx >> j;
        A.ll0 = j + 1 < J ? (void*)P(c, c->lay.wtmp[b0][j + 1]) : nullptr;
        A.llstride = j + 1 < J ? G.tstride[j + 1] : 0;
        A.out0 = P(c, c->lay.wtmp[b0][j]);
        A.outstride = G.tstride[j];
        HIP_TRY(launch_dwt_inv_all(s.dtype, A, c->stream));
    }
    A.sy = s.ny;
    A.sx = s.nx;
    A.ll0 = J > 1 ? (void*)P(c, c->lay.wtmp[b0][1]) : nullptr;
    A.llstride = J > 1 ? G.tstride[1] : 0;
    A.out0 = out;
    A.scale = scale;
    HIP_TRY(launch_dwt_inv0_all(s.dtype, A, c->stream));
    return MUFFIN_OK;
}

// steps III and VI of every wavelet basis from X (z_b updated) and their
// terms of B_rest (added to it); with update = false only the B_rest terms
// of the stored z_b.  Analysis: one launch per level for every basis;
// synthesis: one launch per coarser level for every basis, then the finest
// level of every basis summed into B_rest (a fixed summation order).
int dict_run(muffin_ctx* c, bool update) {
    if (c->lay.n_w == 0) return MUFFIN_OK;
    DictGeom G;
    if (int rc = dict_geom(c, G)) return rc;
    const DwtLevel A = dict_level(c, G, 0, c->lay.n_w);
    if (update)
        if (int rc = dict_analysis(c, G, A, 0, P(c, c->lay.x), nullptr)) return rc;
    return dict_synthesis(c, G, A, 0, P(c, c->lay.brest), c->params.rho_T);
}

// The base and element stride of the n_w cubes at p[0 .. n_w - 1], which
// the all-bases launches need evenly spaced.
int spaced(muffin_ctx* c, void* const* p, void** base, long* stride) {
    const int nw = c->lay.n_w;
    const long es = long(elem_size(c->shape));
    *base = p[0];
    *stride = nw > 1 ? long(((char*)p[1] - (char*)p[0]) / es) : 0L;
    for (int b = 1; b < nw; ++b)
        if ((char*)p[b] - (char*)p[0] != b * *stride * es) {
            set_error("the wavelet coefficient cubes of a sweep slot are not evenly spaced");
            return MUFFIN_EDEVICE;
        }
    return MUFFIN_OK;
}

}  // namespace

static_assert(GRAD_NQ <= kWPartQ, "wavelet work-group sums");

int dict_pass(muffin_ctx* c) { return dict_run(c, true); }

int dict_pass_io(muffin_ctx* c, const void* X, void* const* zin, void* const* zout) {
    DictGeom G;
    if (int rc = dict_geom(c, G)) return rc;
    DwtLevel A = dict_level(c, G, 0, c->lay.n_w);
    void *zi, *zo;
    if (int rc = spaced(c, zin, &zi, &A.zstride)) return rc;
    if (int rc = spaced(c, zout, &zo, &A.zostride)) return rc;
    A.z0 = zi;
    A.zo0 = zo == zi ? nullptr : zo;
    if (int rc = dict_analysis(c, G, A, 0, X, nullptr)) return rc;
    return dict_brest_from(c, zout);
}

int dict_brest_from(muffin_ctx* c, void* const* z) {
    DictGeom G;
    if (int rc = dict_geom(c, G)) return rc;
    DwtLevel A = dict_level(c, G, 0, c->lay.n_w);
    void* zb;
    if (int rc = spaced(c, z, &zb, &A.zstride)) return rc;
    A.z0 = zb;
    return dict_synthesis(c, G, A, 0, P(c, c->lay.brest), c->params.rho_T);
}

int dict_adj_x(muffin_ctx* c, void* const* zbar, void* Xb) {
    DictGeom G;
    if (int rc = dict_geom(c, G)) return rc;
    DwtLevel A = dict_level(c, G, 0, c->lay.n_w);
    void* zb;
    if (int rc = spaced(c, zbar, &zb, &A.zstride)) return rc;
    A.z0 = zb;
    A.mode = 1;              // the cotangents as they are
    return dict_synthesis(c, G, A, 0, Xb, 1.0);
}

int dict_adj_b(muffin_ctx* c, const void* Bb, void* const* zbar, void* const* zs, double* acc) {
    DictGeom G;
    if (int rc = dict_geom(c, G)) return rc;
    DwtLevel A = dict_level(c, G, 0, c->lay.n_w);
    void *zb, *sb;
    if (int rc = spaced(c, zbar, &zb, &A.zstride)) return rc;
    if (int rc = spaced(c, zs, &sb, &A.sstride)) return rc;
    A.z0 = zb;
    A.s0 = sb;
    A.mode = 3;
    long pos = 0;
    if (int rc = dict_analysis(c, G, A, 0, Bb, &pos)) return rc;
    HIP_TRY(launch_grad_accum((const double*)P(c, c->lay.wpart), int(pos), acc, c->stream));
    return MUFFIN_OK;
}
int dict_brest(muffin_ctx* c) { return dict_run(c, false); }

// A reporting pass, before steps II-VI: steps III and VI of every wavelet
// basis (z_b updated exactly as dict_pass does) with the elementwise report
// terms summed (FP64) into sums[WREP_SLOT ..] = r^2, E and ||T||^2 parts,
// and the two cubes the report kernel needs:
//   wrep[1] = rho_T sum_b W_b^T (T_b' - T_b),  wrep[2] = sum_b W_b^T Gamma_T,b'.
// Basis by basis (the difference cube wrep[0] holds one basis at a time).
int dict_report_pre(muffin_ctx* c, double* sums) {
    const muffin_shape& s = c->shape;
    DictGeom G;
    if (int rc = dict_geom(c, G)) return rc;
    const size_t cube = voxels(s) * elem_size(s);
    void* D = P(c, c->lay.wrep[0]);
    void* Wd = P(c, c->lay.wrep[1]);
    void* Wg = P(c, c->lay.wrep[2]);
    HIP_TRY(launch_fill_zero(Wd, cube, c->stream));
    HIP_TRY(launch_fill_zero(Wg, cube, c->stream));
    long pos = 0;
    for (int b = 0; b < c->lay.n_w; ++b) {
        DwtLevel A = dict_level(c, G, b, 1);
        A.mode = 1;
        A.d0 = D;
        if (int rc = dict_analysis(c, G, A, b, P(c, c->lay.x), &pos)) return rc;
        // rho_T W_b^T dT_b: the differences as they are (coefficient function 1)
        DwtLevel B = dict_level(c, G, b, 1);
        B.z0 = D;
        B.zstride = 0;
        B.mode = 1;
        if (int rc = dict_synthesis(c, G, B, b, Wd, c->params.rho_T)) return rc;
    }
    HIP_TRY(launch_reduce_final((const double*)P(c, c->lay.wpart), int(pos), 3, sums, c->stream));
    // W^T Gamma_T,b' = rho_T W_b^T (-clip(z_b')), every basis at once
    DwtLevel A = dict_level(c, G, 0, c->lay.n_w);
    A.mode = 2;
    return dict_synthesis(c, G, A, 0, Wg, c->params.rho_T);
}

// sum_b ||W_b P||_1 for P = max(0, z_P) (the objective's wavelet terms):
// P into the scratch cube wrep[1], its analysis by every basis, into *sum1.
int dict_report_l1(muffin_ctx* c, const void* zP, double* sum1) {
    const muffin_shape& s = c->shape;
    DictGeom G;
    if (int rc = dict_geom(c, G)) return rc;
    void* Pc = P(c, c->lay.wrep[1]);
    HIP_TRY(launch_positive(s.dtype, zP, Pc, voxels(s), c->stream));
    DwtLevel A = dict_level(c, G, 0, c->lay.n_w);
    A.mode = 2;
    long pos = 0;
    if (int rc = dict_analysis(c, G, A, 0, Pc, &pos)) return rc;
    HIP_TRY(launch_reduce_final((const double*)P(c, c->lay.wpart), int(pos), 1, sum1, c->stream));
    return MUFFIN_OK;
}

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
