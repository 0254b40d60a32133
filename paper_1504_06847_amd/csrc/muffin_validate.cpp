// Host-only part of the C ABI: parameter defaults, validation, workspace
// sizing and the thread-local error message.  No HIP runtime calls, so it
// builds and runs without a GPU (and under the host sanitizers).
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <vector>

#include "muffin.h"
#include "muffin_layout.hpp"

namespace muffin {

static thread_local char g_err[512] = "";

void set_error(const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
}

static bool pow2_in_range(int n) { return n >= 8 && n <= 4096 && (n & (n - 1)) == 0; }

int validate_shape(const muffin_shape* s) {
    if (!s) { set_error("shape is NULL"); return MUFFIN_EINVAL; }
    if (s->L < 1) { set_error("L = %d < 1", s->L); return MUFFIN_EINVAL; }
    if (s->nx <= 0 || s->ny <= 0) { set_error("image size %d x %d is not positive", s->ny, s->nx); return MUFFIN_EINVAL; }
    if (!pow2_in_range(s->nx) || !pow2_in_range(s->ny)) {
        set_error("image size %d x %d: each side must be a power of two in [8, 4096]", s->ny, s->nx);
        return MUFFIN_EUNSUPPORTED;
    }
    if (s->L > MUFFIN_MAX_BANDS) {
        set_error("L = %d exceeds MUFFIN_MAX_BANDS = %d", s->L, MUFFIN_MAX_BANDS);
        return MUFFIN_EUNSUPPORTED;
    }
    if (s->L > 32 && (s->L & (s->L - 1)) != 0) {
        set_error("L = %d: band counts above 32 must be powers of two", s->L);
        return MUFFIN_EUNSUPPORTED;
    }
    if (s->dtype != MUFFIN_F32 && s->dtype != MUFFIN_F64) {
        set_error("dtype %d is neither MUFFIN_F32 nor MUFFIN_F64", s->dtype);
        return MUFFIN_EUNSUPPORTED;
    }
    const double vox = double(s->L) * s->nx * s->ny;
    if (vox > 4.0e9) { set_error("cube of %.3g voxels is too large", vox); return MUFFIN_EUNSUPPORTED; }
    return MUFFIN_OK;
}

int validate_params(const muffin_params* p) {
    if (!p) { set_error("params is NULL"); return MUFFIN_EINVAL; }
    const double mus[3] = {p->mu_eps, p->mu_s, p->mu_nu};
    const char* mun[3] = {"mu_eps", "mu_s", "mu_nu"};
    for (int i = 0; i < 3; ++i) {
        if (!std::isfinite(mus[i]) || mus[i] < 0.0) {
            set_error("%s = %g must be finite and >= 0", mun[i], mus[i]);
            return MUFFIN_EINVAL;
        }
    }
    const double rhos[4] = {p->rho_P, p->rho_T, p->rho_V, p->rho_S};
    const char* rhon[4] = {"rho_P", "rho_T", "rho_V", "rho_S"};
    for (int i = 0; i < 4; ++i) {
        if (!std::isfinite(rhos[i]) || rhos[i] <= 0.0) {
            set_error("%s = %g must be finite and > 0", rhon[i], rhos[i]);
            return MUFFIN_EINVAL;
        }
    }
    if (!std::isfinite(p->eps_abs) || p->eps_abs < 0.0 || !std::isfinite(p->eps_rel) || p->eps_rel < 0.0) {
        set_error("eps_abs = %g, eps_rel = %g must be finite and >= 0", p->eps_abs, p->eps_rel);
        return MUFFIN_EINVAL;
    }
    if (p->check_every < 1) { set_error("check_every = %d < 1", p->check_every); return MUFFIN_EINVAL; }
    if (p->n_s < 1 || p->n_s > 1 + kMaxWavelets) {
        set_error("n_s = %d spatial bases: 1 to %d are supported", p->n_s, 1 + kMaxWavelets);
        return MUFFIN_EUNSUPPORTED;
    }
    if (p->spatial[0] != MUFFIN_DIRAC) {
        set_error("spatial[0] = %d: the first spatial basis must be MUFFIN_DIRAC", p->spatial[0]);
        return MUFFIN_EUNSUPPORTED;
    }
    for (int b = 1; b < p->n_s; ++b) {
        if (p->spatial[b] < MUFFIN_DB1 || p->spatial[b] > MUFFIN_DB8) {
            set_error("spatial[%d] = %d is not one of MUFFIN_DB1 .. MUFFIN_DB8", b, p->spatial[b]);
            return MUFFIN_EUNSUPPORTED;
        }
    }
    if (p->n_nu < 1 || p->n_nu > kMaxSpectral) {
        set_error("n_nu = %d spectral bases: 1 to %d are supported", p->n_nu, kMaxSpectral);
        return MUFFIN_EUNSUPPORTED;
    }
    for (int j = 0; j < p->n_nu; ++j) {
        const int b = p->spectral[j];
        if (b != MUFFIN_DCT2_ORTHO && b != MUFFIN_CHEBYSHEV && b != MUFFIN_SPECTRAL_DIRAC) {
            set_error("spectral[%d] = %d is not a spectral basis code", j, b);
            return MUFFIN_EUNSUPPORTED;
        }
        for (int i = 0; i < j; ++i) {
            if (p->spectral[i] == b) {
                set_error("spectral[%d] = spectral[%d] = %d: the bases of a union are distinct", i, j, b);
                return MUFFIN_EINVAL;
            }
        }
    }
    return MUFFIN_OK;
}

bool spectral_dense(const muffin_shape& s, const muffin_params& p) {
    const bool pow2 = (s.L & (s.L - 1)) == 0;
    return !(p.n_nu == 1 && p.spectral[0] == MUFFIN_DCT2_ORTHO && pow2);
}

int spectral_basis_ld(int code, int L, long double* W) {
    if (!W || L < 1 || L > 4096) { set_error("spectral basis: bad L = %d or NULL output", L); return MUFFIN_EINVAL; }
    const long double pi = 3.141592653589793238462643383279502884L;
    if (code == MUFFIN_DCT2_ORTHO) {
        for (int l = 0; l < L; ++l)
            for (int k = 0; k < L; ++k)
                W[size_t(l) * L + k] = (k == 0 ? sqrtl(1.0L / L) : sqrtl(2.0L / L)) *
                                       cosl(pi * (long double)((2 * l + 1) * k) / (2.0L * L));
        return MUFFIN_OK;
    }
    if (code == MUFFIN_SPECTRAL_DIRAC) {
        for (int l = 0; l < L; ++l)
            for (int k = 0; k < L; ++k) W[size_t(l) * L + k] = l == k ? 1.0L : 0.0L;
        return MUFFIN_OK;
    }
    if (code != MUFFIN_CHEBYSHEV) { set_error("spectral basis code %d unknown", code); return MUFFIN_EINVAL; }
    // The polynomials of degree < L at the band positions x_l, orthonormal
    // under the plain sum over the bands: the span of T_0 .. T_k is that of
    // 1, x, .., x^k, so the orthonormalised Chebyshev columns are the
    // discrete orthonormal polynomials, built by the Lanczos recurrence on
    // diag(x): p_0 = 1 / sqrt(L), p_{k+1} = the part of x p_k orthogonal to
    // p_0 .. p_k (projected out twice), normalised.  The degree-(k+1)
    // coefficient of x p_k is p_k's, so every column keeps a positive one.
    std::vector<long double> x(L), q(L);
    for (int l = 0; l < L; ++l) x[l] = L == 1 ? 0.0L : -1.0L + 2.0L * l / (L - 1);
    for (int l = 0; l < L; ++l) W[size_t(l) * L] = 1.0L / sqrtl((long double)L);
    for (int k = 0; k + 1 < L; ++k) {
        for (int l = 0; l < L; ++l) q[l] = x[l] * W[size_t(l) * L + k];
        for (int pass = 0; pass < 2; ++pass) {
            for (int j = 0; j <= k; ++j) {
                long double c = 0.0L;
                for (int l = 0; l < L; ++l) c += q[l] * W[size_t(l) * L + j];
                for (int l = 0; l < L; ++l) q[l] -= c * W[size_t(l) * L + j];
            }
        }
        long double nrm = 0.0L;
        for (int l = 0; l < L; ++l) nrm += q[l] * q[l];
        nrm = sqrtl(nrm);
        for (int l = 0; l < L; ++l) W[size_t(l) * L + k + 1] = q[l] / nrm;
    }
    return MUFFIN_OK;
}

static size_t align_up(size_t v) { return (v + kAlign - 1) & ~(kAlign - 1); }

int dwt_levels(int nx, int ny) {
    int m = nx < ny ? nx : ny, lg = 0;
    while ((1 << (lg + 1)) <= m) ++lg;
    int J = lg - 1;
    if (J > kMaxDwtLevels) J = kMaxDwtLevels;
    return J < 1 ? 1 : J;
}

long dwt_tiles(int sy, int sx) {
    const int hy = sy / 2, hx = sx / 2;
    const int oty = hy < kDwtTileY ? hy : kDwtTileY, otx = hx < kDwtTileX ? hx : kDwtTileX;
    return long(hy / oty) * (hx / otx);
}

Layout make_layout(const muffin_shape* s, int n_s, int n_nu) {
    Layout lay{};
    const size_t sz = s->dtype == MUFFIN_F64 ? 8 : 4;
    const size_t V = size_t(s->L) * s->ny * s->nx;
    const size_t M = size_t(s->nx) / 2;
    const size_t HS = size_t(s->L) * s->ny * M;               // packed half-spectrum entries
    const int NT = s->nx > s->ny ? s->nx : s->ny;
    size_t off = 0;
    auto take = [&](size_t bytes) { size_t o = off; off = align_up(off + bytes); return o; };
    for (int set = 0; set < 2; ++set)
        for (int i = 0; i < kNumState; ++i) lay.state[set][i] = take(V * sz);
    lay.brest = take(V * sz);
    lay.x = take(V * sz);
    lay.n_nu = n_nu;
    if (n_nu > 1)
        for (int set = 0; set < 2; ++set)
            for (int j = 0; j < n_nu; ++j) lay.uz[set][j] = take(V * sz);
    lay.n_w = n_s > 1 ? n_s - 1 : 0;
    lay.levels = dwt_levels(s->nx, s->ny);
    for (int b = 0; b < lay.n_w; ++b) lay.wz[b] = take(V * sz);
    for (int b = 0; b < lay.n_w; ++b)
        for (int j = 1; j < lay.levels; ++j)
            lay.wtmp[b][j] = take(size_t(s->L) * size_t(s->ny >> j) * size_t(s->nx >> j) * sz);
    if (lay.n_w) {
        for (int i = 0; i < 3; ++i) lay.wrep[i] = take(V * sz);
        // the analysis launches of every basis and level, up to kWPartQ sums per block
        for (int j = 0; j < lay.levels; ++j) lay.wblocks += dwt_tiles(s->ny >> j, s->nx >> j) * s->L * lay.n_w;
        lay.wpart = take(size_t(lay.wblocks) * kWPartQ * 8);
    }
    lay.z = take(HS * 2 * sz);
    lay.yf = take(HS * 2 * sz);
    lay.yfnyq = take(size_t(s->L) * s->ny * 2 * sz);
    lay.h2 = take(HS * sz);
    lay.h2nyq = take(size_t(s->L) * s->ny * sz);
    lay.hh = take(HS * 2 * sz);
    lay.hhnyq = take(size_t(s->L) * s->ny * 2 * sz);
    lay.tw = take(size_t(NT) * 2 * sz);
    lay.tw64 = take(size_t(NT) * 16);
    lay.dctm = take(size_t(n_nu) * dense_width(s->L) * dense_width(s->L) * sz);
    lay.nblk = max_blocks_host(s->L, s->ny, s->nx);
    lay.partials = take(size_t(lay.nblk) * kNumRed * 8);
    lay.vpart = take(size_t(lay.nblk) * 8);
    lay.sums = take(64 * 8);
    // outside the region zero_state clears (state sets .. Z)
    if (lay.n_w) lay.wfilt = take(size_t(kMaxWavelets) * 32 * sz);
    lay.total = off;
    // setup scratch: two FP64 packed spectra, carved out of the state region
    lay.setup_scratch_bytes = 2 * HS * 16;
    lay.state_region_bytes = lay.x - lay.state[0][0];
    return lay;
}

int max_blocks_host(int L, int ny, int nx) {
    const long npix = long(ny) * nx;
    const long spec = (npix + 255) / 256;
    const long col = long(L) * (nx / 2);
    long m = spec > col ? spec : col;
    if (m < 8192) m = 8192;
    return int(m);
}

}  // namespace muffin

using namespace muffin;

extern "C" {

void muffin_default_params(muffin_params* p) {
    if (!p) return;
    std::memset(p, 0, sizeof(*p));
    p->mu_eps = 1e-3;
    p->mu_s = 0.5;
    p->mu_nu = 1.0;
    p->rho_P = 1.0;
    p->rho_T = 5.0;
    p->rho_V = 2.0;
    p->rho_S = 1.0;
    p->n_s = 1;
    p->spatial[0] = MUFFIN_DIRAC;
    p->n_nu = 1;
    p->spectral[0] = MUFFIN_DCT2_ORTHO;
    p->check_every = 10;
    p->eps_abs = 1e-5;
    p->eps_rel = 1e-4;
}

int muffin_validate(const muffin_shape* shape, const muffin_params* params) {
    int rc = validate_shape(shape);
    if (rc != MUFFIN_OK) return rc;
    if ((rc = validate_params(params)) != MUFFIN_OK) return rc;
    if (spectral_dense(*shape, *params) && shape->L > 32 && shape->L != 64) {
        set_error("L = %d: spectral bases other than the DCT alone take L <= 32 or L = 64", shape->L);
        return MUFFIN_EUNSUPPORTED;
    }
    return MUFFIN_OK;
}

size_t muffin_workspace_bytes(const muffin_shape* shape, const muffin_params* params) {
    if (muffin_validate(shape, params) != MUFFIN_OK) return 0;
    return make_layout(shape, params->n_s, params->n_nu).total;
}

int muffin_spectral_basis(int code, int L, double* W) {
    if (!W || L < 1 || L > 4096) { set_error("muffin_spectral_basis: bad L = %d or NULL output", L); return MUFFIN_EINVAL; }
    std::vector<long double> w(size_t(L) * L);
    if (int rc = spectral_basis_ld(code, L, w.data())) return rc;
    for (size_t i = 0; i < w.size(); ++i) W[i] = double(w[i]);
    return MUFFIN_OK;
}

const char* muffin_last_error(void) { return g_err; }

}  // extern "C"
