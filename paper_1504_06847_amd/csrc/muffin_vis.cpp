// The visibility-domain model behind muffin_setup_vis (Section 2: the data
// are the sampled visibilities, H_l maps the sky to the visibilities of band
// l; step I of Algorithm 1 by conjugate gradients on Q_l of eq. Qlsimp).
//
// A visibility context is an ordinary context of the image shape (its state,
// steps II-VI, graph replay and state calls serve unchanged) whose step I is
// the CG of muffin_vis.hip.  Its Q_l applies Re(H_l^H H_l) as a circular
// convolution on the 2ny x 2nx grid: a second, inner context of that shape,
// set up with the Toeplitz kernel c as its PSF, supplies the kernel's
// transfer function, its twiddles and its spectrum and padded buffers, and
// each CG iteration runs its row and column passes (the column pass in
// transfer-function mode) on the zero-padded search direction.
#include <cmath>
#include <cstring>
#include <new>
#include <vector>

#include "muffin_ctx.hpp"

struct muffin_vis {
    muffin_ctx* conv;     // the inner 2ny x 2nx context
    int n_cg;
    long n_total;
    void *hty, *r, *Ap;   // plain cubes of the image shape
    double *partials, *rr, *alpha, *beta;
};

using namespace muffin;

namespace {

constexpr int kMaxCg = 100000;

size_t align_up(size_t n) { return (n + kAlign - 1) / kAlign * kAlign; }

muffin_shape conv_shape(const muffin_shape& s) {
    muffin_shape t = s;
    t.nx = 2 * s.nx;
    t.ny = 2 * s.ny;
    return t;
}

// the workspace: the image context's, the inner context's, then the CG
// vectors (Re(H^H y), r, Ap) and the per-band FP64 scalars and partials
struct VisLayout {
    size_t outer, inner, hty, r, ap, scal, partials, total;
};

VisLayout vis_layout(const muffin_shape& s, const muffin_params& p) {
    VisLayout v{};
    const muffin_shape t = conv_shape(s);
    const size_t cube = voxels(s) * elem_size(s);
    v.outer = 0;
    v.inner = align_up(make_layout(&s, p.n_s, p.n_nu).total);
    v.hty = v.inner + align_up(make_layout(&t, 1, p.n_nu).total);
    v.r = v.hty + align_up(cube);
    v.ap = v.r + align_up(cube);
    v.scal = v.ap + align_up(cube);
    v.partials = v.scal + align_up(3 * size_t(s.L) * sizeof(double));
    v.total = v.partials + align_up(size_t(s.L) * size_t(cg_blocks(long(s.ny) * s.nx)) * sizeof(double));
    return v;
}

int vis_validate(const muffin_shape* shape, const muffin_params* params) {
    int rc = muffin_validate(shape, params);
    if (rc) return rc;
    if (shape->nx > 2048 || shape->ny > 2048) {
        set_error("the visibility model convolves on a 2ny x 2nx grid: nx, ny <= 2048 (got %d x %d)", shape->ny,
                  shape->nx);
        return MUFFIN_EUNSUPPORTED;
    }
    if (params->n_s != 1) {
        set_error("the visibility model is built for the Dirac spatial basis alone (n_s = %d)", params->n_s);
        return MUFFIN_EUNSUPPORTED;
    }
    return MUFFIN_OK;
}

}  // namespace

namespace muffin {

int vis_unsupported(const muffin_ctx* c, const char* what) {
    if (!c || !c->vis) return MUFFIN_OK;
    set_error("%s: not built for the visibility-domain model", what);
    return MUFFIN_EUNSUPPORTED;
}

void vis_destroy(muffin_ctx* c) {
    if (!c || !c->vis) return;
    muffin_destroy(c->vis->conv);
    delete c->vis;
    c->vis = nullptr;
}

int vis_step_one(muffin_ctx* c) {
    const muffin_vis& v = *c->vis;
    muffin_ctx* in = v.conv;
    const muffin_shape& s = c->shape;
    const muffin_shape& t = in->shape;
    const int dt = s.dtype;
    hipStream_t st_ = c->stream;
    CgVectors g;
    g.L = s.L;
    g.ny = s.ny;
    g.nx = s.nx;
    g.x = P(c, c->lay.x);
    g.r = v.r;
    g.Ap = v.Ap;
    g.P2 = P(in, in->lay.brest);       // the padded search direction (its padding stays zero)
    g.A2 = P(in, in->lay.x);           // Re(H^H H) p on the padded grid
    g.hty = v.hty;
    g.brest = P(c, c->lay.brest);
    g.partials = v.partials;
    g.rr = v.rr;
    g.alpha = v.alpha;
    g.beta = v.beta;
    const double rho = rho_Q(c->params);
    char* Z2 = P(in, in->lay.z);
    const int nrows = t.L * t.ny;
    // A2 = c (*) P2 on the 2ny x 2nx grid: row pass, column pass multiplying
    // by the kernel's transfer function, inverse row pass
    auto conv = [&]() -> int {
        HIP_TRY(launch_row_fwd(dt, dt == MUFFIN_F64, g.P2, Z2, nrows, t.nx, t.ny, false, false, P(in, in->lay.tw),
                               in->twlog, st_, in->row_v));
        HIP_TRY(launch_col(dt, COL_CONV, Z2, P(in, in->lay.hh), nullptr, nullptr, P(in, in->lay.hhnyq), 0.0,
                           fft_scale(t), t.L, t.ny, t.nx, P(in, in->lay.tw), in->twlog, nullptr, nullptr, st_,
                           in->col_v));
        HIP_TRY(launch_row_inv(dt, Z2, (void*)g.A2, nrows, t.nx, P(in, in->lay.tw), in->twlog, st_, in->row_v));
        return MUFFIN_OK;
    };
    // r = b - Q x0 with x0 the previous X and b = Re(H^H y) + B_rest (eq. matB)
    HIP_TRY(launch_cg(dt, CG_PAD, g, rho, st_));
    if (int rc = conv()) return rc;
    HIP_TRY(launch_cg(dt, CG_INIT, g, rho, st_));
    for (int it = 0; it < v.n_cg; ++it) {
        if (int rc = conv()) return rc;
        HIP_TRY(launch_cg(dt, CG_AP, g, rho, st_));
        HIP_TRY(launch_cg(dt, CG_XR, g, rho, st_));
        if (it + 1 < v.n_cg) HIP_TRY(launch_cg(dt, CG_P, g, rho, st_));
    }
    return MUFFIN_OK;
}

}  // namespace muffin

extern "C" {

size_t muffin_vis_workspace_bytes(const muffin_shape* shape, const muffin_params* params) {
    if (vis_validate(shape, params) != MUFFIN_OK) return 0;
    return vis_layout(*shape, *params).total;
}

int muffin_setup_vis(muffin_ctx** out, const muffin_shape* shape, const muffin_params* params, const int* n_vis,
                     const double* uv, const double* vis, int n_cg, void* workspace, size_t ws_bytes,
                     void* stream) {
    if (!out) { set_error("ctx output pointer is NULL"); return MUFFIN_EINVAL; }
    *out = nullptr;
    int rc = vis_validate(shape, params);
    if (rc) return rc;
    if (!n_vis || !workspace) { set_error("n_vis and workspace must be non-NULL"); return MUFFIN_EINVAL; }
    if (n_cg < 1 || n_cg > kMaxCg) { set_error("n_cg = %d outside [1, %d]", n_cg, kMaxCg); return MUFFIN_EINVAL; }
    const int L = shape->L;
    std::vector<long> off(size_t(L) + 1, 0);
    for (int l = 0; l < L; ++l) {
        if (n_vis[l] < 0) { set_error("n_vis[%d] = %d < 0", l, n_vis[l]); return MUFFIN_EINVAL; }
        off[size_t(l) + 1] = off[size_t(l)] + n_vis[l];
    }
    const long M = off[size_t(L)];
    if (M > 0 && (!uv || !vis)) { set_error("uv and vis must be non-NULL host arrays"); return MUFFIN_EINVAL; }
    for (long j = 0; j < 2 * M; ++j) {
        if (!std::isfinite(uv[j]) || !std::isfinite(vis[j])) {
            set_error("uv / vis hold a non-finite value (entry %ld)", j);
            return MUFFIN_ENONFINITE;
        }
    }
    const VisLayout lay = vis_layout(*shape, *params);
    if (ws_bytes < lay.total) {
        set_error("workspace of %zu bytes is smaller than the %zu bytes needed", ws_bytes, lay.total);
        return MUFFIN_EWORKSPACE;
    }
    if ((reinterpret_cast<uintptr_t>(workspace) & (kAlign - 1)) != 0) {
        set_error("workspace must be %zu-byte aligned", kAlign);
        return MUFFIN_EWORKSPACE;
    }
    char* ws = (char*)workspace;
    hipStream_t s = (hipStream_t)stream;
    const muffin_shape t = conv_shape(*shape);
    const size_t es = elem_size(*shape);
    // setup temporaries: the visibilities on the device, the Toeplitz kernel
    // (the inner context's PSF) and the unit impulses (the image context's)
    double *uv_d = nullptr, *vis_d = nullptr;
    long* off_d = nullptr;
    void *kern = nullptr, *delta = nullptr;
    auto cleanup = [&]() {
        if (uv_d) hipFree(uv_d);
        if (vis_d) hipFree(vis_d);
        if (off_d) hipFree(off_d);
        if (kern) hipFree(kern);
        if (delta) hipFree(delta);
    };
    const size_t nvb = size_t(M > 0 ? M : 1) * 2 * sizeof(double);
    hipError_t e = hipMalloc((void**)&uv_d, nvb);
    if (e == hipSuccess) e = hipMalloc((void**)&vis_d, nvb);
    if (e == hipSuccess) e = hipMalloc((void**)&off_d, off.size() * sizeof(long));
    if (e == hipSuccess) e = hipMalloc(&kern, voxels(t) * es);
    if (e == hipSuccess) e = hipMalloc(&delta, voxels(*shape) * es);
    if (e == hipSuccess && M > 0) e = hipMemcpyAsync(uv_d, uv, size_t(M) * 2 * sizeof(double), hipMemcpyHostToDevice, s);
    if (e == hipSuccess && M > 0) e = hipMemcpyAsync(vis_d, vis, size_t(M) * 2 * sizeof(double), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(off_d, off.data(), off.size() * sizeof(long), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = launch_vis_sum(shape->dtype, 0, uv_d, vis_d, off_d, L, shape->ny, shape->nx, kern, s);
    if (e == hipSuccess)
        e = launch_vis_sum(shape->dtype, 1, uv_d, vis_d, off_d, L, shape->ny, shape->nx, ws + lay.hty, s);
    if (e == hipSuccess) e = launch_vis_delta(shape->dtype, delta, L, shape->ny, shape->nx, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
        set_error("visibility setup: %s", hipGetErrorString(e));
        cleanup();
        return MUFFIN_EDEVICE;
    }
    // the image context (its data term is unused: step I is the CG) and the
    // inner convolution context; muffin_setup synchronises the stream
    muffin_ctx* c = nullptr;
    muffin_ctx* in = nullptr;
    rc = muffin_setup(&c, shape, params, delta, ws + lay.hty, ws + lay.outer, lay.inner - lay.outer, stream);
    if (rc == MUFFIN_OK) {
        muffin_params q = *params;
        rc = muffin_setup(&in, &t, &q, kern, kern, ws + lay.inner, lay.hty - lay.inner, stream);
    }
    cleanup();
    if (rc != MUFFIN_OK) {
        if (c) muffin_destroy(c);
        return rc;
    }
    muffin_vis* v = new (std::nothrow) muffin_vis();
    if (!v) {
        muffin_destroy(in);
        muffin_destroy(c);
        set_error("out of host memory");
        return MUFFIN_EDEVICE;
    }
    v->conv = in;
    v->n_cg = n_cg;
    v->n_total = M;
    v->hty = ws + lay.hty;
    v->r = ws + lay.r;
    v->Ap = ws + lay.ap;
    v->rr = (double*)(ws + lay.scal);
    v->alpha = v->rr + L;
    v->beta = v->alpha + L;
    v->partials = (double*)(ws + lay.partials);
    c->vis = v;
    c->fused = 0;
    c->version++;
    *out = c;
    return MUFFIN_OK;
}

int muffin_vis_cg_iters(const muffin_ctx* c) {
    if (int rc = check_ctx(c)) return rc;
    if (!c->vis) { set_error("not a visibility-domain context"); return MUFFIN_EINVAL; }
    return c->vis->n_cg;
}

}  // extern "C"
