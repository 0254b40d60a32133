// C ABI of the gfx950 ADMM reconstruction: context, setup, the iteration
// driver, convergence checks and state management.  Every step of the
// iteration runs in the HIP kernels of muffin_fft.hip / muffin_spectral.hip.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstring>
#include <new>
#include <vector>

#include "muffin.h"
#include "muffin_ctx.hpp"
#include "muffin_kernels.hpp"
#include "muffin_layout.hpp"

using namespace muffin;

namespace {

// the fused row/spectral launch exists for the fast DCT and the Dirac spatial basis
bool fused_possible(const muffin_ctx* c) {
    return !c->vis && c->lay.n_w == 0 && !spectral_dense(c->shape, c->params) &&
           fused_supported(c->shape.dtype, c->shape.nx, c->shape.ny, c->shape.L);
}

bool use_fused(const muffin_ctx* c) { return c->fused && fused_possible(c); }

// the coefficient cubes z_V,j of a union of spectral bases (current set, or the other)
void* uz(muffin_ctx* c, int j) { return c->ws + c->lay.uz[c->cur][j]; }
void* uz_alt(muffin_ctx* c, int j) { return c->ws + c->lay.uz[1 - c->cur][j]; }

// the row pass of step I: Z = row spectra of B_rest, unless Z holds them
// already (after a fused pass)
int row_forward(muffin_ctx* c) {
    if (c->zvalid) return MUFFIN_OK;
    const muffin_shape& s = c->shape;
    HIP_TRY(launch_row_fwd(s.dtype, s.dtype == MUFFIN_F64, P(c, c->lay.brest), P(c, c->lay.z), s.L * s.ny,
                           s.nx, s.ny, false, false, P(c, c->lay.tw), c->twlog, c->stream, c->row_v));
    c->zvalid = 1;
    return MUFFIN_OK;
}

int col_solve(muffin_ctx* c) {
    const muffin_shape& s = c->shape;
    HIP_TRY(launch_col(s.dtype, COL_SOLVE, P(c, c->lay.z), P(c, c->lay.yf), P(c, c->lay.yfnyq), P(c, c->lay.h2),
                       P(c, c->lay.h2nyq), rho_Q(c->params), fft_scale(s), s.L, s.ny, s.nx,
                       P(c, c->lay.tw), c->twlog, nullptr, nullptr, c->stream, c->col_v));
    c->zvalid = 0;
    return MUFFIN_OK;
}

// step I of one pass: X = Q^{-1} (H^T Y + B_rest), band by band
int step_one(muffin_ctx* c) {
    const muffin_shape& s = c->shape;
    if (int rc = row_forward(c)) return rc;
    if (int rc = col_solve(c)) return rc;
    HIP_TRY(launch_row_inv(s.dtype, P(c, c->lay.z), P(c, c->lay.x), s.L * s.ny, s.nx, P(c, c->lay.tw),
                           c->twlog, c->stream, c->row_v));
    return MUFFIN_OK;
}

// the inverse row pass, steps II-VI and the forward row pass of the next
// step I in one launch: X and the state as step_one + step_spectral, and Z
// holds the row spectra of the new B_rest (B_rest itself is not written)
int fused_rows_io(muffin_ctx* c, void* const in[4], void* const out[4], void* xo) {
    const muffin_shape& s = c->shape;
    FusedArrays A{};
    A.X = (char*)xo;
    A.zP = (char*)in[ST_ZP];
    A.zT = (char*)in[ST_ZT];
    A.zV = (char*)in[ST_ZV];
    A.GS = (char*)in[ST_GS];
    A.zPo = (char*)out[ST_ZP];
    A.zTo = (char*)out[ST_ZT];
    A.zVo = (char*)out[ST_ZV];
    A.GSo = (char*)out[ST_GS];
    A.Z = P(c, c->lay.z);
    A.band_bytes = unsigned(long(s.ny) * s.nx * long(elem_size(s)));
    A.gshift = 0;
    HIP_TRY(launch_fused(s.dtype, A, P(c, c->lay.dctm), s.L, s.ny, s.nx, spec_args(c->params),
                         P(c, c->lay.tw), c->twlog, c->stream, c->fused));
    c->zvalid = 1;
    return MUFFIN_OK;
}

// wx: X goes to the context (the last pass of a run); the passes before it
// leave X unwritten, as the next pass overwrites it unread
int fused_rows(muffin_ctx* c, bool wx = true) {
    void* cur[4];
    for (int i = 0; i < kNumState; ++i) cur[i] = st(c, i);
    return fused_rows_io(c, cur, cur, wx ? P(c, c->lay.x) : nullptr);
}

// steps II-VI from the state `in` and X, the new state to `out` (a
// reporting pass: the alternate set); a reporting pass also writes the FP64
// partials of the convergence quantities, and the sets swap
int step_spectral_io(muffin_ctx* c, bool report, int* nblocks, void* const in[4], void* const out[4],
                     const void* X) {
    const muffin_shape& s = c->shape;
    SpecLaunch g{};
    g.X = X;
    for (int i = 0; i < kNumState; ++i) {
        g.st[i] = in[i];
        g.out[i] = out[i];
    }
    g.brest = P(c, c->lay.brest);
    g.dctm = P(c, c->lay.dctm);
    g.L = s.L;
    g.npix = long(s.ny) * s.nx;
    g.report = report;
    g.vpart = (double*)P(c, c->lay.vpart);
    g.partials = (double*)P(c, c->lay.partials);
    g.dense = spectral_dense(s, c->params);
    g.n_nu = c->params.n_nu;
    if (report && c->lay.n_w) {
        g.wdt = P(c, c->lay.wrep[1]);
        g.wg = P(c, c->lay.wrep[2]);
    }
    if (g.n_nu > 1)
        for (int j = 0; j < g.n_nu; ++j) {
            g.uz[j] = uz(c, j);
            g.uzo[j] = report ? uz_alt(c, j) : uz(c, j);
        }
    HIP_TRY(launch_spectral(s.dtype, g, spec_args(c->params), nblocks, c->stream));
    c->zvalid = 0;        // B_rest written; Z holds the previous step I's spectrum
    if (report) {
        c->cur = 1 - c->cur;
        c->version++;
    }
    return MUFFIN_OK;
}

int step_spectral(muffin_ctx* c, bool report, int* nblocks) {
    void* in[4];
    void* out[4];
    for (int i = 0; i < kNumState; ++i) {
        in[i] = st(c, i);
        out[i] = report ? st_alt(c, i) : st(c, i);
    }
    return step_spectral_io(c, report, nblocks, in, out, P(c, c->lay.x));
}

// One pass launched without a graph, its state read from `in` and the new
// state written to `out` (in place when they are the same arrays), X to xo;
// B_rest (or Z after a fused pass) is the context's and follows the chain of
// passes.  The reverse sweep runs its forward passes this way, straight into
// its checkpoints and segment stores.  One spectral basis; in and out hold
// the four state arrays, then with wavelet bases in W_s their z_b.
int pass_io(muffin_ctx* c, void* const* in, void* const* out, void* xo) {
    const muffin_shape& s = c->shape;
    if (int rc = row_forward(c)) return rc;
    if (int rc = col_solve(c)) return rc;
    if (use_fused(c)) {
        if (int rc = fused_rows_io(c, in, out, xo)) return rc;
    } else {
        HIP_TRY(launch_row_inv(s.dtype, P(c, c->lay.z), xo, s.L * s.ny, s.nx, P(c, c->lay.tw), c->twlog,
                               c->stream, c->row_v));
        if (int rc = step_spectral_io(c, false, nullptr, in, out, xo)) return rc;
        if (c->lay.n_w)
            if (int rc = dict_pass_io(c, xo, in + kNumState, out + kNumState)) return rc;
    }
    c->iters++;
    return MUFFIN_OK;
}

int pass_kernels(muffin_ctx* c, bool wx = true) {
    if (c->vis) {
        // the visibility-domain model: step I by CG, then steps II-VI
        if (int rc = vis_step_one(c)) return rc;
        return step_spectral(c, false, nullptr);
    }
    if (use_fused(c)) {
        if (int rc = row_forward(c)) return rc;
        if (int rc = col_solve(c)) return rc;
        return fused_rows(c, wx);
    }
    int rc = step_one(c);
    if (rc) return rc;
    if ((rc = step_spectral(c, false, nullptr))) return rc;
    return c->lay.n_w ? dict_pass(c) : MUFFIN_OK;
}

void drop_graphs(muffin_ctx* c) {
    for (int i = 0; i < 2; ++i)
        for (int w = 0; w < 2; ++w) {
            if (c->gexec[i][w]) hipGraphExecDestroy(c->gexec[i][w]);
            c->gexec[i][w] = nullptr;
        }
}

// record the kernels of one pass (state set c->cur; X written or not) into an
// executable graph
int capture_pass(muffin_ctx* c, bool wx) {
    if (!c->cap) HIP_TRY(hipStreamCreateWithFlags(&c->cap, hipStreamNonBlocking));
    hipStream_t user = c->stream;
    c->stream = c->cap;
    hipError_t e = hipStreamBeginCapture(c->cap, hipStreamCaptureModeThreadLocal);
    int rc = e == hipSuccess ? pass_kernels(c, wx) : MUFFIN_EDEVICE;
    hipGraph_t g = nullptr;
    hipError_t e2 = hipStreamEndCapture(c->cap, &g);
    c->stream = user;
    if (e != hipSuccess || e2 != hipSuccess || rc != MUFFIN_OK) {
        if (g) hipGraphDestroy(g);
        if (rc == MUFFIN_OK)
            set_error("graph capture failed: %s", hipGetErrorString(e != hipSuccess ? e : e2));
        return rc == MUFFIN_OK ? MUFFIN_EDEVICE : rc;
    }
    e = hipGraphInstantiate(&c->gexec[c->cur][wx], g, nullptr, nullptr, 0);
    hipGraphDestroy(g);
    if (e != hipSuccess) {
        c->gexec[c->cur][wx] = nullptr;
        set_error("graph instantiation failed: %s", hipGetErrorString(e));
        return MUFFIN_EDEVICE;
    }
    return MUFFIN_OK;
}

// one pass; wx: its X is read afterwards (a fused pass writes X only then)
int one_pass(muffin_ctx* c, bool wx = true) {
    if (c->use_graph) {
        // a recorded fused pass starts from Z (the graph holds the column
        // and fused launches only)
        if (use_fused(c))
            if (int rc = row_forward(c)) return rc;
        if (!c->gexec[c->cur][wx]) {
            int rc = capture_pass(c, wx);
            if (rc) return rc;
        }
        HIP_TRY(hipGraphLaunch(c->gexec[c->cur][wx], c->stream));
        c->zvalid = use_fused(c) ? 1 : 0;
    } else {
        int rc = pass_kernels(c, wx);
        if (rc) return rc;
    }
    c->iters++;
    return MUFFIN_OK;
}

int recompute_brest(muffin_ctx* c) {
    // with a union of spectral bases the third state array is S itself
    HIP_TRY(launch_brest(c->shape.dtype, st(c, ST_ZP), st(c, ST_ZT), st(c, ST_ZV), st(c, ST_GS),
                         P(c, c->lay.brest), voxels(c->shape), spec_args(c->params), c->stream,
                         spectral_union(c->params)));
    c->zvalid = 0;
    return c->lay.n_w ? dict_brest(c) : MUFFIN_OK;
}

int zero_state(muffin_ctx* c) {
    // both state sets, B_rest and X are contiguous
    HIP_TRY(launch_fill_zero(P(c, c->lay.state[0][0]), c->lay.z - c->lay.state[0][0], c->stream));
    c->cur = 0;
    c->iters = 0;
    c->zvalid = 0;
    c->version++;
    return MUFFIN_OK;
}

// cos/sin(2 pi k / n) in extended precision, with exact octant reduction
void twiddle(long k, long n, long double* cr, long double* sr) {
    const long double pi = 3.141592653589793238462643383279502884L;
    *cr = cosl(2.0L * pi * (long double)k / (long double)n);
    *sr = sinl(2.0L * pi * (long double)k / (long double)n);
    // snap the exactly representable values
    if ((4 * k) % n == 0) {
        const long q = ((4 * k) / n) % 4;
        *cr = (q == 0) ? 1.0L : (q == 2 ? -1.0L : 0.0L);
        *sr = (q == 1) ? 1.0L : (q == 3 ? -1.0L : 0.0L);
    }
}

int upload_tables(muffin_ctx* c) {
    const muffin_shape& s = c->shape;
    const int NT = s.nx > s.ny ? s.nx : s.ny;
    std::vector<double> t64(2 * size_t(NT));
    std::vector<float> t32(2 * size_t(NT));
    for (int k = 0; k < NT; ++k) {
        long double cr, sr;
        twiddle(k, NT, &cr, &sr);
        t64[2 * k] = double(cr);
        t64[2 * k + 1] = double(-sr);            // exp(-2 pi i k / NT)
        t32[2 * k] = float(cr);
        t32[2 * k + 1] = float(-sr);
    }
    // the dense band transform of each spectral basis j, zero-padded to the
    // kernels' register width: D_j[k * LT + l] = W_j[l][k]
    const int L = s.L, LT = dense_width(L), m = c->params.n_nu;
    std::vector<double> d64(size_t(m) * LT * LT, 0.0);
    std::vector<float> d32(size_t(m) * LT * LT, 0.0f);
    std::vector<long double> W(size_t(L) * L);
    for (int j = 0; j < m; ++j) {
        if (int rc = spectral_basis_ld(c->params.spectral[j], L, W.data())) return rc;
        for (int k = 0; k < L; ++k)
            for (int l = 0; l < L; ++l) {
                const size_t o = size_t(j) * LT * LT + size_t(k) * LT + l;
                d64[o] = double(W[size_t(l) * L + k]);
                d32[o] = float(W[size_t(l) * L + k]);
            }
    }
    HIP_TRY(hipMemcpy(P(c, c->lay.tw64), t64.data(), t64.size() * 8, hipMemcpyHostToDevice));
    if (s.dtype == MUFFIN_F64) {
        HIP_TRY(hipMemcpy(P(c, c->lay.tw), t64.data(), t64.size() * 8, hipMemcpyHostToDevice));
        HIP_TRY(hipMemcpy(P(c, c->lay.dctm), d64.data(), d64.size() * 8, hipMemcpyHostToDevice));
    } else {
        HIP_TRY(hipMemcpy(P(c, c->lay.tw), t32.data(), t32.size() * 4, hipMemcpyHostToDevice));
        HIP_TRY(hipMemcpy(P(c, c->lay.dctm), d32.data(), d32.size() * 4, hipMemcpyHostToDevice));
    }
    return MUFFIN_OK;
}

int read_sums(muffin_ctx* c, int n, double* out) {
    HIP_TRY(hipMemcpyAsync(out, P(c, c->lay.sums), size_t(n) * 8, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    return MUFFIN_OK;
}

// one pass with the FP64 reductions of the spectral step, then the data term
// of the objective at P = max(0, z_P) through a forward FFT pass.  With
// wavelet bases in W_s their steps III and VI run before steps II-VI (they
// read X and z_b only) with their report terms, their B_rest terms after.
int pass_with_report(muffin_ctx* c, muffin_report* rep) {
    const muffin_shape& s = c->shape;
    const bool wav = c->lay.n_w > 0;
    double* partials = (double*)P(c, c->lay.partials);
    double* sums = (double*)P(c, c->lay.sums);
    constexpr int WREP = 16;            // the wavelet sums: r^2, E, ||T||^2 parts, l1 of W_b P
    int rc = step_one(c);
    if (rc) return rc;
    if (wav && (rc = dict_report_pre(c, sums + WREP))) return rc;
    int nb = 0;
    rc = step_spectral(c, true, &nb);
    if (rc) return rc;
    if (wav && (rc = dict_brest(c))) return rc;
    c->iters++;
    HIP_TRY(launch_reduce_final(partials, nb, RED_NQ, sums, c->stream));
    const int nrows = s.L * s.ny;
    HIP_TRY(launch_row_fwd(s.dtype, s.dtype == MUFFIN_F64, st(c, ST_ZP), P(c, c->lay.z), nrows,
                           s.nx, s.ny, false, true, P(c, c->lay.tw), c->twlog, c->stream));
    int nbc = 0;
    HIP_TRY(launch_col(s.dtype, COL_OBJ, P(c, c->lay.z), P(c, c->lay.yf), P(c, c->lay.yfnyq), P(c, c->lay.h2),
                       P(c, c->lay.h2nyq), 0.0, 1.0, s.L, s.ny, s.nx, P(c, c->lay.tw), c->twlog,
                       partials, &nbc, c->stream));
    HIP_TRY(launch_reduce_final(partials, nbc, 1, sums + RED_NQ, c->stream));
    if (wav && (rc = dict_report_l1(c, st(c, ST_ZP), sums + WREP + 3))) return rc;
    double h[WREP + 4] = {};
    rc = read_sums(c, wav ? WREP + 4 : RED_NQ + 1, h);
    if (rc) return rc;
    for (int i = 0; i < WREP + 4; ++i) {
        if (!std::isfinite(h[i])) {
            set_error("non-finite FP64 reduction (slot %d) at iteration %d", i, c->iters);
            return MUFFIN_ENONFINITE;
        }
    }
    const muffin_params& p = c->params;
    const double nv = double(voxels(s));
    const double n_s = double(p.n_s);
    // ||W_s X||^2 = n_s ||X||^2 (orthonormal bases)
    const double Ax = std::sqrt((2.0 + n_s) * h[RED_X2] + h[RED_V2]);
    const double Bz = std::sqrt(h[RED_BZ2] + h[WREP + 2]);
    const double Aty = std::sqrt(h[RED_ATY2]);
    rep->iters = c->iters;
    rep->r_pri = std::sqrt(h[RED_R2] + h[WREP]);
    rep->r_dual = std::sqrt(h[RED_S2]);
    // constraint space (2 + n_s + m_nu) nv entries, block 1 (1 + m_nu) nv
    rep->eps_pri = std::sqrt((2.0 + n_s + p.n_nu) * nv) * p.eps_abs + p.eps_rel * (Ax > Bz ? Ax : Bz);
    rep->eps_dual = std::sqrt((1.0 + p.n_nu) * nv) * p.eps_abs + p.eps_rel * Aty;
    rep->objective = 0.5 * (c->ynorm2 + h[RED_NQ]) + 0.5 * p.mu_eps * h[RED_P2] +
                     p.mu_s * (h[RED_P1] + h[WREP + 3]) + p.mu_nu * h[RED_DCTP1];
    rep->E = h[RED_E] + h[WREP + 1];
    rep->converged = (rep->r_pri <= rep->eps_pri && rep->r_dual <= rep->eps_dual) ? 1 : 0;
    return MUFFIN_OK;
}

size_t state_array_bytes(const muffin_ctx* c) {
    return (voxels(c->shape) * elem_size(c->shape) + kAlign - 1) & ~(kAlign - 1);
}


// ---------------------------------------------------------------- reverse sweep
// Gradient of a loss of X^K (K passes from the zero state) by the adjoint of
// the reduced pass, with the state checkpointed every C passes: a forward
// sweep writes the checkpoints (and the whole last segment), then each other
// segment (last first) is run again from its checkpoint, its passes writing
// the state before every pass and its X into a segment store, and its passes
// are reversed.  Scratch (device, owned by the context):
//   ckpt : ceil(K / C) x 4 state arrays (the state before each segment's
//          first pass, for the recompute and for that pass's adjoint)
//   seg  : 2 x C x 5 arrays (state before the pass, X of the pass; the
//          state slots of pass 0 hold no input), two stores used in turn by
//          consecutive segments (one with a single segment)
//   adj  : 4 state cotangents, X-bar, B-bar
//   gyac : (with gy_out) the sum over the passes of B-bar
//   partials, partials1 (FP64 block sums), acc
// With gy_out, the cotangent of the dirty images goes there too: Y enters
// every pass through H^T Y in step I's right-hand side (eq. matB), so
// dL/dY = H sum_k B-bar_k.
// FP64 block sums of one adjoint launch
size_t grad_nparts(const muffin_ctx* c) {
    const long npix = long(c->shape.ny) * c->shape.nx;
    return size_t(npix / 64 > 8192 ? npix / 64 : 8192);
}

}  // namespace

namespace muffin {

size_t grad_scratch_bytes(const muffin_ctx* c, int K, int C, bool dirty) {
    if (C > K) C = K;
    const int nseg = (K + C - 1) / C;
    const int nbuf = nseg > 1 ? 2 : 1;
    const int nw = c->lay.n_w, ns = kNumState + nw;     // state arrays per slot
    const size_t n_arrays = size_t(nseg) * ns + size_t(nbuf) * C * (ns + 1) + (kNumState + 2 + nw) +
                            (dirty ? 1 : 0);
    return n_arrays * state_array_bytes(c) + 2 * grad_nparts(c) * GRAD_NQ * 8 + GRAD_NQ * 8;
}

// The reverse sweep in the device scratch g (at least grad_scratch_bytes,
// 256-B aligned; every part of it that is read is written first).
int grad_sweep(muffin_ctx* c, int K, int C, const void* sky_or_gx, int mode, double* loss,
               double grad[7], void* gy_out, char* g, size_t g_bytes, int phase, bool dirty) {
    const muffin_shape& s = c->shape;
    if (phase != 1) dirty = gy_out != nullptr;
    const size_t need = grad_scratch_bytes(c, K, C, dirty);
    if (!g || g_bytes < need) {
        set_error("the reverse sweep of %d passes with checkpoints every %d needs %zu bytes of scratch "
                  "(muffin_grad_workspace_bytes), %zu given (muffin_set_grad_workspace)",
                  K, C, need, g ? g_bytes : size_t(0));
        return MUFFIN_EWORKSPACE;
    }
    if (C > K) C = K;
    const int nseg = (K + C - 1) / C;
    const size_t ab = state_array_bytes(c), nb = voxels(s) * elem_size(s);
    const long npix = long(s.ny) * s.nx;
    const size_t nparts = grad_nparts(c);
    const int nbuf = nseg > 1 ? 2 : 1;
    // a stored state: the four state arrays, then the z_b of the wavelet bases
    const int nw = c->lay.n_w, ns = kNumState + nw;
    auto ckpt = [&](int seg, int i) { return g + (size_t(seg) * ns + i) * ab; };
    char* seg0 = g + size_t(nseg) * ns * ab;
    // store b, pass j of the segment, array i (i = ns: X)
    auto segs = [&](int b, int j, int i) { return seg0 + ((size_t(b) * C + j) * (ns + 1) + i) * ab; };
    // the state before pass j of segment sg in store b: its checkpoint for
    // j = 0 (never overwritten, so not copied into the store)
    auto stv = [&](int b, int sg, int j, int i) { return j == 0 ? ckpt(sg, i) : segs(b, j, i); };
    // aP, aT, aS, aG, Xb, Bb, then the cotangents of the z_b
    char* adj = seg0 + size_t(nbuf) * C * (ns + 1) * ab;
    char* gyac = adj + (kNumState + 2 + nw) * ab;
    double* partials = (double*)(gyac + (dirty ? ab : 0));
    double* partials1 = partials + nparts * GRAD_NQ;      // step-I sums of a fused launch
    double* acc = partials1 + nparts * GRAD_NQ;
    const int dt = s.dtype, nrows = s.L * s.ny;
    const SpecArgs a = spec_args(c->params);
    hipStream_t st_ = c->stream;

    auto copy = [&](void* dst, const void* src) {
        return hipMemcpyAsync(dst, src, nb, hipMemcpyDeviceToDevice, st_);
    };
    // Where the forward passes keep their state and X.  Pass k (segment seg,
    // j = (k - 1) mod C) reads the state before it from checkpoint seg (j = 0),
    // from slot j of a segment store (the last segment, and every segment
    // when it is recomputed) or from the context's own arrays (the other
    // segments on the way forward, in place), and writes the state after it
    // where pass k + 1 reads it: the context's arrays after pass K.  X of a
    // stored pass goes to its slot, X^K to the context.  No state is copied.
    // The state arrays of slot 0 of a store are never read (slot 0's state is
    // the checkpoint): a recomputed segment's last pass writes its (already
    // checkpointed) output there.
    // The sweep starts from the zero state: checkpoint 0 and B_rest are
    // cleared (pass 1 reads nothing else), the context's state set 0 will
    // hold the state after K passes.
    if (phase != 2) {
        c->cur = 0;
        c->iters = 0;
        c->zvalid = 0;
        c->version++;
    }
    constexpr int kMaxSt = kNumState + kMaxWavelets;
    void* ctx_st[kMaxSt];
    for (int i = 0; i < kNumState; ++i) ctx_st[i] = st(c, i);
    for (int w = 0; w < nw; ++w) ctx_st[kNumState + w] = P(c, c->lay.wz[w]);
    auto set_ptrs = [&](void* dst[kMaxSt], auto&& loc) {
        for (int i = 0; i < ns; ++i) dst[i] = loc(i);
    };
    const int blast = (nseg - 1) & (nbuf - 1);
    int rc = MUFFIN_OK;
    if (phase != 2) HIP_TRY(launch_fill_zero(P(c, c->lay.brest), nb, st_));
    if (phase != 2)
        for (int i = 0; i < ns; ++i) HIP_TRY(launch_fill_zero(ckpt(0, i), nb, st_));
    for (int k = 1; k <= K && phase != 2; ++k) {
        const int seg = (k - 1) / C, j = (k - 1) % C;
        const bool last = seg == nseg - 1;
        void *in[kMaxSt], *out[kMaxSt];
        if (j == 0) set_ptrs(in, [&](int i) -> void* { return ckpt(seg, i); });
        else if (last) set_ptrs(in, [&](int i) -> void* { return segs(blast, j, i); });
        else set_ptrs(in, [&](int i) -> void* { return ctx_st[i]; });
        if (k == K) set_ptrs(out, [&](int i) -> void* { return ctx_st[i]; });
        else if (j == C - 1) set_ptrs(out, [&](int i) -> void* { return ckpt(seg + 1, i); });
        else if (last) set_ptrs(out, [&](int i) -> void* { return segs(blast, j + 1, i); });
        else set_ptrs(out, [&](int i) -> void* { return ctx_st[i]; });
        void* xo = (last && k < K) ? (void*)segs(blast, j, ns) : (void*)P(c, c->lay.x);
        if ((rc = pass_io(c, in, out, xo)) != MUFFIN_OK) return rc;
    }
    if (phase == 1) return MUFFIN_OK;
    // X of pass k: its slot, X^K in the context
    auto xloc = [&](int b_, int j_, int k_) -> char* {
        return k_ == K ? (char*)P(c, c->lay.x) : segs(b_, j_, ns);
    };
    void* wbar[kMaxWavelets];
    for (int w = 0; w < nw; ++w) wbar[w] = adj + (kNumState + 2 + w) * ab;
    // seed: the cotangent of X^K
    char* Xb = adj + kNumState * ab;
    char* Bb = adj + (kNumState + 1) * ab;
    HIP_TRY(launch_fill_zero(acc, GRAD_NQ * 8, st_));
    if (mode == MUFFIN_MODE_MSE) {
        int nbk = 0;
        HIP_TRY(launch_mse_seed(dt, P(c, c->lay.x), sky_or_gx, Xb, voxels(s), partials, &nbk, st_));
        HIP_TRY(launch_grad_accum(partials, nbk, acc, st_));
    } else {
        HIP_TRY(copy(Xb, sky_or_gx));
    }
    for (int i = 0; i < kNumState; ++i) HIP_TRY(launch_fill_zero(adj + i * ab, nb, st_));
    for (int w = 0; w < nw; ++w) HIP_TRY(launch_fill_zero(wbar[w], nb, st_));
    if (gy_out) HIP_TRY(launch_fill_zero(gyac, nb, st_));

    const unsigned bb = unsigned(npix * long(elem_size(s)));
    const int gsh = spectral_gshift(bb);
    // with wavelet bases the step-I adjoint of every pass runs on its own,
    // after the wavelet part of B-bar's pass
    const bool fuse_ok = adj_single_descriptor(s.L, bb) && nw == 0;
    for (int seg = nseg - 1; seg >= 0; --seg) {
        const int k0 = seg * C, k1 = (k0 + C < K) ? k0 + C : K;
        const int b = seg & (nbuf - 1);
        if (seg < nseg - 1) {
            // recompute the segment from its checkpoint into store b (B_rest
            // from the checkpoint's state)
            HIP_TRY(launch_brest(dt, ckpt(seg, ST_ZP), ckpt(seg, ST_ZT), ckpt(seg, ST_ZV), ckpt(seg, ST_GS),
                                 P(c, c->lay.brest), voxels(s), a, st_, false));
            if (nw) {
                void* zc[kMaxWavelets];
                for (int w = 0; w < nw; ++w) zc[w] = ckpt(seg, kNumState + w);
                if ((rc = dict_brest_from(c, zc)) != MUFFIN_OK) return rc;
            }
            c->zvalid = 0;
            for (int k = k0 + 1; k <= k1; ++k) {
                const int j = k - k0 - 1;
                void *in[kMaxSt], *out[kMaxSt];
                set_ptrs(in, [&](int i) -> void* { return stv(b, seg, j, i); });
                const int jo = j + 1 < C ? j + 1 : 0;
                set_ptrs(out, [&](int i) -> void* { return segs(b, jo, i); });
                if ((rc = pass_io(c, in, out, segs(b, j, ns))) != MUFFIN_OK) return rc;
            }
        }
        // pass k's step-I adjoint runs inside the band-coupled launch of pass
        // k - 1 (its operands stay in the segment store: the first pass of a
        // segment is in the other store while the segment before it is
        // processed); pass 1's runs on its own.  The same launches for any
        // checkpoint spacing, and the parameter sums added in one order:
        // steps II-VI of k, step I of k, steps II-VI of k - 1, ...
        for (int k = k1; k > k0; --k) {
            const int j = k - k0 - 1;
            const bool fused = k < K && fuse_ok;       // step I of pass k + 1 is pending
            AdjArrays A;
            A.zP = stv(b, seg, j, ST_ZP);
            A.zT = stv(b, seg, j, ST_ZT);
            A.zV = stv(b, seg, j, ST_ZV);
            A.GS = stv(b, seg, j, ST_GS);
            A.X = xloc(b, j, k);
            A.aP = adj;
            A.aT = adj + ab;
            A.aS = adj + 2 * ab;
            A.aG = adj + 3 * ab;
            A.Xb = Xb;
            A.band_bytes = bb;
            A.gshift = gsh;
            if (fused) {
                // pass k + 1: the next slot of this store, or the first of the other
                const int b1 = k < k1 ? b : b ^ 1, s1 = k < k1 ? seg : seg + 1, j1 = k < k1 ? j + 1 : 0;
                A.Bb = Bb;
                A.zP1 = stv(b1, s1, j1, ST_ZP);
                A.zT1 = stv(b1, s1, j1, ST_ZT);
                A.zV1 = stv(b1, s1, j1, ST_ZV);
                A.GS1 = stv(b1, s1, j1, ST_GS);
                A.X1 = xloc(b1, j1, k + 1);
            }
            int nbk = 0;
            const int mode = fused ? 2 : (k == K ? 1 : 0);
            HIP_TRY(launch_adj_spectral(dt, A, P(c, c->lay.dctm), s.L, npix, a, mode, partials, partials1, &nbk,
                                        st_, spectral_dense(s, c->params)));
            if (fused) HIP_TRY(launch_grad_accum(partials1, nbk, acc, st_));
            HIP_TRY(launch_grad_accum(partials, nbk, acc, st_));
            // the wavelet updates of pass k: X-bar += sum_b W_b^T zbar_b
            if (nw && (rc = dict_adj_x(c, wbar, Xb)) != MUFFIN_OK) return rc;
            // B-bar = Q^{-1} X-bar (Q is symmetric)
            HIP_TRY(launch_row_fwd(dt, dt == MUFFIN_F64, Xb, P(c, c->lay.z), nrows, s.nx, s.ny, false, false,
                                   P(c, c->lay.tw), c->twlog, st_, c->row_v));
            HIP_TRY(launch_col(dt, COL_FILTER, P(c, c->lay.z), nullptr, nullptr, P(c, c->lay.h2), P(c, c->lay.h2nyq),
                               rho_Q(c->params), fft_scale(s), s.L, s.ny, s.nx, P(c, c->lay.tw), c->twlog,
                               nullptr, nullptr, st_));
            HIP_TRY(launch_row_inv(dt, P(c, c->lay.z), Bb, nrows, s.nx, P(c, c->lay.tw), c->twlog, st_,
                                   c->row_v));
            if (gy_out) HIP_TRY(launch_add(dt, gyac, Bb, voxels(s), st_));
            if (k == 1 || !fuse_ok) {
                HIP_TRY(launch_adj_step1(dt, Bb, A.zP, A.zT, A.zV, A.GS, A.X, A.aP, A.aT, A.aS, A.aG, npix, s.L, a,
                                         partials, &nbk, st_));
                HIP_TRY(launch_grad_accum(partials, nbk, acc, st_));
            }
            if (nw) {
                // the cotangents of the z_b before pass k: through their update
                // (clip) and through step I of pass k (B_rest), at the state
                // before it
                void* zs[kMaxWavelets];
                for (int w = 0; w < nw; ++w) zs[w] = stv(b, seg, j, kNumState + w);
                if ((rc = dict_adj_b(c, Bb, wbar, zs, acc)) != MUFFIN_OK) return rc;
            }
        }
    }
    // the context holds the state after K passes (pass K wrote it there)
    if (gy_out) {
        // dL/dY = H (sum of B-bar): the transfer function applied in the
        // Fourier domain (Z is scratch here; B_rest is rebuilt below)
        HIP_TRY(launch_row_fwd(dt, dt == MUFFIN_F64, gyac, P(c, c->lay.z), nrows, s.nx, s.ny, false, false,
                               P(c, c->lay.tw), c->twlog, st_, c->row_v));
        HIP_TRY(launch_col(dt, COL_CONV, P(c, c->lay.z), P(c, c->lay.hh), nullptr, nullptr, P(c, c->lay.hhnyq), 0.0,
                           fft_scale(s), s.L, s.ny, s.nx, P(c, c->lay.tw), c->twlog, nullptr, nullptr, st_));
        HIP_TRY(launch_row_inv(dt, P(c, c->lay.z), gy_out, nrows, s.nx, P(c, c->lay.tw), c->twlog, st_,
                               c->row_v));
    }
    if ((rc = recompute_brest(c)) != MUFFIN_OK) return rc;
    c->iters = K;
    double h[GRAD_NQ];
    HIP_TRY(hipMemcpyAsync(h, acc, sizeof(h), hipMemcpyDeviceToHost, st_));
    HIP_TRY(hipStreamSynchronize(st_));
    for (int q = 0; q < GRAD_NQ; ++q) {
        if (!std::isfinite(h[q])) {
            set_error("non-finite gradient accumulator (slot %d)", q);
            return MUFFIN_ENONFINITE;
        }
    }
    const muffin_params& p = c->params;
    // rho of eq. Qlsimp counts n_s rho_T
    const double rT = h[G_RHO_T] - h[G_TAU_T] * p.mu_s / (p.rho_T * p.rho_T) + p.n_s * h[G_RHO_Q];
    const double rV = h[G_RHO_V] - h[G_TAU_V] * p.mu_nu / (p.rho_V * p.rho_V);
    const double rP = h[G_RHO_P] + h[G_RHO_Q];
    const double rS = h[G_RHO_S] + h[G_RHO_Q];
    // d/d(mu_eps, mu_s, mu_nu, rho_P, rho_T, rho_V, rho_S): mu_eps enters
    // through rho of eq. Qlsimp only, mu_s and mu_nu through the thresholds
    grad[0] = h[G_RHO_Q];
    grad[1] = h[G_TAU_T] / p.rho_T;
    grad[2] = h[G_TAU_V] / p.rho_V;
    grad[3] = rP;
    grad[4] = rT;
    grad[5] = rV;
    grad[6] = rS;
    if (loss) *loss = mode == MUFFIN_MODE_MSE ? h[G_LOSS] : 0.0;
    return MUFFIN_OK;
}

// the checks shared by the gradient entry points
int grad_args(const muffin_ctx* c, int K, int ckpt_every, const void* sky_or_gx, int mode, const void* out,
              const char* what) {
    if (int rc = check_ctx(c)) return rc;
    if (int rc = vis_unsupported(c, what)) return rc;
    if (c->shape.L > 128) {
        set_error("%s: the reverse sweep is built for band counts up to 128 (L = %d)", what, c->shape.L);
        return MUFFIN_EUNSUPPORTED;
    }
    if (spectral_union(c->params)) {
        set_error("%s: the reverse sweep is built for one spectral basis (n_nu = %d)", what, c->params.n_nu);
        return MUFFIN_EUNSUPPORTED;
    }
    if (spectral_dense(c->shape, c->params) && c->shape.L > 32) {
        set_error("%s: the reverse sweep's dense band transform is built for L <= 32 (L = %d)", what, c->shape.L);
        return MUFFIN_EUNSUPPORTED;
    }
    if (K < 1 || ckpt_every < 1) {
        set_error("K = %d and ckpt_every = %d must be >= 1", K, ckpt_every);
        return MUFFIN_EINVAL;
    }
    if (!sky_or_gx || !out || (mode != MUFFIN_MODE_MSE && mode != MUFFIN_MODE_VJP)) {
        set_error("%s: sky_or_gx and the output must be non-NULL, mode MSE or VJP", what);
        return MUFFIN_EINVAL;
    }
    return MUFFIN_OK;
}

}  // namespace muffin

namespace muffin {
int refresh_brest(muffin_ctx* c) { return recompute_brest(c); }
int ensure_z(muffin_ctx* c) { return row_forward(c); }
bool fused_pass(const muffin_ctx* c) { return use_fused(c); }
}  // namespace muffin

extern "C" {

int muffin_setup(muffin_ctx** out, const muffin_shape* shape, const muffin_params* params,
                 const void* psf, const void* dirty, void* workspace, size_t ws_bytes, void* stream) {
    if (!out) { set_error("ctx output pointer is NULL"); return MUFFIN_EINVAL; }
    *out = nullptr;
    int rc = muffin_validate(shape, params);
    if (rc != MUFFIN_OK) return rc;
    if (!psf || !dirty || !workspace) {
        set_error("psf, dirty and workspace must be non-NULL device pointers");
        return MUFFIN_EINVAL;
    }
    const Layout lay = make_layout(shape, params->n_s, params->n_nu);
    if (ws_bytes < lay.total) {
        set_error("workspace of %zu bytes is smaller than the %zu bytes needed", ws_bytes, lay.total);
        return MUFFIN_EWORKSPACE;
    }
    if ((reinterpret_cast<uintptr_t>(workspace) & (kAlign - 1)) != 0) {
        set_error("workspace must be %zu-byte aligned", kAlign);
        return MUFFIN_EWORKSPACE;
    }
    muffin_ctx* c = new (std::nothrow) muffin_ctx();
    if (!c) { set_error("out of host memory"); return MUFFIN_EDEVICE; }
    c->shape = *shape;
    c->params = *params;
    c->stream = (hipStream_t)stream;
    c->ws = (char*)workspace;
    c->ws_bytes = ws_bytes;
    c->lay = lay;
    c->cur = 0;
    c->iters = 0;
    const int NT = shape->nx > shape->ny ? shape->nx : shape->ny;
    c->twlog = ilog2i(NT);
    c->row_v = kDefaultRowVariant;
    c->col_v = kDefaultColVariant;
    c->fused = lay.n_w ? 0 : kDefaultFused;    // the fused kernel serves the Dirac basis alone
    c->zvalid = 0;
    c->version = 0;
    c->batch = nullptr;
    c->grad_buf = nullptr;
    c->grad_bytes = 0;
    c->use_graph = 0;
    c->cap = nullptr;
    c->gexec[0][0] = c->gexec[0][1] = c->gexec[1][0] = c->gexec[1][1] = nullptr;

    auto fail = [&](int code) {
        if (c->cap) hipStreamDestroy(c->cap);
        delete c;
        return code;
    };
    // the private stream of graph capture, created here: measured on MI355X,
    // the spectral pass on the caller's stream runs about 14 % faster once the
    // process holds a second stream (the other passes within 2 %)
    if (hipStreamCreateWithFlags(&c->cap, hipStreamNonBlocking) != hipSuccess) {
        c->cap = nullptr;
        set_error("could not create the context's private stream");
        return fail(MUFFIN_EDEVICE);
    }
    const bool in64 = shape->dtype == MUFFIN_F64;
    const size_t n = voxels(*shape);
    // non-finite scan and ||y||^2
    int nb = 0;
    double* partials = (double*)P(c, lay.partials);
    double* sums = (double*)P(c, lay.sums);
    hipError_t e = launch_scan(in64, psf, dirty, n, partials, &nb, c->stream);
    if (e == hipSuccess) e = launch_reduce_final(partials, nb, 2, sums, c->stream);
    if (e != hipSuccess) { set_error("setup scan launch failed: %s", hipGetErrorString(e)); return fail(MUFFIN_EDEVICE); }
    double h[2];
    if ((rc = read_sums(c, 2, h)) != MUFFIN_OK) return fail(rc);
    if (h[0] != 0.0 || !std::isfinite(h[1])) {
        set_error("psf/dirty hold %.0f non-finite values", h[0]);
        return fail(MUFFIN_ENONFINITE);
    }
    c->ynorm2 = h[1];
    if ((rc = upload_tables(c)) != MUFFIN_OK) return fail(rc);
    if ((rc = dict_setup(c)) != MUFFIN_OK) return fail(rc);
    // FP64 transforms of the shifted PSF and of the dirty image, in the (not yet
    // used) state region
    char* Ch = P(c, lay.state[0][0]);
    char* Cy = Ch + lay.setup_scratch_bytes / 2;
    const int nrows = shape->L * shape->ny;
    e = launch_row_fwd(MUFFIN_F64, in64, psf, Ch, nrows, shape->nx, shape->ny, true, false,
                       P(c, lay.tw64), c->twlog, c->stream);
    if (e == hipSuccess)
        e = launch_col(MUFFIN_F64, COL_FWD, Ch, nullptr, nullptr, nullptr, nullptr, 0.0, 1.0, shape->L, shape->ny,
                       shape->nx, P(c, lay.tw64), c->twlog, nullptr, nullptr, c->stream);
    if (e == hipSuccess)
        e = launch_row_fwd(MUFFIN_F64, in64, dirty, Cy, nrows, shape->nx, shape->ny, false, false,
                           P(c, lay.tw64), c->twlog, c->stream);
    if (e == hipSuccess)
        e = launch_col(MUFFIN_F64, COL_FWD, Cy, nullptr, nullptr, nullptr, nullptr, 0.0, 1.0, shape->L, shape->ny,
                       shape->nx, P(c, lay.tw64), c->twlog, nullptr, nullptr, c->stream);
    if (e == hipSuccess)
        e = launch_setup_combine(shape->dtype, Ch, Cy, P(c, lay.yf), P(c, lay.yfnyq), P(c, lay.h2), P(c, lay.h2nyq), P(c, lay.hh),
                                 P(c, lay.hhnyq),
                                 shape->L, shape->ny, shape->nx, c->stream);
    if (e != hipSuccess) { set_error("setup transform launch failed: %s", hipGetErrorString(e)); return fail(MUFFIN_EDEVICE); }
    if ((rc = zero_state(c)) != MUFFIN_OK) return fail(rc);
    e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) { set_error("setup failed: %s", hipGetErrorString(e)); return fail(MUFFIN_EDEVICE); }
    *out = c;
    return MUFFIN_OK;
}

int muffin_iterate(muffin_ctx* c, int n_iter) {
    if (c && c->batch) return batch_iterate(c->batch, n_iter);
    if (int rc = check_ctx(c)) return rc;
    if (n_iter < 0) { set_error("n_iter = %d < 0", n_iter); return MUFFIN_EINVAL; }
    // X of a pass is read only after the last (muffin_get_x, the state
    // snapshot); every pass computes it
    for (int i = 0; i < n_iter; ++i) {
        int rc = one_pass(c, i + 1 == n_iter);
        if (rc) return rc;
    }
    return MUFFIN_OK;
}

int muffin_step_report(muffin_ctx* c, muffin_report* rep) {
    if (int rc = check_ctx(c)) return rc;
    if (int rc = vis_unsupported(c, "muffin_step_report")) return rc;
    if (!rep) { set_error("report is NULL"); return MUFFIN_EINVAL; }
    return pass_with_report(c, rep);
}

int muffin_solve(muffin_ctx* c, int max_iter, muffin_report* report) {
    if (int rc = check_ctx(c)) return rc;
    if (int rc = vis_unsupported(c, "muffin_solve")) return rc;
    if (max_iter < 1) { set_error("max_iter = %d < 1", max_iter); return MUFFIN_EINVAL; }
    muffin_report rep{};
    int done = 0;
    while (done < max_iter) {
        const int left = max_iter - done;
        const int plain = (c->params.check_every - 1 < left - 1) ? c->params.check_every - 1 : left - 1;
        int rc = muffin_iterate(c, plain);
        if (rc) return rc;
        rc = pass_with_report(c, &rep);
        if (rc) return rc;
        done += plain + 1;
        if (rep.converged) break;
    }
    if (report) *report = rep;
    return rep.converged ? MUFFIN_OK : MUFFIN_NOT_CONVERGED;
}

int muffin_solve_adaptive(muffin_ctx* c, int max_iter, double mu, double tau, muffin_report* report) {
    if (int rc = check_ctx(c)) return rc;
    if (int rc = vis_unsupported(c, "muffin_solve_adaptive")) return rc;
    if (max_iter < 1) { set_error("max_iter = %d < 1", max_iter); return MUFFIN_EINVAL; }
    if (!std::isfinite(mu) || !std::isfinite(tau) || mu <= 1.0 || tau <= 1.0) {
        set_error("residual balancing needs finite mu > 1 and tau > 1 (mu = %g, tau = %g)", mu, tau);
        return MUFFIN_EINVAL;
    }
    muffin_report rep{};
    int done = 0;
    while (done < max_iter) {
        const int left = max_iter - done;
        const int plain = (c->params.check_every - 1 < left - 1) ? c->params.check_every - 1 : left - 1;
        int rc = muffin_iterate(c, plain);
        if (rc) return rc;
        rc = pass_with_report(c, &rep);
        if (rc) return rc;
        done += plain + 1;
        if (rep.converged || done >= max_iter) break;
        // residual balancing: the four rho's together, multipliers held
        double f = 1.0;
        if (rep.r_pri > mu * rep.r_dual) f = tau;
        else if (rep.r_dual > mu * rep.r_pri) f = 1.0 / tau;
        if (f != 1.0) {
            muffin_params np = c->params;
            np.rho_P *= f;
            np.rho_T *= f;
            np.rho_V *= f;
            np.rho_S *= f;
            if ((rc = muffin_set_params(c, &np))) return rc;
        }
    }
    if (report) *report = rep;
    return rep.converged ? MUFFIN_OK : MUFFIN_NOT_CONVERGED;
}

int muffin_get_params(const muffin_ctx* c, muffin_params* out) {
    if (int rc = check_ctx(c)) return rc;
    if (!out) { set_error("params output is NULL"); return MUFFIN_EINVAL; }
    *out = c->params;
    return MUFFIN_OK;
}

int muffin_get_x(muffin_ctx* c, void* x_out) {
    if (int rc = check_ctx(c)) return rc;
    if (!x_out) { set_error("x_out is NULL"); return MUFFIN_EINVAL; }
    HIP_TRY(hipMemcpyAsync(x_out, P(c, c->lay.x), voxels(c->shape) * elem_size(c->shape),
                           hipMemcpyDeviceToDevice, c->stream));
    return MUFFIN_OK;
}

int muffin_get_p(muffin_ctx* c, void* p_out) {
    if (int rc = check_ctx(c)) return rc;
    if (!p_out) { set_error("p_out is NULL"); return MUFFIN_EINVAL; }
    HIP_TRY(launch_positive(c->shape.dtype, st(c, ST_ZP), p_out, voxels(c->shape), c->stream));
    return MUFFIN_OK;
}

// state arrays of a snapshot: the four of the reduced state, X, the
// coefficient cube z_b of every wavelet basis, then (a union of spectral
// bases) the coefficient cube z_V,j of every spectral basis
static int snapshot_unions(const muffin_ctx* c) { return c->params.n_nu > 1 ? c->params.n_nu : 0; }
static int snapshot_arrays(const muffin_ctx* c) { return kNumState + 1 + c->lay.n_w + snapshot_unions(c); }
static char* snapshot_array(muffin_ctx* c, int i) {
    if (i < kNumState) return (char*)st(c, i);
    if (i == kNumState) return P(c, c->lay.x);
    if (i < kNumState + 1 + c->lay.n_w) return P(c, c->lay.wz[i - kNumState - 1]);
    return (char*)uz(c, i - kNumState - 1 - c->lay.n_w);
}

size_t muffin_state_bytes(const muffin_ctx* c) {
    if (!c) return 0;
    return kAlign + snapshot_arrays(c) * state_array_bytes(c);
}

int muffin_get_state(muffin_ctx* c, void* dst) {
    if (int rc = check_ctx(c)) return rc;
    if (!dst || (reinterpret_cast<uintptr_t>(dst) & (kAlign - 1))) {
        set_error("state buffer must be a non-NULL, %zu-byte aligned device pointer", kAlign);
        return MUFFIN_EINVAL;
    }
    const size_t ab = state_array_bytes(c), nb = voxels(c->shape) * elem_size(c->shape);
    char* d = (char*)dst;
    HIP_TRY(hipStreamSynchronize(c->stream));
    // every byte of the blob is defined: header block zero-padded, gaps zeroed
    int64_t hdr[kAlign / 8] = {0x4d554646494e5354LL, c->iters, c->shape.dtype, (int64_t)voxels(c->shape)};
    HIP_TRY(hipMemcpy(d, hdr, sizeof(hdr), hipMemcpyHostToDevice));
    for (int i = 0; i < snapshot_arrays(c); ++i) {
        char* a = d + kAlign + i * ab;
        HIP_TRY(hipMemcpyAsync(a, snapshot_array(c, i), nb, hipMemcpyDeviceToDevice, c->stream));
        if (ab > nb) HIP_TRY(launch_fill_zero(a + nb, ab - nb, c->stream));
    }
    return MUFFIN_OK;
}

int muffin_set_state(muffin_ctx* c, const void* src) {
    if (int rc = check_ctx(c)) return rc;
    if (!src || (reinterpret_cast<uintptr_t>(src) & (kAlign - 1))) {
        set_error("state buffer must be a non-NULL, %zu-byte aligned device pointer", kAlign);
        return MUFFIN_EINVAL;
    }
    const size_t ab = state_array_bytes(c), nb = voxels(c->shape) * elem_size(c->shape);
    const char* s = (const char*)src;
    int64_t hdr[4];
    HIP_TRY(hipStreamSynchronize(c->stream));
    HIP_TRY(hipMemcpy(hdr, s, sizeof(hdr), hipMemcpyDeviceToHost));
    if (hdr[0] != 0x4d554646494e5354LL || hdr[2] != c->shape.dtype || hdr[3] != (int64_t)voxels(c->shape)) {
        set_error("state buffer does not hold a state of this shape and dtype");
        return MUFFIN_EINVAL;
    }
    for (int i = 0; i < snapshot_arrays(c); ++i)
        HIP_TRY(hipMemcpyAsync(snapshot_array(c, i), s + kAlign + i * ab, nb, hipMemcpyDeviceToDevice, c->stream));
    c->iters = (int)hdr[1];
    return recompute_brest(c);
}

int muffin_set_params(muffin_ctx* c, const muffin_params* params) {
    if (int rc = check_ctx(c)) return rc;
    int rc = validate_params(params);
    if (rc) return rc;
    if (params->n_s != c->params.n_s ||
        std::memcmp(params->spatial, c->params.spatial, sizeof(int) * size_t(params->n_s)) != 0) {
        set_error("the spatial dictionary (n_s, spatial) is fixed at setup");
        return MUFFIN_EINVAL;
    }
    if (params->n_nu != c->params.n_nu ||
        std::memcmp(params->spectral, c->params.spectral, sizeof(int) * size_t(params->n_nu)) != 0) {
        set_error("the spectral dictionary (n_nu, spectral) is fixed at setup");
        return MUFFIN_EINVAL;
    }
    const muffin_params old = c->params;
    drop_graphs(c);      // the parameters are kernel arguments of the recorded pass
    if (old.rho_P != params->rho_P || old.rho_T != params->rho_T || old.rho_V != params->rho_V) {
        // keep P, Gamma_P, S and T, Gamma_T of the stored state under the new
        // rho's (a union keeps S itself; its z_V,j re-encode below)
        const bool un = spectral_union(old);
        HIP_TRY(launch_reencode(c->shape.dtype, st(c, ST_ZP), st(c, ST_ZT), un ? nullptr : st(c, ST_ZV),
                                st(c, ST_GS), voxels(c->shape), old.rho_P / params->rho_P,
                                old.rho_T / params->rho_T, old.mu_s / old.rho_T,
                                old.rho_V != params->rho_V ? 1.0 / old.rho_V - 1.0 / params->rho_V : 0.0,
                                c->stream));
        if (un && old.rho_V != params->rho_V) {
            void* z[kMaxSpectral];
            for (int j = 0; j < old.n_nu; ++j) z[j] = uz(c, j);
            HIP_TRY(launch_union_reencode(c->shape.dtype, st(c, ST_ZV), z, old.n_nu, P(c, c->lay.dctm),
                                          c->shape.L, long(c->shape.ny) * c->shape.nx, old.rho_V / params->rho_V,
                                          c->stream));
        }
        if (old.rho_T != params->rho_T)
            if (int rc2 = dict_reencode(c, old.rho_T / params->rho_T, old.mu_s / old.rho_T)) return rc2;
    }
    c->params = *params;
    c->version++;
    return recompute_brest(c);
}

int muffin_reset(muffin_ctx* c) {
    if (int rc = check_ctx(c)) return rc;
    return zero_state(c);
}

int muffin_iterations(const muffin_ctx* c) {
    if (!c) return -1;
    return c->batch ? batch_iterations(c->batch) : c->iters;
}

int muffin_profile(muffin_ctx* c, int n_iter, double* ms, const char** names, int cap) {
    if (int rc = check_ctx(c)) return rc;
    if (int rc = vis_unsupported(c, "muffin_profile")) return rc;
    if (n_iter < 1 || !ms || cap < 1) { set_error("muffin_profile: bad arguments"); return MUFFIN_EINVAL; }
    // the kernels of one pass of the context's schedule, timed with events
    // between the launches (each pass runs: the state advances)
    static const char* unfused[5] = {"row_fwd", "col_solve", "row_inv", "spectral", "dictionary"};
    static const char* fused[2] = {"col_solve", "fused"};
    const bool fu = use_fused(c);
    const int K = fu ? 2 : (c->lay.n_w ? 5 : 4);
    const char** knames = fu ? fused : unfused;
    hipEvent_t ev[6];
    for (int i = 0; i <= K; ++i) HIP_TRY(hipEventCreate(&ev[i]));
    double acc[5] = {0, 0, 0, 0, 0};
    const muffin_shape& s = c->shape;
    int rc = MUFFIN_OK;
    if (fu) rc = row_forward(c);
    for (int it = 0; it < n_iter && rc == MUFFIN_OK; ++it) {
        hipError_t e = hipEventRecord(ev[0], c->stream);
        if (fu) {
            if (e == hipSuccess && (rc = col_solve(c)) != MUFFIN_OK) break;
            if (e == hipSuccess) e = hipEventRecord(ev[1], c->stream);
            if (e == hipSuccess && (rc = fused_rows(c, it + 1 == n_iter)) != MUFFIN_OK) break;
            if (e == hipSuccess) e = hipEventRecord(ev[2], c->stream);
        } else {
            if (e == hipSuccess && (rc = row_forward(c)) != MUFFIN_OK) break;
            if (e == hipSuccess) e = hipEventRecord(ev[1], c->stream);
            if (e == hipSuccess && (rc = col_solve(c)) != MUFFIN_OK) break;
            if (e == hipSuccess) e = hipEventRecord(ev[2], c->stream);
            if (e == hipSuccess)
                e = launch_row_inv(s.dtype, P(c, c->lay.z), P(c, c->lay.x), s.L * s.ny, s.nx, P(c, c->lay.tw),
                                   c->twlog, c->stream, c->row_v);
            if (e == hipSuccess) e = hipEventRecord(ev[3], c->stream);
            if (e == hipSuccess && (rc = step_spectral(c, false, nullptr)) != MUFFIN_OK) break;
            if (e == hipSuccess) e = hipEventRecord(ev[4], c->stream);
            if (K == 5) {
                if (e == hipSuccess && (rc = dict_pass(c)) != MUFFIN_OK) break;
                if (e == hipSuccess) e = hipEventRecord(ev[5], c->stream);
            }
        }
        if (e == hipSuccess) e = hipEventSynchronize(ev[K]);
        if (e != hipSuccess) { set_error("profile: %s", hipGetErrorString(e)); rc = MUFFIN_EDEVICE; break; }
        // a fused pass writes X on the last of the passes only (as a run's
        // passes do); the average is over the others when there are others
        if (!(fu && n_iter > 1 && it + 1 == n_iter))
            for (int k = 0; k < K; ++k) {
                float t = 0.f;
                hipEventElapsedTime(&t, ev[k], ev[k + 1]);
                acc[k] += t;
            }
        c->iters++;
    }
    for (int i = 0; i <= K; ++i) hipEventDestroy(ev[i]);
    if (rc) return rc;
    const int m = cap < K ? cap : K;
    for (int k = 0; k < m; ++k) {
        ms[k] = acc[k] / ((fu && n_iter > 1) ? n_iter - 1 : n_iter);
        if (names) names[k] = knames[k];
    }
    return K;
}

int muffin_grad(muffin_ctx* c, int K, int ckpt_every, const void* sky_or_gx, int mode,
                double* loss, double grad[3]) {
    if (int rc = grad_args(c, K, ckpt_every, sky_or_gx, mode, grad, "muffin_grad")) return rc;
    double full[7];
    const int rc = grad_sweep(c, K, ckpt_every, sky_or_gx, mode, loss, full, nullptr, (char*)c->grad_buf,
                              c->grad_bytes);
    if (rc) return rc;
    grad[0] = full[1];
    grad[1] = full[2];
    grad[2] = full[3] + full[4] + full[5] + full[6];
    return MUFFIN_OK;
}

int muffin_grad_dirty(muffin_ctx* c, int K, int ckpt_every, const void* sky_or_gx, int mode, double* loss,
                      void* gy_out) {
    if (int rc = grad_args(c, K, ckpt_every, sky_or_gx, mode, gy_out, "muffin_grad_dirty")) return rc;
    double full[7];
    return grad_sweep(c, K, ckpt_every, sky_or_gx, mode, loss, full, gy_out, (char*)c->grad_buf, c->grad_bytes);
}

int muffin_grad_params(muffin_ctx* c, int K, int ckpt_every, const void* sky_or_gx, int mode, double* loss,
                       double grad[7]) {
    if (int rc = grad_args(c, K, ckpt_every, sky_or_gx, mode, grad, "muffin_grad_params")) return rc;
    return grad_sweep(c, K, ckpt_every, sky_or_gx, mode, loss, grad, nullptr, (char*)c->grad_buf, c->grad_bytes);
}

int muffin_grad_record(muffin_ctx* c, int K, int ckpt_every, int dirty) {
    if (int rc = check_ctx(c)) return rc;
    c->grec.valid = 0;
    // the argument checks of the sweep, with a stand-in for the cotangent it
    // will take (given to muffin_grad_replay)
    if (int rc = grad_args(c, K, ckpt_every, c, MUFFIN_MODE_VJP, c, "muffin_grad_record")) return rc;
    double unused[7];
    const int rc = grad_sweep(c, K, ckpt_every, nullptr, MUFFIN_MODE_VJP, nullptr, unused, nullptr,
                              (char*)c->grad_buf, c->grad_bytes, 1, dirty != 0);
    if (rc) return rc;
    c->grec.valid = 1;
    c->grec.K = K;
    c->grec.C = ckpt_every;
    c->grec.dirty = dirty != 0;
    c->grec.iters = c->iters;
    c->grec.version = c->version;
    c->grec.buf = c->grad_buf;
    c->grec.bytes = c->grad_bytes;
    return MUFFIN_OK;
}

int muffin_grad_replay(muffin_ctx* c, const void* sky_or_gx, int mode, double* loss, double grad[7],
                       void* gy_out) {
    if (int rc = check_ctx(c)) return rc;
    const auto& r = c->grec;
    if (!r.valid || r.iters != c->iters || r.version != c->version || r.buf != c->grad_buf ||
        r.bytes != c->grad_bytes) {
        set_error("muffin_grad_replay: no recorded forward sweep, or the context, its parameters or the "
                  "gradient workspace changed since muffin_grad_record");
        return MUFFIN_EINVAL;
    }
    if (r.dirty != (gy_out != nullptr)) {
        set_error("muffin_grad_replay: the sweep was recorded %s a dirty-image cotangent",
                  r.dirty ? "for" : "without");
        return MUFFIN_EINVAL;
    }
    if (int rc = grad_args(c, r.K, r.C, sky_or_gx, mode, grad, "muffin_grad_replay")) return rc;
    c->grec.valid = 0;
    return grad_sweep(c, r.K, r.C, sky_or_gx, mode, loss, grad, gy_out, (char*)c->grad_buf, c->grad_bytes, 2);
}

size_t muffin_grad_workspace_bytes(const muffin_ctx* c, int K, int ckpt_every, int dirty) {
    if (check_ctx(c) != MUFFIN_OK || K < 1 || ckpt_every < 1) return 0;
    return grad_scratch_bytes(c, K, ckpt_every, dirty != 0);
}

int muffin_set_grad_workspace(muffin_ctx* c, void* ws, size_t bytes) {
    if (int rc = check_ctx(c)) return rc;
    if (ws && (reinterpret_cast<uintptr_t>(ws) & (kAlign - 1)) != 0) {
        set_error("the gradient workspace must be %zu-byte aligned", kAlign);
        return MUFFIN_EWORKSPACE;
    }
    c->grad_buf = ws;
    c->grad_bytes = ws ? bytes : 0;
    return MUFFIN_OK;
}

int muffin_autotune(muffin_ctx* c, int reps, int schedule[3]) {
    if (int rc = check_ctx(c)) return rc;
    if (int rc = vis_unsupported(c, "muffin_autotune")) return rc;
    if (reps < 1) { set_error("reps = %d < 1", reps); return MUFFIN_EINVAL; }
    const muffin_shape& s = c->shape;
    const int dt = s.dtype, nrows = s.L * s.ny;
    // Scratch only: Z, B_rest (recomputed from the state at the end) and the
    // second state set; X and the state stay as they are.
    void* scratch = st_alt(c, 0);
    hipEvent_t e0, e1;
    HIP_TRY(hipEventCreate(&e0));
    HIP_TRY(hipEventCreate(&e1));
    hipError_t e = hipSuccess;
    auto timeit = [&](auto&& launch) -> double {
        if (e == hipSuccess) e = launch();
        if (e == hipSuccess) e = hipEventRecord(e0, c->stream);
        for (int r = 0; r < reps && e == hipSuccess; ++r) e = launch();
        if (e == hipSuccess) e = hipEventRecord(e1, c->stream);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        float ms = 0.f;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
        return double(ms) / reps;
    };
    double t[3][kNumVariants];
    for (int v = 0; v < kNumVariants; ++v) {
        t[0][v] = timeit([&] {
            return launch_row_fwd(dt, dt == MUFFIN_F64, P(c, c->lay.brest), P(c, c->lay.z), nrows, s.nx, s.ny,
                                  false, false, P(c, c->lay.tw), c->twlog, c->stream, v);
        });
        t[1][v] = timeit([&] {
            return launch_col(dt, COL_SOLVE, P(c, c->lay.z), P(c, c->lay.yf), P(c, c->lay.yfnyq), P(c, c->lay.h2),
                              P(c, c->lay.h2nyq), rho_Q(c->params), fft_scale(s), s.L, s.ny, s.nx,
                              P(c, c->lay.tw), c->twlog, nullptr, nullptr, c->stream, v);
        });
        t[2][v] = timeit([&] {
            return launch_row_inv(dt, P(c, c->lay.z), scratch, nrows, s.nx, P(c, c->lay.tw), c->twlog, c->stream, v);
        });
    }
    int rv = kDefaultRowVariant, cv = kDefaultColVariant;
    for (int v = 0; v < kNumVariants; ++v) {
        if (t[0][v] + t[2][v] < t[0][rv] + t[2][rv]) rv = v;
        if (t[1][v] < t[1][cv]) cv = v;
    }
    // fused or not: the spectral pass and the fused kernel on a copy of the
    // state in the second set (X of the fused kernel into the B_rest buffer)
    int fu = 0;
    if (e == hipSuccess && fused_possible(c)) {
        const size_t nb = voxels(s) * elem_size(s);
        for (int i = 0; i < kNumState && e == hipSuccess; ++i)
            e = hipMemcpyAsync(st_alt(c, i), st(c, i), nb, hipMemcpyDeviceToDevice, c->stream);
        SpecLaunch g{};
        g.X = P(c, c->lay.x);
        for (int i = 0; i < kNumState; ++i) g.st[i] = g.out[i] = st_alt(c, i);
        g.brest = P(c, c->lay.brest);
        g.dctm = P(c, c->lay.dctm);
        g.L = s.L;
        g.npix = long(s.ny) * s.nx;
        g.report = false;
        g.vpart = (double*)P(c, c->lay.vpart);
        g.partials = (double*)P(c, c->lay.partials);
        const SpecArgs a = spec_args(c->params);
        const double tspec = timeit([&] { return launch_spectral(dt, g, a, nullptr, c->stream); });
        FusedArrays A{};
        A.X = P(c, c->lay.brest);
        A.zP = A.zPo = (char*)st_alt(c, ST_ZP);
        A.zT = A.zTo = (char*)st_alt(c, ST_ZT);
        A.zV = A.zVo = (char*)st_alt(c, ST_ZV);
        A.GS = A.GSo = (char*)st_alt(c, ST_GS);
        A.Z = P(c, c->lay.z);
        A.band_bytes = unsigned(long(s.ny) * s.nx * long(elem_size(s)));
        A.gshift = 0;
        double best = t[0][rv] + t[2][rv] + tspec;
        const int nfv = fused_two_pixel_variant(s.nx, s.L) ? 2 : 1;
        for (int fv = 1; fv <= nfv; ++fv) {
            const double tfu = timeit([&] {
                return launch_fused(dt, A, P(c, c->lay.dctm), s.L, s.ny, s.nx, a, P(c, c->lay.tw), c->twlog,
                                    c->stream, fv);
            });
            if (tfu < best) { best = tfu; fu = fv; }
        }
    }
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    if (e != hipSuccess) { set_error("autotune: %s", hipGetErrorString(e)); return MUFFIN_EDEVICE; }
    if (int rc = recompute_brest(c)) return rc;      // Z and B_rest were scratch
    const int sch[3] = {rv, cv, fu};
    if (schedule) { schedule[0] = rv; schedule[1] = cv; schedule[2] = fu; }
    return muffin_set_schedule(c, sch);
}

int muffin_set_schedule(muffin_ctx* c, const int schedule[3]) {
    if (int rc = check_ctx(c)) return rc;
    if (int rc = vis_unsupported(c, "muffin_set_schedule")) return rc;
    if (!schedule || schedule[0] < 0 || schedule[0] >= kNumVariants || schedule[1] < 0 ||
        schedule[1] >= kNumVariants || schedule[2] < 0 || schedule[2] > 2) {
        set_error("schedule must hold two variant indices in [0, %d) and a fused form in [0, 2]", kNumVariants);
        return MUFFIN_EINVAL;
    }
    if (c->row_v != schedule[0] || c->col_v != schedule[1] || c->fused != schedule[2]) {
        const bool was_fused = use_fused(c);
        c->row_v = schedule[0];
        c->col_v = schedule[1];
        c->fused = schedule[2];
        if (was_fused && !use_fused(c))
            if (int rc = recompute_brest(c)) return rc;    // B_rest was not kept up to date
        drop_graphs(c);
        c->version++;
    }
    return MUFFIN_OK;
}

int muffin_get_schedule(const muffin_ctx* c, int schedule[3]) {
    if (int rc = check_ctx(c)) return rc;
    if (!schedule) { set_error("schedule is NULL"); return MUFFIN_EINVAL; }
    schedule[0] = c->row_v;
    schedule[1] = c->col_v;
    schedule[2] = c->fused;
    return MUFFIN_OK;
}

int muffin_fused_available(const muffin_ctx* c) {
    return c && !c->batch && fused_possible(c) ? 1 : 0;
}

int muffin_set_graph(muffin_ctx* c, int enable) {
    if (c && c->batch) return batch_set_graph(c->batch, enable);
    if (int rc = check_ctx(c)) return rc;
    c->use_graph = enable ? 1 : 0;
    return MUFFIN_OK;
}

int muffin_destroy(muffin_ctx* c) {
    if (!c) return MUFFIN_OK;
    if (c->batch) return batch_destroy(c);
    drop_graphs(c);
    if (c->vis) vis_destroy(c);
    if (c->cap) hipStreamDestroy(c->cap);
    delete c;
    return MUFFIN_OK;
}

}  // extern "C"
