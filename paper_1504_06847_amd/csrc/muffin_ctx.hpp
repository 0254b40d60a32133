// The context of one cube and the small host helpers shared by the C ABI
// translation units (muffin_api.cpp, muffin_batch.cpp).
#pragma once
#include <hip/hip_runtime.h>

#include "muffin.h"
#include "muffin_kernels.hpp"
#include "muffin_layout.hpp"

struct muffin_batch;
struct muffin_vis;

struct muffin_ctx {
    // a batch context (muffin_setup_batch) holds its cubes here and none of
    // the per-cube fields below; a cube context has batch == nullptr
    muffin_batch* batch;
    muffin_shape shape;
    muffin_params params;
    hipStream_t stream;
    char* ws;
    size_t ws_bytes;
    muffin::Layout lay;
    int cur;          // which state set holds the current state
    int iters;
    int twlog;
    double ynorm2;
    // tile schedules of the row and column passes, and whether a pass runs
    // the fused row/spectral kernel (muffin_autotune)
    int row_v, col_v, fused;
    // Z holds the row spectra of the current B_rest (set by the forward row
    // pass and by the fused kernel, which does not write B_rest itself)
    int zvalid;
    // bumped whenever the arrays, parameters or schedules of the next pass
    // change (a batch rebuilds its launch descriptors then)
    unsigned version;
    // the caller's workspace of the reverse sweep (muffin_set_grad_workspace)
    void* grad_buf;
    size_t grad_bytes;
    // a recorded forward sweep (muffin_grad_record) awaiting its reverse half:
    // valid while the context's version, pass count and workspace are the ones
    // it left
    struct {
        int valid, K, C, dirty, iters;
        unsigned version;
        void* buf;
        size_t bytes;
    } grec;
    // graph replay of one pass: captured on a private stream, one executable
    // graph per state set and per form of the pass (X written or not),
    // replayed on `stream`
    int use_graph;
    hipStream_t cap;
    hipGraphExec_t gexec[2][2];
    // wavelet bases of the spatial dictionary: filter length and the FP64
    // scaling filter of each (lay.n_w of them)
    int wK[muffin::kMaxWavelets];
    double wh[muffin::kMaxWavelets][16];
    // the visibility-domain model (muffin_setup_vis): step I by conjugate
    // gradients; nullptr for the dirty-image model
    muffin_vis* vis;
};

namespace muffin {

#define HIP_TRY(expr)                                                                 \
    do {                                                                              \
        hipError_t e_ = (expr);                                                       \
        if (e_ != hipSuccess) {                                                       \
            muffin::set_error("%s failed: %s", #expr, hipGetErrorString(e_));         \
            return MUFFIN_EDEVICE;                                                    \
        }                                                                             \
    } while (0)

inline size_t elem_size(const muffin_shape& s) { return s.dtype == MUFFIN_F64 ? 8 : 4; }
inline size_t voxels(const muffin_shape& s) { return size_t(s.L) * s.ny * s.nx; }
inline int ilog2i(int n) { int r = 0; while ((1 << r) < n) ++r; return r; }

inline char* P(muffin_ctx* c, size_t off) { return c->ws + off; }
inline void* st(muffin_ctx* c, int i) { return c->ws + c->lay.state[c->cur][i]; }
inline void* st_alt(muffin_ctx* c, int i) { return c->ws + c->lay.state[1 - c->cur][i]; }

inline SpecArgs spec_args(const muffin_params& p) {
    SpecArgs a;
    a.rho_P = p.rho_P;
    a.rho_T = p.rho_T;
    a.rho_V = p.rho_V;
    a.rho_S = p.rho_S;
    a.tau_T = p.mu_s / p.rho_T;
    a.tau_V = p.mu_nu / p.rho_V;
    return a;
}

// rho of eq. Qlsimp for a union of n_s orthonormal bases
inline double rho_Q(const muffin_params& p) {
    return p.mu_eps + p.rho_S + p.rho_P + double(p.n_s) * p.rho_T;
}

// scale of the unnormalised packed 2-D transform pair, folded into the filter
inline double fft_scale(const muffin_shape& s) { return 1.0 / (double(s.nx / 2) * double(s.ny)); }

// recompute B_rest from the stored state; make Z hold the row spectra of
// B_rest; whether the context's passes are fused passes (muffin_api.cpp)
int refresh_brest(muffin_ctx* c);
int ensure_z(muffin_ctx* c);
bool fused_pass(const muffin_ctx* c);

// the wavelet bases of the spatial dictionary (muffin_dict.cpp): filters at
// setup; steps III, VI and the B_rest terms of one pass (after the spectral
// pass); the B_rest terms of the stored state; re-encoding for new rho_T
int daubechies_filter(int p, double* h);
int dict_setup(muffin_ctx* c);
int dict_pass(muffin_ctx* c);
int dict_brest(muffin_ctx* c);
int dict_reencode(muffin_ctx* c, double ratio, double tau);
// reporting pass with wavelet bases: sums[0..2] (r^2, E, ||T||^2 parts) and
// the report kernel's cubes; after it, sum_b ||W_b max(0, z_P)||_1 into *sum1
int dict_report_pre(muffin_ctx* c, double* sums);
// steps III and VI of every wavelet basis out of place (X given, z_b read
// from zin[b], written to zout[b]) and their B_rest terms from zout
int dict_pass_io(muffin_ctx* c, const void* X, void* const* zin, void* const* zout);
// the B_rest terms of the wavelet bases from the cubes z[b], added to B_rest
int dict_brest_from(muffin_ctx* c, void* const* z);
// reverse sweep: X-bar += sum_b W_b^T zbar_b (zbar_b the cotangent of z_b
// after a pass)
int dict_adj_x(muffin_ctx* c, void* const* zbar, void* Xb);
// reverse sweep, after B-bar of the pass: zbar_b <- the cotangent of z_b
// before the pass (zs[b] the state's z_b then), tau_T and rho_T sums into acc
int dict_adj_b(muffin_ctx* c, const void* Bb, void* const* zbar, void* const* zs, double* acc);
int dict_report_l1(muffin_ctx* c, const void* zP, double* sum1);

// a cube context (not NULL, not a batch context)
inline int check_ctx(const muffin_ctx* c) {
    if (!c) { set_error("context is NULL"); return MUFFIN_EINVAL; }
    if (c->batch) {
        set_error("a batch context: this call works on one cube (muffin_batch_cube)");
        return MUFFIN_EINVAL;
    }
    return MUFFIN_OK;
}

// the reverse sweep of the gradient entry points (muffin_api.cpp): bytes of
// its device scratch for K passes with checkpoints every C (one more cube
// for the cotangent of the dirty images), and the sweep itself with its
// scratch at g (g_bytes of it; MUFFIN_EWORKSPACE when short); grad receives
// the derivatives along (mu_eps, mu_s, mu_nu, rho_P, rho_T, rho_V, rho_S)
size_t grad_scratch_bytes(const muffin_ctx* c, int K, int C, bool dirty);
// phase 0: the whole sweep; 1: its forward passes only (scratch laid out
// for a dirty-image cotangent when `dirty`), leaving the context after K
// passes; 2: the reverse half of a sweep whose forward passes phase 1 ran
// in the same scratch, the context untouched since
int grad_sweep(muffin_ctx* c, int K, int C, const void* sky_or_gx, int mode, double* loss, double grad[7],
               void* gy_out, char* g, size_t g_bytes, int phase = 0, bool dirty = false);
// argument checks of the gradient entry points (`out`: their output pointer)
int grad_args(const muffin_ctx* c, int K, int ckpt_every, const void* sky_or_gx, int mode, const void* out,
              const char* what);

// the visibility-domain model (muffin_vis.cpp): step I of one pass by CG
// (launches only, capturable); freeing its parts; EUNSUPPORTED for a call
// the model does not have
int vis_step_one(muffin_ctx* c);
void vis_destroy(muffin_ctx* c);
int vis_unsupported(const muffin_ctx* c, const char* what);

// the batch calls behind muffin_iterate, muffin_set_graph, muffin_iterations
// and muffin_destroy on a batch context (muffin_batch.cpp)
int batch_iterate(muffin_batch* b, int n_iter);
int batch_set_graph(muffin_batch* b, int enable);
int batch_iterations(const muffin_batch* b);
int batch_destroy(muffin_ctx* c);

}  // namespace muffin
