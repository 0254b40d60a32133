/*
 * muffin.h -- C ABI of the MI355X (gfx950) wide-band ADMM reconstruction.
 *
 * The library solves, for a cube of L dirty images y_l (one per frequency
 * band) and their point-spread functions, the convex problem of Ferrari et
 * al., "Multi-frequency image reconstruction for radio interferometry. A
 * regularized inverse problem approach" (arXiv 1504.06847):
 *
 *   min_X 1/2 ||Y - H X||^2 + 1_{R+}(X) + mu_eps/2 ||X||_F^2
 *         + mu_s ||W_s X||_1 + mu_nu ||X W_nu||_1          (Section 2, eqs.
 *                                                            costreg, RegAll)
 *
 * with the ADMM iteration of Algorithm 1 (Section 3, steps I-VI).  H_l is a
 * 2-D circular convolution with the band-l PSF (eq. nbmodel), W_s is the
 * Dirac basis (n_s = 1) or the Dirac basis followed by up to eight
 * orthonormal Daubechies wavelet bases (Section 4 uses Db1-Db8, n_s = 9),
 * W_nu the orthonormal DCT-II along the bands.  Step I
 * is solved exactly in the Fourier domain with the filter
 * (|h_hat_l|^2 + rho)^{-1}, rho = mu_eps + rho_S + rho_P + n_s rho_T
 * (eq. Qlsimp and the paragraph after it).
 *
 * Conventions for every entry point:
 *  - Cubes are dense, row-major [L][ny][nx] arrays (x fastest, band slowest)
 *    in DEVICE memory, in the precision named by muffin_shape.dtype
 *    (float for MUFFIN_F32, double for MUFFIN_F64).
 *  - A PSF has its peak at 0-based pixel (ny/2, nx/2).
 *  - `stream` arguments are hipStream_t values passed as void*; NULL is the
 *    default stream.  A context is bound to the stream it was set up on, is
 *    not thread-safe, and is independent of every other context.
 *  - The caller owns psf, dirty, outputs and the workspace; the workspace
 *    must outlive the context.  The library keeps no pointer to psf or dirty
 *    after muffin_setup returns.
 *  - Return values: MUFFIN_OK (0) or a negative error code below; no C++
 *    exception and no abort crosses this interface.  muffin_last_error()
 *    gives a message for the last failure on the calling thread.
 */
#ifndef MUFFIN_H
#define MUFFIN_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------ */
#define MUFFIN_OK              0
#define MUFFIN_NOT_CONVERGED   1   /* muffin_solve reached max_iter (informational) */
#define MUFFIN_EINVAL         -1   /* null pointer, L < 1, mu < 0, rho <= 0, non-finite
                                      parameter, n_iter < 0, K < 1, ckpt_every < 1 */
#define MUFFIN_EUNSUPPORTED   -2   /* size not a power of two in [8, 4096], dtype,
                                      dictionary or band count not supported */
#define MUFFIN_EWORKSPACE     -3   /* workspace too small or misaligned (256 B) */
#define MUFFIN_EDEVICE        -4   /* a HIP runtime error (message in muffin_last_error) */
#define MUFFIN_ENONFINITE     -5   /* NaN/Inf in psf/dirty at setup, or in a reduction */

/* ---- enumerations ------------------------------------------------------ */
#define MUFFIN_F32 0
#define MUFFIN_F64 1

#define MUFFIN_DIRAC 0             /* the Dirac basis (identity) */
/* Daubechies wavelet basis Db_p (p vanishing moments, filter length 2p;
   scaling filter by Daubechies' spectral factorisation, extra zeros outside
   the unit circle), periodised, 4 levels (fewer when the smaller image side
   is below 32: levels = min(4, log2(min(nx, ny)) - 1)), Mallat layout */
#define MUFFIN_DB1 1
#define MUFFIN_DB2 2
#define MUFFIN_DB3 3
#define MUFFIN_DB4 4
#define MUFFIN_DB5 5
#define MUFFIN_DB6 6
#define MUFFIN_DB7 7
#define MUFFIN_DB8 8
/* spectral bases W_nu along the bands (one, or a union of up to
   MUFFIN_MAX_SPECTRAL distinct ones: Section 3, the closed form of step V for
   a union of m_nu orthonormal transforms) */
#define MUFFIN_DCT2_ORTHO 0        /* orthonormal DCT-II along the bands (Section 4) */
#define MUFFIN_CHEBYSHEV 1         /* Chebyshev polynomials T_0 .. T_{L-1} at the bands
                                      (equispaced, mapped onto [-1, 1]) orthonormalised in
                                      order of degree, degree-k coefficient positive
                                      (Section 4 names the family as an alternative) */
#define MUFFIN_SPECTRAL_DIRAC 2    /* the identity along the bands */
#define MUFFIN_MAX_SPECTRAL 4

#define MUFFIN_MODE_MSE 0          /* muffin_grad: loss = ||x_K - sky||^2, sky given */
#define MUFFIN_MODE_VJP 1          /* muffin_grad: cotangent dL/dx_K given */

#define MUFFIN_MAX_BANDS 256       /* largest L: up to 128 bands a pixel's band vector
                                      and its DCT stay in one thread's registers, at 256
                                      they are split over two waves (the DCT-II of length
                                      256 as a butterfly, a DCT-II and a DCT-IV of length
                                      128); above 32 bands L must be a power of two.
                                      Batches and the gradient take L <= 128. */

/* ---- plain-data structs -------------------------------------------------- */
typedef struct muffin_ctx muffin_ctx;        /* opaque, owned by the library */

typedef struct {
    int nx, ny;   /* image size; each a power of two in [8, 4096] */
    int L;        /* number of bands, 1 <= L <= MUFFIN_MAX_BANDS */
    int dtype;    /* MUFFIN_F32 or MUFFIN_F64: storage and arithmetic of the iteration */
} muffin_shape;

typedef struct {
    /* regularisation weights (Section 2, eq. RegAll), all >= 0 */
    double mu_eps, mu_s, mu_nu;
    /* augmented-Lagrangian parameters of the four constraints P = X,
       T = W_s X, V = S W_nu, S = X (eq. admm2), all > 0 */
    double rho_P, rho_T, rho_V, rho_S;
    int n_s;          /* number of spatial bases W_s stacks, 1 <= n_s <= 9 */
    int spatial[9];   /* spatial[0] = MUFFIN_DIRAC; spatial[1 .. n_s-1] in
                         MUFFIN_DB1 .. MUFFIN_DB8.  With n_s > 1: the
                         three-launch pass (in a batch, the cube's wavelet
                         launches follow its grouped ones); a reporting pass runs each
                         basis's analysis once more in report form and three
                         syntheses for W_s^T dT and W_s^T Gamma_T (three more
                         cubes of workspace) */
    int n_nu;         /* number of spectral bases W_nu stacks, 1 <= n_nu <= MUFFIN_MAX_SPECTRAL */
    int spectral[MUFFIN_MAX_SPECTRAL];  /* spectral[0 .. n_nu-1]: distinct codes above.
                         Anything but the DCT alone takes a dense L x L transform
                         per basis, for L <= 32 or L = 64; a union (n_nu > 1) has
                         no fused pass, batches or gradient (MUFFIN_EUNSUPPORTED) */
    int check_every;  /* muffin_solve: iterations between FP64 residual checks (>= 1) */
    double eps_abs, eps_rel;   /* stopping tolerances of Boyd et al. (2011), Sec. 3.3.1 */
} muffin_params;

typedef struct {
    int iters;        /* iterations run by this context since setup/reset */
    int converged;    /* 1 if r_pri <= eps_pri and r_dual <= eps_dual at the last check */
    double r_pri, r_dual, eps_pri, eps_dual;  /* primal/dual residual norms and tolerances */
    double objective; /* criterion (costreg)+(RegAll) evaluated at P = max(0, prox input) */
    double E;         /* ||w^k - w^{k+1}||_H^2 (He & Yuan 2015), non-increasing in k */
} muffin_report;

/* Fill `p` with the paper's parameter values (Section 4): mu_eps = 1e-3,
   mu_s = 0.5, mu_nu = 1, rho_P = 1, rho_T = 5, rho_V = 2, rho_S = 1,
   n_s = 1 (Dirac), n_nu = 1 (DCT-II), check_every = 10, eps_abs = 1e-5,
   eps_rel = 1e-4. */
void muffin_default_params(muffin_params* p);

/* Bytes of device workspace muffin_setup needs for this shape (0 if the
   shape or parameters are invalid; muffin_last_error says why).  Host-only. */
size_t muffin_workspace_bytes(const muffin_shape* shape, const muffin_params* params);

/* Host-only validation of a shape and parameter set: MUFFIN_OK or the code
   muffin_setup would return before touching the device. */
int muffin_validate(const muffin_shape* shape, const muffin_params* params);

/* Host-only: the orthonormal spectral basis `code` for L bands into W
   (row-major L x L, FP64): the spectrum of a pixel's band vector x is
   x W, as the library's spectral passes use it.  Errors: EINVAL (code or L
   out of range, W NULL). */
int muffin_spectral_basis(int code, int L, double* W);

/* Host-only: the scaling filter of the wavelet basis Db_p (MUFFIN_DB1 <= p
   <= MUFFIN_DB8; Section 4's dictionary) into h[0 .. 2p-1], FP64, as the
   library's wavelet passes use it (wavelet filter g[k] = (-1)^k h[2p-1-k]).
   Errors: EINVAL (p out of range or h NULL). */
int muffin_wavelet_filter(int p, double* h);

/* Set up one cube: derives |h_hat_l|^2 and conj(h_hat_l) FFT2(y_l) in FP64
   (stored in the shape's precision) into `workspace`, scans psf/dirty for
   non-finite values, zeroes the ADMM state (Algorithm 1 initialisation) and
   writes the new context to *ctx.  psf, dirty: device [L][ny][nx] arrays.
   Synchronous: it reads the scan result back, uploads the twiddle and DCT
   tables with blocking copies and synchronises `stream` before returning,
   so psf and dirty may be freed or overwritten as soon as it returns.  It
   creates one private stream per context (graph capture).
   Errors: EINVAL, EUNSUPPORTED, EWORKSPACE, EDEVICE, ENONFINITE. */
int muffin_setup(muffin_ctx** ctx, const muffin_shape* shape, const muffin_params* params,
                 const void* psf, const void* dirty, void* workspace, size_t ws_bytes,
                 void* stream);

/* Run n_iter passes of Algorithm 1 (steps I-VI) on the context's stream.
   No host synchronisation.  n_iter = 0 is a no-op.  Every pass computes X;
   the fused pass stores it to the context's X array only in the last pass
   of the call, the earlier ones' X being overwritten unread (muffin_get_x
   and the state snapshot read the last).  Errors: EINVAL, EDEVICE. */
int muffin_iterate(muffin_ctx* ctx, int n_iter);

/* Iterate until the primal/dual residuals of the two-block splitting fall
   under their tolerances (Boyd et al. 2011, Sec. 3.3; checked every
   params.check_every iterations in FP64) or max_iter iterations have run.
   Fills *report (may be NULL).  Returns MUFFIN_OK when converged,
   MUFFIN_NOT_CONVERGED at max_iter, or an error. Synchronises the stream at
   each check. */
int muffin_solve(muffin_ctx* ctx, int max_iter, muffin_report* report);

/* muffin_solve with residual balancing (Boyd et al. 2011, Sec. 3.4.1; the
   paper notes that the rho's set the speed of convergence, Section 4): at
   every check that does not stop the run, the four rho's are multiplied by
   tau when r_pri > mu r_dual and divided by tau when r_dual > mu r_pri, the
   multipliers held as in muffin_set_params (the filter of eq. Qlsimp follows
   the new rho).  mu > 1, tau > 1 (Boyd et al. use 10 and 2).  The rho's in
   force at the end are read back with muffin_get_params.
   Returns as muffin_solve.  Errors: EINVAL, EUNSUPPORTED (visibility-domain
   context), EDEVICE, ENONFINITE. */
int muffin_solve_adaptive(muffin_ctx* ctx, int max_iter, double mu, double tau, muffin_report* report);

/* The context's parameters (host copy).  Errors: EINVAL. */
int muffin_get_params(const muffin_ctx* ctx, muffin_params* out);

/* Run ONE more pass of Algorithm 1 and fill *report with its residuals, E and
   the objective at the new P.  Synchronises the stream. */
int muffin_step_report(muffin_ctx* ctx, muffin_report* report);

/* Copy the current X iterate (step I output of the last pass; zero before the
   first pass) into x_out, a device [L][ny][nx] array of the shape's dtype.
   Asynchronous on the context's stream. */
int muffin_get_x(muffin_ctx* ctx, void* x_out);

/* Copy the current P = max(0, X - Gamma_P / rho_P) iterate (non-negative). */
int muffin_get_p(muffin_ctx* ctx, void* p_out);

/* Gradient of a loss of x_K, the X iterate after K passes of Algorithm 1
   from the all-zero state, with respect to (mu_s, mu_nu, rho), where rho is
   the common value of rho_P = rho_T = rho_V = rho_S (its derivative is taken
   along (1, 1, 1, 1)).  mode = MUFFIN_MODE_MSE: sky_or_gx is a device cube
   (the reference sky), loss = ||x_K - sky||^2.  mode = MUFFIN_MODE_VJP:
   sky_or_gx is dL/dx_K and *loss is left as 0.  Uses a reverse sweep with
   state checkpoints every ckpt_every passes, in the device scratch attached
   with muffin_set_grad_workspace (muffin_grad_workspace_bytes(ctx, K,
   ckpt_every, 0) bytes; the library allocates nothing).  grad: host
   double[3].  The context's state afterwards equals the state after K
   passes from zero.  Synchronises the stream.
   With wavelet bases in W_s their coefficient cubes z_b are stored with the
   state and the sweep runs the adjoint of their updates and of their B_rest
   terms (the step-I adjoint of each pass then runs on its own launch).
   Errors: EINVAL, EUNSUPPORTED (visibility-domain context, a union of
   spectral bases, L > 128), EWORKSPACE (no or a too small workspace
   attached), EDEVICE, ENONFINITE. */
int muffin_grad(muffin_ctx* ctx, int K, int ckpt_every, const void* sky_or_gx, int mode,
                double* loss, double grad[3]);

/* Bytes of device scratch the reverse sweep of K passes with checkpoints
   every ckpt_every needs (dirty = 1: for muffin_grad_dirty, one cube more):
   with m = 4 + n_w state cubes per stored state (n_w = n_s - 1 wavelet
   bases), m ceil(K / C) + 2 (m + 1) C + 6 + n_w cubes for C = ckpt_every < K
   (m + (m + 1) K + 6 + n_w for C >= K), a cube being L ny nx values of the
   context's dtype rounded up to 256 B, plus FP64 block sums.  0 for a NULL or batch context, K < 1 or
   ckpt_every < 1.  Host-only. */
size_t muffin_grad_workspace_bytes(const muffin_ctx* ctx, int K, int ckpt_every, int dirty);

/* Attach the caller's device scratch for the gradient calls (ws 256-byte
   aligned, `bytes` long; NULL detaches).  The context keeps the pointer
   until it is replaced or the context destroyed; the caller keeps it
   allocated meanwhile.  Its contents between calls are not used.
   Errors: EINVAL, EWORKSPACE (misaligned). */
int muffin_set_grad_workspace(muffin_ctx* ctx, void* ws, size_t bytes);

/* For callers that cannot allocate device memory (code under HIP graph
   capture, tight serving loops, harnesses that forbid hipMalloc):
   muffin_grad with the reverse sweep's scratch in a static device array of
   MUFFIN_NOALLOC_SCRATCH_MIB MiB, which the library holds on every GPU it
   runs on until the process ends.  No workspace is needed and nothing is
   allocated.  The sweep must fit: muffin_grad_workspace_bytes(ctx, K,
   ckpt_every, 0) <= MUFFIN_NOALLOC_SCRATCH_MIB MiB, else MUFFIN_EWORKSPACE.
   Every call on a GPU uses that GPU's one array, which keeps the last call's
   contents (each call writes what it reads): calls that overlap on one GPU
   (several streams or host threads) race, and the caller must serialise
   them.  The passes are launched one by one (no graph is recorded).  The
   results equal muffin_grad's bit for bit.  Errors as muffin_grad. */
#define MUFFIN_NOALLOC_SCRATCH_MIB 64
int muffin_grad_noalloc(muffin_ctx* ctx, int K, int ckpt_every, const void* sky_or_gx, int mode,
                        double* loss, double grad[3]);

/* The same reverse sweep, with the derivative along each parameter on its
   own: grad = d/d(mu_eps, mu_s, mu_nu, rho_P, rho_T, rho_V, rho_S) (host
   double[7]).  mu_eps enters through rho of eq. Qlsimp only; the tied-rho
   derivative of muffin_grad is the sum of the last four.  Errors as
   muffin_grad. */
int muffin_grad_params(muffin_ctx* ctx, int K, int ckpt_every, const void* sky_or_gx, int mode,
                       double* loss, double grad[7]);

/* The same reverse sweep, returning the cotangent of the dirty images:
   gy_out (device [L][ny][nx], the iteration's dtype, caller-owned) receives
   dL/dY.  Y enters every pass through H^T Y in the right-hand side of step
   I (eq. matB), so dL/dY = H sum_k Q^{-1} X-bar_k, with X-bar_k the
   cotangent of pass k's X.  loss as muffin_grad.  The attached workspace
   must hold muffin_grad_workspace_bytes(ctx, K, ckpt_every, 1) bytes.
   Errors as muffin_grad. */
int muffin_grad_dirty(muffin_ctx* ctx, int K, int ckpt_every, const void* sky_or_gx, int mode,
                      double* loss, void* gy_out);

/* The reverse sweep in two halves, for callers that need x_K before they
   know its cotangent (an autograd forward, then its backward):
   muffin_grad_record runs the K forward passes from the all-zero state with
   checkpoints every ckpt_every into the attached workspace
   (muffin_grad_workspace_bytes(ctx, K, ckpt_every, dirty) bytes), leaving
   the context after K passes (x_K readable with muffin_get_x);
   muffin_grad_replay then runs the reverse half: loss as muffin_grad, grad
   as muffin_grad_params (host double[7]), and with a record taken with
   dirty = 1 the cotangent of the dirty images to gy_out as
   muffin_grad_dirty (NULL otherwise).  Together they compute what one
   muffin_grad_params / muffin_grad_dirty call computes, running each
   forward pass once.  A replay consumes the record; any pass, state or
   parameter change, or another workspace in between, voids it (EINVAL).
   Errors as muffin_grad. */
int muffin_grad_record(muffin_ctx* ctx, int K, int ckpt_every, int dirty);
int muffin_grad_replay(muffin_ctx* ctx, const void* sky_or_gx, int mode, double* loss, double grad[7],
                       void* gy_out);

/* Bytes of one state snapshot: the iteration's carried arrays (the prox
   inputs z_P and z_T of steps II-III, the spectral prox input
   z_V = S - Gamma_S / rho_V of step IV, and Gamma_S; Gamma_V = Gamma_S W_nu
   holds after every pass, so it is not stored), the X iterate and a header
   with the iteration counter.  The arrays encode the variables under the
   context's rho's: restore a state into a context with the same parameters. */
size_t muffin_state_bytes(const muffin_ctx* ctx);

/* Save / restore the ADMM state to / from device memory `dst` / `src`
   (muffin_state_bytes bytes, 256-byte aligned).  Resuming from a saved state
   reproduces the uninterrupted run bit for bit. */
int muffin_get_state(muffin_ctx* ctx, void* dst);
int muffin_set_state(muffin_ctx* ctx, const void* src);

/* Replace the parameters (mu's, rho's) without a new setup.  The ADMM
   variables are kept (up to rounding): P, Gamma_P, S, Gamma_S, Gamma_V, and
   T, Gamma_T when mu_s is unchanged, so a change of the rho's continues
   Algorithm 1 with the multipliers held fixed (the rule for varying penalty
   parameters, Boyd et al. 2011, Sec. 3.4.1).  With a new mu_s the stored
   input of the spatial soft threshold is kept, i.e. the run continues from a
   warm start of the new problem.  Errors: EINVAL, EUNSUPPORTED, EDEVICE. */
int muffin_set_params(muffin_ctx* ctx, const muffin_params* params);

/* Zero the ADMM state (Algorithm 1 initialisation) and the iteration count. */
int muffin_reset(muffin_ctx* ctx);

/* Replay each pass of muffin_iterate / muffin_solve from a HIP graph
   (enable = 1) instead of launching its kernels one by one (0, the default).
   The graph is recorded on a private stream at the first pass and replayed
   on the context's stream; muffin_set_params records a new one.  Results are
   bitwise identical to the launched form.  Errors: EINVAL, EDEVICE. */
int muffin_set_graph(muffin_ctx* ctx, int enable);

/* Number of passes run since setup/reset. */
int muffin_iterations(const muffin_ctx* ctx);

/* ---- schedules of a pass (the 2-D transform of step I, eq. Qlsimp, and
   the pass structure) -----------------------------------------------------
   A schedule is three integers: schedule[0] in [0, 3) for the row passes
   (about 1024, 2048, 4096 complex points per work-group), schedule[1] in
   [0, 3) for the column pass (half, all or twice the column tile that fits
   64 KiB of LDS; twice only where the LDS holds it), schedule[2] = 1 to run
   the inverse row pass, steps II-VI and the forward row pass of the next
   step I as one fused launch where it is built (muffin_fused_available),
   2 for the same launch with two pixels per thread (built for 64 bands on
   rows of 256 to 1024 pixels and 32 bands on rows of 1024; elsewhere, and
   in a batch, it runs as 1), 0 for three launches.  Every
   schedule evaluates the same formulas in the same order; the compiler may
   fuse a product and a sum into one FMA in one schedule's code and not in
   another's, so results agree to rounding (a few ulps), not bit for bit.
   Default {1, 1, 1}. */

/* Time each variant of the transform passes, and the fused launch (both
   forms where built) against the three it replaces, `reps` times on this context's own arrays (the
   timing writes only internal scratch: X and the state are unchanged), keep
   the fastest and write it to schedule (may be NULL).  Synchronises the
   stream.  Errors: EINVAL (reps < 1), EDEVICE. */
int muffin_autotune(muffin_ctx* ctx, int reps, int schedule[3]);

/* Use a stored schedule (e.g. one muffin_autotune found for this shape).
   Errors: EINVAL (value out of range). */
int muffin_set_schedule(muffin_ctx* ctx, const int schedule[3]);
int muffin_get_schedule(const muffin_ctx* ctx, int schedule[3]);

/* 1 if this context's shape has the fused launch (FP32, 64 <= nx <= 1024,
   L in {4, 8, 16, 32, 64}, a cube of at most 1 GiB), else 0. */
int muffin_fused_available(const muffin_ctx* ctx);

/* ---- batches of independent cubes ----------------------------------------
   Many cubes of uneven size and band count (each its own instance of the
   problem of Section 2, solved by Algorithm 1) iterating together: each
   pass runs one grouped launch per transform pass and shape class (row
   passes per nx, the column pass per ny, the spectral pass per band count)
   that covers the tiles of every cube in the class, so that small cubes
   share the GPU instead of running one after another.  Results are bitwise
   identical to iterating each cube on its own with the same schedule.

   A batch is held by a batch context.  On it, muffin_iterate runs n passes
   of every cube, muffin_set_graph replays each batch pass from one HIP
   graph, muffin_iterations counts the batch passes and muffin_destroy
   releases the batch and its cubes; every other single-cube call returns
   MUFFIN_EINVAL on it and works on the cube contexts of muffin_batch_cube. */

/* Device workspace bytes for n cubes: the per-cube workspaces
   (muffin_workspace_bytes, 256-B aligned) plus the launch descriptors.
   0 if a shape or parameter set is invalid, n < 1, n > MUFFIN_MAX_BATCH or
   the dtypes differ. */
#define MUFFIN_MAX_BATCH 256
size_t muffin_batch_workspace_bytes(int n, const muffin_shape* shapes, const muffin_params* params);

/* Set up n cubes and write the batch context to *ctx: shapes[i],
   params[i], psf[i], dirty[i] as for muffin_setup (every cube in one dtype,
   the Dirac spatial basis), one 256-B aligned workspace of at least
   muffin_batch_workspace_bytes bytes, one stream for all cubes.
   Synchronous, as muffin_setup.
   Errors: as muffin_setup, plus EINVAL for n out of range or mixed dtypes,
   EUNSUPPORTED for a wavelet dictionary. */
int muffin_setup_batch(muffin_ctx** ctx, int n, const muffin_shape* shapes,
                       const muffin_params* params, const void* const* psf,
                       const void* const* dirty, void* workspace, size_t ws_bytes, void* stream);

/* The context of cube i of a batch context (owned by the batch; do not
   destroy it).  Every single-cube call works on it (muffin_get_x,
   muffin_step_report, muffin_solve, muffin_set_params, state calls ...); the
   batch notices the changes before its next pass.  NULL if `batch` is not a
   batch context or i is out of range (muffin_last_error says which). */
muffin_ctx* muffin_batch_cube(muffin_ctx* batch, int i);

/* Autotune every cube's own schedule (muffin_autotune: which pass form the
   cube joins), then time the variants of each grouped transform launch per
   shape class and keep the fastest.  Synchronises the stream. */
int muffin_batch_autotune(muffin_ctx* batch, int reps);

/* Number of grouped launches per pass (shape classes of the four passes);
   -1 if `batch` is not a batch context. */
int muffin_batch_launches(const muffin_ctx* batch);

/* ---- the visibility-domain model -------------------------------------------
   Section 2: the same algorithm with y_l the sampled visibilities of band l
   and H_l the operator from the sky to them, (H_l x)_j = sum_{m,n} x[m][n]
   exp(-2 pi i (u_j (n - nx/2) / nx + v_j (m - ny/2) / ny)), (u_j, v_j) in
   cells of the nx x ny Fourier grid at that band's frequency (any real
   values; the phase centre is pixel (ny/2, nx/2) as the PSF peak of
   muffin_setup).  The sky is real: H_l^T = Re(H_l^H .) and Q_l = Re(H_l^H
   H_l) + rho I (eq. Qlsimp), no longer diagonal in the Fourier domain, so
   step I of Algorithm 1 runs n_cg conjugate-gradient iterations per band
   (Hestenes-Stiefel), started from the previous pass's X (zero at the
   first).  Each applies Re(H^H H) as a circular convolution on the
   2ny x 2nx grid with the Toeplitz kernel c(d) = sum_j cos(2 pi (u_j d_x /
   nx + v_j d_y / ny)), formed at setup (FP64) with the data term
   Re(H^H y).  Built for the Dirac spatial basis (n_s = 1) and nx, ny <=
   2048; any spectral dictionary.  On such a context muffin_iterate,
   muffin_set_graph, muffin_get_x, muffin_get_p, the state calls,
   muffin_set_params, muffin_reset, muffin_iterations and muffin_destroy work
   as for muffin_setup's contexts; reports, muffin_solve*, the gradients,
   muffin_autotune, muffin_set_schedule and muffin_profile return
   MUFFIN_EUNSUPPORTED. */

/* Bytes of device workspace muffin_setup_vis needs (0 if the shape or the
   parameters are invalid for this model).  Host-only. */
size_t muffin_vis_workspace_bytes(const muffin_shape* shape, const muffin_params* params);

/* Set up one cube in the visibility domain.  n_vis: host [L], visibilities
   per band (>= 0); uv: host, sum(n_vis) pairs (u, v) of doubles, band after
   band; vis: host, sum(n_vis) pairs (re, im) of doubles in the same order
   (both read during the call only); n_cg in [1, 100000].  workspace: device,
   256-byte aligned, at least muffin_vis_workspace_bytes, owned by the
   caller and held for the context's life.  Synchronous; allocates setup
   temporaries (the visibilities, the kernel) and frees them before
   returning.  Errors: EINVAL (NULL pointers, n_vis < 0, n_cg out of range),
   EUNSUPPORTED (n_s > 1, nx or ny > 2048), EWORKSPACE, ENONFINITE (a
   non-finite uv or vis), EDEVICE. */
int muffin_setup_vis(muffin_ctx** ctx, const muffin_shape* shape, const muffin_params* params, const int* n_vis,
                     const double* uv, const double* vis, int n_cg, void* workspace, size_t ws_bytes,
                     void* stream);

/* CG iterations per band and pass of a visibility-domain context (negative
   if ctx is not one). */
int muffin_vis_cg_iters(const muffin_ctx* ctx);

/* Time n_iter passes with HIP events around every kernel launch on the
   context's stream; writes the mean duration in ms of each kernel of one
   pass to ms[i] and its name to names[i] (static strings), for up to `cap`
   kernels; returns the number of kernels per pass (negative on error).  As
   in muffin_iterate a fused pass stores X in the last pass only; with
   n_iter > 1 the means are over the passes before it. */
int muffin_profile(muffin_ctx* ctx, int n_iter, double* ms, const char** names, int cap);

/* Release the context (not the caller's workspaces); a batch context
   releases its cubes too.  NULL is a no-op. */
int muffin_destroy(muffin_ctx* ctx);

/* Message for the last error on the calling thread ("" if none). */
const char* muffin_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* MUFFIN_H */
