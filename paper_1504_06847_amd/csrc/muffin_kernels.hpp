// Host-side declarations of the kernel launchers (implemented in
// muffin_kernels.hip).  All pointers are device pointers; every launcher
// returns the hipError_t of its launch.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>

namespace muffin {

enum ColMode { COL_SOLVE = 0, COL_FWD = 1, COL_OBJ = 2, COL_FILTER = 3, COL_CONV = 4 };

// Number of FP64 partial sums per block written by the spectral pass in
// reduction mode, and their meaning.
enum RedSlot {
    RED_R2 = 0,    // ||r||^2, primal residual
    RED_S2,        // ||s||^2, dual residual
    RED_X2,        // ||X||^2
    RED_V2,        // ||V||^2
    RED_BZ2,       // ||P||^2 + ||T||^2 + 2 ||S||^2
    RED_ATY2,      // ||Gamma_P + Gamma_T + Gamma_S||^2 + ||Gamma_V||^2
    RED_E,         // E^k
    RED_P2,        // ||P||^2
    RED_P1,        // sum |P|
    RED_DCTP1,     // sum |P W_nu|
    RED_NQ
};

struct SpecArgs {
    double rho_P, rho_T, rho_V, rho_S, tau_T, tau_V;
};

// Tile schedules of the FFT passes (all compute the same values in the same
// order; only the work split differs).  Row passes: rows per work-group
// (1024, 2048 or 4096 complex points per group for variants 0, 1, 2).
// Column pass: columns per tile (half, all or twice the largest tile that
// fits 64 KiB of LDS, at most 16; twice only where the LDS holds it).
constexpr int kNumVariants = 3;
constexpr int kDefaultRowVariant = 1;
constexpr int kDefaultColVariant = 1;
constexpr int kDefaultFused = 1;      // the fused row/spectral kernel where it is built

// Row pass, forward: every row of `in` (nrows rows of nx reals, type float or
// double per in_f64) -> packed half spectrum `out` (nrows x nx/2 complex of
// type T).  shift: read the row through ifftshift (rows of each band of ny
// rows rotated by ny/2, columns by nx/2).  positive: read max(0, v).
hipError_t launch_row_fwd(int dtype, bool in_f64, const void* in, void* out, int nrows, int nx,
                          int ny, bool shift, bool positive, const void* tw, int twlog,
                          hipStream_t s, int variant = kDefaultRowVariant);

// Row pass, inverse: packed half spectrum -> real rows (unnormalised).
hipError_t launch_row_inv(int dtype, const void* in, void* out, int nrows, int nx,
                          const void* tw, int twlog, hipStream_t s, int variant = kDefaultRowVariant);

// Column pass over L bands of ny x (nx/2) packed spectra, in place.
// COL_SOLVE: FFT along y, X_hat = (Z + Yf) * scale / (H2 + rhoQ), inverse FFT.
// COL_FWD: FFT along y only.  COL_OBJ: FFT along y, then per-block FP64
// partials of sum w (H2 |Z|^2 - 2 Re(conj(Yf) Z)) / (nx ny) into partials.
// COL_FILTER: as COL_SOLVE without the data term (Yf unused).  COL_CONV:
// FFT along y, multiplication by h_hat * scale (the convolution H; Yf points
// at the packed h_hat, H2nyq at its kx = nx/2 column, complex), inverse FFT.
// Yf, H2 and h_hat are in the column-block order launch_setup_combine
// writes; Yf's slot 0 holds the kx = 0 column alone and Yfnyq ([L][ny]
// complex) the kx = nx/2 column (H2nyq: [L][ny]; the h_hat column: [L][ny]
// complex).  In COL_SOLVE and COL_FILTER the two real columns packed in
// slot 0 are transformed apart (one rounding each).
hipError_t launch_col(int dtype, int mode, void* data, const void* Yf, const void* Yfnyq, const void* H2,
                      const void* H2nyq, double rhoQ, double scale, int L, int ny, int nx,
                      const void* tw, int twlog, double* partials, int* nblocks_out,
                      hipStream_t s, int variant = kDefaultColVariant);

// ---------------------------------------------------------------- grouped launches
// One launch covers the tiles of several independent cubes of one shape
// class.  Each cube's descriptor holds its arrays and the first and count of
// the blocks that work on it; blocks of the launch in no cube's range exit.
// The descriptor arrays live in device memory.
struct RowDesc {             // a row pass (forward: in = B_rest, out = Z; inverse: in = Z, out = X)
    const void* in;
    void* out;
    const void* tw;
    int nrows, twlog, first, nblk;
};
struct ColDesc {             // the solving column pass of one cube
    void* data;
    const void* Yf;
    const void* Yfn;
    const void* H2;
    const void* H2nyq;
    const void* tw;
    double rhoQ, scale;
    int L, M, twlog, first, nblk, pad;
};
// the [L][npix] arrays of the spectral pass: X, the state it reads (z_P,
// z_T, z_V = S - Gamma_S / rho_V, Gamma_S), the state it writes (the same
// arrays, or a second set in a reporting pass) and B_rest
struct SpecArrays {
    char *X, *zP, *zT, *zV, *GS;
    char *zPo, *zTo, *zVo, *GSo;
    char *Brest;
    unsigned band_bytes;
    int gshift;
};
struct SpecDesc {
    SpecArrays A;
    const void* D;
    SpecArgs a;
    long npix;
    int Lrt, first, nblk, pad;
};

// the host (g++) and device (hipcc) compilers must agree on these layouts
static_assert(sizeof(SpecArgs) == 48 && sizeof(RowDesc) == 40 && sizeof(ColDesc) == 88 &&
                  sizeof(SpecArrays) == 88 && sizeof(SpecDesc) == 168,
              "descriptor layout");

// blocks of one cube in a grouped launch (and its block size, spectral pass)
int spectral_gshift(unsigned band_bytes);     // SpecArrays::gshift for this band size
int row_blocks(int nrows, int nx, int variant);
int col_blocks(int dtype, int L, int ny, int nx, int variant);
int spectral_block_threads(long npix);
// pixels per block of the (grouped) spectral pass of L bands over npix
// pixels of elem bytes: the `nth` of launch_spectral_group (128 bands: 64
// pixels on two waves where spectral_pair_fits, i.e. 64 bands of an array
// span at most 2^31 bytes; otherwise one pixel per thread)
bool spectral_pair_fits(long npix, int elem);
int spectral_block_pixels(int L, long npix, int elem);
hipError_t launch_row_fwd_group(int dtype, int nx, int variant, const RowDesc* d, int n, int nblocks,
                                hipStream_t s);
hipError_t launch_row_inv_group(int dtype, int nx, int variant, const RowDesc* d, int n, int nblocks,
                                hipStream_t s);
hipError_t launch_col_group(int dtype, int ny, int variant, const ColDesc* d, int n, int nblocks,
                            hipStream_t s);
// cubes of one band count L and one block size; nth = spectral_block_pixels
// (npix >= 256 or all equal npix)
hipError_t launch_spectral_group(int dtype, int L, int nth, const SpecDesc* d, int n, int nblocks,
                                 hipStream_t s);

// ---------------------------------------------------------------- visibility model
// (muffin_vis.hip) Setup sums over the visibilities of each band (uv, vis:
// device, 2 doubles per visibility, band l from off[l] to off[l + 1]):
// mode 0 the Toeplitz kernel c on the 2ny x 2nx grid of lags, lag (0, 0) at
// (ny, nx); mode 1 the data term Re(H^H y) on the ny x nx image.
hipError_t launch_vis_sum(int dtype, int mode, const double* uv, const double* vis, const long* off, int L,
                          int ny, int nx, void* out, hipStream_t s);
// a cube of L unit impulses at pixel (ny/2, nx/2)
hipError_t launch_vis_delta(int dtype, void* out, int L, int ny, int nx, hipStream_t s);
// CG on Q_l x = b_l for every band: x, r, Ap, hty, brest plain cubes; P2 the
// zero-padded 2ny x 2nx cube holding p; A2 = Re(H^H H) p on the padded grid
// (the convolution's output); partials per (band, block); rr, alpha, beta
// per band (FP64, device).  CG_PAD: x into P2.  CG_INIT: r = hty + brest -
// (A2 + rho x), p = r, rr = r.r.  CG_AP: Ap = A2 + rho p, alpha = rr / p.Ap.
// CG_XR: x += alpha p, r -= alpha Ap, beta = r.r / rr, rr = r.r.  CG_P:
// p = r + beta p.
enum CgOp { CG_PAD = 0, CG_INIT = 1, CG_AP = 2, CG_XR = 3, CG_P = 4 };
struct CgVectors {
    int L, ny, nx;
    void *x, *r, *Ap, *P2;
    const void *A2, *hty, *brest;
    double *partials, *rr, *alpha, *beta;
};
int cg_blocks(long npix);       // blocks per band of the CG kernels (partials per band)
hipError_t launch_cg(int dtype, int op, const CgVectors& v, double rho, hipStream_t s);

// ---------------------------------------------------------------- reverse sweep
// FP64 cotangent slots accumulated per block by the adjoint kernels
enum GradSlot {
    G_TAU_T = 0,   // d/d tau_T
    G_TAU_V,       // d/d tau_V
    G_RHO_P,       // d/d rho_P, explicit terms
    G_RHO_T,
    G_RHO_V,
    G_RHO_S,
    G_RHO_Q,       // d/d rho of eq. Qlsimp
    G_LOSS,        // the MSE loss
    GRAD_NQ
};

// [L][npix] arrays of the adjoint of one pass: the state before the pass
// (z_P, z_T, z_V, Gamma_S), the pass's X, the state cotangents (in place;
// those of z_P, z_T, S and Gamma_S) and the cotangent of X; for the fused
// step-I adjoint of the pass after, its B-bar, state and X
struct AdjArrays {
    char *zP, *zT, *zV, *GS, *X;
    char *aP, *aT, *aS, *aG, *Xb;
    char *Bb = nullptr, *zP1 = nullptr, *zT1 = nullptr, *zV1 = nullptr, *GS1 = nullptr, *X1 = nullptr;
    unsigned band_bytes;
    int gshift;
};

// mode: 0 plain, 1 with an outside cotangent of X in Xb, 2 with the step-I
// adjoint of the pass after first (its parameter sums to partials1; only
// where adj_single_descriptor holds: every band array within 2^30 bytes).
// Both kernels run one thread per pixel (npix a power of two, at least 64).
bool adj_single_descriptor(int L, unsigned band_bytes);
// dense: the band transform is the dense product with D (up to 32 bands)
hipError_t launch_adj_spectral(int dtype, const AdjArrays& A, const void* D, int L, long npix,
                               const SpecArgs& a, int mode, double* partials, double* partials1, int* nblocks,
                               hipStream_t s, bool dense = false);
hipError_t launch_adj_step1(int dtype, const void* Bb, const void* zP, const void* zT, const void* zV,
                            const void* GS, const void* X, void* aP, void* aT, void* aS, void* aG, long npix, int L,
                            const SpecArgs& a, double* partials, int* nblocks, hipStream_t s);
hipError_t launch_mse_seed(int dtype, const void* X, const void* sky, void* Xb, size_t n,
                           double* partials, int* nblocks, hipStream_t s);
// acc[q] += the block sums of partials (GRAD_NQ per block), deterministic
hipError_t launch_grad_accum(const double* partials, int nblocks, double* acc, hipStream_t s);

// ---------------------------------------------------------------- fused row/spectral pass
// The inverse row pass, steps II-VI and the forward row pass in one launch
// (FP32, 64 <= nx <= 1024, L in {4, 8, 16, 32, 64}, a cube of at most 1 GiB):
// reads the column pass's
// spectrum Z and the state, writes X, the new state and the spectrum of
// B_rest over Z.
// the state is read from zP .. GS and written to zPo .. GSo (the same
// arrays for a pass in place)
struct FusedArrays {
    char *X, *zP, *zT, *zV, *GS;
    char *zPo, *zTo, *zVo, *GSo;
    char* Z;
    unsigned band_bytes;
    int gshift;
};
struct FusedDesc {                   // one cube of a grouped fused launch
    FusedArrays A;
    const void* D;
    SpecArgs a;
    const void* tw;
    int twlog, L, ny, first, nblk, pad;
};
static_assert(sizeof(FusedArrays) == 88 && sizeof(FusedDesc) == 176, "descriptor layout");
bool fused_supported(int dtype, int nx, int ny, int L);
hipError_t launch_fused_group(int dtype, int nx, int L, const FusedDesc* d, int n, int nblocks,
                              hipStream_t s);
// variant 1: one pixel per thread; 2: two pixels per thread where
// fused_two_pixel_variant(nx, L) (otherwise as 1); results agree to rounding.
// Every array of A must be set (for a pass in place zPo = zP, ...): a null
// one is rejected (hipErrorInvalidValue).
hipError_t launch_fused(int dtype, const FusedArrays& A, const void* D, int L, int ny, int nx,
                        const SpecArgs& a, const void* tw, int twlog, hipStream_t s, int variant);
bool fused_two_pixel_variant(int nx, int L);

// Arrays of one spectral pass.  st: the state read (z_P, z_T, z_V, Gamma_S;
// for a union of spectral bases z_P, z_T, S, Gamma_S); out: where the new
// state goes (= st except in a reporting pass).
struct SpecLaunch {
    const void* X = nullptr;
    void* st[4] = {nullptr, nullptr, nullptr, nullptr};
    void* out[4] = {nullptr, nullptr, nullptr, nullptr};   // = st for a pass in place
    void* brest = nullptr;
    const void* dctm;   // the dense transform(s): per basis D[k * LT + l] = W[l][k], LT = dense_width(L)
    int L;
    long npix;
    bool report;        // also run the reporting kernels: FP64 partials (RED_NQ per block)
    double* vpart;      // one double per block: sum of V^2 (reporting pass)
    double* partials;   // RED_NQ doubles per block (reporting pass)
    bool dense = false; // the band transform is the dense product with dctm (else the fast DCT)
    int n_nu = 1;       // spectral bases; > 1: a union, with the coefficient cubes below
    void* uz[4] = {nullptr, nullptr, nullptr, nullptr};    // z_V,j read
    void* uzo[4] = {nullptr, nullptr, nullptr, nullptr};   // z_V,j written
    // reporting pass with wavelet bases in W_s: rho_T W^T dT and W^T Gamma_T
    // summed over them (cubes like X), else null
    const void* wdt = nullptr;
    const void* wg = nullptr;
};

// Spectral pass (steps II-VI of one iteration) over every pixel.
hipError_t launch_spectral(int dtype, const SpecLaunch& g, const SpecArgs& a, int* nblocks_out,
                           hipStream_t s);

// Setup: combine the FP64 packed column spectra of the shifted PSF (Ch) and of
// the dirty image (Cy) into conj(h_hat) y_hat (Yf, and Yfnyq for the kx = nx/2
// column), |h_hat|^2 (H2, and H2nyq for the kx = nx/2 column), stored in the
// iteration's precision.  Yf and H2
// go in column-block order: per band, blocks of W adjacent kx columns (W =
// min(16, 64 KiB / (ny complex values), nx/2), the default column tile),
// each block's ny rows contiguous.
hipError_t launch_setup_combine(int dtype, const void* Ch, const void* Cy, void* Yf, void* Yfnyq, void* H2,
                                void* H2nyq, void* Hh, void* Hhnyq, int L, int ny, int nx, hipStream_t s);

// dst[i] += src[i], i < n
hipError_t launch_add(int dtype, void* dst, const void* src, size_t n, hipStream_t s);

// Non-finite scan of psf and dirty plus sum dirty^2; writes per-block
// partials (2 per block: count of non-finite values, sum of squares).
hipError_t launch_scan(bool in_f64, const void* psf, const void* dirty, size_t n,
                       double* partials, int* nblocks_out, hipStream_t s);

// out[q] = sum over blocks b of partials[b * nq + q], fixed order (deterministic).
hipError_t launch_reduce_final(const double* partials, int nblocks, int nq, double* out,
                               hipStream_t s);

// ---------------------------------------------------------------- wavelet bases
// One level of the periodised 2-D DWT of n wavelet bases over L images of
// sy x sx (powers of two >= 4), one launch for every basis and band.  Basis b
// uses the filter at ftab + 32 b (h then g, 16 taps each, in the iteration's
// precision; K / 2 in bits 4b .. 4b+3 of kpack), its input at in0 + b
// in_bstride elements (row stride in_ld, band stride in_bs), its coefficient
// cube at z0 + b zstride (row stride ld, band stride z_bs) and its dense LL
// image ([L][sy/2][sx/2]) at ll0 + b llstride, or LL in the cube when ll0 is
// null.  Analysis: z <- c + clip(z, tau) for the coefficients, LL to ll0.
// Synthesis (a level above the finest): the sy x sx images of
// u = 2 soft(z, tau) - z, into out0 + b outstride ([L][sy][sx]).
struct DwtLevel {
    const void* ftab;
    unsigned kpack;
    int n, L, sy, sx;
    const void* in0;
    long in_bstride, in_bs;
    int in_ld, ld;
    void* z0;
    long zstride, z_bs;
    void* ll0;
    long llstride;
    void* out0;
    long outstride;
    double tau;
    // analysis: 0 z_b <- c + clip(z_b, tau); 1 the same, with d_b = soft(z_b')
    // - soft(z_b) written to d0 (z_b's layout, basis stride dstride) and per
    // work-group the FP64 sums of (clip(z_b) - clip(z_b'))^2, rho_T ((clip(z_b)
    // - clip(z_b'))^2 + d_b^2) and soft(z_b')^2 to partials; 2 z_b untouched,
    // the sum of |c| per work-group to partials.  Synthesis: the coefficient
    // function, 0 u = 2 soft(z, tau) - z, 1 z itself, 2 -clip(z, tau)
    // 3 the adjoint of the update: z_b holds its cotangent after the pass,
    // overwritten with the one before it; the state's z_b before the pass
    // at s0 (stride sstride); GRAD_NQ sums per work-group (tau_T, rho_T)
    int mode = 0;
    void* d0 = nullptr;
    long dstride = 0;
    void* zo0 = nullptr;     // mode 0: the updated z_b to here (stride zostride) instead of in place
    long zostride = 0;
    const void* s0 = nullptr;
    long sstride = 0;
    double* partials = nullptr;
    double rho_T = 0.0;
    double scale = 1.0;      // the finest synthesis: out0 += scale * (sum over the bases)
};
// finest: one work-group per tile and band runs every basis over one staged
// image tile (grid z = L, one input image per band); else grid z = n L
hipError_t launch_dwt_fwd_all(int dtype, const DwtLevel& A, hipStream_t s, bool finest = false);
hipError_t launch_dwt_inv_all(int dtype, const DwtLevel& A, hipStream_t s);
// The finest synthesis level (sy x sx = ny x nx) of every basis, summed:
// out0 += scale * sum_b W_b^T f(z_b) at that level (LL from ll0, dense
// [L][ny/2][nx/2] per basis, or from z_b when null).
hipError_t launch_dwt_inv0_all(int dtype, const DwtLevel& A, hipStream_t s);

// Elementwise helpers.
hipError_t launch_fill_zero(void* p, size_t bytes, hipStream_t s);
// B_rest from the stored state; s_stored: the third array holds S itself (a
// union of spectral bases) instead of z_V = S - Gamma_S / rho_V
hipError_t launch_brest(int dtype, const void* zP, const void* zT, const void* zV, const void* GS,
                        void* Brest, size_t n, const SpecArgs& a, hipStream_t s, bool s_stored = false);
// A union of spectral bases under a new rho_V (ratio = rho_V / rho_V'):
// z_V,j <- (S W_j) (1 - ratio) + z_V,j ratio, which keeps S and Gamma_V,j
hipError_t launch_union_reencode(int dtype, const void* S, void* const* uz, int n_nu, const void* D, int L,
                                 long npix, double ratio, hipStream_t s);
hipError_t launch_positive(int dtype, const void* z, void* out, size_t n, hipStream_t s);
// z_P <- max(0, z_P) - rP max(0, -z_P);  z_T <- soft(z_T, tau) + rT clip(z_T, tau);
// z_V <- z_V + dV Gamma_S (dV = 1 / rho_V - 1 / rho_V', skipped when 0); a
// null zP, zT or zV is left out
hipError_t launch_reencode(int dtype, void* zP, void* zT, void* zV, const void* GS, size_t n, double rP,
                           double rT, double tau, double dV, hipStream_t s);

}  // namespace muffin
