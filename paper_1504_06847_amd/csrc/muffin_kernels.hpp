// Host-side declarations of the kernel launchers (implemented in
// muffin_kernels.hip).  All pointers are device pointers; every launcher
// returns the hipError_t of its launch.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>

namespace muffin {

enum ColMode { COL_SOLVE = 0, COL_FWD = 1, COL_OBJ = 2 };

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

// Row pass, forward: every row of `in` (nrows rows of nx reals, type float or
// double per in_f64) -> packed half spectrum `out` (nrows x nx/2 complex of
// type T).  shift: read the row through ifftshift (rows of each band of ny
// rows rotated by ny/2, columns by nx/2).  positive: read max(0, v).
hipError_t launch_row_fwd(int dtype, bool in_f64, const void* in, void* out, int nrows, int nx,
                          int ny, bool shift, bool positive, const void* tw, int twlog,
                          hipStream_t s);

// Row pass, inverse: packed half spectrum -> real rows (unnormalised).
hipError_t launch_row_inv(int dtype, const void* in, void* out, int nrows, int nx,
                          const void* tw, int twlog, hipStream_t s);

// Column pass over L bands of ny x (nx/2) packed spectra, in place.
// COL_SOLVE: FFT along y, X_hat = (Z + Yf) * scale / (H2 + rhoQ), inverse FFT.
// COL_FWD: FFT along y only.  COL_OBJ: FFT along y, then per-block FP64
// partials of sum w (H2 |Z|^2 - 2 Re(conj(Yf) Z)) / (nx ny) into partials.
hipError_t launch_col(int dtype, int mode, void* data, const void* Yf, const void* H2,
                      const void* H2nyq, double rhoQ, double scale, int L, int ny, int nx,
                      const void* tw, int twlog, double* partials, int* nblocks_out,
                      hipStream_t s);

// Arrays of one spectral pass.  st: the state read (z_P, z_T, S, Gamma_S);
// out: where the new state goes (= st except in a reporting pass).
struct SpecLaunch {
    const void* X;
    void* st[4];
    void* out[4];
    void* brest;
    const void* dctm;
    int L;
    long npix;
    bool report;        // also run k_report: FP64 partials (RED_NQ per block)
    double* vpart;      // one double per block: sum of V^2 (reporting pass)
    double* partials;   // RED_NQ doubles per block (reporting pass)
};

// Spectral pass (steps II-VI of one iteration) over every pixel.
hipError_t launch_spectral(int dtype, const SpecLaunch& g, const SpecArgs& a, int* nblocks_out,
                           hipStream_t s);

// Setup: combine the FP64 packed column spectra of the shifted PSF (Ch) and of
// the dirty image (Cy) into conj(h_hat) y_hat (Yf), |h_hat|^2 (H2, and H2nyq
// for the kx = nx/2 column), stored in the iteration's precision.
hipError_t launch_setup_combine(int dtype, const void* Ch, const void* Cy, void* Yf, void* H2,
                                void* H2nyq, int L, int ny, int nx, hipStream_t s);

// Non-finite scan of psf and dirty plus sum dirty^2; writes per-block
// partials (2 per block: count of non-finite values, sum of squares).
hipError_t launch_scan(bool in_f64, const void* psf, const void* dirty, size_t n,
                       double* partials, int* nblocks_out, hipStream_t s);

// out[q] = sum over blocks b of partials[b * nq + q], fixed order (deterministic).
hipError_t launch_reduce_final(const double* partials, int nblocks, int nq, double* out,
                               hipStream_t s);

// Elementwise helpers.
hipError_t launch_fill_zero(void* p, size_t bytes, hipStream_t s);
hipError_t launch_brest(int dtype, const void* zP, const void* zT, const void* S, const void* GS,
                        void* Brest, size_t n, const SpecArgs& a, hipStream_t s);
hipError_t launch_positive(int dtype, const void* z, void* out, size_t n, hipStream_t s);
// z_P <- max(0, z_P) - rP max(0, -z_P);  z_T <- soft(z_T, tau) + rT clip(z_T, tau)
hipError_t launch_reencode(int dtype, void* zP, void* zT, size_t n, double rP, double rT, double tau,
                           hipStream_t s);

}  // namespace muffin
