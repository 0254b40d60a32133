// Workspace layout and host-only helpers shared by the C ABI translation
// units.  Byte offsets into the caller's device workspace, each 256-B aligned.
#pragma once
#include <stddef.h>

#include "muffin.h"

namespace muffin {

constexpr size_t kAlign = 256;
constexpr int kNumState = 4;     // z_P, z_T, z_V = S - Gamma_S / rho_V, Gamma_S (Gamma_V = Gamma_S W_nu implied)
constexpr int kNumRed = 10;      // FP64 partial sums per block (see RedSlot)
enum StateIdx { ST_ZP = 0, ST_ZT = 1, ST_ZV = 2, ST_GS = 3 };

constexpr int kMaxWavelets = 8;  // Db1..Db8 beside the Dirac basis
constexpr int kMaxDwtLevels = 4;
// coefficients per sub-band of one DWT work-group tile (rows, columns)
constexpr int kDwtTileY = 16, kDwtTileX = 32;
// FP64 sums per work-group of a wavelet launch, at most (report: 3, the
// reverse sweep: one per gradient slot)
constexpr int kWPartQ = 8;
constexpr int kMaxSpectral = MUFFIN_MAX_SPECTRAL;

struct Layout {
    size_t state[2][kNumState];   // current and alternate state sets (a reporting
                                  // pass writes the alternate set, then they swap)
    size_t brest, x, z, yf, yfnyq, h2, h2nyq, tw, tw64, dctm, partials, vpart, sums;
    size_t hh, hhnyq;             // h_hat packed like Yf, and its kx = nx/2 column (complex)
    // wavelet bases of the spatial dictionary: one coefficient cube z_b per
    // basis, per basis the scratch image of each DWT level j >= 1 (its LL
    // block going down, its reconstruction coming back), and the filter
    // table (per basis h then g, 16 taps each, in the iteration's precision)
    size_t wz[kMaxWavelets];
    size_t wtmp[kMaxWavelets][kMaxDwtLevels];
    size_t wfilt;
    // a reporting pass with wavelet bases: three cubes (soft(z_b') -
    // soft(z_b) of the basis in hand, rho_T W^T dT and W^T Gamma_T summed
    // over the bases) and FP64 block sums of every analysis launch (also
    // the reverse sweep's)
    size_t wrep[3], wpart;
    long wblocks;
    int n_w, levels;
    // spectral bases: their number, and with more than one (a union) the
    // prox input of each basis's soft threshold, z_V,j = S W_j - Gamma_V,j /
    // rho_V in that basis's coefficients, in both state sets
    int n_nu;
    size_t uz[2][kMaxSpectral];
    size_t total;
    size_t setup_scratch_bytes, state_region_bytes;
    int nblk;
};

void set_error(const char* fmt, ...);
int validate_shape(const muffin_shape* s);
int validate_params(const muffin_params* p);
Layout make_layout(const muffin_shape* s, int n_s = 1, int n_nu = 1);
// whether the spectral transform of these parameters is a dense L x L
// product (any basis but the DCT alone at a power-of-two band count) and
// whether W_nu is a union of bases
bool spectral_dense(const muffin_shape& s, const muffin_params& p);
inline bool spectral_union(const muffin_params& p) { return p.n_nu > 1; }
// the orthonormal spectral basis `code` for L bands, row-major L x L,
// spectrum of a pixel = x W (long double; EINVAL for a bad code or L)
int spectral_basis_ld(int code, int L, long double* W);
// DWT depth of the wavelet bases: 4 levels, fewer when the smaller image side
// would leave a coarsest band under 2 x 2
int dwt_levels(int nx, int ny);
// work-groups of one DWT level over an sy x sx image, per band and basis
long dwt_tiles(int sy, int sx);
int max_blocks_host(int L, int ny, int nx);

// register width of the dense DCT used for band counts that are not powers of two
inline int dense_width(int L) { return L <= 8 ? 8 : (L <= 16 ? 16 : (L <= 32 ? 32 : (L <= 64 ? 64 : L))); }

}  // namespace muffin
