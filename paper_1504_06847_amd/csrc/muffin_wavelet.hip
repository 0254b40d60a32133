// The wavelet part of the spatial dictionary W_s (Section 4: the Dirac basis
// and the orthonormal Daubechies bases Db1-Db8) in steps III and VI of
// Algorithm 1 and in the right-hand side of step I (eq. matB), on gfx950.
//
// Per wavelet basis b the state holds z_b, the input of the spatial soft
// threshold in the coefficient domain (as z_T for the Dirac basis):
//   T_b = soft(z_b, tau_T),  Gamma_T,b = -rho_T clip(z_b, tau_T),
//   z_b <- W_b X + clip(z_b, tau_T)                       (steps III, VI)
// and the basis adds rho_T W_b^T (2 soft(z_b) - z_b) = W_b^T (rho_T T_b +
// Gamma_T,b) to B_rest.
//
// W_b is the periodised multi-level 2-D DWT with the length-K Daubechies
// filter h (wavelet filter g[k] = (-1)^k h[K-1-k]):
//   a[m] = sum_k h[k] x[(2m + k) mod n],  d[m] = sum_k g[k] x[(2m + k) mod n]
// along x, then along y, coefficients in Mallat layout (LL top-left, then
// x-high top-right, y-high bottom-left, both high bottom-right); each level
// recurses on LL.  A work-group transforms one tile (16 rows x 32 columns of
// coefficients per sub-band, so each row of a sub-band block is one 128-B
// line) staged with its periodic halo in LDS.
//   k_dwt_fwd_all: one analysis level of every basis and band in one launch;
//     the detail coefficients (and at the last level the LL block) go
//     straight into the z_b update, LL otherwise to the basis's dense
//     scratch image for the next level.
//   k_dwt_inv_all: one synthesis level above the finest of every basis, of
//     u_b = 2 soft(z_b) - z_b (the LL input from the coarser level's scratch
//     image, or from z_b at the last level).
//   k_dwt_inv0_all: the finest synthesis level of every basis, the bases
//     in order inside each work-group and their sum added into B_rest, so
//     B_rest is read and written once and the sum has a fixed order.
#include "muffin_device.hpp"
#include "muffin_kernels.hpp"
#include "muffin_layout.hpp"

namespace muffin {

constexpr int DWT_OTY = kDwtTileY;     // coefficient rows per sub-band per tile
constexpr int DWT_OTX = kDwtTileX;     // coefficient columns per sub-band per tile
constexpr int DWT_NTH = 256;

#define MUFFIN_DWT_K_CASES(F) F(2) F(4) F(6) F(8) F(10) F(12) F(14) F(16)

// LDS of one tile, in elements, for the longest filter (K = 16)
constexpr int DWT_FWD_LDS = (2 * DWT_OTY + 14) * (2 * DWT_OTX + 14) + 2 * (2 * DWT_OTY + 14) * DWT_OTX;
// row stride of the row synthesis's output in LDS: at least the tile's
// coefficient columns and 1 modulo 4, so that the column synthesis's reads
// (8 lanes per row, 4 columns apart) fall in distinct banks across rows
constexpr int dwt_xstride(int H2) { return DWT_OTX + H2 + ((1 - (DWT_OTX + H2)) & 3); }
constexpr int DWT_INV_LDS = 4 * (DWT_OTY + 7) * (DWT_OTX + 7) + 2 * (2 * DWT_OTY) * dwt_xstride(7);

// clip to [-t, t] (t >= 0, finite z: the median of z, -t and t) and soft
// threshold, soft(z) = z - clip(z) (exactly z - t, z + t or +0)
template <typename T> __device__ __forceinline__ T wclip(T z, T t) {
    if constexpr (sizeof(T) == 4) return __builtin_amdgcn_fmed3f(z, -t, t);
    else return fmin(fmax(z, -t), t);
}
template <typename T> __device__ __forceinline__ T wsoft(T z, T t) { return z - wclip(z, t); }
// z_b <- c + clip(z_b, tau)
template <typename T> __device__ __forceinline__ void zupdate(T* p, T c, T tau) { *p = c + wclip(*p, tau); }
// u = 2 soft(z, tau) - z = z - 2 clip(z, tau), one rounding
template <typename T> __device__ __forceinline__ T ucoef(T z, T tau) { return z - T(2) * wclip(z, tau); }
// the synthesis input of coefficient z: u (CF 0), z (CF 1), -clip(z) (CF 2)
template <typename T, int CF> __device__ __forceinline__ T scoef(T z, T tau) {
    if constexpr (CF == 0) return ucoef(z, tau);
    else if constexpr (CF == 1) return z;
    else return -wclip(z, tau);
}

// The report terms of one updated coefficient (old z, new zn): with
// T_b = soft(z_b), Gamma_T,b = -rho_T clip(z_b) and W_b X = zn - clip(z),
//   T_b' - W_b X = clip(z) - clip(zn),  dGamma_T,b = rho_T (clip(z) - clip(zn)),
// so r^2 gains dc^2, E gains rho_T dT^2 + rho_T dc^2, ||T||^2 gains soft(zn)^2.
struct WStats {
    double r2 = 0.0, e = 0.0, bz = 0.0;
};
template <typename T>
__device__ __forceinline__ T wstat(T z, T zn, T tau, T rT, WStats& st) {
    const T dc = wclip(z, tau) - wclip(zn, tau);
    const T tn = wsoft(zn, tau);
    const T dt = tn - wsoft(z, tau);
    st.r2 += double(dc * dc);
    st.e += double(rT * (dt * dt + dc * dc));
    st.bz += double(tn * tn);
    return dt;
}

// One analysis tile of an sy x sx image (one band): src with row stride
// in_ld; zb the band's coefficient block (row stride ld); llb the band's
// dense LL image ([sy/2][sx/2]) or null (last level: LL into zb).
// One analysis tile: oty x otx coefficients of each sub-band of an sy x sx
// image (one band) from the image rows and columns it needs (periodic
// halo of K - 2), staged in LDS.  Register blocking: a thread of the row
// pass forms DWT_MB adjacent outputs of one row from 2 DWT_MB + K - 2 LDS
// values, a thread of the column pass DWT_IB adjacent coefficient rows of
// one column (all four sub-bands) from 2 DWT_IB + K - 2 values of each row
// image, so each staged value is read a few times instead of K.  Each
// output's taps are summed in k order.
// MODE 0: update z_b; 1: update, soft(z_b') - soft(z_b) to db and the
// report terms into st; 2: no z_b access, sum |c| (LL at the last level
// included) into st.r2.
// The tile (x, y) and slice z of this work-group.  Work-groups go to the 8
// XCDs in turn (their linear id modulo 8), each XCD with its own L2; the
// tiles are renumbered so that each XCD takes one contiguous run of them,
// and neighbouring tiles, whose reads share the lines of their halos, meet
// in one L2.
struct Tile {
    int x, y, z;
};
__device__ __forceinline__ Tile xcd_tile() {
    const unsigned gx = gridDim.x, gy = gridDim.y, n = gx * gy * gridDim.z;
    unsigned l = (blockIdx.z * gy + blockIdx.y) * gx + blockIdx.x;
    if ((n & 7u) == 0) l = (l & 7u) * (n >> 3) + (l >> 3);
    Tile t;
    t.x = int(l % gx);
    l /= gx;
    t.y = int(l % gy);
    t.z = int(l / gy);
    return t;
}

constexpr int DWT_MB = 4;
constexpr int DWT_IB = 2;
// LDS of an analysis tile: the staged image (row stride for the longest
// filter, whatever the basis), then the row pass's low and high halves
constexpr int DWT_HMX = 2 * DWT_OTX + 14, DWT_HMY = 2 * DWT_OTY + 14;

// this thread's column-pass item: coefficient rows ci .. ci + DWT_IB - 1 of
// column cm (oty >= 2, so (oty / DWT_IB) otx <= 256 items)
struct FwdItem {
    bool on;
    int ci, cm;
};
__device__ __forceinline__ FwdItem fwd_item(int oty, int otx) {
    return {(int)threadIdx.x < (oty / DWT_IB) * otx, (int)(threadIdx.x / otx) * DWT_IB, (int)(threadIdx.x % otx)};
}

// The coefficients the item updates (zq[r][sub-band]; the LL one only at
// the last level), and with MODE 3 the state's at the same places (sq),
// loaded ahead of the tile so that their latency overlaps it.
template <typename T, int MODE>
__device__ __forceinline__ void fwd_load_z(const T* __restrict__ zb, const T* __restrict__ zs, int ld, bool last,
                                           int sy, int sx, const Tile& tl, const FwdItem& it, T (&zq)[DWT_IB][4],
                                           T (&sq)[DWT_IB][4]) {
    if (MODE == 2 || !it.on) return;
    const int hy = sy >> 1, hx = sx >> 1;
    const int oty = hy < DWT_OTY ? hy : DWT_OTY, otx = hx < DWT_OTX ? hx : DWT_OTX;
    const int i0 = tl.y * oty, m0 = tl.x * otx;
#pragma unroll
    for (int r = 0; r < DWT_IB; ++r) {
        const long gi = i0 + it.ci + r, gm = m0 + it.cm;
        zq[r][0] = zb[gi * ld + hx + gm];
        zq[r][1] = zb[(hy + gi) * ld + gm];
        zq[r][2] = zb[(hy + gi) * ld + hx + gm];
        zq[r][3] = last ? zb[gi * ld + gm] : T(0);
        if constexpr (MODE == 3) {
            sq[r][0] = zs[gi * ld + hx + gm];
            sq[r][1] = zs[(hy + gi) * ld + gm];
            sq[r][2] = zs[(hy + gi) * ld + hx + gm];
            sq[r][3] = last ? zs[gi * ld + gm] : T(0);
        }
    }
}

// The adjoint of one coefficient (MODE 3): zb the cotangent of z_b after the
// pass, s the state's z_b before it, c the coefficient of W_b B-bar.  The
// pass maps z_b to W_b X + clip(z_b) and its step I reads rho_T W_b^T
// (2 soft(z_b) - z_b), so the cotangent of z_b before the pass is
// clip'(s) zb + rho_T (2 soft'(s) - 1) c; tau_T gains
// sgn(s) 1[|s| > tau] (zb - 2 rho_T c), rho_T gains c (2 soft(s) - s).
template <typename T>
__device__ __forceinline__ T wadj(T zb, T s, T c, T tau, T rT, WStats& st) {
    const bool out = fabs(s) > tau;
    const T sg = s > T(0) ? T(1) : (s < T(0) ? T(-1) : T(0));
    st.r2 += double(out ? sg * (zb - T(2) * rT * c) : T(0));
    st.e += double(c * (T(2) * wsoft(s, tau) - s));
    return (out ? T(0) : zb) + (out ? rT : -rT) * c;
}

// Stage the image rows and columns an analysis tile with filters of up to
// K taps needs (periodic halo of K - 2 below and right) into tin.
template <typename T>
__device__ __forceinline__ void fwd_stage(const T* __restrict__ src, int in_ld, int sy, int sx, int K, const Tile& tl,
                                          T* tin) {
    const int hy = sy >> 1, hx = sx >> 1;
    const int oty = hy < DWT_OTY ? hy : DWT_OTY, otx = hx < DWT_OTX ? hx : DWT_OTX;
    const int i0 = tl.y * oty, m0 = tl.x * otx;
    const int HY = 2 * oty + K - 2, HX = 2 * otx + K - 2;
    for (int e = threadIdx.x; e < HY * HX; e += DWT_NTH) {
        const int r = e / HX, c = e - r * HX;
        tin[r * DWT_HMX + c] = src[(long)((2 * i0 + r) & (sy - 1)) * in_ld + ((2 * m0 + c) & (sx - 1))];
    }
}

// One analysis tile of one basis (filter length K) from the staged image:
// oty x otx coefficients of each sub-band of an sy x sx image.  Register
// blocking: a thread of the row pass forms DWT_MB adjacent outputs of one
// row from 2 DWT_MB + K - 2 LDS values, a thread of the column pass DWT_IB
// adjacent coefficient rows of one column (all four sub-bands) from
// 2 DWT_IB + K - 2 values of each row image, so each staged value is read a
// few times instead of K.  Each output's taps are summed in k order.
// MODE 0: z_b <- c + clip(z_b) (written to zo: zb itself, or another cube
// of the same layout); 1: the same in place, soft(z_b') - soft(z_b) to db
// and the report terms into st; 2: no z_b access, sum |c| (LL at the last
// level included) into st.r2; 3: the adjoint (wadj) in place, with the
// state's z_b in sq.  Starts and ends between barriers: the caller
// synchronises after the staging and before the next tile's row pass.
template <typename T, int K, int MODE>
__device__ __forceinline__ void dwt_fwd_tile(T* __restrict__ zb, T* __restrict__ zo, int ld, T* __restrict__ llb,
                                             int sy, int sx, const T (&h)[K], const T (&g)[K], T tau, T* smem,
                                             T* __restrict__ db, T rT, WStats& st, const Tile& tl,
                                             const FwdItem& it, const T (&zq)[DWT_IB][4],
                                             const T (&sq)[DWT_IB][4]) {
    constexpr int NV = 2 * DWT_MB + K - 2, NR = 2 * DWT_IB + K - 2;
    const T* tin = smem;
    T* rl = smem + DWT_HMY * DWT_HMX;
    T* rh = rl + DWT_HMY * DWT_OTX;
    const int hy = sy >> 1, hx = sx >> 1;
    const int oty = hy < DWT_OTY ? hy : DWT_OTY, otx = hx < DWT_OTX ? hx : DWT_OTX;
    const int i0 = tl.y * oty, m0 = tl.x * otx;
    const int HY = 2 * oty + K - 2;
    // along x: row r, outputs mb .. mb + DWT_MB - 1 (DWT_OTX / DWT_MB items
    // per row whatever the tile's width: a narrower tile reads past its
    // columns inside the LDS array and keeps only its own outputs)
    constexpr int NMB = DWT_OTX / DWT_MB;
    for (int e = threadIdx.x; e < HY * NMB; e += DWT_NTH) {
        const int r = e / NMB, mb = (e - r * NMB) * DWT_MB;
        const T* row = tin + r * DWT_HMX + 2 * mb;
        T v[NV];
#pragma unroll
        for (int t = 0; t < NV; ++t) v[t] = row[t];
#pragma unroll
        for (int o = 0; o < DWT_MB; ++o) {
            T lo = T(0), hi = T(0);
#pragma unroll
            for (int k = 0; k < K; ++k) {
                lo += h[k] * v[2 * o + k];
                hi += g[k] * v[2 * o + k];
            }
            if (mb + o < otx) {
                rl[r * DWT_OTX + mb + o] = lo;
                rh[r * DWT_OTX + mb + o] = hi;
            }
        }
    }
    __syncthreads();
    if (!it.on) return;
    // along y: the four sub-bands of rows ci + r; z <- c + clip(z, tau)
    const int ci = it.ci, cm = it.cm;
    T vl[NR], vh[NR];
#pragma unroll
    for (int t = 0; t < NR; ++t) {
        vl[t] = rl[(2 * ci + t) * DWT_OTX + cm];
        vh[t] = rh[(2 * ci + t) * DWT_OTX + cm];
    }
#pragma unroll
    for (int r = 0; r < DWT_IB; ++r) {
        T a = T(0), by = T(0), bx = T(0), d = T(0);
#pragma unroll
        for (int k = 0; k < K; ++k) {
            a += h[k] * vl[2 * r + k];
            by += g[k] * vl[2 * r + k];
            bx += h[k] * vh[2 * r + k];
            d += g[k] * vh[2 * r + k];
        }
        const long gi = i0 + ci + r, gm = m0 + cm;
        if constexpr (MODE == 0) {
            zo[gi * ld + hx + gm] = bx + wclip(zq[r][0], tau);               // x high, y low
            zo[(hy + gi) * ld + gm] = by + wclip(zq[r][1], tau);             // x low, y high
            zo[(hy + gi) * ld + hx + gm] = d + wclip(zq[r][2], tau);
            if (llb) llb[gi * hx + gm] = a;
            else zo[gi * ld + gm] = a + wclip(zq[r][3], tau);
            continue;
        }
        if constexpr (MODE == 3) {
            zb[gi * ld + hx + gm] = wadj(zq[r][0], sq[r][0], bx, tau, rT, st);
            zb[(hy + gi) * ld + gm] = wadj(zq[r][1], sq[r][1], by, tau, rT, st);
            zb[(hy + gi) * ld + hx + gm] = wadj(zq[r][2], sq[r][2], d, tau, rT, st);
            if (llb) llb[gi * hx + gm] = a;
            else zb[gi * ld + gm] = wadj(zq[r][3], sq[r][3], a, tau, rT, st);
            continue;
        }
        if (llb) llb[gi * hx + gm] = a;
        if constexpr (MODE == 2) {
            st.r2 += double(fabs(bx)) + double(fabs(by)) + double(fabs(d));
            if (!llb) st.r2 += double(fabs(a));
            continue;
        }
        const long o0 = gi * ld + hx + gm, o1 = (hy + gi) * ld + gm, o2 = (hy + gi) * ld + hx + gm,
                   o3 = gi * ld + gm;
        const T n0 = bx + wclip(zq[r][0], tau);               // x high, y low
        const T n1 = by + wclip(zq[r][1], tau);               // x low, y high
        const T n2 = d + wclip(zq[r][2], tau);
        const T n3 = a + wclip(zq[r][3], tau);
        zb[o0] = n0;
        zb[o1] = n1;
        zb[o2] = n2;
        if (!llb) zb[o3] = n3;
        if constexpr (MODE == 1) {
            db[o0] = wstat(zq[r][0], n0, tau, rT, st);
            db[o1] = wstat(zq[r][1], n1, tau, rT, st);
            db[o2] = wstat(zq[r][2], n2, tau, rT, st);
            if (!llb) db[o3] = wstat(zq[r][3], n3, tau, rT, st);
        }
    }
}

// Synthesis output ownership: thread t forms 8 adjacent pixels (columns
// c0 .. c0 + 7) of row rr of the 2 DWT_OTY x 2 DWT_OTX pixels a tile
// computes; n of them lie in the image's 2 oty x 2 otx tile (fewer than 8
// only when the image is narrower than 4 coefficients).  False for threads
// whose pixels all lie outside it.
constexpr int DWT_C2 = 4;    // coefficient columns per thread in the column synthesis (8 pixels)
constexpr int DWT_XT = DWT_OTX / DWT_C2;    // threads per output row
static_assert(2 * DWT_OTY * DWT_XT == DWT_NTH, "one thread per 8 output pixels");
__device__ __forceinline__ bool inv_out(int oty, int otx, int& rr, int& c0, int& n) {
    const int t = threadIdx.x;
    rr = t / DWT_XT;
    c0 = (t % DWT_XT) * 2 * DWT_C2;
    n = 2 * otx - c0 < 2 * DWT_C2 ? 2 * otx - c0 : 2 * DWT_C2;
    return rr < 2 * oty && c0 < 2 * otx;
}

// The coefficients of one synthesis tile, whatever its filter: the
// (DWT_OTY + 7) x (DWT_OTX + 7) block of each sub-band that starts 7 rows
// and columns before the tile's own (the halo of the longest filter),
// periodic, fetched into registers ahead of their use and committed to LDS
// with that row stride, so a block element's LDS index is its fetch index.
// A filter of length 2 H2 + 2 reads the block from (7 - H2, 7 - H2).  A
// tile narrower or shorter than DWT_OTY x DWT_OTX (small images) still
// fills and computes the whole block from the periodic extension and keeps
// only its own pixels.
constexpr int DWT_SY = DWT_OTY + 7, DWT_SX = DWT_OTX + 7, DWT_SE = DWT_SY * DWT_SX;
constexpr int DWT_PF = (DWT_SE + DWT_NTH - 1) / DWT_NTH;
// Where this thread's block elements lie in a sub-band, the same for every
// basis of a level: periodic coefficient row gi and column gm, packed as
// gi << 16 | gm (sub-bands below 65536 x 65536).
struct InvOffsets {
    unsigned rc[DWT_PF];
};
__device__ __forceinline__ InvOffsets inv_offsets(int sy, int sx, const Tile& tl) {
    const int hy = sy >> 1, hx = sx >> 1;
    const int oty = hy < DWT_OTY ? hy : DWT_OTY, otx = hx < DWT_OTX ? hx : DWT_OTX;
    const int i0 = tl.y * oty, m0 = tl.x * otx;
    InvOffsets f;
#pragma unroll
    for (int j = 0; j < DWT_PF; ++j) {
        const int e = threadIdx.x + j * DWT_NTH;
        const int n = e / DWT_SX, q = e - n * DWT_SX;
        // periodic coefficient indices i0 - 7 + n, m0 - 7 + q (hy, hx powers of two)
        const unsigned gi = unsigned(i0 - 7 + n + 8 * hy) & unsigned(hy - 1);
        const unsigned gm = unsigned(m0 - 7 + q + 8 * hx) & unsigned(hx - 1);
        f.rc[j] = gi << 16 | gm;
    }
    return f;
}
// the block into registers: from the band's coefficient block zb (row
// stride ld; LL from llb, the band's dense [sy/2][sx/2] image, when not null)
template <typename T>
__device__ __forceinline__ void inv_fetch(const T* __restrict__ llb, const T* __restrict__ zb, int ld, int sy,
                                          int sx, const InvOffsets& f, T (&pf)[DWT_PF][4]) {
    const long hy = sy >> 1, hx = sx >> 1;
    const T* __restrict__ zx = zb + hx;
    const T* __restrict__ zy = zb + hy * ld;
    const T* __restrict__ zd = zy + hx;
#pragma unroll
    for (int j = 0; j < DWT_PF; ++j) {
        if (j + 1 < DWT_PF || int(threadIdx.x) + j * DWT_NTH < DWT_SE) {
            const unsigned gi = f.rc[j] >> 16, gm = f.rc[j] & 0xffffu;
            const unsigned zo = gi * unsigned(ld) + gm;
            pf[j][0] = llb ? llb[gi * unsigned(hx) + gm] : zb[zo];
            pf[j][1] = zx[zo];
            pf[j][2] = zy[zo];
            pf[j][3] = zd[zo];
        }
    }
}

// The fetched coefficients into LDS as f(z) (scoef; the LL block as it is
// when it came from a coarser level's image).  The caller synchronises
// before the tile reads them.
template <typename T, int CF>
__device__ __forceinline__ void inv_commit(const T (&pf)[DWT_PF][4], bool ll_image, T tau, T* smem) {
#pragma unroll
    for (int j = 0; j < DWT_PF; ++j) {
        const int e = threadIdx.x + j * DWT_NTH;
        if (j + 1 < DWT_PF || e < DWT_SE) {
            smem[e] = ll_image ? pf[j][0] : scoef<T, CF>(pf[j][0], tau);
            smem[DWT_SE + e] = scoef<T, CF>(pf[j][1], tau);
            smem[2 * DWT_SE + e] = scoef<T, CF>(pf[j][2], tau);
            smem[3 * DWT_SE + e] = scoef<T, CF>(pf[j][3], tau);
        }
    }
}

// One synthesis tile producing 2 DWT_OTY x 2 DWT_OTX pixels of one band
// from the four sub-bands committed to LDS (inv_commit; the caller
// synchronises after committing), added to the thread's 8 pixels acc
// (inv_out).  Register blocking: a thread of the row synthesis forms both
// output parities of 2 coefficient rows of one column from K / 2 + 1 rows of
// each sub-band, one pair of sub-bands at a time (LL with y-high, then x-high
// with diagonal); a thread of the column synthesis forms 8 adjacent pixels
// from K / 2 + 3 values of each half.  Each output's taps are summed in tap
// order, the low-pass term of a tap before its high-pass term, one fused
// multiply-add each.  Ends with a barrier, so the next tile may reuse the
// LDS at once.
template <typename T, int K>
__device__ __forceinline__ void dwt_inv_tile(const T (&h)[K], const T (&g)[K], T* smem, T (&acc)[2 * DWT_C2]) {
    constexpr int H2 = K / 2 - 1;                 // coefficient halo below the tile
    constexpr int OFF = 7 - H2;                   // where this filter's block starts in the fetched one
    constexpr int CX = DWT_OTX + H2;              // coefficient columns the row synthesis forms
    constexpr int NY = K / 2 + 1, NX = K / 2 + DWT_C2 - 1;
    const T* ca = smem + OFF * DWT_SX + OFF;
    const T* cbx = ca + DWT_SE;
    const T* cby = cbx + DWT_SE;
    const T* cd = cby + DWT_SE;
    constexpr int CMX = dwt_xstride(H2);
    T* xl = smem + 4 * DWT_SE;
    T* xh = xl + 2 * DWT_OTY * CMX;
    // along y: coefficient rows r2 = rb + r (r < 2) of column q, output rows
    // 2 r2 + p; row r2 takes coefficient rows r2 + H2 - kk, kk < K / 2 (one
    // item at a time: two unrolled would double the registers it holds)
#pragma unroll 1
    for (int e = threadIdx.x; e < (DWT_OTY / 2) * CX; e += DWT_NTH) {
        const int rb = (e / CX) * 2, q = e - (e / CX) * CX;
        // the low half (LL, y-high) then the high half (x-high, diagonal):
        // two sub-bands' rows held at a time
#pragma unroll
        for (int half = 0; half < 2; ++half) {
            const T* c0 = half ? cbx : ca;
            const T* c1 = half ? cd : cby;
            T* xo = half ? xh : xl;
            T v0[NY], v1[NY];
#pragma unroll
            for (int t = 0; t < NY; ++t) {
                v0[t] = c0[(rb + t) * DWT_SX + q];
                v1[t] = c1[(rb + t) * DWT_SX + q];
            }
#pragma unroll
            for (int r = 0; r < 2; ++r)
#pragma unroll
                for (int p = 0; p < 2; ++p) {
                    T a = T(0);
#pragma unroll
                    for (int kk = 0; kk < K / 2; ++kk) {
                        const int t = r + H2 - kk;
                        a += h[2 * kk + p] * v0[t];
                        a += g[2 * kk + p] * v1[t];
                    }
                    xo[(2 * (rb + r) + p) * CMX + q] = a;
                }
            __builtin_amdgcn_sched_barrier(0);
        }
    }
    __syncthreads();
    // along x: row rr, coefficient columns c2 = cb + c (c < DWT_C2), output
    // columns 2 c2 + p; column c2 takes c2 + H2 - kk, kk < K / 2
    {
        const int rr = threadIdx.x / DWT_XT, cb = (threadIdx.x % DWT_XT) * DWT_C2;
        T ul[NX], uh[NX];
#pragma unroll
        for (int t = 0; t < NX; ++t) {
            ul[t] = xl[rr * CMX + cb + t];
            uh[t] = xh[rr * CMX + cb + t];
        }
#pragma unroll
        for (int c = 0; c < DWT_C2; ++c)
#pragma unroll
            for (int p = 0; p < 2; ++p) {
                T v = T(0);
#pragma unroll
                for (int kk = 0; kk < K / 2; ++kk) {
                    const int t = c + H2 - kk;
                    v += h[2 * kk + p] * ul[t];
                    v += g[2 * kk + p] * uh[t];
                }
                acc[2 * c + p] += v;
            }
    }
    __syncthreads();
}

template <typename T, int K>
__device__ __forceinline__ void load_taps(const T* __restrict__ fb, T (&h)[K], T (&g)[K]) {
#pragma unroll
    for (int k = 0; k < K; ++k) {
        h[k] = fb[k];
        g[k] = fb[16 + k];
    }
}

// The work-group's FP64 report sums (MODE 1: 3, MODE 2: 1) into
// partials[work-group * nq + q].
// (MODE 3: GRAD_NQ per work-group, the tau_T and rho_T slots filled)
template <int MODE>
__device__ __forceinline__ void fwd_sums(const WStats& st, double* partials) {
    if constexpr (MODE != 0) {
        __shared__ double sh[DWT_NTH / 64];
        const long wg = ((long)blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x;
        constexpr int nq = MODE == 1 ? 3 : (MODE == 2 ? 1 : 2);
        const double v[3] = {st.r2, st.e, st.bz};
        double out[3];
#pragma unroll
        for (int q = 0; q < nq; ++q) out[q] = block_sum_s<DWT_NTH>(v[q], sh);
        if (threadIdx.x == 0) {
            if constexpr (MODE == 3) {
                for (int q = 0; q < GRAD_NQ; ++q) partials[wg * GRAD_NQ + q] = 0.0;
                partials[wg * GRAD_NQ + G_TAU_T] = out[0];
                partials[wg * GRAD_NQ + G_RHO_T] = out[1];
            } else {
#pragma unroll
                for (int q = 0; q < nq; ++q) partials[wg * nq + q] = out[q];
            }
        }
    }
}

#define MUFFIN_DWT_FWD_CASE(KK)                                                                  \
    case KK: {                                                                                   \
        T h[KK], g[KK];                                                                          \
        load_taps<T, KK>(fb, h, g);                                                              \
        dwt_fwd_tile<T, KK, MODE>(zb, zo, A.ld, llb, A.sy, A.sx, h, g, T(A.tau), smem, db,       \
                                  T(A.rho_T), st, tl, it, zq, sq);                               \
        break;                                                                                   \
    }

// One analysis level of every basis and band (a level above the finest).
// MODE 1 and 2 end with the work-group's FP64 sums (fwd_sums).
template <typename T, int MODE>
__global__ void __launch_bounds__(DWT_NTH, (sizeof(T) == 4 && MODE == 0) ? 6 : 1) k_dwt_fwd_all(DwtLevel A) {
    __shared__ T smem[DWT_FWD_LDS];
    // slice z = band * n + basis: the bases of one band run side by side, so
    // the re-reads of its image hit the caches
    const Tile tl = xcd_tile();
    const long band = tl.z / A.n;
    const int b = tl.z - int(band) * A.n;
    const T* src = (const T*)A.in0 + b * A.in_bstride + band * A.in_bs;
    T* zb = MODE == 2 ? nullptr : (T*)A.z0 + b * A.zstride + band * A.z_bs;
    T* zo = A.zo0 ? (T*)A.zo0 + b * A.zostride + band * A.z_bs : zb;
    const T* zs = MODE == 3 ? (const T*)A.s0 + b * A.sstride + band * A.z_bs : nullptr;
    T* db = MODE == 1 ? (T*)A.d0 + b * A.dstride + band * A.z_bs : nullptr;
    T* llb = A.ll0 ? (T*)A.ll0 + b * A.llstride + band * long(A.sy / 2) * (A.sx / 2) : nullptr;
    const T* fb = (const T*)A.ftab + 32 * b;
    const int K = 2 * int((A.kpack >> (4 * b)) & 15u);
    const int hy = A.sy >> 1, hx = A.sx >> 1;
    const FwdItem it = fwd_item(hy < DWT_OTY ? hy : DWT_OTY, hx < DWT_OTX ? hx : DWT_OTX);
    T zq[DWT_IB][4], sq[DWT_IB][4];
    fwd_load_z<T, MODE>(zb, zs, A.ld, llb == nullptr, A.sy, A.sx, tl, it, zq, sq);
    fwd_stage<T>(src, A.in_ld, A.sy, A.sx, K, tl, smem);
    __syncthreads();
    WStats st;
    switch (K) {
        MUFFIN_DWT_K_CASES(MUFFIN_DWT_FWD_CASE)
        default: break;
    }
    fwd_sums<MODE>(st, A.partials);
}

// The finest analysis level of every basis: one work-group per tile and
// band stages the image tile once (with the longest filter's halo) and
// runs the bases over it in order.  MODE 1 and 2 end with the work-group's
// FP64 sums (fwd_sums).
template <typename T, int MODE>
__global__ void __launch_bounds__(DWT_NTH) k_dwt_fwd0_all(DwtLevel A) {
    __shared__ T smem[DWT_FWD_LDS];
    const Tile tl = xcd_tile();
    const long band = tl.z;
    const T* src = (const T*)A.in0 + band * A.in_bs;
    const int hy = A.sy >> 1, hx = A.sx >> 1;
    const FwdItem it = fwd_item(hy < DWT_OTY ? hy : DWT_OTY, hx < DWT_OTX ? hx : DWT_OTX);
    int kmax = 2;
    for (int b = 0; b < A.n; ++b) {
        const int K = 2 * int((A.kpack >> (4 * b)) & 15u);
        kmax = K > kmax ? K : kmax;
    }
    T zq[DWT_IB][4], sq[DWT_IB][4];
    fwd_load_z<T, MODE>(MODE == 2 ? nullptr : (const T*)A.z0 + band * A.z_bs,
                        MODE == 3 ? (const T*)A.s0 + band * A.z_bs : nullptr, A.ld, A.ll0 == nullptr, A.sy, A.sx,
                        tl, it, zq, sq);
    fwd_stage<T>(src, A.in_ld, A.sy, A.sx, kmax, tl, smem);
    __syncthreads();
    WStats st;
    for (int b = 0; b < A.n; ++b) {
        T* zb = MODE == 2 ? nullptr : (T*)A.z0 + b * A.zstride + band * A.z_bs;
        T* zo = A.zo0 ? (T*)A.zo0 + b * A.zostride + band * A.z_bs : zb;
        const T* zs = MODE == 3 ? (const T*)A.s0 + b * A.sstride + band * A.z_bs : nullptr;
        T* db = MODE == 1 ? (T*)A.d0 + b * A.dstride + band * A.z_bs : nullptr;
        T* llb = A.ll0 ? (T*)A.ll0 + b * A.llstride + band * long(A.sy / 2) * (A.sx / 2) : nullptr;
        const T* fb = (const T*)A.ftab + 32 * b;
        if (b > 0) fwd_load_z<T, MODE>(zb, zs, A.ld, llb == nullptr, A.sy, A.sx, tl, it, zq, sq);
        switch (2 * int((A.kpack >> (4 * b)) & 15u)) {
            MUFFIN_DWT_K_CASES(MUFFIN_DWT_FWD_CASE)
            default: break;
        }
        // the next basis's row pass overwrites the row images
        __syncthreads();
    }
    fwd_sums<MODE>(st, A.partials);
}
#undef MUFFIN_DWT_FWD_CASE

// One synthesis level (not the finest) of every basis and band into the
// bases' dense scratch images: slice z = basis * L + band, the tiles
// numbered so that each XCD takes a contiguous run (the halos that
// neighbouring tiles share meet in one L2).
template <typename T, int CF>
__global__ void __launch_bounds__(DWT_NTH) k_dwt_inv_all(DwtLevel A) {
    __shared__ T smem[DWT_INV_LDS];
    const Tile tl = xcd_tile();
    const int b = tl.z / A.L;
    const long band = tl.z - b * A.L;
    const T* zb = (const T*)A.z0 + b * A.zstride + band * A.z_bs;
    const T* llb = A.ll0 ? (const T*)A.ll0 + b * A.llstride + band * long(A.sy / 2) * (A.sx / 2) : nullptr;
    T* ob = (T*)A.out0 + b * A.outstride + band * long(A.sy) * A.sx;
    const T* fb = (const T*)A.ftab + 32 * b;
    T acc[2 * DWT_C2] = {};
    const int K = 2 * int((A.kpack >> (4 * b)) & 15u);
    {
        T pf[DWT_PF][4];
        inv_fetch<T>(llb, zb, A.ld, A.sy, A.sx, inv_offsets(A.sy, A.sx, tl), pf);
        inv_commit<T, CF>(pf, llb != nullptr, T(A.tau), smem);
    }
    __syncthreads();
    switch (K) {
#define F(KK)                                                                              \
    case KK: {                                                                             \
        T h[KK], g[KK];                                                                    \
        load_taps<T, KK>(fb, h, g);                                                        \
        dwt_inv_tile<T, KK>(h, g, smem, acc);                                              \
        break;                                                                             \
    }
        MUFFIN_DWT_K_CASES(F)
#undef F
        default: break;
    }
    const int hy = A.sy >> 1, hx = A.sx >> 1;
    const int oty = hy < DWT_OTY ? hy : DWT_OTY, otx = hx < DWT_OTX ? hx : DWT_OTX;
    int rr, c0, n;
    if (inv_out(oty, otx, rr, c0, n)) {
        T* o = ob + long(2 * tl.y * oty + rr) * A.sx + 2 * tl.x * otx + c0;
#pragma unroll
        for (int c = 0; c < 2 * DWT_C2; ++c)
            if (c < n) o[c] = acc[c];
    }
}

// The finest synthesis level of every basis, summed and added into out
// ([L][sy][sx], row stride sx): out += scale * sum_b x_b, the bases in
// order inside the work-group, so out is read and written once and the sum
// has a fixed order.  Slice z = band.
template <typename T, int CF>
__global__ void __launch_bounds__(DWT_NTH, sizeof(T) == 4 ? 4 : 3) k_dwt_inv0_all(DwtLevel A) {
    __shared__ T smem[DWT_INV_LDS];
    const Tile tl = xcd_tile();
    const long band = tl.z;
    const long vb = long(A.sy) * A.sx;
    const int hy = A.sy >> 1, hx = A.sx >> 1;
    const int oty = hy < DWT_OTY ? hy : DWT_OTY, otx = hx < DWT_OTX ? hx : DWT_OTX;
    const int i0 = tl.y * oty, m0 = tl.x * otx;
    T* ob = (T*)A.out0 + band * vb;
    int rr, c0, n;
    const bool own = inv_out(oty, otx, rr, c0, n);
    T* o = ob + long(2 * i0 + rr) * A.sx + 2 * m0 + c0;
    T oq[2 * DWT_C2], acc[2 * DWT_C2] = {};
    // the coefficients of basis b + 1 are fetched while basis b is
    // synthesised, the outputs while the last basis is
    auto zb_of = [&](int b) { return (const T*)A.z0 + b * A.zstride + band * A.z_bs; };
    auto llb_of = [&](int b) { return A.ll0 ? (const T*)A.ll0 + b * A.llstride + band * (vb / 4) : nullptr; };
    auto k_of = [&](int b) { return 2 * int((A.kpack >> (4 * b)) & 15u); };
    const InvOffsets fo = inv_offsets(A.sy, A.sx, tl);
    T pf[DWT_PF][4];
    inv_fetch<T>(llb_of(0), zb_of(0), A.ld, A.sy, A.sx, fo, pf);
    for (int b = 0; b < A.n; ++b) {
        const int K = k_of(b);
        inv_commit<T, CF>(pf, A.ll0 != nullptr, T(A.tau), smem);
        __syncthreads();
        if (b + 1 < A.n) {
            inv_fetch<T>(llb_of(b + 1), zb_of(b + 1), A.ld, A.sy, A.sx, fo, pf);
        } else if (own) {
#pragma unroll
            for (int c = 0; c < 2 * DWT_C2; ++c)
                if (c < n) oq[c] = o[c];
        }
        const T* fb = (const T*)A.ftab + 32 * b;
        switch (K) {
#define F(KK)                                                                              \
    case KK: {                                                                             \
        T h[KK], g[KK];                                                                    \
        load_taps<T, KK>(fb, h, g);                                                        \
        dwt_inv_tile<T, KK>(h, g, smem, acc);                                              \
        break;                                                                             \
    }
            MUFFIN_DWT_K_CASES(F)
#undef F
            default: break;
        }
    }
    const T scale = T(A.scale);
    if (own) {
#pragma unroll
        for (int c = 0; c < 2 * DWT_C2; ++c)
            if (c < n) o[c] = oq[c] + scale * acc[c];
    }
}

// ------------------------------------------------------------------ launchers

static dim3 dwt_grid(int sy, int sx, int nz) {
    const int hy = sy / 2, hx = sx / 2;
    const int oty = hy < DWT_OTY ? hy : DWT_OTY, otx = hx < DWT_OTX ? hx : DWT_OTX;
    return dim3((unsigned)(hx / otx), (unsigned)(hy / oty), (unsigned)nz);
}

static bool level_ok(const DwtLevel& A) {
    if (A.n < 1 || A.n > 8 || A.L < 1 || A.sy < 4 || A.sx < 4 || (A.sy & (A.sy - 1)) || (A.sx & (A.sx - 1)))
        return false;
    // the synthesis packs a sub-band row and column in 16 bits each and
    // addresses a band's coefficient block with 32-bit offsets
    if (A.sy > 65536 || A.sx > 65536 || long(A.sy) * A.ld >= (1L << 32)) return false;
    for (int b = 0; b < A.n; ++b) {
        const unsigned k2 = (A.kpack >> (4 * b)) & 15u;
        if (k2 < 1 || k2 > 8) return false;
    }
    return true;
}

template <typename T, bool FINEST>
static void fwd_all_t(const DwtLevel& A, dim3 grid, hipStream_t s) {
    if (FINEST) {
        if (A.mode == 1) hipLaunchKernelGGL((k_dwt_fwd0_all<T, 1>), grid, dim3(DWT_NTH), 0, s, A);
        else if (A.mode == 2) hipLaunchKernelGGL((k_dwt_fwd0_all<T, 2>), grid, dim3(DWT_NTH), 0, s, A);
        else if (A.mode == 3) hipLaunchKernelGGL((k_dwt_fwd0_all<T, 3>), grid, dim3(DWT_NTH), 0, s, A);
        else hipLaunchKernelGGL((k_dwt_fwd0_all<T, 0>), grid, dim3(DWT_NTH), 0, s, A);
    } else {
        if (A.mode == 1) hipLaunchKernelGGL((k_dwt_fwd_all<T, 1>), grid, dim3(DWT_NTH), 0, s, A);
        else if (A.mode == 2) hipLaunchKernelGGL((k_dwt_fwd_all<T, 2>), grid, dim3(DWT_NTH), 0, s, A);
        else if (A.mode == 3) hipLaunchKernelGGL((k_dwt_fwd_all<T, 3>), grid, dim3(DWT_NTH), 0, s, A);
        else hipLaunchKernelGGL((k_dwt_fwd_all<T, 0>), grid, dim3(DWT_NTH), 0, s, A);
    }
}

hipError_t launch_dwt_fwd_all(int dtype, const DwtLevel& A, hipStream_t s, bool finest) {
    if (!level_ok(A) || A.mode < 0 || A.mode > 3 || !A.in0) return hipErrorInvalidValue;
    if ((A.mode != 2 && !A.z0) || (A.mode == 1 && !A.d0) || (A.mode == 3 && !A.s0) || (A.mode != 0 && !A.partials))
        return hipErrorInvalidValue;
    if (A.zo0 && A.mode != 0) return hipErrorInvalidValue;
    // the finest form reads one image per band (no per-basis input stride)
    if (finest && A.in_bstride != 0) return hipErrorInvalidValue;
    const dim3 grid = dwt_grid(A.sy, A.sx, finest ? A.L : A.n * A.L);
    if (finest) {
        if (dtype == 0) fwd_all_t<float, true>(A, grid, s);
        else fwd_all_t<double, true>(A, grid, s);
    } else {
        if (dtype == 0) fwd_all_t<float, false>(A, grid, s);
        else fwd_all_t<double, false>(A, grid, s);
    }
    return hipGetLastError();
}

template <typename T>
static void inv_all_t(const DwtLevel& A, dim3 grid, hipStream_t s) {
    if (A.mode == 1) hipLaunchKernelGGL((k_dwt_inv_all<T, 1>), grid, dim3(DWT_NTH), 0, s, A);
    else if (A.mode == 2) hipLaunchKernelGGL((k_dwt_inv_all<T, 2>), grid, dim3(DWT_NTH), 0, s, A);
    else hipLaunchKernelGGL((k_dwt_inv_all<T, 0>), grid, dim3(DWT_NTH), 0, s, A);
}

hipError_t launch_dwt_inv_all(int dtype, const DwtLevel& A, hipStream_t s) {
    if (!level_ok(A) || !A.out0 || !A.z0 || A.mode < 0 || A.mode > 2) return hipErrorInvalidValue;
    const dim3 grid = dwt_grid(A.sy, A.sx, A.n * A.L);
    if (dtype == 0) inv_all_t<float>(A, grid, s);
    else inv_all_t<double>(A, grid, s);
    return hipGetLastError();
}

template <typename T>
static void inv0_all_t(const DwtLevel& A, dim3 grid, hipStream_t s) {
    if (A.mode == 1) hipLaunchKernelGGL((k_dwt_inv0_all<T, 1>), grid, dim3(DWT_NTH), 0, s, A);
    else if (A.mode == 2) hipLaunchKernelGGL((k_dwt_inv0_all<T, 2>), grid, dim3(DWT_NTH), 0, s, A);
    else hipLaunchKernelGGL((k_dwt_inv0_all<T, 0>), grid, dim3(DWT_NTH), 0, s, A);
}

hipError_t launch_dwt_inv0_all(int dtype, const DwtLevel& A, hipStream_t s) {
    if (!level_ok(A) || !A.out0 || !A.z0 || A.mode < 0 || A.mode > 2) return hipErrorInvalidValue;
    const dim3 grid = dwt_grid(A.sy, A.sx, A.L);
    if (dtype == 0) inv0_all_t<float>(A, grid, s);
    else inv0_all_t<double>(A, grid, s);
    return hipGetLastError();
}

}  // namespace muffin
