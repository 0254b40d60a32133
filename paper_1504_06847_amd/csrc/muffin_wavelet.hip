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
//   k_dwt_inv0: the finest synthesis level of one basis, added into B_rest;
//     one launch per basis, so the sum over the bases has a fixed order.
#include "muffin_device.hpp"
#include "muffin_kernels.hpp"
#include "muffin_layout.hpp"

namespace muffin {

constexpr int DWT_OTY = kDwtTileY;     // coefficient rows per sub-band per tile
constexpr int DWT_OTX = kDwtTileX;     // coefficient columns per sub-band per tile
constexpr int DWT_NTH = 256;

template <typename T> struct WFilt {
    T h[16], g[16];
};
#define MUFFIN_DWT_K_CASES(F) F(2) F(4) F(6) F(8) F(10) F(12) F(14) F(16)

// LDS of one tile, in elements, for the longest filter (K = 16)
constexpr int DWT_FWD_LDS = (2 * DWT_OTY + 14) * (2 * DWT_OTX + 14) + 2 * (2 * DWT_OTY + 14) * DWT_OTX;
constexpr int DWT_INV_LDS = 4 * (DWT_OTY + 7) * (DWT_OTX + 7) + 2 * (2 * DWT_OTY) * (DWT_OTX + 7);

template <typename T> __device__ __forceinline__ T wclip(T z, T t) { return z > t ? t : (z < -t ? -t : z); }
template <typename T> __device__ __forceinline__ T wsoft(T z, T t) {
    return z > t ? z - t : (z < -t ? z + t : T(0));
}
// z_b <- c + clip(z_b, tau)
template <typename T> __device__ __forceinline__ void zupdate(T* p, T c, T tau) { *p = c + wclip(*p, tau); }
// u = 2 soft(z, tau) - z
template <typename T> __device__ __forceinline__ T ucoef(T z, T tau) { return T(2) * wsoft(z, tau) - z; }
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
// MODE 0: update z_b; 1: update, soft(z_b') - soft(z_b) to db and the
// report terms into st; 2: no z_b access, sum |c| (LL at the last level
// included) into st.r2.
template <typename T, int K, int MODE>
__device__ __forceinline__ void dwt_fwd_tile(const T* __restrict__ src, int in_ld, T* __restrict__ zb, int ld,
                                             T* __restrict__ llb, int sy, int sx, const T (&h)[K],
                                             const T (&g)[K], T tau, T* smem, T* __restrict__ db, T rT,
                                             WStats& st) {
    constexpr int HMX = 2 * DWT_OTX + K - 2;
    constexpr int HMY = 2 * DWT_OTY + K - 2;
    T* tin = smem;
    T* rl = smem + HMY * HMX;
    T* rh = rl + HMY * DWT_OTX;
    const int hy = sy >> 1, hx = sx >> 1;
    const int oty = hy < DWT_OTY ? hy : DWT_OTY, otx = hx < DWT_OTX ? hx : DWT_OTX;
    const int i0 = blockIdx.y * oty, m0 = blockIdx.x * otx;
    const int HY = 2 * oty + K - 2, HX = 2 * otx + K - 2;
    // the coefficients this thread updates, loaded first so that their
    // latency overlaps the tile load and the row pass
    constexpr int IPT = (DWT_OTY * DWT_OTX + DWT_NTH - 1) / DWT_NTH;
    T zq[IPT][4];
#pragma unroll
    for (int j = 0; j < IPT; ++j) {
        const int e = threadIdx.x + j * DWT_NTH;
        if (MODE != 2 && e < oty * otx) {
            const int i = e / otx, m = e - i * otx;
            const long gi = i0 + i, gm = m0 + m;
            zq[j][0] = zb[gi * ld + hx + gm];
            zq[j][1] = zb[(hy + gi) * ld + gm];
            zq[j][2] = zb[(hy + gi) * ld + hx + gm];
            zq[j][3] = llb ? T(0) : zb[gi * ld + gm];
        }
    }
    for (int e = threadIdx.x; e < HY * HX; e += DWT_NTH) {
        const int r = e / HX, c = e - r * HX;
        tin[r * HMX + c] = src[(long)((2 * i0 + r) & (sy - 1)) * in_ld + ((2 * m0 + c) & (sx - 1))];
    }
    __syncthreads();
    // along x
    for (int e = threadIdx.x; e < HY * otx; e += DWT_NTH) {
        const int r = e / otx, m = e - r * otx;
        T lo = T(0), hi = T(0);
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const T v = tin[r * HMX + 2 * m + k];
            lo += h[k] * v;
            hi += g[k] * v;
        }
        rl[r * DWT_OTX + m] = lo;
        rh[r * DWT_OTX + m] = hi;
    }
    __syncthreads();
    // along y: the four sub-bands; z <- c + clip(z, tau)
#pragma unroll
    for (int j = 0; j < IPT; ++j) {
        const int e = threadIdx.x + j * DWT_NTH;
        if (e < oty * otx) {
            const int i = e / otx, m = e - i * otx;
            T a = T(0), by = T(0), bx = T(0), d = T(0);
#pragma unroll
            for (int k = 0; k < K; ++k) {
                const T vl = rl[(2 * i + k) * DWT_OTX + m], vh = rh[(2 * i + k) * DWT_OTX + m];
                a += h[k] * vl;
                by += g[k] * vl;
                bx += h[k] * vh;
                d += g[k] * vh;
            }
            const long gi = i0 + i, gm = m0 + m;
            if constexpr (MODE == 0) {
                zb[gi * ld + hx + gm] = bx + wclip(zq[j][0], tau);               // x high, y low
                zb[(hy + gi) * ld + gm] = by + wclip(zq[j][1], tau);             // x low, y high
                zb[(hy + gi) * ld + hx + gm] = d + wclip(zq[j][2], tau);
                if (llb) llb[gi * hx + gm] = a;
                else zb[gi * ld + gm] = a + wclip(zq[j][3], tau);
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
            const T n0 = bx + wclip(zq[j][0], tau);               // x high, y low
            const T n1 = by + wclip(zq[j][1], tau);               // x low, y high
            const T n2 = d + wclip(zq[j][2], tau);
            const T n3 = a + wclip(zq[j][3], tau);
            zb[o0] = n0;
            zb[o1] = n1;
            zb[o2] = n2;
            if (!llb) zb[o3] = n3;
            if constexpr (MODE == 1) {
                db[o0] = wstat(zq[j][0], n0, tau, rT, st);
                db[o1] = wstat(zq[j][1], n1, tau, rT, st);
                db[o2] = wstat(zq[j][2], n2, tau, rT, st);
                if (!llb) db[o3] = wstat(zq[j][3], n3, tau, rT, st);
            }
        }
    }
}

// One synthesis tile producing 2 oty x 2 otx pixels of an sy x sx image (one
// band) from the four sub-bands of u = 2 soft(z, tau) - z (LL from llb, the
// band's dense [sy/2][sx/2] image, or from zb when null); ob with row stride
// out_ld: ob = x, or ob += scale x.
template <typename T, int K, int CF>
__device__ __forceinline__ void dwt_inv_tile(const T* __restrict__ llb, const T* __restrict__ zb, int ld,
                                             T* __restrict__ ob, int out_ld, int sy, int sx, const T (&h)[K],
                                             const T (&g)[K], T tau, T scale, bool accumulate, T* smem) {
    constexpr int H2 = K / 2 - 1;                 // coefficient halo below the tile
    constexpr int CMY = DWT_OTY + H2, CM = DWT_OTX + H2;
    T* ca = smem;
    T* cbx = ca + CMY * CM;
    T* cby = cbx + CMY * CM;
    T* cd = cby + CMY * CM;
    T* xl = cd + CMY * CM;
    T* xh = xl + 2 * DWT_OTY * CM;
    const int hy = sy >> 1, hx = sx >> 1;
    const int oty = hy < DWT_OTY ? hy : DWT_OTY, otx = hx < DWT_OTX ? hx : DWT_OTX;
    const int i0 = blockIdx.y * oty, m0 = blockIdx.x * otx;
    const int CY = oty + H2, CX = otx + H2;
    // the outputs this thread adds to, loaded first (accumulating form)
    constexpr int OPT = (2 * DWT_OTY * DWT_OTX + DWT_NTH - 1) / DWT_NTH;
    T oq[2][OPT];
    if (accumulate) {
#pragma unroll
        for (int p = 0; p < 2; ++p)
#pragma unroll
            for (int j = 0; j < OPT; ++j) {
                const int e = threadIdx.x + j * DWT_NTH;
                if (e < 2 * oty * otx) {
                    const int rr = e / otx, c2 = e - rr * otx;
                    oq[p][j] = ob[long(2 * i0 + rr) * out_ld + 2 * m0 + 2 * c2 + p];
                }
            }
    }
    for (int e = threadIdx.x; e < CY * CX; e += DWT_NTH) {
        const int n = e / CX, q = e - n * CX;
        // periodic coefficient indices i0 - H2 + n, m0 - H2 + q (hy, hx powers of two)
        const long gi = (i0 - H2 + n + 8 * hy) & (hy - 1), gm = (m0 - H2 + q + 8 * hx) & (hx - 1);
        ca[n * CM + q] = llb ? llb[gi * hx + gm] : scoef<T, CF>(zb[gi * ld + gm], tau);
        cbx[n * CM + q] = scoef<T, CF>(zb[gi * ld + hx + gm], tau);
        cby[n * CM + q] = scoef<T, CF>(zb[(hy + gi) * ld + gm], tau);
        cd[n * CM + q] = scoef<T, CF>(zb[(hy + gi) * ld + hx + gm], tau);
    }
    __syncthreads();
    // along y: output rows rr = 2 r2 + p of the tile (the parity p picks the
    // filter taps, so it is the outer, unrolled loop), coefficient columns q
#pragma unroll
    for (int p = 0; p < 2; ++p) {
        for (int e = threadIdx.x; e < oty * CX; e += DWT_NTH) {
            const int r2 = e / CX, q = e - r2 * CX;
            const int base = r2 + H2;
            T lo = T(0), hi = T(0);
#pragma unroll
            for (int kk = 0; kk < K / 2; ++kk) {
                const int n = base - kk;
                lo += h[2 * kk + p] * ca[n * CM + q] + g[2 * kk + p] * cby[n * CM + q];
                hi += h[2 * kk + p] * cbx[n * CM + q] + g[2 * kk + p] * cd[n * CM + q];
            }
            xl[(2 * r2 + p) * CM + q] = lo;
            xh[(2 * r2 + p) * CM + q] = hi;
        }
    }
    __syncthreads();
    // along x: output columns cc = 2 c2 + p
#pragma unroll
    for (int p = 0; p < 2; ++p) {
#pragma unroll
        for (int j = 0; j < OPT; ++j) {
            const int e = threadIdx.x + j * DWT_NTH;
            if (e < 2 * oty * otx) {
                const int rr = e / otx, c2 = e - rr * otx;
                const int base = c2 + H2;
                T v = T(0);
#pragma unroll
                for (int kk = 0; kk < K / 2; ++kk) {
                    const int q = base - kk;
                    v += h[2 * kk + p] * xl[rr * CM + q] + g[2 * kk + p] * xh[rr * CM + q];
                }
                T* o = ob + long(2 * i0 + rr) * out_ld + 2 * m0 + 2 * c2 + p;
                *o = accumulate ? oq[p][j] + scale * v : v;
            }
        }
    }
}

template <typename T, int K>
__device__ __forceinline__ void load_taps(const T* __restrict__ fb, T (&h)[K], T (&g)[K]) {
#pragma unroll
    for (int k = 0; k < K; ++k) {
        h[k] = fb[k];
        g[k] = fb[16 + k];
    }
}

// One analysis level of every basis and band: blockIdx.z = basis * L + band.
// MODE 1 and 2 end with the work-group's FP64 sums in
// A.partials[work-group * nq + q], nq = 3 (MODE 1) or 1 (MODE 2).
template <typename T, int MODE>
__global__ void __launch_bounds__(DWT_NTH) k_dwt_fwd_all(DwtLevel A) {
    __shared__ T smem[DWT_FWD_LDS];
    const int b = blockIdx.z / A.L;
    const long band = blockIdx.z - b * A.L;
    const T* src = (const T*)A.in0 + b * A.in_bstride + band * A.in_bs;
    T* zb = MODE == 2 ? nullptr : (T*)A.z0 + b * A.zstride + band * A.z_bs;
    T* db = MODE == 1 ? (T*)A.d0 + b * A.dstride + band * A.z_bs : nullptr;
    T* llb = A.ll0 ? (T*)A.ll0 + b * A.llstride + band * long(A.sy / 2) * (A.sx / 2) : nullptr;
    const T* fb = (const T*)A.ftab + 32 * b;
    WStats st;
    switch (2 * int((A.kpack >> (4 * b)) & 15u)) {
#define F(KK)                                                                                           \
    case KK: {                                                                                          \
        T h[KK], g[KK];                                                                                 \
        load_taps<T, KK>(fb, h, g);                                                                     \
        dwt_fwd_tile<T, KK, MODE>(src, A.in_ld, zb, A.ld, llb, A.sy, A.sx, h, g, T(A.tau), smem, db,    \
                                  T(A.rho_T), st);                                                      \
        break;                                                                                          \
    }
        MUFFIN_DWT_K_CASES(F)
#undef F
        default: break;
    }
    if constexpr (MODE != 0) {
        __shared__ double sh[DWT_NTH / 64];
        const long wg = ((long)blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x;
        constexpr int nq = MODE == 1 ? 3 : 1;
        const double v[3] = {st.r2, st.e, st.bz};
#pragma unroll
        for (int q = 0; q < nq; ++q) {
            const double sq = block_sum_s<DWT_NTH>(v[q], sh);
            if (threadIdx.x == 0) A.partials[wg * nq + q] = sq;
        }
    }
}

// One synthesis level (not the finest) of every basis and band into the
// bases' dense scratch images: blockIdx.z = basis * L + band.
template <typename T, int CF>
__global__ void __launch_bounds__(DWT_NTH) k_dwt_inv_all(DwtLevel A) {
    __shared__ T smem[DWT_INV_LDS];
    const int b = blockIdx.z / A.L;
    const long band = blockIdx.z - b * A.L;
    const T* zb = (const T*)A.z0 + b * A.zstride + band * A.z_bs;
    const T* llb = A.ll0 ? (const T*)A.ll0 + b * A.llstride + band * long(A.sy / 2) * (A.sx / 2) : nullptr;
    T* ob = (T*)A.out0 + b * A.outstride + band * long(A.sy) * A.sx;
    const T* fb = (const T*)A.ftab + 32 * b;
    switch (2 * int((A.kpack >> (4 * b)) & 15u)) {
#define F(KK)                                                                                          \
    case KK: {                                                                                         \
        T h[KK], g[KK];                                                                                \
        load_taps<T, KK>(fb, h, g);                                                                    \
        dwt_inv_tile<T, KK, CF>(llb, zb, A.ld, ob, A.sx, A.sy, A.sx, h, g, T(A.tau), T(1), false, smem); \
        break;                                                                                         \
    }
        MUFFIN_DWT_K_CASES(F)
#undef F
        default: break;
    }
}

// The finest synthesis level of one basis, added into B_rest (row stride nx,
// band stride ny nx): Brest += scale * x.
template <typename T, int K, int CF>
__global__ void __launch_bounds__(DWT_NTH)
k_dwt_inv0(const T* __restrict__ llin, const T* __restrict__ z, T* __restrict__ Brest, int ny, int nx,
           WFilt<T> f, T tau, T scale) {
    constexpr int CMY = DWT_OTY + K / 2 - 1, CM = DWT_OTX + K / 2 - 1;
    __shared__ T smem[4 * CMY * CM + 2 * (2 * DWT_OTY) * CM];
    const long band = blockIdx.z;
    T h[K], g[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        h[k] = f.h[k];
        g[k] = f.g[k];
    }
    const long vb = long(ny) * nx;
    dwt_inv_tile<T, K, CF>(llin ? llin + band * (vb / 4) : nullptr, z + band * vb, nx, Brest + band * vb, nx, ny,
                           nx, h, g, tau, scale, true, smem);
}

// ------------------------------------------------------------------ launchers
template <typename T> static WFilt<T> make_filt(const double* h, int K) {
    WFilt<T> f{};
    for (int k = 0; k < K; ++k) {
        f.h[k] = T(h[k]);
        f.g[k] = T((k & 1) ? -h[K - 1 - k] : h[K - 1 - k]);
    }
    return f;
}

static dim3 dwt_grid(int sy, int sx, int nz) {
    const int hy = sy / 2, hx = sx / 2;
    const int oty = hy < DWT_OTY ? hy : DWT_OTY, otx = hx < DWT_OTX ? hx : DWT_OTX;
    return dim3((unsigned)(hx / otx), (unsigned)(hy / oty), (unsigned)nz);
}

static bool level_ok(const DwtLevel& A) {
    if (A.n < 1 || A.n > 8 || A.L < 1 || A.sy < 4 || A.sx < 4 || (A.sy & (A.sy - 1)) || (A.sx & (A.sx - 1)))
        return false;
    for (int b = 0; b < A.n; ++b) {
        const unsigned k2 = (A.kpack >> (4 * b)) & 15u;
        if (k2 < 1 || k2 > 8) return false;
    }
    return true;
}

template <typename T>
static void fwd_all_t(const DwtLevel& A, dim3 grid, hipStream_t s) {
    if (A.mode == 1) hipLaunchKernelGGL((k_dwt_fwd_all<T, 1>), grid, dim3(DWT_NTH), 0, s, A);
    else if (A.mode == 2) hipLaunchKernelGGL((k_dwt_fwd_all<T, 2>), grid, dim3(DWT_NTH), 0, s, A);
    else hipLaunchKernelGGL((k_dwt_fwd_all<T, 0>), grid, dim3(DWT_NTH), 0, s, A);
}

hipError_t launch_dwt_fwd_all(int dtype, const DwtLevel& A, hipStream_t s) {
    if (!level_ok(A) || A.mode < 0 || A.mode > 2 || !A.in0) return hipErrorInvalidValue;
    if ((A.mode != 2 && !A.z0) || (A.mode == 1 && !A.d0) || (A.mode != 0 && !A.partials))
        return hipErrorInvalidValue;
    const dim3 grid = dwt_grid(A.sy, A.sx, A.n * A.L);
    if (dtype == 0) fwd_all_t<float>(A, grid, s);
    else fwd_all_t<double>(A, grid, s);
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

template <typename T, int K>
static hipError_t inv0_t(const double* h, const void* llin, const void* z, void* Brest, int ny, int nx, int L,
                         double tau, double scale, hipStream_t s, int cmode) {
    const dim3 grid = dwt_grid(ny, nx, L);
    const WFilt<T> f = make_filt<T>(h, K);
    if (cmode == 1)
        hipLaunchKernelGGL((k_dwt_inv0<T, K, 1>), grid, dim3(DWT_NTH), 0, s, (const T*)llin, (const T*)z, (T*)Brest,
                           ny, nx, f, T(tau), T(scale));
    else if (cmode == 2)
        hipLaunchKernelGGL((k_dwt_inv0<T, K, 2>), grid, dim3(DWT_NTH), 0, s, (const T*)llin, (const T*)z, (T*)Brest,
                           ny, nx, f, T(tau), T(scale));
    else
        hipLaunchKernelGGL((k_dwt_inv0<T, K, 0>), grid, dim3(DWT_NTH), 0, s, (const T*)llin, (const T*)z, (T*)Brest,
                           ny, nx, f, T(tau), T(scale));
    return hipGetLastError();
}

hipError_t launch_dwt_inv0(int dtype, int K, const double* h, const void* llin, const void* z, void* Brest, int ny,
                           int nx, int L, double tau, double scale, hipStream_t s, int cmode) {
    if (K < 2 || K > 16 || (K & 1) || ny < 4 || nx < 4 || L < 1 || (ny & (ny - 1)) || (nx & (nx - 1)) || !z ||
        !Brest || cmode < 0 || cmode > 2)
        return hipErrorInvalidValue;
    switch (K) {
#define F(KK)                                                                                          \
    case KK:                                                                                           \
        return dtype == 0 ? inv0_t<float, KK>(h, llin, z, Brest, ny, nx, L, tau, scale, s, cmode)      \
                          : inv0_t<double, KK>(h, llin, z, Brest, ny, nx, L, tau, scale, s, cmode);
        MUFFIN_DWT_K_CASES(F)
#undef F
    }
    return hipErrorInvalidValue;
}

}  // namespace muffin
