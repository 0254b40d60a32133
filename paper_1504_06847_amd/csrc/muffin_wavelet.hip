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
// recurses on LL.  One launch per level and direction, all bands at once: a
// work-group transforms one tile (16 x 16 coefficients per sub-band) staged
// with its periodic halo in LDS.
//   k_dwt_fwd: one analysis level; the detail coefficients (and at the last
//     level the LL block) go straight into the z_b update; LL otherwise to a
//     dense scratch image for the next level.
//   k_dwt_inv: one synthesis level of u_b = 2 soft(z_b) - z_b (the LL input
//     from the coarser level's scratch image, or from z_b at the last level);
//     the finest level adds scale * W_b^T u_b into B_rest.
#include "muffin_device.hpp"
#include "muffin_kernels.hpp"

namespace muffin {

constexpr int DWT_OT = 16;      // coefficients per sub-band per tile side
constexpr int DWT_NTH = 256;

template <typename T> struct WFilt {
    T h[16], g[16];
};

template <typename T> __device__ __forceinline__ T wclip(T z, T t) { return z > t ? t : (z < -t ? -t : z); }
template <typename T> __device__ __forceinline__ T wsoft(T z, T t) {
    return z > t ? z - t : (z < -t ? z + t : T(0));
}
// z_b <- c + clip(z_b, tau)
template <typename T> __device__ __forceinline__ void zupdate(T* p, T c, T tau) { *p = c + wclip(*p, tau); }
// u = 2 soft(z, tau) - z
template <typename T> __device__ __forceinline__ T ucoef(T z, T tau) { return T(2) * wsoft(z, tau) - z; }

// One analysis level of an sy x sx image per band.  in: [L] images with row
// stride in_ld and band stride in_bs; z: the basis's coefficient cube (row
// stride ld, band stride z_bs); llout: dense [L][sy/2][sx/2] or null (last
// level: LL into z).  Grid: (hx / otx, hy / oty, L).
template <typename T, int K>
__global__ void __launch_bounds__(DWT_NTH)
k_dwt_fwd(const T* __restrict__ in, int in_ld, long in_bs, T* __restrict__ z, int ld, long z_bs,
          T* __restrict__ llout, int sy, int sx, WFilt<T> f, T tau) {
    constexpr int HM = 2 * DWT_OT + K - 2;
    __shared__ T tin[HM * HM];
    __shared__ T rl[HM * DWT_OT], rh[HM * DWT_OT];
    const int hy = sy >> 1, hx = sx >> 1;
    const int oty = hy < DWT_OT ? hy : DWT_OT, otx = hx < DWT_OT ? hx : DWT_OT;
    const int i0 = blockIdx.y * oty, m0 = blockIdx.x * otx;
    const long band = blockIdx.z;
    const int HY = 2 * oty + K - 2, HX = 2 * otx + K - 2;
    const T* src = in + band * in_bs;
    for (int e = threadIdx.x; e < HY * HX; e += DWT_NTH) {
        const int r = e / HX, c = e - r * HX;
        tin[r * HM + c] = src[(long)((2 * i0 + r) & (sy - 1)) * in_ld + ((2 * m0 + c) & (sx - 1))];
    }
    __syncthreads();
    // along x
    for (int e = threadIdx.x; e < HY * otx; e += DWT_NTH) {
        const int r = e / otx, m = e - r * otx;
        T lo = T(0), hi = T(0);
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const T v = tin[r * HM + 2 * m + k];
            lo += f.h[k] * v;
            hi += f.g[k] * v;
        }
        rl[r * DWT_OT + m] = lo;
        rh[r * DWT_OT + m] = hi;
    }
    __syncthreads();
    // along y: the four sub-bands
    T* zb = z + band * z_bs;
    for (int e = threadIdx.x; e < oty * otx; e += DWT_NTH) {
        const int i = e / otx, m = e - i * otx;
        T a = T(0), by = T(0), bx = T(0), d = T(0);
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const T vl = rl[(2 * i + k) * DWT_OT + m], vh = rh[(2 * i + k) * DWT_OT + m];
            a += f.h[k] * vl;
            by += f.g[k] * vl;
            bx += f.h[k] * vh;
            d += f.g[k] * vh;
        }
        const long gi = i0 + i, gm = m0 + m;
        zupdate(zb + gi * ld + hx + gm, bx, tau);               // x high, y low
        zupdate(zb + (hy + gi) * ld + gm, by, tau);             // x low, y high
        zupdate(zb + (hy + gi) * ld + hx + gm, d, tau);
        if (llout) llout[band * long(hy) * hx + gi * hx + gm] = a;
        else zupdate(zb + gi * ld + gm, a, tau);
    }
}

// One synthesis level producing an sy x sx image per band from the four
// sub-bands of u = 2 soft(z, tau) - z (LL from llin, dense [L][sy/2][sx/2],
// or from z when llin is null).  out: row stride out_ld, band stride out_bs;
// accumulate: out += scale * x, else out = x.  Grid: (hx / otx, hy / oty, L).
template <typename T, int K>
__global__ void __launch_bounds__(DWT_NTH)
k_dwt_inv(const T* __restrict__ llin, const T* __restrict__ z, int ld, long z_bs, T* __restrict__ out,
          int out_ld, long out_bs, int sy, int sx, WFilt<T> f, T tau, T scale, int accumulate) {
    constexpr int H2 = K / 2 - 1;                 // coefficient halo below the tile
    constexpr int CM = DWT_OT + H2;
    __shared__ T ca[CM * CM], cbx[CM * CM], cby[CM * CM], cd[CM * CM];
    __shared__ T xl[2 * DWT_OT * CM], xh[2 * DWT_OT * CM];
    const int hy = sy >> 1, hx = sx >> 1;
    const int oty = hy < DWT_OT ? hy : DWT_OT, otx = hx < DWT_OT ? hx : DWT_OT;
    const int i0 = blockIdx.y * oty, m0 = blockIdx.x * otx;
    const long band = blockIdx.z;
    const int CY = oty + H2, CX = otx + H2;
    const T* zb = z + band * z_bs;
    for (int e = threadIdx.x; e < CY * CX; e += DWT_NTH) {
        const int n = e / CX, q = e - n * CX;
        // periodic coefficient indices i0 - H2 + n, m0 - H2 + q (hy, hx powers of two)
        const long gi = (i0 - H2 + n + 8 * hy) & (hy - 1), gm = (m0 - H2 + q + 8 * hx) & (hx - 1);
        ca[n * CM + q] = llin ? llin[band * long(hy) * hx + gi * hx + gm] : ucoef(zb[gi * ld + gm], tau);
        cbx[n * CM + q] = ucoef(zb[gi * ld + hx + gm], tau);
        cby[n * CM + q] = ucoef(zb[(hy + gi) * ld + gm], tau);
        cd[n * CM + q] = ucoef(zb[(hy + gi) * ld + hx + gm], tau);
    }
    __syncthreads();
    // along y: output rows rr of the tile, coefficient columns q
    for (int e = threadIdx.x; e < 2 * oty * CX; e += DWT_NTH) {
        const int rr = e / CX, q = e - rr * CX;
        const int p = rr & 1, base = (rr >> 1) + H2;
        T lo = T(0), hi = T(0);
#pragma unroll
        for (int kk = 0; kk < K / 2; ++kk) {
            const int k = 2 * kk + p, n = base - kk;
            lo += f.h[k] * ca[n * CM + q] + f.g[k] * cby[n * CM + q];
            hi += f.h[k] * cbx[n * CM + q] + f.g[k] * cd[n * CM + q];
        }
        xl[rr * CM + q] = lo;
        xh[rr * CM + q] = hi;
    }
    __syncthreads();
    // along x
    T* ob = out + band * out_bs;
    for (int e = threadIdx.x; e < 4 * oty * otx; e += DWT_NTH) {
        const int rr = e / (2 * otx), cc = e - rr * (2 * otx);
        const int p = cc & 1, base = (cc >> 1) + H2;
        T v = T(0);
#pragma unroll
        for (int kk = 0; kk < K / 2; ++kk) {
            const int k = 2 * kk + p, q = base - kk;
            v += f.h[k] * xl[rr * CM + q] + f.g[k] * xh[rr * CM + q];
        }
        T* o = ob + long(2 * i0 + rr) * out_ld + 2 * m0 + cc;
        if (accumulate) *o += scale * v;
        else *o = v;
    }
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

static dim3 dwt_grid(int sy, int sx, int L) {
    const int hy = sy / 2, hx = sx / 2;
    const int oty = hy < DWT_OT ? hy : DWT_OT, otx = hx < DWT_OT ? hx : DWT_OT;
    return dim3((unsigned)(hx / otx), (unsigned)(hy / oty), (unsigned)L);
}

template <typename T, int K>
static hipError_t dwt_fwd_t(const double* h, const void* in, int in_ld, long in_bs, void* z, int ld, long z_bs,
                            void* llout, int sy, int sx, int L, double tau, hipStream_t s) {
    hipLaunchKernelGGL((k_dwt_fwd<T, K>), dwt_grid(sy, sx, L), dim3(DWT_NTH), 0, s, (const T*)in, in_ld, in_bs,
                       (T*)z, ld, z_bs, (T*)llout, sy, sx, make_filt<T>(h, K), T(tau));
    return hipGetLastError();
}

template <typename T, int K>
static hipError_t dwt_inv_t(const double* h, const void* llin, const void* z, int ld, long z_bs, void* out,
                            int out_ld, long out_bs, int sy, int sx, int L, double tau, double scale,
                            bool accumulate, hipStream_t s) {
    hipLaunchKernelGGL((k_dwt_inv<T, K>), dwt_grid(sy, sx, L), dim3(DWT_NTH), 0, s, (const T*)llin,
                       (const T*)z, ld, z_bs, (T*)out, out_ld, out_bs, sy, sx, make_filt<T>(h, K), T(tau),
                       T(scale), accumulate ? 1 : 0);
    return hipGetLastError();
}

#define MUFFIN_DWT_K_CASES(F) F(2) F(4) F(6) F(8) F(10) F(12) F(14) F(16)

static bool dwt_args_ok(int K, int sy, int sx, int L) {
    return K >= 2 && K <= 16 && (K & 1) == 0 && sy >= 4 && sx >= 4 && (sy & (sy - 1)) == 0 &&
           (sx & (sx - 1)) == 0 && L >= 1;
}

hipError_t launch_dwt_fwd(int dtype, int K, const double* h, const void* in, int in_ld, long in_bs, void* z,
                          int ld, long z_bs, void* llout, int sy, int sx, int L, double tau, hipStream_t s) {
    if (!dwt_args_ok(K, sy, sx, L)) return hipErrorInvalidValue;
    switch (K) {
#define F(KK)                                                                                              \
    case KK:                                                                                               \
        return dtype == 0 ? dwt_fwd_t<float, KK>(h, in, in_ld, in_bs, z, ld, z_bs, llout, sy, sx, L, tau, s) \
                          : dwt_fwd_t<double, KK>(h, in, in_ld, in_bs, z, ld, z_bs, llout, sy, sx, L, tau, s);
        MUFFIN_DWT_K_CASES(F)
#undef F
    }
    return hipErrorInvalidValue;
}

hipError_t launch_dwt_inv(int dtype, int K, const double* h, const void* llin, const void* z, int ld, long z_bs,
                          void* out, int out_ld, long out_bs, int sy, int sx, int L, double tau, double scale,
                          bool accumulate, hipStream_t s) {
    if (!dwt_args_ok(K, sy, sx, L)) return hipErrorInvalidValue;
    switch (K) {
#define F(KK)                                                                                           \
    case KK:                                                                                            \
        return dtype == 0 ? dwt_inv_t<float, KK>(h, llin, z, ld, z_bs, out, out_ld, out_bs, sy, sx, L, tau, \
                                                 scale, accumulate, s)                                   \
                          : dwt_inv_t<double, KK>(h, llin, z, ld, z_bs, out, out_ld, out_bs, sy, sx, L,  \
                                                  tau, scale, accumulate, s);
        MUFFIN_DWT_K_CASES(F)
#undef F
    }
    return hipErrorInvalidValue;
}

}  // namespace muffin
