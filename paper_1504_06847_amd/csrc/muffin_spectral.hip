// Steps II-VI of one ADMM pass on gfx950 (Section 3, Algorithm 1), fused
// into one HBM pass over every pixel, plus the element-wise helpers and the
// deterministic FP64 reductions.
//
// One thread owns one pixel and keeps a single length-L band vector in
// registers; band l of pixel p sits at [l * npix + p], so every load/store
// of a wavefront covers 64 consecutive pixels of one band.
//
// The state is the reduced form of Algorithm 1's nine arrays with W_s = I:
//   z_P (input of the positivity prox, step II), z_T (input of the spatial
//   soft threshold, step III), S, Gamma_S, Gamma_V.
// With these, P = max(0, z_P), Gamma_P = rho_P max(0, -z_P),
// T = soft(z_T, mu_s/rho_T), Gamma_T = -rho_T clip(z_T, mu_s/rho_T), and the
// right-hand side of step I (eq. matB) is H^T Y + B_rest with
// B_rest = rho_T (2 T - z_T) + rho_P |z_P| + Gamma_S + rho_S S.
// Per pixel, given the new X from step I:
//   a = DCT(S_old)                                  (step IV uses the old S)
//   V = soft(a - Gamma_V / rho_V, mu_nu / rho_V);  a = Gamma_V + rho_V V
//   a = IDCT(a);  S = (a - Gamma_S + rho_S X) / (rho_V + rho_S)      (step V)
//   Gamma_S += rho_S (S - X);  a -= rho_V S;  Gamma_V = DCT(a)       (step VI:
//       Gamma_V + rho_V (V - S W_nu) = (Gamma_V + rho_V V) - rho_V S W_nu)
//   z_P <- X - max(0, -z_P);  z_T <- X + clip(z_T, tau_T)     (steps II, III, VI)
#include "muffin_device.hpp"
#include "muffin_kernels.hpp"

namespace muffin {

constexpr int SPEC_NTH = 256;

// deterministic block sum (valid in thread 0): wavefront tree, then the
// per-wave sums in wave order; blockDim.x is a multiple of 64, at most NTH
template <int NTH> __device__ __forceinline__ double block_sum_s(double v, double* sh) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) sh[w] = v;
    __syncthreads();
    double r = 0.0;
    if (threadIdx.x == 0) {
        for (int i = 0; i < (int)(blockDim.x >> 6); ++i) r += sh[i];
    }
    __syncthreads();
    return r;
}

template <typename T> __device__ __forceinline__ T softt(T z, T t) {
    const T m = fabs(z) - t;
    return m > T(0) ? copysign(m, z) : T(0);
}
template <typename T> __device__ __forceinline__ T clipt(T z, T t) {
    return z > t ? t : (z < -t ? -t : z);
}

// dense orthonormal DCT-II (INV = false) or DCT-III (INV = true) for band
// counts that are not powers of two.  D is zero-padded to LT x LT:
// D[k * LT + l] = a_k cos(pi (2l+1) k / 2L) for k, l < L, else 0, so the
// padded entries of v stay zero.
template <typename T, int LT, bool INV>
__device__ __forceinline__ void dct_dense(T (&v)[LT], const T* __restrict__ D) {
    T o[LT];
#pragma unroll
    for (int k = 0; k < LT; ++k) o[k] = T(0);
#pragma unroll
    for (int l = 0; l < LT; ++l) {
#pragma unroll
        for (int k = 0; k < LT; ++k) o[k] += (INV ? D[l * LT + k] : D[k * LT + l]) * v[l];
    }
#pragma unroll
    for (int k = 0; k < LT; ++k) v[k] = o[k];
}

template <typename T, int LT, bool DENSE, bool INV>
__device__ __forceinline__ void dct_any(T (&v)[LT], const T* __restrict__ D, int L) {
    if constexpr (DENSE) dct_dense<T, LT, INV>(v, D);
    else if constexpr (INV) dct3_ortho<T, LT>(v);
    else dct2_ortho<T, LT>(v);
}

// the seven [L][npix] arrays of the spectral pass
struct SpecArrays {
    char *X, *zP, *zT, *S, *GS, *GV, *Brest;
    unsigned band_bytes;
    int gshift;
};

template <typename T, int LT, bool DENSE, bool REDUCE>
__global__ void __launch_bounds__(SPEC_NTH)
k_spectral(SpecArrays A, const T* __restrict__ D, int Lrt, long npix, SpecArgs a,
           double* __restrict__ partials) {
    // the launch covers npix exactly (npix is a power of two >= 64 and the
    // block size min(256, npix) divides it), so every lane owns a pixel
    const long p = (long)blockIdx.x * blockDim.x + threadIdx.x;
    const unsigned off = (unsigned)p * (unsigned)sizeof(T);
    const BandArray<T> X{A.X, A.band_bytes, A.gshift}, zP{A.zP, A.band_bytes, A.gshift},
        zT{A.zT, A.band_bytes, A.gshift}, S{A.S, A.band_bytes, A.gshift},
        GS{A.GS, A.band_bytes, A.gshift}, GV{A.GV, A.band_bytes, A.gshift},
        Brest{A.Brest, A.band_bytes, A.gshift};
    const int L = DENSE ? Lrt : LT;
    const T rhoP = T(a.rho_P), rhoT = T(a.rho_T), rhoV = T(a.rho_V), rhoS = T(a.rho_S);
    const T tauT = T(a.tau_T), tauV = T(a.tau_V);
    const T inv_rhoV = T(1.0 / a.rho_V), inv_VS = T(1.0 / (a.rho_V + a.rho_S));
    double acc[REDUCE ? RED_NQ : 1];
#pragma unroll
    for (int q = 0; q < (REDUCE ? RED_NQ : 1); ++q) acc[q] = 0.0;

    T v[LT];
    // previous Gamma_V, held for the residual / E^k sums of the reduction variant
    T gvold[REDUCE ? LT : 1];
    // step IV input: DCT of the previous S
#pragma unroll
    for (int l = 0; l < LT; ++l) v[l] = (l < L) ? S.load(l, off) : T(0);
    dct_any<T, LT, DENSE, false>(v, D, L);
    // Phase boundaries: keep each phase's loads inside it.  Left free, the
    // scheduler hoists the next phase's band loads above the register DCT
    // and the kernel needs 200+ VGPRs (occupancy 2) or spills.
    __builtin_amdgcn_sched_barrier(0);
    // step IV: V = soft(S W - Gamma_V / rho_V); keep Gamma_V + rho_V V
#pragma unroll
    for (int k = 0; k < LT; ++k) {
        if (k < L) {
            const T gv = GV.load(k, off);
            const T V = softt(v[k] - gv * inv_rhoV, tauV);
            v[k] = gv + rhoV * V;
            if constexpr (REDUCE) {
                acc[RED_V2] += double(V) * V;
                gvold[k] = gv;
            }
        }
    }
    __builtin_amdgcn_sched_barrier(0);
    dct_any<T, LT, DENSE, true>(v, D, L);
    __builtin_amdgcn_sched_barrier(0);
    // steps II, III, V and the Gamma_P, Gamma_T, Gamma_S updates, band by band
#pragma unroll
    for (int l = 0; l < LT; ++l) {
        if (l < L) {
            const T x = X.load(l, off), gs = GS.load(l, off), zp = zP.load(l, off), zt = zT.load(l, off);
            const T s = (v[l] - gs + rhoS * x) * inv_VS;
            const T gs2 = gs + rhoS * (s - x);
            const T zp2 = x - (zp < T(0) ? -zp : T(0));
            const T zt2 = x + clipt(zt, tauT);
            const T tt = softt(zt2, tauT);
            const T b = rhoT * (T(2) * tt - zt2) + rhoP * fabs(zp2) + gs2 + rhoS * s;
            if constexpr (REDUCE) {
                const T sold = S.load(l, off);
                const double P = zp2 > T(0) ? double(zp2) : 0.0;
                const double Pold = zp > T(0) ? double(zp) : 0.0;
                const double Told = double(softt(zt, tauT));
                const double dP = P - Pold, dT = double(tt) - Told, dS = double(s) - double(sold);
                const double gp = double(rhoP) * (zp2 < T(0) ? -double(zp2) : 0.0);
                const double gpo = double(rhoP) * (zp < T(0) ? -double(zp) : 0.0);
                const double gt = -double(rhoT) * double(clipt(zt2, tauT));
                const double gto = -double(rhoT) * double(clipt(zt, tauT));
                const double xd = double(x);
                acc[RED_R2] += (P - xd) * (P - xd) + (double(tt) - xd) * (double(tt) - xd)
                               + (double(s) - xd) * (double(s) - xd);
                const double sx = a.rho_P * dP + a.rho_T * dT + a.rho_S * dS;
                acc[RED_S2] += sx * sx + a.rho_V * a.rho_V * dS * dS;
                acc[RED_X2] += xd * xd;
                acc[RED_BZ2] += P * P + double(tt) * tt + 2.0 * double(s) * s;
                const double gsum = gp + gt + double(gs2);
                acc[RED_ATY2] += gsum * gsum;
                acc[RED_E] += a.rho_P * dP * dP + a.rho_T * dT * dT + (a.rho_S + a.rho_V) * dS * dS
                              + (gp - gpo) * (gp - gpo) / a.rho_P + (gt - gto) * (gt - gto) / a.rho_T
                              + (double(gs2) - gs) * (double(gs2) - gs) / a.rho_S;
                acc[RED_P2] += P * P;
                acc[RED_P1] += P;
            }
            S.store(l, off, s);
            GS.store(l, off, gs2);
            zP.store(l, off, zp2);
            zT.store(l, off, zt2);
            Brest.store(l, off, b);
            v[l] -= rhoV * s;
        }
        // the reduction variant carries 10 FP64 sums and their operands: keep
        // each band's loads inside its own iteration
        if constexpr (REDUCE) __builtin_amdgcn_sched_barrier(0);
    }
    // step VI for Gamma_V
    __builtin_amdgcn_sched_barrier(0);
    dct_any<T, LT, DENSE, false>(v, D, L);
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int k = 0; k < LT; ++k) {
        if (k < L) {
            if constexpr (REDUCE) {
                const double gvo = double(gvold[k]);
                const double dg = double(v[k]) - gvo;
                acc[RED_R2] += dg * dg / (a.rho_V * a.rho_V);
                acc[RED_E] += dg * dg / a.rho_V;
                acc[RED_ATY2] += double(v[k]) * v[k];
            }
            GV.store(k, off, v[k]);
        }
        if constexpr (REDUCE) __builtin_amdgcn_sched_barrier(0);
    }
    if constexpr (REDUCE) {
        // spectral l1 norm of P for the objective
#pragma unroll
        for (int l = 0; l < LT; ++l) {
            const T z = (l < L) ? zP.load(l, off) : T(0);
            v[l] = z > T(0) ? z : T(0);
        }
        dct_any<T, LT, DENSE, false>(v, D, L);
#pragma unroll
        for (int k = 0; k < LT; ++k)
            if (k < L) acc[RED_DCTP1] += fabs(double(v[k]));
        __shared__ double sh[SPEC_NTH / 64];
#pragma unroll
        for (int q = 0; q < RED_NQ; ++q) {
            const double sq = block_sum_s<SPEC_NTH>(acc[q], sh);
            if (threadIdx.x == 0) partials[(long)blockIdx.x * RED_NQ + q] = sq;
        }
    }
}

template <typename T, int LT, bool DENSE>
static hipError_t spectral_t(bool reduce, const void* X, void* zP, void* zT, void* S, void* GS,
                             void* GV, void* Brest, const void* D, int L, long npix,
                             const SpecArgs& a, double* partials, int* nb, hipStream_t s) {
    // npix = nx ny is a power of two >= 64: the block size divides it
    const int nth = npix < SPEC_NTH ? (int)npix : SPEC_NTH;
    if (npix < 64 || (npix & (npix - 1)) != 0) return hipErrorInvalidValue;
    dim3 grid((unsigned)(npix / nth));
    if (nb) *nb = (int)grid.x;
    SpecArrays A{(char*)X, (char*)zP, (char*)zT, (char*)S, (char*)GS, (char*)GV, (char*)Brest,
                 (unsigned)(npix * (long)sizeof(T)), band_group_shift((unsigned long long)npix * sizeof(T))};
    if (reduce)
        hipLaunchKernelGGL((k_spectral<T, LT, DENSE, true>), grid, dim3(nth), 0, s, A,
                           (const T*)D, L, npix, a, partials);
    else
        hipLaunchKernelGGL((k_spectral<T, LT, DENSE, false>), grid, dim3(nth), 0, s, A,
                           (const T*)D, L, npix, a, partials);
    return hipGetLastError();
}

template <typename T>
static hipError_t spectral_dispatch(bool reduce, const void* X, void* zP, void* zT, void* S,
                                    void* GS, void* GV, void* Brest, const void* D, int L,
                                    long npix, const SpecArgs& a, double* partials, int* nb,
                                    hipStream_t s) {
#define ARGS reduce, X, zP, zT, S, GS, GV, Brest, D, L, npix, a, partials, nb, s
    switch (L) {
        case 1: return spectral_t<T, 1, false>(ARGS);
        case 2: return spectral_t<T, 2, false>(ARGS);
        case 4: return spectral_t<T, 4, false>(ARGS);
        case 8: return spectral_t<T, 8, false>(ARGS);
        case 16: return spectral_t<T, 16, false>(ARGS);
        case 32: return spectral_t<T, 32, false>(ARGS);
        case 64: return spectral_t<T, 64, false>(ARGS);
        default: break;
    }
    // band counts that are not powers of two: dense DCT, up to 32 bands
    if (L < 1 || L > 32) return hipErrorInvalidValue;
    if (L <= 8) return spectral_t<T, 8, true>(ARGS);
    if (L <= 16) return spectral_t<T, 16, true>(ARGS);
    return spectral_t<T, 32, true>(ARGS);
#undef ARGS
}

hipError_t launch_spectral(int dtype, bool reduce, const void* X, void* zP, void* zT, void* S,
                           void* GS, void* GV, void* Brest, const void* dctm, int L, int npix,
                           const SpecArgs& a, double* partials, int* nblocks_out, hipStream_t s) {
    if (dtype == 0)
        return spectral_dispatch<float>(reduce, X, zP, zT, S, GS, GV, Brest, dctm, L, npix, a,
                                        partials, nblocks_out, s);
    return spectral_dispatch<double>(reduce, X, zP, zT, S, GS, GV, Brest, dctm, L, npix, a,
                                     partials, nblocks_out, s);
}

// ------------------------------------------------------------------ element-wise
template <typename T>
__global__ void __launch_bounds__(256)
k_brest(const T* __restrict__ zP, const T* __restrict__ zT, const T* __restrict__ S,
        const T* __restrict__ GS, T* __restrict__ Brest, long n, SpecArgs a) {
    const T rhoP = T(a.rho_P), rhoT = T(a.rho_T), rhoS = T(a.rho_S), tauT = T(a.tau_T);
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
        const T zt = zT[i];
        Brest[i] = rhoT * (T(2) * softt(zt, tauT) - zt) + rhoP * fabs(zP[i]) + GS[i] + rhoS * S[i];
    }
}

// Re-encode the prox inputs for new parameters so that P, Gamma_P (always)
// and T, Gamma_T (when mu_s is unchanged) keep their values:
//   z_P' = max(0, z_P) - (rho_P / rho_P') max(0, -z_P)          (= P - Gamma_P / rho_P')
//   z_T' = soft(z_T, tau) + (rho_T / rho_T') clip(z_T, tau)     (= T - Gamma_T / rho_T')
template <typename T>
__global__ void __launch_bounds__(256)
k_reencode(T* __restrict__ zP, T* __restrict__ zT, long n, double rP, double rT, double tau) {
    const T ratioP = T(rP), ratioT = T(rT), t = T(tau);
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
        const T zp = zP[i], zt = zT[i];
        zP[i] = (zp > T(0) ? zp : T(0)) - ratioP * (zp < T(0) ? -zp : T(0));
        zT[i] = softt(zt, t) + ratioT * clipt(zt, t);
    }
}

template <typename T>
__global__ void __launch_bounds__(256) k_positive(const T* __restrict__ z, T* __restrict__ o, long n) {
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
        const T v = z[i];
        o[i] = v > T(0) ? v : T(0);
    }
}

__global__ void __launch_bounds__(256) k_fill_zero(uint32_t* __restrict__ p, long n) {
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
        p[i] = 0u;
}

template <typename Tin>
__global__ void __launch_bounds__(256)
k_scan(const Tin* __restrict__ psf, const Tin* __restrict__ dirty, long n, double* __restrict__ partials) {
    double bad = 0.0, y2 = 0.0;
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
        const double a = double(psf[i]), b = double(dirty[i]);
        if (!isfinite(a)) bad += 1.0;
        if (!isfinite(b)) bad += 1.0;
        else y2 += b * b;
    }
    __shared__ double sh[256 / 64];
    const double sb = block_sum_s<256>(bad, sh);
    const double sy = block_sum_s<256>(y2, sh);
    if (threadIdx.x == 0) { partials[blockIdx.x * 2] = sb; partials[blockIdx.x * 2 + 1] = sy; }
}

__global__ void __launch_bounds__(256)
k_reduce_final(const double* __restrict__ partials, int nblocks, int nq, double* __restrict__ out) {
    const int q = blockIdx.x;
    double s = 0.0;
    for (int b = threadIdx.x; b < nblocks; b += 256) s += partials[(long)b * nq + q];
    __shared__ double sh[256 / 64];
    const double r = block_sum_s<256>(s, sh);
    if (threadIdx.x == 0) out[q] = r;
}

static unsigned grid_for(long n) {
    long b = (n + 255) / 256;
    if (b > 8192) b = 8192;
    if (b < 1) b = 1;
    return (unsigned)b;
}

hipError_t launch_brest(int dtype, const void* zP, const void* zT, const void* S, const void* GS,
                        void* Brest, size_t n, const SpecArgs& a, hipStream_t s) {
    if (dtype == 0)
        hipLaunchKernelGGL((k_brest<float>), dim3(grid_for(n)), dim3(256), 0, s, (const float*)zP,
                           (const float*)zT, (const float*)S, (const float*)GS, (float*)Brest, (long)n, a);
    else
        hipLaunchKernelGGL((k_brest<double>), dim3(grid_for(n)), dim3(256), 0, s, (const double*)zP,
                           (const double*)zT, (const double*)S, (const double*)GS, (double*)Brest, (long)n, a);
    return hipGetLastError();
}

hipError_t launch_reencode(int dtype, void* zP, void* zT, size_t n, double rP, double rT, double tau,
                           hipStream_t s) {
    if (dtype == 0)
        hipLaunchKernelGGL((k_reencode<float>), dim3(grid_for(n)), dim3(256), 0, s, (float*)zP, (float*)zT, (long)n, rP, rT, tau);
    else
        hipLaunchKernelGGL((k_reencode<double>), dim3(grid_for(n)), dim3(256), 0, s, (double*)zP, (double*)zT, (long)n, rP, rT, tau);
    return hipGetLastError();
}

hipError_t launch_positive(int dtype, const void* z, void* out, size_t n, hipStream_t s) {
    if (dtype == 0)
        hipLaunchKernelGGL((k_positive<float>), dim3(grid_for(n)), dim3(256), 0, s, (const float*)z, (float*)out, (long)n);
    else
        hipLaunchKernelGGL((k_positive<double>), dim3(grid_for(n)), dim3(256), 0, s, (const double*)z, (double*)out, (long)n);
    return hipGetLastError();
}

hipError_t launch_fill_zero(void* p, size_t bytes, hipStream_t s) {
    const long n = (long)(bytes / 4);
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_zero, dim3(grid_for(n)), dim3(256), 0, s, (uint32_t*)p, n);
    return hipGetLastError();
}

hipError_t launch_scan(bool in_f64, const void* psf, const void* dirty, size_t n, double* partials,
                       int* nblocks_out, hipStream_t s) {
    const unsigned g = grid_for((long)n);
    if (nblocks_out) *nblocks_out = (int)g;
    if (in_f64)
        hipLaunchKernelGGL((k_scan<double>), dim3(g), dim3(256), 0, s, (const double*)psf, (const double*)dirty, (long)n, partials);
    else
        hipLaunchKernelGGL((k_scan<float>), dim3(g), dim3(256), 0, s, (const float*)psf, (const float*)dirty, (long)n, partials);
    return hipGetLastError();
}

hipError_t launch_reduce_final(const double* partials, int nblocks, int nq, double* out, hipStream_t s) {
    hipLaunchKernelGGL(k_reduce_final, dim3(nq), dim3(256), 0, s, partials, nblocks, nq, out);
    return hipGetLastError();
}

}  // namespace muffin
