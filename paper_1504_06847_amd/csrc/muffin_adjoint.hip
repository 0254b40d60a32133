// Reverse sweep of K unrolled passes of Algorithm 1 (Section 3) on gfx950:
// the adjoint of the reduced pass of muffin_spectral.hip, one launch per
// pass for the band-coupled part (steps II-VI) and the adjoint of the
// right-hand side of step I (eq. matB), either on its own or inside the
// band-coupled launch of the pass before (in sweep order: the next launch),
// which saves a read-modify-write of the four state cotangents.  The step I
// solve itself is symmetric (Q = H^T H + rho I, eq. Qlsimp), so its adjoint
// reuses the column pass in filter mode.
//
// Forward pass k, per pixel, from the state (z_P, z_T, S, Gamma_S):
//   B   = H^T Y + rho_T (2 soft(z_T, tau_T) - z_T) + rho_P |z_P| + Gamma_S + rho_S S
//   X   = Q^{-1} B
//   c   = DCT(S - Gamma_S / rho_V),  V = soft(c, tau_V),  q = IDCT(V)
//   S'  = (rho_V q + rho_S X) / (rho_V + rho_S)
//   G'  = Gamma_S + rho_V (q - S')
//   z_P' = X - max(0, -z_P),  z_T' = X + clip(z_T, tau_T)
// with tau_T = mu_s / rho_T, tau_V = mu_nu / rho_V.  The sweep differentiates
// this map, with cotangents of (z_P, z_T, S, Gamma_S); the stored states
// hold z_V = S - Gamma_S / rho_V in place of S (the DCT input above), and
// S = z_V + Gamma_S / rho_V where S itself enters.  Derivatives at the
// kinks: soft' = 1[|z| > tau], clip' = 1[|z| <= tau], max(0, .)' = 1[. > 0],
// |z|' = sign(z) (0 at 0).
//
// The parameter cotangents are accumulated in FP64 per block into
// partials[block * GRAD_NQ + slot] (GradSlot).
#include "muffin_device.hpp"
#include "muffin_kernels.hpp"

namespace muffin {

constexpr int ADJ_NTH = 256;

template <typename T> __device__ __forceinline__ T sgnt(T z) {
    return z > T(0) ? T(1) : (z < T(0) ? T(-1) : T(0));
}

// Step-I part of the adjoint at one voxel: b = B-bar there (the cotangent of
// the right-hand side, eq. matB), (zp, zt, zv, gs, x) the state before the
// pass and the pass's X.  Adds b's terms to the state cotangents (pb, tb, sb,
// gb) and to the parameter sums, -<b, X> for rho_Q included.  Products that
// are added are explicit fma's: every kernel that inlines it rounds alike.
struct Step1Sums {
    double tT = 0.0, rP = 0.0, rT = 0.0, rS = 0.0, rQ = 0.0;
};

template <typename T> __device__ __forceinline__ void step1_sg(T b, T rhoS, T& sb, T& gb) {
    sb = fma(rhoS, b, sb);
    gb = gb + b;
}

template <typename T>
__device__ __forceinline__ void step1_elem(T b, T zp, T zt, T zv, T gs, T x, const SpecArgs& a, T& pb, T& tb,
                                           T& sb, T& gb, Step1Sums& h) {
    const T rhoP = T(a.rho_P), rhoT = T(a.rho_T), rhoS = T(a.rho_S), tauT = T(a.tau_T);
    const T inv_rhoV = T(1.0 / a.rho_V);
    const bool out = fabs(zt) > tauT;
    tb = fma(out ? rhoT : -rhoT, b, tb);
    pb = fma(rhoP * sgnt(zp), b, pb);
    step1_sg(b, rhoS, sb, gb);
    h.tT += double(out ? (T(-2) * rhoT * sgnt(zt)) * b : T(0));
    h.rT += double(b * fma(T(2), softt(zt, tauT), -zt));
    h.rP += double(b * fabs(zp));
    h.rS += double(b * fma(gs, inv_rhoV, zv));
    h.rQ -= double(b * x);
}

// writes the GRAD_NQ block sums of vals (thread 0 of each block)
__device__ __forceinline__ void store_grad_partials(const double (&vals)[GRAD_NQ], double* partials,
                                                    unsigned blk) {
    __shared__ double sh[ADJ_NTH / 64];
#pragma unroll
    for (int q = 0; q < GRAD_NQ; ++q) {
        const double s = block_sum_s<ADJ_NTH>(vals[q], sh);
        if (threadIdx.x == 0) partials[(long)blk * GRAD_NQ + q] = s;
    }
}

// compiler fence between the stages of the kernel: memory accesses are not
// moved (nor merged) across it, nor is other code scheduled across it
__device__ __forceinline__ void stage_fence() {
    asm volatile("" ::: "memory");
    __builtin_amdgcn_sched_barrier(0);
}

// the value is computed here: without it the compiler sinks the sums of a
// stage (and so every band's operands, live) to where the sums are stored
__device__ __forceinline__ void settle(double& x) { asm volatile("" : "+v"(x)); }

enum AdjMode { ADJ_PLAIN = 0, ADJ_EXT = 1, ADJ_STEP1 = 2 };

// the value as if read from memory: the arithmetic that follows is not
// combined with the arithmetic that made it, so the fused step-I adjoint
// rounds as the separate launch does, whose results pass through memory
template <typename T> __device__ __forceinline__ void opaque(T& x) { asm volatile("" : "+v"(x)); }

// Adjoint of steps II-VI of pass k at one pixel.  In: the state before the
// pass (zP, zT, zV, GS), the pass's X, the cotangents of the state after the
// pass (aP, aT, aS, aG, overwritten in place by those of the state before
// it, this part of them) and, with ADJ_EXT, an outside cotangent of X in Xb.
// Out: Xb = the total cotangent of X.  With ADJ_STEP1 the step-I part of
// pass k + 1 comes first (its B-bar bB, its state zP1.., its X1; parameter
// sums to partials1): the cotangents read are the ones it leaves.
template <typename T, int LT, bool DENSE, int MODE, typename BA>
__device__ __forceinline__ void adj_spectral_body(const BA& zP, const BA& zT, const BA& zV, const BA& GS,
                                                  const BA& X, const BA& aP, const BA& aT, const BA& aS,
                                                  const BA& aG, const BA& Xb, const BA& bB, const BA& zP1,
                                                  const BA& zT1, const BA& zV1, const BA& GS1, const BA& X1,
                                                  unsigned off, const T* __restrict__ D, int Lrt, const SpecArgs& a,
                                                  double* __restrict__ partials, double* __restrict__ partials1) {
    constexpr bool EXT = MODE == ADJ_EXT, S1 = MODE == ADJ_STEP1;
    const int L = DENSE ? Lrt : LT;
    const T rhoV = T(a.rho_V), rhoS = T(a.rho_S), tauT = T(a.tau_T), tauV = T(a.tau_V);
    const T inv_rhoV = T(1.0 / a.rho_V), inv_VS = T(1.0 / (a.rho_V + a.rho_S));
    const T inv_rhoV2 = T(1.0 / (a.rho_V * a.rho_V));
    constexpr int W = (LT + 31) / 32;
    unsigned mc[W], sc[W];
#pragma unroll
    for (int w = 0; w < W; ++w) mc[w] = sc[w] = 0u;

    T v[LT];
    // forward: c = DCT(z_V); keep the kink pattern of soft(c)
#pragma unroll
    for (int l = 0; l < LT; ++l) v[l] = (l < L) ? zV.load(l, off) : T(0);
    dct_any<T, LT, DENSE, false>(v, D, L);
    stage_fence();
#pragma unroll
    for (int k = 0; k < LT; ++k) {
        if (fabs(v[k]) > tauV) mc[k >> 5] |= 1u << (k & 31);
        if (v[k] < T(0)) sc[k >> 5] |= 1u << (k & 31);
        v[k] = softt(v[k], tauV);
    }
    dct_any<T, LT, DENSE, true>(v, D, L);        // q
    stage_fence();

    double g_tT = 0.0, g_tV = 0.0, g_rV = 0.0, g_rS = 0.0;
    Step1Sums h1;
    // steps VI and V backwards, band by band: v becomes the cotangent of q
    // (the cotangent of S' in total is sig = aS - rho_V aG)
#pragma unroll
    for (int l = 0; l < LT; ++l) {
        if (l < L) {
            const T x = X.load(l, off);
            T sb = aS.load(l, off), gb = aG.load(l, off);
            if constexpr (S1) {
                step1_sg(bB.load(l, off), rhoS, sb, gb);
                opaque(sb);
                opaque(gb);
            }
            const T q = v[l];
            const T s2 = (rhoV * q + rhoS * x) * inv_VS;
            const T sig = sb - rhoV * gb;
            v[l] = rhoV * gb + sig * rhoV * inv_VS;
            g_rV += double(gb * (q - s2) + sig * (q - s2) * inv_VS);
            g_rS += double(sig * (x - s2) * inv_VS);
        }
    }
    settle(g_rV);
    settle(g_rS);
    // the cotangents read above are read again after the DCTs: the fences
    // keep every band's reads beside their use, not live across the DCTs
    stage_fence();
    // step IV backwards: V-bar = DCT(q-bar), c-bar = V-bar on the support of soft
    dct_any<T, LT, DENSE, false>(v, D, L);
#pragma unroll
    for (int k = 0; k < LT; ++k) {
        // selects, not branches: a branch here copies all of v at every k
        const bool m = (mc[k >> 5] >> (k & 31)) & 1u;
        const bool neg = (sc[k >> 5] >> (k & 31)) & 1u;
        const T vk = m ? v[k] : T(0);
        g_tV += double(neg ? vk : -vk);
        v[k] = vk;
    }
    settle(g_tV);
    dct_any<T, LT, DENSE, true>(v, D, L);         // u-bar = IDCT(c-bar)
    stage_fence();
    // the state cotangents before the pass, X-bar, and steps III, II backwards
#pragma unroll
    for (int l = 0; l < LT; ++l) {
        if (l < L) {
            T sb = aS.load(l, off), gb = aG.load(l, off), pb = aP.load(l, off), tb = aT.load(l, off);
            if constexpr (S1) {
                step1_elem(bB.load(l, off), zP1.load(l, off), zT1.load(l, off), zV1.load(l, off), GS1.load(l, off),
                           X1.load(l, off), a, pb, tb, sb, gb, h1);
                opaque(pb);
                opaque(tb);
                opaque(sb);
                opaque(gb);
            }
            const T zp = zP.load(l, off), zt = zT.load(l, off), gs = GS.load(l, off);
            const T ext = EXT ? Xb.load(l, off) : T(0);
            const T sig = sb - rhoV * gb;
            const T ub = v[l];
            Xb.store(l, off, ext + pb + tb + sig * rhoS * inv_VS);
            aS.store(l, off, ub);
            aG.store(l, off, gb - ub * inv_rhoV);
            g_rV += double(ub * gs * inv_rhoV2);
            aP.store(l, off, zp < T(0) ? pb : T(0));
            const bool out = fabs(zt) > tauT;
            aT.store(l, off, out ? T(0) : tb);
            const T tbo = out ? tb : T(0);
            g_tT += double(zt > T(0) ? tbo : -tbo);
            if constexpr (S1) {
                // band by band: left to itself the scheduler defers the FP64
                // sums of this loop to its end, every band's operands live
                settle(g_tT);
                settle(g_rV);
                settle(h1.tT);
                settle(h1.rP);
                settle(h1.rT);
                settle(h1.rS);
                settle(h1.rQ);
            }
        }
    }
    settle(g_tT);
    settle(g_rV);
    if constexpr (S1) {
        settle(h1.tT);
        settle(h1.rP);
        settle(h1.rT);
        settle(h1.rS);
        settle(h1.rQ);
    }
    const double vals[GRAD_NQ] = {g_tT, g_tV, 0.0, 0.0, g_rV, g_rS, 0.0, 0.0};
    store_grad_partials(vals, partials, blockIdx.x);
    if constexpr (S1) {
        const double v1[GRAD_NQ] = {h1.tT, 0.0, h1.rP, h1.rT, 0.0, h1.rS, h1.rQ, 0.0};
        store_grad_partials(v1, partials1, blockIdx.x);
    }
}

// MODE (AdjMode) is a template argument, so that no branch splits the band
// loops.  ONE: every array lies within 2^30 bytes of its base, one buffer
// descriptor per array (BandArray1); else one per band group (BandArray),
// whose run-time group shift makes them per array and band (scalar
// registers, spilled in the fused mode, which is built with ONE only).
template <typename T, int LT, bool DENSE, int MODE, bool ONE>
__global__ void __launch_bounds__(ADJ_NTH)
k_adj_spectral(AdjArrays A, const T* __restrict__ D, int Lrt, SpecArgs a, double* __restrict__ partials,
               double* __restrict__ partials1) {
    static_assert(ONE || MODE != ADJ_STEP1, "the fused mode takes single-descriptor arrays");
    const long p = (long)blockIdx.x * blockDim.x + threadIdx.x;
    const unsigned off = (unsigned)p * (unsigned)sizeof(T);
    const unsigned bb = A.band_bytes;
    if constexpr (ONE) {
        const BandArray1<T> zP(A.zP, bb), zT(A.zT, bb), zV(A.zV, bb), GS(A.GS, bb), X(A.X, bb), aP(A.aP, bb),
            aT(A.aT, bb), aS(A.aS, bb), aG(A.aG, bb), Xb(A.Xb, bb);
        if constexpr (MODE == ADJ_STEP1) {
            const BandArray1<T> bB(A.Bb, bb), zP1(A.zP1, bb), zT1(A.zT1, bb), zV1(A.zV1, bb), GS1(A.GS1, bb),
                X1(A.X1, bb);
            adj_spectral_body<T, LT, DENSE, MODE>(zP, zT, zV, GS, X, aP, aT, aS, aG, Xb, bB, zP1, zT1, zV1, GS1,
                                                  X1, off, D, Lrt, a, partials, partials1);
        } else {
            adj_spectral_body<T, LT, DENSE, MODE>(zP, zT, zV, GS, X, aP, aT, aS, aG, Xb, X, X, X, X, X, X, off, D,
                                                  Lrt, a, partials, partials1);
        }
    } else {
        const int gs_ = A.gshift;
        const BandArray<T> zP{A.zP, bb, gs_}, zT{A.zT, bb, gs_}, zV{A.zV, bb, gs_}, GS{A.GS, bb, gs_},
            X{A.X, bb, gs_}, aP{A.aP, bb, gs_}, aT{A.aT, bb, gs_}, aS{A.aS, bb, gs_}, aG{A.aG, bb, gs_},
            Xb{A.Xb, bb, gs_};
        adj_spectral_body<T, LT, DENSE, MODE>(zP, zT, zV, GS, X, aP, aT, aS, aG, Xb, X, X, X, X, X, X, off, D,
                                              Lrt, a, partials, partials1);
    }
}

// Adjoint of the right-hand side of step I (eq. matB) on its own: Bb =
// Q^{-1} X-bar is the cotangent of B.  One thread per pixel over the bands,
// as in k_adj_spectral, so that its parameter sums are those of the fused
// form bit for bit.
template <typename T>
__global__ void __launch_bounds__(ADJ_NTH)
k_adj_step1(const T* __restrict__ Bb, const T* __restrict__ zP, const T* __restrict__ zT,
            const T* __restrict__ zV, const T* __restrict__ GS, const T* __restrict__ X, T* __restrict__ aP,
            T* __restrict__ aT, T* __restrict__ aS, T* __restrict__ aG, long npix, int L, SpecArgs a,
            double* __restrict__ partials) {
    const long p = (long)blockIdx.x * blockDim.x + threadIdx.x;
    Step1Sums h;
    for (int l = 0; l < L; ++l) {
        const long i = (long)l * npix + p;
        T pb = aP[i], tb = aT[i], sb = aS[i], gb = aG[i];
        step1_elem(Bb[i], zP[i], zT[i], zV[i], GS[i], X[i], a, pb, tb, sb, gb, h);
        aP[i] = pb;
        aT[i] = tb;
        aS[i] = sb;
        aG[i] = gb;
    }
    const double vals[GRAD_NQ] = {h.tT, 0.0, h.rP, h.rT, 0.0, h.rS, h.rQ, 0.0};
    store_grad_partials(vals, partials, blockIdx.x);
}

// seed of the MSE loss: Xb = 2 (X - sky), loss partials sum (X - sky)^2
template <typename T>
__global__ void __launch_bounds__(ADJ_NTH)
k_mse_seed(const T* __restrict__ X, const T* __restrict__ sky, T* __restrict__ Xb, long n,
           double* __restrict__ partials) {
    double l2 = 0.0;
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
        const T d = X[i] - sky[i];
        Xb[i] = T(2) * d;
        l2 += double(d) * double(d);
    }
    const double vals[GRAD_NQ] = {0, 0, 0, 0, 0, 0, 0, l2};
    store_grad_partials(vals, partials, blockIdx.x);
}

// acc[q] += sum over blocks of partials[b * GRAD_NQ + q], fixed order
__global__ void __launch_bounds__(256)
k_grad_accum(const double* __restrict__ partials, int nblocks, double* __restrict__ acc) {
    const int q = blockIdx.x;
    double s = 0.0;
    for (int b = threadIdx.x; b < nblocks; b += 256) s += partials[(long)b * GRAD_NQ + q];
    __shared__ double sh[256 / 64];
    const double r = block_sum_s<256>(s, sh);
    if (threadIdx.x == 0) acc[q] += r;
}

static unsigned adj_grid(long n) {
    long b = (n + ADJ_NTH - 1) / ADJ_NTH;
    if (b > 8192) b = 8192;
    if (b < 1) b = 1;
    return (unsigned)b;
}

bool adj_single_descriptor(int L, unsigned band_bytes) {
    return (unsigned long long)L * band_bytes <= (1ull << 30);
}

// one thread per pixel: npix a power of two, at least 64
static bool pixel_grid(long npix, int* nth, unsigned* g) {
    if (npix < 64 || (npix & (npix - 1)) != 0) return false;
    *nth = npix < ADJ_NTH ? (int)npix : ADJ_NTH;
    *g = (unsigned)(npix / *nth);
    return true;
}

template <typename T, int LT, bool DENSE>
static hipError_t adj_t(const AdjArrays& A, const void* D, int L, long npix, const SpecArgs& a,
                        int mode, double* partials, double* partials1, int* nblocks, hipStream_t s) {
    int nth;
    unsigned g;
    if (!pixel_grid(npix, &nth, &g)) return hipErrorInvalidValue;
    *nblocks = (int)g;
    const bool one = adj_single_descriptor(L, A.band_bytes);
    if (mode == ADJ_STEP1 && !one) return hipErrorInvalidValue;
#define MUFFIN_ADJ_LAUNCH(M, O)                                                                                 \
    hipLaunchKernelGGL((k_adj_spectral<T, LT, DENSE, M, O>), dim3(g), dim3(nth), 0, s, A, (const T*)D, L, a,     \
                       partials, partials1)
    if (mode == ADJ_STEP1) MUFFIN_ADJ_LAUNCH(ADJ_STEP1, true);
    else if (mode == ADJ_EXT && one) MUFFIN_ADJ_LAUNCH(ADJ_EXT, true);
    else if (mode == ADJ_EXT) MUFFIN_ADJ_LAUNCH(ADJ_EXT, false);
    else if (one) MUFFIN_ADJ_LAUNCH(ADJ_PLAIN, true);
    else MUFFIN_ADJ_LAUNCH(ADJ_PLAIN, false);
#undef MUFFIN_ADJ_LAUNCH
    return hipGetLastError();
}

template <typename T>
static hipError_t adj_dispatch(const AdjArrays& A, const void* D, int L, long npix, const SpecArgs& a,
                               int mode, double* partials, double* partials1, int* nb, hipStream_t s,
                               bool dense) {
    if (!dense) switch (L) {
        case 1: return adj_t<T, 1, false>(A, D, L, npix, a, mode, partials, partials1, nb, s);
        case 2: return adj_t<T, 2, false>(A, D, L, npix, a, mode, partials, partials1, nb, s);
        case 4: return adj_t<T, 4, false>(A, D, L, npix, a, mode, partials, partials1, nb, s);
        case 8: return adj_t<T, 8, false>(A, D, L, npix, a, mode, partials, partials1, nb, s);
        case 16: return adj_t<T, 16, false>(A, D, L, npix, a, mode, partials, partials1, nb, s);
        case 32: return adj_t<T, 32, false>(A, D, L, npix, a, mode, partials, partials1, nb, s);
        case 64: return adj_t<T, 64, false>(A, D, L, npix, a, mode, partials, partials1, nb, s);
        case 128: return adj_t<T, 128, false>(A, D, L, npix, a, mode, partials, partials1, nb, s);
        default: break;
    }
    // the dense product with D: band counts that are not powers of two, and
    // the spectral bases other than the DCT, up to 32 bands
    if (L < 1 || L > 32) return hipErrorInvalidValue;
    if (L <= 8) return adj_t<T, 8, true>(A, D, L, npix, a, mode, partials, partials1, nb, s);
    if (L <= 16) return adj_t<T, 16, true>(A, D, L, npix, a, mode, partials, partials1, nb, s);
    return adj_t<T, 32, true>(A, D, L, npix, a, mode, partials, partials1, nb, s);
}

hipError_t launch_adj_spectral(int dtype, const AdjArrays& A, const void* D, int L, long npix,
                               const SpecArgs& a, int mode, double* partials, double* partials1, int* nblocks,
                               hipStream_t s, bool dense) {
    if (mode < ADJ_PLAIN || mode > ADJ_STEP1 || (mode == ADJ_STEP1 && !partials1)) return hipErrorInvalidValue;
    return dtype == 0 ? adj_dispatch<float>(A, D, L, npix, a, mode, partials, partials1, nblocks, s, dense)
                      : adj_dispatch<double>(A, D, L, npix, a, mode, partials, partials1, nblocks, s, dense);
}

hipError_t launch_adj_step1(int dtype, const void* Bb, const void* zP, const void* zT, const void* zV,
                            const void* GS, const void* X, void* aP, void* aT, void* aS, void* aG, long npix, int L,
                            const SpecArgs& a, double* partials, int* nblocks, hipStream_t s) {
    int nth;
    unsigned g;
    if (!pixel_grid(npix, &nth, &g) || L < 1) return hipErrorInvalidValue;
    *nblocks = (int)g;
    if (dtype == 0)
        hipLaunchKernelGGL((k_adj_step1<float>), dim3(g), dim3(nth), 0, s, (const float*)Bb, (const float*)zP,
                           (const float*)zT, (const float*)zV, (const float*)GS, (const float*)X, (float*)aP,
                           (float*)aT, (float*)aS, (float*)aG, npix, L, a, partials);
    else
        hipLaunchKernelGGL((k_adj_step1<double>), dim3(g), dim3(nth), 0, s, (const double*)Bb,
                           (const double*)zP, (const double*)zT, (const double*)zV, (const double*)GS,
                           (const double*)X, (double*)aP, (double*)aT, (double*)aS, (double*)aG, npix, L, a,
                           partials);
    return hipGetLastError();
}

hipError_t launch_mse_seed(int dtype, const void* X, const void* sky, void* Xb, size_t n,
                           double* partials, int* nblocks, hipStream_t s) {
    const unsigned g = adj_grid((long)n);
    *nblocks = (int)g;
    if (dtype == 0)
        hipLaunchKernelGGL((k_mse_seed<float>), dim3(g), dim3(ADJ_NTH), 0, s, (const float*)X,
                           (const float*)sky, (float*)Xb, (long)n, partials);
    else
        hipLaunchKernelGGL((k_mse_seed<double>), dim3(g), dim3(ADJ_NTH), 0, s, (const double*)X,
                           (const double*)sky, (double*)Xb, (long)n, partials);
    return hipGetLastError();
}

hipError_t launch_grad_accum(const double* partials, int nblocks, double* acc, hipStream_t s) {
    hipLaunchKernelGGL(k_grad_accum, dim3(GRAD_NQ), dim3(256), 0, s, partials, nblocks, acc);
    return hipGetLastError();
}

}  // namespace muffin
