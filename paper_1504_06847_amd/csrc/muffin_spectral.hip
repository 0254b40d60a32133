// Steps II-VI of one ADMM pass on gfx950 (Section 3, Algorithm 1), fused
// into one HBM pass over every pixel, plus the element-wise helpers and the
// deterministic FP64 reductions.
//
// One thread owns one pixel and keeps a single length-L band vector in
// registers; band l of pixel p sits at [l * npix + p], so every load/store
// of a wavefront covers 64 consecutive pixels of one band.
//
// State: the reduced form of Algorithm 1's nine arrays with W_s = I, four
// arrays z_P, z_T, z_V, Gamma_S.
//  * z_P, z_T are the inputs of the positivity prox (step II) and of the
//    spatial soft threshold (step III): P = max(0, z_P),
//    Gamma_P = rho_P max(0, -z_P), T = soft(z_T, tau_T),
//    Gamma_T = -rho_T clip(z_T, tau_T).
//  * Gamma_V is not stored.  Step V minimises the augmented Lagrangian in S
//    exactly, and its optimality condition is Gamma_S^+ = Gamma_V^+ W_nu^T
//    after every pass (and at the all-zero start), so Gamma_V = Gamma_S W_nu.
//  * z_V = S - Gamma_S / rho_V is the pixel-domain input of the spectral
//    soft threshold (step IV), stored in place of S: step IV reads only z_V
//    and steps V, VI only Gamma_S, one band vector per pixel each, and
//    S = z_V + Gamma_S / rho_V where S itself is needed.
// Per pixel, given the new X from step I:
//   V = soft(DCT(z_V), mu_nu / rho_V)                          (step IV)
//   q = IDCT(V)
//   S^+ = (rho_V q + rho_S X) / (rho_V + rho_S)               (step V)
//   Gamma_S^+ = Gamma_S + rho_V (q - S^+)                      (step VI; also
//       = Gamma_S + rho_S (S^+ - X) by the S-step's closed form)
//   z_V <- S^+ - Gamma_S^+ / rho_V
//   z_P <- X - max(0, -z_P);  z_T <- X + clip(z_T, tau_T)     (steps II, III, VI)
// and the right-hand side of the next step I (eq. matB) is H^T Y + B_rest with
// B_rest = rho_T (2 T - z_T) + rho_P |z_P| + Gamma_S + rho_S S.
#include "muffin_device.hpp"
#include "muffin_kernels.hpp"

namespace muffin {

constexpr int SPEC_NTH = 256;

// One ADMM pass after step I, the state read from zP .. GS and the new one
// written to zPo .. GSo.  REDUCE (a reporting pass): the new state goes to
// the second array set, so k_report can compare old and new, and the
// block sums of ||V||^2 (the only DCT-domain quantity of the convergence
// checks) are written to partials[block].
template <typename T, int LT, bool DENSE, bool REDUCE>
__device__ __forceinline__ void spectral_body(const SpecArrays& A, const T* __restrict__ D, int Lrt,
                                              const SpecArgs& a, double* __restrict__ partials,
                                              unsigned blk) {
    // the launch covers npix exactly (npix is a power of two >= 64 and the
    // block size min(256, npix) divides it), so every lane owns a pixel
    const long p = (long)blk * blockDim.x + threadIdx.x;
    const unsigned off = (unsigned)p * (unsigned)sizeof(T);
    const unsigned bb = A.band_bytes;
    const int gs_ = A.gshift;
    // X (written by the row pass just before) and B_rest (read by the next
    // one) through the caches; the state streams through (non-temporal)
    const BandArray<T> X{A.X, bb, gs_}, Brest{A.Brest, bb, gs_};
    const BandArray<T, kStreamCpol> zP{A.zP, bb, gs_}, zT{A.zT, bb, gs_}, zV{A.zV, bb, gs_},
        GS{A.GS, bb, gs_};
    // the new state: the other set in a reporting pass, the same arrays for
    // a pass in place, or wherever the caller directs it
    const BandArray<T, kStreamCpol> zPo{A.zPo, bb, gs_}, zTo{A.zTo, bb, gs_}, zVo{A.zVo, bb, gs_},
        GSo{A.GSo, bb, gs_};
    const int L = DENSE ? Lrt : LT;
    const T rhoP = T(a.rho_P), rhoT = T(a.rho_T), rhoV = T(a.rho_V), rhoS = T(a.rho_S);
    const T tauT = T(a.tau_T), tauV = T(a.tau_V);
    const T inv_rhoV = T(1.0 / a.rho_V), inv_VS = T(1.0 / (a.rho_V + a.rho_S));
    double v2 = 0.0;

    T v[LT];
    // step IV: V = soft(DCT(z_V)) with the previous z_V = S - Gamma_S / rho_V
#pragma unroll
    for (int l = 0; l < LT; ++l) v[l] = (l < L) ? zV.load(l, off) : T(0);
    dct_any<T, LT, DENSE, false>(v, D, L);
    // Phase boundaries keep each phase's band loads inside it: left free, the
    // scheduler hoists the next phase's loads above the register DCT and the
    // kernel needs 200+ VGPRs or spills.
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int k = 0; k < LT; ++k) {
        const T V = softt(v[k], tauV);
        v[k] = V;
        if constexpr (REDUCE) v2 += double(V) * V;
    }
    dct_any<T, LT, DENSE, true>(v, D, L);        // q = V W_nu^T
    __builtin_amdgcn_sched_barrier(0);
    // steps II, III, V, VI, band by band
#pragma unroll
    for (int l = 0; l < LT; ++l) {
        if (l < L) {
            const T x = X.load(l, off), gs = GS.load(l, off), zp = zP.load(l, off), zt = zT.load(l, off);
            const T q = v[l];
            const T s = (rhoV * q + rhoS * x) * inv_VS;
            const T gs2 = gs + rhoV * (q - s);
            const T zp2 = x - (zp < T(0) ? -zp : T(0));
            const T zt2 = x + clipt(zt, tauT);
            const T tt = softt(zt2, tauT);
            // B_rest from S as the stored state gives it (as k_brest forms
            // it), so a pass from a restored state repeats this one exactly
            const T zv2 = s - gs2 * inv_rhoV;
            const T sv = zv2 + gs2 * inv_rhoV;
            const T b = rhoT * (T(2) * tt - zt2) + rhoP * fabs(zp2) + gs2 + rhoS * sv;
            zVo.store(l, off, zv2);
            GSo.store(l, off, gs2);
            zPo.store(l, off, zp2);
            zTo.store(l, off, zt2);
            Brest.store(l, off, b);
        }
    }
    if constexpr (REDUCE) {
        __shared__ double sh[SPEC_NTH / 64];
        const double sv = block_sum_s<SPEC_NTH>(v2, sh);
        if (threadIdx.x == 0) partials[blk] = sv;
    }
}

template <typename T, int LT, bool DENSE, bool REDUCE>
__global__ void __launch_bounds__(SPEC_NTH)
k_spectral(SpecArrays A, const T* __restrict__ D, int Lrt, long npix, SpecArgs a,
           double* __restrict__ partials) {
    spectral_body<T, LT, DENSE, REDUCE>(A, D, Lrt, a, partials, blockIdx.x);
}

// the spectral pass over the pixels of several cubes with the same band
// count and block size
template <typename T, int LT, bool DENSE>
__global__ void __launch_bounds__(SPEC_NTH)
k_spectral_group(const SpecDesc* __restrict__ d, int n) {
    int j = 0;
    while (j + 1 < n && blockIdx.x >= (unsigned)d[j + 1].first) ++j;
    const unsigned b = blockIdx.x - (unsigned)d[j].first;
    if (blockIdx.x < (unsigned)d[j].first || b >= (unsigned)d[j].nblk) return;
    spectral_body<T, LT, DENSE, false>(d[j].A, (const T*)d[j].D, d[j].Lrt, d[j].a, nullptr, b);
}

// ---------------------------------------------------------------- 256 bands
// A pixel's 256 band values do not fit one thread's registers beside the
// transform.  The orthonormal DCT-II of length 2N (N = 128) splits into a
// butterfly of the two halves, u_n = (x_n + x_{2N-1-n}) / sqrt 2 and
// w_n = (x_n - x_{2N-1-n}) / sqrt 2, followed by c_{2k} = DCT-II_N(u)_k and
// c_{2k+1} = DCT-IV_N(w)_k; the inverse takes the same steps backwards
// (DCT-III_N of the even and DCT-IV_N of the odd coefficients, then the
// butterfly).  A work-group of two waves serves 64 pixels: wave 0 holds
// bands 0..127 of its pixels and then the even coefficients, wave 1 bands
// 128..255 and the odd ones, so each wave runs one transform and every band
// access is uniform over the wave.  The butterflies exchange the halves
// through LDS, 64 registers per round.  Steps IV and V touch the
// coefficients one by one, so which wave holds which does not matter.
constexpr int SPLIT_N = 128;       // bands per wave
constexpr int SPLIT_NTH = 128;     // two waves, 64 pixels

// (the exchange rounds: round_reg, slot_of in muffin_device.hpp)
// the forward butterfly of a 2N-band vector held as two halves of N:
// wave 0 (h = 0) ends with u_n in register n, wave 1 with w_j in register j
// (its register r held band N + r = x_{2N-1 - (N-1 - r)})
template <typename T, int N>
__device__ __forceinline__ void split_fwd(T (&v)[N], int h, T (*xch)[SPLIT_NTH]) {
    const T rs = T(0.70710678118654752440084436210484903928);
    const int t = threadIdx.x, o = t ^ 64;      // the partner: same lane of the other wave
#pragma unroll
    for (int q = 0; q < 2; ++q) {
#pragma unroll
        for (int i = 0; i < N / 2; ++i) xch[i][t] = v[round_reg<N>(q, i)];
        __syncthreads();
        if (h == 0) {
#pragma unroll
            for (int i = 0; i < N / 2; ++i) {
                const int n = round_reg<N>(q, i);
                v[n] = (v[n] + xch[slot_of<N>(N - 1 - n)][o]) * rs;
            }
        } else {
#pragma unroll
            for (int i = 0; i < N / 4; ++i) {
                const int j = q == 0 ? i : N / 4 + i;
                const T a = v[j], b = v[N - 1 - j];
                v[j] = (xch[slot_of<N>(j)][o] - b) * rs;
                v[N - 1 - j] = (xch[slot_of<N>(N - 1 - j)][o] - a) * rs;
            }
        }
        __syncthreads();
    }
}

// the inverse butterfly: from u_n (wave 0) and w_n (wave 1) in register n
// back to bands 0..N-1 (wave 0) and N..2N-1 (wave 1)
template <typename T, int N>
__device__ __forceinline__ void split_inv(T (&v)[N], int h, T (*xch)[SPLIT_NTH]) {
    const T rs = T(0.70710678118654752440084436210484903928);
    const int t = threadIdx.x, o = t ^ 64;
#pragma unroll
    for (int q = 0; q < 2; ++q) {
#pragma unroll
        for (int i = 0; i < N / 2; ++i) xch[i][t] = v[round_reg<N>(q, i)];
        __syncthreads();
        if (h == 0) {
#pragma unroll
            for (int i = 0; i < N / 2; ++i) {
                const int n = round_reg<N>(q, i);
                v[n] = (v[n] + xch[slot_of<N>(n)][o]) * rs;               // x_n = (u_n + w_n) / sqrt 2
            }
        } else {
#pragma unroll
            for (int i = 0; i < N / 4; ++i) {
                const int j = q == 0 ? i : N / 4 + i;
                const T a = v[j], b = v[N - 1 - j];
                v[N - 1 - j] = (xch[slot_of<N>(j)][o] - a) * rs;         // x_{2N-1-j} = (u_j - w_j) / sqrt 2
                v[j] = (xch[slot_of<N>(N - 1 - j)][o] - b) * rs;         // x_{N+j}
            }
        }
        __syncthreads();
    }
}

// 128 bands: the same split at N = 64 in one launch.  With 64 band values
// per thread the transforms fit beside the element-wise steps (as the
// one-thread pass at 64 bands), so q stays in registers: wave h forms
// steps II, III, V, VI for bands 64 h .. 64 h + 63 of its 64 pixels.  The
// one-thread pass at 128 bands holds 128 values (192 registers, 2 waves per
// SIMD); the reporting pass still uses it.
constexpr int PAIR_N = 64;

template <typename T>
__device__ __forceinline__ void spectral_pair_body(const SpecArrays& A, const SpecArgs& a, unsigned blk) {
    constexpr int N = PAIR_N;
    __shared__ T xch[N / 2][SPLIT_NTH];
    const int h = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const long p = (long)blk * 64 + (threadIdx.x & 63);
    const unsigned off = (unsigned)p * (unsigned)sizeof(T);
    const unsigned bb = A.band_bytes;
    // one buffer descriptor per array for the wave's 64 bands (64 band_bytes
    // within 2^31 bytes: checked on the host, spectral_pair_fits)
    const size_t h0 = (size_t)h * N * bb;
    const BandArray1<T> X(A.X + h0, bb), Brest(A.Brest + h0, bb);
    const BandArray1<T, kStreamCpol> zP(A.zP + h0, bb), zT(A.zT + h0, bb), zV(A.zV + h0, bb), GS(A.GS + h0, bb);
    const BandArray1<T, kStreamCpol> zPo(A.zPo + h0, bb), zTo(A.zTo + h0, bb), zVo(A.zVo + h0, bb),
        GSo(A.GSo + h0, bb);
    const T rhoP = T(a.rho_P), rhoT = T(a.rho_T), rhoV = T(a.rho_V), rhoS = T(a.rho_S);
    const T tauT = T(a.tau_T), tauV = T(a.tau_V);
    const T inv_rhoV = T(1.0 / a.rho_V), inv_VS = T(1.0 / (a.rho_V + a.rho_S));
    T v[N];
#pragma unroll
    for (int l = 0; l < N; ++l) v[l] = zV.load(l, off);
    // step IV: DCT-II of 128 = butterfly, DCT-II of 64 (even coefficients,
    // wave 0) and DCT-IV of 64 (odd, wave 1); soft threshold; back
    split_fwd<T, N>(v, h, xch);
    if (h == 0) dct2_ortho<T, N>(v);
    else dct4_ortho<T, N>(v);
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int k = 0; k < N; ++k) v[k] = softt(v[k], tauV);
    if (h == 0) dct3_ortho<T, N>(v);
    else dct4_ortho<T, N>(v);
    split_inv<T, N>(v, h, xch);
    __builtin_amdgcn_sched_barrier(0);
    // steps II, III, V, VI for this wave's bands (the formulas of spectral_body)
#pragma unroll
    for (int i = 0; i < N; ++i) {
        const int l = i;              // band 64 h + i
        const T x = X.load(l, off), gs = GS.load(l, off), zp = zP.load(l, off), zt = zT.load(l, off);
        const T q = v[i];
        const T s = (rhoV * q + rhoS * x) * inv_VS;
        const T gs2 = gs + rhoV * (q - s);
        const T zp2 = x - (zp < T(0) ? -zp : T(0));
        const T zt2 = x + clipt(zt, tauT);
        const T tt = softt(zt2, tauT);
        const T zv2 = s - gs2 * inv_rhoV;
        const T sv = zv2 + gs2 * inv_rhoV;
        const T b = rhoT * (T(2) * tt - zt2) + rhoP * fabs(zp2) + gs2 + rhoS * sv;
        zVo.store(l, off, zv2);
        GSo.store(l, off, gs2);
        zPo.store(l, off, zp2);
        zTo.store(l, off, zt2);
        Brest.store(l, off, b);
        if ((i & 7) == 7) __builtin_amdgcn_sched_barrier(0);
    }
}

template <typename T>
__global__ void __launch_bounds__(SPLIT_NTH)
k_spectral_pair(SpecArrays A, SpecArgs a) {
    spectral_pair_body<T>(A, a, blockIdx.x);
}

// the 128-band pass over the pixels of several cubes (64 pixels per block)
template <typename T>
__global__ void __launch_bounds__(SPLIT_NTH)
k_spectral_pair_group(const SpecDesc* __restrict__ d, int n) {
    int j = 0;
    while (j + 1 < n && blockIdx.x >= (unsigned)d[j + 1].first) ++j;
    const unsigned b = blockIdx.x - (unsigned)d[j].first;
    if (blockIdx.x < (unsigned)d[j].first || b >= (unsigned)d[j].nblk) return;
    spectral_pair_body<T>(d[j].A, d[j].a, b);
}

// The pass runs in two launches, each with the occupancy it can have: the
// transforms (q = IDCT(soft(DCT(z_V))), 128 registers of band values per
// thread) write q into the B_rest array, then an element-wise launch forms
// steps II, III, V, VI and B_rest from it at full occupancy.  That is 8 B
// per voxel more than one launch (q out and back in); measured at
// 2048 x 2048 x 256 FP32 the two launches take 11.9 ms, one launch with
// both halves (344 registers, one wave per SIMD) 16.7 ms.
template <typename T, bool REDUCE>
__global__ void __launch_bounds__(SPLIT_NTH)
k_spectral_split_q(SpecArrays A, SpecArgs a, double* __restrict__ partials) {
    __shared__ T xch[64][SPLIT_NTH];
    const int h = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const long p = (long)blockIdx.x * 64 + (threadIdx.x & 63);
    const unsigned off = (unsigned)p * (unsigned)sizeof(T);
    const unsigned bb = A.band_bytes;
    const int gs_ = A.gshift;
    const BandArray<T, kStreamCpol> zV{A.zV, bb, gs_};
    const BandArray<T> Q{A.Brest, bb, gs_};
    const int l0 = h * SPLIT_N;
    const T tauV = T(a.tau_V);
    double v2 = 0.0;
    T v[SPLIT_N];
#pragma unroll
    for (int l = 0; l < SPLIT_N; ++l) v[l] = zV.load(l0 + l, off);
    split_fwd<T, SPLIT_N>(v, h, xch);
    if (h == 0) dct2_ortho<T, SPLIT_N>(v);
    else dct4_ortho<T, SPLIT_N>(v);
#pragma unroll
    for (int k = 0; k < SPLIT_N; ++k) {
        const T V = softt(v[k], tauV);
        v[k] = V;
        if constexpr (REDUCE) v2 += double(V) * V;
    }
    if (h == 0) dct3_ortho<T, SPLIT_N>(v);
    else dct4_ortho<T, SPLIT_N>(v);
    split_inv<T, SPLIT_N>(v, h, xch);
#pragma unroll
    for (int i = 0; i < SPLIT_N; ++i) Q.store(l0 + i, off, v[i]);
    if constexpr (REDUCE) {
        __shared__ double sh[SPLIT_NTH / 64];
        const double sv = block_sum_s<SPLIT_NTH>(v2, sh);
        if (threadIdx.x == 0) partials[blockIdx.x] = sv;
    }
}

// steps II, III, V, VI element by element from q (in B_rest), 4 voxels per
// thread: the arrays are [L][npix] with npix a multiple of 64, so the L npix
// voxels split into whole 16-B (FP32) or 32-B (FP64) groups
template <typename T>
__global__ void __launch_bounds__(256)
k_spectral_elem(SpecArrays A, SpecArgs a, long n4) {
    typedef T T4 __attribute__((ext_vector_type(4)));
    const T4* X = (const T4*)A.X;
    const T4 *zP = (const T4*)A.zP, *zT = (const T4*)A.zT, *GS = (const T4*)A.GS;
    T4 *zPo = (T4*)A.zPo, *zTo = (T4*)A.zTo, *zVo = (T4*)A.zVo, *GSo = (T4*)A.GSo;
    T4* B = (T4*)A.Brest;
    const T rhoP = T(a.rho_P), rhoT = T(a.rho_T), rhoV = T(a.rho_V), rhoS = T(a.rho_S);
    const T tauT = T(a.tau_T);
    const T inv_rhoV = T(1.0 / a.rho_V), inv_VS = T(1.0 / (a.rho_V + a.rho_S));
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n4; i += (long)gridDim.x * blockDim.x) {
        const T4 x4 = X[i], q4 = B[i];
        const T4 gs4 = __builtin_nontemporal_load(GS + i), zp4 = __builtin_nontemporal_load(zP + i),
                 zt4 = __builtin_nontemporal_load(zT + i);
        T4 zv_o, gs_o, zp_o, zt_o, b_o;
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const T x = x4[c], q = q4[c], gs = gs4[c], zp = zp4[c], zt = zt4[c];
            const T s = (rhoV * q + rhoS * x) * inv_VS;
            const T gs2 = gs + rhoV * (q - s);
            const T zp2 = x - (zp < T(0) ? -zp : T(0));
            const T zt2 = x + clipt(zt, tauT);
            const T tt = softt(zt2, tauT);
            const T zv2 = s - gs2 * inv_rhoV;
            const T sv = zv2 + gs2 * inv_rhoV;
            zv_o[c] = zv2;
            gs_o[c] = gs2;
            zp_o[c] = zp2;
            zt_o[c] = zt2;
            b_o[c] = rhoT * (T(2) * tt - zt2) + rhoP * fabs(zp2) + gs2 + rhoS * sv;
        }
        __builtin_nontemporal_store(zv_o, zVo + i);
        __builtin_nontemporal_store(gs_o, GSo + i);
        __builtin_nontemporal_store(zp_o, zPo + i);
        __builtin_nontemporal_store(zt_o, zTo + i);
        B[i] = b_o;
    }
}

// sum over pixels of |P W_nu|_1 for 256 bands (blocks of 64 pixels)
template <typename T>
__global__ void __launch_bounds__(SPLIT_NTH)
k_dct_l1_split(SpecArrays A, double* __restrict__ partials) {
    __shared__ T xch[64][SPLIT_NTH];
    const int h = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const long p = (long)blockIdx.x * 64 + (threadIdx.x & 63);
    const unsigned off = (unsigned)p * (unsigned)sizeof(T);
    const BandArray<T> zP{A.zP, A.band_bytes, A.gshift};
    T v[SPLIT_N];
#pragma unroll
    for (int l = 0; l < SPLIT_N; ++l) {
        const T z = zP.load(h * SPLIT_N + l, off);
        v[l] = z > T(0) ? z : T(0);
    }
    split_fwd<T, SPLIT_N>(v, h, xch);
    if (h == 0) dct2_ortho<T, SPLIT_N>(v);
    else dct4_ortho<T, SPLIT_N>(v);
    double pd = 0.0;
#pragma unroll
    for (int k = 0; k < SPLIT_N; ++k) pd += fabs(double(v[k]));
    __shared__ double sh[SPLIT_NTH / 64];
    const double sq = block_sum_s<SPLIT_NTH>(pd, sh);
    if (threadIdx.x == 0) partials[(long)blockIdx.x * RED_NQ + RED_DCTP1] = sq;
}

// FP64 sums of a reporting pass from the old state (z_P, z_T, z_V, Gamma_S),
// the new state (primed) and X, per block into partials[block * RED_NQ + q]
// (RED_V2 copied from vpart[block], written by the spectral pass; RED_DCTP1
// written by k_dct_l1):
//   r^2  = ||P - X||^2 + ||T - X||^2 + ||S - X||^2 + ||d Gamma_S||^2 / rho_V^2
//          (the last term is ||V - S W_nu||^2 = ||d Gamma_V||^2 / rho_V^2)
//   s^2  = ||rho_P dP + rho_T dT + rho_S dS||^2 + rho_V^2 ||dS||^2
//   E    = rho_P ||dP||^2 + rho_T ||dT||^2 + (rho_S + rho_V) ||dS||^2
//          + ||dGamma_P||^2 / rho_P + ||dGamma_T||^2 / rho_T
//          + ||dGamma_S||^2 (1 / rho_S + 1 / rho_V)
//   ||X||^2, ||P||^2 + ||T||^2 + 2 ||S||^2, ||Gamma_P + Gamma_T + Gamma_S||^2
//   + ||Gamma_S||^2, ||P||^2, sum P
// using Gamma_V = Gamma_S W_nu and the orthonormality of W_nu.  Each band's
// terms are formed in the iteration's precision T and accumulated in FP64.
// With wavelet bases in W_s (Wd, Wg not null), rho_T W_b^T dT_b and
// W_b^T Gamma_T,b summed over them (Wd, Wg) join the Dirac basis's dT and
// Gamma_T in s^2 and in the dual tolerance's norm; their elementwise terms
// are summed by the analysis itself.
template <typename T>
__global__ void __launch_bounds__(SPEC_NTH)
k_report(SpecArrays A, int L, long npix, SpecArgs a, const double* __restrict__ vpart,
         double* __restrict__ partials, char* Wd, char* Wg) {
    const long p = (long)blockIdx.x * blockDim.x + threadIdx.x;
    const unsigned off = (unsigned)p * (unsigned)sizeof(T);
    const unsigned bb = A.band_bytes;
    const int gs_ = A.gshift;
    const BandArray<T> X{A.X, bb, gs_}, zP{A.zP, bb, gs_}, zT{A.zT, bb, gs_}, zV{A.zV, bb, gs_},
        GS{A.GS, bb, gs_}, zPo{A.zPo, bb, gs_}, zTo{A.zTo, bb, gs_}, zVo{A.zVo, bb, gs_},
        GSo{A.GSo, bb, gs_};
    const BandArray<T> Wdt{Wd, bb, gs_}, Wgt{Wg, bb, gs_};
    const bool wav = Wd != nullptr;
    const T rP = T(a.rho_P), rT = T(a.rho_T), rV = T(a.rho_V), rS = T(a.rho_S), tT = T(a.tau_T);
    const T irP = T(1.0 / a.rho_P), irT = T(1.0 / a.rho_T), irV2 = T(1.0 / (a.rho_V * a.rho_V));
    const T irV = T(1.0 / a.rho_V);
    const T ieS = T(1.0 / a.rho_S + 1.0 / a.rho_V), rSV = T(a.rho_S + a.rho_V);
    double r2 = 0, s2 = 0, x2 = 0, bz2 = 0, aty2 = 0, e = 0, p2 = 0, p1 = 0;
#pragma unroll 2
    for (int l = 0; l < L; ++l) {
        const T x = X.load(l, off);
        const T zp = zP.load(l, off), zt = zT.load(l, off), go = GS.load(l, off);
        const T zp2 = zPo.load(l, off), zt2 = zTo.load(l, off), gn = GSo.load(l, off);
        const T so = zV.load(l, off) + go * irV, sn = zVo.load(l, off) + gn * irV;
        const T P = zp2 > T(0) ? zp2 : T(0), Po = zp > T(0) ? zp : T(0);
        const T Tn = softt(zt2, tT), To = softt(zt, tT);
        const T gp = rP * (zp2 < T(0) ? -zp2 : T(0)), gpo = rP * (zp < T(0) ? -zp : T(0));
        const T gt = -rT * clipt(zt2, tT), gto = -rT * clipt(zt, tT);
        const T dP = P - Po, dT = Tn - To, dS = sn - so, dg = gn - go;
        const T a1 = P - x, a2 = Tn - x, a3 = sn - x;
        r2 += double(a1 * a1 + a2 * a2 + a3 * a3 + dg * dg * irV2);
        T sx = rP * dP + rT * dT + rS * dS;
        if (wav) sx += Wdt.load(l, off);
        s2 += double(sx * sx + rV * rV * dS * dS);
        x2 += double(x * x);
        bz2 += double(P * P + Tn * Tn + T(2) * sn * sn);
        T g = gp + gt + gn;
        if (wav) g += Wgt.load(l, off);
        aty2 += double(g * g + gn * gn);
        const T dgp = gp - gpo, dgt = gt - gto;
        e += double(rP * dP * dP + rT * dT * dT + rSV * dS * dS + dgp * dgp * irP + dgt * dgt * irT
                    + dg * dg * ieS);
        p2 += double(P * P);
        p1 += double(P);
    }
    __shared__ double sh[SPEC_NTH / 64];
    const double vals[RED_NQ] = {r2, s2, x2, 0.0, bz2, aty2, e, p2, p1, 0.0};
#pragma unroll
    for (int q = 0; q < RED_NQ; ++q) {
        if (q == RED_V2 || q == RED_DCTP1) continue;
        const double sq = block_sum_s<SPEC_NTH>(vals[q], sh);
        if (threadIdx.x == 0) partials[(long)blockIdx.x * RED_NQ + q] = sq;
    }
    if (threadIdx.x == 0) partials[(long)blockIdx.x * RED_NQ + RED_V2] = vpart[blockIdx.x];
}

// sum over pixels of |P W_nu|_1 with P = max(0, z_P): block sums into
// partials[block * RED_NQ + RED_DCTP1]
template <typename T, int LT, bool DENSE>
__global__ void __launch_bounds__(SPEC_NTH)
k_dct_l1(SpecArrays A, const T* __restrict__ D, int Lrt, long npix, double* __restrict__ partials) {
    const long p = (long)blockIdx.x * blockDim.x + threadIdx.x;
    const unsigned off = (unsigned)p * (unsigned)sizeof(T);
    const BandArray<T> zP{A.zP, A.band_bytes, A.gshift};
    const int L = DENSE ? Lrt : LT;
    T v[LT];
#pragma unroll
    for (int l = 0; l < LT; ++l) {
        const T z = (l < L) ? zP.load(l, off) : T(0);
        v[l] = z > T(0) ? z : T(0);
    }
    dct_any<T, LT, DENSE, false>(v, D, L);
    double pd = 0.0;
#pragma unroll
    for (int k = 0; k < LT; ++k) pd += fabs(double(v[k]));
    __shared__ double sh[SPEC_NTH / 64];
    const double sq = block_sum_s<SPEC_NTH>(pd, sh);
    if (threadIdx.x == 0) partials[(long)blockIdx.x * RED_NQ + RED_DCTP1] = sq;
}

template <typename T, int LT, bool DENSE>
static hipError_t spectral_t(const SpecLaunch& g, const SpecArgs& a, hipStream_t s) {
    // npix = nx ny is a power of two >= 64: the block size divides it
    const long npix = g.npix;
    const int nth = npix < SPEC_NTH ? (int)npix : SPEC_NTH;
    if (npix < 64 || (npix & (npix - 1)) != 0) return hipErrorInvalidValue;
    dim3 grid((unsigned)(npix / nth));
    const unsigned bb = (unsigned)(npix * (long)sizeof(T));
    SpecArrays A{(char*)g.X, (char*)g.st[0], (char*)g.st[1], (char*)g.st[2], (char*)g.st[3],
                 (char*)g.out[0], (char*)g.out[1], (char*)g.out[2], (char*)g.out[3], (char*)g.brest,
                 bb, band_group_shift(bb)};
    if (g.report) {
        hipLaunchKernelGGL((k_spectral<T, LT, DENSE, true>), grid, dim3(nth), 0, s, A,
                           (const T*)g.dctm, g.L, npix, a, g.vpart);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL((k_report<T>), grid, dim3(nth), 0, s, A, g.L, npix, a,
                           (const double*)g.vpart, g.partials,
                           (char*)g.wdt, (char*)g.wg);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
        // the spectral l1 term reads the new z_P
        SpecArrays B = A;
        B.zP = A.zPo;
        hipLaunchKernelGGL((k_dct_l1<T, LT, DENSE>), grid, dim3(nth), 0, s, B, (const T*)g.dctm, g.L,
                           npix, g.partials);
    } else if (LT == 2 * PAIR_N && !DENSE && spectral_pair_fits(npix, (int)sizeof(T))) {
        hipLaunchKernelGGL((k_spectral_pair<T>), dim3((unsigned)(npix / 64)), dim3(SPLIT_NTH), 0, s, A, a);
    } else {
        hipLaunchKernelGGL((k_spectral<T, LT, DENSE, false>), grid, dim3(nth), 0, s, A,
                           (const T*)g.dctm, g.L, npix, a, g.vpart);
    }
    return hipGetLastError();
}

// 256 bands: blocks of 64 pixels (two waves); a reporting pass runs k_report
// with 64-thread blocks, so that its blocks are the spectral pass's
template <typename T>
static hipError_t spectral_split_t(const SpecLaunch& g, const SpecArgs& a, hipStream_t s) {
    const long npix = g.npix;
    if (npix < 64 || (npix & (npix - 1)) != 0) return hipErrorInvalidValue;
    dim3 grid((unsigned)(npix / 64));
    const unsigned bb = (unsigned)(npix * (long)sizeof(T));
    SpecArrays A{(char*)g.X, (char*)g.st[0], (char*)g.st[1], (char*)g.st[2], (char*)g.st[3],
                 (char*)g.out[0], (char*)g.out[1], (char*)g.out[2], (char*)g.out[3], (char*)g.brest,
                 bb, band_group_shift(bb)};
    const long n4 = (long)g.L * npix / 4;
    long eb = (n4 + 255) / 256;
    if (eb > 65536) eb = 65536;
    if (g.report) {
        hipLaunchKernelGGL((k_spectral_split_q<T, true>), grid, dim3(SPLIT_NTH), 0, s, A, a, g.vpart);
        hipLaunchKernelGGL((k_spectral_elem<T>), dim3((unsigned)eb), dim3(256), 0, s, A, a, n4);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL((k_report<T>), grid, dim3(64), 0, s, A, g.L, npix, a, (const double*)g.vpart,
                           g.partials, (char*)g.wdt, (char*)g.wg);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
        SpecArrays B = A;
        B.zP = A.zPo;
        hipLaunchKernelGGL((k_dct_l1_split<T>), grid, dim3(SPLIT_NTH), 0, s, B, g.partials);
    } else {
        hipLaunchKernelGGL((k_spectral_split_q<T, false>), grid, dim3(SPLIT_NTH), 0, s, A, a, g.vpart);
        hipLaunchKernelGGL((k_spectral_elem<T>), dim3((unsigned)eb), dim3(256), 0, s, A, a, n4);
    }
    return hipGetLastError();
}

template <typename T>
static hipError_t spectral_dispatch(const SpecLaunch& g, const SpecArgs& a, hipStream_t s) {
    if (!g.dense) {
        switch (g.L) {
            case 1: return spectral_t<T, 1, false>(g, a, s);
            case 2: return spectral_t<T, 2, false>(g, a, s);
            case 4: return spectral_t<T, 4, false>(g, a, s);
            case 8: return spectral_t<T, 8, false>(g, a, s);
            case 16: return spectral_t<T, 16, false>(g, a, s);
            case 32: return spectral_t<T, 32, false>(g, a, s);
            case 64: return spectral_t<T, 64, false>(g, a, s);
            case 128: return spectral_t<T, 128, false>(g, a, s);
            case 256: return spectral_split_t<T>(g, a, s);
            default: break;
        }
    }
    // the dense product with dctm: band counts that are not powers of two
    // (the DCT), and the other spectral bases, up to 32 bands or 64
    if (g.L < 1 || (g.L > 32 && g.L != 64)) return hipErrorInvalidValue;
    if (g.L <= 8) return spectral_t<T, 8, true>(g, a, s);
    if (g.L <= 16) return spectral_t<T, 16, true>(g, a, s);
    if (g.L <= 32) return spectral_t<T, 32, true>(g, a, s);
    return spectral_t<T, 64, true>(g, a, s);
}

int spectral_block_threads(long npix) { return npix < SPEC_NTH ? (int)npix : SPEC_NTH; }
bool spectral_pair_fits(long npix, int elem) { return (long long)PAIR_N * npix * elem <= (1ll << 31); }
int spectral_block_pixels(int L, long npix, int elem) {
    return L == 2 * PAIR_N && spectral_pair_fits(npix, elem) ? 64 : spectral_block_threads(npix);
}
int spectral_gshift(unsigned band_bytes) { return band_group_shift(band_bytes); }

template <typename T>
static hipError_t spectral_group_t(int L, const SpecDesc* d, int n, int nblocks, int nth, hipStream_t s) {
    const dim3 g((unsigned)nblocks), b((unsigned)nth);
    switch (L) {
        case 1: hipLaunchKernelGGL((k_spectral_group<T, 1, false>), g, b, 0, s, d, n); return hipGetLastError();
        case 2: hipLaunchKernelGGL((k_spectral_group<T, 2, false>), g, b, 0, s, d, n); return hipGetLastError();
        case 4: hipLaunchKernelGGL((k_spectral_group<T, 4, false>), g, b, 0, s, d, n); return hipGetLastError();
        case 8: hipLaunchKernelGGL((k_spectral_group<T, 8, false>), g, b, 0, s, d, n); return hipGetLastError();
        case 16: hipLaunchKernelGGL((k_spectral_group<T, 16, false>), g, b, 0, s, d, n); return hipGetLastError();
        case 32: hipLaunchKernelGGL((k_spectral_group<T, 32, false>), g, b, 0, s, d, n); return hipGetLastError();
        case 64: hipLaunchKernelGGL((k_spectral_group<T, 64, false>), g, b, 0, s, d, n); return hipGetLastError();
        case 128:
            // 64 pixels per block: the two-wave pass (every cube within
            // spectral_pair_fits), else one pixel per thread
            if (nth == 64) hipLaunchKernelGGL((k_spectral_pair_group<T>), g, dim3(SPLIT_NTH), 0, s, d, n);
            else hipLaunchKernelGGL((k_spectral_group<T, 128, false>), g, b, 0, s, d, n);
            return hipGetLastError();
        default: break;
    }
    if (L < 1 || L > 32) return hipErrorInvalidValue;
    if (L <= 8) hipLaunchKernelGGL((k_spectral_group<T, 8, true>), g, b, 0, s, d, n);
    else if (L <= 16) hipLaunchKernelGGL((k_spectral_group<T, 16, true>), g, b, 0, s, d, n);
    else hipLaunchKernelGGL((k_spectral_group<T, 32, true>), g, b, 0, s, d, n);
    return hipGetLastError();
}

hipError_t launch_spectral_group(int dtype, int L, int nth, const SpecDesc* d, int n, int nblocks,
                                 hipStream_t s) {
    if (n <= 0 || nblocks <= 0) return hipSuccess;
    if (nth < 64 || nth > SPEC_NTH || (nth & 63)) return hipErrorInvalidValue;
    return dtype == 0 ? spectral_group_t<float>(L, d, n, nblocks, nth, s)
                      : spectral_group_t<double>(L, d, n, nblocks, nth, s);
}

// a union of spectral bases (defined with its kernels below)
template <typename T>
static hipError_t union_dispatch(const SpecLaunch& g, const SpecArgs& a, hipStream_t s);

hipError_t launch_spectral(int dtype, const SpecLaunch& g, const SpecArgs& a, int* nblocks_out,
                           hipStream_t s) {
    // every array the kernels read or write must be set (out = st in place)
    if (!g.X || !g.brest || g.n_nu < 1 || g.n_nu > 4) return hipErrorInvalidValue;
    for (int i = 0; i < 4; ++i)
        if (!g.st[i] || !g.out[i]) return hipErrorInvalidValue;
    for (int j = 0; g.n_nu > 1 && j < g.n_nu; ++j)
        if (!g.uz[j] || !g.uzo[j]) return hipErrorInvalidValue;
    const bool split = g.L == 2 * SPLIT_N && !g.dense && g.n_nu == 1;
    if (nblocks_out) *nblocks_out = (int)(split ? g.npix / 64 : g.npix / (g.npix < SPEC_NTH ? g.npix : SPEC_NTH));
    if (g.n_nu > 1) return dtype == 0 ? union_dispatch<float>(g, a, s) : union_dispatch<double>(g, a, s);
    return dtype == 0 ? spectral_dispatch<float>(g, a, s) : spectral_dispatch<double>(g, a, s);
}

// ------------------------------------------------------------------ a union of spectral bases
// W_nu = [W_1 .. W_m], m orthonormal bases, each applied as a dense product
// (D + j LT^2 holds W_j as D_j[k * LT + l] = W_j[l][k]).  With m > 1 the
// multiplier Gamma_V has m coefficient blocks that Gamma_S = Gamma_V W_nu^T
// does not determine, so the state is z_P, z_T, S, Gamma_S and, per basis,
// z_V,j = S W_j - Gamma_V,j / rho_V (the input of step IV's soft threshold,
// in basis j's coefficients).  Per pixel (Section 3, steps IV-VI):
//   V_j = soft(z_V,j, mu_nu / rho_V)                           (step IV)
//   q = sum_j V_j W_j^T,  S' = (rho_V q + rho_S X) / (m rho_V + rho_S)
//       (step V: sum_j Gamma_V,j W_j^T = Gamma_S + ... cancels exactly;
//        the oracle's closed form with the m_nu rho_V denominator)
//   Gamma_S' = Gamma_S + rho_S (S' - X)                         (step VI)
//   z_V,j' = S' W_j - Gamma_V,j' / rho_V = (2 S' - S) W_j + z_V,j - V_j
//          = (2 S' - S) W_j + clip(z_V,j, mu_nu / rho_V)
// and B_rest = rho_T (2 T - z_T) + rho_P |z_P| + Gamma_S' + rho_S S'.
struct UnionZ {
    char* in[4];
    char* out[4];
};

template <typename T, int LT>
__device__ __forceinline__ void dense_fwd(T (&c)[LT], const T (&u)[LT], const T* __restrict__ Dj) {
#pragma unroll
    for (int k = 0; k < LT; ++k) {
        T acc = T(0);
#pragma unroll
        for (int l = 0; l < LT; ++l) acc += Dj[k * LT + l] * u[l];
        c[k] = acc;
    }
}

template <typename T, int LT>
__global__ void __launch_bounds__(SPEC_NTH)
k_spectral_union(SpecArrays A, UnionZ Z, const T* __restrict__ D, int Lrt, int m, SpecArgs a) {
    const long p = (long)blockIdx.x * blockDim.x + threadIdx.x;
    const unsigned off = (unsigned)p * (unsigned)sizeof(T);
    const unsigned bb = A.band_bytes;
    const int gs_ = A.gshift;
    const int L = Lrt;
    const BandArray<T> X{A.X, bb, gs_}, Brest{A.Brest, bb, gs_};
    const BandArray<T, kStreamCpol> zP{A.zP, bb, gs_}, zT{A.zT, bb, gs_}, S{A.zV, bb, gs_}, GS{A.GS, bb, gs_};
    const BandArray<T, kStreamCpol> zPo{A.zPo, bb, gs_}, zTo{A.zTo, bb, gs_}, So{A.zVo, bb, gs_},
        GSo{A.GSo, bb, gs_};
    const T rhoP = T(a.rho_P), rhoT = T(a.rho_T), rhoV = T(a.rho_V), rhoS = T(a.rho_S);
    const T tauT = T(a.tau_T), tauV = T(a.tau_V);
    const T inv_mVS = T(1.0 / (double(m) * a.rho_V + a.rho_S));
    T q[LT];
#pragma unroll
    for (int l = 0; l < LT; ++l) q[l] = T(0);
    // steps IV and V: q = sum_j soft(z_V,j) W_j^T
    for (int j = 0; j < m; ++j) {
        const BandArray<T, kStreamCpol> zv{Z.in[j], bb, gs_};
        const T* Dj = D + (long)j * LT * LT;
        T c[LT];
#pragma unroll
        for (int k = 0; k < LT; ++k) c[k] = k < L ? softt(zv.load(k, off), tauV) : T(0);
#pragma unroll
        for (int k = 0; k < LT; ++k)
#pragma unroll
            for (int l = 0; l < LT; ++l) q[l] += Dj[k * LT + l] * c[k];
    }
    __builtin_amdgcn_sched_barrier(0);
    // steps II, III, V, VI band by band; q[l] becomes 2 S' - S
#pragma unroll
    for (int l = 0; l < LT; ++l) {
        if (l < L) {
            const T x = X.load(l, off), so = S.load(l, off), gs = GS.load(l, off), zp = zP.load(l, off),
                    zt = zT.load(l, off);
            const T sn = (rhoV * q[l] + rhoS * x) * inv_mVS;
            const T gs2 = gs + rhoS * (sn - x);
            const T zp2 = x - (zp < T(0) ? -zp : T(0));
            const T zt2 = x + clipt(zt, tauT);
            const T tt = softt(zt2, tauT);
            So.store(l, off, sn);
            GSo.store(l, off, gs2);
            zPo.store(l, off, zp2);
            zTo.store(l, off, zt2);
            Brest.store(l, off, rhoT * (T(2) * tt - zt2) + rhoP * fabs(zp2) + gs2 + rhoS * sn);
            q[l] = T(2) * sn - so;
        } else {
            q[l] = T(0);
        }
    }
    __builtin_amdgcn_sched_barrier(0);
    // z_V,j' = (2 S' - S) W_j + clip(z_V,j)
    for (int j = 0; j < m; ++j) {
        const BandArray<T, kStreamCpol> zv{Z.in[j], bb, gs_}, zvo{Z.out[j], bb, gs_};
        T c[LT];
        dense_fwd<T, LT>(c, q, D + (long)j * LT * LT);
#pragma unroll
        for (int k = 0; k < LT; ++k)
            if (k < L) zvo.store(k, off, c[k] + clipt(zv.load(k, off), tauV));
    }
}

// The FP64 sums of a reporting pass for a union (every RED slot), from the
// old state (z_P, z_T, S, Gamma_S, z_V,j), the new one (primed) and X:
//   r^2  = ||P - X||^2 + ||T - X||^2 + ||S' - X||^2 + sum_j ||V_j - S' W_j||^2
//   s^2  = ||rho_P dP + rho_T dT + rho_S dS||^2 + m rho_V^2 ||dS||^2
//   E    = rho_P ||dP||^2 + rho_T ||dT||^2 + (rho_S + m rho_V) ||dS||^2
//          + ||dGamma_P||^2 / rho_P + ||dGamma_T||^2 / rho_T + ||dGamma_S||^2 / rho_S
//          + rho_V sum_j ||V_j - S' W_j||^2         (dGamma_V,j = rho_V (V_j - S' W_j))
//   ||X||^2, sum_j ||V_j||^2, ||P||^2 + ||T||^2 + (m + 1) ||S'||^2,
//   ||Gamma_P + Gamma_T + Gamma_S'||^2 + sum_j ||Gamma_V,j'||^2 with
//   Gamma_V,j' = rho_V (S' W_j - z_V,j'), ||P||^2, sum P, sum_j |P W_j|_1
// (V_j = soft(z_V,j) of the old state; W_nu orthonormal per basis).
// With wavelet bases in W_s, Wd and Wg as in k_report.
template <typename T, int LT>
__global__ void __launch_bounds__(SPEC_NTH)
k_report_union(SpecArrays A, UnionZ Z, const T* __restrict__ D, int Lrt, int m, SpecArgs a,
               double* __restrict__ partials, char* Wd, char* Wg) {
    const long p = (long)blockIdx.x * blockDim.x + threadIdx.x;
    const unsigned off = (unsigned)p * (unsigned)sizeof(T);
    const unsigned bb = A.band_bytes;
    const int gs_ = A.gshift;
    const int L = Lrt;
    const BandArray<T> X{A.X, bb, gs_}, zP{A.zP, bb, gs_}, zT{A.zT, bb, gs_}, S{A.zV, bb, gs_}, GS{A.GS, bb, gs_},
        zPo{A.zPo, bb, gs_}, zTo{A.zTo, bb, gs_}, So{A.zVo, bb, gs_}, GSo{A.GSo, bb, gs_};
    const BandArray<T> Wdt{Wd, bb, gs_}, Wgt{Wg, bb, gs_};
    const bool wav = Wd != nullptr;
    const T rP = T(a.rho_P), rT = T(a.rho_T), rV = T(a.rho_V), rS = T(a.rho_S), tT = T(a.tau_T), tV = T(a.tau_V);
    const T irP = T(1.0 / a.rho_P), irT = T(1.0 / a.rho_T), irS = T(1.0 / a.rho_S);
    const T mT = T(m);
    double r2 = 0, s2 = 0, x2 = 0, v2 = 0, bz2 = 0, aty2 = 0, e = 0, p2 = 0, p1 = 0, pd = 0;
    T sv[LT], pv[LT];
#pragma unroll
    for (int l = 0; l < LT; ++l) {
        sv[l] = T(0);
        pv[l] = T(0);
        if (l < L) {
            const T x = X.load(l, off);
            const T zp = zP.load(l, off), zt = zT.load(l, off), go = GS.load(l, off), so = S.load(l, off);
            const T zp2 = zPo.load(l, off), zt2 = zTo.load(l, off), gn = GSo.load(l, off), sn = So.load(l, off);
            const T P = zp2 > T(0) ? zp2 : T(0), Po = zp > T(0) ? zp : T(0);
            const T Tn = softt(zt2, tT), To = softt(zt, tT);
            const T gp = rP * (zp2 < T(0) ? -zp2 : T(0)), gpo = rP * (zp < T(0) ? -zp : T(0));
            const T gt = -rT * clipt(zt2, tT), gto = -rT * clipt(zt, tT);
            const T dP = P - Po, dT = Tn - To, dS = sn - so, dg = gn - go;
            const T a1 = P - x, a2 = Tn - x, a3 = sn - x;
            r2 += double(a1 * a1 + a2 * a2 + a3 * a3);
            T sx = rP * dP + rT * dT + rS * dS;
            if (wav) sx += Wdt.load(l, off);
            s2 += double(sx * sx + mT * rV * rV * dS * dS);
            x2 += double(x * x);
            bz2 += double(P * P + Tn * Tn + (mT + T(1)) * sn * sn);
            T g = gp + gt + gn;
            if (wav) g += Wgt.load(l, off);
            aty2 += double(g * g);
            const T dgp = gp - gpo, dgt = gt - gto;
            e += double(rP * dP * dP + rT * dT * dT + (rS + mT * rV) * dS * dS + dgp * dgp * irP +
                        dgt * dgt * irT + dg * dg * irS);
            p2 += double(P * P);
            p1 += double(P);
            sv[l] = sn;
            pv[l] = P;
        }
    }
    for (int j = 0; j < m; ++j) {
        const BandArray<T> zv{Z.in[j], bb, gs_}, zvo{Z.out[j], bb, gs_};
        const T* Dj = D + (long)j * LT * LT;
        T c[LT];
        dense_fwd<T, LT>(c, sv, Dj);
#pragma unroll
        for (int k = 0; k < LT; ++k) {
            if (k < L) {
                const T V = softt(zv.load(k, off), tV);
                const T dv = V - c[k];
                const T gv = rV * (c[k] - zvo.load(k, off));
                r2 += double(dv * dv);
                e += double(rV * dv * dv);
                v2 += double(V * V);
                aty2 += double(gv * gv);
            }
        }
        dense_fwd<T, LT>(c, pv, Dj);
#pragma unroll
        for (int k = 0; k < LT; ++k) pd += fabs(double(c[k]));
    }
    __shared__ double sh[SPEC_NTH / 64];
    const double vals[RED_NQ] = {r2, s2, x2, v2, bz2, aty2, e, p2, p1, pd};
#pragma unroll
    for (int q = 0; q < RED_NQ; ++q) {
        const double sq = block_sum_s<SPEC_NTH>(vals[q], sh);
        if (threadIdx.x == 0) partials[(long)blockIdx.x * RED_NQ + q] = sq;
    }
}

// z_V,j <- (S W_j)(1 - ratio) + z_V,j ratio (new rho_V, ratio = rho_V / rho_V')
template <typename T, int LT>
__global__ void __launch_bounds__(SPEC_NTH)
k_union_reencode(const T* __restrict__ S, UnionZ Z, const T* __restrict__ D, int Lrt, int m, long npix, T ratio) {
    const long p = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= npix) return;
    T sv[LT];
#pragma unroll
    for (int l = 0; l < LT; ++l) sv[l] = l < Lrt ? S[(long)l * npix + p] : T(0);
    for (int j = 0; j < m; ++j) {
        T c[LT];
        dense_fwd<T, LT>(c, sv, D + (long)j * LT * LT);
        T* z = (T*)Z.in[j];
#pragma unroll
        for (int k = 0; k < LT; ++k)
            if (k < Lrt) z[(long)k * npix + p] = c[k] * (T(1) - ratio) + z[(long)k * npix + p] * ratio;
    }
}

template <typename T, int LT>
static hipError_t union_t(const SpecLaunch& g, const SpecArgs& a, hipStream_t s) {
    const long npix = g.npix;
    const int nth = npix < SPEC_NTH ? (int)npix : SPEC_NTH;
    if (npix < 64 || (npix & (npix - 1)) != 0) return hipErrorInvalidValue;
    dim3 grid((unsigned)(npix / nth));
    const unsigned bb = (unsigned)(npix * (long)sizeof(T));
    SpecArrays A{(char*)g.X, (char*)g.st[0], (char*)g.st[1], (char*)g.st[2], (char*)g.st[3],
                 (char*)g.out[0], (char*)g.out[1], (char*)g.out[2], (char*)g.out[3], (char*)g.brest,
                 bb, band_group_shift(bb)};
    UnionZ Z{};
    for (int j = 0; j < g.n_nu; ++j) {
        Z.in[j] = (char*)g.uz[j];
        Z.out[j] = (char*)g.uzo[j];
    }
    hipLaunchKernelGGL((k_spectral_union<T, LT>), grid, dim3(nth), 0, s, A, Z, (const T*)g.dctm, g.L, g.n_nu, a);
    if (g.report) {
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        // every partial sum of the convergence checks, the spectral terms included
        hipLaunchKernelGGL((k_report_union<T, LT>), grid, dim3(nth), 0, s, A, Z, (const T*)g.dctm, g.L, g.n_nu, a,
                           g.partials, (char*)g.wdt, (char*)g.wg);
    }
    return hipGetLastError();
}

template <typename T>
static hipError_t union_dispatch(const SpecLaunch& g, const SpecArgs& a, hipStream_t s) {
    if (g.L < 1 || (g.L > 32 && g.L != 64) || g.n_nu < 2 || g.n_nu > 4) return hipErrorInvalidValue;
    if (g.L <= 8) return union_t<T, 8>(g, a, s);
    if (g.L <= 16) return union_t<T, 16>(g, a, s);
    if (g.L <= 32) return union_t<T, 32>(g, a, s);
    return union_t<T, 64>(g, a, s);
}

template <typename T>
static hipError_t union_reencode_t(const void* S, void* const* uz, int n_nu, const void* D, int L, long npix,
                                   double ratio, hipStream_t s) {
    UnionZ Z{};
    for (int j = 0; j < n_nu; ++j) Z.in[j] = (char*)uz[j];
    const dim3 grid((unsigned)((npix + SPEC_NTH - 1) / SPEC_NTH)), blk(SPEC_NTH);
    if (L <= 8) hipLaunchKernelGGL((k_union_reencode<T, 8>), grid, blk, 0, s, (const T*)S, Z, (const T*)D, L, n_nu, npix, T(ratio));
    else if (L <= 16) hipLaunchKernelGGL((k_union_reencode<T, 16>), grid, blk, 0, s, (const T*)S, Z, (const T*)D, L, n_nu, npix, T(ratio));
    else if (L <= 32) hipLaunchKernelGGL((k_union_reencode<T, 32>), grid, blk, 0, s, (const T*)S, Z, (const T*)D, L, n_nu, npix, T(ratio));
    else hipLaunchKernelGGL((k_union_reencode<T, 64>), grid, blk, 0, s, (const T*)S, Z, (const T*)D, L, n_nu, npix, T(ratio));
    return hipGetLastError();
}

hipError_t launch_union_reencode(int dtype, const void* S, void* const* uz, int n_nu, const void* D, int L,
                                 long npix, double ratio, hipStream_t s) {
    if (n_nu < 2 || n_nu > 4 || L < 1 || (L > 32 && L != 64)) return hipErrorInvalidValue;
    return dtype == 0 ? union_reencode_t<float>(S, uz, n_nu, D, L, npix, ratio, s)
                      : union_reencode_t<double>(S, uz, n_nu, D, L, npix, ratio, s);
}

// ------------------------------------------------------------------ element-wise
template <typename T>
__global__ void __launch_bounds__(256)
k_brest(const T* __restrict__ zP, const T* __restrict__ zT, const T* __restrict__ zV,
        const T* __restrict__ GS, T* __restrict__ Brest, long n, SpecArgs a, bool s_stored) {
    const T rhoP = T(a.rho_P), rhoT = T(a.rho_T), rhoS = T(a.rho_S), tauT = T(a.tau_T);
    const T inv_rhoV = s_stored ? T(0) : T(1.0 / a.rho_V);
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
        const T zt = zT[i], gs = GS[i];
        const T sv = zV[i] + gs * inv_rhoV;
        Brest[i] = rhoT * (T(2) * softt(zt, tauT) - zt) + rhoP * fabs(zP[i]) + gs + rhoS * sv;
    }
}

// Re-encode the prox inputs for new parameters so that P, Gamma_P, S
// (always) and T, Gamma_T (when mu_s is unchanged) keep their values:
//   z_P' = max(0, z_P) - (rho_P / rho_P') max(0, -z_P)          (= P - Gamma_P / rho_P')
//   z_T' = soft(z_T, tau) + (rho_T / rho_T') clip(z_T, tau)     (= T - Gamma_T / rho_T')
//   z_V' = z_V + (1 / rho_V - 1 / rho_V') Gamma_S               (= S - Gamma_S / rho_V')
template <typename T>
__global__ void __launch_bounds__(256)
k_reencode(T* __restrict__ zP, T* __restrict__ zT, T* __restrict__ zV, const T* __restrict__ GS, long n,
           double rP, double rT, double tau, double dV) {
    const T ratioP = T(rP), ratioT = T(rT), t = T(tau), dv = T(dV);
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
        if (zP) {
            const T zp = zP[i];
            zP[i] = (zp > T(0) ? zp : T(0)) - ratioP * (zp < T(0) ? -zp : T(0));
        }
        if (zT) {
            const T zt = zT[i];
            zT[i] = softt(zt, t) + ratioT * clipt(zt, t);
        }
        if (zV && dV != 0.0) zV[i] += dv * GS[i];
    }
}

template <typename T>
__global__ void __launch_bounds__(256) k_add(T* __restrict__ d, const T* __restrict__ a, long n) {
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
        d[i] += a[i];
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

hipError_t launch_brest(int dtype, const void* zP, const void* zT, const void* zV, const void* GS,
                        void* Brest, size_t n, const SpecArgs& a, hipStream_t s, bool s_stored) {
    if (dtype == 0)
        hipLaunchKernelGGL((k_brest<float>), dim3(grid_for(n)), dim3(256), 0, s, (const float*)zP,
                           (const float*)zT, (const float*)zV, (const float*)GS, (float*)Brest, (long)n, a,
                           s_stored);
    else
        hipLaunchKernelGGL((k_brest<double>), dim3(grid_for(n)), dim3(256), 0, s, (const double*)zP,
                           (const double*)zT, (const double*)zV, (const double*)GS, (double*)Brest, (long)n, a,
                           s_stored);
    return hipGetLastError();
}

hipError_t launch_reencode(int dtype, void* zP, void* zT, void* zV, const void* GS, size_t n, double rP,
                           double rT, double tau, double dV, hipStream_t s) {
    if (dtype == 0)
        hipLaunchKernelGGL((k_reencode<float>), dim3(grid_for(n)), dim3(256), 0, s, (float*)zP, (float*)zT,
                           (float*)zV, (const float*)GS, (long)n, rP, rT, tau, dV);
    else
        hipLaunchKernelGGL((k_reencode<double>), dim3(grid_for(n)), dim3(256), 0, s, (double*)zP, (double*)zT,
                           (double*)zV, (const double*)GS, (long)n, rP, rT, tau, dV);
    return hipGetLastError();
}

hipError_t launch_add(int dtype, void* dst, const void* src, size_t n, hipStream_t s) {
    if (dtype == 0)
        hipLaunchKernelGGL((k_add<float>), dim3(grid_for(n)), dim3(256), 0, s, (float*)dst, (const float*)src, (long)n);
    else
        hipLaunchKernelGGL((k_add<double>), dim3(grid_for(n)), dim3(256), 0, s, (double*)dst, (const double*)src,
                           (long)n);
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
