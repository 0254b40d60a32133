// The inverse row pass of step I, steps II-VI and the forward row pass of the
// next step I fused into one launch (Section 3, Algorithm 1; the 2-D FFT of
// the Fourier-domain solve of eq. Qlsimp split as in muffin_fft.hip).
//
// A work-group owns one image row y of every band: one thread per pixel x,
// holding the pixel's band vector in registers for the spectral steps (as
// k_spectral), and the row of G bands at a time in LDS for the row
// transforms:
//   A  V = soft(DCT(z_V)), q = IDCT(V)                         (registers)
//   B  for each group of G bands:
//        inverse real FFT of the column pass's spectrum rows -> X rows (LDS)
//        steps II, III, V, VI per pixel; X and the new state to HBM; B_rest
//          into the LDS rows in place of X
//        forward real FFT of B_rest -> the spectrum rows of the next column
//          pass (written over the rows read)
// X and B_rest never make an HBM round trip between kernels: 44 B/voxel in
// FP32 (Z, z_P, z_T, z_V, Gamma_S in; Z, X, z_P, z_T, z_V, Gamma_S out; the
// new state in place or into other arrays)
// against 56 B for the inverse row pass, spectral pass and forward row pass
// launched one after another.  The state is that of muffin_spectral.hip
// (z_V = S - Gamma_S / rho_V in place of S).
#include "muffin_device.hpp"
#include "muffin_kernels.hpp"

namespace muffin {

// PPT pixels per thread (x = t + p NX / PPT).  One pixel per thread runs NX
// threads at 4 waves per SIMD (at most 128 registers a lane); two pixels per
// thread run NX / 2 threads at 2 waves per SIMD (256 registers).  With 64
// bands on rows of 1024 (32 bands too) the first spills (the register-held
// part of q next to the row transforms), the second does not; the autotuner
// times both where both are built.  Both evaluate the same formulas per
// pixel and per butterfly; the compiler contracts products and sums into
// FMAs differently in the two, so results agree to rounding.
constexpr bool fused_two_pixels_at(int nx, int lt) { return (lt == 64 && nx >= 256) || (lt == 32 && nx == 1024); }
template <int NX, int LT> constexpr bool fused_two_pixels() { return fused_two_pixels_at(NX, LT); }

template <int LT> constexpr int fused_g() { return LT < 16 ? LT : (LT >= 64 ? 8 : 16); }
// with 64 bands, q of the last fused_qb bands waits in LDS: the band vector
// of the others plus the row transforms fill the registers
template <int LT> constexpr int fused_qb() { return LT >= 64 ? 28 : 0; }

template <typename T, int NX, int LT> struct FusedLds {
    cx<T> rows[fused_g<LT>() * lds_len<true>(NX / 2)];   // G spectrum / image rows
    cx<T> twl[tw_at<4>(NX)];                              // w_NX^i, i < NX (padded)
    T q[fused_qb<LT>() > 0 ? fused_qb<LT>() * NX : 1];   // PPT x NTH = NX values per band
};
static_assert(sizeof(FusedLds<float, 1024, 64>) <= 160 * 1024, "fused LDS exceeds 160 KiB");

// One image row y of every band (see the head of this file).
template <typename T, int NX, int LT, bool DENSE, int PPT>
__device__ __forceinline__ void fused_body(const FusedArrays& A, const T* __restrict__ D, int Lrt, int ny,
                                           const SpecArgs& a, const cx<T>* __restrict__ tw, int twlog, int y,
                                           FusedLds<T, NX, LT>& sh) {
    constexpr int NTH = NX / PPT;
    constexpr int M = NX / 2;
    constexpr int G = fused_g<LT>();                // bands per LDS row group
    constexpr int TS = lds_len<true>(M);
    constexpr int NK = M / 2 + 1;
    constexpr int TPR = NTH / G;                    // threads per LDS row in B1, B3
    static_assert(NTH % G == 0, "row split");
    cx<T>* lds = sh.rows;
    cx<T>* twl = sh.twl;
    constexpr int QB = fused_qb<LT>();
    T* qlds = sh.q;
    const int t = threadIdx.x;
    for (int i = t; i < NX; i += NTH) twl[tw_at<4>(i)] = tw[i << (twlog - ilog2c(NX))];
    __syncthreads();
    unsigned off[PPT];
#pragma unroll
    for (int p = 0; p < PPT; ++p) off[p] = (unsigned)((long)y * NX + t + p * NTH) * (unsigned)sizeof(T);
    const unsigned bb = A.band_bytes;
    // every band of an array within 2^30 bytes of its base (checked on the host)
    // the state and X stream through once per pass: non-temporal
    const BandArray1<T, kStreamCpol> X(A.X, bb), zP(A.zP, bb), zT(A.zT, bb), zV(A.zV, bb), GS(A.GS, bb);
    const BandArray1<T, kStreamCpol> zPo(A.zPo, bb), zTo(A.zTo, bb), zVo(A.zVo, bb), GSo(A.GSo, bb);
    // X goes out only when the caller reads it (A.X not null): the passes of a
    // run before its last overwrite it unread
    const bool wx = A.X != nullptr;
    cx<T>* Z = (cx<T>*)A.Z;
    const int L = DENSE ? Lrt : LT;
    const T rhoP = T(a.rho_P), rhoT = T(a.rho_T), rhoV = T(a.rho_V), rhoS = T(a.rho_S);
    const T tauT = T(a.tau_T), tauV = T(a.tau_V);
    const T inv_rhoV = T(1.0 / a.rho_V), inv_VS = T(1.0 / (a.rho_V + a.rho_S));

    T v[PPT][LT];
    // A: step IV with the previous z_V
#pragma unroll
    for (int p = 0; p < PPT; ++p) {
#pragma unroll
        for (int l = 0; l < LT; ++l) v[p][l] = (l < L) ? zV.load(l, off[p]) : T(0);
        dct_any<T, LT, DENSE, false>(v[p], D, L);
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int k = 0; k < LT; ++k) v[p][k] = softt(v[p][k], tauV);
        dct_any<T, LT, DENSE, true>(v[p], D, L);        // q = V W_nu^T
        // the last QB bands wait in LDS: the register-held ones are consumed
        // by the first groups, so fewer of them stay live across the row
        // transforms.  Stored as the inverse transform produces them (no
        // scheduling barrier in between), so all LT outputs are never live
        // together.
#pragma unroll
        for (int l = 0; l < QB; ++l) qlds[(l * PPT + p) * NTH + t] = v[p][LT - QB + l];
        __builtin_amdgcn_sched_barrier(0);
    }

    T* lrow = reinterpret_cast<T*>(lds);
#pragma unroll
    for (int g = 0; g < LT / G; ++g) {
        // the thread's addresses (LDS positions, twiddle indices, row
        // offsets) are the same in every group; computed from a copy of the
        // thread index that the compiler cannot see through, they are
        // recomputed per group instead of held in registers across all
        // groups next to the register-held part of q
        int tg = t;
        asm volatile("" : "+v"(tg));
        const int r0 = tg / TPR, k0 = tg % TPR;
        // B1: spectrum rows of bands g G .. g G + G - 1 at image row y; TPR
        // threads per row (one wavefront per row for NX = 1024)
        {
            const int l = g * G + r0;
            const cx<T>* prow = Z + ((long)l * ny + y) * M;
#pragma unroll
            for (int j = 0; j < (NK + TPR - 1) / TPR; ++j) {
                const int k = k0 + j * TPR;
                if (k < NK && l < L) irfft_pre<T, NX, 4>(prow, lds + r0 * TS, k, twl, ilog2c(NX));
            }
        }
        __syncthreads();
        __builtin_amdgcn_sched_barrier(0);
        tile_fft<T, M, G, NTH, TS, 1, false, true, true, 4>(lds, twl, ilog2c(NX), tg);
        __builtin_amdgcn_sched_barrier(0);
        // B2: steps II, III, V, VI at the thread's pixels for the group's bands
#pragma unroll
        for (int r = 0; r < G; ++r) {
            const int l = g * G + r;
#pragma unroll
            for (int p = 0; p < PPT; ++p) {
                if (l < L) {
                    const int x = tg + p * NTH;
                    const unsigned offp = (unsigned)((long)y * NX + x) * (unsigned)sizeof(T);
                    const int e = r * TS * 2 + 2 * lds_pos<true>(x >> 1) + (x & 1);
                    const T xv = lrow[e];
                    const T gs = GS.load(l, offp), zp = zP.load(l, offp), zt = zT.load(l, offp);
                    const T q = (l >= LT - QB) ? qlds[((l - (LT - QB)) * PPT + p) * NTH + tg] : v[p][l];
                    const T s = (rhoV * q + rhoS * xv) * inv_VS;
                    const T gs2 = gs + rhoV * (q - s);
                    const T zp2 = xv - (zp < T(0) ? -zp : T(0));
                    const T zt2 = xv + clipt(zt, tauT);
                    const T tt = softt(zt2, tauT);
                    const T zv2 = s - gs2 * inv_rhoV;
                    const T sv = zv2 + gs2 * inv_rhoV;       // S as stored (see k_spectral)
                    lrow[e] = rhoT * (T(2) * tt - zt2) + rhoP * fabs(zp2) + gs2 + rhoS * sv;
                    if (wx) X.store(l, offp, xv);
                    zVo.store(l, offp, zv2);
                    GSo.store(l, offp, gs2);
                    zPo.store(l, offp, zp2);
                    zTo.store(l, offp, zt2);
                }
            }
            if ((r & 3) == 3) __builtin_amdgcn_sched_barrier(0);
        }
        __syncthreads();
        __builtin_amdgcn_sched_barrier(0);
        asm volatile("" : "+v"(tg));       // as above: not held across B2
        tile_fft<T, M, G, NTH, TS, 1, false, true, false, 4>(lds, twl, ilog2c(NX), tg);
        __builtin_amdgcn_sched_barrier(0);
        // B3: packed spectrum rows of B_rest, over the rows read in B1
        {
            const int r0 = tg / TPR, k0 = tg % TPR;
            const int l = g * G + r0;
            cx<T>* prow = Z + ((long)l * ny + y) * M;
#pragma unroll
            for (int j = 0; j < (NK + TPR - 1) / TPR; ++j) {
                const int k = k0 + j * TPR;
                if (k < NK && l < L) rfft_post<T, NX, 4>(lds + r0 * TS, prow, k, twl, ilog2c(NX));
            }
        }
        __syncthreads();
        __builtin_amdgcn_sched_barrier(0);
    }
}

// one pixel per thread: at most 128 registers (4 waves per SIMD), so that a
// CU holds 16 waves at every row length (two 512-thread work-groups, four
// of 256, ...) as at 1024; two pixels per thread: 256 (2 waves per SIMD)
template <typename T, int NX, int LT, bool DENSE, int PPT>
__global__ void __launch_bounds__(NX / PPT, PPT == 1 ? 4 : 2)
k_fused(FusedArrays A, const T* __restrict__ D, int Lrt, int ny, SpecArgs a,
        const cx<T>* __restrict__ tw, int twlog) {
    __shared__ FusedLds<T, NX, LT> sh;
    fused_body<T, NX, LT, DENSE, PPT>(A, D, Lrt, ny, a, tw, twlog, blockIdx.x, sh);
}

// the fused pass over the rows of several cubes of one row length and band
// count (one block per image row of each cube)
template <typename T, int NX, int LT, bool DENSE>
__global__ void __launch_bounds__(NX, 4)
k_fused_group(const FusedDesc* __restrict__ d, int n) {
    __shared__ FusedLds<T, NX, LT> sh;
    int j = 0;
    while (j + 1 < n && blockIdx.x >= (unsigned)d[j + 1].first) ++j;
    const unsigned y = blockIdx.x - (unsigned)d[j].first;
    if (blockIdx.x < (unsigned)d[j].first || y >= (unsigned)d[j].nblk) return;
    fused_body<T, NX, LT, DENSE, 1>(d[j].A, (const T*)d[j].D, d[j].L, d[j].ny, d[j].a, (const cx<T>*)d[j].tw,
                                    d[j].twlog, (int)y, sh);
}

template <typename T, int NX, int LT, bool DENSE>
static hipError_t fused_t(const FusedArrays& A, const void* D, int L, int ny, const SpecArgs& a,
                          const void* tw, int twlog, hipStream_t s, int variant) {
    if constexpr (fused_two_pixels<NX, LT>()) {
        if (variant == 2) {
            hipLaunchKernelGGL((k_fused<T, NX, LT, DENSE, 2>), dim3(ny), dim3(NX / 2), 0, s, A, (const T*)D, L, ny,
                               a, (const cx<T>*)tw, twlog);
            return hipGetLastError();
        }
    }
    hipLaunchKernelGGL((k_fused<T, NX, LT, DENSE, 1>), dim3(ny), dim3(NX), 0, s, A, (const T*)D, L, ny, a,
                       (const cx<T>*)tw, twlog);
    return hipGetLastError();
}

template <typename T, int NX>
static hipError_t fused_l(const FusedArrays& A, const void* D, int L, int ny, const SpecArgs& a,
                          const void* tw, int twlog, hipStream_t s, int v) {
    switch (L) {
        case 4: return fused_t<T, NX, 4, false>(A, D, L, ny, a, tw, twlog, s, v);
        case 8: return fused_t<T, NX, 8, false>(A, D, L, ny, a, tw, twlog, s, v);
        case 16: return fused_t<T, NX, 16, false>(A, D, L, ny, a, tw, twlog, s, v);
        case 32: return fused_t<T, NX, 32, false>(A, D, L, ny, a, tw, twlog, s, v);
        case 64: return fused_t<T, NX, 64, false>(A, D, L, ny, a, tw, twlog, s, v);
        default: return hipErrorInvalidValue;
    }
}

bool fused_supported(int dtype, int nx, int ny, int L) {
    return dtype == 0 && nx >= 64 && nx <= 1024 && (L == 4 || L == 8 || L == 16 || L == 32 || L == 64) &&
           (long long)L * ny * nx * 4 <= (1ll << 30);
}

bool fused_two_pixel_variant(int nx, int L) { return fused_two_pixels_at(nx, L); }

hipError_t launch_fused(int dtype, const FusedArrays& A, const void* D, int L, int ny, int nx,
                        const SpecArgs& a, const void* tw, int twlog, hipStream_t s, int variant) {
    if (!fused_supported(dtype, nx, ny, L) || variant < 1 || variant > 2) return hipErrorInvalidValue;
    if (!A.zP || !A.zT || !A.zV || !A.GS || !A.zPo || !A.zTo || !A.zVo || !A.GSo || !A.Z)
        return hipErrorInvalidValue;
    switch (nx) {
        case 64: return fused_l<float, 64>(A, D, L, ny, a, tw, twlog, s, variant);
        case 128: return fused_l<float, 128>(A, D, L, ny, a, tw, twlog, s, variant);
        case 256: return fused_l<float, 256>(A, D, L, ny, a, tw, twlog, s, variant);
        case 512: return fused_l<float, 512>(A, D, L, ny, a, tw, twlog, s, variant);
        case 1024: return fused_l<float, 1024>(A, D, L, ny, a, tw, twlog, s, variant);
        default: return hipErrorInvalidValue;
    }
}

template <typename T, int NX, int LT>
static hipError_t fused_group_t(const FusedDesc* d, int n, int nblocks, hipStream_t s) {
    hipLaunchKernelGGL((k_fused_group<T, NX, LT, false>), dim3(nblocks), dim3(NX), 0, s,
                       d, n);
    return hipGetLastError();
}

template <int NX>
static hipError_t fused_group_l(int L, const FusedDesc* d, int n, int nblocks, hipStream_t s) {
    switch (L) {
        case 4: return fused_group_t<float, NX, 4>(d, n, nblocks, s);
        case 8: return fused_group_t<float, NX, 8>(d, n, nblocks, s);
        case 16: return fused_group_t<float, NX, 16>(d, n, nblocks, s);
        case 32: return fused_group_t<float, NX, 32>(d, n, nblocks, s);
        case 64: return fused_group_t<float, NX, 64>(d, n, nblocks, s);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_fused_group(int dtype, int nx, int L, const FusedDesc* d, int n, int nblocks,
                              hipStream_t s) {
    if (n <= 0 || nblocks <= 0) return hipSuccess;
    if (dtype != 0) return hipErrorInvalidValue;
    switch (nx) {
        case 64: return fused_group_l<64>(L, d, n, nblocks, s);
        case 128: return fused_group_l<128>(L, d, n, nblocks, s);
        case 256: return fused_group_l<256>(L, d, n, nblocks, s);
        case 512: return fused_group_l<512>(L, d, n, nblocks, s);
        case 1024: return fused_group_l<1024>(L, d, n, nblocks, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace muffin
