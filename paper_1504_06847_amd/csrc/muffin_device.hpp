// Device building blocks of the gfx950 ADMM path: complex arithmetic,
// compile-time trigonometry, LDS-staged Stockham FFT stages and
// register-resident DCT-II / DCT-III along the band axis.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace muffin {

// ---------------------------------------------------------------- complex
template <typename T> struct alignas(2 * sizeof(T)) cx { T x, y; };

template <typename T> __device__ __forceinline__ cx<T> operator+(cx<T> a, cx<T> b) { return {a.x + b.x, a.y + b.y}; }
template <typename T> __device__ __forceinline__ cx<T> operator-(cx<T> a, cx<T> b) { return {a.x - b.x, a.y - b.y}; }
template <typename T> __device__ __forceinline__ cx<T> operator*(cx<T> a, T s) { return {a.x * s, a.y * s}; }
template <typename T> __device__ __forceinline__ cx<T> cmul(cx<T> a, cx<T> b) {
    return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
template <typename T> __device__ __forceinline__ cx<T> cmulc(cx<T> a, cx<T> b) {   // a * conj(b)
    return {a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y};
}
template <typename T> __device__ __forceinline__ cx<T> conj(cx<T> a) { return {a.x, -a.y}; }
template <typename T> __device__ __forceinline__ cx<T> mul_i(cx<T> a) { return {-a.y, a.x}; }    //  i a
template <typename T> __device__ __forceinline__ cx<T> mul_mi(cx<T> a) { return {a.y, -a.x}; }   // -i a

// ---------------------------------------------------------------- compile-time trig
// cos(pi n / d) and sin(pi n / d) evaluated by the front end: exact integer
// argument reduction to [0, pi/4], then Taylor series.
constexpr double kPi = 3.141592653589793238462643383279502884;

constexpr double taylor_sin(double x) {
    double x2 = x * x, term = x, sum = x;
    for (int k = 1; k < 14; ++k) { term *= -x2 / double((2 * k) * (2 * k + 1)); sum += term; }
    return sum;
}
constexpr double taylor_cos(double x) {
    double x2 = x * x, term = 1.0, sum = 1.0;
    for (int k = 1; k < 14; ++k) { term *= -x2 / double((2 * k - 1) * (2 * k)); sum += term; }
    return sum;
}
constexpr double cospi_ratio(long n, long d) {
    long p = 2 * d;
    n %= p;
    if (n < 0) n += p;
    if (n > d) n = p - n;                       // cos(2pi - a) = cos a
    double sgn = 1.0;
    if (2 * n > d) { n = d - n; sgn = -1.0; }   // cos(pi - a) = -cos a
    if (4 * n > d) return sgn * taylor_sin(kPi * double(d - 2 * n) / double(2 * d));
    return sgn * taylor_cos(kPi * double(n) / double(d));
}
constexpr double sinpi_ratio(long n, long d) { return cospi_ratio(2 * n - d, 2 * d); }

constexpr int ilog2c(int n) { return n <= 1 ? 0 : 1 + ilog2c(n >> 1); }

// square root of a positive double by Newton's iteration (front-end constant)
constexpr double sqrt_c(double v) {
    double x = v > 1.0 ? v : 1.0;
    for (int i = 0; i < 64; ++i) x = 0.5 * (x + v / x);
    return x;
}

// ---------------------------------------------------------------- band-strided access
// Element (l, p) of a [L][npix] array through raw buffer instructions: the
// descriptor (SGPRs) points at the first band of a group of 2^gshift bands,
// the band offset inside the group is a scalar offset and the pixel offset is
// one VGPR shared by every access of the thread.  With global loads the
// compiler keeps one 64-bit address per band live, which costs two VGPRs per
// band.  Groups keep every offset below 2^31 bytes (gshift from
// band_group_shift, groups of at most 1 GiB).  Callers mask lanes whose pixel lies outside the array.
constexpr int kBufWord3 = 0x00020000;   // raw 32-bit data format, gfx9 family
typedef unsigned u32x2_t __attribute__((ext_vector_type(2)));
// Cache-policy operand of the buffer instructions (CP below): 0 = default,
// kStreamCpol = non-temporal (the NT bit), for arrays read and written once
// per pass, so that they do not displace what the caches hold for reuse
// (the spectrum between the two kernels of a pass, register spills).
constexpr int kStreamCpol = 2;

template <typename T, int CP = 0> struct BandArray {
    char* base;
    unsigned band_bytes;
    int gshift;
    __device__ __forceinline__ __amdgpu_buffer_rsrc_t rsrc(int l) const {
        const int g = l >> gshift;
        return __builtin_amdgcn_make_buffer_rsrc(base + (size_t)(g << gshift) * band_bytes, (short)0,
                                                 0x7fffffff, kBufWord3);
    }
    __device__ __forceinline__ unsigned soff(int l) const {
        return (unsigned)(l & ((1 << gshift) - 1)) * band_bytes;
    }
    __device__ __forceinline__ T load(int l, unsigned lane_off) const {
        if constexpr (sizeof(T) == 4) {
            return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b32(rsrc(l), lane_off, soff(l), CP));
        } else {
            return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b64(rsrc(l), lane_off, soff(l), CP));
        }
    }
    __device__ __forceinline__ void store(int l, unsigned lane_off, T v) const {
        if constexpr (sizeof(T) == 4) {
            __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), rsrc(l), lane_off, soff(l), CP);
        } else {
            __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2_t, v), rsrc(l), lane_off, soff(l), CP);
        }
    }
};

// The same for an array whose L bands all lie within 2^30 bytes of its base:
// one descriptor for every band (the band offset is the scalar offset).
template <typename T, int CP = 0> struct BandArray1 {
    __amdgpu_buffer_rsrc_t r;
    unsigned band_bytes;
    __device__ __forceinline__ BandArray1(char* base, unsigned bb)
        : r(__builtin_amdgcn_make_buffer_rsrc(base, (short)0, 0x7fffffff, kBufWord3)), band_bytes(bb) {}
    __device__ __forceinline__ T load(int l, unsigned lane_off) const {
        if constexpr (sizeof(T) == 4)
            return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b32(r, lane_off, (unsigned)l * band_bytes, CP));
        else
            return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b64(r, lane_off, (unsigned)l * band_bytes, CP));
    }
    __device__ __forceinline__ void store(int l, unsigned lane_off, T v) const {
        if constexpr (sizeof(T) == 4)
            __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, lane_off, (unsigned)l * band_bytes, CP);
        else
            __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2_t, v), r, lane_off, (unsigned)l * band_bytes, CP);
    }
};

// largest gshift with 2^gshift bands of band_bytes each within 2^30 bytes
__host__ __device__ inline int band_group_shift(unsigned long long band_bytes) {
    int g = 0;
    while (g < 29 && (band_bytes << (g + 1)) <= (1ull << 30)) ++g;
    return g;
}

// ---------------------------------------------------------------- small DFTs in registers
// Forward: y_q = sum_r v_r exp(-2 pi i r q / R); inverse uses exp(+...).
template <typename T, bool INV> __device__ __forceinline__ void dft2(cx<T>* v) {
    cx<T> a = v[0];
    v[0] = a + v[1];
    v[1] = a - v[1];
}

template <typename T, bool INV> __device__ __forceinline__ void dft4(cx<T>& a0, cx<T>& a1, cx<T>& a2, cx<T>& a3) {
    cx<T> s02 = a0 + a2, d02 = a0 - a2, s13 = a1 + a3, d13 = a1 - a3;
    cx<T> j13 = INV ? mul_i(d13) : mul_mi(d13);
    a0 = s02 + s13;
    a2 = s02 - s13;
    a1 = d02 + j13;
    a3 = d02 - j13;
}

template <typename T, bool INV> __device__ __forceinline__ void dft8(cx<T>* v) {
    const T h = T(0.70710678118654752440084436210484903928);
    cx<T> e0 = v[0], e1 = v[2], e2 = v[4], e3 = v[6];
    cx<T> o0 = v[1], o1 = v[3], o2 = v[5], o3 = v[7];
    dft4<T, INV>(e0, e1, e2, e3);
    dft4<T, INV>(o0, o1, o2, o3);
    // o_q *= w8^q, w8 = exp(-+ i pi / 4)
    if (!INV) {
        o1 = {(o1.x + o1.y) * h, (o1.y - o1.x) * h};
        o2 = mul_mi(o2);
        o3 = {(o3.y - o3.x) * h, -(o3.x + o3.y) * h};
    } else {
        o1 = {(o1.x - o1.y) * h, (o1.x + o1.y) * h};
        o2 = mul_i(o2);
        o3 = {-(o3.x + o3.y) * h, (o3.x - o3.y) * h};
    }
    v[0] = e0 + o0; v[4] = e0 - o0;
    v[1] = e1 + o1; v[5] = e1 - o1;
    v[2] = e2 + o2; v[6] = e2 - o2;
    v[3] = e3 + o3; v[7] = e3 - o3;
}

template <typename T, int R, bool INV> __device__ __forceinline__ void dftR(cx<T>* v) {
    if constexpr (R == 2) dft2<T, INV>(v);
    else if constexpr (R == 4) dft4<T, INV>(v[0], v[1], v[2], v[3]);
    else dft8<T, INV>(v);
}

// ---------------------------------------------------------------- FFT plans
// Radix sequence for a power-of-two length: radix-8 stages, with one radix-4
// (or two for lengths 2^(3q+1)) where 8 does not divide.
constexpr int plan_nstages(int n) {
    int m = ilog2c(n);
    if (n == 2) return 1;
    int q = m / 3, r = m % 3;
    return r == 0 ? q : (r == 2 ? q + 1 : q + 1);
}
constexpr int plan_radix(int n, int s) {
    int m = ilog2c(n);
    if (n == 2) return 2;
    int q = m / 3, r = m % 3;
    if (r == 0) return 8;
    if (r == 2) return s < q ? 8 : 4;
    return s < q - 1 ? 8 : 4;       // 2^(3q+1) = 8^(q-1) * 4 * 4
}
constexpr int plan_ns(int n, int s) {   // product of the radices before stage s
    int p = 1;
    for (int i = 0; i < s; ++i) p *= plan_radix(n, i);
    return p;
}

// LDS position of element e of a transform: with PAD, one spare slot after
// every 8 elements, which spreads the stride-R writes of a Stockham stage
// over the LDS banks (without it they collide 8 to 16 ways).
template <bool PAD> __host__ __device__ constexpr int lds_pos(int e) { return PAD ? e + (e >> 3) : e; }
template <bool PAD> __host__ __device__ constexpr int lds_len(int n) { return PAD ? n + (n >> 3) : n; }

// Twiddles w^r, r = 1..R-1, of one butterfly, w = exp(-2 pi i k / (NS R)):
// w, w^2 and w^4 come from the table (exact to the table's rounding), the
// others as one product of two table values.
// Entry i of a twiddle table with one spare slot after every 2^TWP entries
// (TWP > 0, tables in LDS: the stride-2^s reads of a stage then spread over
// the banks instead of hitting one).
template <int TWP> __host__ __device__ constexpr int tw_at(int i) { return TWP > 0 ? i + (i >> TWP) : i; }

template <typename T, int R, int TWP = 0>
__device__ __forceinline__ void stage_twiddles(cx<T>* w, const cx<T>* __restrict__ tw, int k, int shift) {
    w[1] = tw[tw_at<TWP>(k << shift)];
    if constexpr (R >= 4) {
        w[2] = tw[tw_at<TWP>((2 * k) << shift)];
        w[3] = cmul(w[1], w[2]);
    }
    if constexpr (R == 8) {
        w[4] = tw[tw_at<TWP>((4 * k) << shift)];
        w[5] = cmul(w[1], w[4]);
        w[6] = cmul(w[2], w[4]);
        w[7] = cmul(w[3], w[4]);
    }
}

// Element e of transform tr of an LDS tile.  ES > 0: at tr * TS + pos(e) * ES.
// ES == 0: column tiles (transform index fastest, NTRANS per row, no
// padding) with the rows of each window of W consecutive rows permuted,
// W = min(32 / NTRANS, first radix): row e goes to slot (e + e / R0) mod W
// of its window.  A wavefront then hits distinct banks both when it reads
// consecutive rows (every stage) and when the first stage writes rows R0
// apart.
template <int LEN, int NTRANS>
__device__ __forceinline__ int swz_pos(int e, int tr) {
    constexpr int R0 = plan_radix(LEN, 0);
    constexpr int W0 = NTRANS >= 32 ? 1 : 32 / NTRANS;
    constexpr int W = W0 < R0 ? W0 : R0;
    const int q = (e + (e >> ilog2c(R0))) & (W - 1);
    return ((e & ~(W - 1)) + q) * NTRANS + tr;
}
template <int LEN, int NTRANS, int TS, int ES, bool PAD>
__device__ __forceinline__ int tile_index(int tr, int e) {
    if constexpr (ES == 0) return swz_pos<LEN, NTRANS>(e, tr);
    else return tr * TS + lds_pos<PAD>(e) * ES;
}

// One Stockham autosort stage over a tile of NTRANS transforms of length LEN
// in LDS.  Element e of transform t sits at buf[tile_index(t, e)].
// Butterfly j (0 <= j < LEN/R) reads elements j + r LEN/R, multiplies input r
// by w_{NS R}^{r (j mod NS)}, applies an R-point DFT and writes output q to
// (j - j mod NS) R + (j mod NS) + q NS.  Work items (transform, butterfly) are
// spread over NTH threads: TFAST puts the transform index fastest across
// threads (strided tiles), otherwise the butterfly index.
template <typename T, int LEN, int R, int NS, int NTRANS, int NTH, int TS, int ES, bool TFAST, bool PAD, bool INV,
          int TWP = 0>
__device__ __forceinline__ void fft_stage(cx<T>* buf, const cx<T>* __restrict__ tw, int twlog, int t) {
    constexpr int NB = LEN / R;
    constexpr int ITEMS = NB * NTRANS;
    constexpr int IPT = (ITEMS + NTH - 1) / NTH;
    constexpr int LOGNR = ilog2c(NS * R);
    cx<T> v[IPT][R];
#pragma unroll
    for (int i = 0; i < IPT; ++i) {
        const int item = t + i * NTH;
        if ((ITEMS % NTH) == 0 || item < ITEMS) {
            const int tr = TFAST ? item % NTRANS : item / NB;
            const int j = TFAST ? item / NTRANS : item % NB;
#pragma unroll
            for (int r = 0; r < R; ++r) v[i][r] = buf[tile_index<LEN, NTRANS, TS, ES, PAD>(tr, j + r * NB)];
            if constexpr (NS > 1) {
                const int k = j & (NS - 1);
                cx<T> w[R];
                stage_twiddles<T, R, TWP>(w, tw, k, twlog - LOGNR);
#pragma unroll
                for (int r = 1; r < R; ++r) v[i][r] = INV ? cmulc(v[i][r], w[r]) : cmul(v[i][r], w[r]);
            }
            dftR<T, R, INV>(v[i]);
        }
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < IPT; ++i) {
        const int item = t + i * NTH;
        if ((ITEMS % NTH) == 0 || item < ITEMS) {
            const int tr = TFAST ? item % NTRANS : item / NB;
            const int j = TFAST ? item / NTRANS : item % NB;
            const int k = j & (NS - 1);
            const int base = (j - k) * R + k;
#pragma unroll
            for (int r = 0; r < R; ++r) buf[tile_index<LEN, NTRANS, TS, ES, PAD>(tr, base + r * NS)] = v[i][r];
        }
    }
    __syncthreads();
}

template <typename T, int LEN, int NTRANS, int NTH, int TS, int ES, bool TFAST, bool PAD, bool INV, int S,
          int TWP = 0>
__device__ __forceinline__ void fft_stages(cx<T>* buf, const cx<T>* __restrict__ tw, int twlog, int t) {
    if constexpr (S < plan_nstages(LEN)) {
        fft_stage<T, LEN, plan_radix(LEN, S), plan_ns(LEN, S), NTRANS, NTH, TS, ES, TFAST, PAD, INV, TWP>(buf, tw, twlog, t);
        fft_stages<T, LEN, NTRANS, NTH, TS, ES, TFAST, PAD, INV, S + 1, TWP>(buf, tw, twlog, t);
    }
}

// In-place FFT of NTRANS transforms of length LEN held in LDS (natural order
// in and out, unnormalised).  Must be called by all NTH threads of the block.
// Stages S .. E-1 of the plan.
template <typename T, int LEN, int NTRANS, int NTH, int TS, int ES, bool TFAST, bool PAD, bool INV, int S, int E,
          int TWP = 0>
__device__ __forceinline__ void fft_stage_range(cx<T>* buf, const cx<T>* __restrict__ tw, int twlog, int t) {
    if constexpr (S < E) {
        fft_stage<T, LEN, plan_radix(LEN, S), plan_ns(LEN, S), NTRANS, NTH, TS, ES, TFAST, PAD, INV, TWP>(buf, tw, twlog, t);
        fft_stage_range<T, LEN, NTRANS, NTH, TS, ES, TFAST, PAD, INV, S + 1, E, TWP>(buf, tw, twlog, t);
    }
}

// The first stage (no twiddles) with its input read from global memory:
// element e of transform tr at src[e * ld + tr], zero for tr >= ntr; with
// re0, transform 0 reads only the real parts (its imaginary parts as zero).
// Its output goes to the LDS tile; ends with a barrier.
template <typename T, int LEN, int NTRANS, int NTH, int TS, int ES, bool TFAST, bool PAD, bool INV>
__device__ __forceinline__ void fft_first_stage_global(cx<T>* buf, const cx<T>* __restrict__ src, long ld,
                                                       int ntr, int t, bool re0 = false) {
    constexpr int R = plan_radix(LEN, 0);
    constexpr int NB = LEN / R;
    constexpr int ITEMS = NB * NTRANS;
    constexpr int IPT = (ITEMS + NTH - 1) / NTH;
    cx<T> v[IPT][R];
#pragma unroll
    for (int i = 0; i < IPT; ++i) {
        const int item = t + i * NTH;
        if ((ITEMS % NTH) == 0 || item < ITEMS) {
            const int tr = TFAST ? item % NTRANS : item / NB;
            const int j = TFAST ? item / NTRANS : item % NB;
#pragma unroll
            for (int r = 0; r < R; ++r) {
                v[i][r] = tr < ntr ? src[(long)(j + r * NB) * ld + tr] : cx<T>{T(0), T(0)};
                if (re0 && tr == 0) v[i][r].y = T(0);
            }
            dftR<T, R, INV>(v[i]);
        }
    }
#pragma unroll
    for (int i = 0; i < IPT; ++i) {
        const int item = t + i * NTH;
        if ((ITEMS % NTH) == 0 || item < ITEMS) {
            const int tr = TFAST ? item % NTRANS : item / NB;
            const int j = TFAST ? item / NTRANS : item % NB;
#pragma unroll
            for (int r = 0; r < R; ++r) buf[tile_index<LEN, NTRANS, TS, ES, PAD>(tr, j * R + r)] = v[i][r];
        }
    }
    __syncthreads();
}

// The last stage with its output written to global memory: element e of
// transform tr to dst[e * ld + tr] for tr < ntr.  No barrier at the end.
template <typename T, int LEN, int NTRANS, int NTH, int TS, int ES, bool TFAST, bool PAD, bool INV, int TWP = 0>
__device__ __forceinline__ void fft_last_stage_global(const cx<T>* buf, const cx<T>* __restrict__ tw, int twlog,
                                                      cx<T>* dst, long ld, int ntr, int t) {
    constexpr int S = plan_nstages(LEN) - 1;
    constexpr int R = plan_radix(LEN, S), NS = plan_ns(LEN, S);
    constexpr int NB = LEN / R;
    constexpr int ITEMS = NB * NTRANS;
    constexpr int IPT = (ITEMS + NTH - 1) / NTH;
    constexpr int LOGNR = ilog2c(NS * R);
#pragma unroll
    for (int i = 0; i < IPT; ++i) {
        const int item = t + i * NTH;
        if ((ITEMS % NTH) == 0 || item < ITEMS) {
            const int tr = TFAST ? item % NTRANS : item / NB;
            const int j = TFAST ? item / NTRANS : item % NB;
            cx<T> v[R];
#pragma unroll
            for (int r = 0; r < R; ++r) v[r] = buf[tile_index<LEN, NTRANS, TS, ES, PAD>(tr, j + r * NB)];
            const int k = j & (NS - 1);
            if constexpr (NS > 1) {
                cx<T> w[R];
                stage_twiddles<T, R, TWP>(w, tw, k, twlog - LOGNR);
#pragma unroll
                for (int r = 1; r < R; ++r) v[r] = INV ? cmulc(v[r], w[r]) : cmul(v[r], w[r]);
            }
            dftR<T, R, INV>(v);
            const int base = (j - k) * R + k;
            if (tr < ntr) {
#pragma unroll
                for (int r = 0; r < R; ++r) dst[(long)(base + r * NS) * ld + tr] = v[r];
            }
        }
    }
}

template <typename T, int LEN, int NTRANS, int NTH, int TS, int ES, bool TFAST, bool PAD, bool INV, int TWP = 0>
__device__ __forceinline__ void tile_fft(cx<T>* buf, const cx<T>* __restrict__ tw, int twlog, int t) {
    fft_stages<T, LEN, NTRANS, NTH, TS, ES, TFAST, PAD, INV, 0, TWP>(buf, tw, twlog, t);
}

// ---------------------------------------------------------------- real rows
// A real row x_0 .. x_{nx-1} is transformed as the M = nx/2 point complex
// sequence z_m = x_{2m} + i x_{2m+1}.  Packed half spectrum of the row:
// slot 0 holds the two real values (X_0, X_{nx/2}), slot k (0 < k < M) X_k.
// l: the row's M-point spectrum Z in LDS (padded positions); o: the packed
// output row; k in [0, M/2] produces slots k and M - k.
template <typename T, int NX, int TWP = 0>
__device__ __forceinline__ void rfft_post(const cx<T>* l, cx<T>* o, int k, const cx<T>* __restrict__ tw,
                                          int twlog) {
    constexpr int M = NX / 2;
    const cx<T> zk = l[lds_pos<true>(k)];
    if (k == 0) {
        o[0] = {zk.x + zk.y, zk.x - zk.y};           // (X_0, X_{nx/2}), both real
    } else if (k == M / 2) {
        o[k] = conj(zk);
    } else {
        const cx<T> zm = l[lds_pos<true>(M - k)];
        // even/odd sample spectra E = (Z_k + conj Z_{M-k})/2, O = -i (Z_k - conj Z_{M-k})/2
        const cx<T> e = {T(0.5) * (zk.x + zm.x), T(0.5) * (zk.y - zm.y)};
        const cx<T> od = {T(0.5) * (zk.y + zm.y), T(-0.5) * (zk.x - zm.x)};
        const cx<T> wo = cmul(od, tw[tw_at<TWP>(k << (twlog - ilog2c(NX)))]);
        o[k] = e + wo;                                // X_k = E + w^k O
        o[M - k] = conj(e - wo);                      // X_{M-k} = conj(E - w^k O)
    }
}

// The inverse: from the packed half spectrum p of a row, slots k and M - k of
// the M-point spectrum whose inverse FFT is z_m = x_{2m} + i x_{2m+1}
// (unnormalised), written to the LDS row l.
template <typename T, int NX, int TWP = 0>
__device__ __forceinline__ void irfft_pre(const cx<T>* p, cx<T>* l, int k, const cx<T>* __restrict__ tw,
                                          int twlog) {
    constexpr int M = NX / 2;
    const cx<T> xk = p[k];
    if (k == 0) {
        l[0] = {T(0.5) * (xk.x + xk.y), T(0.5) * (xk.x - xk.y)};
    } else if (k == M / 2) {
        l[lds_pos<true>(k)] = conj(xk);
    } else {
        const cx<T> xm = p[M - k];
        const cx<T> e = {T(0.5) * (xk.x + xm.x), T(0.5) * (xk.y - xm.y)};
        const cx<T> d = {T(0.5) * (xk.x - xm.x), T(0.5) * (xk.y + xm.y)};
        const cx<T> o = cmulc(d, tw[tw_at<TWP>(k << (twlog - ilog2c(NX)))]);   // O = w^{-k} D
        l[lds_pos<true>(k)] = e + mul_i(o);                         // Z_k = E + i O
        l[lds_pos<true>(M - k)] = conj(e) + mul_i(conj(o));
    }
}

// non-temporal loads of constants read once per pass
template <typename T> __device__ __forceinline__ T stream_load(const T* p) { return __builtin_nontemporal_load(p); }
template <typename T> __device__ __forceinline__ cx<T> stream_load(const cx<T>* p) {
    typedef T v2 __attribute__((ext_vector_type(2)));
    const v2 v = __builtin_nontemporal_load(reinterpret_cast<const v2*>(p));
    return {v.x, v.y};
}

// ---------------------------------------------------------------- register FFT / DCT
// Complex FFT of N points held in registers (radix-2, decimation in time
// after a compile-time bit reversal).  Every twiddle is a template-argument
// constant expression, so the whole transform is straight-line code.
template <int N> constexpr int bitrev(int i) {
    int r = 0;
    for (int b = 0; b < ilog2c(N); ++b) r |= ((i >> b) & 1) << (ilog2c(N) - 1 - b);
    return r;
}

template <typename T, int N, bool INV, int LEN, int K>
__host__ __device__ __forceinline__ void reg_fft_k(T (&re)[N], T (&im)[N]) {
    if constexpr (K < LEN / 2) {
        constexpr double c = cospi_ratio(2 * K, LEN);
        constexpr double s = INV ? sinpi_ratio(2 * K, LEN) : -sinpi_ratio(2 * K, LEN);
#pragma unroll
        for (int i = 0; i < N; i += LEN) {
            const int a = i + K, b = i + K + LEN / 2;
            T tr, ti;
            if constexpr (K == 0) { tr = re[b]; ti = im[b]; }
            else { tr = re[b] * T(c) - im[b] * T(s); ti = re[b] * T(s) + im[b] * T(c); }
            re[b] = re[a] - tr; im[b] = im[a] - ti;
            re[a] = re[a] + tr; im[a] = im[a] + ti;
        }
        reg_fft_k<T, N, INV, LEN, K + 1>(re, im);
    }
}

template <typename T, int N, bool INV, int LEN>
__host__ __device__ __forceinline__ void reg_fft_len(T (&re)[N], T (&im)[N]) {
    if constexpr (LEN <= N) {
        reg_fft_k<T, N, INV, LEN, 0>(re, im);
        reg_fft_len<T, N, INV, 2 * LEN>(re, im);
    }
}

template <typename T, int N, bool INV> __host__ __device__ __forceinline__ void reg_fft(T (&re)[N], T (&im)[N]) {
#pragma unroll
    for (int i = 0; i < N; ++i) {
        const int j = bitrev<N>(i);
        if (j > i) {
            T a = re[i]; re[i] = re[j]; re[j] = a;
            T b = im[i]; im[i] = im[j]; im[j] = b;
        }
    }
    reg_fft_len<T, N, INV, 2>(re, im);
}

// DCT-II post-processing of output index K (0 <= K <= M = L/2) from the
// L/2-point FFT Z of (v_{2m} + i v_{2m+1}):
//   V_K = E + w^K O, E = (Z_K + conj Z_{M-K}) / 2, O = -i (Z_K - conj Z_{M-K}) / 2,
//   w = exp(-2 pi i / L);  q = exp(-i pi K / 2L) V_K;  c_K = Re q, c_{L-K} = -Im q.
template <typename T, int L, int K>
__host__ __device__ __forceinline__ void dct2_one(T zr, T zi, T mr, T mi, T& qr, T& qi) {
    constexpr double wc = cospi_ratio(2 * K, L), ws = -sinpi_ratio(2 * K, L);
    constexpr double qc = cospi_ratio(K, 2 * L), qs = -sinpi_ratio(K, 2 * L);
    const T er = T(0.5) * (zr + mr), ei = T(0.5) * (zi - mi);
    const T orr = T(0.5) * (zi + mi), oi = T(-0.5) * (zr - mr);
    const T vr = er + (orr * T(wc) - oi * T(ws)), vi = ei + (orr * T(ws) + oi * T(wc));
    qr = vr * T(qc) - vi * T(qs);
    qi = vr * T(qs) + vi * T(qc);
}

// Outputs K and M - K are produced together from Z_K and Z_{M-K}, so the four
// registers consumed become the four outputs (the transform stays in place).
template <typename T, int L, int K>
__host__ __device__ __forceinline__ void dct2_post(T (&a)[L], T (&re)[L / 2], T (&im)[L / 2]) {
    constexpr int M = L / 2;
    constexpr double s0 = 1.0 / sqrt_c(double(L)), sk = sqrt_c(2.0 / double(L));
    if constexpr (K == 0) {
        T q0r, q0i, qmr, qmi;
        dct2_one<T, L, 0>(re[0], im[0], re[0], im[0], q0r, q0i);
        dct2_one<T, L, M>(re[0], im[0], re[0], im[0], qmr, qmi);
        a[0] = q0r * T(s0);
        a[M] = qmr * T(sk);
        dct2_post<T, L, 1>(a, re, im);
    } else if constexpr (2 * K < M) {
        constexpr int J = M - K;
        T qkr, qki, qjr, qji;
        dct2_one<T, L, K>(re[K], im[K], re[J], im[J], qkr, qki);
        dct2_one<T, L, J>(re[J], im[J], re[K], im[K], qjr, qji);
        a[K] = qkr * T(sk); a[L - K] = -qki * T(sk);
        a[J] = qjr * T(sk); a[L - J] = -qji * T(sk);
        dct2_post<T, L, K + 1>(a, re, im);
    } else if constexpr (2 * K == M) {
        T qr, qi;
        dct2_one<T, L, K>(re[K], im[K], re[K], im[K], qr, qi);
        a[K] = qr * T(sk); a[L - K] = -qi * T(sk);
    }
}

// Orthonormal DCT-II of L (power of two) values in registers:
// c_k = a_k sum_l x_l cos(pi (2l + 1) k / (2L)), a_0 = sqrt(1/L), a_k = sqrt(2/L).
// Makhoul (1980): reorder v_n = x_{2n}, v_{L-1-n} = x_{2n+1}; the DCT is
// Re(exp(-i pi k / (2L)) V_k) with V the L-point DFT of v, obtained from an
// L/2-point complex FFT of (v_{2m} + i v_{2m+1}).
template <typename T, int L> __host__ __device__ __forceinline__ void dct2_ortho(T (&a)[L]) {
    if constexpr (L == 1) {
        return;
    } else if constexpr (L == 2) {
        const T h = T(0.70710678118654752440084436210484903928);
        T s = (a[0] + a[1]) * h, d = (a[0] - a[1]) * h;
        a[0] = s; a[1] = d;
    } else {
        constexpr int M = L / 2;
        T re[M], im[M];
#pragma unroll
        for (int m = 0; m < M; ++m) {
            const int j0 = 2 * m, j1 = 2 * m + 1;            // positions in v
            re[m] = j0 < M ? a[2 * j0] : a[2 * (L - 1 - j0) + 1];
            im[m] = j1 < M ? a[2 * j1] : a[2 * (L - 1 - j1) + 1];
        }
        reg_fft<T, M, false>(re, im);
        dct2_post<T, L, 0>(a, re, im);      // inputs now live in re/im
    }
}

// DCT-III pre-processing for index K (0 <= K <= M): with the orthonormal
// scaling undone and the 1/M of the inverse FFT folded in,
//   V_K = exp(i pi K / 2L) (X_K - i X_{L-K})  (X_L = 0).
template <typename T, int L, int K>
__host__ __device__ __forceinline__ void dct3_v(T xk, T xlk, T& vr, T& vi) {
    constexpr int M = L / 2;
    constexpr double s0 = sqrt_c(double(L)) / double(M);
    constexpr double sk = sqrt_c(double(L) / 2.0) / double(M);
    constexpr double qc = cospi_ratio(K, 2 * L), qs = sinpi_ratio(K, 2 * L);
    const T xr = (K == 0 ? T(s0) : T(sk)) * xk;
    const T xi = K == 0 ? T(0) : -(T(sk) * xlk);
    vr = xr * T(qc) - xi * T(qs);
    vi = xr * T(qs) + xi * T(qc);
}

// Z_K = E + i O with E = (V_K + conj V_{M-K}) / 2, O = exp(2 pi i K / L) (V_K - conj V_{M-K}) / 2
template <typename T, int L, int K>
__host__ __device__ __forceinline__ void dct3_z(T vkr, T vki, T vjr, T vji, T& zr, T& zi) {
    constexpr double wc = cospi_ratio(2 * K, L), ws = sinpi_ratio(2 * K, L);
    const T er = T(0.5) * (vkr + vjr), ei = T(0.5) * (vki - vji);
    const T dr = T(0.5) * (vkr - vjr), di = T(0.5) * (vki + vji);
    const T orr = dr * T(wc) - di * T(ws), oi = dr * T(ws) + di * T(wc);
    zr = er - oi;
    zi = ei + orr;
}

// pairs (K, M - K): inputs X_K, X_{L-K}, X_{M-K}, X_{M+K} -> Z_K, Z_{M-K}
template <typename T, int L, int K>
__host__ __device__ __forceinline__ void dct3_pre(const T (&a)[L], T (&re)[L / 2], T (&im)[L / 2]) {
    constexpr int M = L / 2;
    if constexpr (K == 0) {
        T v0r, v0i, vmr, vmi;
        dct3_v<T, L, 0>(a[0], T(0), v0r, v0i);
        dct3_v<T, L, M>(a[M], a[M], vmr, vmi);
        dct3_z<T, L, 0>(v0r, v0i, vmr, vmi, re[0], im[0]);
        dct3_pre<T, L, 1>(a, re, im);
    } else if constexpr (2 * K < M) {
        constexpr int J = M - K;
        T vkr, vki, vjr, vji;
        dct3_v<T, L, K>(a[K], a[L - K], vkr, vki);
        dct3_v<T, L, J>(a[J], a[L - J], vjr, vji);
        dct3_z<T, L, K>(vkr, vki, vjr, vji, re[K], im[K]);
        dct3_z<T, L, J>(vjr, vji, vkr, vki, re[J], im[J]);
        dct3_pre<T, L, K + 1>(a, re, im);
    } else if constexpr (2 * K == M) {
        T vr, vi;
        dct3_v<T, L, K>(a[K], a[L - K], vr, vi);
        dct3_z<T, L, K>(vr, vi, vr, vi, re[K], im[K]);
    }
}

// Orthonormal DCT-III (the inverse / transpose of dct2_ortho).
template <typename T, int L> __host__ __device__ __forceinline__ void dct3_ortho(T (&a)[L]) {
    if constexpr (L == 1) {
        return;
    } else if constexpr (L == 2) {
        const T h = T(0.70710678118654752440084436210484903928);
        T s = (a[0] + a[1]) * h, d = (a[0] - a[1]) * h;
        a[0] = s; a[1] = d;
    } else {
        constexpr int M = L / 2;
        T re[M], im[M];
        dct3_pre<T, L, 0>(a, re, im);
        reg_fft<T, M, true>(re, im);
        // v_{2m} = Re z_m, v_{2m+1} = Im z_m; x_{2n} = v_n, x_{2n+1} = v_{L-1-n}
#pragma unroll
        for (int m = 0; m < M; ++m) {
            const int j0 = 2 * m, j1 = 2 * m + 1;
            if (j0 < M) a[2 * j0] = re[m]; else a[2 * (L - 1 - j0) + 1] = re[m];
            if (j1 < M) a[2 * j1] = im[m]; else a[2 * (L - 1 - j1) + 1] = im[m];
        }
    }
}

// The two-wave split of a 2N-band vector (the spectral passes at 128 and
// 256 bands) exchanges its N registers through LDS in two rounds: round q
// moves registers [0, N/4) and [3N/4, N) (q = 0), then [N/4, 3N/4) (q = 1),
// so that register r and register N - 1 - r travel together; slot i of a
// round holds register round_reg(q, i), register r sits in slot slot_of(r).
template <int N> __host__ __device__ constexpr int round_reg(int q, int i) {
    return q == 0 ? (i < N / 4 ? i : N / 2 + i) : N / 4 + i;
}
template <int N> __host__ __device__ constexpr int slot_of(int r) {
    return r < N / 4 ? r : (r < 3 * N / 4 ? r - N / 4 : r - N / 2);
}

// Orthonormal DCT-IV of N (a power of two) values in registers, its own
// inverse: y_k = sqrt(2/N) sum_n w_n cos(pi (2n + 1)(2k + 1) / (4N)).
// With M = N/2: z_m = (w_{2m} + i w_{N-1-2m}) exp(-i pi (4m + 1) / (4N)),
// Z the M-point DFT of z, u_k = Z_k exp(-i pi k / N); then
// y_{2k} = sqrt(2/N) Re u_k and y_{N-1-2k} = -sqrt(2/N) Im u_k.
template <typename T, int N, int K>
__host__ __device__ __forceinline__ void dct4_pre(const T (&a)[N], T (&re)[N / 2], T (&im)[N / 2]) {
    if constexpr (K < N / 2) {
        constexpr double c = cospi_ratio(4 * K + 1, 4 * N), s = sinpi_ratio(4 * K + 1, 4 * N);
        const T x = a[2 * K], y = a[N - 1 - 2 * K];
        re[K] = x * T(c) + y * T(s);
        im[K] = y * T(c) - x * T(s);
        dct4_pre<T, N, K + 1>(a, re, im);
    }
}

template <typename T, int N, int K>
__host__ __device__ __forceinline__ void dct4_post(T (&a)[N], const T (&re)[N / 2], const T (&im)[N / 2]) {
    if constexpr (K < N / 2) {
        constexpr double c = cospi_ratio(K, N), s = sinpi_ratio(K, N);
        constexpr double sc = sqrt_c(2.0 / double(N));
        const T ur = re[K] * T(c) + im[K] * T(s);
        const T ui = im[K] * T(c) - re[K] * T(s);
        a[2 * K] = ur * T(sc);
        a[N - 1 - 2 * K] = -(ui * T(sc));
        dct4_post<T, N, K + 1>(a, re, im);
    }
}

template <typename T, int N> __host__ __device__ __forceinline__ void dct4_ortho(T (&a)[N]) {
    if constexpr (N == 1) {
        return;
    } else {
        constexpr int M = N / 2;
        T re[M], im[M];
        dct4_pre<T, N, 0>(a, re, im);
        reg_fft<T, M, false>(re, im);
        dct4_post<T, N, 0>(a, re, im);
    }
}

// ---------------------------------------------------------------- band-axis helpers
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

}  // namespace muffin
