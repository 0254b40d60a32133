// 2-D FFT passes of step I for gfx950: the exact per-band solve
// (H_l^T H_l + rho I) x_l = b_l as a Fourier-domain filter (Section 3, eq.
// Qlsimp and the closing paragraph of the section), split in three HBM passes:
//   row pass   : real FFT along x of every row of every band, packed half
//                spectrum (slot 0 holds the kx = 0 and kx = nx/2 values, both
//                real for real rows, as real and imaginary part);
//   column pass: FFT along y of a tile of adjacent kx columns held in LDS,
//                multiplication by scale / (|h_hat|^2 + rho) after adding the
//                data term conj(h_hat) y_hat, inverse FFT along y;
//   row pass   : inverse real FFT along x.
// The same kernels, instantiated in double, compute the setup transforms.
#include "muffin_device.hpp"
#include "muffin_kernels.hpp"

namespace muffin {

constexpr int ROW_NTH = 256;

// rows per block: about 1024, 2048 or 4096 complex points per block (variant 0, 1, 2)
template <int M, int V> constexpr int row_rpw() {
    const int b = M >= 2048 ? 1 : 2048 / M;
    const int r = (b << V) >> 1;
    return r < 1 ? 1 : r;
}

template <typename T, int NY> constexpr int col_tc_base() {
    int tc = int(65536 / (NY * int(sizeof(cx<T>))));
    return tc > 16 ? 16 : (tc < 1 ? 1 : tc);
}
template <typename T, int NY> constexpr bool col_twl() { return NY * int(sizeof(cx<T>)) <= 16384; }
constexpr int COL_TWP = 4;                 // LDS twiddle table: one spare slot per 16 entries
template <int NY> constexpr int col_twl_len() { return tw_at<COL_TWP>(NY); }
template <typename T, int NY, int TC> constexpr int col_lds_bytes() {
    return NY * TC * int(sizeof(cx<T>)) + (col_twl<T, NY>() ? col_twl_len<NY>() * int(sizeof(cx<T>)) : 0) + 64;
}
// columns per tile of variant V: half, all or twice the 64-KiB tile
template <typename T, int NY, int V> constexpr int col_tc() {
    constexpr int b = col_tc_base<T, NY>();
    if (V == 0) return b > 1 ? b / 2 : 1;
    if (V == 1) return b;
    return (2 * b <= 16 && col_lds_bytes<T, NY, 2 * b>() <= 160 * 1024) ? 2 * b : b;
}
template <typename T, int NY, int TC> constexpr int col_nth() {
    int n = TC * NY / 8;
    return n > 512 ? 512 : (n < 64 ? 64 : n);
}

// The column pass's constants (the data term conj(h_hat) y_hat and
// |h_hat|^2, one value per packed half-spectrum point of each band) are
// stored in column-block order: blocks of W adjacent kx columns, each
// block's ny rows of W values contiguous, with W the tile width of the
// default column schedule (col_tc_base, at most M).  A column tile then
// reads them as consecutive runs instead of one short run per spectrum row.
template <typename T> __device__ __forceinline__ int filt_shift(int ny, int M) {
    int w = 65536 / (ny * int(sizeof(cx<T>)));
    w = w > 16 ? 16 : (w < 1 ? 1 : w);
    return __builtin_ctz(w < M ? w : M);
}
// offset of (ky, kx) in one band's block-ordered constants (sh = filt_shift)
__device__ __forceinline__ long filt_pos(int ny, int sh, int ky, int kx) {
    return ((long)(kx >> sh) * ny << sh) + ((long)ky << sh) + (kx & ((1 << sh) - 1));
}

template <int NTH> __device__ __forceinline__ double block_sum(double v, double* sh) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) sh[w] = v;
    __syncthreads();
    double r = 0.0;
    if (threadIdx.x == 0) {
        for (int i = 0; i < NTH / 64; ++i) r += sh[i];
    }
    __syncthreads();
    return r;
}

// cube of a grouped launch that block b works on, or -1 for a padding block
template <typename D>
__device__ __forceinline__ int group_find(const D* __restrict__ d, int n, unsigned b) {
    int j = 0;
    while (j + 1 < n && b >= (unsigned)d[j + 1].first) ++j;
    return (b >= (unsigned)d[j].first && b < (unsigned)(d[j].first + d[j].nblk)) ? j : -1;
}

// ------------------------------------------------------------------ row passes
template <typename Tin, typename T, int NX, bool SHIFT, bool POS, int RPW>
__device__ __forceinline__ void row_fwd_body(const Tin* __restrict__ in, cx<T>* __restrict__ out,
                                             int nrows, int ny, const cx<T>* __restrict__ tw,
                                             int twlog, long blk, cx<T>* lds) {
    constexpr int M = NX / 2;
    constexpr int TS = lds_len<true>(M);
    const int t = threadIdx.x;
    const long row0 = blk * RPW;
#pragma unroll
    for (int j = 0; j < (RPW * M + ROW_NTH - 1) / ROW_NTH; ++j) {
        const int i = t + j * ROW_NTH;
        if ((RPW * M) % ROW_NTH != 0 && i >= RPW * M) break;
        const int r = i / M, m = i % M;
        const long grow = row0 + r;
        cx<T> v = {T(0), T(0)};
        if (grow < nrows) {
            long srow = grow;
            int sm = m;
            if constexpr (SHIFT) {
                const long band = grow / ny;
                const int y = int(grow - band * ny);
                srow = band * ny + ((y + ny / 2) & (ny - 1));
                sm = (m + M / 2) & (M - 1);
            }
            const cx<Tin> q = reinterpret_cast<const cx<Tin>*>(in + srow * NX)[sm];
            T a = T(q.x), b = T(q.y);
            if constexpr (POS) {
                a = a > T(0) ? a : T(0);
                b = b > T(0) ? b : T(0);
            }
            v = {a, b};
        }
        lds[r * TS + lds_pos<true>(m)] = v;
    }
    __syncthreads();
    tile_fft<T, M, RPW, ROW_NTH, TS, 1, false, true, false>(lds, tw, twlog, t);
    constexpr int NK = M / 2 + 1;
#pragma unroll
    for (int j = 0; j < (RPW * NK + ROW_NTH - 1) / ROW_NTH; ++j) {
        const int i = t + j * ROW_NTH;
        if (i >= RPW * NK) break;
        const int r = i / NK, k = i % NK;
        const long grow = row0 + r;
        if (grow >= nrows) continue;
        rfft_post<T, NX>(lds + r * TS, out + grow * M, k, tw, twlog);
    }
}

template <typename Tin, typename T, int NX, bool SHIFT, bool POS, int V>
__global__ void __launch_bounds__(ROW_NTH)
k_row_fwd(const Tin* __restrict__ in, cx<T>* __restrict__ out, int nrows, int ny,
          const cx<T>* __restrict__ tw, int twlog) {
    constexpr int RPW = row_rpw<NX / 2, V>();
    __shared__ cx<T> lds[RPW * lds_len<true>(NX / 2)];
    row_fwd_body<Tin, T, NX, SHIFT, POS, RPW>(in, out, nrows, ny, tw, twlog, blockIdx.x, lds);
}

template <typename T, int NX, int V>
__global__ void __launch_bounds__(ROW_NTH)
k_row_fwd_group(const RowDesc* __restrict__ d, int n) {
    constexpr int RPW = row_rpw<NX / 2, V>();
    __shared__ cx<T> lds[RPW * lds_len<true>(NX / 2)];
    const int j = group_find(d, n, blockIdx.x);
    if (j < 0) return;
    row_fwd_body<T, T, NX, false, false, RPW>((const T*)d[j].in, (cx<T>*)d[j].out, d[j].nrows, 0,
                                             (const cx<T>*)d[j].tw, d[j].twlog,
                                             (long)(blockIdx.x - d[j].first), lds);
}

template <typename T, int NX, int RPW>
__device__ __forceinline__ void row_inv_body(const cx<T>* __restrict__ in, T* __restrict__ out,
                                             int nrows, const cx<T>* __restrict__ tw, int twlog,
                                             long blk, cx<T>* lds) {
    constexpr int M = NX / 2;
    constexpr int TS = lds_len<true>(M);
    const int t = threadIdx.x;
    const long row0 = blk * RPW;
    constexpr int NK = M / 2 + 1;
#pragma unroll
    for (int j = 0; j < (RPW * NK + ROW_NTH - 1) / ROW_NTH; ++j) {
        const int i = t + j * ROW_NTH;
        if (i >= RPW * NK) break;
        const int r = i / NK, k = i % NK;
        const long grow = row0 + r;
        if (grow >= nrows) continue;
        irfft_pre<T, NX>(in + grow * M, lds + r * TS, k, tw, twlog);
    }
    __syncthreads();
    tile_fft<T, M, RPW, ROW_NTH, TS, 1, false, true, true>(lds, tw, twlog, t);
#pragma unroll
    for (int j = 0; j < (RPW * M + ROW_NTH - 1) / ROW_NTH; ++j) {
        const int i = t + j * ROW_NTH;
        if ((RPW * M) % ROW_NTH != 0 && i >= RPW * M) break;
        const int r = i / M, m = i % M;
        const long grow = row0 + r;
        if (grow < nrows) reinterpret_cast<cx<T>*>(out + grow * NX)[m] = lds[r * TS + lds_pos<true>(m)];
    }
}

template <typename T, int NX, int V>
__global__ void __launch_bounds__(ROW_NTH)
k_row_inv(const cx<T>* __restrict__ in, T* __restrict__ out, int nrows,
          const cx<T>* __restrict__ tw, int twlog) {
    constexpr int RPW = row_rpw<NX / 2, V>();
    __shared__ cx<T> lds[RPW * lds_len<true>(NX / 2)];
    row_inv_body<T, NX, RPW>(in, out, nrows, tw, twlog, blockIdx.x, lds);
}

template <typename T, int NX, int V>
__global__ void __launch_bounds__(ROW_NTH)
k_row_inv_group(const RowDesc* __restrict__ d, int n) {
    constexpr int RPW = row_rpw<NX / 2, V>();
    __shared__ cx<T> lds[RPW * lds_len<true>(NX / 2)];
    const int j = group_find(d, n, blockIdx.x);
    if (j < 0) return;
    row_inv_body<T, NX, RPW>((const cx<T>*)d[j].in, (T*)d[j].out, d[j].nrows, (const cx<T>*)d[j].tw,
                             d[j].twlog, (long)(blockIdx.x - d[j].first), lds);
}

// ------------------------------------------------------------------ column pass
// One tile of TC adjacent kx columns of one band.  wg: the tile's index in
// the launch (or in its cube's block range), nwg: tiles of the cube, ntiles:
// tiles per band.
template <typename T, int NY, int MODE, int TC>
__device__ __forceinline__ void col_body(cx<T>* data, const cx<T>* __restrict__ Yf,
                                         const cx<T>* __restrict__ Yfn,
                                         const T* __restrict__ H2, const T* __restrict__ H2nyq,
                                         T rhoQ, T scale, int M, const cx<T>* __restrict__ tw,
                                         int twlog, double* __restrict__ partials, double inv_n,
                                         unsigned wg, unsigned nwg, unsigned ntiles, cx<T>* lds,
                                         cx<T>* twl, double* red) {
    constexpr int NTH = col_nth<T, NY, TC>();
    // the NY-point twiddle table lives in LDS when it is small: every stage
    // reads its twiddles there instead of from the global table
    constexpr bool TWL = col_twl<T, NY>();
    const unsigned wg_in = wg;
    const int t = threadIdx.x;
    // XCD-aware tile order.  Work-groups go to the 8 XCDs round-robin in
    // dispatch order, each XCD with its own L2.  Adjacent column tiles share
    // the 128-B lines of Z, Yf and |h|^2 (a tile row is TC * 8 B of Z, TC * 4 B
    // of |h|^2), so logical tiles 4j .. 4j+3 run as work-groups i, i+8, i+16,
    // i+24: on one XCD, in consecutive dispatch rounds.
    if ((nwg & 31u) == 0) {
        const unsigned r = wg >> 3, x = wg & 7u;
        wg = (r >> 2) * 32u + x * 4u + (r & 3u);
    }
    const int band = int(wg / ntiles);
    const int c0 = int(wg % ntiles) * TC;
    const long base = (long)band * NY * M;
    const int fsh = filt_shift<T>(NY, M);
    constexpr int NIT = (NY * TC + NTH - 1) / NTH;
    constexpr int NST = plan_nstages(NY);
    const int ntr = M - c0 < TC ? M - c0 : TC;      // columns of this tile inside the spectrum
    if constexpr (TWL) {
        for (int i = t; i < NY; i += NTH) twl[tw_at<COL_TWP>(i)] = tw[i << (twlog - ilog2c(NY))];
    }
    // Slot 0 of a spectrum row packs the kx = 0 and kx = nx/2 values of the
    // row transform (both real).  Transformed along y as one complex column,
    // the two would share its rounding: the error of the large kx = 0 column
    // (the image mean and its slow variations) would land on the kx = nx/2
    // column, whose filter gain 1 / (|h_hat|^2 + rho) is the largest of the
    // band.  In the solving modes the tile holding slot 0 therefore
    // transforms the real parts (kx = 0) with its other columns and the
    // imaginary parts (kx = nx/2) as a column of their own.
    constexpr bool FILT = MODE == COL_SOLVE || MODE == COL_FILTER;
    const bool dc = FILT && c0 == 0;
    // the data term and the filter of this thread's elements, loaded before
    // the forward transform so that their latency hides behind it (up to 8
    // elements per thread: more would cost the occupancy of wide tiles)
    constexpr int IPT = NIT;
    constexpr bool PRE = FILT && IPT <= 8;
    cx<T> yfp[MODE == COL_SOLVE && PRE ? IPT : 1];
    T gp[PRE ? IPT : 1];
    if constexpr (PRE) {
#pragma unroll
        for (int j = 0; j < IPT; ++j) {
            const int i = t + j * NTH;
            const int y = i / TC, c = i % TC, kx = c0 + c;
            gp[j] = T(0);
            if constexpr (MODE == COL_SOLVE) yfp[j] = {T(0), T(0)};
            if (i < NY * TC && kx < M) {
                const long g = base + filt_pos(NY, fsh, y, kx);
                if constexpr (MODE == COL_SOLVE) yfp[j] = stream_load(Yf + g);
                gp[j] = scale / (stream_load(H2 + g) + rhoQ);
            }
        }
    }
    // forward FFT along y; its first stage reads the tile straight from Z
    // (the barrier that ends it also publishes the twiddle table)
    fft_first_stage_global<T, NY, TC, NTH, 1, 0, true, false, false>(lds, data + base + c0, M, ntr, t, dc);
    if constexpr (TWL) fft_stage_range<T, NY, TC, NTH, 1, 0, true, false, false, 1, NST, COL_TWP>(lds, twl, ilog2c(NY), t);
    else fft_stage_range<T, NY, TC, NTH, 1, 0, true, false, false, 1, NST>(lds, tw, twlog, t);

    if constexpr (FILT) {
        // COL_FILTER: Q^{-1} alone (no data term), the adjoint's solve
#pragma unroll
        for (int j = 0; j < IPT; ++j) {
            const int i = t + j * NTH;
            const int y = i / TC, c = i % TC, kx = c0 + c;
            if (i >= NY * TC || kx >= M) continue;
            cx<T> v = lds[swz_pos<NY, TC>(y, c)];
            if constexpr (PRE) {
                if constexpr (MODE == COL_SOLVE) v = v + yfp[j];
                lds[swz_pos<NY, TC>(y, c)] = v * gp[j];
            } else {
                const long g = base + filt_pos(NY, fsh, y, kx);
                if constexpr (MODE == COL_SOLVE) v = v + stream_load(Yf + g);
                lds[swz_pos<NY, TC>(y, c)] = v * (scale / (stream_load(H2 + g) + rhoQ));
            }
        }
        __syncthreads();
        if (!dc) {
            // inverse FFT along y; its last stage writes the tile straight to Z
            if constexpr (TWL) {
                fft_stage_range<T, NY, TC, NTH, 1, 0, true, false, true, 0, NST - 1, COL_TWP>(lds, twl, ilog2c(NY), t);
                fft_last_stage_global<T, NY, TC, NTH, 1, 0, true, false, true, COL_TWP>(lds, twl, ilog2c(NY),
                                                                                       data + base + c0, M, ntr, t);
            } else {
                fft_stage_range<T, NY, TC, NTH, 1, 0, true, false, true, 0, NST - 1>(lds, tw, twlog, t);
                fft_last_stage_global<T, NY, TC, NTH, 1, 0, true, false, true>(lds, tw, twlog, data + base + c0, M,
                                                                              ntr, t);
            }
        } else {
            // the tile of slot 0: the whole inverse in LDS, the other columns
            // written out, the kx = 0 results kept in registers (element y of
            // the column by thread y mod NTH)
            if constexpr (TWL) fft_stage_range<T, NY, TC, NTH, 1, 0, true, false, true, 0, NST, COL_TWP>(lds, twl, ilog2c(NY), t);
            else fft_stage_range<T, NY, TC, NTH, 1, 0, true, false, true, 0, NST>(lds, tw, twlog, t);
            for (int i = t; i < NY * TC; i += NTH) {
                const int y = i / TC, c = i % TC;
                if (c > 0 && c < ntr) data[base + (long)y * M + c] = lds[swz_pos<NY, TC>(y, c)];
            }
            constexpr int NA = (NY + NTH - 1) / NTH;
            T a0[NA];
#pragma unroll
            for (int j = 0; j < NA; ++j) {
                const int y = t + j * NTH;
                a0[j] = y < NY ? lds[swz_pos<NY, TC>(y, 0)].x : T(0);
            }
            __syncthreads();
            // the kx = nx/2 column (imaginary parts of slot 0, still in Z):
            // forward FFT, data term and filter, inverse FFT, contiguous in LDS
            for (int y = t; y < NY; y += NTH) lds[y] = {data[base + (long)y * M].y, T(0)};
            __syncthreads();
            if constexpr (TWL) fft_stages<T, NY, 1, NTH, 0, 1, false, false, false, 0, COL_TWP>(lds, twl, ilog2c(NY), t);
            else fft_stages<T, NY, 1, NTH, 0, 1, false, false, false, 0>(lds, tw, twlog, t);
            for (int y = t; y < NY; y += NTH) {
                cx<T> v = lds[y];
                if constexpr (MODE == COL_SOLVE) v = v + Yfn[(long)band * NY + y];
                lds[y] = v * (scale / (H2nyq[(long)band * NY + y] + rhoQ));
            }
            __syncthreads();
            if constexpr (TWL) fft_stages<T, NY, 1, NTH, 0, 1, false, false, true, 0, COL_TWP>(lds, twl, ilog2c(NY), t);
            else fft_stages<T, NY, 1, NTH, 0, 1, false, false, true, 0>(lds, tw, twlog, t);
#pragma unroll
            for (int j = 0; j < NA; ++j) {
                const int y = t + j * NTH;
                if (y < NY) data[base + (long)y * M] = {a0[j], lds[y].x};
            }
        }
    }

    if constexpr (MODE == COL_CONV) {
        // multiplication by the transfer function h_hat (Yf holds it packed,
        // H2nyq its kx = nx/2 column as complex values), then the inverse FFT
        const cx<T>* Hh = Yf;
        const cx<T>* Hn = reinterpret_cast<const cx<T>*>(H2nyq);
#pragma unroll
        for (int j = 0; j < IPT; ++j) {
            const int i = t + j * NTH;
            const int y = i / TC, c = i % TC, kx = c0 + c;
            if (i >= NY * TC || kx == 0 || kx >= M) continue;
            const long g = base + filt_pos(NY, fsh, y, kx);
            lds[swz_pos<NY, TC>(y, c)] = cmul(lds[swz_pos<NY, TC>(y, c)], Hh[g]) * scale;
        }
        if (c0 == 0) {
            for (int ky = t; ky <= NY / 2; ky += NTH) {
                const int kn = (NY - ky) & (NY - 1);
                const cx<T> c1 = lds[swz_pos<NY, TC>(ky, 0)], c2 = lds[swz_pos<NY, TC>(kn, 0)];
                cx<T> A = {T(0.5) * (c1.x + c2.x), T(0.5) * (c1.y - c2.y)};
                cx<T> B = {T(0.5) * (c1.y + c2.y), T(-0.5) * (c1.x - c2.x)};
                A = cmul(A, Hh[base + filt_pos(NY, fsh, ky, 0)]) * scale;
                B = cmul(B, Hn[(long)band * NY + ky]) * scale;
                lds[swz_pos<NY, TC>(ky, 0)] = A + mul_i(B);
                if (kn != ky) lds[swz_pos<NY, TC>(kn, 0)] = conj(A) + mul_i(conj(B));
            }
        }
        __syncthreads();
        if constexpr (TWL) {
            fft_stage_range<T, NY, TC, NTH, 1, 0, true, false, true, 0, NST - 1, COL_TWP>(lds, twl, ilog2c(NY), t);
            fft_last_stage_global<T, NY, TC, NTH, 1, 0, true, false, true, COL_TWP>(lds, twl, ilog2c(NY),
                                                                                   data + base + c0, M, ntr, t);
        } else {
            fft_stage_range<T, NY, TC, NTH, 1, 0, true, false, true, 0, NST - 1>(lds, tw, twlog, t);
            fft_last_stage_global<T, NY, TC, NTH, 1, 0, true, false, true>(lds, tw, twlog, data + base + c0, M,
                                                                          ntr, t);
        }
    }

    if constexpr (MODE == COL_FWD) {
#pragma unroll
        for (int j = 0; j < NIT; ++j) {
            const int i = t + j * NTH;
            const int y = i / TC, c = i % TC;
            if (i < NY * TC && c0 + c < M) data[base + (long)y * M + c0 + c] = lds[swz_pos<NY, TC>(y, c)];
        }
    }

    if constexpr (MODE == COL_OBJ) {
        // sum over the full spectrum of |h|^2 |P|^2 - 2 Re(conj(Yf) P), from the half plane
        double acc = 0.0;
        for (int i = t; i < NY * TC; i += NTH) {
            const int y = i / TC, c = i % TC, kx = c0 + c;
            if (kx == 0 || kx >= M) continue;
            const long g = base + filt_pos(NY, fsh, y, kx);
            const cx<T> z = lds[swz_pos<NY, TC>(y, c)], f = Yf[g];
            const double zz = double(z.x) * z.x + double(z.y) * z.y;
            const double cr = double(f.x) * z.x + double(f.y) * z.y;
            acc += 2.0 * (double(H2[g]) * zz - 2.0 * cr);
        }
        if (c0 == 0) {
            for (int ky = t; ky <= NY / 2; ky += NTH) {
                const int kn = (NY - ky) & (NY - 1);
                const long g1 = base + filt_pos(NY, fsh, ky, 0);
                const cx<T> c1 = lds[swz_pos<NY, TC>(ky, 0)], c2 = lds[swz_pos<NY, TC>(kn, 0)];
                const cx<T> A = {T(0.5) * (c1.x + c2.x), T(0.5) * (c1.y - c2.y)};
                const cx<T> B = {T(0.5) * (c1.y + c2.y), T(-0.5) * (c1.x - c2.x)};
                // the data terms of the kx = 0 and kx = nx/2 columns, stored apart
                const cx<T> FA = Yf[g1], FB = Yfn[(long)band * NY + ky];
                const double wgt = (kn == ky) ? 1.0 : 2.0;
                const double a2 = double(A.x) * A.x + double(A.y) * A.y;
                const double b2 = double(B.x) * B.x + double(B.y) * B.y;
                const double ar = double(FA.x) * A.x + double(FA.y) * A.y;
                const double br = double(FB.x) * B.x + double(FB.y) * B.y;
                acc += wgt * (double(H2[g1]) * a2 - 2.0 * ar
                              + double(H2nyq[(long)band * NY + ky]) * b2 - 2.0 * br);
            }
        }
        const double s = block_sum<NTH>(acc * inv_n, red);
        if (t == 0) partials[wg_in] = s;
    }
}

template <typename T, int NY, int MODE, int V>
__global__ void __launch_bounds__((col_nth<T, NY, col_tc<T, NY, V>()>()))
k_col(cx<T>* data, const cx<T>* __restrict__ Yf, const cx<T>* __restrict__ Yfn, const T* __restrict__ H2,
      const T* __restrict__ H2nyq, T rhoQ, T scale, int M, const cx<T>* __restrict__ tw,
      int twlog, double* __restrict__ partials, double inv_n) {
    constexpr int TC = col_tc<T, NY, V>();
    __shared__ cx<T> lds[NY * TC];
    __shared__ cx<T> twl[col_twl<T, NY>() ? col_twl_len<NY>() : 1];
    __shared__ double red[col_nth<T, NY, TC>() / 64];
    col_body<T, NY, MODE, TC>(data, Yf, Yfn, H2, H2nyq, rhoQ, scale, M, tw, twlog, partials, inv_n,
                              blockIdx.x + blockIdx.y * gridDim.x, gridDim.x * gridDim.y, gridDim.x,
                              lds, twl, red);
}

// the solving column pass over the tiles of several cubes of one ny; each
// cube's block range starts at a multiple of 32 (the tile order above)
template <typename T, int NY, int V>
__global__ void __launch_bounds__((col_nth<T, NY, col_tc<T, NY, V>()>()))
k_col_group(const ColDesc* __restrict__ d, int n) {
    constexpr int TC = col_tc<T, NY, V>();
    __shared__ cx<T> lds[NY * TC];
    __shared__ cx<T> twl[col_twl<T, NY>() ? col_twl_len<NY>() : 1];
    __shared__ double red[col_nth<T, NY, TC>() / 64];
    const int j = group_find(d, n, blockIdx.x);
    if (j < 0) return;
    const int M = d[j].M;
    const unsigned ntiles = (unsigned)((M + TC - 1) / TC);
    col_body<T, NY, COL_SOLVE, TC>((cx<T>*)d[j].data, (const cx<T>*)d[j].Yf, (const cx<T>*)d[j].Yfn,
                                   (const T*)d[j].H2,
                                   (const T*)d[j].H2nyq, T(d[j].rhoQ), T(d[j].scale), M,
                                   (const cx<T>*)d[j].tw, d[j].twlog, nullptr, 0.0,
                                   blockIdx.x - (unsigned)d[j].first, (unsigned)d[j].nblk, ntiles,
                                   lds, twl, red);
}

// ------------------------------------------------------------------ setup combine
template <typename T>
__global__ void __launch_bounds__(256)
k_setup_combine(const cx<double>* __restrict__ Ch, const cx<double>* __restrict__ Cy,
                cx<T>* __restrict__ Yf, cx<T>* __restrict__ Yfnyq, T* __restrict__ H2, T* __restrict__ H2nyq,
                cx<T>* __restrict__ Hh, cx<T>* __restrict__ Hhnyq, int L, int ny, int M) {
    // Ch, Cy in spectrum order [L][ny][M]; Yf, H2 written in column-block order
    const long n = (long)L * ny * M;
    const int fsh = filt_shift<T>(ny, M);
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
        const long band = i / ((long)ny * M);
        const long rem = i - band * ny * M;
        const int ky = int(rem / M), kx = int(rem % M);
        const long o = band * ny * M + filt_pos(ny, fsh, ky, kx);
        if (kx != 0) {
            const cx<double> h = Ch[i], y = Cy[i];
            const cx<double> f = {h.x * y.x + h.y * y.y, h.x * y.y - h.y * y.x};   // conj(h) y
            Yf[o] = {T(f.x), T(f.y)};
            H2[o] = T(h.x * h.x + h.y * h.y);
            Hh[o] = {T(h.x), T(h.y)};
        } else if (ky <= ny / 2) {
            const int kn = (ny - ky) & (ny - 1);
            const long i2 = band * ny * M + (long)kn * M;
            const long o2 = band * ny * M + filt_pos(ny, fsh, kn, 0);
            const cx<double> h1 = Ch[i], h2 = Ch[i2], y1 = Cy[i], y2 = Cy[i2];
            const cx<double> Ah = {0.5 * (h1.x + h2.x), 0.5 * (h1.y - h2.y)};
            const cx<double> Bh = {0.5 * (h1.y + h2.y), -0.5 * (h1.x - h2.x)};
            const cx<double> Ay = {0.5 * (y1.x + y2.x), 0.5 * (y1.y - y2.y)};
            const cx<double> By = {0.5 * (y1.y + y2.y), -0.5 * (y1.x - y2.x)};
            const cx<double> FA = {Ah.x * Ay.x + Ah.y * Ay.y, Ah.x * Ay.y - Ah.y * Ay.x};
            const cx<double> FB = {Bh.x * By.x + Bh.y * By.y, Bh.x * By.y - Bh.y * By.x};
            // the data terms of the two columns stored apart (each Hermitian
            // in ky): kx = 0 in slot 0, kx = nx/2 in its own column.  Packed
            // into one complex value, the rounding of the large kx = 0 term
            // would fall on the small kx = nx/2 one.
            Yf[o] = {T(FA.x), T(FA.y)};
            Yf[o2] = {T(FA.x), T(-FA.y)};
            Yfnyq[band * ny + ky] = {T(FB.x), T(FB.y)};
            Yfnyq[band * ny + kn] = {T(FB.x), T(-FB.y)};
            const T a2 = T(Ah.x * Ah.x + Ah.y * Ah.y), b2 = T(Bh.x * Bh.x + Bh.y * Bh.y);
            H2[o] = a2;
            H2[o2] = a2;
            H2nyq[band * ny + ky] = b2;
            H2nyq[band * ny + kn] = b2;
            // the transfer functions of the kx = 0 and kx = nx/2 columns
            // (each Hermitian in ky)
            Hh[o] = {T(Ah.x), T(Ah.y)};
            Hh[o2] = {T(Ah.x), T(-Ah.y)};
            Hhnyq[band * ny + ky] = {T(Bh.x), T(Bh.y)};
            Hhnyq[band * ny + kn] = {T(Bh.x), T(-Bh.y)};
        }
    }
}

// ------------------------------------------------------------------ launchers
#define MUFFIN_POW2_CASES(F) F(8) F(16) F(32) F(64) F(128) F(256) F(512) F(1024) F(2048) F(4096)
// runtime variant -> template argument V
#define MUFFIN_VARIANT(v, CALL)            \
    switch (v) {                           \
        case 0: { constexpr int V = 0; CALL; } \
        case 1: { constexpr int V = 1; CALL; } \
        case 2: { constexpr int V = 2; CALL; } \
        default: return hipErrorInvalidValue;  \
    }

template <int V> static int row_rpw_rt(int nx) {
    switch (nx) {
#define F(N) case N: return row_rpw<N / 2, V>();
        MUFFIN_POW2_CASES(F)
#undef F
    }
    return 1;
}

int row_blocks(int nrows, int nx, int variant) {
    const int rpw = variant == 0 ? row_rpw_rt<0>(nx) : (variant == 2 ? row_rpw_rt<2>(nx) : row_rpw_rt<1>(nx));
    return (nrows + rpw - 1) / rpw;
}

template <typename Tin, typename T, bool SHIFT, bool POS, int V>
static hipError_t row_fwd_t(const void* in, void* out, int nrows, int nx, int ny, const void* tw,
                            int twlog, hipStream_t s) {
    switch (nx) {
#define F(N)                                                                                 \
    case N: {                                                                                \
        constexpr int RPW = row_rpw<N / 2, V>();                                             \
        dim3 grid((nrows + RPW - 1) / RPW);                                                  \
        hipLaunchKernelGGL((k_row_fwd<Tin, T, N, SHIFT, POS, V>), grid, dim3(ROW_NTH), 0, s, \
                           (const Tin*)in, (cx<T>*)out, nrows, ny, (const cx<T>*)tw, twlog); \
        return hipGetLastError();                                                            \
    }
        MUFFIN_POW2_CASES(F)
#undef F
    }
    return hipErrorInvalidValue;
}

hipError_t launch_row_fwd(int dtype, bool in_f64, const void* in, void* out, int nrows, int nx,
                          int ny, bool shift, bool positive, const void* tw, int twlog,
                          hipStream_t s, int variant) {
    if (nrows <= 0) return hipSuccess;
    const bool plain = !shift && !positive;
    if (dtype == 0) {       // float output
        if (in_f64 || shift) return hipErrorInvalidValue;
        if (positive) return row_fwd_t<float, float, false, true, 1>(in, out, nrows, nx, ny, tw, twlog, s);
        MUFFIN_VARIANT(variant, return (row_fwd_t<float, float, false, false, V>(in, out, nrows, nx, ny, tw, twlog, s)))
    }
    // double output
    if (in_f64) {
        if (positive) return row_fwd_t<double, double, false, true, 1>(in, out, nrows, nx, ny, tw, twlog, s);
        if (shift) return row_fwd_t<double, double, true, false, 1>(in, out, nrows, nx, ny, tw, twlog, s);
        if (plain) {
            MUFFIN_VARIANT(variant, return (row_fwd_t<double, double, false, false, V>(in, out, nrows, nx, ny, tw, twlog, s)))
        }
    }
    if (positive) return hipErrorInvalidValue;
    if (shift) return row_fwd_t<float, double, true, false, 1>(in, out, nrows, nx, ny, tw, twlog, s);
    return row_fwd_t<float, double, false, false, 1>(in, out, nrows, nx, ny, tw, twlog, s);
}

template <typename T, int V>
static hipError_t row_inv_t(const void* in, void* out, int nrows, int nx, const void* tw, int twlog,
                            hipStream_t s) {
    switch (nx) {
#define F(N)                                                                            \
    case N: {                                                                           \
        constexpr int RPW = row_rpw<N / 2, V>();                                        \
        dim3 grid((nrows + RPW - 1) / RPW);                                             \
        hipLaunchKernelGGL((k_row_inv<T, N, V>), grid, dim3(ROW_NTH), 0, s,             \
                           (const cx<T>*)in, (T*)out, nrows, (const cx<T>*)tw, twlog);  \
        return hipGetLastError();                                                       \
    }
        MUFFIN_POW2_CASES(F)
#undef F
    }
    return hipErrorInvalidValue;
}

hipError_t launch_row_inv(int dtype, const void* in, void* out, int nrows, int nx, const void* tw,
                          int twlog, hipStream_t s, int variant) {
    if (nrows <= 0) return hipSuccess;
    if (dtype == 0) {
        MUFFIN_VARIANT(variant, return (row_inv_t<float, V>(in, out, nrows, nx, tw, twlog, s)))
    }
    MUFFIN_VARIANT(variant, return (row_inv_t<double, V>(in, out, nrows, nx, tw, twlog, s)))
}

template <typename T, int V> static int col_tc_rt(int ny) {
    switch (ny) {
#define F(N) case N: return col_tc<T, N, V>();
        MUFFIN_POW2_CASES(F)
#undef F
    }
    return 1;
}

int col_blocks(int dtype, int L, int ny, int nx, int variant) {
    int tc = 1;
    if (dtype == 0) tc = variant == 0 ? col_tc_rt<float, 0>(ny) : (variant == 2 ? col_tc_rt<float, 2>(ny) : col_tc_rt<float, 1>(ny));
    else tc = variant == 0 ? col_tc_rt<double, 0>(ny) : (variant == 2 ? col_tc_rt<double, 2>(ny) : col_tc_rt<double, 1>(ny));
    const int M = nx / 2;
    return ((M + tc - 1) / tc) * L;
}

template <typename T, int MODE, int V>
static hipError_t col_t(void* data, const void* Yf, const void* Yfn, const void* H2, const void* H2nyq,
                        double rhoQ, double scale, int L, int ny, int nx, const void* tw, int twlog,
                        double* partials, int* nblocks_out, hipStream_t s) {
    const int M = nx / 2;
    switch (ny) {
#define F(N)                                                                                  \
    case N: {                                                                                 \
        constexpr int TC = col_tc<T, N, V>();                                                 \
        dim3 grid((M + TC - 1) / TC, L);                                                      \
        if (nblocks_out) *nblocks_out = int(grid.x * grid.y);                                 \
        hipLaunchKernelGGL((k_col<T, N, MODE, V>), grid, dim3(col_nth<T, N, TC>()), 0, s,     \
                           (cx<T>*)data, (const cx<T>*)Yf, (const cx<T>*)Yfn, (const T*)H2,   \
                           (const T*)H2nyq,                                                   \
                           T(rhoQ), T(scale), M, (const cx<T>*)tw, twlog, partials,           \
                           1.0 / (double(nx) * double(ny)));                                  \
        return hipGetLastError();                                                             \
    }
        MUFFIN_POW2_CASES(F)
#undef F
    }
    return hipErrorInvalidValue;
}

hipError_t launch_col(int dtype, int mode, void* data, const void* Yf, const void* Yfnyq, const void* H2,
                      const void* H2nyq, double rhoQ, double scale, int L, int ny, int nx,
                      const void* tw, int twlog, double* partials, int* nblocks_out,
                      hipStream_t s, int variant) {
    constexpr int D = kDefaultColVariant;
    if (dtype == 0) {
        if (mode == COL_SOLVE) {
            MUFFIN_VARIANT(variant, return (col_t<float, COL_SOLVE, V>(data, Yf, Yfnyq, H2, H2nyq, rhoQ, scale, L, ny, nx, tw, twlog, partials, nblocks_out, s)))
        }
        if (mode == COL_OBJ)
            return col_t<float, COL_OBJ, D>(data, Yf, Yfnyq, H2, H2nyq, rhoQ, scale, L, ny, nx, tw, twlog, partials, nblocks_out, s);
        if (mode == COL_FILTER)
            return col_t<float, COL_FILTER, D>(data, Yf, Yfnyq, H2, H2nyq, rhoQ, scale, L, ny, nx, tw, twlog, partials, nblocks_out, s);
        if (mode == COL_CONV)
            return col_t<float, COL_CONV, D>(data, Yf, Yfnyq, H2, H2nyq, rhoQ, scale, L, ny, nx, tw, twlog, partials, nblocks_out, s);
        return hipErrorInvalidValue;
    }
    if (mode == COL_FILTER)
        return col_t<double, COL_FILTER, D>(data, Yf, Yfnyq, H2, H2nyq, rhoQ, scale, L, ny, nx, tw, twlog, partials, nblocks_out, s);
    if (mode == COL_CONV)
        return col_t<double, COL_CONV, D>(data, Yf, Yfnyq, H2, H2nyq, rhoQ, scale, L, ny, nx, tw, twlog, partials, nblocks_out, s);
    if (mode == COL_SOLVE) {
        MUFFIN_VARIANT(variant, return (col_t<double, COL_SOLVE, V>(data, Yf, Yfnyq, H2, H2nyq, rhoQ, scale, L, ny, nx, tw, twlog, partials, nblocks_out, s)))
    }
    if (mode == COL_FWD)
        return col_t<double, COL_FWD, D>(data, Yf, Yfnyq, H2, H2nyq, rhoQ, scale, L, ny, nx, tw, twlog, partials, nblocks_out, s);
    return col_t<double, COL_OBJ, D>(data, Yf, Yfnyq, H2, H2nyq, rhoQ, scale, L, ny, nx, tw, twlog, partials, nblocks_out, s);
}

// ------------------------------------------------------------------ grouped launchers
template <typename T, int V>
static hipError_t row_group_t(bool inv, int nx, const RowDesc* d, int n, int nblocks, hipStream_t s) {
    switch (nx) {
#define F(N)                                                                                     \
    case N:                                                                                      \
        if (inv) hipLaunchKernelGGL((k_row_inv_group<T, N, V>), dim3(nblocks), dim3(ROW_NTH), 0, s, d, n); \
        else hipLaunchKernelGGL((k_row_fwd_group<T, N, V>), dim3(nblocks), dim3(ROW_NTH), 0, s, d, n);     \
        return hipGetLastError();
        MUFFIN_POW2_CASES(F)
#undef F
    }
    return hipErrorInvalidValue;
}

hipError_t launch_row_fwd_group(int dtype, int nx, int variant, const RowDesc* d, int n, int nblocks,
                                hipStream_t s) {
    if (n <= 0 || nblocks <= 0) return hipSuccess;
    if (dtype == 0) { MUFFIN_VARIANT(variant, return (row_group_t<float, V>(false, nx, d, n, nblocks, s))) }
    MUFFIN_VARIANT(variant, return (row_group_t<double, V>(false, nx, d, n, nblocks, s)))
}

hipError_t launch_row_inv_group(int dtype, int nx, int variant, const RowDesc* d, int n, int nblocks,
                                hipStream_t s) {
    if (n <= 0 || nblocks <= 0) return hipSuccess;
    if (dtype == 0) { MUFFIN_VARIANT(variant, return (row_group_t<float, V>(true, nx, d, n, nblocks, s))) }
    MUFFIN_VARIANT(variant, return (row_group_t<double, V>(true, nx, d, n, nblocks, s)))
}

template <typename T, int V>
static hipError_t col_group_t(int ny, const ColDesc* d, int n, int nblocks, hipStream_t s) {
    switch (ny) {
#define F(N)                                                                                       \
    case N:                                                                                        \
        hipLaunchKernelGGL((k_col_group<T, N, V>), dim3(nblocks), dim3(col_nth<T, N, col_tc<T, N, V>()>()), \
                           0, s, d, n);                                                            \
        return hipGetLastError();
        MUFFIN_POW2_CASES(F)
#undef F
    }
    return hipErrorInvalidValue;
}

hipError_t launch_col_group(int dtype, int ny, int variant, const ColDesc* d, int n, int nblocks,
                            hipStream_t s) {
    if (n <= 0 || nblocks <= 0) return hipSuccess;
    if (dtype == 0) { MUFFIN_VARIANT(variant, return (col_group_t<float, V>(ny, d, n, nblocks, s))) }
    MUFFIN_VARIANT(variant, return (col_group_t<double, V>(ny, d, n, nblocks, s)))
}

hipError_t launch_setup_combine(int dtype, const void* Ch, const void* Cy, void* Yf, void* Yfnyq, void* H2,
                                void* H2nyq, void* Hh, void* Hhnyq, int L, int ny, int nx, hipStream_t s) {
    const int M = nx / 2;
    const long n = (long)L * ny * M;
    const int blocks = int((n + 255) / 256 < 65536 ? (n + 255) / 256 : 65536);
    if (dtype == 0)
        hipLaunchKernelGGL((k_setup_combine<float>), dim3(blocks), dim3(256), 0, s,
                           (const cx<double>*)Ch, (const cx<double>*)Cy, (cx<float>*)Yf, (cx<float>*)Yfnyq,
                           (float*)H2, (float*)H2nyq, (cx<float>*)Hh, (cx<float>*)Hhnyq, L, ny, M);
    else
        hipLaunchKernelGGL((k_setup_combine<double>), dim3(blocks), dim3(256), 0, s,
                           (const cx<double>*)Ch, (const cx<double>*)Cy, (cx<double>*)Yf, (cx<double>*)Yfnyq,
                           (double*)H2, (double*)H2nyq, (cx<double>*)Hh, (cx<double>*)Hhnyq, L, ny, M);
    return hipGetLastError();
}

}  // namespace muffin
