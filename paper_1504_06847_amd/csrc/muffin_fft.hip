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

// rows per block: about 2048 complex points per block
template <int M> constexpr int row_rpw() { return M >= 2048 ? 1 : 2048 / M; }

template <typename T, int NY> constexpr int col_tc() {
    int tc = int(65536 / (NY * int(sizeof(cx<T>))));
    return tc > 16 ? 16 : (tc < 1 ? 1 : tc);
}
template <typename T, int NY> constexpr int col_nth() {
    int n = col_tc<T, NY>() * NY / 8;
    return n > 512 ? 512 : (n < 64 ? 64 : n);
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

// ------------------------------------------------------------------ row passes
template <typename Tin, typename T, int NX, bool SHIFT, bool POS>
__global__ void __launch_bounds__(ROW_NTH)
k_row_fwd(const Tin* __restrict__ in, cx<T>* __restrict__ out, int nrows, int ny,
          const cx<T>* __restrict__ tw, int twlog) {
    constexpr int M = NX / 2;
    constexpr int RPW = row_rpw<M>();
    constexpr int TS = lds_len<true>(M);
    __shared__ cx<T> lds[RPW * TS];
    const int t = threadIdx.x;
    const long row0 = (long)blockIdx.x * RPW;
    for (int i = t; i < RPW * M; i += ROW_NTH) {
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
    for (int i = t; i < RPW * NK; i += ROW_NTH) {
        const int r = i / NK, k = i % NK;
        const long grow = row0 + r;
        if (grow >= nrows) continue;
        cx<T>* o = out + grow * M;
        const cx<T> zk = lds[r * TS + lds_pos<true>(k)];
        if (k == 0) {
            o[0] = {zk.x + zk.y, zk.x - zk.y};           // (X_0, X_{nx/2}), both real
        } else if (k == M / 2) {
            o[k] = conj(zk);
        } else {
            const cx<T> zm = lds[r * TS + lds_pos<true>(M - k)];
            // even/odd sample spectra E = (Z_k + conj Z_{M-k})/2, O = -i (Z_k - conj Z_{M-k})/2
            const cx<T> e = {T(0.5) * (zk.x + zm.x), T(0.5) * (zk.y - zm.y)};
            const cx<T> od = {T(0.5) * (zk.y + zm.y), T(-0.5) * (zk.x - zm.x)};
            const cx<T> wo = cmul(od, tw[k << (twlog - ilog2c(NX))]);
            o[k] = e + wo;                                // X_k = E + w^k O
            o[M - k] = conj(e - wo);                      // X_{M-k} = conj(E - w^k O)
        }
    }
}

template <typename T, int NX>
__global__ void __launch_bounds__(ROW_NTH)
k_row_inv(const cx<T>* __restrict__ in, T* __restrict__ out, int nrows,
          const cx<T>* __restrict__ tw, int twlog) {
    constexpr int M = NX / 2;
    constexpr int RPW = row_rpw<M>();
    constexpr int TS = lds_len<true>(M);
    __shared__ cx<T> lds[RPW * TS];
    const int t = threadIdx.x;
    const long row0 = (long)blockIdx.x * RPW;
    constexpr int NK = M / 2 + 1;
    for (int i = t; i < RPW * NK; i += ROW_NTH) {
        const int r = i / NK, k = i % NK;
        const long grow = row0 + r;
        cx<T>* l = lds + r * TS;
        if (grow >= nrows) continue;
        const cx<T>* p = in + grow * M;
        const cx<T> xk = p[k];
        if (k == 0) {
            l[0] = {T(0.5) * (xk.x + xk.y), T(0.5) * (xk.x - xk.y)};
        } else if (k == M / 2) {
            l[lds_pos<true>(k)] = conj(xk);
        } else {
            const cx<T> xm = p[M - k];
            const cx<T> e = {T(0.5) * (xk.x + xm.x), T(0.5) * (xk.y - xm.y)};
            const cx<T> d = {T(0.5) * (xk.x - xm.x), T(0.5) * (xk.y + xm.y)};
            const cx<T> o = cmulc(d, tw[k << (twlog - ilog2c(NX))]);   // O = w^{-k} D
            l[lds_pos<true>(k)] = e + mul_i(o);                         // Z_k = E + i O
            l[lds_pos<true>(M - k)] = conj(e) + mul_i(conj(o));
        }
    }
    __syncthreads();
    tile_fft<T, M, RPW, ROW_NTH, TS, 1, false, true, true>(lds, tw, twlog, t);
    for (int i = t; i < RPW * M; i += ROW_NTH) {
        const int r = i / M, m = i % M;
        const long grow = row0 + r;
        if (grow < nrows) reinterpret_cast<cx<T>*>(out + grow * NX)[m] = lds[r * TS + lds_pos<true>(m)];
    }
}

// ------------------------------------------------------------------ column pass
template <typename T, int NY, int MODE>
__global__ void __launch_bounds__((col_nth<T, NY>()))
k_col(cx<T>* data, const cx<T>* __restrict__ Yf, const T* __restrict__ H2,
      const T* __restrict__ H2nyq, T rhoQ, T scale, int M, const cx<T>* __restrict__ tw,
      int twlog, double* __restrict__ partials, double inv_n) {
    constexpr int TC = col_tc<T, NY>();
    constexpr int NTH = col_nth<T, NY>();
    constexpr int TCP = TC + 1;          // padded row stride: spreads stride-R writes over the banks
    // the NY-point twiddle table lives in LDS when it is small: every stage
    // reads its twiddles there instead of from the global table
    constexpr bool TWL = NY * int(sizeof(cx<T>)) <= 16384;
    __shared__ cx<T> lds[NY * TCP];
    __shared__ cx<T> twl[TWL ? NY : 1];
    __shared__ double red[NTH / 64];
    const int t = threadIdx.x;
    // XCD-aware tile order.  Work-groups go to the 8 XCDs round-robin in
    // dispatch order, each XCD with its own L2.  Adjacent column tiles share
    // the 128-B lines of Z, Yf and |h|^2 (a tile row is TC * 8 B of Z, TC * 4 B
    // of |h|^2), so logical tiles 4j .. 4j+3 run as work-groups i, i+8, i+16,
    // i+24: on one XCD, in consecutive dispatch rounds.
    const unsigned ntiles = gridDim.x, nwg = gridDim.x * gridDim.y;
    unsigned wg = blockIdx.x + blockIdx.y * gridDim.x;
    if ((nwg & 31u) == 0) {
        const unsigned r = wg >> 3, x = wg & 7u;
        wg = (r >> 2) * 32u + x * 4u + (r & 3u);
    }
    const int band = int(wg / ntiles);
    const int c0 = int(wg % ntiles) * TC;
    const long base = (long)band * NY * M;
    for (int i = t; i < NY * TC; i += NTH) {
        const int y = i / TC, c = i % TC;
        cx<T> v = {T(0), T(0)};
        if (c0 + c < M) v = data[base + (long)y * M + c0 + c];
        lds[y * TCP + c] = v;
    }
    if constexpr (TWL) {
        for (int i = t; i < NY; i += NTH) twl[i] = tw[i << (twlog - ilog2c(NY))];
    }
    __syncthreads();
    if constexpr (TWL) tile_fft<T, NY, TC, NTH, 1, TCP, true, false, false>(lds, twl, ilog2c(NY), t);
    else tile_fft<T, NY, TC, NTH, 1, TCP, true, false, false>(lds, tw, twlog, t);

    if constexpr (MODE == COL_SOLVE) {
        for (int i = t; i < NY * TC; i += NTH) {
            const int y = i / TC, c = i % TC, kx = c0 + c;
            if (kx == 0 || kx >= M) continue;
            const long g = base + (long)y * M + kx;
            const cx<T> v = lds[y * TCP + c] + Yf[g];
            lds[y * TCP + c] = v * (scale / (H2[g] + rhoQ));
        }
        if (c0 == 0) {
            // slot 0 packs the real columns kx = 0 (A) and kx = nx/2 (B): C = A + i B
            for (int ky = t; ky <= NY / 2; ky += NTH) {
                const int kn = (NY - ky) & (NY - 1);
                const long g1 = base + (long)ky * M, g2 = base + (long)kn * M;
                const cx<T> c1 = lds[ky * TCP] + Yf[g1];
                const cx<T> c2 = lds[kn * TCP] + Yf[g2];
                const T g0 = scale / (H2[g1] + rhoQ);
                const T gm = scale / (H2nyq[(long)band * NY + ky] + rhoQ);
                cx<T> A = {T(0.5) * (c1.x + c2.x), T(0.5) * (c1.y - c2.y)};
                cx<T> B = {T(0.5) * (c1.y + c2.y), T(-0.5) * (c1.x - c2.x)};
                A = A * g0;
                B = B * gm;
                lds[ky * TCP] = A + mul_i(B);
                if (kn != ky) lds[kn * TCP] = conj(A) + mul_i(conj(B));
            }
        }
        __syncthreads();
        if constexpr (TWL) tile_fft<T, NY, TC, NTH, 1, TCP, true, false, true>(lds, twl, ilog2c(NY), t);
        else tile_fft<T, NY, TC, NTH, 1, TCP, true, false, true>(lds, tw, twlog, t);
    }

    if constexpr (MODE == COL_SOLVE || MODE == COL_FWD) {
        for (int i = t; i < NY * TC; i += NTH) {
            const int y = i / TC, c = i % TC;
            if (c0 + c < M) data[base + (long)y * M + c0 + c] = lds[y * TCP + c];
        }
    }

    if constexpr (MODE == COL_OBJ) {
        // sum over the full spectrum of |h|^2 |P|^2 - 2 Re(conj(Yf) P), from the half plane
        double acc = 0.0;
        for (int i = t; i < NY * TC; i += NTH) {
            const int y = i / TC, c = i % TC, kx = c0 + c;
            if (kx == 0 || kx >= M) continue;
            const long g = base + (long)y * M + kx;
            const cx<T> z = lds[y * TCP + c], f = Yf[g];
            const double zz = double(z.x) * z.x + double(z.y) * z.y;
            const double cr = double(f.x) * z.x + double(f.y) * z.y;
            acc += 2.0 * (double(H2[g]) * zz - 2.0 * cr);
        }
        if (c0 == 0) {
            for (int ky = t; ky <= NY / 2; ky += NTH) {
                const int kn = (NY - ky) & (NY - 1);
                const long g1 = base + (long)ky * M, g2 = base + (long)kn * M;
                const cx<T> c1 = lds[ky * TCP], c2 = lds[kn * TCP];
                const cx<T> f1 = Yf[g1], f2 = Yf[g2];
                const cx<T> A = {T(0.5) * (c1.x + c2.x), T(0.5) * (c1.y - c2.y)};
                const cx<T> B = {T(0.5) * (c1.y + c2.y), T(-0.5) * (c1.x - c2.x)};
                const cx<T> FA = {T(0.5) * (f1.x + f2.x), T(0.5) * (f1.y - f2.y)};
                const cx<T> FB = {T(0.5) * (f1.y + f2.y), T(-0.5) * (f1.x - f2.x)};
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
        if (t == 0) partials[(long)blockIdx.y * gridDim.x + blockIdx.x] = s;
    }
}

// ------------------------------------------------------------------ setup combine
template <typename T>
__global__ void __launch_bounds__(256)
k_setup_combine(const cx<double>* __restrict__ Ch, const cx<double>* __restrict__ Cy,
                cx<T>* __restrict__ Yf, T* __restrict__ H2, T* __restrict__ H2nyq, int L,
                int ny, int M) {
    const long n = (long)L * ny * M;
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
        const long band = i / ((long)ny * M);
        const long rem = i - band * ny * M;
        const int ky = int(rem / M), kx = int(rem % M);
        if (kx != 0) {
            const cx<double> h = Ch[i], y = Cy[i];
            const cx<double> f = {h.x * y.x + h.y * y.y, h.x * y.y - h.y * y.x};   // conj(h) y
            Yf[i] = {T(f.x), T(f.y)};
            H2[i] = T(h.x * h.x + h.y * h.y);
        } else if (ky <= ny / 2) {
            const int kn = (ny - ky) & (ny - 1);
            const long i2 = band * ny * M + (long)kn * M;
            const cx<double> h1 = Ch[i], h2 = Ch[i2], y1 = Cy[i], y2 = Cy[i2];
            const cx<double> Ah = {0.5 * (h1.x + h2.x), 0.5 * (h1.y - h2.y)};
            const cx<double> Bh = {0.5 * (h1.y + h2.y), -0.5 * (h1.x - h2.x)};
            const cx<double> Ay = {0.5 * (y1.x + y2.x), 0.5 * (y1.y - y2.y)};
            const cx<double> By = {0.5 * (y1.y + y2.y), -0.5 * (y1.x - y2.x)};
            const cx<double> FA = {Ah.x * Ay.x + Ah.y * Ay.y, Ah.x * Ay.y - Ah.y * Ay.x};
            const cx<double> FB = {Bh.x * By.x + Bh.y * By.y, Bh.x * By.y - Bh.y * By.x};
            // packed: FA + i FB at ky, conj(FA) + i conj(FB) at -ky
            Yf[i] = {T(FA.x - FB.y), T(FA.y + FB.x)};
            Yf[i2] = {T(FA.x + FB.y), T(FB.x - FA.y)};
            const T a2 = T(Ah.x * Ah.x + Ah.y * Ah.y), b2 = T(Bh.x * Bh.x + Bh.y * Bh.y);
            H2[i] = a2;
            H2[i2] = a2;
            H2nyq[band * ny + ky] = b2;
            H2nyq[band * ny + kn] = b2;
        }
    }
}

// ------------------------------------------------------------------ launchers
#define MUFFIN_POW2_CASES(F) F(8) F(16) F(32) F(64) F(128) F(256) F(512) F(1024) F(2048) F(4096)

template <typename Tin, typename T, bool SHIFT, bool POS>
static hipError_t row_fwd_t(const void* in, void* out, int nrows, int nx, int ny, const void* tw,
                            int twlog, hipStream_t s) {
    switch (nx) {
#define F(N)                                                                              \
    case N: {                                                                             \
        constexpr int RPW = row_rpw<N / 2>();                                             \
        dim3 grid((nrows + RPW - 1) / RPW);                                               \
        hipLaunchKernelGGL((k_row_fwd<Tin, T, N, SHIFT, POS>), grid, dim3(ROW_NTH), 0, s, \
                           (const Tin*)in, (cx<T>*)out, nrows, ny, (const cx<T>*)tw, twlog); \
        return hipGetLastError();                                                         \
    }
        MUFFIN_POW2_CASES(F)
#undef F
    }
    return hipErrorInvalidValue;
}

hipError_t launch_row_fwd(int dtype, bool in_f64, const void* in, void* out, int nrows, int nx,
                          int ny, bool shift, bool positive, const void* tw, int twlog,
                          hipStream_t s) {
    if (nrows <= 0) return hipSuccess;
    if (dtype == 0) {       // float output
        if (in_f64) return hipErrorInvalidValue;
        if (positive) return row_fwd_t<float, float, false, true>(in, out, nrows, nx, ny, tw, twlog, s);
        if (shift) return hipErrorInvalidValue;
        return row_fwd_t<float, float, false, false>(in, out, nrows, nx, ny, tw, twlog, s);
    }
    // double output
    if (in_f64) {
        if (positive) return row_fwd_t<double, double, false, true>(in, out, nrows, nx, ny, tw, twlog, s);
        if (shift) return row_fwd_t<double, double, true, false>(in, out, nrows, nx, ny, tw, twlog, s);
        return row_fwd_t<double, double, false, false>(in, out, nrows, nx, ny, tw, twlog, s);
    }
    if (positive) return hipErrorInvalidValue;
    if (shift) return row_fwd_t<float, double, true, false>(in, out, nrows, nx, ny, tw, twlog, s);
    return row_fwd_t<float, double, false, false>(in, out, nrows, nx, ny, tw, twlog, s);
}

template <typename T>
static hipError_t row_inv_t(const void* in, void* out, int nrows, int nx, const void* tw, int twlog,
                            hipStream_t s) {
    switch (nx) {
#define F(N)                                                                            \
    case N: {                                                                           \
        constexpr int RPW = row_rpw<N / 2>();                                           \
        dim3 grid((nrows + RPW - 1) / RPW);                                             \
        hipLaunchKernelGGL((k_row_inv<T, N>), grid, dim3(ROW_NTH), 0, s,                \
                           (const cx<T>*)in, (T*)out, nrows, (const cx<T>*)tw, twlog);  \
        return hipGetLastError();                                                       \
    }
        MUFFIN_POW2_CASES(F)
#undef F
    }
    return hipErrorInvalidValue;
}

hipError_t launch_row_inv(int dtype, const void* in, void* out, int nrows, int nx, const void* tw,
                          int twlog, hipStream_t s) {
    if (nrows <= 0) return hipSuccess;
    return dtype == 0 ? row_inv_t<float>(in, out, nrows, nx, tw, twlog, s)
                      : row_inv_t<double>(in, out, nrows, nx, tw, twlog, s);
}

template <typename T, int MODE>
static hipError_t col_t(void* data, const void* Yf, const void* H2, const void* H2nyq, double rhoQ,
                        double scale, int L, int ny, int nx, const void* tw, int twlog,
                        double* partials, int* nblocks_out, hipStream_t s) {
    const int M = nx / 2;
    switch (ny) {
#define F(N)                                                                                  \
    case N: {                                                                                 \
        constexpr int TC = col_tc<T, N>();                                                    \
        dim3 grid((M + TC - 1) / TC, L);                                                      \
        if (nblocks_out) *nblocks_out = int(grid.x * grid.y);                                 \
        hipLaunchKernelGGL((k_col<T, N, MODE>), grid, dim3(col_nth<T, N>()), 0, s,            \
                           (cx<T>*)data, (const cx<T>*)Yf, (const T*)H2, (const T*)H2nyq,     \
                           T(rhoQ), T(scale), M, (const cx<T>*)tw, twlog, partials,           \
                           1.0 / (double(nx) * double(ny)));                                  \
        return hipGetLastError();                                                             \
    }
        MUFFIN_POW2_CASES(F)
#undef F
    }
    return hipErrorInvalidValue;
}

hipError_t launch_col(int dtype, int mode, void* data, const void* Yf, const void* H2,
                      const void* H2nyq, double rhoQ, double scale, int L, int ny, int nx,
                      const void* tw, int twlog, double* partials, int* nblocks_out,
                      hipStream_t s) {
    if (dtype == 0) {
        if (mode == COL_SOLVE)
            return col_t<float, COL_SOLVE>(data, Yf, H2, H2nyq, rhoQ, scale, L, ny, nx, tw, twlog, partials, nblocks_out, s);
        if (mode == COL_OBJ)
            return col_t<float, COL_OBJ>(data, Yf, H2, H2nyq, rhoQ, scale, L, ny, nx, tw, twlog, partials, nblocks_out, s);
        return hipErrorInvalidValue;
    }
    if (mode == COL_SOLVE)
        return col_t<double, COL_SOLVE>(data, Yf, H2, H2nyq, rhoQ, scale, L, ny, nx, tw, twlog, partials, nblocks_out, s);
    if (mode == COL_FWD)
        return col_t<double, COL_FWD>(data, Yf, H2, H2nyq, rhoQ, scale, L, ny, nx, tw, twlog, partials, nblocks_out, s);
    return col_t<double, COL_OBJ>(data, Yf, H2, H2nyq, rhoQ, scale, L, ny, nx, tw, twlog, partials, nblocks_out, s);
}

hipError_t launch_setup_combine(int dtype, const void* Ch, const void* Cy, void* Yf, void* H2,
                                void* H2nyq, int L, int ny, int nx, hipStream_t s) {
    const int M = nx / 2;
    const long n = (long)L * ny * M;
    const int blocks = int((n + 255) / 256 < 65536 ? (n + 255) / 256 : 65536);
    if (dtype == 0)
        hipLaunchKernelGGL((k_setup_combine<float>), dim3(blocks), dim3(256), 0, s,
                           (const cx<double>*)Ch, (const cx<double>*)Cy, (cx<float>*)Yf,
                           (float*)H2, (float*)H2nyq, L, ny, M);
    else
        hipLaunchKernelGGL((k_setup_combine<double>), dim3(blocks), dim3(256), 0, s,
                           (const cx<double>*)Ch, (const cx<double>*)Cy, (cx<double>*)Yf,
                           (double*)H2, (double*)H2nyq, L, ny, M);
    return hipGetLastError();
}

}  // namespace muffin
