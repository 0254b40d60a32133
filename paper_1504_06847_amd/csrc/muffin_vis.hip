// The visibility-domain model (Section 2: the data are the sampled
// visibilities and H_l maps the sky to the visibilities of band l; step I
// of Algorithm 1 by conjugate gradients on Q_l = Re(H_l^H H_l) + rho I,
// eq. Qlsimp).
//
// (H_l x)_j = sum_{m,n} x[m, n] exp(-2 pi i (u_j (n - nx/2) / nx + v_j (m - ny/2) / ny))
// at visibility j = (u_j, v_j) in cells of the Fourier grid.  Re(H^H H) is
// two-level Toeplitz with kernel c(d) = sum_j cos(2 pi (u_j d_x / nx +
// v_j d_y / ny)): with the kernel on a 2ny x 2nx grid it is a circular
// convolution of the zero-padded image, cropped, so each CG iteration runs
// the existing row and column FFT passes on the padded cube (the column pass
// multiplying by the kernel's transfer function).  Setup forms c and the data
// term Re(H^H y) by direct sums over the visibilities in FP64; both sums are
// matrix products over the separable phase e^{i(a + b)} = e^{ia} e^{ib}, so a
// work-group computes a 64 x 64 tile of outputs from chunks of 16
// visibilities whose phases it stages in LDS.
#include "muffin_device.hpp"
#include "muffin_kernels.hpp"

namespace muffin {

constexpr int VT = 64;        // output tile (rows and columns)
constexpr int VK = 16;        // visibilities per LDS chunk
constexpr int VNTH = 256;     // 16 x 16 threads, 4 x 4 outputs each

// MODE 0: out[l][Y][X] = c(Y - ny, X - nx) on the 2ny x 2nx grid of lags
// (zero at the unused lags -ny and -nx).  MODE 1: out[l][Y][X] =
// Re(H^H y)[Y][X] = sum_j Re(y_j e^{i(a + b)}), a = 2 pi u_j (X - nx/2) / nx,
// b = 2 pi v_j (Y - ny/2) / ny.  Both: sum_j (B1[Y] A1[X] - B2[Y] A2[X]) with
// B1 = cos b, B2 = sin b and (A1, A2) = (cos a, sin a) (MODE 0) or
// (Re y cos a - Im y sin a, Re y sin a + Im y cos a) (MODE 1).
template <typename T, int MODE>
__global__ void __launch_bounds__(VNTH)
k_vis_sum(const double* __restrict__ uv, const double* __restrict__ vis, const long* __restrict__ off, int ny,
          int nx, T* __restrict__ out) {
    __shared__ double a1[VK][VT], a2[VK][VT], b1[VK][VT], b2[VK][VT];
    const int l = blockIdx.z;
    const int W = MODE == 0 ? 2 * nx : nx, H = MODE == 0 ? 2 * ny : ny;
    const int X0 = blockIdx.x * VT, Y0 = blockIdx.y * VT;
    const int t = threadIdx.x, tx = t & 15, ty = t >> 4;
    const long j0 = off[l], j1 = off[l + 1];
    double acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int k = 0; k < 4; ++k) acc[i][k] = 0.0;
    for (long jc = j0; jc < j1; jc += VK) {
        // phases of this chunk: VK x VT for the columns and for the rows
        for (int e = t; e < VK * VT; e += VNTH) {
            const int k = e / VT, c = e % VT;
            const long j = jc + k;
            double ca = 0.0, sa = 0.0, cb = 0.0, sb = 0.0, yr = 0.0, yi = 0.0;
            if (j < j1) {
                const double u = uv[2 * j], v = uv[2 * j + 1];
                const int X = X0 + c, Y = Y0 + c;
                const double dx = MODE == 0 ? double(X - nx) : double(X - nx / 2);
                const double dy = MODE == 0 ? double(Y - ny) : double(Y - ny / 2);
                sincospi(2.0 * u * dx / nx, &sa, &ca);
                sincospi(2.0 * v * dy / ny, &sb, &cb);
                if (MODE == 1) { yr = vis[2 * j]; yi = vis[2 * j + 1]; }
            }
            if (MODE == 0) {
                a1[k][c] = ca;
                a2[k][c] = sa;
            } else {
                a1[k][c] = yr * ca - yi * sa;
                a2[k][c] = yr * sa + yi * ca;
            }
            b1[k][c] = cb;
            b2[k][c] = sb;
        }
        __syncthreads();
#pragma unroll 4
        for (int k = 0; k < VK; ++k) {
            double ra1[4], ra2[4], rb1[4], rb2[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                ra1[i] = a1[k][tx + 16 * i];
                ra2[i] = a2[k][tx + 16 * i];
                rb1[i] = b1[k][ty + 16 * i];
                rb2[i] = b2[k][ty + 16 * i];
            }
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int q = 0; q < 4; ++q) acc[i][q] = fma(rb1[i], ra1[q], fma(-rb2[i], ra2[q], acc[i][q]));
        }
        __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int Y = Y0 + ty + 16 * i;
        if (Y >= H) continue;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int X = X0 + tx + 16 * q;
            if (X >= W) continue;
            const bool unused = MODE == 0 && (X == 0 || Y == 0);
            out[((long)l * H + Y) * W + X] = T(unused ? 0.0 : acc[i][q]);
        }
    }
}

template <typename T>
__global__ void __launch_bounds__(VNTH) k_vis_delta(T* __restrict__ out, long npix, long centre, long n) {
    for (long i = (long)blockIdx.x * VNTH + threadIdx.x; i < n; i += (long)gridDim.x * VNTH)
        out[i] = (i % npix) == centre ? T(1) : T(0);
}

hipError_t launch_vis_delta(int dtype, void* out, int L, int ny, int nx, hipStream_t s) {
    const long npix = (long)ny * nx, n = npix * L, centre = (long)(ny / 2) * nx + nx / 2;
    long nb = (n + VNTH - 1) / VNTH;
    if (nb > 65536) nb = 65536;
    if (dtype == 0) hipLaunchKernelGGL((k_vis_delta<float>), dim3((unsigned)nb), dim3(VNTH), 0, s, (float*)out, npix, centre, n);
    else hipLaunchKernelGGL((k_vis_delta<double>), dim3((unsigned)nb), dim3(VNTH), 0, s, (double*)out, npix, centre, n);
    return hipGetLastError();
}

template <typename T>
static hipError_t vis_sum_t(int mode, const double* uv, const double* vis, const long* off, int L, int ny, int nx,
                            void* out, hipStream_t s) {
    const int W = mode == 0 ? 2 * nx : nx, H = mode == 0 ? 2 * ny : ny;
    const dim3 grid((unsigned)((W + VT - 1) / VT), (unsigned)((H + VT - 1) / VT), (unsigned)L);
    if (mode == 0) hipLaunchKernelGGL((k_vis_sum<T, 0>), grid, dim3(VNTH), 0, s, uv, vis, off, ny, nx, (T*)out);
    else hipLaunchKernelGGL((k_vis_sum<T, 1>), grid, dim3(VNTH), 0, s, uv, vis, off, ny, nx, (T*)out);
    return hipGetLastError();
}

hipError_t launch_vis_sum(int dtype, int mode, const double* uv, const double* vis, const long* off, int L,
                          int ny, int nx, void* out, hipStream_t s) {
    if (mode < 0 || mode > 1 || L < 1 || ny < 1 || nx < 1) return hipErrorInvalidValue;
    return dtype == 0 ? vis_sum_t<float>(mode, uv, vis, off, L, ny, nx, out, s)
                      : vis_sum_t<double>(mode, uv, vis, off, L, ny, nx, out, s);
}

// ------------------------------------------------------------------ CG vectors
// Element kernels over the pixels of every band: grid (nb, L), block VNTH;
// block b of band l takes pixels b VNTH + t, then every nb VNTH further.  A
// pixel (y, x) of band l sits at l npix + y nx + x in a plain cube and at
// l 4 npix + y 2nx + x in the zero-padded 2ny x 2nx cube.  The dot products
// accumulate in FP64 per thread, then per block (fixed order), into
// partials[l nb + b].
struct CgGeom {
    int nx, ny, nb;
    long npix;
};

__device__ __forceinline__ long padded(const CgGeom& g, int l, long i) {
    return (long)l * 4 * g.npix + (i / g.nx) * 2 * g.nx + (i % g.nx);
}

template <typename T>
__device__ __forceinline__ void put_partial(double v, double* partials, const CgGeom& g) {
    __shared__ double sh[VNTH / 64];
    const double s = block_sum_s<VNTH>(v, sh);
    if (threadIdx.x == 0) partials[(long)blockIdx.y * g.nb + blockIdx.x] = s;
}

// x0 into the padded cube
template <typename T>
__global__ void __launch_bounds__(VNTH) k_cg_pad(CgGeom g, const T* __restrict__ x, T* __restrict__ P2) {
    const int l = blockIdx.y;
    for (long i = (long)blockIdx.x * VNTH + threadIdx.x; i < g.npix; i += (long)g.nb * VNTH)
        P2[padded(g, l, i)] = x[(long)l * g.npix + i];
}

// r = HtY + B_rest - (A2 + rho x);  p = r;  partial r.r
template <typename T>
__global__ void __launch_bounds__(VNTH)
k_cg_init(CgGeom g, const T* __restrict__ hty, const T* __restrict__ brest, const T* __restrict__ x,
          const T* __restrict__ A2, double rho, T* __restrict__ r, T* __restrict__ P2, double* __restrict__ partials) {
    const int l = blockIdx.y;
    const T rh = T(rho);
    double acc = 0.0;
    for (long i = (long)blockIdx.x * VNTH + threadIdx.x; i < g.npix; i += (long)g.nb * VNTH) {
        const long o = (long)l * g.npix + i, po = padded(g, l, i);
        const T rv = (hty[o] + brest[o]) - (A2[po] + rh * x[o]);
        r[o] = rv;
        P2[po] = rv;
        acc += double(rv) * double(rv);
    }
    put_partial<T>(acc, partials, g);
}

// Ap = A2 + rho p;  partial p.Ap
template <typename T>
__global__ void __launch_bounds__(VNTH)
k_cg_ap(CgGeom g, const T* __restrict__ P2, const T* __restrict__ A2, double rho, T* __restrict__ Ap,
        double* __restrict__ partials) {
    const int l = blockIdx.y;
    const T rh = T(rho);
    double acc = 0.0;
    for (long i = (long)blockIdx.x * VNTH + threadIdx.x; i < g.npix; i += (long)g.nb * VNTH) {
        const long o = (long)l * g.npix + i, po = padded(g, l, i);
        const T p = P2[po];
        const T q = A2[po] + rh * p;
        Ap[o] = q;
        acc += double(p) * double(q);
    }
    put_partial<T>(acc, partials, g);
}

// x += alpha p;  r -= alpha Ap;  partial r.r
template <typename T>
__global__ void __launch_bounds__(VNTH)
k_cg_xr(CgGeom g, T* __restrict__ x, T* __restrict__ r, const T* __restrict__ P2, const T* __restrict__ Ap,
        const double* __restrict__ alpha, double* __restrict__ partials) {
    const int l = blockIdx.y;
    const T a = T(alpha[l]);
    double acc = 0.0;
    for (long i = (long)blockIdx.x * VNTH + threadIdx.x; i < g.npix; i += (long)g.nb * VNTH) {
        const long o = (long)l * g.npix + i;
        x[o] = x[o] + a * P2[padded(g, l, i)];
        const T rv = r[o] - a * Ap[o];
        r[o] = rv;
        acc += double(rv) * double(rv);
    }
    put_partial<T>(acc, partials, g);
}

// p = r + beta p
template <typename T>
__global__ void __launch_bounds__(VNTH)
k_cg_p(CgGeom g, const T* __restrict__ r, T* __restrict__ P2, const double* __restrict__ beta) {
    const int l = blockIdx.y;
    const T b = T(beta[l]);
    for (long i = (long)blockIdx.x * VNTH + threadIdx.x; i < g.npix; i += (long)g.nb * VNTH) {
        const long po = padded(g, l, i);
        P2[po] = r[(long)l * g.npix + i] + b * P2[po];
    }
}

// the per-band scalars from the partial sums s of one band (one work-group
// of 64 per band, fixed summation order): mode 0: rr = s; 1: alpha =
// rr / s (0 if s <= 0); 2: beta = s / rr (0 if rr <= 0), rr = s
__global__ void __launch_bounds__(64)
k_cg_scalar(const double* __restrict__ partials, int nb, int mode, double* __restrict__ rr,
            double* __restrict__ alpha, double* __restrict__ beta) {
    const int l = blockIdx.x;
    double v = 0.0;
    for (int b = threadIdx.x; b < nb; b += 64) v += partials[(long)l * nb + b];
    __shared__ double sh[1];
    const double s = block_sum_s<64>(v, sh);
    if (threadIdx.x == 0) {
        if (mode == 0) {
            rr[l] = s;
        } else if (mode == 1) {
            alpha[l] = s > 0.0 ? rr[l] / s : 0.0;
        } else {
            beta[l] = rr[l] > 0.0 ? s / rr[l] : 0.0;
            rr[l] = s;
        }
    }
}

int cg_blocks(long npix) {
    long nb = npix / (VNTH * 4);
    if (nb < 1) nb = 1;
    if (nb > 256) nb = 256;
    return (int)nb;
}

template <typename T>
static hipError_t cg_t(int op, const CgVectors& v, double rho, hipStream_t s) {
    CgGeom g{v.nx, v.ny, cg_blocks((long)v.nx * v.ny), (long)v.nx * v.ny};
    const dim3 grid((unsigned)g.nb, (unsigned)v.L), blk(VNTH);
    switch (op) {
        case CG_PAD:
            hipLaunchKernelGGL((k_cg_pad<T>), grid, blk, 0, s, g, (const T*)v.x, (T*)v.P2);
            break;
        case CG_INIT:
            hipLaunchKernelGGL((k_cg_init<T>), grid, blk, 0, s, g, (const T*)v.hty, (const T*)v.brest,
                               (const T*)v.x, (const T*)v.A2, rho, (T*)v.r, (T*)v.P2, v.partials);
            break;
        case CG_AP:
            hipLaunchKernelGGL((k_cg_ap<T>), grid, blk, 0, s, g, (const T*)v.P2, (const T*)v.A2, rho, (T*)v.Ap,
                               v.partials);
            break;
        case CG_XR:
            hipLaunchKernelGGL((k_cg_xr<T>), grid, blk, 0, s, g, (T*)v.x, (T*)v.r, (const T*)v.P2, (const T*)v.Ap,
                               (const double*)v.alpha, v.partials);
            break;
        case CG_P:
            hipLaunchKernelGGL((k_cg_p<T>), grid, blk, 0, s, g, (const T*)v.r, (T*)v.P2, (const double*)v.beta);
            break;
        default: return hipErrorInvalidValue;
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || op == CG_PAD || op == CG_P) return e;
    // the per-band scalar that follows each reduction
    const int mode = op == CG_INIT ? 0 : (op == CG_AP ? 1 : 2);
    hipLaunchKernelGGL(k_cg_scalar, dim3((unsigned)v.L), dim3(64), 0, s, (const double*)v.partials, g.nb, mode,
                       v.rr, v.alpha, v.beta);
    return hipGetLastError();
}

hipError_t launch_cg(int dtype, int op, const CgVectors& v, double rho, hipStream_t s) {
    if (v.L < 1 || v.nx < 1 || v.ny < 1) return hipErrorInvalidValue;
    return dtype == 0 ? cg_t<float>(op, v, rho, s) : cg_t<double>(op, v, rho, s);
}

}  // namespace muffin
