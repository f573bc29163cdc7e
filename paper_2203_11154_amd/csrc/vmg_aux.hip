// Kernels around the shifted solves: the shift sensitivity reduction used by
// the adjoint, the backward-Euler all-at-once heat operator and residual that
// the alpha-circulant ParaDIAG preconditioner is iterated on, and the vector
// operations of the Krylov (flexible GMRES) outer solver.  All reductions are
// two-stage with a fixed summation order.
#include "vmg_internal.h"

namespace vmg {

namespace {

constexpr int NT = 256;
constexpr int CHUNK = 4096;  // nodes per block of the reductions

__device__ __forceinline__ double wave_sum(double v) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// block-wide fixed-order sum; every thread returns the total
__device__ double block_sum(double v, double* red) {
    v = wave_sum(v);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    double t = 0.0;
    for (int w = 0; w < NT / 64; ++w) t += red[w];
    __syncthreads();
    return t;
}

// partial[s * ntiles + tile] = sum over the tile's nodes of conj(z) g
__global__ __launch_bounds__(NT) void k_cdot_partial(const double2* __restrict__ z, const double2* __restrict__ g,
                                                     int64_t m, int ntiles, double2* __restrict__ partial) {
    __shared__ double red[NT / 64];
    const int s = blockIdx.y, tile = blockIdx.x;
    const int64_t p0 = (int64_t)tile * CHUNK;
    const int64_t p1 = p0 + CHUNK < m ? p0 + CHUNK : m;
    double re = 0.0, im = 0.0;
    for (int64_t p = p0 + threadIdx.x; p < p1; p += NT) {
        const double2 a = z[(int64_t)s * m + p], b = g[(int64_t)s * m + p];
        // conj(a) * b
        re += a.x * b.x + a.y * b.y;
        im += a.x * b.y - a.y * b.x;
    }
    re = block_sum(re, red);
    im = block_sum(im, red);
    if (threadIdx.x == 0) partial[(int64_t)s * ntiles + tile] = make_double2(re, im);
}

__global__ __launch_bounds__(NT) void k_cdot_finalize(const double2* __restrict__ partial, int ntiles, double scale,
                                                      double2* __restrict__ out) {
    __shared__ double red[NT / 64];
    const int s = blockIdx.x;
    double re = 0.0, im = 0.0;
    for (int t = threadIdx.x; t < ntiles; t += NT) {
        re += partial[(int64_t)s * ntiles + t].x;
        im += partial[(int64_t)s * ntiles + t].y;
    }
    re = block_sum(re, red);
    im = block_sum(im, red);
    if (threadIdx.x == 0) out[s] = make_double2(scale * re, scale * im);
}

// R^m = F^m - ((U^m - U^{m-1})/tau + A U^m) (or U^{m+1} for the transpose);
// with F == NULL, R^m = (K U)^m instead; block (tile of CHUNK nodes, slice m);
// partial |R|^2 per block.
__global__ __launch_bounds__(NT) void k_heat_residual(const double2* __restrict__ U, const double2* F,
                                                      double2* R, int n, int nx, int ny, double h, double tau,
                                                      int transpose, int ntiles, double* __restrict__ partial) {
    __shared__ double red[NT / 64];
    const int sl = blockIdx.y, tile = blockIdx.x;
    const int64_t m = (int64_t)nx * ny;
    const int64_t p0 = (int64_t)tile * CHUNK;
    const int64_t p1 = p0 + CHUNK < m ? p0 + CHUNK : m;
    const int nb = transpose ? sl + 1 : sl - 1;  // neighbouring time slice
    const bool has_nb = nb >= 0 && nb < n;
    const double ih2 = 1.0 / (h * h), itau = 1.0 / tau;
    const double2* u = U + (int64_t)sl * m;
    double acc = 0.0;
    for (int64_t p = p0 + threadIdx.x; p < p1; p += NT) {
        const int k = (int)(p / nx), i = (int)(p - (int64_t)k * nx);
        const double2 c = u[p];
        double2 s = make_double2(0.0, 0.0);
        if (i > 0) { s.x += u[p - 1].x; s.y += u[p - 1].y; }
        if (i < nx - 1) { s.x += u[p + 1].x; s.y += u[p + 1].y; }
        if (k > 0) { s.x += u[p - nx].x; s.y += u[p - nx].y; }
        if (k < ny - 1) { s.x += u[p + nx].x; s.y += u[p + nx].y; }
        double2 prev = make_double2(0.0, 0.0);
        if (has_nb) prev = U[(int64_t)nb * m + p];
        double2 r;
        if (F) {
            const double2 f = F[(int64_t)sl * m + p];
            r.x = f.x - ((c.x - prev.x) * itau + (4.0 * c.x - s.x) * ih2);
            r.y = f.y - ((c.y - prev.y) * itau + (4.0 * c.y - s.y) * ih2);
        } else {
            r.x = (c.x - prev.x) * itau + (4.0 * c.x - s.x) * ih2;
            r.y = (c.y - prev.y) * itau + (4.0 * c.y - s.y) * ih2;
        }
        R[(int64_t)sl * m + p] = r;
        acc += r.x * r.x + r.y * r.y;
    }
    acc = block_sum(acc, red);
    if (threadIdx.x == 0) partial[(int64_t)sl * ntiles + tile] = acc;
}

__global__ __launch_bounds__(NT) void k_sum_all(const double* __restrict__ partial, int64_t count,
                                                double* __restrict__ out) {
    __shared__ double red[NT / 64];
    double acc = 0.0;
    for (int64_t t = threadIdx.x; t < count; t += NT) acc += partial[t];
    acc = block_sum(acc, red);
    if (threadIdx.x == 0) out[0] = acc;
}

// y += sign * a * x with a = *coef (device) or the value `a` when coef is NULL
__global__ __launch_bounds__(NT) void k_zaxpy(double2* __restrict__ y, const double2* __restrict__ x, int64_t N,
                                              const double2* coef, double sign, double2 a) {
    if (coef) a = *coef;
    a.x *= sign;
    a.y *= sign;
    for (int64_t p = (int64_t)blockIdx.x * NT + threadIdx.x; p < N; p += (int64_t)gridDim.x * NT) {
        const double2 v = x[p];
        double2 w = y[p];
        w.x += a.x * v.x - a.y * v.y;
        w.y += a.x * v.y + a.y * v.x;
        y[p] = w;
    }
}

// y *= 1 / sqrt(nrm2->x) (y unchanged when the norm is zero), or by `s` when
// nrm2 is NULL
__global__ __launch_bounds__(NT) void k_zscale(double2* __restrict__ y, int64_t N, const double2* nrm2, double s) {
    if (nrm2) s = nrm2->x > 0.0 ? 1.0 / sqrt(nrm2->x) : 1.0;
    for (int64_t p = (int64_t)blockIdx.x * NT + threadIdx.x; p < N; p += (int64_t)gridDim.x * NT) {
        double2 w = y[p];
        w.x *= s;
        w.y *= s;
        y[p] = w;
    }
}

inline int stream_blocks(int64_t N) {
    const int64_t b = (N + NT - 1) / NT;
    return (int)(b < 8192 ? (b > 0 ? b : 1) : 8192);
}

}  // namespace

void launch_zdot(const double2* a, const double2* b, int64_t N, double2* partial, double2* out, hipStream_t st) {
    const int nt = aux_tiles(N);
    hipLaunchKernelGGL(k_cdot_partial, dim3(nt, 1), dim3(NT), 0, st, a, b, N, nt, partial);
    hipLaunchKernelGGL(k_cdot_finalize, dim3(1), dim3(NT), 0, st, partial, nt, 1.0, out);
}

void launch_zaxpy(double2* y, const double2* x, int64_t N, const double2* coef, double sign, double2 a,
                  hipStream_t st) {
    hipLaunchKernelGGL(k_zaxpy, dim3(stream_blocks(N)), dim3(NT), 0, st, y, x, N, coef, sign, a);
}

void launch_zscale(double2* y, int64_t N, const double2* nrm2, double s, hipStream_t st) {
    hipLaunchKernelGGL(k_zscale, dim3(stream_blocks(N)), dim3(NT), 0, st, y, N, nrm2, s);
}

int aux_tiles(int64_t m) { return (int)((m + CHUNK - 1) / CHUNK); }

void launch_shift_gradient(const double2* z, const double2* g, int64_t m, int nsys, double2* partial,
                           double2* out, hipStream_t st) {
    const int nt = aux_tiles(m);
    hipLaunchKernelGGL(k_cdot_partial, dim3(nt, nsys), dim3(NT), 0, st, z, g, m, nt, partial);
    hipLaunchKernelGGL(k_cdot_finalize, dim3(nsys), dim3(NT), 0, st, partial, nt, -1.0, out);
}

void launch_heat_residual(const double2* U, const double2* F, double2* R, int n, int nx, int ny, double h,
                          double tau, int transpose, double* partial, double* out_norm2, hipStream_t st) {
    const int nt = aux_tiles((int64_t)nx * ny);
    hipLaunchKernelGGL(k_heat_residual, dim3(nt, n), dim3(NT), 0, st, U, F, R, n, nx, ny, h, tau, transpose, nt,
                       partial);
    hipLaunchKernelGGL(k_sum_all, dim3(1), dim3(NT), 0, st, partial, (int64_t)nt * n, out_norm2);
}

}  // namespace vmg
