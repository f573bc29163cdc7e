// Stencil kernels of the Vanka multigrid solver for gfx950.
//
// Every kernel works on a batch of systems that share one level geometry:
// blockIdx.z is the system, and a system whose active flag is 0 is left
// untouched (its solve has stopped).  Complex values are interleaved
// (double2 / float2); planes are padded with a zero Dirichlet ring so the
// interior stencils need no boundary branches on their loads, only on the
// tile halo outside the padded plane.
#include "vmg_internal.h"

namespace vmg {

namespace {

constexpr int NT = 256;  // threads per block (4 wave64)

// ---------------------------------------------------------------------------
// Additive Vanka sweep (eq. (3) with the explicit stencil of eq. (6)):
//   r = b - L x on the tile plus a one-node halo (zero off the interior),
//   x' = x + ca r_c + cb (edge sum of r) + cc (corner sum of r).
// Out of place: every update uses the residual of the old x.
// Tile: TX = 64 columns (one wave per row segment) by TY rows.
// ---------------------------------------------------------------------------
template <typename T, int TY>
__global__ __launch_bounds__(NT) void k_sweep(SegTable<T> tab) {
    using C = cplx<T>;
    constexpr int TX = 64;
    constexpr int XW = TX + 4, XH = TY + 4;
    constexpr int RW = TX + 2, RH = TY + 2;
    __shared__ C sx[XH * XW];
    __shared__ C sr[RH * RW];
    const LevelSeg<T> S = seg_of(tab, blockIdx.z);
    const int sys = blockIdx.z - S.z0;
    if ((int)blockIdx.x >= S.gx || (int)blockIdx.y >= S.gy) return;
    if (!S.active[sys]) return;
    const LevelView lv = S.lf;
    const int x_zero = S.x_zero;
    const int i0 = blockIdx.x * TX + 1;
    const int k0 = blockIdx.y * TY + 1;
    const int64_t base = (int64_t)sys * lv.plane;
    const C* xs = S.x + base;
    const C* bs = S.b + base;
    const Coef<T> cf = S.coef[sys];
    const T s = S.s;

    if (!x_zero) {
        for (int t = threadIdx.x; t < XH * XW; t += NT) {
            const int ry = t / XW, rx = t - ry * XW;
            const int i = i0 - 2 + rx, k = k0 - 2 + ry;
            C v = czero<C>();
            if (i >= 0 && i <= lv.nx + 1 && k >= 0 && k <= lv.ny + 1) v = xs[(int64_t)k * lv.pitch + i];
            sx[t] = v;
        }
        __syncthreads();
    }
    for (int t = threadIdx.x; t < RH * RW; t += NT) {
        const int ry = t / RW, rx = t - ry * RW;
        const int i = i0 - 1 + rx, k = k0 - 1 + ry;
        C r = czero<C>();
        if (i >= 1 && i <= lv.nx && k >= 1 && k <= lv.ny) {
            r = bs[(int64_t)k * lv.pitch + i];
            if (!x_zero) {
                const int c = (ry + 1) * XW + rx + 1;
                const C nb = cadd(cadd(sx[c - XW], sx[c + XW]), cadd(sx[c - 1], sx[c + 1]));
                // r = b - (d x - s nb)
                r = csub(r, csub(cmul(cf.d, sx[c]), cscale(nb, s)));
            }
        }
        sr[t] = r;
    }
    __syncthreads();
    for (int t = threadIdx.x; t < TX * TY; t += NT) {
        const int ty = t / TX, tx = t - ty * TX;
        const int i = i0 + tx, k = k0 + ty;
        if (i > lv.nx || k > lv.ny) continue;
        const int c = (ty + 1) * RW + tx + 1;
        const C edge = cadd(cadd(sr[c - RW], sr[c + RW]), cadd(sr[c - 1], sr[c + 1]));
        const C corner = cadd(cadd(sr[c - RW - 1], sr[c - RW + 1]), cadd(sr[c + RW - 1], sr[c + RW + 1]));
        C v = x_zero ? czero<C>() : sx[(ty + 2) * XW + tx + 2];
        v = cfma(v, cf.ca, sr[c]);
        v = cfma(v, cf.cb, edge);
        v = cfma(v, cf.cc, corner);
        S.xo[base + (int64_t)k * lv.pitch + i] = v;
    }
}

// ---------------------------------------------------------------------------
// Residual + full-weighting restriction: r_H(I, K) = FW(b - L x) around fine
// node (2I, 2K), written into the coarse right-hand side.
// Tile: TXC x TYC coarse nodes; the fine residual is formed in LDS on the
// (2 TXC + 1) x (2 TYC + 1) nodes they cover.
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(NT) void k_restrict(SegTable<T> tab) {
    using C = cplx<T>;
    constexpr int TXC = 32, TYC = 8;
    constexpr int RW = 2 * TXC + 1, RH = 2 * TYC + 1;
    constexpr int XW = RW + 2, XH = RH + 2;
    __shared__ C sx[XH * XW];
    __shared__ C sr[RH * RW];
    const LevelSeg<T> S = seg_of(tab, blockIdx.z);
    const int sys = blockIdx.z - S.z0;
    if ((int)blockIdx.x >= S.gx || (int)blockIdx.y >= S.gy) return;
    if (!S.active[sys]) return;
    const LevelView lf = S.lf, lc = S.lc;
    const int x_zero = S.x_zero;
    const int I0 = blockIdx.x * TXC + 1, K0 = blockIdx.y * TYC + 1;
    const int fi0 = 2 * I0 - 1, fk0 = 2 * K0 - 1;  // first fine node of the residual region
    const int64_t basef = (int64_t)sys * lf.plane;
    const C* xs = S.x + basef;
    const C* bs = S.b + basef;
    const Coef<T> cf = S.coef[sys];
    const T s = S.s;
    if (!x_zero) {
        for (int t = threadIdx.x; t < XH * XW; t += NT) {
            const int ry = t / XW, rx = t - ry * XW;
            const int i = fi0 - 1 + rx, k = fk0 - 1 + ry;
            C v = czero<C>();
            if (i >= 0 && i <= lf.nx + 1 && k >= 0 && k <= lf.ny + 1) v = xs[(int64_t)k * lf.pitch + i];
            sx[t] = v;
        }
        __syncthreads();
    }
    for (int t = threadIdx.x; t < RH * RW; t += NT) {
        const int ry = t / RW, rx = t - ry * RW;
        const int i = fi0 + rx, k = fk0 + ry;
        C r = czero<C>();
        if (i >= 1 && i <= lf.nx && k >= 1 && k <= lf.ny) {
            r = bs[(int64_t)k * lf.pitch + i];
            if (!x_zero) {
                const int c = (ry + 1) * XW + rx + 1;
                const C nb = cadd(cadd(sx[c - XW], sx[c + XW]), cadd(sx[c - 1], sx[c + 1]));
                r = csub(r, csub(cmul(cf.d, sx[c]), cscale(nb, s)));
            }
        }
        sr[t] = r;
    }
    __syncthreads();
    for (int t = threadIdx.x; t < TXC * TYC; t += NT) {
        const int ty = t / TXC, tx = t - ty * TXC;
        const int I = I0 + tx, K = K0 + ty;
        if (I > lc.nx || K > lc.ny) continue;
        const int c = (2 * ty + 1) * RW + 2 * tx + 1;  // fine (2I, 2K) in the region
        const C edge = cadd(cadd(sr[c - RW], sr[c + RW]), cadd(sr[c - 1], sr[c + 1]));
        const C corner = cadd(cadd(sr[c - RW - 1], sr[c - RW + 1]), cadd(sr[c + RW - 1], sr[c + RW + 1]));
        C v = cscale(sr[c], (T)0.25);
        v = cadd(v, cscale(edge, (T)0.125));
        v = cadd(v, cscale(corner, (T)0.0625));
        S.c[(int64_t)sys * lc.plane + (int64_t)K * lc.pitch + I] = v;
    }
}

// ---------------------------------------------------------------------------
// Bilinear interpolation of the coarse correction and update:
//   x(i, k) += sum of e over the 1, 2 or 4 coarse nodes around fine (i, k),
// with weights 1, 1/2, 1/4 (the coarse ring holds zeros).
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(NT) void k_prolong(SegTable<T> tab) {
    using C = cplx<T>;
    constexpr int TX = 64, TY = 16;
    const LevelSeg<T> S = seg_of(tab, blockIdx.z);
    const int sys = blockIdx.z - S.z0;
    if ((int)blockIdx.x >= S.gx || (int)blockIdx.y >= S.gy) return;
    if (!S.active[sys]) return;
    const LevelView lf = S.lf, lc = S.lc;
    const int i = blockIdx.x * TX + (threadIdx.x & 63) + 1;
    if (i > lf.nx) return;
    const C* es = S.c + (int64_t)sys * lc.plane;
    const C* xs = S.x + (int64_t)sys * lf.plane;
    C* xos = S.xo + (int64_t)sys * lf.plane;
    const int il = i >> 1, ir = (i + 1) >> 1;       // coarse columns around fine i
    const T wx = (i & 1) ? (T)0.5 : (T)1.0;         // odd: average of two
    for (int k = blockIdx.y * TY + (threadIdx.x >> 6) + 1; k <= min(lf.ny, (int)(blockIdx.y + 1) * TY);
         k += NT / 64) {
        const int kl = k >> 1, kr = (k + 1) >> 1;
        const T wy = (k & 1) ? (T)0.5 : (T)1.0;
        C v;
        if (!(i & 1) && !(k & 1)) {
            v = es[(int64_t)kl * lc.pitch + il];
        } else {
            const C a = es[(int64_t)kl * lc.pitch + il];
            const C bq = es[(int64_t)kl * lc.pitch + ir];
            const C c = es[(int64_t)kr * lc.pitch + il];
            const C d = es[(int64_t)kr * lc.pitch + ir];
            // for even i, il == ir and wx = 1: the pair collapses to one node
            C row0 = (i & 1) ? cadd(a, bq) : a;
            C row1 = (i & 1) ? cadd(c, d) : c;
            v = (k & 1) ? cadd(row0, row1) : row0;
            v = cscale(v, wx * wy);
        }
        const int64_t o = (int64_t)k * lf.pitch + i;
        xos[o] = S.x_zero ? v : cadd(xs[o], v);
    }
}

// ---------------------------------------------------------------------------
// Residual r = b - L x with optional store (as TO) and per-tile sums of |r|^2.
// Tile 64 x 16 nodes, neighbours read directly (cached).
// ---------------------------------------------------------------------------
template <typename T, typename TO>
__global__ __launch_bounds__(NT) void k_residual(const cplx<T>* __restrict__ x, const cplx<T>* __restrict__ b,
                                                 cplx<TO>* __restrict__ rout, LevelView lv, LevelView lo, T s,
                                                 const Coef<T>* __restrict__ coef,
                                                 const int* __restrict__ active, int x_zero,
                                                 double* __restrict__ partial) {
    using C = cplx<T>;
    using CO = cplx<TO>;
    constexpr int TX = 64, TY = 16;
    __shared__ double red[NT / 64];
    const int sys = blockIdx.z;
    if (!active[sys]) return;
    const int i = blockIdx.x * TX + (threadIdx.x & 63) + 1;
    const int64_t base = (int64_t)sys * lv.plane;
    const Coef<T> cf = coef[sys];
    double acc = 0.0;
    if (i <= lv.nx) {
        for (int k = blockIdx.y * TY + (threadIdx.x >> 6) + 1; k <= min(lv.ny, (int)(blockIdx.y + 1) * TY);
             k += NT / 64) {
            const int64_t o = base + (int64_t)k * lv.pitch + i;
            C r = b[o];
            if (!x_zero) {
                const C nb = cadd(cadd(x[o - lv.pitch], x[o + lv.pitch]), cadd(x[o - 1], x[o + 1]));
                r = csub(r, csub(cmul(cf.d, x[o]), cscale(nb, s)));
            }
            acc += (double)r.x * (double)r.x + (double)r.y * (double)r.y;
            if (rout) {
                CO ro;
                ro.x = (TO)r.x;
                ro.y = (TO)r.y;
                rout[(int64_t)sys * lo.plane + (int64_t)k * lo.pitch + i] = ro;
            }
        }
    }
    // fixed-order block reduction: butterfly within each wave, then waves in order
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0 && partial) {
        double tsum = 0.0;
        for (int w = 0; w < NT / 64; ++w) tsum += red[w];
        partial[(int64_t)sys * (gridDim.x * gridDim.y) + blockIdx.y * gridDim.x + blockIdx.x] = tsum;
    }
}

// ---------------------------------------------------------------------------
// Coarsest grid: x = (A_c + lambda_j I)^{-1} b with the inverse precomputed
// on the host (stored transposed: cinvT[k * nc + row]).  One block per system.
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(NT) void k_coarse(SegTable<T> tab) {
    using C = cplx<T>;
    __shared__ C sb[NT];
    const LevelSeg<T> S = seg_of(tab, blockIdx.z);
    const int sys = blockIdx.z - S.z0;
    if (!S.active[sys]) return;
    const LevelView lc = S.lf;
    const int nc = S.nc;
    const int t = threadIdx.x;
    const int64_t base = (int64_t)sys * lc.plane;
    int64_t o = 0;
    if (t < nc) {
        const int k = t / lc.nx + 1, i = t - (k - 1) * lc.nx + 1;
        o = base + (int64_t)k * lc.pitch + i;
        sb[t] = S.b[o];
    }
    __syncthreads();
    if (t < nc) {
        const C* ci = S.cinvT + (int64_t)sys * nc * nc;
        C acc = czero<C>();
        for (int k = 0; k < nc; ++k) acc = cfma(acc, ci[(int64_t)k * nc + t], sb[k]);
        S.xo[o] = acc;
    }
}

// One refinement step's end: x' = x + e (FP64 iterate plus the complex64
// correction; x = 0 with x_zero), written to a second buffer, and the FP64
// residual of x' (stored as complex64, the next step's right-hand side) with
// its per-tile |r|^2 sums, in one pass.  x' at the neighbours is formed from
// x and e on the fly (their rings are zero).
__global__ __launch_bounds__(NT) void k_ir_residual(const double2* __restrict__ x, const float2* __restrict__ e,
                                                    const double2* __restrict__ b, double2* __restrict__ xn,
                                                    float2* __restrict__ rout, LevelView lv, LevelView le, double s,
                                                    const Coef<double>* __restrict__ coef,
                                                    const int* __restrict__ active, double* __restrict__ partial) {
    constexpr int TX = 64, TY = 16;
    __shared__ double red[NT / 64];
    const int sys = blockIdx.z;
    if (!active[sys]) return;
    const int i = blockIdx.x * TX + (threadIdx.x & 63) + 1;
    const int64_t base = (int64_t)sys * lv.plane, ebase = (int64_t)sys * le.plane;
    const Coef<double> cf = coef[sys];
    auto xv = [&](int k, int c) {
        const float2 ev = e[ebase + (int64_t)k * le.pitch + c];
        double2 v = x ? x[base + (int64_t)k * lv.pitch + c] : make_double2(0.0, 0.0);
        v.x += (double)ev.x;
        v.y += (double)ev.y;
        return v;
    };
    double acc = 0.0;
    if (i <= lv.nx) {
        for (int k = blockIdx.y * TY + (threadIdx.x >> 6) + 1; k <= min(lv.ny, (int)(blockIdx.y + 1) * TY);
             k += NT / 64) {
            const double2 xc = xv(k, i);
            const double2 nb = cadd(cadd(xv(k - 1, i), xv(k + 1, i)), cadd(xv(k, i - 1), xv(k, i + 1)));
            const int64_t o = base + (int64_t)k * lv.pitch + i;
            const double2 r = csub(b[o], csub(cmul(cf.d, xc), cscale(nb, s)));
            xn[o] = xc;
            acc += r.x * r.x + r.y * r.y;
            rout[ebase + (int64_t)k * le.pitch + i] = make_float2((float)r.x, (float)r.y);
        }
    }
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        double tsum = 0.0;
        for (int w = 0; w < NT / 64; ++w) tsum += red[w];
        partial[(int64_t)sys * (gridDim.x * gridDim.y) + blockIdx.y * gridDim.x + blockIdx.x] = tsum;
    }
}

template <typename T>
__global__ __launch_bounds__(NT) void k_pack(const cplx<T>* __restrict__ src, cplx<T>* __restrict__ dst,
                                             LevelView lv, double* __restrict__ partial) {
    __shared__ double red[NT / 64];
    const int sys = blockIdx.z;
    const int i = blockIdx.x * 64 + (threadIdx.x & 63);
    double acc = 0.0;
    if (i < lv.nx) {
        for (int k = blockIdx.y * 16 + (threadIdx.x >> 6); k < min(lv.ny, (int)(blockIdx.y + 1) * 16); k += NT / 64) {
            const cplx<T> v = src[((int64_t)sys * lv.ny + k) * lv.nx + i];
            dst[(int64_t)sys * lv.plane + (int64_t)(k + 1) * lv.pitch + i + 1] = v;
            acc += (double)v.x * (double)v.x + (double)v.y * (double)v.y;
        }
    }
    if (!partial) return;  // uniform over the grid
    // |b|^2 of the tile, in the residual kernel's tile order and layout
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int w = 0; w < NT / 64; ++w) t += red[w];
        partial[(int64_t)sys * (gridDim.x * gridDim.y) + blockIdx.y * gridDim.x + blockIdx.x] = t;
    }
}

template <typename T>
__global__ __launch_bounds__(NT) void k_unpack(const cplx<T>* __restrict__ src0, const cplx<T>* __restrict__ src1,
                                               cplx<T>* __restrict__ dst, LevelView lv,
                                               const int* __restrict__ iters, int flips) {
    using C = cplx<T>;
    const int sys = blockIdx.z;
    const int i = blockIdx.x * 64 + (threadIdx.x & 63);
    if (i >= lv.nx) return;
    const bool zero = iters && iters[sys] == 0;
    const C* src = (iters && src1 && ((iters[sys] * flips) & 1)) ? src1 : src0;
    for (int k = blockIdx.y * 16 + (threadIdx.x >> 6); k < min(lv.ny, (int)(blockIdx.y + 1) * 16); k += NT / 64)
        dst[((int64_t)sys * lv.ny + k) * lv.nx + i] =
            zero ? czero<C>() : src[(int64_t)sys * lv.plane + (int64_t)(k + 1) * lv.pitch + i + 1];
}

__global__ __launch_bounds__(NT) void k_norm_finalize(const double* __restrict__ partial, int ntiles, int mode,
                                                      double tol, int fixed, double* bb, double* relres,
                                                      int* iters, int* active, const int* target, int* nanflag) {
    __shared__ double red[NT / 64];
    const int sys = blockIdx.x;
    if (mode == 1 && !active[sys]) return;
    double acc = 0.0;
    // strided per-thread sums in a fixed order, then the fixed-order block tree
    for (int t = threadIdx.x; t < ntiles; t += NT) acc += partial[(int64_t)sys * ntiles + t];
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x != 0) return;
    double sum = 0.0;
    for (int w = 0; w < NT / 64; ++w) sum += red[w];
    if (mode == 0) {
        bb[sys] = sum;
        iters[sys] = 0;
        const int on = (sum > 0.0) && (target[sys] > 0);
        active[sys] = on;
        relres[sys] = sum > 0.0 ? 1.0 : 0.0;
        nanflag[sys] = !(sum == sum) || sum > 1.0e300;
        if (nanflag[sys]) active[sys] = 0;
        return;
    }
    const int it = iters[sys] + 1;
    iters[sys] = it;
    const double rel = sqrt(sum / bb[sys]);
    relres[sys] = rel;
    if (!(rel == rel) || rel > 1.0e300) {
        nanflag[sys] = 1;
        active[sys] = 0;
    } else if (it >= target[sys] || (!fixed && rel <= tol)) {
        active[sys] = 0;
    }
}

__global__ void k_fill_int(int* p, int v, int n) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) p[t] = v;
}

inline dim3 grid2(int nx, int ny, int tx, int ty, int nsys) {
    return dim3((nx + tx - 1) / tx, (ny + ty - 1) / ty, nsys);
}

}  // namespace

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
// Fill z0 and the per-segment block extents; return the launch grid.
template <typename T> dim3 seg_grid(SegTable<T>& tab, const int* nsys, int tx, int ty, bool coarse_dims) {
    int z = 0, gx = 1, gy = 1;
    for (int q = 0; q < tab.n; ++q) {
        LevelSeg<T>& S = tab.s[q];
        const LevelView& v = coarse_dims ? S.lc : S.lf;
        S.z0 = z;
        S.gx = (v.nx + tx - 1) / tx;
        S.gy = (v.ny + ty - 1) / ty;
        gx = max(gx, S.gx);
        gy = max(gy, S.gy);
        z += nsys[q];
    }
    return dim3(gx, gy, z);
}

template <typename T> void launch_sweep(SegTable<T> tab, const int* nsys, hipStream_t st) {
    constexpr int TY = 16;
    const dim3 g = seg_grid(tab, nsys, 64, TY, false);
    hipLaunchKernelGGL((k_sweep<T, TY>), g, dim3(NT), 0, st, tab);
}

template <typename T> void launch_restrict(SegTable<T> tab, const int* nsys, hipStream_t st) {
    const dim3 g = seg_grid(tab, nsys, 32, 8, true);
    hipLaunchKernelGGL((k_restrict<T>), g, dim3(NT), 0, st, tab);
}

template <typename T> void launch_prolong(SegTable<T> tab, const int* nsys, hipStream_t st) {
    const dim3 g = seg_grid(tab, nsys, 64, 16, false);
    hipLaunchKernelGGL((k_prolong<T>), g, dim3(NT), 0, st, tab);
}

template <typename T> void launch_coarse(SegTable<T> tab, const int* nsys, hipStream_t st) {
    const dim3 g = seg_grid(tab, nsys, 1 << 20, 1 << 20, false);
    hipLaunchKernelGGL((k_coarse<T>), dim3(1, 1, g.z), dim3(NT), 0, st, tab);
}

int residual_tiles(LevelView lv) { return ((lv.nx + 63) / 64) * ((lv.ny + 15) / 16); }

template <typename T, typename TO>
int launch_residual(const cplx<T>* x, const cplx<T>* b, cplx<TO>* rout, LevelView lv, LevelView lo, T s,
                    const Coef<T>* coef, const int* active, int nsys, int x_zero, double* partial, hipStream_t st) {
    hipLaunchKernelGGL((k_residual<T, TO>), grid2(lv.nx, lv.ny, 64, 16, nsys), dim3(NT), 0, st, x, b, rout, lv, lo, s,
                       coef, active, x_zero, partial);
    return residual_tiles(lv);
}


int launch_ir_residual(const double2* x, const float2* e, const double2* b, double2* xn, float2* rout, LevelView lv,
                       LevelView le, double s, const Coef<double>* coef, const int* active, int nsys, double* partial,
                       hipStream_t st) {
    hipLaunchKernelGGL(k_ir_residual, grid2(lv.nx, lv.ny, 64, 16, nsys), dim3(NT), 0, st, x, e, b, xn, rout, lv, le, s,
                       coef, active, partial);
    return residual_tiles(lv);
}

template <typename T>
void launch_pack(const cplx<T>* src, cplx<T>* dst, LevelView lv, int nsys, hipStream_t st, double* partial) {
    hipLaunchKernelGGL((k_pack<T>), grid2(lv.nx, lv.ny, 64, 16, nsys), dim3(NT), 0, st, src, dst, lv, partial);
}

template <typename T>
void launch_unpack(const cplx<T>* src0, const cplx<T>* src1, cplx<T>* dst, LevelView lv, int nsys, const int* iters,
                   int flips, hipStream_t st) {
    hipLaunchKernelGGL((k_unpack<T>), grid2(lv.nx, lv.ny, 64, 16, nsys), dim3(NT), 0, st, src0, src1, dst, lv, iters,
                       flips);
}

void launch_norm_finalize(const double* partial, int ntiles, int nsys, int sys_off, int mode, double tol, int fixed,
                          double* bb, double* relres, int* iters, int* active, const int* target, int* nanflag,
                          hipStream_t st) {
    hipLaunchKernelGGL(k_norm_finalize, dim3(nsys), dim3(NT), 0, st, partial, ntiles, mode, tol, fixed, bb + sys_off,
                       relres + sys_off, iters + sys_off, active + sys_off, target + sys_off, nanflag + sys_off);
}

void launch_fill_int(int* p, int value, int n, hipStream_t st) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_fill_int, dim3((n + 255) / 256), dim3(256), 0, st, p, value, n);
}

#define VMG_INST(T)                                                                                              \
    template void launch_sweep<T>(SegTable<T>, const int*, hipStream_t);                                         \
    template void launch_restrict<T>(SegTable<T>, const int*, hipStream_t);                                      \
    template void launch_prolong<T>(SegTable<T>, const int*, hipStream_t);                                       \
    template void launch_coarse<T>(SegTable<T>, const int*, hipStream_t);                                        \
    template void launch_pack<T>(const cplx<T>*, cplx<T>*, LevelView, int, hipStream_t, double*);             \
    template void launch_unpack<T>(const cplx<T>*, const cplx<T>*, cplx<T>*, LevelView, int, const int*, int,  \
                                   hipStream_t);
VMG_INST(double)
VMG_INST(float)
template int launch_residual<double, double>(const double2*, const double2*, double2*, LevelView, LevelView, double,
                                             const Coef<double>*, const int*, int, int, double*, hipStream_t);
template int launch_residual<double, float>(const double2*, const double2*, float2*, LevelView, LevelView, double,
                                            const Coef<double>*, const int*, int, int, double*, hipStream_t);
template int launch_residual<float, float>(const float2*, const float2*, float2*, LevelView, LevelView, float,
                                           const Coef<float>*, const int*, int, int, double*, hipStream_t);

}  // namespace vmg
