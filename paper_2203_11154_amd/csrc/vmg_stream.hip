// Fused, register-streaming multigrid kernels for the large levels.
//
// One wave owns a strip of grid columns (lane = column) and walks down a
// block of rows.  Every stage of the level's work is a row-by-row stencil, so
// it runs a fixed number of rows behind the stage it consumes and keeps only
// three rows of each intermediate in registers; left and right neighbours
// come from the adjacent lanes.  Each stage loses one valid lane per side, so
// a wave owns the 64 - 2*HALO middle columns and neighbouring waves overlap by
// HALO columns (read again through L2).
//
//   k_down<NS>: x_0 = x; for s < NS: r_s = b - L x_s, x_{s+1} = x_s + M r_s
//               (the additive Vanka sweep of eq. (3) with the stencil of
//               eq. (6)); then r_NS = b - L x_NS and the coarse right-hand side
//               FW(r_NS).  Writes x_NS (NS > 0) and the coarse b; reads x and b
//               once.
//   k_up<NS>:   x_0 = x + P e (bilinear correction); NS sweeps as above;
//               optionally per-block sums of |b - L x_NS|^2 (the stopping
//               test on the finest level).  Writes x_NS; reads x, e, b once.
//
// Rows or columns outside the interior hold zero in every stage (Dirichlet
// ring for the iterates, zero residual off the interior).
#include "vmg_internal.h"

namespace vmg {

namespace {

constexpr int NT = 256;

template <typename C> __device__ __forceinline__ C z2() { C z; z.x = 0; z.y = 0; return z; }
template <typename C> __device__ __forceinline__ C add(C a, C b) { C r; r.x = a.x + b.x; r.y = a.y + b.y; return r; }
template <typename C> __device__ __forceinline__ C sub(C a, C b) { C r; r.x = a.x - b.x; r.y = a.y - b.y; return r; }
template <typename C, typename T> __device__ __forceinline__ C scl(C a, T s) { C r; r.x = a.x * s; r.y = a.y * s; return r; }
template <typename C> __device__ __forceinline__ C mul(C a, C b) {
    C r;
    r.x = a.x * b.x - a.y * b.y;
    r.y = a.x * b.y + a.y * b.x;
    return r;
}
template <typename C> __device__ __forceinline__ C fma2(C acc, C a, C b) {  // acc + a * b
    C r;
    r.x = acc.x + a.x * b.x - a.y * b.y;
    r.y = acc.y + a.x * b.y + a.y * b.x;
    return r;
}
// Value of the left (lane - 1) and right (lane + 1) neighbour; the wave's
// edge lanes receive values of no meaning and are never owned.  With
// VMG_NEIGHBOR_DPP the move is a DPP wave shift (wave_shr:1 / wave_shl:1, a
// VALU operand modifier; lane direction checked on gfx950), otherwise a
// cross-lane permute through the LDS crossbar.
#ifndef VMG_NEIGHBOR_DPP
#define VMG_NEIGHBOR_DPP 1
#endif
template <int CTRL> __device__ __forceinline__ float dpp_move(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, false));
}
template <int CTRL> __device__ __forceinline__ double dpp_move(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffLL), CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xF, 0xF, false);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
template <typename C> __device__ __forceinline__ C from_left(C v) {
    C r;
#if VMG_NEIGHBOR_DPP
    r.x = dpp_move<0x138>(v.x);
    r.y = dpp_move<0x138>(v.y);
#else
    r.x = __shfl_up(v.x, 1, 64);
    r.y = __shfl_up(v.y, 1, 64);
#endif
    return r;
}
template <typename C> __device__ __forceinline__ C from_right(C v) {
    C r;
#if VMG_NEIGHBOR_DPP
    r.x = dpp_move<0x130>(v.x);
    r.y = dpp_move<0x130>(v.y);
#else
    r.x = __shfl_down(v.x, 1, 64);
    r.y = __shfl_down(v.y, 1, 64);
#endif
    return r;
}

// three-row window, r[2] = newest row
template <typename C> struct Win {
    C r[3];
    __device__ __forceinline__ void init() { r[0] = r[1] = r[2] = z2<C>(); }
    __device__ __forceinline__ void push(C v) {
        r[0] = r[1];
        r[1] = r[2];
        r[2] = v;
    }
};

// residual of the middle row of an iterate window: b - (d x - s (W + E + N + S))
template <typename T, typename C>
__device__ __forceinline__ C residual_mid(const Win<C>& xw, C bv, C d, T s) {
    const C nb = add(add(from_left(xw.r[1]), from_right(xw.r[1])), add(xw.r[0], xw.r[2]));
    return sub(bv, sub(mul(d, xw.r[1]), scl(nb, s)));
}

// Vanka update of the middle row: x + ca r + cb (edge sum) + cc (corner sum),
// with nw holding the left+right neighbour sums of the r rows
template <typename T, typename C>
__device__ __forceinline__ C vanka_mid(C xc, const Win<C>& rw, const Win<C>& nw, const Coef<T>& cf) {
    const C edge = add(nw.r[1], add(rw.r[0], rw.r[2]));
    const C corner = add(nw.r[0], nw.r[2]);
    C v = fma2(xc, cf.ca, rw.r[1]);
    v = fma2(v, cf.cb, edge);
    return fma2(v, cf.cc, corner);
}

__device__ __forceinline__ bool in_rows(int k, int ny) { return k >= 1 && k <= ny; }

// ---------------------------------------------------------------------------
template <typename T, int NS>
__global__ __launch_bounds__(NT) void k_down(SegTable<T> tab, int ty) {
    using C = cplx<T>;
    constexpr int HALO = 2 * NS + 2;
    constexpr int OWN = 64 - 2 * HALO;
    constexpr int NB = 2 * NS + 1;  // b rows in flight
    const int lane = threadIdx.x & 63;
    const LevelSeg<T> S = seg_of(tab, blockIdx.z);
    const int sys = blockIdx.z - S.z0;
    if ((int)blockIdx.x >= S.gx || (int)blockIdx.y >= S.gy) return;
    if (!S.active[sys]) return;
    const LevelView lf = S.lf, lc = S.lc;
    const int x_zero = S.x_zero;
    const T s = S.s;
    const int c0 = 1 + (int)(blockIdx.x * (NT / 64) + (threadIdx.x >> 6)) * OWN;
    if (c0 > lf.nx) return;  // whole wave idle; no block barriers in this kernel
    const int i = c0 - HALO + lane;
    const bool col_in = i >= 1 && i <= lf.nx;
    const bool col_ld = i >= 0 && i <= lf.nx + 1;
    const bool own = lane >= HALO && lane < HALO + OWN && col_in;
    const int k0 = 1 + (int)blockIdx.y * ty;
    const int k1 = min(lf.ny, k0 + ty - 1);
    const int64_t base = (int64_t)sys * lf.plane;
    const C* xs = S.x + base;
    const C* bs = S.b + base;
    C* xos = S.xo + base;
    C* bcs = S.c + (int64_t)sys * lc.plane;
    const Coef<T> cf = S.coef[sys];

    Win<C> X[NS + 1], R[NS + 1], N[NS + 1];
#pragma unroll
    for (int q = 0; q <= NS; ++q) {
        X[q].init();
        R[q].init();
        N[q].init();
    }
    C B[NB];
#pragma unroll
    for (int q = 0; q < NB; ++q) B[q] = z2<C>();

    const int jbeg = k0 - 2 * NS - 2, jend = k1 + 2 * NS + 2;
    // rows are fetched one iteration ahead so their latency overlaps the
    // current row's arithmetic
    auto load_x = [&](int j) {
        C v = z2<C>();
        if (!x_zero && col_ld && j >= 0 && j <= lf.ny + 1) v = xs[(int64_t)j * lf.pitch + i];
        return v;
    };
    auto load_b = [&](int j) {
        C v = z2<C>();
        if (col_in && in_rows(j, lf.ny)) v = bs[(int64_t)j * lf.pitch + i];
        return v;
    };
    C xnext = load_x(jbeg), bnext = load_b(jbeg - 1);
    for (int j = jbeg; j <= jend; ++j) {
        // newest iterate row j and newest right-hand side row j - 1
        const C xn = xnext, bn = bnext;
        xnext = load_x(j + 1);
        bnext = load_b(j);
        X[0].push(xn);
#pragma unroll
        for (int q = 0; q < NB - 1; ++q) B[q] = B[q + 1];
        B[NB - 1] = bn;
#pragma unroll
        for (int q = 0; q <= NS; ++q) {
            // r_q at row j - 2q - 1 from x_q rows j - 2q - 2 .. j - 2q
            const int rrow = j - 2 * q - 1;
            C r = residual_mid<T>(X[q], B[NB - 1 - 2 * q], cf.d, s);
            if (!(col_in && in_rows(rrow, lf.ny))) r = z2<C>();
            R[q].push(r);
            N[q].push(add(from_left(r), from_right(r)));
            if (q < NS) {
                // x_{q+1} at row j - 2q - 2
                const int xrow = j - 2 * q - 2;
                C v = vanka_mid<T>(X[q].r[0], R[q], N[q], cf);
                if (!(col_in && in_rows(xrow, lf.ny))) v = z2<C>();
                X[q + 1].push(v);
            }
        }
        if (NS > 0) {
            const int orow = j - 2 * NS;
            if (own && orow >= k0 && orow <= k1) xos[(int64_t)orow * lf.pitch + i] = X[NS].r[2];
        }
        // full weighting around fine row j - 2NS - 2 (even rows carry coarse nodes)
        const int frow = j - 2 * NS - 2;
        if (own && !(frow & 1) && !(i & 1) && frow >= k0 && frow <= k1 && frow >= 2) {
            const Win<C>& rw = R[NS];
            const Win<C>& nw = N[NS];
            C v = scl(rw.r[1], (T)0.25);
            v = add(v, scl(add(nw.r[1], add(rw.r[0], rw.r[2])), (T)0.125));
            v = add(v, scl(add(nw.r[0], nw.r[2]), (T)0.0625));
            const int K = frow >> 1, I = i >> 1;
            if (K <= lc.ny && I <= lc.nx) bcs[(int64_t)K * lc.pitch + I] = v;
        }
    }
}

// ---------------------------------------------------------------------------
template <typename T, int NS, bool NORM>
__global__ __launch_bounds__(NT) void k_up(SegTable<T> tab, int ty) {
    using C = cplx<T>;
    constexpr int HALO = NORM ? 2 * NS + 1 : (NS > 0 ? 2 * NS : 1);
    constexpr int OWN = 64 - 2 * HALO;
    constexpr int NB = 2 * NS + 1;
    __shared__ double red[NT / 64];
    const int lane = threadIdx.x & 63;
    const LevelSeg<T> S = seg_of(tab, blockIdx.z);
    const int sys = blockIdx.z - S.z0;
    // both exits are uniform over the block (before its only barrier)
    if ((int)blockIdx.x >= S.gx || (int)blockIdx.y >= S.gy) return;
    if (!S.active[sys]) return;
    const LevelView lf = S.lf, lc = S.lc;
    const T s = S.s;
    double* partial = S.partial;
    const int c0 = 1 + (int)(blockIdx.x * (NT / 64) + (threadIdx.x >> 6)) * OWN;
    const bool wave_on = c0 <= lf.nx;
    const int i = c0 - HALO + lane;
    const bool col_in = wave_on && i >= 1 && i <= lf.nx;
    const bool own = lane >= HALO && lane < HALO + OWN && col_in;
    const int k0 = 1 + (int)blockIdx.y * ty;
    const int k1 = min(lf.ny, k0 + ty - 1);
    const int64_t base = (int64_t)sys * lf.plane;
    const C* xs = S.x + base;
    const C* bs = S.b + base;
    const C* es = S.c + (int64_t)sys * lc.plane;
    C* xos = S.xo + base;
    const Coef<T> cf = S.coef[sys];

    Win<C> X[NS + 1], R[NS + 1], N[NS + 1];
#pragma unroll
    for (int q = 0; q <= NS; ++q) {
        X[q].init();
        R[q].init();
        N[q].init();
    }
    C B[NB];
#pragma unroll
    for (int q = 0; q < NB; ++q) B[q] = z2<C>();
    double acc = 0.0;

    const int jbeg = k0 - 2 * NS - 1, jend = k1 + 2 * NS + 1;
    // Bilinear correction, streamed by coarse rows: lane i loads coarse column
    // i/2 of each coarse row once; an odd column averages it with its right
    // neighbour's value (coarse column (i+1)/2), fetched by a lane shift.
    // Fine row j uses the x-interpolated coarse rows j/2 (even j) or
    // (j-1)/2 and (j+1)/2 (odd j).  Raw loads of x, b and the next coarse row
    // are issued one row ahead and combined only when the row is consumed.
    const bool ecol = wave_on && i >= 0 && i <= lf.nx + 1;
    auto load_e = [&](int K) {
        C v = z2<C>();
        if (ecol && K >= 0 && K <= lc.ny + 1) v = es[(int64_t)K * lc.pitch + (i >> 1)];
        return v;
    };
    auto interp_x = [&](C v) {
        const C rv = from_right(v);
        return (i & 1) ? scl(add(v, rv), (T)0.5) : v;
    };
    auto load_x = [&](int j) {
        C v = z2<C>();
        if (col_in && in_rows(j, lf.ny)) v = xs[(int64_t)j * lf.pitch + i];
        return v;
    };
    auto load_b = [&](int j) {
        C v = z2<C>();
        if (col_in && in_rows(j, lf.ny)) v = bs[(int64_t)j * lf.pitch + i];
        return v;
    };
    if (wave_on) {
        C e_lo = z2<C>(), e_hi = z2<C>(), e_raw = z2<C>();
        if (jbeg & 1) {
            e_hi = interp_x(load_e((jbeg - 1) >> 1));
            e_raw = load_e((jbeg + 1) >> 1);
        } else {
            e_hi = interp_x(load_e(jbeg >> 1));
        }
        C xnext = load_x(jbeg), bnext = load_b(jbeg - 1);
        for (int j = jbeg; j <= jend; ++j) {
            const C xr = xnext, bn = bnext;
            xnext = load_x(j + 1);
            bnext = load_b(j);
            if (j & 1) {
                e_lo = e_hi;                 // coarse row (j - 1) / 2
                e_hi = interp_x(e_raw);      // coarse row (j + 1) / 2
            } else {
                e_raw = load_e((j + 2) >> 1);  // needed by row j + 1
            }
            C xn = z2<C>();
            if (col_in && in_rows(j, lf.ny)) xn = add(xr, (j & 1) ? scl(add(e_lo, e_hi), (T)0.5) : e_hi);
            X[0].push(xn);
#pragma unroll
            for (int q = 0; q < NB - 1; ++q) B[q] = B[q + 1];
            B[NB - 1] = bn;
#pragma unroll
            for (int q = 0; q <= NS; ++q) {
                if (q == NS && !NORM) break;
                const int rrow = j - 2 * q - 1;
                C r = residual_mid<T>(X[q], B[NB - 1 - 2 * q], cf.d, s);
                if (!(col_in && in_rows(rrow, lf.ny))) r = z2<C>();
                if (q == NS) {
                    if (own && rrow >= k0 && rrow <= k1) acc += (double)r.x * (double)r.x + (double)r.y * (double)r.y;
                    break;
                }  // (the sum is written only for segments with a partial buffer)
                R[q].push(r);
                N[q].push(add(from_left(r), from_right(r)));
                const int xrow = j - 2 * q - 2;
                C v = vanka_mid<T>(X[q].r[0], R[q], N[q], cf);
                if (!(col_in && in_rows(xrow, lf.ny))) v = z2<C>();
                X[q + 1].push(v);
            }
            const int orow = j - 2 * NS;
            if (own && orow >= k0 && orow <= k1) xos[(int64_t)orow * lf.pitch + i] = X[NS].r[2];
        }
    }
    if (NORM && partial) {
        for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
        if (lane == 0) red[threadIdx.x >> 6] = acc;
        __syncthreads();
        if (threadIdx.x == 0) {
            double t = 0.0;
            for (int w = 0; w < NT / 64; ++w) t += red[w];
            partial[(int64_t)sys * (S.gx * S.gy) + blockIdx.y * S.gx + blockIdx.x] = t;
        }
    }
}

template <typename T>
__global__ __launch_bounds__(NT) void k_fill_zero(cplx<T>* __restrict__ x, LevelView lv) {
    const int i = blockIdx.x * 64 + (threadIdx.x & 63) + 1;
    if (i > lv.nx) return;
    for (int k = blockIdx.y * 16 + (threadIdx.x >> 6) + 1; k <= min(lv.ny, (int)(blockIdx.y + 1) * 16); k += NT / 64)
        x[(int64_t)blockIdx.z * lv.plane + (int64_t)k * lv.pitch + i] = z2<cplx<T>>();
}

template <int NS> constexpr int down_own() { return 64 - 2 * (2 * NS + 2); }
template <int NS, bool NORM> constexpr int up_own() { return 64 - 2 * (NORM ? 2 * NS + 1 : (NS > 0 ? 2 * NS : 1)); }

inline dim3 stream_grid(int nx, int ny, int own, int ty, int nsys) {
    const int tiles = (nx + own - 1) / own;
    return dim3((tiles + NT / 64 - 1) / (NT / 64), (ny + ty - 1) / ty, nsys);
}

template <typename T> dim3 stream_seg_grid(SegTable<T>& tab, const int* nsys, int own, int ty) {
    int z = 0, gx = 1, gy = 1;
    for (int q = 0; q < tab.n; ++q) {
        LevelSeg<T>& S = tab.s[q];
        const dim3 g = stream_grid(S.lf.nx, S.lf.ny, own, ty, 1);
        S.z0 = z;
        S.gx = (int)g.x;
        S.gy = (int)g.y;
        gx = max(gx, S.gx);
        gy = max(gy, S.gy);
        z += nsys[q];
    }
    return dim3(gx, gy, z);
}

}  // namespace

int stream_tiles(int nx, int ny, int nu, bool norm, int ty) {
    int own = 0;
    switch (nu) {
        case 0: own = norm ? up_own<0, true>() : up_own<0, false>(); break;
        case 1: own = norm ? up_own<1, true>() : up_own<1, false>(); break;
        default: own = norm ? up_own<2, true>() : up_own<2, false>(); break;
    }
    const dim3 g = stream_grid(nx, ny, own, ty, 1);
    return (int)(g.x * g.y);
}

template <typename T> void launch_down(SegTable<T> tab, const int* nsys, int nu, int ty, hipStream_t st) {
    switch (nu) {
        case 0: {
            const dim3 g = stream_seg_grid(tab, nsys, down_own<0>(), ty);
            hipLaunchKernelGGL((k_down<T, 0>), g, dim3(NT), 0, st, tab, ty);
            break;
        }
        case 1: {
            const dim3 g = stream_seg_grid(tab, nsys, down_own<1>(), ty);
            hipLaunchKernelGGL((k_down<T, 1>), g, dim3(NT), 0, st, tab, ty);
            break;
        }
        default: {
            const dim3 g = stream_seg_grid(tab, nsys, down_own<2>(), ty);
            hipLaunchKernelGGL((k_down<T, 2>), g, dim3(NT), 0, st, tab, ty);
            break;
        }
    }
}

template <typename T> void launch_up(SegTable<T> tab, const int* nsys, int nu, bool norm, int ty, hipStream_t st) {
#define VMG_UP(NSV, NORMV)                                                          \
    do {                                                                            \
        const dim3 g = stream_seg_grid(tab, nsys, up_own<NSV, NORMV>(), ty);        \
        hipLaunchKernelGGL((k_up<T, NSV, NORMV>), g, dim3(NT), 0, st, tab, ty);     \
    } while (0)
    switch (nu) {
        case 0: if (norm) VMG_UP(0, true); else VMG_UP(0, false); break;
        case 1: if (norm) VMG_UP(1, true); else VMG_UP(1, false); break;
        default: if (norm) VMG_UP(2, true); else VMG_UP(2, false); break;
    }
#undef VMG_UP
}

template <typename T> void launch_fill_zero(cplx<T>* x, LevelView lv, int nsys, hipStream_t st) {
    hipLaunchKernelGGL((k_fill_zero<T>), dim3((lv.nx + 63) / 64, (lv.ny + 15) / 16, nsys), dim3(NT), 0, st, x, lv);
}
template void launch_fill_zero<double>(double2*, LevelView, int, hipStream_t);
template void launch_fill_zero<float>(float2*, LevelView, int, hipStream_t);

template void launch_down<double>(SegTable<double>, const int*, int, int, hipStream_t);
template void launch_down<float>(SegTable<float>, const int*, int, int, hipStream_t);
template void launch_up<double>(SegTable<double>, const int*, int, bool, int, hipStream_t);
template void launch_up<float>(SegTable<float>, const int*, int, bool, int, hipStream_t);

}  // namespace vmg
