// The small levels of a multigrid cycle in one workgroup per system.
//
// Below a few thousand nodes per system a level's kernels are bound by launch
// and drain latency, not by bandwidth.  Here one 1024-thread workgroup runs,
// for one system, the whole cycle MG(lt, x, b) of the levels lt..coarsest
// (sweeps of eqs. (3)/(6), residual and full weighting, gamma recursive
// visits of the next level, bilinear correction, and the direct coarsest
// solve) with every iterate, right-hand side and residual of those levels in
// LDS; only b of level lt is read from global memory (L2), and x of level lt
// is read (unless it starts at zero) and written back once.
//
// LDS layout for a tail whose first level has P0 = (nx+2)(ny+2) padded nodes:
//   region A  [0, P0)          x of level lt
//   region B  [P0, P0 + Q)     the residual of level lt, or (while a deeper
//                              level is active, when that residual is dead)
//                              x and b of every deeper level followed by one
//                              residual buffer shared by the deeper levels.
// Restriction from level lt writes b of level lt+1 over its own residual, so
// the full-weighting values are formed in registers first and stored after a
// barrier.  Every array keeps a zero ring.
#include "vmg_internal.h"

#include <algorithm>

namespace vmg {

namespace {

constexpr int TT = 1024;  // threads per workgroup (16 waves)

__device__ __forceinline__ int padded(const LevelView& v) { return (v.nx + 2) * (v.ny + 2); }

// A tail level's constants for the workgroup's system, gathered into LDS
// once per launch: read from the segment table in global memory (scalar
// loads, the offsets by loops over the levels) they cost every step of a
// cycle about 1,500 clocks before its first node.
template <typename T> struct alignas(16) TailLevel {
    Coef<T> cf;
    T s;
    int nx, ny;
    int xo, bo, ro;      // element offsets of x, b (l >= 1) and the residual of the level
    float inx, ipitch;   // 1 / nx and 1 / (nx + 2), for qdiv
};

// t / p for 0 <= t < 2^16 and p >= 1, from the float reciprocal ip of p: the
// float quotient is then within 1e-3 of t / p, and one correction makes it
// exact (a fraction of the instructions of an integer division)
__device__ __forceinline__ int qdiv(int t, int p, float ip) {
    int q = (int)((float)t * ip);
    const int r = t - q * p;
    q += (r >= p ? 1 : 0) - (r < 0 ? 1 : 0);
    return q;
}

template <typename T> struct TailView {
    const TailSeg<T>* S;
    int sys;
    cplx<T>* lds;
    const TailLevel<T>* L;  // per level, in LDS
    __device__ LevelView lv(int l) const {
        LevelView v;
        v.nx = L[l].nx;
        v.ny = L[l].ny;
        v.pitch = v.nx + 2;
        v.plane = 0;
        return v;
    }
    __device__ int xo(int l) const { return L[l].xo; }
    __device__ int bo(int l) const { return L[l].bo; }
    __device__ int ro(int l) const { return L[l].ro; }
};

// Level l's entry of the table (offsets as laid out in the header comment).
template <typename T> __device__ void fill_level(TailLevel<T>& e, const TailSeg<T>* S, int sys, int l) {
    e.cf = S->coef[l][sys];
    e.s = S->s[l];
    e.nx = S->lv[l].nx;
    e.ny = S->lv[l].ny;
    const int p0 = padded(S->lv[0]);
    int xo = 0;
    if (l > 0) {
        xo = p0;
        for (int q = 1; q < l; ++q) xo += 2 * padded(S->lv[q]);
    }
    int ro = p0;
    if (l > 0)
        for (int q = 1; q < S->nl; ++q) ro += 2 * padded(S->lv[q]);
    e.xo = xo;
    e.bo = xo + padded(S->lv[l]);
    e.ro = ro;
    e.inx = 1.0f / (float)e.nx;
    e.ipitch = 1.0f / (float)(e.nx + 2);
}

template <typename T> __device__ __forceinline__ cplx<T> load_b0(const TailView<T>& V, int k, int i) {
    const LevelView g = V.S->gv;
    return V.S->b[(int64_t)V.sys * g.plane + (int64_t)k * g.pitch + i];
}

// The first tail level's padded nodes a thread visits, t = threadIdx.x + j TT
// (j < JMAX), with their right-hand side kept in registers and a bit per
// node that is set on the interior: the level's passes then read no global
// memory and divide by nothing.  JMAX bounds the nodes per thread of any
// first level whose x and residual fit in LDS (the host checks it).
template <typename T> struct Level0 {
    static constexpr int JMAX = tail_first_nodes_max<T>() / TT;
    cplx<T> b[JMAX];
    unsigned in;
};

// r = b - L x on every padded node of level l (zero on the ring)
template <typename T> __device__ void residual_first(const TailView<T>& V, const Level0<T>& f) {
    using C = cplx<T>;
    const LevelView v = V.lv(0);
    const int pitch = v.nx + 2, P = padded(v);
    const Coef<T> cf = V.L[0].cf;
    const T s = V.L[0].s;
    const C* x = V.lds;
    C* r = V.lds + V.ro(0);
#pragma unroll
    for (int j = 0; j < Level0<T>::JMAX; ++j) {
        const int t = threadIdx.x + j * TT;
        if (t < P) {
            C rv = czero<C>();
            if ((f.in >> j) & 1u) {
                const C nb = cadd(cadd(x[t - pitch], x[t + pitch]), cadd(x[t - 1], x[t + 1]));
                rv = csub(f.b[j], csub(cmul(cf.d, x[t]), cscale(nb, s)));
            }
            r[t] = rv;
        }
    }
    __syncthreads();
}

template <typename T> __device__ void residual(const TailView<T>& V, int l, const Level0<T>& f) {
    using C = cplx<T>;
    if (l == 0) {
        residual_first(V, f);
        return;
    }
    const LevelView v = V.lv(l);
    const int pitch = v.nx + 2, P = padded(v);
    const Coef<T> cf = V.L[l].cf;
    const T s = V.L[l].s;
    const C* x = V.lds + V.xo(l);
    const C* b = V.lds + V.bo(l);
    C* r = V.lds + V.ro(l);
    for (int t = threadIdx.x; t < P; t += TT) {
        const int k = qdiv(t, pitch, V.L[l].ipitch), i = t - k * pitch;
        C rv = czero<C>();
        if (i >= 1 && i <= v.nx && k >= 1 && k <= v.ny) {
            const C bv = b[t];
            const C nb = cadd(cadd(x[t - pitch], x[t + pitch]), cadd(x[t - 1], x[t + 1]));
            rv = csub(bv, csub(cmul(cf.d, x[t]), cscale(nb, s)));
        }
        r[t] = rv;
    }
    __syncthreads();
}

template <typename T, typename C>
__device__ __forceinline__ void vanka_node(C* x, const C* r, int c, int pitch, const Coef<T>& cf) {
    const C edge = cadd(cadd(r[c - pitch], r[c + pitch]), cadd(r[c - 1], r[c + 1]));
    const C corner = cadd(cadd(r[c - pitch - 1], r[c - pitch + 1]), cadd(r[c + pitch - 1], r[c + pitch + 1]));
    C u = cfma(x[c], cf.ca, r[c]);
    u = cfma(u, cf.cb, edge);
    x[c] = cfma(u, cf.cc, corner);
}

// x += ca r + cb (edge sum of r) + cc (corner sum of r), in place
template <typename T> __device__ void smooth(const TailView<T>& V, int l, const Level0<T>& f) {
    using C = cplx<T>;
    residual(V, l, f);
    const LevelView v = V.lv(l);
    const int pitch = v.nx + 2;
    const Coef<T> cf = V.L[l].cf;
    C* x = V.lds + V.xo(l);
    const C* r = V.lds + V.ro(l);
    if (l == 0) {
#pragma unroll
        for (int j = 0; j < Level0<T>::JMAX; ++j)
            if ((f.in >> j) & 1u) vanka_node<T>(x, r, (int)threadIdx.x + j * TT, pitch, cf);
        __syncthreads();
        return;
    }
    for (int t = threadIdx.x; t < v.nx * v.ny; t += TT) {
        const int k = qdiv(t, v.nx, V.L[l].inx) + 1, i = t - (k - 1) * v.nx + 1;
        vanka_node<T>(x, r, k * pitch + i, pitch, cf);
    }
    __syncthreads();
}

// b_{l+1} = FW(b - L x) at level l; x_{l+1} = 0 (ring included)
template <typename T> __device__ void restrict_down(const TailView<T>& V, int l, const Level0<T>& f) {
    using C = cplx<T>;
    residual(V, l, f);
    const LevelView v = V.lv(l), vc = V.lv(l + 1);
    const int pitch = v.nx + 2, pc = vc.nx + 2;
    const C* r = V.lds + V.ro(l);
    // one coarse node per thread (the host keeps the coarse levels of a tail
    // at most TT nodes)
    const int t = threadIdx.x;
    C val = czero<C>();
    const bool on = t < vc.nx * vc.ny;
    int cc = 0;
    if (on) {
        const int K = qdiv(t, vc.nx, V.L[l + 1].inx) + 1, I = t - (K - 1) * vc.nx + 1;
        const int c = 2 * K * pitch + 2 * I;
        const C edge = cadd(cadd(r[c - pitch], r[c + pitch]), cadd(r[c - 1], r[c + 1]));
        const C corner = cadd(cadd(r[c - pitch - 1], r[c - pitch + 1]), cadd(r[c + pitch - 1], r[c + pitch + 1]));
        val = cscale(r[c], (T)0.25);
        val = cadd(val, cscale(edge, (T)0.125));
        val = cadd(val, cscale(corner, (T)0.0625));
        cc = K * pc + I;
    }
    __syncthreads();  // every read of this level's residual is done
    C* xc = V.lds + V.xo(l + 1);
    C* bc = V.lds + V.bo(l + 1);
    for (int q = threadIdx.x; q < padded(vc); q += TT) xc[q] = czero<C>();
    if (on) bc[cc] = val;
    __syncthreads();
}

// x_l += P x_{l+1} (bilinear; the coarse ring holds zeros)
template <typename T> __device__ void prolong_up(const TailView<T>& V, int l) {
    using C = cplx<T>;
    const LevelView v = V.lv(l), vc = V.lv(l + 1);
    const int pitch = v.nx + 2, pc = vc.nx + 2;
    C* x = V.lds + V.xo(l);
    const C* e = V.lds + V.xo(l + 1);
    for (int t = threadIdx.x; t < v.nx * v.ny; t += TT) {
        const int k = qdiv(t, v.nx, V.L[l].inx) + 1, i = t - (k - 1) * v.nx + 1;
        const int il = i >> 1, ir = (i + 1) >> 1, kl = k >> 1, kr = (k + 1) >> 1;
        C w;
        if (!(i & 1) && !(k & 1)) {
            w = e[kl * pc + il];
        } else {
            const C row0 = (i & 1) ? cadd(e[kl * pc + il], e[kl * pc + ir]) : e[kl * pc + il];
            const C row1 = (i & 1) ? cadd(e[kr * pc + il], e[kr * pc + ir]) : e[kr * pc + il];
            w = (k & 1) ? cadd(row0, row1) : row0;
            w = cscale(w, (T)((i & 1) ? 0.5 : 1.0) * (T)((k & 1) ? 0.5 : 1.0));
        }
        const int c = k * pitch + i;
        x[c] = cadd(x[c], w);
    }
    __syncthreads();
}

// coarsest level: x = (A_c + lambda I)^{-1} b by the precomputed inverse
template <typename T> __device__ void coarse_solve(const TailView<T>& V, int l) {
    using C = cplx<T>;
    const LevelView v = V.lv(l);
    const int pitch = v.nx + 2, nc = V.S->nc;
    C* x = V.lds + V.xo(l);
    C* sb = V.lds + V.ro(l);  // right-hand side gathered densely (scratch)
    for (int t = threadIdx.x; t < nc; t += TT) {
        const int k = qdiv(t, v.nx, V.L[l].inx) + 1, i = t - (k - 1) * v.nx + 1;
        sb[t] = l == 0 ? load_b0(V, k, i) : V.lds[V.bo(l) + k * pitch + i];
    }
    __syncthreads();
    // CS consecutive lanes share an output row: lane q sums the products of
    // k = q, q + CS, ... (all its loads in flight at once), and the lanes'
    // sums meet in a fixed shuffle order
    constexpr int CS = 16;
    const C* ci = V.S->cinvT + (int64_t)V.sys * nc * nc;
    const int q = threadIdx.x & (CS - 1);
    for (int t0 = 0; t0 < nc; t0 += TT / CS) {
        const int t = t0 + (int)threadIdx.x / CS;
        C acc = czero<C>();
        if (t < nc)
            for (int k = q; k < nc; k += CS) acc = cfma(acc, ci[(int64_t)k * nc + t], sb[k]);
        for (int off = CS / 2; off > 0; off >>= 1) {
            acc.x += __shfl_xor(acc.x, off, 64);
            acc.y += __shfl_xor(acc.y, off, 64);
        }
        if (t < nc && q == 0) {
            const int kk = qdiv(t, v.nx, V.L[l].inx) + 1, i = t - (kk - 1) * v.nx + 1;
            x[kk * pitch + i] = acc;
        }
    }
    __syncthreads();
}

template <typename T>
__global__ __launch_bounds__(TT) void k_tail(const TailSeg<T>* __restrict__ segs, TailLaunch<T> tl, int nu1, int nu2,
                                             int gamma) {
    using C = cplx<T>;
    extern __shared__ __align__(16) double tail_lds[];
    // entry of this workgroup (selected without indexing the argument arrays)
    int seg = tl.seg[0], z0 = tl.z0[0], xz = tl.xz[0], sys0 = tl.sys0[0];
    C* xg = tl.x[0];
#pragma unroll
    for (int j = 1; j < MAXSEG; ++j)
        if (j < tl.n && (int)blockIdx.x >= tl.z0[j]) {
            seg = tl.seg[j];
            z0 = tl.z0[j];
            xz = tl.xz[j];
            xg = tl.x[j];
            sys0 = tl.sys0[j];
        }
    TailView<T> V;
    V.S = segs + seg;
    V.sys = (int)blockIdx.x - z0;
    V.lds = reinterpret_cast<C*>(tail_lds);
    if (!V.S->active[V.sys]) return;  // uniform over the workgroup
    const int nl = V.S->nl;
    __shared__ TailLevel<T> tlev[MAXT];
    if ((int)threadIdx.x < nl) fill_level(tlev[threadIdx.x], V.S, V.sys, (int)threadIdx.x);
    V.L = tlev;  // (read after the barrier below)
    const LevelView v0 = V.S->lv[0], g0 = V.S->gv;
    C* x0 = V.lds;
    C* gx = xg + (int64_t)V.sys * g0.plane;
    Level0<T> f;
    f.in = 0u;
#pragma unroll
    for (int j = 0; j < Level0<T>::JMAX; ++j) {
        const int t = threadIdx.x + j * TT;
        const int k = t / (v0.nx + 2), i = t - k * (v0.nx + 2);
        const bool inner = t < padded(v0) && i >= 1 && i <= v0.nx && k >= 1 && k <= v0.ny;
        f.b[j] = inner ? load_b0(V, k, i) : czero<C>();
        f.in |= (inner ? 1u : 0u) << j;
        if (t < padded(v0)) x0[t] = (xz || !inner) ? czero<C>() : gx[(int64_t)k * g0.pitch + i];
    }
    __syncthreads();
    // whole solves: cycles until the system stops (at most tl.maxc); else one.
    // red: the per-wave norm sums and (last slot) the go-on flag; 144 bytes,
    // so that the static LDS (with the level table, whose entries are 16-byte
    // aligned) stays a multiple of 16 bytes and the dynamic LDS after it
    // 16-byte aligned for the double2 accesses
    __shared__ __align__(16) double red[TT / 64 + 2];
    const int ncyc = tl.maxc > 0 ? tl.maxc : 1;
    for (int cyc = 0; cyc < ncyc; ++cyc) {
    // MG(0) with gamma visits of every coarser level, without recursion:
    // cnt holds, 4 bits per level, the visits of the next level made so far
    unsigned cnt = 0;
    int l = 0;
    bool down = true;
    for (;;) {
        if (down) {
            if (l == nl - 1) {
                coarse_solve(V, l);
                down = false;
                continue;
            }
            for (int it = 0; it < nu1; ++it) smooth(V, l, f);
            restrict_down(V, l, f);
            cnt &= ~(15u << (4 * l));
            ++l;
            continue;
        }
        if (l == 0) break;
        const int p = l - 1;
        const unsigned c = ((cnt >> (4 * p)) & 15u) + 1u;
        cnt = (cnt & ~(15u << (4 * p))) | (c << (4 * p));
        if ((int)c < gamma) {
            down = true;  // another visit of level l, from its current iterate
            continue;
        }
        prolong_up(V, p);
        for (int it = 0; it < nu2; ++it) smooth(V, p, f);
        l = p;
    }
    if (tl.maxc == 0) break;
    // the stopping test of k_norm_finalize on |b - L x|^2 of the finest
    // level (fixed-order sums: per thread, wave, then the waves in order)
    residual_first(V, f);
    {
        const C* r = V.lds + V.ro(0);
        double acc = 0.0;
#pragma unroll
        for (int j = 0; j < Level0<T>::JMAX; ++j)
            if ((f.in >> j) & 1u) {
                const C rv = r[threadIdx.x + j * TT];
                acc += (double)rv.x * (double)rv.x + (double)rv.y * (double)rv.y;
            }
        for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
        if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double sum = 0.0;
        for (int w = 0; w < TT / 64; ++w) sum += red[w];
        const int gs = sys0 + V.sys;
        const int it = tl.iters[gs] + 1;
        tl.iters[gs] = it;
        const double rel = sqrt(sum / tl.bb[gs]);
        tl.relres[gs] = rel;
        int on = 1;
        if (!(rel == rel) || rel > 1.0e300) {
            tl.nanflag[gs] = 1;
            on = 0;
        } else if (it >= tl.target[gs] || (!tl.fixed && rel <= tl.tol)) {
            on = 0;
        }
        if (!on) tl.active[gs] = 0;
        red[TT / 64] = on ? 1.0 : 0.0;
    }
    __syncthreads();
    if (red[TT / 64] == 0.0) break;
    }
    for (int t = threadIdx.x; t < v0.nx * v0.ny; t += TT) {
        const int k = t / v0.nx + 1, i = t - (k - 1) * v0.nx + 1;
        gx[(int64_t)k * g0.pitch + i] = x0[k * (v0.nx + 2) + i];
    }
}

}  // namespace

template <typename T> int64_t tail_lds_bytes(const LevelView* lv, int nl) {
    auto pad = [](const LevelView& v) { return (int64_t)(v.nx + 2) * (v.ny + 2); };
    int64_t a = pad(lv[0]);
    int64_t deep = 0;
    for (int q = 1; q < nl; ++q) deep += 2 * pad(lv[q]);
    if (nl > 1) deep += pad(lv[1]);  // residual buffer shared by the deeper levels
    int64_t b = std::max(pad(lv[0]), deep);
    // the coarsest solve gathers its right-hand side into the residual buffer
    return (a + b) * (int64_t)sizeof(cplx<T>);
}
template int64_t tail_lds_bytes<double>(const LevelView*, int);
template int64_t tail_lds_bytes<float>(const LevelView*, int);

int tail_max_lds() {
    static int max_lds = -1;
    if (max_lds < 0) {
        int dev = 0, v = 0;
        if (hipGetDevice(&dev) != hipSuccess) dev = 0;
        if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess) v = 65536;
        // (less the kernel's own static LDS: the per-level constants and the
        // whole-solve reduction slots)
        max_lds = v - 1280;
        // allow the dynamic allocation above the default limit
        (void)hipFuncSetAttribute((const void*)&k_tail<double>, hipFuncAttributeMaxDynamicSharedMemorySize, max_lds);
        (void)hipFuncSetAttribute((const void*)&k_tail<float>, hipFuncAttributeMaxDynamicSharedMemorySize, max_lds);
        (void)hipGetLastError();
    }
    return max_lds;
}

template <typename T>
void launch_tail(const TailSeg<T>* segs, const TailLaunch<T>& tl, int total_sys, int64_t lds_bytes, int nu1, int nu2,
                 int gamma, hipStream_t st) {
    if (total_sys <= 0) return;
    hipLaunchKernelGGL((k_tail<T>), dim3(total_sys), dim3(TT), (size_t)lds_bytes, st, segs, tl, nu1, nu2, gamma);
}
template void launch_tail<double>(const TailSeg<double>*, const TailLaunch<double>&, int, int64_t, int, int, int,
                                  hipStream_t);
template void launch_tail<float>(const TailSeg<float>*, const TailLaunch<float>&, int, int64_t, int, int, int,
                                 hipStream_t);

}  // namespace vmg
