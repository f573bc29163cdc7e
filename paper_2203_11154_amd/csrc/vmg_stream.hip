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
//               As the finishing pass it rebuilds the last cycle's iterate
//               of every system from the inputs of that cycle's k_edge pass
//               and writes it to a dense output.
//   k_edge<NA, NB>: the finest level across the boundary of two V-cycles:
//               k_up<NA> with the stopping-test sums, then k_down<NB> from its
//               result, in one pass (reads x, b, e once; writes the next
//               cycle's pre-smoothed iterate and coarse right-hand side).
//
// The last template argument of each kernel is the precision of the coarse
// level it writes (the restricted residual) and reads (the correction e): the
// level's own, or complex64 under an FP64 level when the coarse-grid
// correction runs in complex64; values are rounded to it as they are stored
// and widened (exactly) as they are read.
//
// Rows or columns outside the interior hold zero in every stage (Dirichlet
// ring for the iterates, zero residual off the interior).
#include "vmg_internal.h"

#include <algorithm>
#include <type_traits>
#include <map>
#include <mutex>

namespace vmg {

namespace {

constexpr int NT = 256;

// a * b + c rounded once, in the precision of the operands
__device__ __forceinline__ double fmar(double a, double b, double c) { return __builtin_fma(a, b, c); }
__device__ __forceinline__ float fmar(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
// complex value in another precision (round to nearest; the identity when
// the types agree)
template <typename D, typename S> __device__ __forceinline__ D cvt(S v) {
    if constexpr (std::is_same<D, S>::value) {
        return v;
    } else {
        D r;
        r.x = v.x;
        r.y = v.y;
        return r;
    }
}
// Value of the left (lane - 1) and right (lane + 1) neighbour; the wave's
// edge lanes receive values of no meaning and are never owned.  The move is a
// DPP wave shift (wave_shr:1 / wave_shl:1, a VALU operand modifier; lane
// direction checked on gfx950).
template <int CTRL> __device__ __forceinline__ int dpp_move_i(int v) {
    // bound_ctrl set: a lane whose source is off the wave receives 0, so no
    // "old" operand has to be materialised
    return __builtin_amdgcn_mov_dpp(v, CTRL, 0xF, 0xF, true);
}
template <int CTRL> __device__ __forceinline__ float dpp_move(float v) {
    return __int_as_float(dpp_move_i<CTRL>(__float_as_int(v)));
}
template <int CTRL> __device__ __forceinline__ double dpp_move(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = dpp_move_i<CTRL>((int)(b & 0xffffffffLL));
    const int hi = dpp_move_i<CTRL>((int)(b >> 32));
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
template <typename C> __device__ __forceinline__ C from_left(C v) {
    C r;
    r.x = dpp_move<0x138>(v.x);
    r.y = dpp_move<0x138>(v.y);
    return r;
}
template <typename C> __device__ __forceinline__ C from_right(C v) {
    C r;
    r.x = dpp_move<0x130>(v.x);
    r.y = dpp_move<0x130>(v.y);
    return r;
}

// Left + right neighbour sum.
template <typename C> __device__ __forceinline__ C lr_sum(C v) { return cadd(from_left(v), from_right(v)); }

// Residual of a middle row: b - (d x - s (W + E + N + S)), from the rows
// above (xo), at (xm) and below (xn); three fused multiply-adds a component
// after the neighbour sum.
template <typename T, typename C>
__device__ __forceinline__ C residual_row(C xo, C xm, C xn, C bv, C d, T s) {
    const C nb = cadd(lr_sum(xm), cadd(xo, xn));
    C r;
    r.x = fmar(d.y, xm.y, fmar(-d.x, xm.x, fmar(s, nb.x, bv.x)));
    r.y = fmar(-d.y, xm.x, fmar(-d.x, xm.y, fmar(s, nb.y, bv.y)));
    return r;
}

// Vanka update of a middle row from the residual rows above (ro), at (rm)
// and below (rn):  x + ca r + cb (edge sum) + cc (corner sum).  With
// vs = ro + rn the edge sum is vs + LR(rm) and the corner sum LR(vs); the lane
// shifts commute with the (uniform) coefficients, so with alpha = ca / cb and
// gamma = cc / cb (per system and level) the update takes one neighbour sum
// and three complex multiply-adds:
//   x + cb (alpha rm + vs + LR(rm + gamma vs)).
// Off the interior (mk = 0) every term but the neighbour sum is zero already
// (zero iterate and residual there); mk multiplies that sum, so the update is
// zero there without a select.  JAC: the damped Jacobi smoother, x + ca r.
template <typename T, bool JAC, typename C>
__device__ __forceinline__ C vanka_row(C xc, C ro, C rm, C rn, const Coef<T>& cf, T mk) {
    if constexpr (JAC) {
        return cfma(xc, cf.ca, rm);
    } else {
        const C vs = cadd(ro, rn);
        const C t = cfma(rm, cf.gamma, vs);
        C u = cfma(vs, cf.alpha, rm);
        const C lr = lr_sum(t);
        u.x = fmar(mk, lr.x, u.x);
        u.y = fmar(mk, lr.y, u.y);
        return cfma(xc, cf.cb, u);
    }
}

// Full weighting around a middle row, the same way: with
// w = rm/8 + (ro + rn)/16 it is rm/4 + (ro + rn)/8 + LR(w) = 2 w + LR(w).
template <typename T, typename C> __device__ __forceinline__ C full_weight_row(C ro, C rm, C rn) {
    const C vs = cadd(ro, rn);
    C w;
    w.x = fmar(vs.x, (T)0.0625, rm.x * (T)0.125);
    w.y = fmar(vs.y, (T)0.0625, rm.y * (T)0.125);
    const C lr = lr_sum(w);
    C r;
    r.x = fmar((T)2, w.x, lr.x);
    r.y = fmar((T)2, w.y, lr.y);
    return r;
}

__device__ __forceinline__ bool in_rows(int k, int ny) { return k >= 1 && k <= ny; }

// Plane access through buffer resources.  The hardware range check returns
// zero for a load, and drops a store, at a byte offset at or beyond the
// plane's size; an invalid row or column therefore just adds OOB to the
// offset (planes are kept below 1 GiB, so any sum holding OOB is out of
// range).  Loads and stores then need no branches, which keeps the memory
// counter waits exact and lets rows be fetched ahead.
constexpr unsigned OOB = 0x40000000u;
using rsrc_t = __amdgpu_buffer_rsrc_t;
template <typename C> __device__ __forceinline__ rsrc_t plane_rsrc(const C* p, int64_t elems) {
    return __builtin_amdgcn_make_buffer_rsrc((void*)p, (short)0, (int)(elems * (int64_t)sizeof(C)), 0x00020000);
}
// voff: per-lane byte offset (range checked); soff: uniform byte offset,
// only ever non-zero for rows known to lie inside the plane
__device__ __forceinline__ void bload(rsrc_t r, unsigned voff, unsigned soff, double2& v) {
    v = __builtin_bit_cast(double2, __builtin_amdgcn_raw_buffer_load_b128(r, (int)voff, (int)soff, 0));
}
__device__ __forceinline__ void bload(rsrc_t r, unsigned voff, unsigned soff, float2& v) {
    v = __builtin_bit_cast(float2, __builtin_amdgcn_raw_buffer_load_b64(r, (int)voff, (int)soff, 0));
}
// Stores carry the non-temporal hint (iterates written once per pass; the
// cache keeps the rows that neighbouring waves read again).
constexpr int STORE_POLICY = 2;  // non-temporal
__device__ __forceinline__ void bstore(rsrc_t r, unsigned voff, unsigned soff, double2 v) {
    using V = __attribute__((ext_vector_type(4))) unsigned int;
    __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(V, v), r, (int)voff, (int)soff, STORE_POLICY);
}
__device__ __forceinline__ void bstore(rsrc_t r, unsigned voff, unsigned soff, float2 v) {
    using V = __attribute__((ext_vector_type(2))) unsigned int;
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(V, v), r, (int)voff, (int)soff, STORE_POLICY);
}
// row * bytes-per-row, computed where it is used: an opaque scalar multiply
// keeps the compiler from hoisting every (row + constant) * rx of an unrolled
// block into its own scalar register
__device__ __forceinline__ unsigned srow(int row, unsigned rx) {
    unsigned r;
    asm volatile("s_mul_i32 %0, %1, %2" : "=s"(r) : "s"(row), "s"(rx));
    return r;
}
// byte offset of row j when ok, else OOB (uniform)
__device__ __forceinline__ unsigned row_off(bool ok, int j, int pitch, int es) {
    return ok ? (unsigned)(j * pitch * es) : OOB;
}

// Row pipelines.  Both kernels advance one grid row per step and are
// unrolled by UNR steps, so that every ring of rows below has a length that
// divides UNR and all ring slots are compile-time constants (no register
// rotation): a value pushed at phase P of the unrolled block sits in slot
// P mod L, the one pushed k steps earlier in (P - k) mod L.  Raw x and b rows
// are fetched PF steps ahead of their use.  Every block of UNR rows starts at
// an even row, so the parity of a row is that of its phase.
//
// Columns off the interior: b and x read zero there (out-of-range offsets),
// and d, s are replaced by zero in those lanes, so the residual vanishes
// there without a select; the smoothed iterate is cleared there by a lane
// select.  Rows off the interior only occur in the unrolled blocks at the two
// ends of a block's range ("edge" blocks); the interior blocks run a copy of
// the step with every row test removed.
constexpr int UNR = 6;
constexpr int PF = 2;  // rows of x and b fetched ahead
static_assert(UNR % 6 == 0 && UNR % (PF + 1) == 0, "ring lengths must divide the unroll");
template <int L> __host__ __device__ constexpr int slot(int p) { return ((p % L) + L * UNR) % L; }

// An empty asm statement that takes v in registers: everything v depends on
// is computed before this point.  Ends each step, so the compiler cannot sink
// a step's arithmetic into a later one (which keeps many rows alive at once).
__device__ __forceinline__ void pin(double& v) { asm volatile("" : "+v"(v)); }
__device__ __forceinline__ void pin(float& v) { asm volatile("" : "+v"(v)); }
__device__ __forceinline__ void pin(double2& v) { asm volatile("" : "+v"(v.x), "+v"(v.y)); }
__device__ __forceinline__ void pin(float2& v) { asm volatile("" : "+v"(v.x), "+v"(v.y)); }

// TC: precision of the coarse level (the restricted residual is rounded to
// it when the coarse levels run in complex64 under an FP64 finest level).
template <typename T, int NS, typename TC = T, bool JAC = false>
struct DownPipe {
    using C = cplx<T>;
    using CC = cplx<TC>;
    static constexpr int HALO = 2 * NS + 2;
    static constexpr int OWN = 64 - 2 * HALO;
    C X[NS + 1][3], R[NS + 1][3];
    C B[6];             // b rows j-1, j-2, ... (ring of 6 >= 2 NS + 1)
    C xr[PF + 1], br[PF + 1];
    rsrc_t xs, bs, xos, bcs;
    LevelView lf, lc;
    Coef<T> cf;
    C dl;               // d on interior columns, else 0
    T sl;               // s on interior columns, else 0
    int k0, k1;
    bool col_in;
    bool xz;            // the iterate read is zero: its residual is b itself
    T mk;  // 1 on interior columns, 0 off them
    unsigned ox, ob, oo, of;  // lane byte offsets: x, b, x written, coarse b (or OOB)
    unsigned rx;              // bytes per fine row
    unsigned rc;              // bytes per coarse row
    // physical fine / coarse row of pipeline row j / coarse row K: the
    // identity, or the reflection j -> ny + 1 - j for runs that stream upward
    int fa, fs, ca, cs;
    __device__ __forceinline__ int fph(int j) const { return fa + fs * j; }
    __device__ __forceinline__ int cph(int K) const { return ca + cs * K; }

    template <bool EDGE> __device__ __forceinline__ C load_x(int j) const {
        C v;
        if constexpr (EDGE) bload(xs, ox + (j >= 0 && j <= lf.ny + 1 ? fph(j) * rx : OOB), 0, v);
        else bload(xs, ox, fph(j) * rx, v);
        return v;
    }
    template <bool EDGE> __device__ __forceinline__ C load_b(int j) const {
        C v;
        if constexpr (EDGE) bload(bs, ob + (in_rows(j, lf.ny) ? fph(j) * rx : OOB), 0, v);
        else bload(bs, ob, fph(j) * rx, v);
        return v;
    }
    // step at row j, phase P: push x_0 row j and b row j - 1; stage q turns
    // x_q rows j-2q-2..j-2q into r_q row j-2q-1 and x_{q+1} row j-2q-2
    template <int P, bool EDGE> __device__ __forceinline__ void step(int j) {
        xr[slot<PF + 1>(P + PF)] = load_x<EDGE>(j + PF);
        br[slot<PF + 1>(P + PF)] = load_b<EDGE>(j + PF - 1);
        constexpr int n0 = slot<3>(P), n1 = slot<3>(P - 1), n2 = slot<3>(P - 2);
        X[0][n0] = xr[slot<PF + 1>(P)];
        B[slot<6>(P)] = br[slot<PF + 1>(P)];
#pragma unroll
        for (int q = 0; q <= NS; ++q) {
            C r;
            // (a zero start: b - L 0 is b, up to the sign of a zero; the ring
            // holds zero rows outside the grid)
            if (q == 0 && xz) {
                r = B[slot<6>(P)];
            } else {
                r = residual_row<T>(X[q][n2], X[q][n1], X[q][n0], B[slot<6>(P - 2 * q)], dl, sl);
                if constexpr (EDGE)
                    if (!in_rows(j - 2 * q - 1, lf.ny)) r = czero<C>();
            }
            R[q][n0] = r;
            if (q < NS) {
                C v = vanka_row<T, JAC>(X[q][n2], R[q][n2], R[q][n1], R[q][n0], cf, mk);
                if constexpr (EDGE)
                    if (!in_rows(j - 2 * q - 2, lf.ny)) v = czero<C>();
                X[q + 1][n0] = v;
            }
            pin(R[q][n0]);
            if (q < NS) pin(X[q + 1][n0]);
        }
        if constexpr (NS > 0) {
            const int orow = j - 2 * NS;
            if constexpr (EDGE) bstore(xos, oo + (orow >= k0 && orow <= k1 ? fph(orow) * rx : OOB), 0, X[NS][n0]);
            else bstore(xos, oo, fph(orow) * rx, X[NS][n0]);
        }
        // full weighting around fine row j - 2NS - 2 (even rows carry coarse nodes)
        if constexpr ((P & 1) == 0) {
            const int frow = j - 2 * NS - 2;
            const CC v = cvt<CC>(full_weight_row<T>(R[NS][n2], R[NS][n1], R[NS][n0]));
            const int K = frow >> 1;
            if constexpr (EDGE)
                bstore(bcs, of + (frow >= k0 && frow <= k1 && frow >= 2 && K <= lc.ny ? cph(K) * rc : OOB), 0, v);
            else bstore(bcs, of, cph(K) * rc, v);
        }
    }
    // (the scheduling barriers keep each step's loads in their step, so that
    // the fetch-ahead distance stays PF rows and the registers bounded)
    template <bool EDGE> __device__ __forceinline__ void block(int j) {
        step<0, EDGE>(j);
        __builtin_amdgcn_sched_barrier(0);
        step<1, EDGE>(j + 1);
        __builtin_amdgcn_sched_barrier(0);
        step<2, EDGE>(j + 2);
        __builtin_amdgcn_sched_barrier(0);
        step<3, EDGE>(j + 3);
        __builtin_amdgcn_sched_barrier(0);
        step<4, EDGE>(j + 4);
        __builtin_amdgcn_sched_barrier(0);
        step<5, EDGE>(j + 5);
        __builtin_amdgcn_sched_barrier(0);
    }
};

// Rows of a run.  Neighbouring runs of a strip walk in opposite directions:
// an odd run takes its rows from the bottom up, through the reflection
// j -> ny + 1 - j of the fine grid and K -> nyc + 1 - K of the coarse one
// (every level has an odd row count, so the reflection keeps the parity of a
// row and the pairing of fine row 2K with coarse row K).  Two runs that share
// halo rows then reach them at the end of both walks, about the same time, and
// the second reads come from L2.  k0, k1 become pipeline rows.
template <typename Pipe> __device__ __forceinline__ void set_rows(Pipe& p, bool rev, int& k0, int& k1) {
    const bool r = rev && (p.lf.ny & 1) != 0;
    p.fa = r ? p.lf.ny + 1 : 0;
    p.fs = r ? -1 : 1;
    p.ca = r ? p.lc.ny + 1 : 0;
    p.cs = p.fs;
    if (r) {
        const int t = p.lf.ny + 1 - k1;
        k1 = p.lf.ny + 1 - k0;
        k0 = t;
    }
    p.k0 = k0;
    p.k1 = k1;
}

// One wave's share of the work: rows k0..k1 of strip `strip` of system
// `sys` of segment S (the pipeline adds its halo rows itself).
template <typename T, int NS, typename TC, bool JAC, bool PACE = false>
__device__ __forceinline__ void down_piece(const LevelSeg<T>& S, int sys, int strip, int k0, int k1, bool rev,
                                           int lane) {
    using C = cplx<T>;
    using Pipe = DownPipe<T, NS, TC, JAC>;
    constexpr int HALO = Pipe::HALO, OWN = Pipe::OWN;
    Pipe p;
    p.lf = S.lf;
    p.lc = S.lc;
    const int i = 1 + strip * OWN - HALO + lane;
    p.col_in = i >= 1 && i <= p.lf.nx;
    p.mk = p.col_in ? (T)1 : (T)0;
    const bool col_ld = i >= 0 && i <= p.lf.nx + 1 && !S.x_zero;
    p.xz = S.x_zero != 0;
    const bool own = lane >= HALO && lane < HALO + OWN && p.col_in;
    const unsigned es = sizeof(C);
    p.ox = col_ld ? i * es : OOB;
    p.ob = p.col_in ? i * es : OOB;
    p.oo = own ? i * es : OOB;
    const unsigned ec = sizeof(cplx<TC>);
    p.of = (own && !(i & 1) && (i >> 1) <= p.lc.nx) ? (i >> 1) * ec : OOB;
    p.rx = p.lf.pitch * es;
    p.rc = p.lc.pitch * ec;
    set_rows(p, rev, k0, k1);
    const int64_t base = (int64_t)sys * p.lf.plane;
    p.xs = plane_rsrc(S.x + base, p.lf.plane);
    p.bs = plane_rsrc(S.b + base, p.lf.plane);
    // (no iterate output, S.xo null: its ascent recomputes it, see k_recomp;
    // an empty range drops every store)
    p.xos = S.xo ? plane_rsrc(S.xo + base, p.lf.plane) : plane_rsrc(S.b + base, 0);
    p.bcs = plane_rsrc(reinterpret_cast<const cplx<TC>*>(S.c) + (int64_t)sys * p.lc.plane, p.lc.plane);
    p.cf = S.coef[sys];
    p.dl = p.col_in ? p.cf.d : czero<C>();
    p.sl = p.col_in ? S.s : (T)0;
#pragma unroll
    for (int q = 0; q <= NS; ++q)
#pragma unroll
        for (int w = 0; w < 3; ++w) p.X[q][w] = p.R[q][w] = czero<C>();
#pragma unroll
    for (int w = 0; w < 6; ++w) p.B[w] = czero<C>();
    int jbeg = k0 - 2 * NS - 2;
    jbeg -= jbeg & 1;
    const int jend = k1 + 2 * NS + 2;
    // unrolled blocks whose rows (and the rows they load and store) all lie
    // inside the grid and the piece
    const int jlo = max(k0 + 2 * NS + 2, 2 * NS + 4), jhi = min(p.lf.ny - 4 - PF, k1 + 2 * NS - 5);
#pragma unroll
    for (int d = 0; d < PF; ++d) {
        p.xr[d] = p.template load_x<true>(jbeg + d);
        p.br[d] = p.template load_b<true>(jbeg + d - 1);
    }
    int j = jbeg;
    // (PACE: as in edge_piece)
    for (; j <= jend && j < jlo; j += UNR) {
        p.template block<true>(j);
        if constexpr (PACE) __syncthreads();
    }
    for (; j <= jhi; j += UNR) {
        p.template block<false>(j);
        if constexpr (PACE) __syncthreads();
    }
    for (; j <= jend; j += UNR) {
        p.template block<true>(j);
        if constexpr (PACE) __syncthreads();
    }
}

// Segment of global wave gw (segments own consecutive wave ranges).
template <typename T> __device__ __forceinline__ LevelSeg<T> seg_of_wave(const SegTable<T>& t, int gw) {
    LevelSeg<T> r = t.s[0];
#pragma unroll
    for (int q = 1; q < MAXSEG; ++q)
        if (q < t.n && gw >= t.s[q].w0) r = t.s[q];
    return r;
}

// Work split: every strip of every system is cut into S.pieces runs of
// S.rows rows (the last one shorter), one per wave; the host picks the cut so
// that the waves fill the device evenly.  Waves are numbered with the strip
// fastest, then the run, then the system: the waves of a block, and
// neighbouring blocks, cover adjacent strips of the same rows, so the halo
// columns two strips share are read close together in time (mostly from L2).
struct Piece {
    int sys, strip, k0, k1, slot;
    bool rev;  // odd runs stream their rows upward (see set_rows)
};
template <typename T> __device__ __forceinline__ Piece piece_of(const LevelSeg<T>& S, int lw) {
    Piece pc;
    const int t = lw / S.strips;
    pc.strip = lw - t * S.strips;
    pc.sys = t / S.pieces;
    const int run = t - pc.sys * S.pieces;
    pc.slot = lw;  // == (sys * pieces + run) * strips + strip
    pc.k0 = 1 + run * S.rows;
    pc.k1 = min(S.lf.ny, pc.k0 + S.rows - 1);
    pc.rev = (run & 1) != 0;
    return pc;
}

// ---------------------------------------------------------------------------
// WB waves a block (more than NT / 64: paced blocks, see edge_piece)
template <typename T, int NS, typename TC, bool JAC = false, int WB = NT / 64>
__global__ __launch_bounds__(64 * WB) void k_down(SegTable<T> tab) {
    // the wave index is uniform over the wave; say so, so that everything
    // derived from it (segment, buffer resources, row bounds) lives in SGPRs
    const int gw = (int)xcd_block().x * WB + __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int lane = threadIdx.x & 63;
    const LevelSeg<T> S = seg_of_wave(tab, gw);
    const int lw = gw - S.w0;
    if (lw >= S.waves) return;  // whole wave idle (paced blocks: see edge_piece)
    const Piece pc = piece_of(S, lw);
    if (pc.k0 > pc.k1 || !S.active[pc.sys]) return;
    down_piece<T, NS, TC, JAC, (WB > NT / 64)>(S, pc.sys, pc.strip, pc.k0, pc.k1, pc.rev, lane);
}

template <typename T, int NS, bool NORM, typename TC = T, bool JAC = false>
struct UpPipe {
    using C = cplx<T>;
    static constexpr int HALO = NORM ? 2 * NS + 1 : (NS > 0 ? 2 * NS : 1);
    static constexpr int OWN = 64 - 2 * HALO;
    // The correction at an odd column takes the right lane's coarse value, so
    // lane 63 is wrong there and the error spreads one lane per stage.  With
    // an even HALO lane 63 sits on an even column; with the odd HALO of the
    // norm variant the strips start one column earlier (at the zero ring
    // column) to the same effect.
    static constexpr int COL0 = (HALO & 1) ? 0 : 1;
    C X[NS + 1][3], R[NS + 1][3];
    C B[6];
    C xr[PF + 1], br[PF + 1];
    C er[3], ei[3];     // coarse rows: raw, and interpolated along x
    rsrc_t xs, bs, es, xos;
    LevelView lf, lc;
    Coef<T> cf;
    C dl;
    T sl;
    int k0, k1;
    bool col_in, odd;
    T mk, hf;  // 1 / 0 on interior / other columns; 1/2 / 0 on odd / even columns
    unsigned ox, oe, oo;  // lane byte offsets: x and b, coarse e, x written (or OOB)
    unsigned rx, rc, ro;  // row strides in bytes: x and b, coarse e, x written
    // physical fine / coarse row of pipeline row j / coarse row K: the
    // identity, or the reflection j -> ny + 1 - j for runs that stream upward
    int fa, fs, ca, cs;
    __device__ __forceinline__ int fph(int j) const { return fa + fs * j; }
    __device__ __forceinline__ int cph(int K) const { return ca + cs * K; }
    double acc;

    template <bool EDGE> __device__ __forceinline__ C load_x(int j) const {
        C v;
        if constexpr (EDGE) bload(xs, ox + (in_rows(j, lf.ny) ? fph(j) * rx : OOB), 0, v);
        else bload(xs, ox, fph(j) * rx, v);
        return v;
    }
    template <bool EDGE> __device__ __forceinline__ C load_b(int j) const {
        C v;
        if constexpr (EDGE) bload(bs, ox + (in_rows(j, lf.ny) ? fph(j) * rx : OOB), 0, v);
        else bload(bs, ox, fph(j) * rx, v);
        return v;
    }
    template <bool EDGE> __device__ __forceinline__ C load_e(int K) const {
        cplx<TC> v;
        if constexpr (EDGE) bload(es, oe + (K >= 0 && K <= lc.ny + 1 ? cph(K) * rc : OOB), 0, v);
        else bload(es, oe, cph(K) * rc, v);
        return cvt<C>(v);
    }
    // coarse column i/2 at an even fine column; the average of coarse columns
    // (i-1)/2 and (i+1)/2 at an odd one (the right one via a lane shift)
    __device__ __forceinline__ C interp_x(C v) const {
        // v + hf (right - v): the average at odd columns (hf = 1/2), v at even ones
        const C rv = from_right(v);
        C r;
        r.x = fmar(hf, rv.x - v.x, v.x);
        r.y = fmar(hf, rv.y - v.y, v.y);
        return r;
    }
    // Step at fine row j, phase P.  Coarse row K = jb/2 + c (jb the unrolled
    // block's first row) lives in coarse slot c mod 3: its raw load is issued
    // four fine rows ahead of row 2K - 1, where it is interpolated along x.
    // Off the interior the interpolated correction is zero by itself (odd
    // level sizes: the ring of the coarse grid lies on the fine ring).
    template <int P, bool EDGE> __device__ __forceinline__ void step(int j) {
        xr[slot<PF + 1>(P + PF)] = load_x<EDGE>(j + PF);
        br[slot<PF + 1>(P + PF)] = load_b<EDGE>(j + PF - 1);
        C e;
        if constexpr ((P & 1) != 0) {
            constexpr int lo = slot<3>((P - 1) / 2), hi = slot<3>((P + 1) / 2);
            ei[hi] = interp_x(er[hi]);
            e = cscale(cadd(ei[lo], ei[hi]), (T)0.5);
        } else {
            er[slot<3>(P / 2 + 2)] = load_e<EDGE>((j >> 1) + 2);
            e = ei[slot<3>(P / 2)];
        }
        constexpr int n0 = slot<3>(P), n1 = slot<3>(P - 1), n2 = slot<3>(P - 2);
        X[0][n0] = cadd(xr[slot<PF + 1>(P)], e);
        B[slot<6>(P)] = br[slot<PF + 1>(P)];
#pragma unroll
        for (int q = 0; q <= NS; ++q) {
            if (q == NS && !NORM) break;
            const int rrow = j - 2 * q - 1;
            C r = residual_row<T>(X[q][n2], X[q][n1], X[q][n0], B[slot<6>(P - 2 * q)], dl, sl);
            if constexpr (EDGE)
                if (!in_rows(rrow, lf.ny)) r = czero<C>();
            if (q == NS) {
                // the owned-lane mask is applied once, at the end
                if (!EDGE || (rrow >= k0 && rrow <= k1)) acc += (double)r.x * (double)r.x + (double)r.y * (double)r.y;
                pin(acc);
                break;
            }
            R[q][n0] = r;
            C v = vanka_row<T, JAC>(X[q][n2], R[q][n2], R[q][n1], R[q][n0], cf, mk);
            if constexpr (EDGE)
                if (!in_rows(j - 2 * q - 2, lf.ny)) v = czero<C>();
            X[q + 1][n0] = v;
            pin(R[q][n0]);
            pin(X[q + 1][n0]);
        }
        pin(X[0][n0]);
        const int orow = j - 2 * NS;
        if constexpr (EDGE) bstore(xos, oo + (orow >= k0 && orow <= k1 ? fph(orow) * ro : OOB), 0, X[NS][n0]);
        else bstore(xos, oo, fph(orow) * ro, X[NS][n0]);
    }
    template <bool EDGE> __device__ __forceinline__ void block(int j) {
        step<0, EDGE>(j);
        __builtin_amdgcn_sched_barrier(0);
        step<1, EDGE>(j + 1);
        __builtin_amdgcn_sched_barrier(0);
        step<2, EDGE>(j + 2);
        __builtin_amdgcn_sched_barrier(0);
        step<3, EDGE>(j + 3);
        __builtin_amdgcn_sched_barrier(0);
        step<4, EDGE>(j + 4);
        __builtin_amdgcn_sched_barrier(0);
        step<5, EDGE>(j + 5);
        __builtin_amdgcn_sched_barrier(0);
    }
};

// Rows k0..k1 of one strip of one system; returns the lane's share of
// sum |b - L x|^2 over the owned columns and rows (NORM).
template <typename T, int NS, bool NORM, typename TC, bool JAC, bool PACE = false>
__device__ __forceinline__ double up_piece(const LevelSeg<T>& S, int sys, int strip, int k0, int k1, bool rev,
                                           int lane) {
    using C = cplx<T>;
    using Pipe = UpPipe<T, NS, NORM, TC, JAC>;
    constexpr int HALO = Pipe::HALO, OWN = Pipe::OWN;
    Pipe p;
    p.lf = S.lf;
    p.lc = S.lc;
    const int i = Pipe::COL0 + strip * OWN - HALO + lane;
    p.col_in = i >= 1 && i <= p.lf.nx;
    p.mk = p.col_in ? (T)1 : (T)0;
    p.odd = (i & 1) != 0;
    p.hf = p.odd ? (T)0.5 : (T)0;
    const bool ecol = i >= 0 && i <= p.lf.nx + 1;
    const bool own = lane >= HALO && lane < HALO + OWN && p.col_in;
    const unsigned es = sizeof(C), ec = sizeof(cplx<TC>);
    p.ox = p.col_in ? i * es : OOB;
    p.oe = ecol ? (i >> 1) * ec : OOB;
    p.oo = own ? i * es : OOB;
    p.rx = p.lf.pitch * es;
    p.rc = p.lc.pitch * ec;
    set_rows(p, rev, k0, k1);
    const int64_t base = (int64_t)sys * p.lf.plane;
    // finishing pass (S.iters set): the iterate read is the one the system's
    // last cycle-edge pass read, x after an even number of cycles and xalt
    // after an odd one; no cycle at all means a zero result (every read
    // through an empty range returns zero)
    const C* xsrc = S.x;
    int64_t len = p.lf.plane, clen = p.lc.plane;
    if (S.iters) {
        const int it = S.iters[sys];
        if (it & 1) xsrc = S.xalt;
        if (it == 0) len = clen = 0;
    }
    p.xs = plane_rsrc(xsrc + base, len);
    p.bs = plane_rsrc(S.b + base, len);
    p.es = plane_rsrc(reinterpret_cast<const cplx<TC>*>(S.c) + (int64_t)sys * p.lc.plane, clen);
    if (S.zd) {
        // dense rows of nx nodes: row r, column i (both from 1) at (r - 1) nx + i - 1
        const int64_t m = (int64_t)p.lf.nx * p.lf.ny;
        p.xos = plane_rsrc(S.zd + sys * m - (p.lf.nx + 1), m + p.lf.nx + 1);
        p.ro = p.lf.nx * es;
    } else {
        p.xos = plane_rsrc(S.xo + base, p.lf.plane);
        p.ro = p.rx;
    }
    p.cf = S.coef[sys];
    p.dl = p.col_in ? p.cf.d : czero<C>();
    p.sl = p.col_in ? S.s : (T)0;
    p.acc = 0.0;
#pragma unroll
    for (int q = 0; q <= NS; ++q)
#pragma unroll
        for (int w = 0; w < 3; ++w) p.X[q][w] = p.R[q][w] = czero<C>();
#pragma unroll
    for (int w = 0; w < 6; ++w) p.B[w] = czero<C>();
    int jbeg = k0 - 2 * NS - 1;
    jbeg -= jbeg & 1;
    const int jend = k1 + 2 * NS + 1;
    const int jlo = max(k0 + 2 * NS + 1, 2 * NS + 2);
    const int jhi = min(min(p.lf.ny - 5 - PF, p.lf.ny - 7), k1 + 2 * NS - 5);
    // coarse rows jbeg/2 (interpolated) and jbeg/2 + 1 (raw) before the first step
    p.ei[0] = p.interp_x(p.template load_e<true>(jbeg >> 1));
    p.er[1] = p.template load_e<true>((jbeg >> 1) + 1);
#pragma unroll
    for (int d = 0; d < PF; ++d) {
        p.xr[d] = p.template load_x<true>(jbeg + d);
        p.br[d] = p.template load_b<true>(jbeg + d - 1);
    }
    int j = jbeg;
    // (PACE: as in edge_piece)
    for (; j <= jend && j < jlo; j += UNR) {
        p.template block<true>(j);
        if constexpr (PACE) __syncthreads();
    }
    for (; j <= jhi; j += UNR) {
        p.template block<false>(j);
        if constexpr (PACE) __syncthreads();
    }
    for (; j <= jend; j += UNR) {
        p.template block<true>(j);
        if constexpr (PACE) __syncthreads();
    }
    return own ? p.acc : 0.0;
}

// ---------------------------------------------------------------------------
// With NORM, every wave leaves its run's sum in the segment's partial buffer
// (slot = the wave's index in the segment, S.pieces * S.strips per system).
template <typename T, int NS, bool NORM, typename TC, bool JAC = false, int WB = NT / 64>
__global__ __launch_bounds__(64 * WB) void k_up(SegTable<T> tab) {
    // the wave index is uniform over the wave; say so, so that everything
    // derived from it (segment, buffer resources, row bounds) lives in SGPRs
    const int gw = (int)xcd_block().x * WB + __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int lane = threadIdx.x & 63;
    const LevelSeg<T> S = seg_of_wave(tab, gw);
    const int lw = gw - S.w0;
    if (lw >= S.waves) return;  // whole wave idle (paced blocks: see edge_piece)
    const Piece pc = piece_of(S, lw);
    if (!S.iters && !S.active[pc.sys]) return;  // (the finishing pass runs for every system)
    double acc = 0.0;
    if (pc.k0 <= pc.k1)
        acc = up_piece<T, NS, NORM, TC, JAC, (WB > NT / 64)>(S, pc.sys, pc.strip, pc.k0, pc.k1, pc.rev, lane);
    if (NORM && S.partial) {
        for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
        if (lane == 0) S.partial[pc.slot] = acc;
    }
}

// ---------------------------------------------------------------------------
// Finest level at the boundary of two V-cycles, in one pass: the bilinear
// correction and NA post-smoothing sweeps that end cycle k, the residual norm
// of that iterate (the stopping test), then NB pre-smoothing sweeps of cycle
// k+1 from it (written to xo), their residual and its full weighting (the
// next coarse right-hand side, written to cb).  Reads x, b and the coarse
// correction once instead of twice per cycle.  Cycle k's finished iterate is
// not stored: once a system stops, its inputs to this pass (x and the coarse
// correction) are left untouched, and the finishing pass of k_up rebuilds the
// iterate from them once.  Unrolled by 12 steps: the right-hand side ring
// needs 2(NA+NB)+1 rows.
constexpr int UNR_E = 12;
constexpr int EPF = 1;  // rows of x and b fetched ahead
template <int L> __host__ __device__ constexpr int eslot(int p) { return ((p % L) + L * UNR_E) % L; }

template <typename T, int NA, int NB, typename TC = T, bool JAC = false>
struct EdgePipe {
    using C = cplx<T>;
    using CC = cplx<TC>;
    static constexpr int NS = NA + NB;
    static constexpr int HALO = 2 * NS + 2;  // NS+1 residuals, NS updates, the weighting's lane sum
    static constexpr int OWN = 64 - 2 * HALO;
    // an even HALO and strips from column 1 put lane 63 on an even column,
    // where the correction needs no right-lane value
    static constexpr int COL0 = 1;
    static_assert(UNR_E % 12 == 0 && UNR_E % (EPF + 1) == 0 && 2 * NS + 1 <= 12, "ring lengths");
    C X[NS + 1][3], R[NS + 1][3];
    C* B;               // this lane's column of the wave's 12-row ring in LDS (stride 64)
    C xr[EPF + 1], br[EPF + 1];
    C er[3], ei[3];
    rsrc_t xs, bs, es, xos, cbs;
    LevelView lf, lc;
    Coef<T> cf;
    C dl;
    T sl;
    int k0, k1;
    bool col_in, odd;
    T mk, hf;  // 1 / 0 on interior / other columns; 1/2 / 0 on odd / even columns
    unsigned ox, oe, oo, of;
    unsigned rx, rc;
    // physical fine / coarse row of pipeline row j / coarse row K: the
    // identity, or the reflection j -> ny + 1 - j for runs that stream upward
    int fa, fs, ca, cs;
    __device__ __forceinline__ int fph(int j) const { return fa + fs * j; }
    __device__ __forceinline__ int cph(int K) const { return ca + cs * K; }
    double acc;

    template <bool EDGE> __device__ __forceinline__ C load_x(int j) const {
        C v;
        if constexpr (EDGE) bload(xs, ox + (in_rows(j, lf.ny) ? fph(j) * rx : OOB), 0, v);
        else bload(xs, ox, srow(fph(j), rx), v);
        return v;
    }
    template <bool EDGE> __device__ __forceinline__ C load_b(int j) const {
        C v;
        if constexpr (EDGE) bload(bs, ox + (in_rows(j, lf.ny) ? fph(j) * rx : OOB), 0, v);
        else bload(bs, ox, srow(fph(j), rx), v);
        return v;
    }
    template <bool EDGE> __device__ __forceinline__ C load_e(int K) const {
        CC v;
        if constexpr (EDGE) bload(es, oe + (K >= 0 && K <= lc.ny + 1 ? cph(K) * rc : OOB), 0, v);
        else bload(es, oe, srow(cph(K), rc), v);
        return cvt<C>(v);
    }
    __device__ __forceinline__ C interp_x(C v) const {
        // v + hf (right - v): the average at odd columns (hf = 1/2), v at even ones
        const C rv = from_right(v);
        C r;
        r.x = fmar(hf, rv.x - v.x, v.x);
        r.y = fmar(hf, rv.y - v.y, v.y);
        return r;
    }
    template <bool EDGE> __device__ __forceinline__ void store_row(rsrc_t r, int row, C v) const {
        if constexpr (EDGE) bstore(r, oo + (row >= k0 && row <= k1 ? fph(row) * rx : OOB), 0, v);
        else bstore(r, oo, srow(fph(row), rx), v);
    }
    template <int P, bool EDGE> __device__ __forceinline__ void step(int j) {
        xr[eslot<EPF + 1>(P + EPF)] = load_x<EDGE>(j + EPF);
        br[eslot<EPF + 1>(P + EPF)] = load_b<EDGE>(j + EPF - 1);
        C e;
        if constexpr ((P & 1) != 0) {
            constexpr int lo = eslot<3>((P - 1) / 2), hi = eslot<3>((P + 1) / 2);
            ei[hi] = interp_x(er[hi]);
            e = cscale(cadd(ei[lo], ei[hi]), (T)0.5);
        } else {
            er[eslot<3>(P / 2 + 2)] = load_e<EDGE>((j >> 1) + 2);
            e = ei[eslot<3>(P / 2)];
        }
        constexpr int n0 = eslot<3>(P), n1 = eslot<3>(P - 1), n2 = eslot<3>(P - 2);
        X[0][n0] = cadd(xr[eslot<EPF + 1>(P)], e);
        B[eslot<12>(P) * 64] = br[eslot<EPF + 1>(P)];
#pragma unroll
        for (int q = 0; q <= NS; ++q) {
            const int rrow = j - 2 * q - 1;
            const C bq = B[eslot<12>(P - 2 * q) * 64];
            C r = residual_row<T>(X[q][n2], X[q][n1], X[q][n0], bq, dl, sl);
            if constexpr (EDGE)
                if (!in_rows(rrow, lf.ny)) r = czero<C>();
            if (q == NA) {
                // stopping-test residual of cycle k's final iterate (owned-lane
                // mask applied once, at the end)
                if (!EDGE || (rrow >= k0 && rrow <= k1)) acc += (double)r.x * (double)r.x + (double)r.y * (double)r.y;
                pin(acc);
            }
            R[q][n0] = r;
            pin(R[q][n0]);
            if (q < NS) {
                C v = vanka_row<T, JAC>(X[q][n2], R[q][n2], R[q][n1], R[q][n0], cf, mk);
                if constexpr (EDGE)
                    if (!in_rows(j - 2 * q - 2, lf.ny)) v = czero<C>();
                X[q + 1][n0] = v;
                pin(X[q + 1][n0]);
            }
        }
        pin(X[0][n0]);
        store_row<EDGE>(xos, j - 2 * NS, X[NS][n0]);
        if constexpr ((P & 1) == 0) {
            const int frow = j - 2 * NS - 2;
            const CC v = cvt<CC>(full_weight_row<T>(R[NS][n2], R[NS][n1], R[NS][n0]));
            const int K = frow >> 1;
            if constexpr (EDGE)
                bstore(cbs, of + (frow >= k0 && frow <= k1 && frow >= 2 && K <= lc.ny ? cph(K) * rc : OOB), 0, v);
            else bstore(cbs, of, srow(cph(K), rc), v);
        }
    }
    template <bool EDGE> __device__ __forceinline__ void block(int j) {
#define VMG_E(P)                      \
    step<P, EDGE>(j + P);             \
    __builtin_amdgcn_sched_barrier(0);
        VMG_E(0) VMG_E(1) VMG_E(2) VMG_E(3) VMG_E(4) VMG_E(5)
        VMG_E(6) VMG_E(7) VMG_E(8) VMG_E(9) VMG_E(10) VMG_E(11)
#undef VMG_E
    }
};

template <typename T, int NA, int NB, typename TC, bool JAC, bool PACE>
__device__ __forceinline__ double edge_piece(const LevelSeg<T>& S, int sys, int strip, int k0, int k1, bool rev,
                                             int lane, cplx<T>* bring) {
    using C = cplx<T>;
    using Pipe = EdgePipe<T, NA, NB, TC, JAC>;
    constexpr int HALO = Pipe::HALO, OWN = Pipe::OWN, NS = Pipe::NS, U = UNR_E;
    Pipe p;
    p.B = bring + lane;
    p.lf = S.lf;
    p.lc = S.lc;
    const int i = Pipe::COL0 + strip * OWN - HALO + lane;
    p.col_in = i >= 1 && i <= p.lf.nx;
    p.mk = p.col_in ? (T)1 : (T)0;
    p.odd = (i & 1) != 0;
    p.hf = p.odd ? (T)0.5 : (T)0;
    const bool ecol = i >= 0 && i <= p.lf.nx + 1;
    const bool own = lane >= HALO && lane < HALO + OWN && p.col_in;
    const unsigned es = sizeof(C), ec = sizeof(cplx<TC>);
    p.ox = p.col_in ? i * es : OOB;
    p.oe = ecol ? (i >> 1) * ec : OOB;
    p.oo = own ? i * es : OOB;
    p.of = (own && !(i & 1) && (i >> 1) <= p.lc.nx) ? (i >> 1) * ec : OOB;
    p.rx = p.lf.pitch * es;
    p.rc = p.lc.pitch * ec;
    set_rows(p, rev, k0, k1);
    const int64_t base = (int64_t)sys * p.lf.plane;
    p.xs = plane_rsrc(S.x + base, p.lf.plane);
    p.bs = plane_rsrc(S.b + base, p.lf.plane);
    p.es = plane_rsrc(reinterpret_cast<const cplx<TC>*>(S.c) + (int64_t)sys * p.lc.plane, p.lc.plane);
    p.xos = plane_rsrc(S.xo + base, p.lf.plane);
    p.cbs = plane_rsrc(reinterpret_cast<const cplx<TC>*>(S.cb) + (int64_t)sys * p.lc.plane, p.lc.plane);
    p.cf = S.coef[sys];
    p.dl = p.col_in ? p.cf.d : czero<C>();
    p.sl = p.col_in ? S.s : (T)0;
    p.acc = 0.0;
#pragma unroll
    for (int q = 0; q <= NS; ++q)
#pragma unroll
        for (int w = 0; w < 3; ++w) p.X[q][w] = p.R[q][w] = czero<C>();
#pragma unroll
    for (int w = 0; w < 12; ++w) p.B[w * 64] = czero<C>();
    int jbeg = k0 - 2 * NS - 2;
    jbeg -= jbeg & 1;
    const int jend = k1 + 2 * NS + 2;
    const int jlo = max(k0 + 2 * NS + 2, 2 * NS + 4);
    const int jhi = min(min(p.lf.ny - U + 1 - EPF, p.lf.ny - U - 1), k1 - U + 1 + 2 * NA);
    p.ei[0] = p.interp_x(p.template load_e<true>(jbeg >> 1));
    p.er[1] = p.template load_e<true>((jbeg >> 1) + 1);
#pragma unroll
    for (int d = 0; d < EPF; ++d) {
        p.xr[d] = p.template load_x<true>(jbeg + d);
        p.br[d] = p.template load_b<true>(jbeg + d - 1);
    }
    // PACE: the block's waves (adjacent strips of the same rows) meet at a
    // barrier after every block of rows, so that they read and write the
    // same rows of the planes at about the same time.  Only pacing: no data
    // passes between the waves, and a wave that ends early leaves the
    // barrier to the others (its trip count may differ from theirs).
    int j = jbeg;
    for (; j <= jend && j < jlo; j += U) {
        p.template block<true>(j);
        if constexpr (PACE) __syncthreads();
    }
    for (; j <= jhi; j += U) {
        p.template block<false>(j);
        if constexpr (PACE) __syncthreads();
    }
    for (; j <= jend; j += U) {
        p.template block<true>(j);
        if constexpr (PACE) __syncthreads();
    }
    return own ? p.acc : 0.0;
}

// WB waves a block: NT / 64, or EDGE_WB (the waves of a CU at the FP64
// kernel's occupancy) for the paced form.
constexpr int EDGE_WB = 12;
template <typename T, int NA, int NB, typename TC, bool JAC = false, int WB = NT / 64>
__global__ __launch_bounds__(64 * WB) void k_edge(SegTable<T> tab) {
    __shared__ cplx<T> bring[WB][12 * 64];  // right-hand side rows, one ring per wave
    const int gw = (int)xcd_block().x * WB + __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int lane = threadIdx.x & 63;
    const LevelSeg<T> S = seg_of_wave(tab, gw);
    const int lw = gw - S.w0;
    if (lw >= S.waves) return;
    const Piece pc = piece_of(S, lw);
    if (!S.active[pc.sys]) return;
    // (every run walks downward here: the kernel is at its register limit and
    // measured slower with the reflected address arithmetic)
    double acc = edge_piece<T, NA, NB, TC, JAC, (WB > NT / 64)>(S, pc.sys, pc.strip, pc.k0, pc.k1, false, lane,
                                                               bring[threadIdx.x >> 6]);
    if (S.partial) {
        for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
        if (lane == 0) S.partial[pc.slot] = acc;
    }
}

// ---------------------------------------------------------------------------
// A coarse level's ascent that recomputes its pre-smoothed iterate.  Every
// visit of a V-cycle's coarse level starts from zero, so the pre-smoothed
// iterate x' = S^NPRE(0; b) is a function of that level's right-hand side
// alone: the descent (k_down with no iterate output) need not store it, and
// this pass rebuilds it on the way, from the same right-hand side rows it
// reads for the post-smoothing anyway:
//   x_0 = 0, NPRE sweeps  ->  x'   (the descent's stages)
//   x' + P e, NPOST sweeps -> xo   (the plain ascent's stages)
// Each stage is the same row stencil, in the same order, as in the two
// passes it replaces, except that the zero start's residual is b itself, so
// the results equal theirs (up to the sign of a zero, which no later sum or
// product turns into another value); the level moves the iterate's write and
// read (2 of 5.5 complex values a node) less.  The zero start is a runtime
// zero, as the descent's range-checked load of an empty plane gives, so that
// no later stage is simplified differently.  Unrolled by 12 steps: the
// right-hand side ring needs 2 NS - 1 rows.
template <typename T, int NPRE, int NPOST, bool JAC = false>
struct RecompPipe {
    using C = cplx<T>;
    static constexpr int NS = NPRE + NPOST;
    // a lane is wrong once a stage needs a neighbour the wave lacks: the
    // first residual (of the zero start) is right on every lane, each later
    // residual and every update widen the wrong edge by one lane (2 NS - 1)
    static constexpr int HALO = 2 * NS;
    static constexpr int OWN = 64 - 2 * HALO;
    static constexpr int COL0 = 1;
    static_assert(UNR_E % 12 == 0 && UNR_E % (EPF + 1) == 0 && 2 * NS - 1 <= 12 && NPRE >= 1 && NPOST >= 1,
                  "ring lengths");
    C X[NS + 1][3], R[NS][3];
    C* B;  // this lane's column of the wave's 12-row ring in LDS (stride 64)
    C br[EPF + 1];
    C er[3], ei[3];
    rsrc_t bs, es, xos;
    LevelView lf, lc;
    Coef<T> cf;
    C dl;
    T sl;
    int k0, k1;
    bool col_in, odd;
    T mk, hf;
    unsigned ox, oe, oo;
    unsigned rx, rc;

    template <bool EDGE> __device__ __forceinline__ C load_b(int j) const {
        C v;
        if constexpr (EDGE) bload(bs, ox + (in_rows(j, lf.ny) ? j * rx : OOB), 0, v);
        else bload(bs, ox, srow(j, rx), v);
        return v;
    }
    template <bool EDGE> __device__ __forceinline__ C load_e(int K) const {
        C v;
        if constexpr (EDGE) bload(es, oe + (K >= 0 && K <= lc.ny + 1 ? K * rc : OOB), 0, v);
        else bload(es, oe, srow(K, rc), v);
        return v;
    }
    __device__ __forceinline__ C interp_x(C v) const {
        const C rv = from_right(v);
        C r;
        r.x = fmar(hf, rv.x - v.x, v.x);
        r.y = fmar(hf, rv.y - v.y, v.y);
        return r;
    }
    // Step at row j, phase P: push b row j - 1; stage q turns x_q rows
    // j-2q-2..j-2q into r_q row j-2q-1 and x_{q+1} row j-2q-2.  The
    // correction joins x_NPRE, whose newest row is j' = j - 2 NPRE: the coarse
    // rows follow j' (phase Q = P - 2 NPRE, of P's parity) exactly as they
    // follow the loaded row in the plain ascent.
    template <int P, bool EDGE> __device__ __forceinline__ void step(int j) {
        br[eslot<EPF + 1>(P + EPF)] = load_b<EDGE>(j + EPF - 1);
        constexpr int Q = P - 2 * NPRE;
        const int jq = j - 2 * NPRE;
        C e;
        if constexpr ((Q & 1) != 0) {
            constexpr int lo = eslot<3>((Q - 1) / 2), hi = eslot<3>((Q + 1) / 2);
            ei[hi] = interp_x(er[hi]);
            e = cscale(cadd(ei[lo], ei[hi]), (T)0.5);
        } else {
            er[eslot<3>(Q / 2 + 2)] = load_e<EDGE>((jq >> 1) + 2);
            e = ei[eslot<3>(Q / 2)];
        }
        constexpr int n0 = eslot<3>(P), n1 = eslot<3>(P - 1), n2 = eslot<3>(P - 2);
        B[eslot<12>(P) * 64] = br[eslot<EPF + 1>(P)];
#pragma unroll
        for (int q = 0; q < NS; ++q) {
            const C bq = B[eslot<12>(P - 2 * q) * 64];
            // (the zero start's residual is b itself: the ring holds zero rows
            // outside the grid, and the value equals the descent's b - L 0 up
            // to the sign of a zero)
            C r = q == 0 ? bq : residual_row<T>(X[q][n2], X[q][n1], X[q][n0], bq, dl, sl);
            if constexpr (EDGE)
                if (q > 0 && !in_rows(j - 2 * q - 1, lf.ny)) r = czero<C>();
            R[q][n0] = r;
            pin(R[q][n0]);
            C v = vanka_row<T, JAC>(X[q][n2], R[q][n2], R[q][n1], R[q][n0], cf, mk);
            if constexpr (EDGE)
                if (!in_rows(j - 2 * q - 2, lf.ny)) v = czero<C>();
            if (q + 1 == NPRE) v = cadd(v, e);
            X[q + 1][n0] = v;
            pin(X[q + 1][n0]);
        }
        const int orow = j - 2 * NS;
        if constexpr (EDGE) bstore(xos, oo + (orow >= k0 && orow <= k1 ? orow * rx : OOB), 0, X[NS][n0]);
        else bstore(xos, oo, srow(orow, rx), X[NS][n0]);
    }
    template <bool EDGE> __device__ __forceinline__ void block(int j) {
#define VMG_R(P)                      \
    step<P, EDGE>(j + P);             \
    __builtin_amdgcn_sched_barrier(0);
        VMG_R(0) VMG_R(1) VMG_R(2) VMG_R(3) VMG_R(4) VMG_R(5)
        VMG_R(6) VMG_R(7) VMG_R(8) VMG_R(9) VMG_R(10) VMG_R(11)
#undef VMG_R
    }
};

template <typename T, int NPRE, int NPOST, bool JAC>
__device__ __forceinline__ void recomp_piece(const LevelSeg<T>& S, int sys, int strip, int k0, int k1, int lane,
                                             cplx<T>* bring) {
    using C = cplx<T>;
    using Pipe = RecompPipe<T, NPRE, NPOST, JAC>;
    constexpr int HALO = Pipe::HALO, OWN = Pipe::OWN, NS = Pipe::NS, U = UNR_E;
    Pipe p;
    p.B = bring + lane;
    p.lf = S.lf;
    p.lc = S.lc;
    const int i = Pipe::COL0 + strip * OWN - HALO + lane;
    p.col_in = i >= 1 && i <= p.lf.nx;
    p.mk = p.col_in ? (T)1 : (T)0;
    p.odd = (i & 1) != 0;
    p.hf = p.odd ? (T)0.5 : (T)0;
    const bool ecol = i >= 0 && i <= p.lf.nx + 1;
    const bool own = lane >= HALO && lane < HALO + OWN && p.col_in;
    const unsigned es = sizeof(C);
    p.ox = p.col_in ? i * es : OOB;
    p.oe = ecol ? (i >> 1) * es : OOB;
    p.oo = own ? i * es : OOB;
    p.rx = p.lf.pitch * es;
    p.rc = p.lc.pitch * es;
    p.k0 = k0;
    p.k1 = k1;
    const int64_t base = (int64_t)sys * p.lf.plane;
    p.bs = plane_rsrc(S.b + base, p.lf.plane);
    p.es = plane_rsrc(S.c + (int64_t)sys * p.lc.plane, p.lc.plane);
    p.xos = plane_rsrc(S.xo + base, p.lf.plane);
    p.cf = S.coef[sys];
    p.dl = p.col_in ? p.cf.d : czero<C>();
    p.sl = p.col_in ? S.s : (T)0;
    C zero = czero<C>();
    pin(zero);
#pragma unroll
    for (int w = 0; w < 3; ++w) {
        p.X[0][w] = zero;
#pragma unroll
        for (int q = 0; q < NS; ++q) p.X[q + 1][w] = p.R[q][w] = czero<C>();
    }
#pragma unroll
    for (int w = 0; w < 12; ++w) p.B[w * 64] = czero<C>();
    int jbeg = k0 - 2 * NS;
    jbeg -= jbeg & 1;
    const int jend = k1 + 2 * NS;
    // blocks whose rows, loads and stores all lie inside the grid and the piece
    const int jlo = max(k0 + 2 * NS, 2 * NS + 2);
    const int jhi = min(min(p.lf.ny - U + 1 - EPF, p.lf.ny - U - 1), k1 - U + 1 + 2 * NS);
    // coarse rows j'/2 (interpolated) and j'/2 + 1 (raw) of the first step's j'
    const int jq = jbeg - 2 * NPRE;
    p.ei[eslot<3>(-NPRE)] = p.interp_x(p.template load_e<true>(jq >> 1));
    p.er[eslot<3>(1 - NPRE)] = p.template load_e<true>((jq >> 1) + 1);
#pragma unroll
    for (int d = 0; d < EPF; ++d) p.br[d] = p.template load_b<true>(jbeg + d - 1);
    int j = jbeg;
    for (; j <= jend && j < jlo; j += U) p.template block<true>(j);
    for (; j <= jhi; j += U) p.template block<false>(j);
    for (; j <= jend; j += U) p.template block<true>(j);
}

template <typename T, int NPRE, int NPOST, bool JAC = false>
__global__ __launch_bounds__(NT) void k_recomp(SegTable<T> tab) {
    __shared__ cplx<T> bring[NT / 64][12 * 64];  // right-hand side rows, one ring per wave
    const int gw = (int)xcd_block().x * (NT / 64) + __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int lane = threadIdx.x & 63;
    const LevelSeg<T> S = seg_of_wave(tab, gw);
    const int lw = gw - S.w0;
    if (lw >= S.waves) return;
    const Piece pc = piece_of(S, lw);
    if (pc.k0 > pc.k1 || !S.active[pc.sys]) return;
    recomp_piece<T, NPRE, NPOST, JAC>(S, pc.sys, pc.strip, pc.k0, pc.k1, lane, bring[threadIdx.x >> 6]);
}

// ---------------------------------------------------------------------------
// Boundary of two refinement steps (complex64 V-cycles inside FP64
// refinement) on the finest level, in one pass.  Inputs: the last inner
// cycle's pre-smoothed complex64 correction e, its coarse correction, the
// inner right-hand side r (complex64), the FP64 iterate x and right-hand side
// b.  Stages, each a row stencil as in the cycle-edge kernel:
//   e <- e + P e_c, NA sweeps on L e = r           (complex64; ends step k)
//   x' = x + e, r' = b - L x'                        (FP64; norm partials of r',
//                                                    the step's stopping test)
//   u = 0, NB sweeps on L u = r', FW(r' - L u)       (complex64; the first
//                                                    inner cycle of step k+1)
// Writes x' (FP64), r' rounded to complex64 (the next step's right-hand
// side), u (the next cycle's pre-smoothed iterate) and the coarse right-hand
// side.  The first sweep from zero is the update alone (its residual is r').
template <int NA, int NB, bool JAC>
struct IrEdgePipe {
    using T = float;
    using C = float2;
    using D = double2;
    static constexpr int NS = NA + NB;
    static constexpr int HALO = 2 * NS + 2;
    static constexpr int OWN = 64 - 2 * HALO;
    static constexpr int COL0 = 1;
    static_assert(2 * NS + 1 <= 12 && 2 * NB + 1 <= 6, "ring lengths");
    C X[NS + 1][3], R[NS + 1][3];
    C* B;              // this lane's column of the wave's 12-row ring of r (stride 64)
    C RP[6];           // ring of r' rows for the sweeps of step k+1
    C xr[EPF + 1], br[EPF + 1];
    D xhr[EPF + 1], bhr[EPF + 1];  // FP64 x and b rows fetched ahead
    D XP[3];           // x' rows
    C er[3], ei[3];
    rsrc_t xs, bs, es, xos, cbs, xhs, xhos, bhs, bnos;
    LevelView lf, lc;
    Coef<T> cf;
    C dl;
    T sl;
    D dh;              // FP64 d on interior columns, else 0
    double shl;        // FP64 1/h^2 on interior columns, else 0
    int k0, k1;
    bool col_in, odd;
    T mk, hf;
    unsigned ox, oe, oo, of, oxh, ooh;
    unsigned rx, rc, rxh;
    double acc;

    template <bool EDGE> __device__ __forceinline__ C load_x(int j) const {
        C v;
        if constexpr (EDGE) bload(xs, ox + (in_rows(j, lf.ny) ? j * rx : OOB), 0, v);
        else bload(xs, ox, srow(j, rx), v);
        return v;
    }
    template <bool EDGE> __device__ __forceinline__ C load_b(int j) const {
        C v;
        if constexpr (EDGE) bload(bs, ox + (in_rows(j, lf.ny) ? j * rx : OOB), 0, v);
        else bload(bs, ox, srow(j, rx), v);
        return v;
    }
    template <bool EDGE> __device__ __forceinline__ D load_xh(int j) const {
        D v;
        if constexpr (EDGE) bload(xhs, oxh + (in_rows(j, lf.ny) ? j * rxh : OOB), 0, v);
        else bload(xhs, oxh, srow(j, rxh), v);
        return v;
    }
    template <bool EDGE> __device__ __forceinline__ D load_bh(int j) const {
        D v;
        if constexpr (EDGE) bload(bhs, oxh + (in_rows(j, lf.ny) ? j * rxh : OOB), 0, v);
        else bload(bhs, oxh, srow(j, rxh), v);
        return v;
    }
    template <bool EDGE> __device__ __forceinline__ C load_e(int K) const {
        C v;
        if constexpr (EDGE) bload(es, oe + (K >= 0 && K <= lc.ny + 1 ? K * rc : OOB), 0, v);
        else bload(es, oe, srow(K, rc), v);
        return v;
    }
    __device__ __forceinline__ C interp_x(C v) const {
        const C rv = from_right(v);
        C r;
        r.x = fmar(hf, rv.x - v.x, v.x);
        r.y = fmar(hf, rv.y - v.y, v.y);
        return r;
    }
    // store of an owned row (rows k0..k1) of a plane with bytes-per-row rb
    template <bool EDGE, typename V>
    __device__ __forceinline__ void store_at(rsrc_t r, unsigned off, unsigned rb, int row, V v) const {
        if constexpr (EDGE) bstore(r, off + (row >= k0 && row <= k1 ? row * rb : OOB), 0, v);
        else bstore(r, off, srow(row, rb), v);
    }
    template <int P, bool EDGE> __device__ __forceinline__ void step(int j) {
        xr[eslot<EPF + 1>(P + EPF)] = load_x<EDGE>(j + EPF);
        br[eslot<EPF + 1>(P + EPF)] = load_b<EDGE>(j + EPF - 1);
        // FP64 x at the row where e ends (j - 2NA), b one row above
        xhr[eslot<EPF + 1>(P + EPF)] = load_xh<EDGE>(j + EPF - 2 * NA);
        bhr[eslot<EPF + 1>(P + EPF)] = load_bh<EDGE>(j + EPF - 2 * NA - 1);
        C e;
        if constexpr ((P & 1) != 0) {
            constexpr int lo = eslot<3>((P - 1) / 2), hi = eslot<3>((P + 1) / 2);
            ei[hi] = interp_x(er[hi]);
            e = cscale(cadd(ei[lo], ei[hi]), (T)0.5);
        } else {
            er[eslot<3>(P / 2 + 2)] = load_e<EDGE>((j >> 1) + 2);
            e = ei[eslot<3>(P / 2)];
        }
        constexpr int n0 = eslot<3>(P), n1 = eslot<3>(P - 1), n2 = eslot<3>(P - 2);
        X[0][n0] = cadd(xr[eslot<EPF + 1>(P)], e);
        B[eslot<12>(P) * 64] = br[eslot<EPF + 1>(P)];
#pragma unroll
        for (int q = 0; q <= NS; ++q) {
            const int rrow = j - 2 * q - 1;
            C r;
            if (q == NA) {
                // x' = x + e at row j - 2NA, then the FP64 residual of x' at row
                // j - 2NA - 1 (the refinement step's stopping test)
                const C ev = X[NA][n0];
                D xp = xhr[eslot<EPF + 1>(P)];
                xp.x += (double)ev.x;
                xp.y += (double)ev.y;
                XP[n0] = xp;
                store_at<EDGE>(xhos, ooh, rxh, j - 2 * NA, xp);
                D rh = residual_row<double>(XP[n2], XP[n1], XP[n0], bhr[eslot<EPF + 1>(P)], dh, shl);
                if constexpr (EDGE)
                    if (!in_rows(rrow, lf.ny)) rh = czero<D>();
                if (!EDGE || (rrow >= k0 && rrow <= k1)) acc += rh.x * rh.x + rh.y * rh.y;
                pin(acc);
                pin(XP[n0]);
                r = cvt<C>(rh);
                RP[eslot<6>(P)] = r;
                store_at<EDGE>(bnos, oo, rx, rrow, r);
            } else {
                const C bq = q < NA ? B[eslot<12>(P - 2 * q) * 64] : RP[eslot<6>(P - 2 * (q - NA))];
                r = residual_row<T>(X[q][n2], X[q][n1], X[q][n0], bq, dl, sl);
                if constexpr (EDGE)
                    if (!in_rows(rrow, lf.ny)) r = czero<C>();
            }
            R[q][n0] = r;
            pin(R[q][n0]);
            if (q < NS) {
                // (the first sweep of step k+1 starts from zero)
                C v = vanka_row<T, JAC>(q == NA ? czero<C>() : X[q][n2], R[q][n2], R[q][n1], R[q][n0], cf, mk);
                if constexpr (EDGE)
                    if (!in_rows(j - 2 * q - 2, lf.ny)) v = czero<C>();
                X[q + 1][n0] = v;
                pin(X[q + 1][n0]);
            }
        }
        pin(X[0][n0]);
        store_at<EDGE>(xos, oo, rx, j - 2 * NS, X[NS][n0]);
        if constexpr ((P & 1) == 0) {
            const int frow = j - 2 * NS - 2;
            const C v = full_weight_row<T>(R[NS][n2], R[NS][n1], R[NS][n0]);
            const int K = frow >> 1;
            if constexpr (EDGE)
                bstore(cbs, of + (frow >= k0 && frow <= k1 && frow >= 2 && K <= lc.ny ? K * rc : OOB), 0, v);
            else bstore(cbs, of, srow(K, rc), v);
        }
    }
    template <bool EDGE> __device__ __forceinline__ void block(int j) {
#define VMG_E(P)                      \
    step<P, EDGE>(j + P);             \
    __builtin_amdgcn_sched_barrier(0);
        VMG_E(0) VMG_E(1) VMG_E(2) VMG_E(3) VMG_E(4) VMG_E(5)
        VMG_E(6) VMG_E(7) VMG_E(8) VMG_E(9) VMG_E(10) VMG_E(11)
#undef VMG_E
    }
};

template <int NA, int NB, bool JAC, bool PACE>
__device__ __forceinline__ double ir_edge_piece(const LevelSeg<float>& S, int sys, int strip, int k0, int k1, int lane,
                                                float2* bring) {
    using C = float2;
    using D = double2;
    using Pipe = IrEdgePipe<NA, NB, JAC>;
    constexpr int HALO = Pipe::HALO, OWN = Pipe::OWN, NS = Pipe::NS, U = UNR_E;
    Pipe p;
    p.B = bring + lane;
    p.lf = S.lf;
    p.lc = S.lc;
    const int i = Pipe::COL0 + strip * OWN - HALO + lane;
    p.col_in = i >= 1 && i <= p.lf.nx;
    p.mk = p.col_in ? 1.0f : 0.0f;
    p.odd = (i & 1) != 0;
    p.hf = p.odd ? 0.5f : 0.0f;
    const bool ecol = i >= 0 && i <= p.lf.nx + 1;
    const bool own = lane >= HALO && lane < HALO + OWN && p.col_in;
    const unsigned es = sizeof(C), eh = sizeof(D);
    p.ox = p.col_in ? i * es : OOB;
    p.oe = ecol ? (i >> 1) * es : OOB;
    p.oo = own ? i * es : OOB;
    p.of = (own && !(i & 1) && (i >> 1) <= p.lc.nx) ? (i >> 1) * es : OOB;
    p.rx = p.lf.pitch * es;
    p.rc = p.lc.pitch * es;
    // the FP64 planes of the finest level have their own pitch (S.lh); x' is
    // written on owned columns only; with no FP64 iterate yet (x = 0) every
    // read of it goes through an empty range and returns zero
    p.oxh = p.col_in ? i * eh : OOB;
    p.ooh = own ? i * eh : OOB;
    p.rxh = S.lh.pitch * eh;
    const int64_t bhase = (int64_t)sys * S.lh.plane;
    p.xhs = S.xh ? plane_rsrc(S.xh + bhase, S.lh.plane) : plane_rsrc(S.xho + bhase, 0);
    p.bhs = plane_rsrc(S.bh + bhase, S.lh.plane);
    p.xhos = plane_rsrc(S.xho + bhase, S.lh.plane);
    p.k0 = k0;
    p.k1 = k1;
    const int64_t base = (int64_t)sys * p.lf.plane;
    p.xs = plane_rsrc(S.x + base, p.lf.plane);
    p.bs = plane_rsrc(S.b + base, p.lf.plane);
    p.es = plane_rsrc(S.c + (int64_t)sys * p.lc.plane, p.lc.plane);
    p.xos = plane_rsrc(S.xo + base, p.lf.plane);
    p.cbs = plane_rsrc(S.cb + (int64_t)sys * p.lc.plane, p.lc.plane);
    p.bnos = plane_rsrc(S.bno + base, p.lf.plane);
    p.cf = S.coef[sys];
    p.dl = p.col_in ? p.cf.d : czero<C>();
    p.sl = p.col_in ? S.s : 0.0f;
    const Coef<double> ch = S.coefh[sys];
    p.dh = p.col_in ? ch.d : czero<D>();
    p.shl = p.col_in ? S.sh : 0.0;
    p.acc = 0.0;
#pragma unroll
    for (int q = 0; q <= NS; ++q)
#pragma unroll
        for (int w = 0; w < 3; ++w) p.X[q][w] = p.R[q][w] = czero<C>();
#pragma unroll
    for (int w = 0; w < 3; ++w) p.XP[w] = czero<D>();
#pragma unroll
    for (int w = 0; w < 6; ++w) p.RP[w] = czero<C>();
#pragma unroll
    for (int w = 0; w < 12; ++w) p.B[w * 64] = czero<C>();
    int jbeg = k0 - 2 * NS - 2;
    jbeg -= jbeg & 1;
    const int jend = k1 + 2 * NS + 2;
    const int jlo = max(k0 + 2 * NS + 2, 2 * NS + 4);
    const int jhi = min(min(p.lf.ny - U + 1 - EPF, p.lf.ny - U - 1), k1 - U + 1 + 2 * NA);
    p.ei[0] = p.interp_x(p.template load_e<true>(jbeg >> 1));
    p.er[1] = p.template load_e<true>((jbeg >> 1) + 1);
#pragma unroll
    for (int d = 0; d < EPF; ++d) {
        p.xr[d] = p.template load_x<true>(jbeg + d);
        p.br[d] = p.template load_b<true>(jbeg + d - 1);
        p.xhr[d] = p.template load_xh<true>(jbeg + d - 2 * NA);
        p.bhr[d] = p.template load_bh<true>(jbeg + d - 2 * NA - 1);
    }
    // (PACE: as in edge_piece)
    int j = jbeg;
    for (; j <= jend && j < jlo; j += U) {
        p.template block<true>(j);
        if constexpr (PACE) __syncthreads();
    }
    for (; j <= jhi; j += U) {
        p.template block<false>(j);
        if constexpr (PACE) __syncthreads();
    }
    for (; j <= jend; j += U) {
        p.template block<true>(j);
        if constexpr (PACE) __syncthreads();
    }
    return own ? p.acc : 0.0;
}

template <int NA, int NB, bool JAC, int WB = NT / 64>
__global__ __launch_bounds__(64 * WB) void k_ir_edge(SegTable<float> tab) {
    __shared__ float2 bring[WB][12 * 64];  // inner right-hand side rows, one ring per wave
    const int gw = (int)xcd_block().x * WB + __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int lane = threadIdx.x & 63;
    const LevelSeg<float> S = seg_of_wave(tab, gw);
    const int lw = gw - S.w0;
    if (lw >= S.waves) return;
    const Piece pc = piece_of(S, lw);
    if (!S.active[pc.sys]) return;
    double acc = ir_edge_piece<NA, NB, JAC, (WB > NT / 64)>(S, pc.sys, pc.strip, pc.k0, pc.k1, lane,
                                                         bring[threadIdx.x >> 6]);
    if (S.partial) {
        for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
        if (lane == 0) S.partial[pc.slot] = acc;
    }
}

template <typename T>
__global__ __launch_bounds__(NT) void k_fill_zero(cplx<T>* __restrict__ x, LevelView lv) {
    const int i = blockIdx.x * 64 + (threadIdx.x & 63) + 1;
    if (i > lv.nx) return;
    for (int k = blockIdx.y * 16 + (threadIdx.x >> 6) + 1; k <= min(lv.ny, (int)(blockIdx.y + 1) * 16); k += NT / 64)
        x[(int64_t)blockIdx.z * lv.plane + (int64_t)k * lv.pitch + i] = czero<cplx<T>>();
}

template <int NS> constexpr int down_own() { return DownPipe<double, NS>::OWN; }
template <int NS, bool NORM> constexpr int up_own() { return UpPipe<double, NS, NORM>::OWN; }

// Waves of one kernel that are resident on the whole device at once, in
// blocks of `threads`.
int resident_waves(const void* kernel, int threads = NT) {
    static std::mutex mu;
    static std::map<std::pair<const void*, int>, int> cache;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) dev = 0;
    std::lock_guard<std::mutex> lock(mu);
    auto it = cache.find({kernel, dev});
    if (it != cache.end()) return it->second;
    int blocks = 0, cus = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, kernel, threads, 0) != hipSuccess || blocks < 1)
        blocks = 1;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1) cus = 1;
    const int w = blocks * cus * (threads / 64);
    cache[{kernel, dev}] = w;
    return w;
}

// Cut of one segment's strips into runs of rows, one run per wave.  The
// number of runs per strip p minimises (rounds of resident waves) x (rows per
// run + the pipeline's start-up rows), with runs of at least
// max(rmin, MIN_RUN) rows.
constexpr int MIN_RUN = 16;
struct RunGeom {
    int strips, pieces, rows, waves;
};
RunGeom run_geom(int nx, int ny, int nsys, int own, int col0, int halo_rows, int rmin, int resident) {
    RunGeom g;
    g.strips = (nx + 1 - col0 + own - 1) / own;  // strips cover columns col0..nx
    const int64_t runs1 = (int64_t)nsys * g.strips;
    const int pmax = std::max(1, ny / std::max(rmin, MIN_RUN));
    int best = 1;
    int64_t best_cost = -1;
    for (int p = 1; p <= pmax; ++p) {
        const int rows = (ny + p - 1) / p;
        const int64_t rounds = (runs1 * p + resident - 1) / resident;
        const int64_t cost = rounds * (rows + halo_rows);
        if (best_cost < 0 || cost < best_cost) {
            best_cost = cost;
            best = p;
        }
    }
    g.rows = (ny + best - 1) / best;
    g.pieces = (ny + g.rows - 1) / g.rows;
    g.waves = (int)(runs1 * g.pieces);
    return g;
}

template <typename T>
dim3 stream_seg_grid(SegTable<T>& tab, const int* nsys, int own, int col0, int halo_rows, int rmin, int resident) {
    int w = 0;
    for (int q = 0; q < tab.n; ++q) {
        LevelSeg<T>& S = tab.s[q];
        const RunGeom g = run_geom(S.lf.nx, S.lf.ny, nsys[q], own, col0, halo_rows, rmin, resident);
        S.z0 = 0;
        S.nsys = nsys[q];
        S.strips = g.strips;
        S.rows = g.rows;
        S.pieces = g.pieces;
        S.waves = g.waves;
        S.w0 = w;
        w += g.waves;
    }
    return dim3((w + NT / 64 - 1) / (NT / 64));
}

// (the run geometry always follows the occupancy of the kernel whose coarse
// level has the precision of its own, so that a kernel reading or writing
// complex64 coarse values splits its level, and its norm partial sums, the
// same way)
// Paced blocks (see edge_piece) for the FP64 Vanka kernels with two sweeps
// that open and close a solve on the finest level: WB = the waves a CU holds
// of the plain kernel (12 for k_down, 16 for k_up without the norm), launched
// only where a CU holds one block of them, so that the run geometry the plain
// grid was cut for stays the same.
template <int WB, typename T> dim3 paced_grid(const SegTable<T>& tab, const void* kp, int resident) {
    if (resident_waves(kp, 64 * WB) != resident) return dim3(0);
    const int w = tab.s[tab.n - 1].w0 + tab.s[tab.n - 1].waves;
    return dim3((w + WB - 1) / WB);
}
constexpr int DOWN_WB = 12, UP_WB = 16;

template <typename T, int NS, typename TC>
void down_go(SegTable<T> tab, const int* nsys, int rmin, hipStream_t st, bool paced) {
    const void* k = (const void*)&k_down<T, NS, T>;
    const int resident = resident_waves(k);
    const dim3 g = stream_seg_grid(tab, nsys, down_own<NS>(), 1, 4 * NS + 9, rmin, resident);
    if (g.x == 0) return;
    if constexpr (std::is_same<T, double>::value && NS == 2) {
        if (paced && !tab.s[0].jacobi) {
            const dim3 gp = paced_grid<DOWN_WB>(tab, (const void*)&k_down<T, NS, TC, false, DOWN_WB>, resident);
            if (gp.x) {
                hipLaunchKernelGGL((k_down<T, NS, TC, false, DOWN_WB>), gp, dim3(64 * DOWN_WB), 0, st, tab);
                return;
            }
        }
    }
    if (tab.s[0].jacobi) hipLaunchKernelGGL((k_down<T, NS, TC, true>), g, dim3(NT), 0, st, tab);
    else hipLaunchKernelGGL((k_down<T, NS, TC, false>), g, dim3(NT), 0, st, tab);
}
template <typename T, int NS, bool NORM, typename TC>
void up_go(SegTable<T> tab, const int* nsys, int rmin, hipStream_t st, bool paced) {
    const void* k = (const void*)&k_up<T, NS, NORM, T>;
    const int resident = resident_waves(k);
    const dim3 g = stream_seg_grid(tab, nsys, up_own<NS, NORM>(), UpPipe<T, NS, NORM>::COL0, 4 * NS + 7, rmin, resident);
    if (g.x == 0) return;
    if constexpr (std::is_same<T, double>::value && NS == 2 && !NORM) {
        if (paced && !tab.s[0].jacobi) {
            const dim3 gp = paced_grid<UP_WB>(tab, (const void*)&k_up<T, NS, NORM, TC, false, UP_WB>, resident);
            if (gp.x) {
                hipLaunchKernelGGL((k_up<T, NS, NORM, TC, false, UP_WB>), gp, dim3(64 * UP_WB), 0, st, tab);
                return;
            }
        }
    }
    if (tab.s[0].jacobi) hipLaunchKernelGGL((k_up<T, NS, NORM, TC, true>), g, dim3(NT), 0, st, tab);
    else hipLaunchKernelGGL((k_up<T, NS, NORM, TC, false>), g, dim3(NT), 0, st, tab);
}

template <typename T, int NA, int NB, typename TC>
void edge_go(SegTable<T> tab, const int* nsys, int rmin, hipStream_t st, bool paced) {
    using Pipe = EdgePipe<T, NA, NB>;
    const void* k = (const void*)&k_edge<T, NA, NB, T>;
    const int resident = resident_waves(k);
    dim3 g = stream_seg_grid(tab, nsys, Pipe::OWN, Pipe::COL0, 4 * Pipe::NS + 9, rmin, resident);
    if (g.x == 0) return;
    if constexpr (std::is_same<T, double>::value) {
        // paced blocks (Vanka only), where a CU holds as many of their waves as
        // of the plain blocks' (the run geometry above assumes that count)
        const void* kp = (const void*)&k_edge<T, NA, NB, TC, false, EDGE_WB>;
        if (paced && !tab.s[0].jacobi && resident_waves(kp, 64 * EDGE_WB) == resident) {
            const int w = tab.s[tab.n - 1].w0 + tab.s[tab.n - 1].waves;
            g.x = (w + EDGE_WB - 1) / EDGE_WB;
            hipLaunchKernelGGL((k_edge<T, NA, NB, TC, false, EDGE_WB>), g, dim3(64 * EDGE_WB), 0, st, tab);
            return;
        }
    }
    if (tab.s[0].jacobi) hipLaunchKernelGGL((k_edge<T, NA, NB, TC, true>), g, dim3(NT), 0, st, tab);
    else hipLaunchKernelGGL((k_edge<T, NA, NB, TC, false>), g, dim3(NT), 0, st, tab);
}

template <typename T, int NPRE, int NPOST> void recomp_go(SegTable<T> tab, const int* nsys, int rmin, hipStream_t st) {
    using Pipe = RecompPipe<T, NPRE, NPOST>;
    const void* k = (const void*)&k_recomp<T, NPRE, NPOST>;
    const dim3 g = stream_seg_grid(tab, nsys, Pipe::OWN, Pipe::COL0, 4 * Pipe::NS + 1, rmin, resident_waves(k));
    if (g.x == 0) return;
    hipLaunchKernelGGL((k_recomp<T, NPRE, NPOST>), g, dim3(NT), 0, st, tab);
}

template <typename T, int NA, int NB> int edge_tiles_of(int nx, int ny, int nsys, int rmin) {
    using Pipe = EdgePipe<T, NA, NB>;
    const RunGeom g = run_geom(nx, ny, nsys, Pipe::OWN, Pipe::COL0, 4 * Pipe::NS + 9, rmin,
                               resident_waves((const void*)&k_edge<T, NA, NB, T>));
    return g.strips * g.pieces;
}

}  // namespace

bool edge_supported(int nu1, int nu2) { return nu1 >= 1 && nu1 <= 2 && nu2 >= 1 && nu2 <= 2; }

template <typename T, typename TC>
void edge_launch(SegTable<T> tab, const int* nsys, int nu1, int nu2, int rmin, hipStream_t st, bool paced) {
    if (nu2 == 1 && nu1 == 1) edge_go<T, 1, 1, TC>(tab, nsys, rmin, st, paced);
    else if (nu2 == 1 && nu1 == 2) edge_go<T, 1, 2, TC>(tab, nsys, rmin, st, paced);
    else if (nu2 == 2 && nu1 == 1) edge_go<T, 2, 1, TC>(tab, nsys, rmin, st, paced);
    else edge_go<T, 2, 2, TC>(tab, nsys, rmin, st, paced);
}
template <typename T>
void launch_edge(SegTable<T> tab, const int* nsys, int nu1, int nu2, int rmin, hipStream_t st, bool c32, bool paced) {
    if constexpr (std::is_same<T, double>::value) {
        if (c32) {
            edge_launch<double, float>(tab, nsys, nu1, nu2, rmin, st, paced);
            return;
        }
    }
    edge_launch<T, T>(tab, nsys, nu1, nu2, rmin, st, paced);
}
template void launch_edge<double>(SegTable<double>, const int*, int, int, int, hipStream_t, bool, bool);
template void launch_edge<float>(SegTable<float>, const int*, int, int, int, hipStream_t, bool, bool);

template <typename T> void launch_recomp(SegTable<T> tab, const int* nsys, int nu1, int nu2, int rmin, hipStream_t st) {
    if (nu1 == 1 && nu2 == 1) recomp_go<T, 1, 1>(tab, nsys, rmin, st);
    else if (nu1 == 1 && nu2 == 2) recomp_go<T, 1, 2>(tab, nsys, rmin, st);
    else if (nu1 == 2 && nu2 == 1) recomp_go<T, 2, 1>(tab, nsys, rmin, st);
    else recomp_go<T, 2, 2>(tab, nsys, rmin, st);
}
template void launch_recomp<double>(SegTable<double>, const int*, int, int, int, hipStream_t);
template void launch_recomp<float>(SegTable<float>, const int*, int, int, int, hipStream_t);

template <typename T> int edge_tiles(int nx, int ny, int nsys, int nu1, int nu2, int rmin) {
    if (nu2 == 1 && nu1 == 1) return edge_tiles_of<T, 1, 1>(nx, ny, nsys, rmin);
    if (nu2 == 1 && nu1 == 2) return edge_tiles_of<T, 1, 2>(nx, ny, nsys, rmin);
    if (nu2 == 2 && nu1 == 1) return edge_tiles_of<T, 2, 1>(nx, ny, nsys, rmin);
    return edge_tiles_of<T, 2, 2>(nx, ny, nsys, rmin);
}
template int edge_tiles<double>(int, int, int, int, int, int);
template int edge_tiles<float>(int, int, int, int, int, int);

namespace {
// (the run geometry follows the Vanka kernel's occupancy for both smoothers,
// as the norm partial sums are counted with it)
template <int NA, int NB> void ir_edge_go(SegTable<float> tab, const int* nsys, int rmin, hipStream_t st, bool paced) {
    using Pipe = IrEdgePipe<NA, NB, false>;
    const int resident = resident_waves((const void*)&k_ir_edge<NA, NB, false>);
    dim3 g = stream_seg_grid(tab, nsys, Pipe::OWN, Pipe::COL0, 4 * Pipe::NS + 9, rmin, resident);
    if (g.x == 0) return;
    // paced blocks as for the cycle-edge kernel (Vanka; where a CU holds as
    // many of their waves as of the plain blocks')
    const void* kp = (const void*)&k_ir_edge<NA, NB, false, EDGE_WB>;
    if (paced && !tab.s[0].jacobi && resident_waves(kp, 64 * EDGE_WB) == resident) {
        const int w = tab.s[tab.n - 1].w0 + tab.s[tab.n - 1].waves;
        g.x = (w + EDGE_WB - 1) / EDGE_WB;
        hipLaunchKernelGGL((k_ir_edge<NA, NB, false, EDGE_WB>), g, dim3(64 * EDGE_WB), 0, st, tab);
        return;
    }
    if (tab.s[0].jacobi) hipLaunchKernelGGL((k_ir_edge<NA, NB, true>), g, dim3(NT), 0, st, tab);
    else hipLaunchKernelGGL((k_ir_edge<NA, NB, false>), g, dim3(NT), 0, st, tab);
}
template <int NA, int NB> int ir_edge_tiles_of(int nx, int ny, int nsys, int rmin) {
    using Pipe = IrEdgePipe<NA, NB, false>;
    const RunGeom g = run_geom(nx, ny, nsys, Pipe::OWN, Pipe::COL0, 4 * Pipe::NS + 9, rmin,
                               resident_waves((const void*)&k_ir_edge<NA, NB, false>));
    return g.strips * g.pieces;
}
}  // namespace

void launch_ir_edge(SegTable<float> tab, const int* nsys, int nu1, int nu2, int rmin, hipStream_t st, bool paced) {
    if (nu2 == 1 && nu1 == 1) ir_edge_go<1, 1>(tab, nsys, rmin, st, paced);
    else if (nu2 == 1 && nu1 == 2) ir_edge_go<1, 2>(tab, nsys, rmin, st, paced);
    else if (nu2 == 2 && nu1 == 1) ir_edge_go<2, 1>(tab, nsys, rmin, st, paced);
    else ir_edge_go<2, 2>(tab, nsys, rmin, st, paced);
}
int ir_edge_tiles(int nx, int ny, int nsys, int nu1, int nu2, int rmin) {
    if (nu2 == 1 && nu1 == 1) return ir_edge_tiles_of<1, 1>(nx, ny, nsys, rmin);
    if (nu2 == 1 && nu1 == 2) return ir_edge_tiles_of<1, 2>(nx, ny, nsys, rmin);
    if (nu2 == 2 && nu1 == 1) return ir_edge_tiles_of<2, 1>(nx, ny, nsys, rmin);
    return ir_edge_tiles_of<2, 2>(nx, ny, nsys, rmin);
}

template <typename T> int stream_tiles(int nx, int ny, int nsys, int nu, int rmin) {
    const void* k;
    int own;
    switch (nu) {
        case 0: k = (const void*)&k_up<T, 0, true, T>; own = up_own<0, true>(); break;
        case 1: k = (const void*)&k_up<T, 1, true, T>; own = up_own<1, true>(); break;
        default: k = (const void*)&k_up<T, 2, true, T>; own = up_own<2, true>(); break;
    }
    const RunGeom g = run_geom(nx, ny, nsys, own, UpPipe<T, 2, true>::COL0, 4 * (nu < 2 ? nu : 2) + 7, rmin,
                               resident_waves(k));
    return g.strips * g.pieces;
}
template int stream_tiles<double>(int, int, int, int, int);
// Occupancy queries of every streaming kernel up front (not inside a stream
// capture).
void stream_prepare() {
#define VMG_PREP(T)                                                                                   \
    resident_waves((const void*)&k_down<T, 0, T>), resident_waves((const void*)&k_down<T, 1, T>),             \
        resident_waves((const void*)&k_down<T, 2, T>), resident_waves((const void*)&k_up<T, 0, true, T>),      \
        resident_waves((const void*)&k_up<T, 1, true, T>), resident_waves((const void*)&k_up<T, 2, true, T>),  \
        resident_waves((const void*)&k_up<T, 0, false, T>), resident_waves((const void*)&k_up<T, 1, false, T>), \
        resident_waves((const void*)&k_up<T, 2, false, T>), resident_waves((const void*)&k_edge<T, 1, 1, T>),  \
        resident_waves((const void*)&k_edge<T, 1, 2, T>), resident_waves((const void*)&k_edge<T, 2, 1, T>),    \
        resident_waves((const void*)&k_edge<T, 2, 2, T>)
    VMG_PREP(double);
    VMG_PREP(float);
#undef VMG_PREP
    resident_waves((const void*)&k_ir_edge<1, 1, false>), resident_waves((const void*)&k_ir_edge<1, 2, false>),
        resident_waves((const void*)&k_ir_edge<2, 1, false>), resident_waves((const void*)&k_ir_edge<2, 2, false>);
}

int stream_tiles_max(int nx, int ny, int nu) {
    // the narrowest strips of any kernel that forms the norm: the cycle-edge kernel's
    const int own = std::min(EdgePipe<double, 2, 2>::OWN,
                             nu == 0 ? up_own<0, true>() : (nu == 1 ? up_own<1, true>() : up_own<2, true>()));
    return ((nx + own) / own) * std::max(1, ny / MIN_RUN);
}
template int stream_tiles<float>(int, int, int, int, int);

template <typename T, typename TC>
void down_launch(SegTable<T> tab, const int* nsys, int nu, int ty, hipStream_t st, bool paced) {
    switch (nu) {
        case 0: down_go<T, 0, TC>(tab, nsys, ty, st, paced); break;
        case 1: down_go<T, 1, TC>(tab, nsys, ty, st, paced); break;
        default: down_go<T, 2, TC>(tab, nsys, ty, st, paced); break;
    }
}
template <typename T>
void launch_down(SegTable<T> tab, const int* nsys, int nu, int ty, hipStream_t st, bool c32, bool paced) {
    if constexpr (std::is_same<T, double>::value) {
        if (c32) {
            down_launch<double, float>(tab, nsys, nu, ty, st, paced);
            return;
        }
    }
    down_launch<T, T>(tab, nsys, nu, ty, st, paced);
}

template <typename T, typename TC>
void up_launch(SegTable<T> tab, const int* nsys, int nu, bool norm, int ty, hipStream_t st, bool paced) {
    switch (nu) {
        case 0:
            if (norm) up_go<T, 0, true, TC>(tab, nsys, ty, st, paced);
            else up_go<T, 0, false, TC>(tab, nsys, ty, st, paced);
            break;
        case 1:
            if (norm) up_go<T, 1, true, TC>(tab, nsys, ty, st, paced);
            else up_go<T, 1, false, TC>(tab, nsys, ty, st, paced);
            break;
        default:
            if (norm) up_go<T, 2, true, TC>(tab, nsys, ty, st, paced);
            else up_go<T, 2, false, TC>(tab, nsys, ty, st, paced);
            break;
    }
}
template <typename T>
void launch_up(SegTable<T> tab, const int* nsys, int nu, bool norm, int ty, hipStream_t st, bool c32, bool paced) {
    if constexpr (std::is_same<T, double>::value) {
        if (c32) {
            up_launch<double, float>(tab, nsys, nu, norm, ty, st, paced);
            return;
        }
    }
    up_launch<T, T>(tab, nsys, nu, norm, ty, st, paced);
}

template <typename T> void launch_fill_zero(cplx<T>* x, LevelView lv, int nsys, hipStream_t st) {
    hipLaunchKernelGGL((k_fill_zero<T>), dim3((lv.nx + 63) / 64, (lv.ny + 15) / 16, nsys), dim3(NT), 0, st, x, lv);
}
template void launch_fill_zero<double>(double2*, LevelView, int, hipStream_t);
template void launch_fill_zero<float>(float2*, LevelView, int, hipStream_t);

template void launch_down<double>(SegTable<double>, const int*, int, int, hipStream_t, bool, bool);
template void launch_down<float>(SegTable<float>, const int*, int, int, hipStream_t, bool, bool);
template void launch_up<double>(SegTable<double>, const int*, int, bool, int, hipStream_t, bool, bool);
template void launch_up<float>(SegTable<float>, const int*, int, bool, int, hipStream_t, bool, bool);

}  // namespace vmg
