// Internal declarations shared by the kernels and the host runtime of the
// Vanka multigrid library (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace vmg {

template <typename T> struct cplx_t;
template <> struct cplx_t<double> { using type = double2; };
template <> struct cplx_t<float> { using type = float2; };
template <typename T> using cplx = typename cplx_t<T>::type;

// Geometry of one level of one grid.  Every system owns a padded plane of
// (ny + 2) rows of `pitch` elements; interior node (i, k), 1 <= i <= nx,
// 1 <= k <= ny, is element k * pitch + i of its plane, and the ring i or k in
// {0, n + 1} (plus the row padding beyond nx + 1) always holds zero.
struct LevelView {
    int nx, ny;
    int pitch;
    int64_t plane;
};

// Per (system, level) constants of the shifted operator and the smoother:
//   (L x)_p = d x_p - s (x_N + x_S + x_E + x_W),  d = 4/h^2 + lambda,  s = 1/h^2
//   x'_p = x_p + ca r_p + cb (r_N + r_S + r_E + r_W) + cc (r_NE + r_NW + r_SE + r_SW)
// For the Vanka stencil of eq. (6) with weight omega: ca = omega h^2 a,
// cb = omega h^2 b / 2, cc = omega h^2 c / 4, and the ratios alpha = ca / cb,
// gamma = cc / cb (the streaming kernels' form of the update).  For damped
// Jacobi: ca = omega/d (cb = cc = alpha = gamma = 0).
template <typename T> struct Coef {
    cplx<T> d, ca, cb, cc, alpha, gamma;
};

// One grid's share of a batched launch.  A launch covers up to MAXSEG grids
// (segments) that may differ in size; blockIdx.z runs over the systems of all
// segments (segment q owns z0[q] .. z0[q+1]-1) and blocks beyond a segment's
// own grid extent (gx, gy) return at once.
constexpr int MAXSEG = 8;
template <typename T> struct LevelSeg {
    const cplx<T>* x;     // iterate read (padded planes)
    const cplx<T>* b;     // right-hand side
    cplx<T>* xo;          // iterate written
    cplx<T>* c;           // coarse right-hand side written (restriction) or
                          // coarse correction read (prolongation)
    cplx<T>* cb;          // cycle-edge kernel: the next coarse right-hand side
    // refinement boundary (complex64 finest level of FP64 refinement): the
    // FP64 iterate read and written, the FP64 right-hand side, coefficients
    // and 1/h^2 of the finest level, and the next step's complex64
    // right-hand side written
    LevelView lh;         // (the finest level's FP64 planes)
    const double2* xh;
    double2* xho;
    const double2* bh;
    const Coef<double>* coefh;
    double sh;
    cplx<T>* bno;
    // finishing pass of the streaming correction + post-smoothing kernel (finest
    // level after cycle-edge cycles), else NULL: cycles run per system, the
    // iterate read after an odd count (x after an even one), dense destination
    const int* iters;
    const cplx<T>* xalt;
    cplx<T>* zd;
    LevelView lf, lc;     // this level and the next coarser one
    T s;                  // 1 / h^2 of this level
    const Coef<T>* coef;  // per system of the segment
    const int* active;    // per system of the segment
    const cplx<T>* cinvT; // coarsest level: transposed inverses
    double* partial;      // fused norm partial sums, or NULL
    int x_zero;           // the iterate read is zero (not loaded)
    int jacobi;           // damped Jacobi smoother instead of Vanka
    int nc;               // coarsest level: unknowns per system
    int z0;               // first blockIdx.z of the segment
    int gx, gy;           // blocks of the segment in x and y
    // streaming kernels (one wave per run of rows, see vmg_stream.hip)
    int nsys;             // systems of the segment
    int strips;           // column strips per system
    int rows;             // rows per run (one run per wave)
    int pieces;           // runs per strip
    int waves;            // waves of the segment
    int w0;               // first global wave of the segment
};
template <typename T> struct SegTable {
    int n;
    LevelSeg<T> s[MAXSEG];
};

#ifdef __HIPCC__
// Complex arithmetic on double2 / float2 (x the real part, y the imaginary
// part), written out so that every kernel rounds the same way.
template <typename C> __device__ __forceinline__ C czero() { C z; z.x = 0; z.y = 0; return z; }
template <typename C> __device__ __forceinline__ C cadd(C a, C b) { C r; r.x = a.x + b.x; r.y = a.y + b.y; return r; }
template <typename C> __device__ __forceinline__ C csub(C a, C b) { C r; r.x = a.x - b.x; r.y = a.y - b.y; return r; }
template <typename C, typename T> __device__ __forceinline__ C cscale(C a, T s) { C r; r.x = a.x * s; r.y = a.y * s; return r; }
template <typename C> __device__ __forceinline__ C cmul(C a, C b) {
    C r;
    r.x = a.x * b.x - a.y * b.y;
    r.y = a.x * b.y + a.y * b.x;
    return r;
}
// a + b * c
template <typename C> __device__ __forceinline__ C cfma(C a, C b, C c) {
    C r;
    r.x = a.x + b.x * c.x - b.y * c.y;
    r.y = a.y + b.x * c.y + b.y * c.x;
    return r;
}

// The hardware hands consecutive workgroups of a launch to the chip's eight
// XCDs in turn, and each XCD has its own L2.  Renumber the blocks so that
// every XCD receives one contiguous run of the logical order (x fastest):
// strips that share halo columns, or tiles that share the cache lines at
// their ends, then meet in the same L2.
constexpr unsigned NXCD = 8;
__device__ __forceinline__ uint3 xcd_block() {
    const unsigned gx = gridDim.x, gxy = gridDim.x * gridDim.y;
    const unsigned n = gxy * gridDim.z;
    const unsigned L = blockIdx.x + gx * blockIdx.y + gxy * blockIdx.z;
    const unsigned xcd = L % NXCD, k = L / NXCD, q = n / NXCD, r = n % NXCD;
    const unsigned Lp = xcd * q + min(xcd, r) + k;
    return make_uint3(Lp % gx, (Lp % gxy) / gx, Lp / gxy);
}

template <typename T> __device__ __forceinline__ LevelSeg<T> seg_of(const SegTable<T>& t, int z) {
    LevelSeg<T> r = t.s[0];
#pragma unroll
    for (int q = 1; q < MAXSEG; ++q)
        if (q < t.n && z >= t.s[q].z0) r = t.s[q];
    return r;
}
#endif

// Algorithmic (compulsory) bytes per fine node, complex element size E:
//   sweep: read x, b, write x'            3E
//   residual + restriction: read x, b; write r_H on a quarter of the nodes  2E + E/4
//   prolongation + correction: read x, e (quarter), write x               2E + E/4
//   norm: read x, b                        2E
struct KernelStats;

// ---- launchers (defined in vmg_kernels.hip); all enqueue on `st` ----
// Batched launchers: every segment's nsys systems, one launch.  nsys[q] is
// the system count of segment q (z0/gx/gy are filled in here).
//   sweep:    xo = x + omega M (b - L x)                      (x, b, xo)
//   restrict: c = FW(b - L x)                                 (x, b, c)
//   prolong:  xo = x + P c  (in place when xo == x)           (x, c, xo)
//   coarse:   xo = cinvT^T b                                  (b, xo, cinvT, nc)
template <typename T> void launch_sweep(SegTable<T> tab, const int* nsys, hipStream_t st);
template <typename T> void launch_restrict(SegTable<T> tab, const int* nsys, hipStream_t st);
template <typename T> void launch_prolong(SegTable<T> tab, const int* nsys, hipStream_t st);
template <typename T> void launch_coarse(SegTable<T> tab, const int* nsys, hipStream_t st);

// r = b - L x; optionally stores r (as TO, in layout lo) and per-tile partial
// sums of |r|^2 (partial[sys * ntiles + tile]).  Returns ntiles per system.
template <typename T, typename TO>
int launch_residual(const cplx<T>* x, const cplx<T>* b, cplx<TO>* rout, LevelView lv, LevelView lo, T s,
                    const Coef<T>* coef, const int* active, int nsys, int x_zero, double* partial,
                    hipStream_t st);
int residual_tiles(LevelView lv);
// End of a refinement step: xn = x + e (x = NULL: zero), rout = complex64 of
// b - L xn, |b - L xn|^2 per tile as launch_residual; e and rout in layout le.
int launch_ir_residual(const double2* x, const float2* e, const double2* b, double2* xn, float2* rout, LevelView lv,
                       LevelView le, double s, const Coef<double>* coef, const int* active, int nsys, double* partial,
                       hipStream_t st);



// unpadded <-> padded interior copies.  For unpack, if iters != NULL a system
// with iters[s] == 0 is written as zero, and if sel != NULL system s reads
// src1 instead of src0 when ((iters[s] * flips) & 1).
template <typename T>
// pack: with partial set, also |dst|^2 per system in residual_tiles(lv) tiles
// (partial[sys * tiles + t], the layout launch_residual writes)
void launch_pack(const cplx<T>* src, cplx<T>* dst, LevelView lv, int nsys, hipStream_t st, double* partial = nullptr);
template <typename T>
void launch_unpack(const cplx<T>* src0, const cplx<T>* src1, cplx<T>* dst, LevelView lv, int nsys,
                   const int* iters, int flips, hipStream_t st);

// Convergence bookkeeping (one thread block per system, fixed summation order).
// mode 0 (init): bb[s] = sum of partials; iters = 0; active = (bb > 0) && target > 0;
//                relres = active ? 1 : 0.
// mode 1 (check): for active systems: iters++, relres = sqrt(rr / bb), stop if
//                 NaN (flag), iters >= target, or (!fixed && relres <= tol).
void launch_norm_finalize(const double* partial, int ntiles, int nsys, int sys_off, int mode, double tol,
                          int fixed, double* bb, double* relres, int* iters, int* active, const int* target,
                          int* nanflag, hipStream_t st);

void launch_fill_int(int* p, int value, int n, hipStream_t st);

// Small levels in one workgroup per system (vmg_tail.hip): the cycle
// MG(lt, x, b) of levels lt..coarsest with gamma visits, nu1/nu2 sweeps.
// One TailSeg per grid (device table built once); a launch names up to
// MAXSEG of them with their x buffers and system offsets.
constexpr int MAXT = 6;  // levels of a tail, coarsest included
template <typename T> struct TailSeg {
    const cplx<T>* b;          // right-hand side of the first tail level (padded planes)
    LevelView gv;              // its global geometry
    LevelView lv[MAXT];        // every tail level (nx, ny used)
    T s[MAXT];                 // 1 / h^2 per level
    const Coef<T>* coef[MAXT]; // per level, per system
    const cplx<T>* cinvT;      // coarsest inverses, transposed
    const int* active;         // per system
    int nc;                    // coarsest unknowns per system
    int nl;                    // tail levels
};
template <typename T> struct TailLaunch {
    int n;
    int seg[MAXSEG];           // index into the TailSeg table
    int z0[MAXSEG];            // first workgroup (system) of the entry
    int xz[MAXSEG];            // first tail level starts from x = 0
    cplx<T>* x[MAXSEG];        // x of the first tail level (read unless xz, written)
    // whole solves (maxc > 0; the tail starts at the finest level): up to
    // maxc cycles per system, each followed by the stopping test of the
    // finest level's residual, on the per-system state at index sys0 + system
    int maxc;
    int fixed;                 // fixed counts: stop at target only
    double tol;
    int sys0[MAXSEG];
    const double* bb;          // |b|^2
    double* relres;
    int* iters;
    int* active;
    const int* target;
    int* nanflag;
};
template <typename T>
void launch_tail(const TailSeg<T>* segs, const TailLaunch<T>& tl, int total_sys, int64_t lds_bytes, int nu1, int nu2,
                 int gamma, hipStream_t st);
template <typename T> int64_t tail_lds_bytes(const LevelView* lv, int nl);
int tail_max_lds();        // dynamic LDS a workgroup may use (enables it for the tail kernels)
constexpr int TAIL_MAX_COARSE_NODES = 1024;  // nodes of every level below the first
// most padded nodes of a tail's first level (the kernel keeps its right-hand
// side in registers: 5 values a thread in complex128, 10 in complex64)
template <typename T> constexpr int tail_first_nodes_max() { return sizeof(T) == 8 ? 5 * 1024 : 10 * 1024; }

// Complex GEMM out[i, p] = sum_k M[i, k] in[k, p] (M^H with trans_conj),
// added to out when accumulate != 0, on FP64 matrix cores.  in/out rows may be padded planes: element p of row i
// sits at i * row + (p / nx) * pitch + p % nx + off.
struct RowLayout {
    int nx;        // nodes per grid row
    int pitch;     // elements per stored grid row
    int64_t row;   // elements per matrix row (one system / time slice)
    int64_t off;   // element offset of node 0
    // input rows only (the GEMM transforms): with sel set, row i sits alt
    // elements further on when (sel[i] * flips) is odd, and reads as zero
    // when sel[i] == 0 (a solve's iterates left in their two level-0
    // buffers, selected by each system's cycle count)
    const int* sel = nullptr;
    int64_t alt = 0;
    int flips = 0;
};
// With norm_partial set (and accumulate off), also sum |out|^2 per output
// row into norm_partial[row * tiles + t] and return the tile count; 0 when
// this product shape has no fused sums (nothing written there).
// The same products for the alpha-circulant eigenvector matrix V (time
// steps n a power of two, 2..256) as scaled DFTs: inverse = 0 applies V^{-1}
// (conj: V^H), inverse = 1 applies V (conj: V^{-H}).  norm_partial as above.
bool circulant_supported(int n);
int launch_circulant(int n, int64_t m, double alpha, int inverse, int conj, const double2* in, RowLayout li,
                     double2* out, RowLayout lo, hipStream_t st, int accumulate = 0, double* norm_partial = nullptr,
                     int max_tiles = 0);
// o32.p set (with norm_partial): the product rounded to complex64 is also
// written to o32.p in layout o32.l, where the fused sums are formed (n = 8,
// 16, 32, 64); a return of 0 means neither was written.
struct Out32 {
    float2* p = nullptr;
    RowLayout l{};
};
int launch_transform(int n, int64_t m, const double2* M, int trans_conj, const double2* in, RowLayout li,
                     double2* out, RowLayout lo, double2* mbuf, hipStream_t st, int accumulate = 0,
                     double* norm_partial = nullptr, int max_tiles = 0, Out32 o32 = Out32{});
// doubles of the scratch launch_transform expands M into (mbuf): 4 n^2, or
// more for n whose expanded form is padded to whole MFMA fragments (at most
// 4 n^2 for n a multiple of 8, and at most 4 * 256^2 for every n <= 256)
size_t transform_scratch_doubles(int n);

// Fused register-streaming level kernels (vmg_stream.hip), nu in {0, 1, 2},
// batched over segments like the launchers above:
//   down: nu sweeps, residual, full weighting -> xo (x_nu), c (coarse rhs)
//   up:   x + P c, nu sweeps -> xo; with `norm`, the partial sums of
//         |b - L xo|^2 go to a segment's partial buffer when that pointer is
//         not NULL (partial[sys * tiles + t], tiles = stream_tiles(...)).
//         `norm` selects the geometry with the extra halo lane the norm needs.
//         Finishing pass (segment's iters set, norm off): runs for every
//         system whatever its active flag, reads x or xalt by the parity of
//         iters[sys] (zero result for 0) and writes the dense rows of zd.
// The work of a level is split evenly over the device's resident waves, with
// at least rmin rows per wave.  c32 (T = double only): the coarse level (c,
// and cb of the edge kernel) holds complex64 values; the pointers in the
// segment are then float2 data, and the coarse views those of the complex64
// level.  paced (T = double, two Vanka sweeps): as for the cycle-edge
// kernel below, where a CU holds a block of 12 or 16 of the paced waves as
// it holds the plain ones (else the plain launch).
template <typename T>
void launch_down(SegTable<T> tab, const int* nsys, int nu, int rmin, hipStream_t st, bool c32 = false,
                 bool paced = false);
template <typename T>
void launch_up(SegTable<T> tab, const int* nsys, int nu, bool norm, int rmin, hipStream_t st, bool c32 = false,
               bool paced = false);
template <typename T> int stream_tiles(int nx, int ny, int nsys, int nu, int rmin);
int stream_tiles_max(int nx, int ny, int nu);  // over every rmin and kernel
// Cycle-edge kernel (FP64 finest level, nu1, nu2 in {1, 2}): correction +
// nu2 sweeps, norm partials of that iterate (edge_tiles per system), nu1
// sweeps -> xo, full weighting -> cb; reads x, b and the coarse correction c
// and leaves them untouched (the finishing pass of launch_up rebuilds the
// last cycle's iterate from them).  paced (T = double, Vanka): blocks of a
// CU's worth of waves on adjacent strips, held together by a barrier after
// every block of rows (the same run geometry and results).
// Ascent of a coarse level visited from zero (V-cycles): nu1 sweeps from
// zero rebuild the pre-smoothed iterate that the descent, given a null xo,
// did not store, then the correction from c and nu2 sweeps -> xo; reads b
// and c only.  Vanka, nu1 and nu2 in {1, 2} (edge_supported); the results
// equal those of launch_up after a storing launch_down (up to zeros' signs).
template <typename T>
void launch_recomp(SegTable<T> tab, const int* nsys, int nu1, int nu2, int rmin, hipStream_t st);
bool edge_supported(int nu1, int nu2);
template <typename T>
void launch_edge(SegTable<T> tab, const int* nsys, int nu1, int nu2, int rmin, hipStream_t st, bool c32 = false,
                 bool paced = false);
template <typename T> int edge_tiles(int nx, int ny, int nsys, int nu1, int nu2, int rmin);
// The boundary of two refinement steps on a streamed complex64 finest level,
// in one pass: the last inner cycle's correction and nu2 sweeps (complex64),
// x' = x + e and the FP64 residual of x' (its norm partials, ir_edge_tiles per
// system; stored rounded to complex64 as the next step's right-hand side), then
// the next step's first inner cycle from zero: nu1 sweeps, residual and full
// weighting.  nu1, nu2 in {1, 2}.
void launch_ir_edge(SegTable<float> tab, const int* nsys, int nu1, int nu2, int rmin, hipStream_t st,
                    bool paced = false);
int ir_edge_tiles(int nx, int ny, int nsys, int nu1, int nu2, int rmin);
void stream_prepare();  // device occupancy of the streaming kernels (call outside stream capture)
template <typename T> void launch_fill_zero(cplx<T>* x, LevelView lv, int nsys, hipStream_t st);

// Shift sensitivities out[s] = -sum_p conj(z[s*m + p]) g[s*m + p]; partial
// holds nsys * aux_tiles(m) double2.
int aux_tiles(int64_t m);
void launch_shift_gradient(const double2* z, const double2* g, int64_t m, int nsys, double2* partial,
                           double2* out, hipStream_t st);
// Backward-Euler all-at-once heat residual R = F - K U (n slices of nx x ny),
// or R = K U when F is NULL; partial holds n * aux_tiles(nx * ny) doubles;
// *out_norm2 (device) = ||R||^2.
void launch_heat_residual(const double2* U, const double2* F, double2* R, int n, int nx, int ny, double h,
                          double tau, int transpose, double* partial, double* out_norm2, hipStream_t st);

// Krylov vector operations over N complex entries (all on `st`):
//   zdot:  *out = sum conj(a) b (partial holds aux_tiles(N) entries)
//   zaxpy: y += sign * c * x, c = *coef (device) or the value a if coef is NULL
//   zscale: y *= 1/sqrt(nrm2->x) (device norm^2), or by s if nrm2 is NULL
void launch_zdot(const double2* a, const double2* b, int64_t N, double2* partial, double2* out, hipStream_t st);
void launch_zaxpy(double2* y, const double2* x, int64_t N, const double2* coef, double sign, double2 a,
                  hipStream_t st);
void launch_zscale(double2* y, int64_t N, const double2* nrm2, double s, hipStream_t st);

}  // namespace vmg
