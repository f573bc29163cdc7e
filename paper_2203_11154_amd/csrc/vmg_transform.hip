// Time transform of eq. (1): out = (M kron I_m) in, a complex (n x n) by
// (n x m) product, on the FP64 matrix cores of gfx950, and the ParaDIAG step
// that wraps the shifted solves between two such transforms.
//
// The complex product is run as one real GEMM of twice the size: with
// interleaved storage, the real row index 2i + c of `in` is component c of
// complex row i, and the expanded real matrix
//   Mx[2i][2k] = Re M_ik, Mx[2i][2k+1] = -Im M_ik,
//   Mx[2i+1][2k] = Im M_ik, Mx[2i+1][2k+1] = Re M_ik
// maps it to the same interleaved layout of `out` (8 n^2 m flops, no waste).
#include <hip/hip_runtime.h>

#include "vmg_internal.h"

#include <algorithm>

namespace vmg {

namespace {

typedef double dbl4 __attribute__((ext_vector_type(4)));

constexpr int TN = 512;        // threads per block, 8 waves
constexpr int ROWS = 256;      // real output rows per block (32 per wave)
constexpr int COLS = 64;       // grid nodes per block
constexpr int KC = 16;         // real K per chunk (8 complex time slices)

// Mx from M (or M^H when trans_conj), n2 = 2n.
__global__ void k_expand(const double2* __restrict__ M, int n, int trans_conj, double* __restrict__ Mx) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n * n) return;
    const int i = t / n, k = t - i * n;
    double2 v = trans_conj ? M[(int64_t)k * n + i] : M[(int64_t)i * n + k];
    if (trans_conj) v.y = -v.y;
    const int64_t n2 = 2 * (int64_t)n;
    Mx[(2 * i) * n2 + 2 * k] = v.x;
    Mx[(2 * i) * n2 + 2 * k + 1] = -v.y;
    Mx[(2 * i + 1) * n2 + 2 * k] = v.y;
    Mx[(2 * i + 1) * n2 + 2 * k + 1] = v.x;
}

__device__ __forceinline__ int tile_row_perm(int r) { return 2 * ((r & 3) + 4 * (r >> 3)) + ((r >> 2) & 1); }

// Mx in the order k_transform's waves consume it: for row block rb (32 real
// rows, one wave), K chunk c (KC real columns) and lane l, the eight values
//   Mx[32 rb + 16 a + perm(l % 16)][KC c + 4 s + l / 16],  a < 2, s < 4,
// at ((rb * nch + c) * 64 + l) * 8 + 4 a + s, zero outside the 2n x 2n matrix,
// so that a lane reads its chunk as 64 contiguous bytes.
__global__ void k_expand_frag(const double2* __restrict__ M, int n, int trans_conj, int nrb, int nch,
                              double* __restrict__ Mf) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)nrb * nch * 512) return;
    const int v = (int)(t & 7), l = (int)((t >> 3) & 63);
    const int64_t q = t >> 9;
    const int c = (int)(q % nch), rb = (int)(q / nch);
    const int r = 32 * rb + 16 * (v >> 2) + tile_row_perm(l & 15);
    const int k = KC * c + 4 * (v & 3) + (l >> 4);
    double x = 0.0;
    if (r < 2 * n && k < 2 * n) {
        const int i = r >> 1, kk = k >> 1;
        double2 e = trans_conj ? M[(int64_t)kk * n + i] : M[(int64_t)i * n + kk];
        if (trans_conj) e.y = -e.y;
        // [[Re, -Im], [Im, Re]] block of complex entry (i, kk)
        x = (r & 1) ? ((k & 1) ? e.x : e.y) : ((k & 1) ? -e.y : e.x);
    }
    Mf[t] = x;
}

// Element offset of grid node p (< 2^30) in a row layout.  The row index
// p / nx comes from a reciprocal computed once per thread: for p, nx < 2^30
// the rounded product is within one of the quotient, and one compare fixes it
// (a 64-bit integer division would cost tens of VALU instructions a node).
struct NodeMap {
    int nx, pitch;
    int64_t off;
    double inv;
    __device__ __forceinline__ explicit NodeMap(const RowLayout& L)
        : nx(L.nx), pitch(L.pitch), off(L.off), inv(1.0 / (double)L.nx) {}
    __device__ __forceinline__ int64_t operator()(int64_t p64) const {
        const int p = (int)p64;
        int r = (int)((double)p * inv);
        const int c = p - r * nx;
        r += (c >= nx ? 1 : 0) - (c < 0 ? 1 : 0);
        return off + (int64_t)r * pitch + (p - r * nx);
    }
};

// Start of input row k (and whether it holds data): see RowLayout::sel.
__device__ __forceinline__ bool in_row(const RowLayout& L, int k, int64_t& base) {
    base = (int64_t)k * L.row;
    if (!L.sel) return true;
    const int it = L.sel[k];
    if ((it * L.flips) & 1) base += L.alt;
    return it != 0;
}

// One block: real rows [rb*ROWS, +ROWS) x nodes [cb*COLS, +COLS).
// Wave w owns rows w*32..w*32+31 as 2 x 4 MFMA 16x16 tiles.
// v_mfma_f64_16x16x4_f64 lane layout (measured on gfx950): A[i][k] at lane
// i + 16k, B[k][j] at lane j + 16k, D[i][j] at lane j + 16(i%4), element
// i/4.  A lane therefore holds tile rows g, g+4, g+8, g+12 (g = lane/16).
// Feeding MFMA row r from real row perm(r) = 2((r%4) + 4(r/8)) + (r/4)%2
// makes those four values (re, im) of complex rows g and g+4 of the tile's
// eight complex rows, so each lane stores two whole double2 results.
// Each wave reads its own rows of Mx (fragment order, k_expand_frag) straight
// into registers, a chunk ahead; the input chunk all waves share goes
// through a double-buffered LDS tile (one barrier a chunk).  Two blocks a CU.
// Column blocks lie within grid rows of tx nodes, as in k_transform_reg.
__global__ __launch_bounds__(TN) __attribute__((amdgpu_waves_per_eu(4))) void k_transform(
    int n, int tx, const double* __restrict__ Mf, int nch, const double2* __restrict__ in, RowLayout li,
    double2* __restrict__ out, RowLayout lo, int accumulate) {
    __shared__ double sB[2][KC][COLS + 1];
    const int n2 = 2 * n;
    const NodeMap mi(li), mo(lo);
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const uint3 xb = xcd_block();
    const int row0 = xb.y * ROWS;
    const int tpr = (tx + COLS - 1) / COLS;
    const int grow = xb.x / tpr;
    const int gcol0 = (xb.x - grow * tpr) * COLS;  // first column of the block in its grid row
    const int64_t col0 = (int64_t)grow * tx + gcol0;     // its node
    const int wrow = row0 + wave * 32;
    const bool wave_active = wrow < n2;
    const double2* af = reinterpret_cast<const double2*>(Mf + ((int64_t)(wrow >> 5) * nch * 64 + lane) * 8);
    dbl4 acc[2][4];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = dbl4{0.0, 0.0, 0.0, 0.0};

    // input chunk: complex row kr = t / COLS of the chunk, node t % COLS
    const int kr = threadIdx.x / COLS, kcol = threadIdx.x % COLS;
    const bool pin = gcol0 + kcol < tx;
    const int64_t poff = pin ? mi(col0 + kcol) : 0;
    double2 rb;
    auto fetch_b = [&](int c) {
        const int gk = c * (KC / 2) + kr;
        int64_t base = 0;
        const bool live = gk < n && pin && in_row(li, gk, base);
        rb = live ? in[base + poff] : make_double2(0.0, 0.0);
    };
    auto stage = [&](int buf) {
        sB[buf][2 * kr][kcol] = rb.x;
        sB[buf][2 * kr + 1][kcol] = rb.y;
    };
    double2 ac[4], an[4];  // this chunk's and the next chunk's A fragments
    auto fetch_a = [&](int c, double2* dst) {
#pragma unroll
        for (int q = 0; q < 4; ++q) dst[q] = af[(int64_t)c * 256 + q];
    };
    if (wave_active) fetch_a(0, ac);
    fetch_b(0);
    stage(0);
    __syncthreads();
    int buf = 0;
    for (int c = 0; c < nch; ++c) {
        const bool more = c + 1 < nch;
        if (more) {
            fetch_b(c + 1);
            if (wave_active) fetch_a(c + 1, an);
        }
        if (wave_active) {
#pragma unroll
            for (int ks = 0; ks < 4; ++ks) {
                double bv[4];
#pragma unroll
                for (int b = 0; b < 4; ++b) bv[b] = sB[buf][4 * ks + (lane >> 4)][b * 16 + (lane & 15)];
#pragma unroll
                for (int a = 0; a < 2; ++a) {
                    // value 4a + ks of the lane's fragment
                    const double av = (ks & 1) ? ac[2 * a + (ks >> 1)].y : ac[2 * a + (ks >> 1)].x;
#pragma unroll
                    for (int b = 0; b < 4; ++b)
                        acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv[b], acc[a][b], 0, 0, 0);
                }
            }
        }
        if (more) {
            stage(buf ^ 1);
            __syncthreads();
            buf ^= 1;
#pragma unroll
            for (int q = 0; q < 4; ++q) ac[q] = an[q];
        }
    }
    if (!wave_active) return;
#pragma unroll
    for (int a = 0; a < 2; ++a) {
        // complex rows of this lane: cr and cr + 4 (elements 0,1 and 2,3)
        const int cr = (wrow + a * 16) / 2 + (lane >> 4);
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const int j = b * 16 + (lane & 15);
            if (gcol0 + j >= tx) continue;
            const int64_t o = mo(col0 + j);
            if (cr < n) {
                double2 v = make_double2(acc[a][b][0], acc[a][b][1]);
                double2* q = out + (int64_t)cr * lo.row + o;
                if (accumulate) { const double2 w = *q; v.x += w.x; v.y += w.y; }
                *q = v;
            }
            if (cr + 4 < n) {
                double2 v = make_double2(acc[a][b][2], acc[a][b][3]);
                double2* q = out + (int64_t)(cr + 4) * lo.row + o;
                if (accumulate) { const double2 w = *q; v.x += w.x; v.y += w.y; }
                *q = v;
            }
        }
    }
}

// Register-resident variant for 2n = 16 NW (n = 8, 16, 32, 64): a block of
// NW waves keeps the whole expanded matrix in registers (wave w holds real
// rows 16w..16w+15 for every K, KS = 2n/4 MFMA steps, n VGPRs a lane) and
// walks over tiles of CT*16 grid nodes, so Mx is read once per block and the
// input is streamed through a double-buffered LDS tile.  Same lane layout and
// row permutation as k_transform.  Tiles never cross a grid row of tx nodes
// (the shorter row of the two layouts): in a padded plane, whose interior
// rows start on 128-byte boundaries, a tile then reads or writes whole
// cache lines only (the last tile of a row is partly empty).
constexpr int RT_CT = 2;               // 16-node column sub-tiles per tile
constexpr int RT_NODES = 16 * RT_CT;   // nodes per tile

// (two blocks a CU: 4 waves a SIMD for NW = 8)
// NORM: also the sums of |out|^2 per output row (see launch_transform), kept
// per lane in LDS across tiles so that the MFMA loop's registers are untouched;
// C32 (with NORM): also out rounded to complex64 into o32.p, layout o32.l.
template <int NW, bool NORM, bool C32 = false>
__global__ __launch_bounds__(64 * NW) __attribute__((amdgpu_waves_per_eu(4))) void k_transform_reg(int64_t m, const double* __restrict__ Mx,
                                                            const double2* __restrict__ in, RowLayout li,
                                                            double2* __restrict__ out, RowLayout lo, int accumulate,
                                                            int tx, int64_t ntiles, double* __restrict__ partial,
                                                            Out32 o32) {
    __shared__ double sN[NORM ? 2 * 64 * NW : 1];
    constexpr int n = 8 * NW, n2 = 2 * n, KS = n2 / 4, TT = 64 * NW;
    // per thread of the tile load: complex rows x nodes = n x RT_NODES values
    constexpr int LD = n * RT_NODES / TT;  // = 4
    static_assert(LD * TT == n * RT_NODES, "tile load split");
    __shared__ double sB[2][n2][RT_NODES + 1];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int arow = 16 * wave + tile_row_perm(lane & 15);
    double av[KS];
#pragma unroll
    for (int s = 0; s < KS; ++s) av[s] = Mx[(int64_t)arow * n2 + 4 * s + (lane >> 4)];

    // thread t loads complex row t / (RT_NODES / LD), nodes lcol + q LS (q < LD):
    // for n = 64 consecutive threads read consecutive nodes of a row (LS =
    // RT_NODES / LD), for smaller n each thread reads LD consecutive nodes
    // (LS = 1); each measured the faster for its n
    constexpr bool SPREAD = NW >= 8;
    constexpr int LS = SPREAD ? RT_NODES / LD : 1;
    const int lrow = threadIdx.x / (RT_NODES / LD);
    const int lcol = SPREAD ? threadIdx.x % (RT_NODES / LD) : (threadIdx.x % (RT_NODES / LD)) * LD;
    const NodeMap mi(li), mo(lo);
    double2 rb[LD];
    // tile -> node of its first column, and that column within the grid row
    const int tpr = (tx + RT_NODES - 1) / RT_NODES;
    auto tile_at = [&](int64_t tile, int64_t& p0, int& col0) {
        const int64_t r = tile / tpr;
        col0 = (int)(tile - r * tpr) * RT_NODES;
        p0 = r * tx + col0;
    };
    int64_t rbase;
    const bool rlive = in_row(li, lrow, rbase);
    auto fetch = [&](int64_t tile) {
        int64_t p0;
        int col0;
        tile_at(tile, p0, col0);
#pragma unroll
        for (int q = 0; q < LD; ++q) {
            const int c = lcol + q * LS;
            rb[q] = (rlive && col0 + c < tx) ? in[rbase + mi(p0 + c)] : make_double2(0.0, 0.0);
        }
    };
    auto stage = [&](int buf) {
#pragma unroll
        for (int q = 0; q < LD; ++q) {
            sB[buf][2 * lrow][lcol + q * LS] = rb[q].x;
            sB[buf][2 * lrow + 1][lcol + q * LS] = rb[q].y;
        }
    };
    // Tile order: for n <= 32 block b walks the contiguous run [b T / G,
    // (b + 1) T / G) of the T tiles (at least one, as G <= T), for n = 64 the
    // tiles b, b + G, ...; each measured the faster for its n.  Neighbouring
    // tiles, which share the cache lines at their ends in planes that do not
    // start on a line, run in one block or on one XCD.
    constexpr bool RUN = NW < 8;
    const int64_t xb = xcd_block().x;
    int64_t tile = RUN ? xb * ntiles / gridDim.x : xb;
    const int64_t tend = RUN ? (xb + 1) * ntiles / gridDim.x : ntiles;
    const int64_t tstep = RUN ? 1 : gridDim.x;
    if (tile >= tend) return;  // uniform over the block (never with NORM: one tile a block at least)
    if constexpr (NORM) {
        sN[2 * threadIdx.x] = 0.0;  // |out|^2 of the lane's two complex rows
        sN[2 * threadIdx.x + 1] = 0.0;
    }
    fetch(tile);
    stage(0);
    __syncthreads();
    int buf = 0;
    // (contiguous runs) a store into the cache line that the run's next tile
    // completes waits for that tile's stores, so that both parts of the line
    // reach L2 together rather than one part being written back alone
    double2* dq0 = nullptr;
    double2* dq1 = nullptr;
    double2 dv0 = make_double2(0.0, 0.0), dv1 = make_double2(0.0, 0.0);
    for (; tile < tend; tile += tstep) {
        const int64_t next = tile + tstep;
        if (next < tend) fetch(next);
        dbl4 acc[RT_CT];
#pragma unroll
        for (int c = 0; c < RT_CT; ++c) acc[c] = dbl4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int s = 0; s < KS; ++s)
#pragma unroll
            for (int c = 0; c < RT_CT; ++c)
                acc[c] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[s], sB[buf][4 * s + (lane >> 4)][16 * c + (lane & 15)],
                                                              acc[c], 0, 0, 0);
        // complex rows of this lane: cr and cr + 4
        const int cr = 8 * wave + (lane >> 4);
        int64_t p0;
        int col0;
        tile_at(tile, p0, col0);
        // lines of the next tile's first node in this lane's two rows (only
        // the last 16 nodes of a tile can share one: a line holds 8 nodes)
        bool has_next = false;
        uintptr_t ln0 = 0, ln1 = 0;
        if constexpr (RUN) {
            if (dq0) *dq0 = dv0;
            if (dq1) *dq1 = dv1;
            dq0 = dq1 = nullptr;
            if (next < tend) {
                int64_t pn;
                int cn;
                tile_at(next, pn, cn);
                const int64_t on = mo(pn);
                has_next = true;
                ln0 = (uintptr_t)(out + (int64_t)cr * lo.row + on) >> 7;
                ln1 = (uintptr_t)(out + (int64_t)(cr + 4) * lo.row + on) >> 7;
            }
        }
#pragma unroll
        for (int c = 0; c < RT_CT; ++c) {
            const int j = 16 * c + (lane & 15);
            if (col0 + j < tx) {
                const int64_t o = mo(p0 + j);
                double2 v0 = make_double2(acc[c][0], acc[c][1]);
                double2 v1 = make_double2(acc[c][2], acc[c][3]);
                double2* q0 = out + (int64_t)cr * lo.row + o;
                double2* q1 = out + (int64_t)(cr + 4) * lo.row + o;
                if (accumulate) {
                    const double2 w0 = *q0, w1 = *q1;
                    v0.x += w0.x; v0.y += w0.y;
                    v1.x += w1.x; v1.y += w1.y;
                }
                const bool d0 = RUN && c == RT_CT - 1 && has_next && ((uintptr_t)q0 >> 7) == ln0;
                const bool d1 = RUN && c == RT_CT - 1 && has_next && ((uintptr_t)q1 >> 7) == ln1;
                if (d0) {
                    dq0 = q0;
                    dv0 = v0;
                } else {
                    *q0 = v0;
                }
                if (d1) {
                    dq1 = q1;
                    dv1 = v1;
                } else {
                    *q1 = v1;
                }
                if constexpr (NORM) {
                    sN[2 * threadIdx.x] += v0.x * v0.x + v0.y * v0.y;
                    sN[2 * threadIdx.x + 1] += v1.x * v1.x + v1.y * v1.y;
                    if constexpr (C32) {
                        const int64_t o2 = NodeMap(o32.l)(p0 + j);
                        o32.p[(int64_t)cr * o32.l.row + o2] = make_float2((float)v0.x, (float)v0.y);
                        o32.p[(int64_t)(cr + 4) * o32.l.row + o2] = make_float2((float)v1.x, (float)v1.y);
                    }
                }
            }
        }
        if (next < tend) {
            stage(buf ^ 1);
            __syncthreads();
            buf ^= 1;
        }
    }
    if (dq0) *dq0 = dv0;  // (never taken: a store waits only for a next tile)
    if (dq1) *dq1 = dv1;
    if constexpr (NORM) {
        // the 16 lanes of a lane group hold the same two rows
        double s0 = sN[2 * threadIdx.x], s1 = sN[2 * threadIdx.x + 1];
        for (int off = 8; off > 0; off >>= 1) {
            s0 += __shfl_xor(s0, off, 64);
            s1 += __shfl_xor(s1, off, 64);
        }
        if ((lane & 15) == 0) {
            const int cr = 8 * wave + (lane >> 4);
            partial[(int64_t)cr * gridDim.x + blockIdx.x] = s0;
            partial[(int64_t)(cr + 4) * gridDim.x + blockIdx.x] = s1;
        }
    }
}

template <int NW, bool NORM> int reg_blocks() {
    static int blocks = 0;
    if (!blocks) {
        int per_cu = 0, cus = 0, dev = 0;
        if (hipGetDevice(&dev) != hipSuccess) dev = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void*)&k_transform_reg<NW, NORM>, 64 * NW, 0) !=
                hipSuccess || per_cu < 1)
            per_cu = 1;
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1) cus = 1;
        blocks = per_cu * cus;
    }
    return blocks;
}

template <int NW>
int go_reg(int64_t m, const double* Mx, const double2* in, RowLayout li, double2* out, RowLayout lo, int accumulate,
           hipStream_t st, double* partial, int max_tiles, Out32 o32) {
    // tiles within grid rows of the shorter layout row (m is a multiple of it)
    const int tx = std::min(li.nx, lo.nx);
    const int64_t ntiles = (m / tx) * ((tx + RT_NODES - 1) / RT_NODES);
    if (partial && !accumulate) {
        const int64_t blocks = std::min<int64_t>(ntiles, reg_blocks<NW, true>());
        if (blocks >= 1 && blocks <= max_tiles) {
            if (o32.p)
                hipLaunchKernelGGL((k_transform_reg<NW, true, true>), dim3((unsigned)blocks), dim3(64 * NW), 0, st, m, Mx,
                                   in, li, out, lo, 0, tx, ntiles, partial, o32);
            else
                hipLaunchKernelGGL((k_transform_reg<NW, true>), dim3((unsigned)blocks), dim3(64 * NW), 0, st, m, Mx, in,
                                   li, out, lo, 0, tx, ntiles, partial, o32);
            return (int)blocks;
        }
    }
    const int64_t blocks = std::min<int64_t>(ntiles, reg_blocks<NW, false>());
    if (blocks < 1) return 0;
    hipLaunchKernelGGL((k_transform_reg<NW, false>), dim3((unsigned)blocks), dim3(64 * NW), 0, st, m, Mx, in, li, out,
                       lo, accumulate, tx, ntiles, nullptr, Out32{});
    return 0;
}

// ---------------------------------------------------------------------------
// The same products for the alpha-circulant eigenvector matrix of the
// backward-Euler time-stepping matrix, V = diag(alpha^{-i/n}) W with
// W_ik = exp(-2 pi i ik/n) and V^{-1} = W^H diag(alpha^{i/n}) / n (indices
// from 0): each is a length-n DFT along the time index of every node between
// two diagonal scalings,
//   out_k = post_k sum_i exp(sigma 2 pi i ik/n) pre_i in_i.
// A block walks over tiles of FT_TILE / n nodes x n slices held in LDS (rows
// stored in bit-reversed order, so the radix-2 decimation-in-time stages run
// in place and end in natural order); twiddles and scalings are computed once
// per block.  Memory bound: one read and one write of every value.
constexpr int FT = 256;          // threads per block
constexpr int FT_TILE = 2048;    // complex values per tile
constexpr int FT_MAXN = 256;

__device__ __forceinline__ int bit_reverse(int i, int logn) { return (int)(__brev((unsigned)i) >> (32 - logn)); }

template <bool NORM>
__global__ __launch_bounds__(FT) void k_circ_dft(int logn, int64_t m, int sign, double alpha, int variant,
                                                 const double2* __restrict__ in, RowLayout li,
                                                 double2* __restrict__ out, RowLayout lo, int accumulate,
                                                 int64_t ntiles, double* __restrict__ partial) {
    __shared__ double2 s[FT_TILE];
    __shared__ double2 tw[FT_MAXN / 2];
    __shared__ double pre[FT_MAXN], post[FT_MAXN];
    const int n = 1 << logn;
    const int logtn = 11 - logn;  // log2(FT_TILE / n)
    const int tn = 1 << logtn;
    const NodeMap mi(li), mo(lo);
    for (int j = threadIdx.x; j < n / 2; j += FT) {
        double sv, cv;
        sincospi(2.0 * j / n, &sv, &cv);
        tw[j] = make_double2(cv, sign * sv);
    }
    for (int i = threadIdx.x; i < n; i += FT) {
        const double a = pow(alpha, (double)i / n);  // alpha^{i/n}
        // 0: V^{-1} (pre alpha^{i/n}, post 1/n); 1: V (post alpha^{-k/n});
        // 2: V^H (pre alpha^{-i/n}); 3: V^{-H} (post alpha^{k/n} / n)
        pre[i] = variant == 0 ? a : (variant == 2 ? 1.0 / a : 1.0);
        post[i] = variant == 0 ? 1.0 / n : (variant == 1 ? 1.0 / a : (variant == 3 ? a / n : 1.0));
    }
    double acc = 0.0;  // NORM: sum of |out|^2 of row threadIdx.x (< n)
    // the next tile is loaded into registers while the current one is
    // transformed in LDS
    constexpr int LD = FT_TILE / FT;
    double2 rb[LD];
    auto fetch = [&](int64_t t) {
#pragma unroll
        for (int q = 0; q < LD; ++q) {
            const int e = threadIdx.x + q * FT;
            const int i = e >> logtn, c = e & (tn - 1);
            const int64_t p = t * tn + c;
            int64_t base;
            const bool live = in_row(li, i, base);
            rb[q] = (live && p < m) ? in[base + mi(p)] : make_double2(0.0, 0.0);
        }
    };
    const int64_t t0 = xcd_block().x;  // (as in k_transform_reg)
    if (t0 < ntiles) fetch(t0);
    __syncthreads();
    for (int64_t tile = t0; tile < ntiles; tile += gridDim.x) {
        const int64_t p0 = tile * tn;
#pragma unroll
        for (int q = 0; q < LD; ++q) {
            const int e = threadIdx.x + q * FT;
            const int i = e >> logtn, c = e & (tn - 1);
            s[(bit_reverse(i, logn) << logtn) + c] = make_double2(rb[q].x * pre[i], rb[q].y * pre[i]);
        }
        __syncthreads();
        if (tile + gridDim.x < ntiles) fetch(tile + gridDim.x);
        for (int lh = 0; lh < logn; ++lh) {
            const int half = 1 << lh;
            for (int e = threadIdx.x; e < FT_TILE / 2; e += FT) {
                const int c = e & (tn - 1);
                const int b = e >> logtn;  // butterfly of the column
                const int j = b & (half - 1);
                const int k0 = ((b >> lh) << (lh + 1)) + j;
                const double2 w = tw[j << (logn - 1 - lh)];
                const double2 x0 = s[(k0 << logtn) + c];
                const double2 x1 = s[((k0 + half) << logtn) + c];
                const double2 t = make_double2(w.x * x1.x - w.y * x1.y, w.x * x1.y + w.y * x1.x);
                s[(k0 << logtn) + c] = make_double2(x0.x + t.x, x0.y + t.y);
                s[((k0 + half) << logtn) + c] = make_double2(x0.x - t.x, x0.y - t.y);
            }
            __syncthreads();
        }
        for (int e = threadIdx.x; e < FT_TILE; e += FT) {
            const int k = e >> logtn, c = e & (tn - 1);
            const int64_t p = p0 + c;
            if (p < m) {
                double2 v = s[e];
                v.x *= post[k];
                v.y *= post[k];
                double2* q = out + (int64_t)k * lo.row + mo(p);
                if (accumulate) {
                    const double2 w = *q;
                    v.x += w.x;
                    v.y += w.y;
                }
                *q = v;
                if (NORM) s[e] = v;
            }
        }
        if constexpr (NORM) {
            __syncthreads();
            if (threadIdx.x < n) {
                const int k = threadIdx.x;
                for (int c = 0; c < tn && p0 + c < m; ++c) {
                    const double2 v = s[(k << logtn) + c];
                    acc += v.x * v.x + v.y * v.y;
                }
            }
        }
        __syncthreads();  // the tile is read completely before the next one is stored
    }
    if (NORM && threadIdx.x < n) partial[(int64_t)threadIdx.x * gridDim.x + blockIdx.x] = acc;
}

template <bool NORM> int circ_blocks() {
    static int blocks = 0;
    if (!blocks) {
        int per_cu = 0, cus = 0, dev = 0;
        if (hipGetDevice(&dev) != hipSuccess) dev = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void*)&k_circ_dft<NORM>, FT, 0) !=
                hipSuccess || per_cu < 1)
            per_cu = 1;
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1) cus = 1;
        blocks = per_cu * cus;
    }
    return blocks;
}

}  // namespace

bool circulant_supported(int n) { return n >= 2 && n <= FT_MAXN && (n & (n - 1)) == 0; }

int launch_circulant(int n, int64_t m, double alpha, int inverse, int conj, const double2* in, RowLayout li,
                     double2* out, RowLayout lo, hipStream_t st, int accumulate, double* norm_partial, int max_tiles) {
    int logn = 0;
    while ((1 << logn) < n) ++logn;
    const int64_t tn = FT_TILE / n;
    const int64_t ntiles = (m + tn - 1) / tn;
    const int variant = conj ? (inverse ? 3 : 2) : (inverse ? 1 : 0);
    const int sign = inverse ? -1 : 1;
    if (norm_partial && !accumulate) {
        const int64_t blocks = std::min<int64_t>(ntiles, circ_blocks<true>());
        if (blocks >= 1 && blocks <= max_tiles) {
            hipLaunchKernelGGL(k_circ_dft<true>, dim3((unsigned)blocks), dim3(FT), 0, st, logn, m, sign, alpha, variant,
                               in, li, out, lo, 0, ntiles, norm_partial);
            return (int)blocks;
        }
    }
    const int64_t blocks = std::min<int64_t>(ntiles, circ_blocks<false>());
    if (blocks >= 1)
        hipLaunchKernelGGL(k_circ_dft<false>, dim3((unsigned)blocks), dim3(FT), 0, st, logn, m, sign, alpha, variant,
                           in, li, out, lo, accumulate, ntiles, nullptr);
    return 0;
}

bool transform_reg(int n) { return n == 8 || n == 16 || n == 32 || n == 64; }

size_t transform_scratch_doubles(int n) {
    if (transform_reg(n)) return 4 * (size_t)n * n;
    const size_t nrb = (2 * (size_t)n + 31) / 32, nch = (2 * (size_t)n + KC - 1) / KC;
    return std::max(4 * (size_t)n * n, nrb * nch * 512);
}

int launch_transform(int n, int64_t m, const double2* M, int trans_conj, const double2* in, RowLayout li,
                     double2* out, RowLayout lo, double2* mbuf, hipStream_t st, int accumulate, double* norm_partial,
                     int max_tiles, Out32 o32) {
    double* Mx = reinterpret_cast<double*>(mbuf);
    if (transform_reg(n)) {
        hipLaunchKernelGGL(k_expand, dim3((n * n + 255) / 256), dim3(256), 0, st, M, n, trans_conj, Mx);
        switch (n) {
            case 8: return go_reg<1>(m, Mx, in, li, out, lo, accumulate, st, norm_partial, max_tiles, o32);
            case 16: return go_reg<2>(m, Mx, in, li, out, lo, accumulate, st, norm_partial, max_tiles, o32);
            case 32: return go_reg<4>(m, Mx, in, li, out, lo, accumulate, st, norm_partial, max_tiles, o32);
            default: return go_reg<8>(m, Mx, in, li, out, lo, accumulate, st, norm_partial, max_tiles, o32);
        }
    }
    const int nrb = (2 * n + 31) / 32, nch = (2 * n + KC - 1) / KC;
    const int64_t frag = (int64_t)nrb * nch * 512;
    hipLaunchKernelGGL(k_expand_frag, dim3((unsigned)((frag + 255) / 256)), dim3(256), 0, st, M, n, trans_conj, nrb,
                       nch, Mx);
    const int tx = std::min(li.nx, lo.nx);  // m is a multiple of it
    const dim3 grid((unsigned)((m / tx) * ((tx + COLS - 1) / COLS)), (unsigned)((2 * n + ROWS - 1) / ROWS));
    hipLaunchKernelGGL(k_transform, grid, dim3(TN), 0, st, n, tx, Mx, nch, in, li, out, lo, accumulate);
    return 0;
}

}  // namespace vmg
