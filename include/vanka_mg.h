/*
 * vanka_mg.h - C ABI of the MI355X (gfx950) Vanka-multigrid library for the
 * complex-shifted Laplacian systems of diagonalisation-based parallel-in-time
 * (ParaDIAG) methods.
 *
 * Method: He & Liu, "A Vanka-type multigrid solver for complex-shifted
 * Laplacian systems from diagonalization-based parallel-in-time algorithms"
 * (arXiv 2203.11154).
 *   - eq. (1): (B kron I_h + I_t kron A) u = f with B = V D V^{-1} splits into
 *     G = (V^{-1} kron I_h) F, n independent shifted solves, U = (V kron I_h) Z.
 *   - eq. (2): the shifted systems L_j z = (A + lambda_j I) z = b_j, A the
 *     5-point Laplacian (1/h^2)[., -1, .; -1, 4, -1; ., -1, .] on a rectangle
 *     with homogeneous Dirichlet boundary (Sec. 1).
 *   - eqs. (3) and (6): the additive element-wise Vanka smoother, applied as the
 *     explicit stencil M_{e,j} = (h^2/4)[c 2b c; 2b 4a 2b; c 2b c] with one
 *     precomputed patch inverse (a, b, c) per shift and level, relaxation
 *     weight omega = 24/25 (Sec. 2.1, after Theorem 2.1).
 *   - Sec. 3: re-discretised coarse operators (2h), full-weighting
 *     restriction, linear interpolation, a direct solve on the coarsest grid,
 *     and a stop on the reduction of the relative residual norm.
 *
 * Data conventions (all entry points)
 *   - Complex numbers are interleaved (re, im) doubles (C99 double _Complex /
 *     numpy complex128 / torch.complex128 layout).
 *   - A grid has nx x ny interior nodes, x fastest.  A vector of one system is
 *     ny*nx complex values, row-major; the systems of all grids are
 *     concatenated in the order the grids were given to vanka_mg_setup, and
 *     within a grid in system order.
 *   - "device" pointers are HIP device memory of the GPU that was current at
 *     setup; "host" pointers are ordinary host memory.
 *   - hip_stream is a hipStream_t (NULL = the default stream).  Work is
 *     enqueued on that stream; a call returns once its work is enqueued unless
 *     it has host outputs, which imply a synchronisation of that stream.
 *     Solves that stop at a tolerance also read the per-system state between
 *     batches of cycles (stream synchronisations), so that no cycle is
 *     launched after every system has stopped.
 *   - The caller owns every buffer it passes in; the library owns everything
 *     inside a handle.  A handle is used from one host thread and one stream at
 *     a time.
 *
 * Errors: every int-returning call returns one of the VMG_* codes below and
 * never throws or aborts.  On an error no output is valid unless stated.
 */
#ifndef VANKA_MG_H
#define VANKA_MG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    VMG_OK = 0,
    VMG_NOT_CONVERGED = 1,   /* outputs valid; some system hit max_iter      */
    VMG_INVALID_ARG = -1,    /* null pointer, bad size, bad option            */
    VMG_HIP_ERROR = -2,      /* a HIP runtime call failed                     */
    VMG_OOM = -3,            /* device or host allocation failed              */
    VMG_SINGULAR = -4,       /* a shifted coarsest-grid matrix is singular    */
    VMG_NAN_DETECTED = -5    /* a residual norm became NaN or Inf             */
};

/* Operation codes of vanka_mg_apply_op (single kernels, for tests/tuning). */
enum {
    VMG_OP_SWEEP = 0,            /* out = x + omega M_{e,j}(b - L_j x)          */
    VMG_OP_RESIDUAL = 1,         /* out = b - L_j x                              */
    VMG_OP_RESTRICT_RESIDUAL = 2,/* out (coarse) = FW(b - L_j x)                 */
    VMG_OP_PROLONG_CORRECT = 3,  /* out = x + P e, e = b argument on the coarse grid */
    VMG_OP_COARSE_SOLVE = 4,     /* out = (A_c + lambda_j I)^{-1} b, coarsest    */
    VMG_OP_CYCLE = 5             /* out = one multigrid cycle from x with rhs b  */
};

typedef struct vmg_handle vmg_handle;

/* One grid and the systems solved on it. */
typedef struct {
    int32_t nx, ny;       /* interior nodes; each level above the coarsest
                             must have odd nx, ny >= 3 (coarse = (n-1)/2)      */
    double h;             /* mesh width (unit square: 1/(nx+1))                */
    int32_t levels;       /* number of levels; 0 = coarsen until the smaller
                             side has at most 7 nodes (h0 = 1/8, Sec. 3)      */
    int32_t num_systems;  /* shifts solved on this grid                        */
} vmg_grid;

typedef struct {
    double omega;         /* relaxation weight; default 24/25 (Sec. 2.1)      */
    int32_t nu1, nu2;     /* pre-/post-smoothing steps; default 2, 2          */
    int32_t gamma;        /* 1 = V-cycle (default), 2 = W-cycle (Sec. 3)     */
    int32_t max_iter;     /* cycle (or refinement step) limit; default 100    */
    int32_t precision;    /* 0 = complex128 cycles (default);
                             1 = complex64 cycles inside FP64 iterative
                                 refinement (residual and update in FP64);
                             2 = FP64 V-cycles whose coarse-grid correction
                                 runs in complex64 (finest level, stopping
                                 test and result in FP64; gamma must be 1 and
                                 every grid's finest level large enough for
                                 the streaming kernels, else setup returns
                                 VMG_INVALID_ARG)                            */
    int32_t smoother;     /* 0 = additive Vanka (default); 1 = damped Jacobi,
                             the comparison smoother of Sec. 3 (omega 4/5)   */
    int32_t ir_inner;     /* complex64 cycles per refinement step; default 3 */
    int32_t check_every;  /* most cycles enqueued between two host checks of
                             the stop flags; default 64 (the stop itself is
                             exact per system: it is decided on the device
                             after every cycle, and the host sizes batches
                             from the observed convergence rates)            */
    int32_t graphs;       /* 1 (default): replay each cycle as a captured
                             hipGraph (eager launches while kernel timing is
                             on); 0: always launch eagerly                   */
} vmg_opts;

/* Fill *opts with the defaults listed above.  Returns VMG_OK or
 * VMG_INVALID_ARG (opts NULL). */
int vanka_mg_default_opts(vmg_opts* opts);

/*
 * Build the level hierarchy, the per-(shift, level) Vanka coefficients
 * (eq. (6), eta = lambda_j h_l^2, evaluated in FP64 over one common
 * denominator) and the inverse of every shifted coarsest-grid matrix, and
 * allocate all device buffers.
 *   grids    host, n_grids entries (n_grids >= 1).
 *   shifts   host, sum(num_systems) complex lambda_j (interleaved doubles),
 *            copied.
 *   opts     host, NULL = defaults.
 *   out      receives the new handle (NULL on failure).
 * Errors: VMG_INVALID_ARG (sizes, levels that cannot coarsen, a coarsest grid
 * with more than 256 nodes, bad options), VMG_OOM, VMG_SINGULAR, VMG_HIP_ERROR.
 */
int vanka_mg_setup(const vmg_grid* grids, int32_t n_grids, const double* shifts,
                   const vmg_opts* opts, void* hip_stream, vmg_handle** out);

/*
 * Per-system complex relaxation weights omega_j for the smoother (the
 * complex relaxation parameter the paper leaves as future work after
 * Example 3; S_j = I - omega_j M_{e,j} L_j).  omega: host, one complex value
 * per system (interleaved doubles), or NULL to return to opts->omega.  The
 * adjoint systems use conj(omega_j).  Synchronises the device.
 * Returns VMG_OK, VMG_INVALID_ARG, VMG_HIP_ERROR.
 */
int vanka_mg_set_omega(vmg_handle* h, const double* omega);

/*
 * New shifts lambda_j for the handle's systems (eq. (2)), in place: the
 * Vanka coefficients of eq. (6) of every (system, level) and the inverses of
 * the shifted coarsest matrices are recomputed and copied into the buffers
 * the handle already holds, so nothing is allocated and the captured cycle
 * graphs stay valid.  Relaxation weights return to opts->omega (call
 * vanka_mg_set_omega or vanka_mg_optimize_omega again for others).
 * Synchronises the device first (work already enqueued uses the old shifts).
 *   shifts  host, one complex value per system (interleaved doubles), in the
 *           order of vanka_mg_setup.
 * Returns VMG_OK, VMG_INVALID_ARG (NULL, non-finite value), VMG_SINGULAR (a
 * shifted coarsest matrix is singular; the previous shifts are kept),
 * VMG_HIP_ERROR.
 */
int vanka_mg_set_shifts(vmg_handle* h, const double* shifts);

/*
 * Local Fourier analysis (Sec. 2.1): for each eta = lambda h^2 the complex
 * relaxation weight omega minimising the smoothing factor of eq. (4),
 * mu = max over the high frequencies of |1 - omega M(theta) L(theta)| (the
 * symbols of L_j and of the smoother, scaled by h^2), and that minimum.
 * Host computation only (needs no device).
 *   eta       host, count complex values (interleaved doubles).
 *   smoother  0 = additive Vanka (eq. (6)), 1 = point Jacobi.
 *   omega     host output, count complex values (interleaved doubles).
 *   mu        host output, count doubles, or NULL.
 * The high frequencies are sampled on a uniform grid of (cos t1, cos t2)
 * with spacing 1/192; the minimum is exact for the samples up to about 1e-9.
 * Returns VMG_OK or VMG_INVALID_ARG (NULL eta or omega, count < 0, bad
 * smoother).
 */
int vanka_mg_lfa_omega(const double* eta, int32_t count, int32_t smoother, double* omega, double* mu);

/*
 * The complex relaxation parameter per shift (and level): sets, for every
 * system j and level l, the omega vanka_mg_lfa_omega gives for
 * eta = lambda_j h^2 with h the finest mesh width (per_level = 0: one weight
 * per shift on every level) or the level's own h_l (per_level = 1), for the
 * handle's smoother, and uploads the coefficients (the adjoint systems use
 * the conjugates).  Replaces weights set by vanka_mg_set_omega;
 * vanka_mg_set_omega(h, NULL) returns to opts->omega.  Synchronises the
 * device.
 * Returns VMG_OK, VMG_INVALID_ARG (per_level not 0 or 1), VMG_HIP_ERROR.
 */
int vanka_mg_optimize_omega(vmg_handle* h, int32_t per_level);

/*
 * Solve (A + lambda_j I) z_j = b_j for every system (eq. (2)), or with
 * conj != 0 the adjoint systems (A + conj(lambda_j) I) z_j = b_j.
 *   B, Z        device, complex128, all systems concatenated (see above).
 *               Z may not alias B.  The iteration starts from z = 0.
 *   tol         relative residual target ||b_j - L_j z_j||_2 / ||b_j||_2 > 0.
 *   fixed_iters host, NULL or one count per system: run exactly that many
 *               cycles (refinement steps) for system j and ignore tol.
 *   iters       host, NULL or one int per system: cycles (refinement steps)
 *               run.  relres: host, NULL or one double per system: final
 *               relative residual.  If both are NULL and every system has a
 *               fixed count, the call is fully asynchronous (it then returns
 *               VMG_OK without looking at the results: vanka_mg_last_stats
 *               gives the counts and residuals afterwards).
 * A system with b_j = 0 returns z_j = 0 after zero cycles.
 * Returns VMG_OK, VMG_NOT_CONVERGED (some system reached max_iter above tol;
 * outputs valid), VMG_NAN_DETECTED, VMG_INVALID_ARG, VMG_HIP_ERROR.
 */
int vanka_mg_solve(vmg_handle* h, const double* B, double* Z, double tol, int32_t conj,
                   const int32_t* fixed_iters, int32_t* iters, double* relres, void* hip_stream);

/*
 * ParaDIAG step of eq. (1) for a handle whose systems are the n time modes
 * (n = total number of systems, all on one grid with m = nx*ny nodes):
 *   G = (Vinv kron I) F;  Z_j = L_j^{-1} G_j;  U = (V kron I) Z.
 *   V, Vinv  device, complex128 n x n row-major, V Vinv = I expected.
 *   F, U     device, complex128 n x m row-major (row = time slice).  U may
 *            alias F.
 *   conj     apply the adjoint instead,
 *            U = (V^{-H} kron I) blockdiag((A + conj(lambda_j) I)^{-1}) (V^H kron I) F.
 *   fixed_iters  host, NULL or one cycle count per system (as in
 *            vanka_mg_solve; freezes the solve into a fixed linear map).
 * The shifts given at setup must be the eigenvalues D of B = V D V^{-1}.
 * Per-system counts and residuals: vanka_mg_last_stats.
 * Returns as vanka_mg_solve.
 */
int paradiag_apply(vmg_handle* h, const double* V, const double* Vinv, const double* F,
                   double* U, double tol, int32_t conj, const int32_t* fixed_iters, void* hip_stream);

/*
 * Sensitivity of the shifted solves to their shifts (eq. (2)): with
 * z_j = L_j^{-1} b_j, dz_j/dlambda_j = -L_j^{-1} z_j, so for an adjoint
 * solution g_j = L_j^{-H} w_j the vector-Jacobian product is
 *   grad_lambda[j] = -sum_p conj(z_j[p]) g_j[p].
 *   Z, G         device, complex128, the handle's concatenated layout.
 *   grad_lambda  device, complex128, one value per system.
 * Fixed-order reduction (bitwise repeatable).  Returns VMG_OK,
 * VMG_INVALID_ARG, VMG_HIP_ERROR.
 */
int vanka_mg_shift_gradient(vmg_handle* h, const double* Z, const double* G, double* grad_lambda,
                            void* hip_stream);

/*
 * Residual of the backward-Euler all-at-once heat system that the alpha-
 * circulant ParaDIAG preconditioner is iterated on (eq. (1) with
 * B = (1/tau)(I - Z), Z the down-shift, zero initial value):
 *   transpose = 0:  R^m = F^m - ((U^m - U^{m-1})/tau + A U^m),  U^{-1} = 0
 *   transpose = 1:  R^m = F^m - ((U^m - U^{m+1})/tau + A U^m),  U^{n} = 0
 * for the handle's single grid (n = number of systems, m = nx*ny).
 * With F == NULL the operator itself is applied: R = K U (K^T U).
 *   U, F, R  device, complex128 n x m; R may alias F.
 *   norm2    host, NULL or receives ||R||_2^2 (synchronises the stream).
 * Returns VMG_OK, VMG_INVALID_ARG, VMG_HIP_ERROR.
 */
int paradiag_heat_residual(vmg_handle* h, double tau, const double* U, const double* F, double* R,
                           int32_t transpose, double* norm2, void* hip_stream);

/*
 * ParaDIAG-II iteration for the backward-Euler heat all-at-once system
 * K u = f, K = B kron I + I kron A with B = (1/tau)(I - Z) (Z the down-shift,
 * zero initial value), preconditioned by the alpha-circulant system
 * P = C_alpha kron I + I kron A whose eigen-decomposition C_alpha = V D V^{-1}
 * the caller supplies (D = the shifts given at setup; eq. (1)):
 *   u^0 = 0,  u^{k+1} = u^k + P^{-1}(f - K u^k)  until ||f - K u|| <= tol ||f||,
 * every P^{-1} applied by paradiag_apply with inner tolerance inner_tol.
 *   transpose != 0: solve K^T w = f with P^{-T} = P^{-H} (P is real), the
 *            adjoint solve of the heat problem.
 *   replay != 0: repeat exactly the outer and per-system inner iteration
 *            counts recorded by the last call with replay = 0 and the same
 *            transpose flag, making the solve one fixed linear map of f.
 *   F, U     device, complex128 n x m; U may not alias F.
 *   outer    host, NULL or receives the number of preconditioned steps.
 *   relres   host, NULL or receives the final ||f - K u|| / ||f||.
 * Returns VMG_OK, VMG_NOT_CONVERGED (max_outer reached), VMG_INVALID_ARG,
 * VMG_HIP_ERROR, VMG_NAN_DETECTED.
 */
int paradiag_heat_solve(vmg_handle* h, const double* V, const double* Vinv, double tau, const double* F,
                        double* U, double tol, double inner_tol, int32_t transpose, int32_t replay,
                        int32_t max_outer, int32_t* outer, double* relres, void* hip_stream);

/*
 * The same all-at-once heat system K u = f (K^T w = f with transpose) solved
 * by a Krylov method instead of the stationary iteration: restarted flexible
 * GMRES, right-preconditioned by the alpha-circulant ParaDIAG step P^{-1}
 * (the circulant-type preconditioner of Sec. 1; every P^{-1} is applied by
 * paradiag_apply with inner tolerance inner_tol).  From u = 0; a cycle of at
 * most `restart` steps builds v_1 = r/||r||, z_j = P^{-1} v_j, the modified
 * Gram-Schmidt Arnoldi vector of K z_j, and ends with u += sum_j y_j z_j,
 * y minimising the Hessenberg least-squares residual (Givens rotations on the
 * host).  Stops when ||f - K u|| <= tol ||f|| or after max_iter steps in all.
 *   F, U     device, complex128 n x m; U may not alias F.
 *   restart  1..200; the library keeps 2 restart + 1 vectors of n x m.
 *   iters    host, NULL or receives the number of preconditioned steps.
 *   relres   host, NULL or receives the final ||f - K u|| / ||f||.
 * Synchronises the stream once per step.  Returns VMG_OK,
 * VMG_NOT_CONVERGED (max_iter reached), VMG_INVALID_ARG, VMG_OOM,
 * VMG_HIP_ERROR, VMG_NAN_DETECTED.
 */
int paradiag_heat_gmres(vmg_handle* h, const double* V, const double* Vinv, double tau, const double* F,
                        double* U, double tol, double inner_tol, int32_t transpose, int32_t restart,
                        int32_t max_iter, int32_t* iters, double* relres, void* hip_stream);

/*
 * The ParaDIAG step above for the alpha-circulant preconditioner of
 * backward Euler (the circulant-type ParaDIAG preconditioners of Sec. 1):
 * V = diag(alpha^{-i/n}) W with W_ik = exp(-2 pi i ik/n) (indices from 0) and
 * V^{-1} = W^H diag(alpha^{i/n}) / n, so each transform is a length-n DFT
 * along the time index of every node between two diagonal scalings (one
 * read and one write of every value instead of a GEMM).  The shifts given
 * at setup must be the matching eigenvalues, lambda_j =
 * (1 - alpha^{1/n} exp(2 pi i j/n)) / tau.  n = number of systems, a power of
 * two in [2, 256]; 0 < alpha <= 1.  Other arguments and returns as
 * paradiag_apply.
 */
int paradiag_apply_circulant(vmg_handle* h, double alpha, const double* F, double* U, double tol,
                             int32_t conj, const int32_t* fixed_iters, void* hip_stream);

/*
 * The alpha-circulant transforms on their own (n, alpha as above):
 * inverse = 0: out = (V^{-1} kron I) in (conj: V^H); inverse = 1:
 * out = (V kron I) in (conj: V^{-H}).  in, out: device, complex128 n x m
 * row-major, may not alias.  Returns VMG_OK, VMG_INVALID_ARG, VMG_HIP_ERROR.
 */
int paradiag_transform_circulant(int32_t n, int64_t m, double alpha, int32_t inverse, int32_t conj,
                                 const double* in, double* out, void* hip_stream);

/*
 * The time transform of eq. (1) on its own: out = (M kron I_m) in, i.e.
 * out[i, p] = sum_k M[i, k] in[k, p] for i, k < n and p < m, as a complex
 * GEMM on the FP64 matrix cores.  With trans_conj != 0, M^H replaces M.
 *   M        device, complex128 n x n row-major (1 <= n <= 512).
 *   in, out  device, complex128 n x m row-major; may not alias.
 * The expanded real form of M lives in a per-device buffer of the library
 * (allocated on first use, grown when a larger n comes, kept until the
 * process ends).  Its reuse is ordered on the device: each call's stream
 * waits for the previous call's kernels, on whatever stream they ran, so
 * calls on different streams are safe (and serialised there).
 * Returns VMG_OK, VMG_INVALID_ARG, VMG_HIP_ERROR, VMG_OOM.
 */
int paradiag_transform(int32_t n, int64_t m, const double* M, int32_t trans_conj,
                       const double* in, double* out, void* hip_stream);

/*
 * paradiag_transform for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same kernels and results, with the expanded matrix kept in
 * a fixed device array of the library (4 n^2 doubles for n up to
 * VMG_NOALLOC_MAX_N = 256, i.e. 2 MiB per GPU, held until the process ends;
 * its address is looked up once per device on the first call there).  No
 * allocation of any kind is made.  Every call on one GPU uses that GPU's one
 * array: calls that overlap on the device (other streams, other host
 * threads) race and must be ordered by the caller.
 *   n        1 <= n <= VMG_NOALLOC_MAX_N; larger n returns VMG_INVALID_ARG.
 *   other arguments as paradiag_transform.
 * Returns VMG_OK, VMG_INVALID_ARG, VMG_HIP_ERROR.
 */
#define VMG_NOALLOC_MAX_N 256
int paradiag_transform_noalloc(int32_t n, int64_t m, const double* M, int32_t trans_conj,
                               const double* in, double* out, void* hip_stream);

/*
 * Run one operation (VMG_OP_*) of the solver on caller data, for every system
 * of every grid at level `level` (0 = finest), with the handle's shifts (conj
 * as in vanka_mg_solve).  Vectors use the unpadded layout above at that
 * level's size (coarse ops: `out` at level+1 for RESTRICT_RESIDUAL, `b` at
 * level+1 for PROLONG_CORRECT).  x may be NULL for x = 0 (not for
 * PROLONG_CORRECT).  The handle's work buffers at that level are overwritten.
 * Every grid must have more than `level` levels (COARSE_SOLVE: `level` is the
 * coarsest of every grid).  Exists for per-kernel parity tests and tuning.
 * Returns VMG_OK, VMG_INVALID_ARG, VMG_HIP_ERROR.
 */
int vanka_mg_apply_op(vmg_handle* h, int32_t op, int32_t level, int32_t conj,
                      const double* x, const double* b, double* out, void* hip_stream);

/*
 * Kernel timing: with enable != 0 every later kernel launch of the handle is
 * bracketed by HIP events on its stream, and vanka_mg_kernel_stats reports,
 * per kernel class k < VMG_NUM_KCLASS, the launch count, the summed duration
 * (ms) and the summed algorithmic bytes (compulsory HBM bytes of each launch,
 * counted per node as documented for each class).  enable = 0 stops timing;
 * reset clears the sums.
 */
enum {
    VMG_K_SWEEP = 0, VMG_K_RESTRICT = 1, VMG_K_PROLONG = 2, VMG_K_NORM = 3,
    VMG_K_COARSE = 4, VMG_K_PACK = 5, VMG_K_TRANSFORM = 6, VMG_K_IR = 7,
    VMG_K_DOWN = 8,   /* fused pre-smoothing + residual + restriction */
    VMG_K_UP = 9,     /* fused correction + post-smoothing (+ norm)    */
    VMG_K_EDGE = 10,  /* finest level across two V-cycles: correction, post-smoothing, norm,
                         pre-smoothing, residual, restriction in one pass */
    VMG_NUM_KCLASS = 11
};
int vanka_mg_set_timing(vmg_handle* h, int32_t enable, int32_t reset);
/* Kernel classes timed while timing is on: bit k of mask for class k
 * (VMG_K_*), 0 = every class (the default).  Events are recorded only around
 * the launches of those classes, so a single timed class leaves the rest of
 * the work unperturbed.  Returns VMG_OK or VMG_INVALID_ARG (bits beyond the
 * classes). */
int vanka_mg_set_timing_mask(vmg_handle* h, int32_t mask);
int vanka_mg_kernel_stats(vmg_handle* h, int64_t* launches /* [VMG_NUM_KCLASS] */,
                          double* total_ms, double* total_bytes);
/* The same sums for one kernel class split by multigrid level (0 = finest;
 * kernels outside the cycle count as level 0); arrays of nlev entries. */
int vanka_mg_level_stats(vmg_handle* h, int32_t kclass, int32_t nlev, int64_t* launches,
                         double* total_ms, double* total_bytes);

/*
 * Per-system results of the last vanka_mg_solve or paradiag_apply on this
 * handle: cycles (refinement steps) run and final relative residual.  Host
 * arrays of the handle's system count (either may be NULL); synchronises
 * hip_stream.  Returns VMG_OK, VMG_INVALID_ARG, VMG_HIP_ERROR.
 */
int vanka_mg_last_stats(vmg_handle* h, int32_t* iters, double* relres, void* hip_stream);

/*
 * Autotuner: for every grid and level above the coarsest, time each kernel
 * schedule on the handle's own buffers (the LDS-tiled sweep / restriction /
 * prolongation kernels, or the fused streaming kernels with 16, 32, 64 or
 * 128 rows per block; on the finest level also the cycle-edge kernel, see
 * vanka_mg_plan) and keep the fastest.  cache_path (host string, NULL = no
 * cache) is a text file of earlier choices keyed by device, precision, grid,
 * system count and smoothing counts; new choices are appended.  Results of
 * later solves are identical under every schedule up to rounding order.
 * Returns VMG_OK, VMG_INVALID_ARG, VMG_HIP_ERROR.
 */
int vanka_mg_autotune(vmg_handle* h, const char* cache_path, void* hip_stream);

/* Schedule in use for grid g, levels 0..nlev-1: 0 = LDS-tiled kernels, r > 0
 * = streaming kernels with r rows per block, -1 = coarsest / beyond. */
int vanka_mg_schedule(const vmg_handle* h, int32_t g, int32_t nlev, int32_t* sched);

/* Fused kernels in use for grid g (host outputs): *edge = 1 when the finest
 * level runs across the boundary of two V-cycles in one launch (1 or 2 pre-
 * and post-smoothing steps and a streamed finest level; refinement: also the
 * boundary of two refinement steps), 2 when that kernel (refinement: the
 * step boundary pass) runs in paced blocks
 * (a CU's worth of waves on adjacent strips meeting at a barrier after every
 * block of rows; so do the finest level's first pre-smoothing and its
 * finishing pass), else 0; *tail_level = the first level whose work (down to
 * the coarsest solve and back) runs in one workgroup per system, -1 when none
 * does.  Either pointer may be NULL.  Untuned, the cycle-edge kernel runs on
 * grids whose finest levels hold at least 16M nodes over all systems, in
 * plain blocks; vanka_mg_autotune times it against the separate launches per
 * grid, and the paced blocks against the plain ones.  Environment switches
 * read at setup: VMG_EDGE=0 turns it off, VMG_EDGE=2 uses it wherever it
 * applies; VMG_EDGE_PACE=0/1 never/always paces it; VMG_IR_EDGE=0 keeps the
 * refinement step boundary in separate passes; VMG_TAIL=0 turns the tail
 * kernel off; VMG_RECOMP=0/2 never/always (on every streamed coarse level of
 * a V(nu1, nu2) Vanka cycle with nu1, nu2 in {1, 2}; by default on FP64
 * levels of at least 12M nodes and complex64 levels of at least 24M nodes
 * over all systems) lets a coarse level's
 * ascent recompute its pre-smoothed iterate instead of storing it.  Returns VMG_OK or VMG_INVALID_ARG. */
int vanka_mg_plan(const vmg_handle* h, int32_t g, int32_t* edge, int32_t* tail_level);

/* Levels of grid g: writes count and, if non-NULL, nx/ny per level. */
int vanka_mg_levels(const vmg_handle* h, int32_t g, int32_t* count, int32_t* nx, int32_t* ny);

/* Release every resource of the handle (NULL is accepted). */
int vanka_mg_destroy(vmg_handle* h);

/* Static text for a VMG_* code. */
const char* vanka_mg_error_string(int code);

#ifdef __cplusplus
}
#endif

#endif /* VANKA_MG_H */
