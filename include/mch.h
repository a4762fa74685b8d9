/*
 * mch.h -- C ABI of the hierarchical multicontinuum homogenization cell-solve
 * library (libmch.so) for AMD Instinct MI355X (gfx950).
 *
 * The library computes, for every macropoint of a structured macrogrid, the
 * local solutions of the constrained cell problems of multicontinuum
 * homogenization (Xie, Hoang, Yang, Huang, arXiv 2503.01276, Sec. 2,
 * Eqs. phi_avar and phi_grad), either on the fine grid at every macropoint
 * (flat method, levels = 1) or hierarchically (Sec. 3, Algorithm 1): a
 * macropoint of level n >= 2 inherits fine solutions of lower levels (that of
 * the level-1 macropoint of its group, or a multilinear interpolation of its
 * neighbours in T_(n-1)) and solves a correction on the coarsened mesh
 * h*eta^(n-1) (Eqs. phi_avar_corrector and phi_grad_corrector). From the local
 * solutions it forms the effective coefficient tensors (Eq. Bs_defi) and the
 * adjoint gradient of a loss on them with respect to log kappa per fine element.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Fine elements: e = i1 + n1*(i2 + n2*i3) (x1 fastest), uniform size h, on the
 *   unit square / cube; kappa is piecewise constant per element and labels
 *   (continuum index of each element, 0..n_cont-1) are uint8.
 * Macropoints: p = j1 + m1*(j2 + m2*j3); macropoint p is the centre of coarse
 *   block K_p, the H^d block of fine elements starting at H*j (H = n_fine/n_macro).
 * Cell of p: n_cell^d fine elements centred on the macropoint, local
 *   coordinates centred there; kappa and labels are sampled with periodic wrap
 *   of the global grid; homogeneous Dirichlet data on the cell boundary.
 * Constraint regions: the cell is tiled by n_sub^d equal sub-blocks R_q; one
 *   constraint row per (R_q, continuum j) holding the average of the unknown
 *   over R_q intersected with continuum j (rows with an empty intersection are
 *   inactive).
 * Right-hand sides: M = N + N*d per macropoint; alpha = i is phi_i (average
 *   constraints delta_ij), alpha = N + i*d + m is phi_i^m (first-moment
 *   constraints delta_ij*(xbar_{m,qj} - c_mj), c_mj the continuum-j centroid in K_p).
 * Hierarchy: T_n keeps macropoints with index = o (mod eta^(L-n)) per axis,
 *   o = floor(eta^(L-1)/2); S_1 = T_1, S_n = T_n minus T_(n-1) (Sec. 3.1,
 *   Eq. defi_Sn). A level-n point inherits I = sum_t c_t Phi_t (Sec. 3.3,
 *   Eq. phiXiI_all): with interp = 0 the level-1 point of its aligned
 *   eta^(L-1)-per-axis block with weight 1 (the rule of the paper's
 *   experiments); with interp = 1 the points of T_(n-1) that bracket it per
 *   axis (lattice step eta^(L-n+1), periodic in the macropoint index) with
 *   tensor-product linear weights, which sum to 1.
 * Precision: every floating-point quantity is IEEE binary64.
 *
 * Memory and streams
 * ------------------
 * Every pointer argument named kappa, label, A_eff, gA, glogk or out is a
 * device pointer on the plan's device, contiguous, owned by the caller.
 * The plan owns its scratch (local solutions, multipliers, diagnostics).
 * hip_stream is a hipStream_t (NULL = default stream). Calls are asynchronous
 * on that stream unless stated otherwise; a plan must not be used from two
 * streams concurrently.
 *
 * Errors
 * ------
 * Every int-returning call returns MCH_OK (0) or a negative code; nothing
 * throws across the ABI. mch_last_error() returns a thread-local message
 * describing the most recent failure on the calling thread.
 *
 * Tuning knobs
 * ------------
 * mch_build_levels reads these environment variables when it creates a
 * plan. None changes the problems solved, only how they are solved; results
 * agree to the Krylov tolerance (the preconditioner knobs move the iterates)
 * or bitwise where stated:
 *   MCH_RPT_<NC>     node rows per thread of the 2D solve kernel for level
 *                    cell width NC (default 8 for NC >= 64, else 4; a value
 *                    without an instantiated kernel falls back to the first
 *                    valid one of 4, 8, 2, 1, 16);
 *   MCH_PREC         band coarse correction in the 2D preconditioner: 0 off,
 *                    1 on for widths >= 64 (default), 2 on for every width
 *                    with a kernel;
 *   MCH_PREC_<NC>    the same per width: 0 off, 1 bands of a thread's node
 *                    rows, 2 two sub-bands of half as many rows (each only
 *                    where its kernel exists and fits the LDS, else off);
 *   MCH_SPLIT        0 runs level 1 as one launch instead of two (default 1);
 *   MCH_GENERIC      1 puts every level on the generic solve kernels (the
 *                    kernels Neumann cells and wide cells always use);
 *   MCH_XCD          0 numbers the 2D solve's workgroups in plain order
 *                    instead of grouping a cell's right-hand sides on one XCD
 *                    (bitwise the same results);
 *   MCH_SETUP_WIDE   0 keeps 256-thread set-up workgroups on levels of at most
 *                    128 cells (default 1: 1024 threads there; read once per
 *                    process);
 *   MCH_GRAPHS       0 launches every call eagerly instead of replaying
 *                    captured graphs;
 *   MCH_SERIAL       1 puts every launch on the caller's stream (isolated
 *                    per-kernel timings);
 *   MCH_MACRO_GRID   workgroups of the grid-wide macroscopic CG.
 * mch_plan_info reports the shape and preconditioner each level took.
 */
#ifndef MCH_H
#define MCH_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MCH_OK 0
#define MCH_EINVAL (-1)     /* invalid configuration or argument */
#define MCH_ESINGULAR (-2)  /* over-constrained coarsest level or singular Schur matrix */
#define MCH_ENOCONV (-3)    /* a Krylov solve hit max_iter before rtol (results still written) */
#define MCH_EHIP (-4)       /* HIP runtime error */
#define MCH_ESTALE (-5)     /* backward / effective tensors requested without a completed forward */
#define MCH_ENOTIMPL (-6)   /* configuration recognised but not implemented */

typedef struct {
  int32_t dim;          /* 2 or 3 */
  int32_t n_fine[3];    /* fine elements per axis (equal on used axes; unused axes = 1) */
  double h;             /* fine element size, must equal 1/n_fine[0] */
  int32_t n_macro[3];   /* macropoints per axis (equal on used axes); H = n_fine/n_macro, even */
  int32_t n_cell;       /* oversampled cell width in fine elements; even, divisible by n_sub*eta^(L-1) */
  int32_t n_sub;        /* constraint sub-blocks per axis (s) */
  int32_t n_cont;       /* number of continua N (1..3) */
  int32_t levels;       /* L >= 1; L = 1 is the flat method */
  int32_t eta;          /* coarsening factor >= 1; n_macro divisible by eta^(L-1) */
  int32_t interp;       /* 0: inherit the level-1 solution of the group (the paper's experiments);
                           1: multilinear interpolation from T_(n-1) */
  int32_t bc;           /* cell boundary condition (Sec. 2, the artificial conditions on R_p^+):
                           0: homogeneous Dirichlet; 1: natural Neumann, every cell node free
                           (interp = 0; 3D with n_sub = 2; solved by the generic kernels) */
  double rtol;          /* relative tolerance on the projected preconditioned residual norm */
  int32_t max_iter;     /* Krylov iteration cap per solve */
} mch_config;

typedef struct mch_plan mch_plan;

/* Build the macrogrid hierarchy (Algorithm 1 steps 1-2; Sec. 3.1-3.2),
 * validate the configuration, choose kernels per size class, and allocate the
 * plan's device scratch on the current HIP device. Synchronous.
 * 2D levels run on the register-resident solve kernel where one is
 * instantiated for the level's shape (widths 8..64, Dirichlet cells), else on
 * the generic kernel (Krylov vectors in device memory): Neumann cells, cells
 * up to 128 fine elements wide, any width divisible by n_sub, n_sub <= 8.
 * 3D levels run on the column-marching kernel (Dirichlet cells, widths 8, 16,
 * 32, n_sub = 2) or, for Neumann cells, on the generic 3D kernel.
 * Returns MCH_EINVAL for inconsistent sizes, MCH_ESINGULAR when the coarsest
 * level has more constraint rows than free unknowns, MCH_ENOTIMPL for a mode
 * outside the implemented ones, MCH_EHIP on allocation failure.
 * On success *out owns the plan; release it with mch_destroy. */
int mch_build_levels(const mch_config* cfg, mch_plan** out);

/* Host-only form of the hierarchy step (no device needed): level and
 * inherited level-1 macropoint of every macropoint for the given macrogrid
 * (only dim, n_macro, levels and eta are read), into host arrays of length
 * n_macro^dim. Synchronous. MCH_EINVAL for inconsistent sizes. */
int mch_build_hierarchy(const mch_config* cfg, int32_t* level, int32_t* parent);

/* Host-only: the neighbours and weights of the multilinear rule (interp = 1,
 * Sec. 3.3, Eq. phiXiI_all) for every macropoint, whatever cfg->interp says.
 * nbr [n_macro^dim][2^dim] receives neighbour macropoint indices (-1 where
 * unused, and for every slot of a level-1 point), weight the same shape
 * (0 where unused); per point the entries are the tensor products of the
 * per-axis (lower, upper) choices, axis 1 fastest, aligned axes contributing
 * the lower one only. Only dim, n_macro, levels and eta are read. Host
 * arrays owned by the caller. Synchronous. MCH_EINVAL for inconsistent sizes. */
int mch_build_interp(const mch_config* cfg, int32_t* nbr, double* weight);

/* Static description of a built plan (host memory, synchronous):
 * info[0] = P (macropoints), info[1] = M (right-hand sides per macropoint),
 * info[2] = m (constraint rows per cell, including inactive ones),
 * info[3] = L, info[4..4+L) = number of macropoints of each level,
 * info[4+L..4+2L) = node rows per thread of each level's 2D solve kernel (the
 * size-class shape: the workgroup has NC^2 / rows threads; 0 in 3D and for
 * levels on the generic 2D kernel),
 * info[4+2L..4+3L) = the sub-bands per thread's node rows (1 or 2) where the
 * level's 2D solve preconditions with the band coarse correction, 0 where
 * with the diagonal alone (and in 3D), the rest zero. info must hold at
 * least 28 entries (4 + 3 * 8 levels). */
int mch_plan_info(const mch_plan* plan, int64_t* info);

/* Level (1..L) and the level-1 macropoint of its group (-1 for level 1) of
 * every macropoint, into host arrays of length P (with interp = 1 the
 * neighbours are those of mch_build_interp). Synchronous. */
int mch_hierarchy(const mch_plan* plan, int32_t* level, int32_t* parent);

/* Algorithm 1 steps 3-5 (Sec. 3.3): solve every cell problem, level by level,
 * in the hierarchical form (inherited solution plus correction in V_n).
 * kappa: [n_fine^d] f64 > 0, finite; label: [n_fine^d] u8 < n_cont. A
 * device-side check of both runs first in the same launch sequence; a
 * violation is reported as MCH_EINVAL by mch_diagnostics (the call itself
 * stays asynchronous). Asynchronous on hip_stream. Returns MCH_ENOCONV only
 * from mch_diagnostics; here errors are argument and launch errors. */
int mch_solve_cells(mch_plan* plan, const double* kappa, const uint8_t* label, void* hip_stream);

/* Effective tensors (Eq. Bs_defi with R_p = K_p): A_eff[p][a][b] =
 * sum over fine elements e of K_p of kappa_e Phi_a|_e^T K_ref Phi_b|_e for the
 * M local solutions of macropoint p. kappa must be the array passed to the
 * last mch_solve_cells (MCH_EINVAL otherwise). A_eff: [P][M][M] f64 device
 * array. Asynchronous. MCH_ESTALE if no forward solve has been issued on
 * this plan. */
int mch_effective_coeffs(mch_plan* plan, const double* kappa, double* A_eff, void* hip_stream);

/* Adjoint of mch_effective_coeffs o mch_solve_cells: given gA[p][a][b] =
 * dLoss/dA_eff[p][a][b], writes glogk[e] = dLoss/dlog(kappa_e) for every
 * fine element (the gradient flows through the local solutions, through the
 * inherited solutions of the lower levels, and through the explicit kappa in
 * the tensors). Uses the state of the most recent forward on this plan,
 * including its kappa and label arrays, which must still hold the forward's
 * values; kappa must be that forward's array (MCH_EINVAL otherwise).
 * gA: [P][M][M], glogk: [n_fine^d] f64 device. Asynchronous. MCH_ESTALE if
 * no forward solve has been issued. */
int mch_effective_coeffs_backward(mch_plan* plan, const double* kappa, const double* gA,
                                  double* glogk, void* hip_stream);

/* The upscaled multicontinuum system (Sec. 2, Eq. macro_eq with the
 * coefficients of Eq. Bs_defi; the last step of Algorithm 1).
 *
 * mch_macro_load: b[p][j] = int_{K_p} f phi_j for j < n_cont, with f
 * piecewise constant per fine element ([n_fine^d] f64 device array) and phi_j
 * the type-1 local solutions of the most recent forward on this plan.
 * b: [P][n_cont] f64 device array. Asynchronous. MCH_ESTALE without a
 * forward. */
int mch_macro_load(mch_plan* plan, const double* f, double* b, void* hip_stream);

/* mch_macro_solve: the weak form sum_p int_{K_p} w_V^T (A_eff(p)/|K_p|) w_U =
 * sum_p int_{K_p} (b(p)/|K_p|) . V, with w = (U_j, d_m U_j) in the
 * right-hand-side order of the cell problems, discretised by multilinear
 * elements on the coarse blocks (nodes at the block corners of the unit
 * square or cube, U = 0 on its boundary, the block densities integrated exactly),
 * solved by CG preconditioned with the inverse N x N block of each node (its
 * continua) to the relative tolerance rtol on the preconditioned residual
 * (sqrt(r^T M^-1 r) over its initial value), at most max_iter iterations. A_eff: [P][M][M] and
 * b: [P][n_cont] device inputs (any source, e.g. mch_effective_coeffs and
 * mch_macro_load); U: [(n_macro+1)^d][n_cont] nodal values (node
 * k1 + (n_macro+1) (k2 + (n_macro+1) k3)), U_block: [P][n_cont] block
 * averages, device outputs.
 * Systems of up to 19456 / (5 + n_cont) unknowns are solved by one
 * workgroup with its vectors in LDS; larger ones by one cooperative launch
 * over the device (at most two workgroups per CU) with a fixed-order
 * grid-wide reduction, so the result is bitwise reproducible either way.
 * The plan allocates the solve's scratch on the first call (host-synchronous
 * then); otherwise asynchronous. MCH_EINVAL for bad arguments. */
int mch_macro_solve(mch_plan* plan, const double* A_eff, const double* b, double* U, double* U_block,
                    double rtol, int32_t max_iter, void* hip_stream);

/* For callers that cannot allocate device memory when they call (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * mch_macro_solve with every intermediate array in one fixed device buffer of
 * the library instead of the plan's scratch, which mch_macro_solve allocates
 * on its first call. The buffer holds 16 MiB on each device the library runs
 * on, until the process ends; systems whose element matrices, stencil rows
 * and vectors need more ((P (2^d N)^2 + 3^d N n + (6 + N) n + 8192) doubles,
 * n = (n_macro - 1)^d N unknowns: the 512^2 and 128^3 workloads need about
 * 1 MiB) are refused with MCH_EINVAL. Same arguments and results as
 * mch_macro_solve; additionally iters [1] (int32) and resid [1] (f64) are
 * device outputs receiving the iteration count and the final relative
 * residual (mch_macro_diagnostics does not see this call). Makes no
 * hipMalloc, hipFree or other allocation and does not modify the plan.
 * Every call on one device shares the buffer: calls that overlap on one
 * device (two streams, two threads) race on it and must not be issued.
 * Asynchronous on hip_stream. MCH_EINVAL for bad arguments. */
int mch_macro_solve_noalloc(const mch_plan* plan, const double* A_eff, const double* b, double* U,
                            double* U_block, double rtol, int32_t max_iter, int32_t* iters, double* resid,
                            void* hip_stream);

/* Iterations and final relative residual of the most recent mch_macro_solve
 * (host, synchronous). MCH_ENOCONV if it stopped at max_iter above rtol,
 * MCH_ESTALE if none has been issued. */
int mch_macro_diagnostics(const mch_plan* plan, int32_t* iters, double* resid);

/* Test hook: the full fine local solutions Phi of the listed macropoints,
 * out[k][a][node] with node = b1 + (n_cell+1)*(b2 + (n_cell+1)*b3) over all
 * (n_cell+1)^d cell nodes (boundary nodes are zero). cells: host array of n
 * macropoint indices. out: device array. Asynchronous. */
int mch_local_solutions(mch_plan* plan, const int64_t* cells, int64_t n, double* out, void* hip_stream);

/* Per (macropoint, right-hand side) Krylov iteration count and final relative
 * projected residual of the most recent forward solve, into host arrays of
 * length P*M. Synchronous (waits for the plan's last stream). Returns
 * MCH_EINVAL when the forward's kappa was not positive and finite or a label
 * was >= n_cont on some fine element (the message names the first one; the
 * forward checks its inputs on the device before the cell kernels, and its
 * results are then meaningless); otherwise the verdict of
 * mch_classify_solves on the records (MCH_ESINGULAR, MCH_ENOCONV or MCH_OK). */
int mch_diagnostics(const mch_plan* plan, int32_t* iters, double* resid);

/* Host-only rule by which mch_diagnostics and mch_adjoint_diagnostics judge
 * their per-solve records: MCH_ESINGULAR if any iteration count is negative
 * (a singular constraint Schur matrix), else MCH_ENOCONV if any residual is
 * not finite (NaN: the recurrence left the finite numbers) or a solve stopped
 * at max_iter with a residual above rtol, else MCH_OK. iters and resid are
 * host arrays of n entries owned by the caller. Synchronous; MCH_EINVAL for
 * null arrays with n > 0 or n < 0. */
int mch_classify_solves(const int32_t* iters, const double* resid, int64_t n, int32_t max_iter, double rtol);

/* Measurement hook. mode 1 turns profiling on, 0 off; either clears the
 * records. While on, every kernel launch of the plan is bracketed by HIP
 * events recorded on the launch's own stream. Host-side, synchronous. */
int mch_profile(mch_plan* plan, int32_t mode);

/* With idx < 0 returns the number of profile records. Otherwise waits for
 * record idx and writes its kernel name (NUL-terminated, at most cap bytes)
 * and its elapsed milliseconds; returns the record count or an error. */
int mch_profile_read(mch_plan* plan, int32_t idx, char* name, int32_t cap, double* ms);

/* As mch_diagnostics, for the adjoint solves of the most recent
 * mch_effective_coeffs_backward (zeros before the first backward). */
int mch_adjoint_diagnostics(const mch_plan* plan, int32_t* iters, double* resid);

/* Release the plan and its device scratch. NULL is allowed. */
void mch_destroy(mch_plan* plan);

/* Thread-local description of the last error on this thread ("" if none). */
const char* mch_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* MCH_H */
