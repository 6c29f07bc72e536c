/*
 * fe.h -- C ABI of the MI355X implicit finite-element step library.
 *
 * The library implements the per-time-step hot path of the implicit FE
 * method of Zeng & Courtecuisse, "Efficient parallelization strategy for
 * real-time FE simulations" (arXiv 2306.05893):
 *
 *   assembly   element tangents and internal forces, scattered through a map
 *              built once from the topology into a fixed-pattern CSR matrix
 *              A = (1 + h alpha) M + h (beta + h) K and right-hand side b
 *              (Sec. 3.2, Eq. "dynamic equation2"; Sec. 4.2 "fast assembly");
 *   solve      preconditioned CG on A whose preconditioner is the LDL^T
 *              factor of an earlier A (Sec. 3.3, Eq. "asynchronous
 *              preconditioner"), applied by level-scheduled triangular solves
 *              over a nested-dissection partition (Sec. 5.1, Eq. "regional
 *              problem");
 *   step       backward-Euler update (Eq. "implicit integration").
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Every function returns an int: FE_OK (0) or a negative FE_E* code.  No
 *   C++ exception crosses this boundary.  fe_last_error(ctx) returns a
 *   human-readable message for the last failing call on that context.
 * - "host" pointers point to CPU memory, "device" pointers to GPU memory
 *   (hipMalloc'd or a torch CUDA tensor).  Device buffers passed to a call
 *   are owned by the caller and must stay valid until the work queued on
 *   `stream` has completed.  The library allocates no device memory of its
 *   own: fe_query reports how many bytes of device workspace a context needs
 *   and fe_bind hands it a caller-owned buffer of that size.
 * - DOF numbering: DOF 3*i + c is coordinate c of node i.  All state and
 *   force vectors are FP64, length 3*n_nodes.
 * - `stream` is a hipStream_t passed as void* (NULL = the default stream).
 *   Calls on one context are not re-entrant; use one context per stream.
 * - Precision: FE_PREC_FP64 computes everything in FP64.  FE_PREC_MIXED
 *   stores A and the factor panels in FP32 and runs the element arithmetic
 *   and the triangular solves in FP32; the SpMV reads the FP32 values of A
 *   and upcasts them exactly, so its products and row sums are FP64, as are
 *   state, CG vectors, dot products, alpha/beta and the residual check.  The
 *   LDL^T factorisation itself is always FP64, on the GPU (its own stream;
 *   fe_build_opts.factor_on_gpu = 1) or on the host factor thread, and its
 *   panels are rounded to FP32 once when they are written.  The adjoint
 *   element pass of fe_step_adjoint is FP64 in both modes.
 */
#ifndef FE_H
#define FE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------ */
#define FE_OK         0
#define FE_EINVAL    -1  /* bad argument, index or size                        */
#define FE_ENOMEM    -2  /* host allocation failed / workspace too small       */
#define FE_EINVERTED -3  /* an element has det F <= 0 (inverted)               */
#define FE_EINDEF    -4  /* CG breakdown: p^T A p <= 0 (A not SPD)             */
#define FE_ENOTCONV  -5  /* CG hit max_it; x and the stats are still valid     */
#define FE_EFACTOR   -6  /* LDL^T hit a non-positive pivot                     */
#define FE_EBUSY     -7  /* a factorisation job is still running               */
#define FE_EDEVICE   -8  /* a HIP runtime call failed                          */
#define FE_ESTATE    -9  /* call out of order (e.g. not bound yet)             */

/* ---- enumerations ------------------------------------------------------ */
#define FE_TET4 4               /* linear tetrahedron, 1 quadrature point    */
#define FE_HEX8 8               /* trilinear hexahedron, 2x2x2 Gauss points  */

#define FE_NEO_HOOKEAN   0      /* compressible neo-Hookean                  */
#define FE_STVK          1      /* St Venant-Kirchhoff                       */
#define FE_COROTATIONAL  2      /* co-rotational linear elasticity (Sec. 3.1,
                                   Eq. "eqmodel"): f = R K0 (R^T x - X),
                                   K = R K0 R^T, R the rotation of the polar
                                   decomposition of F at the element centre  */
#define FE_MOONEY_RIVLIN 3      /* Mooney-Rivlin in the isochoric invariants
                                   (Sec. 3.1, MJED materials):
                                   C10 (J^-2/3 I1 - 3) + C01 (J^-4/3 I2 - 3)
                                   + kappa/2 (ln J)^2                         */

#define FE_PREC_FP64  0
#define FE_PREC_MIXED 1

#define FE_FACTOR_DETERMINISTIC 0 /* factor of A_{kR} used from step kR+d   */
#define FE_FACTOR_ASYNC         1 /* newest finished factor is swapped in    */

typedef struct fe_ctx fe_ctx;

/* Mesh topology and rest geometry (host arrays, read during the call). */
typedef struct {
  int32_t n_nodes;
  int32_t n_elems;
  int32_t elem_type;          /* FE_TET4 or FE_HEX8                           */
  const int32_t *conn;        /* host [n_elems * nen], element-major          */
  const double *X;            /* host [3 * n_nodes] rest coordinates          */
} fe_mesh;

typedef struct {
  int32_t leaf_nodes;         /* nested-dissection leaf size in nodes (0: 48) */
  int32_t fwd_tile_cols;      /* forward-sweep tile width 16/32/64/128 for every
                                 level; 0: chosen per level (64, or 128 on levels
                                 of supernodes with 65..128 own columns)       */
  int32_t bwd_tile_rows;      /* backward tile height 256/512/1024 for every
                                 level; 0: chosen per level (512, or 256 where
                                 it pads the level's panel rows clearly less) */
  int32_t factor_on_gpu;      /* 1: fe_factor_async runs the FP64 multifrontal
                                 LDL^T on the GPU (own stream, writes the idle
                                 factor slot directly; no host round trip);
                                 0: host factor thread (the paper's scheme)  */
  int32_t n_threads;          /* host factorisation threads (0: the CPU share:
                                 min(cores, OMP_NUM_THREADS, 16) - 1)         */
  int32_t factor_max_blocks;  /* GPU factorisation: upper bound on the work-
                                 groups of one launch (its kernels loop over
                                 their work), i.e. on the share of the GPU the
                                 background refactorisation takes from the
                                 solves; 0: no bound                          */
  int32_t bwd_tile_cols;      /* backward tile width 16/32/64 for every level
                                 (4 columns per wavefront: 4, 8 or 16
                                 wavefronts share a tile's gathered inputs);
                                 0: chosen per level (64, or 32 where 64 pads
                                 the level's own columns more)               */
  int32_t fwd_col_groups;     /* forward tiles of 1, 2 or 4 groups of 64
                                 columns (4 wavefronts each) whose row sums
                                 meet in one atomic, on every 64-column level;
                                 0: chosen per level (4 on levels of wide
                                 supernodes, else 1)                         */
} fe_build_opts;

/* Physical parameters of one assembly.  E and f_nodal are DEVICE pointers. */
typedef struct {
  double h;                   /* time step                                    */
  double alpha, beta;         /* Rayleigh damping B = alpha M + beta K        */
  double rho;                 /* density                                      */
  double nu;                  /* Poisson ratio                                */
  int32_t material;           /* FE_NEO_HOOKEAN, FE_STVK, FE_COROTATIONAL or
                                 FE_MOONEY_RIVLIN                             */
  int32_t pad_;
  double gravity[3];          /* body acceleration                            */
  const double *E;            /* device [n_elems] Young's modulus per element */
  const double *f_nodal;      /* device [3 n_nodes] point loads, or NULL      */
  double mr_c01_share;        /* Mooney-Rivlin: C10 = (1 - s) mu / 2,
                                 C01 = s mu / 2, kappa = lambda + 2 mu / 3
                                 (mu, lambda from E, nu); s in [0, 1]          */
} fe_params;

typedef struct {
  int64_t n_dofs;             /* 3 * n_nodes                                  */
  int64_t nnz;                /* CSR nonzeros of A (structural)               */
  int64_t n_elems;
  int64_t map_len;            /* canonical map entries = n_elems * (3 nen)^2  */
  int64_t n_supernodes;       /* nested-dissection blocks of the factor       */
  int64_t n_levels;           /* dependency levels of the triangular solves   */
  int64_t factor_entries;     /* stored panel entries (incl. explicit zeros)  */
  int64_t factor_lower;       /* panel entries on/below the diagonal          */
  double factor_flops;        /* flops of one numeric factorisation           */
  int64_t ws_bytes;           /* device workspace for the queried precision   */
  int32_t compact_map;        /* 1: 1-byte slot map in use, 0: int32 map      */
  int32_t pad_;
} fe_sizes;

typedef struct {
  int32_t iterations;         /* CG iterations performed                      */
  int32_t status;             /* FE_OK / FE_ENOTCONV / FE_EINDEF              */
  double rel_res;             /* FP64 recomputed ||b - A x|| / ||b||          */
  int64_t factor_tag;         /* tag of the factor used, -1 = Jacobi          */
} fe_solve_stats;

typedef struct {
  double rel_tol;             /* stopping test on the recomputed residual     */
  int32_t max_it;
  int32_t refresh;            /* R: factor A every R steps (0: never)         */
  int32_t lag;                /* d: deterministic mode uses A_{kR} from kR+d  */
  int32_t mode;               /* FE_FACTOR_DETERMINISTIC / FE_FACTOR_ASYNC    */
  int32_t warm_start;         /* initial guess of the CG (the paper is silent;
                                 0, the default, is x0 = 0):
                                 1: the previous step's acceleration;
                                 m = 2..8: the A-norm projection of the
                                 solution onto the last m accelerations,
                                 x0 = V c with (V^T A V) c = V^T b (Fischer's
                                 projection for successive right-hand sides;
                                 m SpMV-like products and a few dot products
                                 per step; vectors that are nearly
                                 combinations of newer ones are dropped).
                                 Values above 8 use 8.                        */
  int32_t rotate_precond;     /* 1: apply the stale factor rotated to the
                                 current state, P^{-1} = Q A_t0^{-1} Q^T with
                                 Q_n = R_n(t) R_n(t0)^T per node (R_n: the
                                 rotation of the polar decomposition of the
                                 summed element-centre deformation gradients
                                 around node n; Q_n = I on nodes with a fixed
                                 DOF).  Not in the paper: a correction of the
                                 asynchronous preconditioner for bodies that
                                 rotate; still symmetric positive definite, so
                                 the results meet the same test.  0: off.     */
} fe_step_opts;

typedef struct {
  fe_solve_stats solve;
  int64_t step;               /* index of the step just taken                 */
  int64_t factor_lag;         /* step - tag of the factor used (-1: Jacobi)   */
} fe_step_stats;

/* ---- context ----------------------------------------------------------- */

/* Build the CSR pattern of A and the element-to-nonzero map by two counting
 * sort transposes of the triplet keys, dropping the rows/columns of fixed
 * DOFs and giving them a lone diagonal entry (Sec. 4.2, Table "build
 * pattern"; Sec. 6.1).  Also computes the nested-dissection ordering, the
 * supernodal structure of L and the level sets of the triangular solves
 * (Sec. 5.1).  Host work only; no GPU is touched.
 *   mesh       topology and rest coordinates (host)
 *   fixed_dof  host [3 n_nodes], 1 = Dirichlet DOF, NULL = none
 *   opts       NULL for defaults
 *   out        receives a new context (free with fe_destroy)
 * Errors: FE_EINVAL (node index out of range, bad element type, an element
 * with non-positive rest volume), FE_ENOMEM. */
int fe_build_pattern(const fe_mesh *mesh, const uint8_t *fixed_dof,
                     const fe_build_opts *opts, fe_ctx **out);

/* Sizes of the context's structures; ws_bytes is for precision `prec`. */
int fe_query(fe_ctx *ctx, int32_t prec, fe_sizes *out);

/* Bind a caller-owned device workspace of at least fe_query().ws_bytes bytes
 * (256-byte aligned) for precision `prec`, upload the pattern, map, mesh and
 * solve schedule into it (queued on `stream`), and start the factor thread.
 * Errors: FE_ENOMEM (buffer too small), FE_EINVAL, FE_EDEVICE. */
int fe_bind(fe_ctx *ctx, int32_t prec, void *d_workspace, int64_t ws_bytes,
            void *stream);

/* Copy the pattern and the canonical triplet map to host arrays:
 *   row_ptr [n_dofs + 1], col_idx [nnz], map [map_len] (triplet t of the
 *   element-major fill order -> CSR slot, -1 = dropped).  Any pointer may be
 *   NULL.  Host work only. */
int fe_export_pattern(fe_ctx *ctx, int32_t *row_ptr, int32_t *col_idx, int32_t *map);

/* Export the nested-dissection permutation (host [n_dofs]: perm[k] = DOF
 * eliminated k-th; fixed DOFs last) and the supernode boundaries
 * (host [n_supernodes + 1] offsets into perm).  Either pointer may be NULL. */
int fe_export_ordering(fe_ctx *ctx, int32_t *perm, int32_t *sn_ptr);

/* Export the supernodal structure of the factor (Sec. 5.1, the regional
 * problems of the level-scheduled solve): per supernode s (host
 * [n_supernodes] each), n_rows[s] = rows of its panel (its own columns,
 * sn_ptr[s+1] - sn_ptr[s] of fe_export_ordering, first, then the rows below
 * them), and level[s] = its level in the assembly tree (0 = leaves; every
 * supernode's level is above its children's; the triangular sweeps run one
 * launch per level).  Either pointer may be NULL.  Host work only. */
int fe_export_supernodes(fe_ctx *ctx, int32_t *n_rows, int32_t *level);

/* Export the triangular sweeps' tile schedule (Sec. 5.1: the level-scheduled
 * solve of the regional problems), for diagnostics and tests.  Counts:
 * *n_levels, *n_fwd, *n_bwd (any may be NULL).  extents (host [n_levels * 4]
 * or NULL): per level, the forward tile width in columns per group, the
 * forward column groups, the backward tile height and width.  fwd / bwd
 * (host [n_fwd * 3] / [n_bwd * 3] or NULL): per tile, in launch order
 * (forward: levels ascending; backward: descending), its supernode, first
 * panel row r0 and first own column c0.  A forward tile covers rows r0 ..
 * r0 + 255 and columns c0 .. c0 + width * groups - 1, a backward tile rows
 * r0 .. r0 + height - 1 and columns c0 .. c0 + width - 1, clipped to the
 * supernode's panel; only entries on or below the diagonal of L11^{-1} are
 * read.  Host work only. */
int fe_export_sweep_tiles(fe_ctx *ctx, int32_t *n_levels, int32_t *n_fwd, int32_t *n_bwd,
                          int32_t *extents, int32_t *fwd, int32_t *bwd);

/* Assemble A (CSR values, FP32 for FE_PREC_MIXED / FP64 for FE_PREC_FP64,
 * device [nnz]) and b (FP64 device [n_dofs]) at state (q, v) (device [n_dofs]
 * each):  A = (1 + h alpha) M + h (beta + h) K(q),
 *         b = p - f(q) - alpha M v - (beta + h) K(q) v,   p = M g + f_nodal,
 * with fixed rows/cols replaced by the identity and b_d = 0 (Sec. 3.2,
 * Sec. 4.2 merged LHS/RHS assembly, Sec. 6.1).  Queued on `stream`; returns
 * FE_EINVERTED if an element with det F <= 0 was met (checked after the
 * stream work completes, so this call synchronises `stream`). */
int fe_assemble(fe_ctx *ctx, const fe_params *params, const double *q,
                const double *v, void *A_vals, double *b, void *stream);

/* Snapshot A (device, the context's precision) after the work queued on
 * `stream`, and factor it as P = L D L^T in FP64 (Sec. 3.3): on the GPU, on
 * the context's own factorisation stream, when the context was built with
 * factor_on_gpu = 1 (the result is written straight into the idle factor
 * slot), else on the host factor thread (the snapshot is copied to pinned
 * host memory first).  Work queued on `stream` after this call waits for
 * the snapshot copy, so A may be overwritten by the next assembly at once.
 * Returns without waiting for the factorisation.  `tag` labels the factor
 * (usually the step index).  FE_EBUSY if a previous job has not finished. */
int fe_factor_async(fe_ctx *ctx, const void *A_vals, int64_t tag, void *stream);

/* Newest finished factor's tag (-1 if none) and the status of the last job. */
int fe_factor_status(fe_ctx *ctx, int64_t *ready_tag);

/* Block until the job with `tag` has finished; returns its status. */
int fe_factor_wait(fe_ctx *ctx, int64_t tag);

/* Make the newest finished factor the preconditioner for later solves (the
 * upload is queued on an internal copy stream and ordered before later work
 * on `stream`).  Returns its tag in *tag (NULL allowed), -1 if none. */
int fe_factor_install(fe_ctx *ctx, int64_t *tag, void *stream);

/* Preconditioned CG on A x = b (Sec. 5, Fig. "DataTransfer": SpMV, vector
 * operations and the preconditioner all on the GPU, one small status word
 * read back per batch of iterations).  A_vals device [nnz] in the context's
 * precision, b and x FP64 device [n_dofs]; x holds x0 on entry.  Stops when
 * the FP64 recomputed ||b - A x|| <= rel_tol ||b||.  Preconditioner: the
 * installed LDL^T factor, else Jacobi.  Synchronises `stream`.
 * Errors: FE_ENOTCONV (x, stats valid), FE_EINDEF. */
int fe_pcg_solve(fe_ctx *ctx, const void *A_vals, const double *b, double *x,
                 double rel_tol, int32_t max_it, void *stream, fe_solve_stats *stats);

/* One full step at state (q, v) (device, FP64, updated in place): assemble,
 * schedule/install factors per opts, solve A a = b, then v += h a,
 * q += h v (Eq. "implicit integration").  a_out (device [n_dofs]) may be
 * NULL.  A, b and the CG vectors live in the workspace. */
int fe_step(fe_ctx *ctx, double *q, double *v, const fe_params *params,
            const fe_step_opts *opts, double *a_out, void *stream, fe_step_stats *stats);

/* One reverse step of the adjoint of fe_step (not in the paper), for the
 * neo-Hookean and St Venant-Kirchhoff materials (FE_EINVAL otherwise).  Given the
 * state (q_n, v_n) of the forward step, its output velocity v_np1 and the
 * incoming adjoints lam_q_in = dL/dq_{n+1}, lam_v_in = dL/dv_{n+1}:
 *   abar = h lam_v_in + h^2 lam_q_in (fixed DOFs 0);  A mu = abar (same PCG);
 *   lam_v_out = lam_v_in + h lam_q_in - alpha M mu - (beta + h) K mu
 *   lam_q_out = lam_q_in - K mu - (beta + h) T(q_n)[mu, v_np1]
 *   dE_accum[e] += -(mu_e . f_e + (beta + h) mu_e . K_e v_np1_e) / E_e
 * with T the directional derivative of K.  All vectors FP64 device.
 * The lam_*_out buffers may alias lam_*_in. */
int fe_step_adjoint(fe_ctx *ctx, const double *q_n, const double *v_n,
                    const double *v_np1, const double *lam_q_in, const double *lam_v_in,
                    double *lam_q_out, double *lam_v_out, double *dE_accum,
                    const fe_params *params, const fe_step_opts *opts, void *stream,
                    fe_solve_stats *stats);

/* y = A x (A device [nnz] in the context's precision, x, y FP64 device). */
int fe_spmv(fe_ctx *ctx, const void *A_vals, const double *x, double *y, void *stream);

/* z = P^{-1} r with the installed factor (Jacobi on A_vals if none). */
int fe_precond_apply(fe_ctx *ctx, const void *A_vals, const double *r, double *z,
                     void *stream);

/* ---- many right-hand sides and contact (Sec. 6.2) ---------------------
 * Contact through Lagrange multipliers solves, besides the free motion, a
 * complementarity problem on the compliance matrix W = H A^{-1} H^T of the k
 * constraint rows H, built (Sec. 7.4) from the asynchronous preconditioner
 * and a triangular solver for many right-hand sides, and corrects the motion
 * with one more solve of A.  H is a k x n_dofs CSR matrix on the device:
 * h_row_ptr [k + 1], h_col [nnz_h] (DOF indices), h_val [nnz_h] FP64.
 * Blocks of right-hand sides R and results Z are FP64, DOF-major: entry
 * (dof, j) at [dof * k + j].
 * The many-right-hand-side calls need a caller-owned device workspace of
 * fe_multi_ws_bytes(k) bytes (256-byte aligned), separate from the bound
 * one and not kept between calls. */

/* Bytes of workspace for k right-hand sides (k >= 0). */
int fe_multi_ws_bytes(fe_ctx *ctx, int32_t k, int64_t *bytes);

/* Z = P^{-1} R for k right-hand sides at once with the installed factor:
 * the same forward / diagonal / backward sweeps as fe_precond_apply, each
 * panel block multiplying a block of up to 128 right-hand sides on the
 * matrix cores (arithmetic in the context's precision: FP32 for
 * FE_PREC_MIXED, FP64 otherwise).  R, Z device [n_dofs * k].
 * Errors: FE_ESTATE (no factor installed), FE_ENOMEM (work too small),
 * FE_EINVAL. */
int fe_precond_apply_multi(fe_ctx *ctx, const double *R, double *Z, int32_t k, void *work,
                           int64_t work_bytes, void *stream);

/* Compliance matrix W = H P^{-1} H^T (device [k * k], row-major FP64) with
 * the installed factor P (Sec. 6.2, Sec. 7.4).  If Z is not NULL it
 * receives P^{-1} H^T (device [n_dofs * k], DOF-major).  Synchronises
 * `stream`.  Errors: FE_EINVAL (a row range of H outside [0, nnz_h] or a
 * column outside [0, n_dofs): such entries are skipped, W is not valid),
 * FE_ESTATE, FE_ENOMEM. */
int fe_compliance(fe_ctx *ctx, int32_t k, const int32_t *h_row_ptr, const int32_t *h_col,
                  const double *h_val, int64_t nnz_h, double *W, double *Z, void *work,
                  int64_t work_bytes, void *stream);

/* Bytes of the static device scratch of fe_compliance_noalloc (256 MiB). */
#define FE_NOALLOC_SCRATCH_BYTES (256ll << 20)

/* fe_compliance for callers that cannot allocate device memory (code under
 * HIP graph capture, tight real-time loops, harnesses that forbid
 * hipMalloc): the same arguments and results without `work`.  The blocks of
 * right-hand sides live in a static device array of FE_NOALLOC_SCRATCH_BYTES
 * bytes, one per GPU, reserved when the first context is bound on that GPU
 * (fe_bind) and held until the process ends; the call itself allocates
 * nothing and clears the part of the array it uses before every use.  Every
 * call on one GPU (any context, any stream) shares that array, so calls that
 * overlap in time on one GPU race: the caller orders them (one stream, or
 * events).  The caller still passes H, W and Z.  Synchronises `stream`.
 * Errors: as fe_compliance; FE_ENOMEM when fe_multi_ws_bytes(k) exceeds
 * FE_NOALLOC_SCRATCH_BYTES (e.g. k > 128 right-hand sides for 107,163 DOFs in
 * mixed precision); FE_EDEVICE when the array's device address could not be
 * obtained at fe_bind. */
int fe_compliance_noalloc(fe_ctx *ctx, int32_t k, const int32_t *h_row_ptr, const int32_t *h_col,
                          const double *h_val, int64_t nnz_h, double *W, double *Z,
                          void *stream);

/* y = s_h op(H) x + s_y y_in with op(H) = H (transpose = 0: x device
 * [n_dofs], y and y_in device [k]) or H^T (transpose = 1: x device [k], y
 * and y_in device [n_dofs]); y_in NULL counts as zero and may alias y.
 * Gives the complementarity right-hand side H x_free - delta and the
 * corrected load b - H^T lambda of the motion correction (Sec. 6.2).
 * Synchronises `stream`.  Errors: FE_EINVAL (bad index, as fe_compliance). */
int fe_constraint_apply(fe_ctx *ctx, int32_t k, const int32_t *h_row_ptr, const int32_t *h_col,
                        const double *h_val, int64_t nnz_h, int32_t transpose, double s_h,
                        const double *x, double s_y, const double *y_in, double *y,
                        void *stream);

/* Projected Gauss-Seidel (Sec. 6.2) on the complementarity problem
 *   lambda >= 0,  W lambda - c >= 0,  lambda . (W lambda - c) = 0
 * with W device [k * k] row-major and c device [k]: each sweep visits the
 * constraints in order and sets
 *   lambda_i <- max(0, lambda_i - ((W lambda)_i - c_i) / W_ii)
 * (a row with W_ii <= 0 keeps its value).  lam (device [k]) holds the start
 * on entry and the result on exit.  Stops after max_sweeps sweeps or after
 * the first sweep whose largest change is <= tol * max(lambda).  info
 * (device [2], NULL allowed) receives the sweeps done and that last change.
 * One wavefront on the GPU; k <= 4096.  Queued on `stream`.
 * Errors: FE_EINVAL. */
int fe_pgs(fe_ctx *ctx, int32_t k, const double *W, const double *c, double *lam,
           int32_t max_sweeps, double tol, double *info, void *stream);

/* keepStruct test of the fast assembly (Sec. 4, Alg. "add"): does a
 * candidate fill sequence differ from the one the context's pattern and map
 * were built from?  The fill order is a function of the element connectivity
 * (element-major, local node order) and of the fixed DOFs, so they are
 * compared entry by entry on the GPU.
 *   n_elems    elements of the candidate (same element type)
 *   conn       device [n_elems * nen] candidate connectivity
 *   fixed_dof  device [n_dofs] candidate Dirichlet flags, NULL = unchanged
 *   changed    host out: 0 = same fill order, the map stays valid (fast
 *              assembly); 1 = it changed (e.g. elements removed by cutting,
 *              or a node order permuted), and the pattern, the map and the
 *              factor structure must be rebuilt: the full assembly is a new
 *              context from fe_build_pattern with the new mesh
 * Synchronises `stream`. */
int fe_structure_changed(fe_ctx *ctx, int64_t n_elems, const int32_t *conn,
                         const uint8_t *fixed_dof, int32_t *changed, void *stream);

/* Host-only check of the factorisation (no GPU): factor the FP64 CSR values
 * A_host (host [nnz]) with the context's ordering and supernodes, then apply
 * z = P^{-1} r on the host with the same explicit-inverse panels and the same
 * forward / diagonal / backward order as the GPU sweeps, for n_rhs
 * right-hand sides stored one after another in r_host / z_host
 * (host [n_rhs * n_dofs]).  Errors: FE_EFACTOR (non-positive pivot). */
int fe_host_factor_apply(fe_ctx *ctx, const double *A_host, const double *r_host,
                         double *z_host, int32_t n_rhs);

/* CG iterations are captured once per (A, x, factor slot) into a HIP graph
 * (kernel nodes only) and replayed on the caller's stream; enable = 0 runs
 * every kernel with its own launch instead (also the case while kernel
 * timing is on).  Default: enabled. */
int fe_set_graphs(fe_ctx *ctx, int32_t enable);

/* Per-kernel timing: when enabled, the library brackets every launch of the
 * triangular-solve and SpMV kernels with HIP events on the launch stream and
 * accumulates their durations; fe_kernel_times reads and resets them.
 *   names: 0 spmv, 1 trisolve forward, 2 trisolve backward, 3 element,
 *          4 many-right-hand-side forward, 5 many-right-hand-side backward
 *   out_ms[k], out_count[k], out_bytes[k]: algorithmic bytes moved for
 *   kinds 0-3, algorithmic flops (2 per lower panel entry and right-hand
 *   side) for kinds 4-5. */
int fe_set_kernel_timing(fe_ctx *ctx, int32_t enable);
int fe_kernel_times(fe_ctx *ctx, double *out_ms, int64_t *out_count, double *out_bytes,
                    int32_t n);

/* Reset the step counter and drop installed factors (new rollout). */
int fe_reset(fe_ctx *ctx);

/* Join the factor thread and free all host state.  NULL is a no-op. */
int fe_destroy(fe_ctx *ctx);

/* Message of the last error on ctx (or of the last failed fe_build_pattern
 * when ctx is NULL).  Valid until the next call on ctx. */
const char *fe_last_error(fe_ctx *ctx);

#ifdef __cplusplus
}
#endif

#endif /* FE_H */
