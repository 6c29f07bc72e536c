// Device-side structures and kernel launchers of the FE step library
// (HIP for gfx950).  Shared by kernels_*.hip and the C-ABI implementation.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>

#include "host.hpp"

namespace fe {

struct SnDev {          // one supernode of the factor, as the GPU sees it
  int32_t nc, m;        // own columns, panel rows
  int64_t panel_off;    // entry offset of the m x nc column-major panel
  int64_t rows_off;     // offset into the rows array (DOF indices)
  int32_t ld, pad;      // leading dimension of the panel (m rounded up to
                        // a multiple of kPanelAlign)
};

// One tile of a triangular sweep with its supernode's fields copied in, so
// that a workgroup's first load (the descriptor) is its only dependent one
// before the index and panel loads.
struct TileDev {
  int64_t panel_off;    // the supernode's panel (entry offset)
  int64_t rows_off;     // its rows (offset into the rows array)
  int32_t nc, m, ld;    // own columns, panel rows, leading dimension
  int32_t r0, c0, pad;  // the tile's first row and column
};

// Control block of one CG solve (device memory, read back by the host).
struct PcgState {
  double rz;            // r . z of the current iterate
  double pAp;
  double rr;            // ||r||^2 (recursive)
  double bb;            // ||b||^2
  double alpha, beta;
  double tol2;          // rel_tol^2 * ||b||^2
  double rr_true;       // recomputed ||b - A x||^2
  int32_t it;           // iterations done
  int32_t done;         // 1: converged candidate / breakdown -> kernels no-op
  int32_t status;       // 0 ok, 4 = p^T A p <= 0
  int32_t elem_status;  // bit 0: an element had det F <= 0 or det J <= 0
};

struct ElemParams {
  double h, alpha, beta, rho, nu;
  double gx, gy, gz;
  int32_t material;     // 0 neo-Hookean, 1 StVK, 2 co-rotational, 3 Mooney-Rivlin
  int32_t pad;
  double mr_c01_share;  // Mooney-Rivlin: share of mu/2 carried by C01
};

// ---------------------------------------------------------------- launchers
// Assembly: A <- 0 with fixed diagonals 1; b <- f_nodal (0 on fixed DOFs).
template <typename T>
void launch_assembly_init(hipStream_t st, int64_t nnz, T *A, int64_t n_fixed,
                          const int32_t *fixed_diag_slot, int64_t n, double *b,
                          const double *f_nodal, const uint8_t *dof_fixed, bool zero_A);

// keepStruct: *flag = 1 if conn differs from ref_conn or (fixed != NULL)
// fixed differs from ref_fixed.
void launch_struct_cmp(hipStream_t st, int64_t n_conn, const int32_t *conn, const int32_t *ref_conn,
                       int64_t n_dofs, const uint8_t *fixed, const uint8_t *ref_fixed,
                       int *flag);

// Element tangents + forces.  With the compact map (slot != NULL) the 3 x 3
// blocks go to ebuf [E][nen*nen][9] and the RHS shares of the nodes to rbuf
// [E][nen][3] (no atomics; launch_assembly_gather sums them into A and b);
// otherwise (smap [E][(3nen)^2]) they are added into A and b with atomics.
template <typename T>
void launch_element(hipStream_t st, int elem_type, int64_t n_elems, const int32_t *conn,
                    const uint8_t *slot, const int32_t *smap, const int32_t *row_ptr,
                    const double *X, const double *q, const double *v, const double *E,
                    const uint8_t *dof_fixed, const ElemParams &prm, T *A, double *b,
                    T *ebuf, double *rbuf, PcgState *state);

// Sum of the element contributions per node block of A (one thread per
// block, contributions in element order) and, on diagonal blocks, of the
// RHS shares of the row node: b = f_nodal + sum.
template <typename T>
void launch_assembly_gather(hipStream_t st, int nen, int64_t n_blocks, const int32_t *blk_ptr,
                            const int32_t *blk_src, const int32_t *blk_pos,
                            const int32_t *blk_node, const int32_t *row_ptr, const T *ebuf,
                            const double *rbuf, const double *f_nodal, T *A, double *b);

// y = A x; if dot_partial != NULL also sum_i w[i] y[i] per block.
template <typename T>
void launch_spmv(hipStream_t st, int64_t n, int rows_per_lanes, const int32_t *row_ptr,
                 const int32_t *col, const T *val, const double *x, double *y,
                 const double *w, double *dot_partial, int *n_partial, const PcgState *state);
int spmv_lanes_for(double avg_row_nnz);

// Triangular sweeps z = P^{-1} r with P = L D L^T in explicit-inverse panels
// (stream: read the panels non-temporally, for a factor larger than the
// last-level cache).
template <typename T>
void launch_tri_prep(hipStream_t st, int64_t n, const double *r, T *w, T *y, double *z,
                     const uint8_t *dof_fixed, const PcgState *state);
template <typename T>
void launch_tri_fwd(hipStream_t st, const TileDev *tiles, int n_tiles,
                    const int32_t *rows, const T *panels, T *w, T *y, const PcgState *state,
                    int tile_cols, int groups, bool stream);
template <typename T>
void launch_tri_bwd(hipStream_t st, const TileDev *tiles, int n_tiles,
                    const int32_t *rows, const T *panels, const T *dinv, const T *y, double *z,
                    const PcgState *state, int tile_rows, int tile_cols, bool stream);

// Many right-hand sides: DOF-major n x ld blocks (ld = k rounded up to the
// tile width bn, 64 or 128), w/y in the factor's precision, z FP64.
template <typename T>
void launch_multi_prep(hipStream_t st, int64_t n, int k, int ld, const double *R, T *w, T *y,
                       double *z, const uint8_t *dof_fixed);
template <typename T>
void launch_multi_zero(hipStream_t st, int64_t total, T *w, T *y, double *z);
void launch_multi_out(hipStream_t st, int64_t n, int k, int ld, const double *z, double *Z);
template <typename T>
void launch_multi_fwd(hipStream_t st, const MTile *tiles, int n_tiles, int n_kb, int bn,
                      const SnDev *sn, const int32_t *rows, const T *panels, T *w, T *y, int ld,
                      int k);
template <typename T>
void launch_multi_bwd(hipStream_t st, const MTile *tiles, int n_tiles, int n_kb, int bn,
                      const SnDev *sn, const int32_t *rows, const T *panels, const T *dinv, T *y,
                      double *z, int ld, int k);
// After each backward level: y <- -z on that level's DOFs (the inputs the
// lower levels read).
template <typename T>
void launch_multi_conv(hipStream_t st, const int32_t *dofs, int64_t cnt, int ld, const double *z,
                       T *y);
// Contact: right-hand sides H^T (w, and z on fixed DOFs; blocks zeroed
// before), W = H Z, y = s_h op(H) x + s_y y_in, projected Gauss-Seidel.  Invalid
// row ranges or column indices of H are skipped and set *err.
template <typename T>
void launch_h_scatter(hipStream_t st, int kc, int64_t n, int64_t nnz_h, const int32_t *hrp,
                      const int32_t *hcol, const double *hval, int ld, T *w, double *z,
                      const uint8_t *dof_fixed, int *err);
void launch_hz(hipStream_t st, int kc, int64_t n, int64_t nnz_h, const int32_t *hrp,
               const int32_t *hcol, const double *hval, int ld, const double *z, double *W);
void launch_h_apply(hipStream_t st, int kc, int64_t n, int64_t nnz_h, const int32_t *hrp,
                    const int32_t *hcol, const double *hval, bool transpose, double s_h,
                    const double *x, double s_y, const double *y_in, double *y, int *err);
int pgs_max_constraints();
void launch_pgs(hipStream_t st, int kc, const double *W, const double *c, double *lam,
                int max_sweeps, double tol, double *info);

// Jacobi: dinv_A[i] = 1 / A_ii ; z = dinv_A * r
template <typename T>
void launch_diag_inv(hipStream_t st, int64_t n, const int32_t *row_ptr, const int32_t *col,
                     const T *val, double *dinv);
void launch_jacobi(hipStream_t st, int64_t n, const double *dinv, const double *r, double *z,
                   const PcgState *state);

// x += alpha p, r -= alpha q with ||r||^2 partials (cg_blocks(n) of them);
// when w != NULL it also writes the sweep inputs w = r, y = 0, z = 0 (r on
// fixed DOFs), replacing the separate preparation pass.
template <typename T>
void launch_update_xr_prep(hipStream_t st, int64_t n, double *x, double *r, const double *p,
                           const double *q, double *part, const PcgState *state, T *w, T *y,
                           double *z, const uint8_t *dof_fixed);

// CG vector kernels (all no-ops once state->done is set).
int cg_blocks(int64_t n);
void launch_residual(hipStream_t st, int64_t n, const double *b, const double *Ax, double *r,
                     double *part_rr, double *part_bb);
void launch_ctl_init(hipStream_t st, PcgState *s, const double *part_rr, const double *part_bb,
                     int np, double rel_tol);
void launch_dot(hipStream_t st, int64_t n, const double *a, const double *b, double *part,
                const PcgState *state);
void launch_ctl_rz(hipStream_t st, PcgState *s, const double *part, int np, int first);
void launch_ctl_alpha(hipStream_t st, PcgState *s, const double *part, int np,
                      double *stage = nullptr);
void launch_ctl_rr(hipStream_t st, PcgState *s, const double *part, int np);
void launch_update_p(hipStream_t st, int64_t n, double *p, const double *z, const PcgState *state,
                     int first);
void launch_ctl_true(hipStream_t st, PcgState *s, const double *part, int np);
void launch_zero(hipStream_t st, int64_t n, double *x);

// Initial guess of a step's CG from the last m (<= kHist) solutions: the
// A-norm projection x = V c, (V^T A V) c = V^T b, with V (n x kHist,
// interleaved: DOF k's values at V[k * kHist + j]) the ring of earlier
// solutions whose newest column is `newest`; W (same shape) receives A V.
// part: hist_part_doubles() doubles of scratch, its last kHist the
// coefficients.  launch_hist_push stores x as column `slot` of V.
constexpr int kHist = 8;
template <typename T>
void launch_hist_guess(hipStream_t st, int64_t n, int m, int newest, const int32_t *row_ptr,
                       const int32_t *col, const T *val, const double *V, double *W,
                       const double *b, double *part, double *coef, double *x);
void launch_hist_push(hipStream_t st, int64_t n, int slot, const double *x, double *V);
int64_t hist_part_doubles();

// Rotation of the stale preconditioner: per-node rotations R_n of state q
// (Fe: 9 FP64 per element, the element-centre deformation gradients; ne_ptr
// / ne_idx: the elements of each node, ascending), the identity,
// Q_n = R_n(t) R_n(t0)^T, and the sweep input w = Q^T r / output z = Q z per
// node.
void launch_node_rotations(hipStream_t st, int elem_type, int64_t n_elems, const int32_t *conn,
                           const double *X, const double *q, int64_t n_nodes,
                           const uint8_t *dof_fixed, const int32_t *ne_ptr,
                           const int32_t *ne_idx, double *Fe, double *Rn);
void launch_rot_identity(hipStream_t st, int64_t n_nodes, double *R);
template <typename T>
void launch_rot_q(hipStream_t st, int64_t n_nodes, const double *Rt, const double *R0, T *Q);
template <typename T>
void launch_rot_in(hipStream_t st, int64_t n_nodes, const T *Q, const double *r, T *w,
                   const PcgState *s);
template <typename T>
void launch_rot_out(hipStream_t st, int64_t n_nodes, const T *Q, double *z, const PcgState *s);
void launch_integrate(hipStream_t st, int64_t n, double h, const double *a, double *q,
                      double *v);

// GPU factorisation: device copies of the GfPlan arrays plus the front store.
struct GfDev {
  const GfFront *fr;
  const int32_t *lvl_sn, *a_csr;
  const int64_t *a_off;
  const int32_t *parent, *rel;
  const int64_t *rel_off;
  const GfExt *ext;
  const int32_t *panel_sn;
  const GfTile *upd;
  const int32_t *rows;
  double *fronts;
  int *status;          // bit 0: non-positive pivot met
  int max_blocks;       // bound on the workgroups of one launch (0: none)
};
// FP64 multifrontal LDL^T of A (values TA) -> explicit-inverse panels and
// 1/d (T), queued on st.  The plan's host arrays drive the launch sequence.
template <typename TA, typename T>
void launch_gpu_factor(hipStream_t st, const GfPlan &P, const GfDev &d, const TA *A, T *panels,
                       T *dinv);

// Adjoint element pass: lam_q_out, lam_v_out, dE (see fe.h fe_step_adjoint)
template <typename T>
void launch_adjoint_element(hipStream_t st, int elem_type, int64_t n_elems,
                            const int32_t *conn, const double *X, const double *q,
                            const double *mu, const double *vnp1, const double *E,
                            const ElemParams &prm, double *Kmu, double *Mmu, double *Tmv,
                            double *dE);
void launch_adjoint_combine(hipStream_t st, int64_t n, double h, double alpha, double beta,
                            const double *lq_in, const double *lv_in, const double *Kmu,
                            const double *Mmu, const double *Tmv, double *lq_out,
                            double *lv_out);
void launch_abar(hipStream_t st, int64_t n, double h, const double *lq, const double *lv,
                 const uint8_t *dof_fixed, double *abar);

}  // namespace fe
