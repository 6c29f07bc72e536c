// Rotation of the stale preconditioner (not in the paper; the paper notes
// that the asynchronous preconditioner can be corrected when the system
// changes quickly, Sec. 3.3).  When the body rotates, the tangent follows
// the rotation: for a state q = R x the element energy is unchanged, so
// K(q) = Q K(x) Q^T and M = Q M Q^T with Q = blockdiag(R) per node.  A factor
// of A_{t0} therefore preconditions A_t better as
//   P_t^{-1} = Q A_{t0}^{-1} Q^T,   Q_n = R_n(t) R_n(t0)^T per node,
// with R_n the rotation of the material around node n: the rotation factor
// of the polar decomposition of the sum of the deformation gradients at the
// centres of the elements around the node.  P_t is symmetric positive
// definite whenever A_{t0} is, so the PCG stays a PCG and its results
// (every step meets the same recomputed-residual test) do not change; only
// the iteration count does.  Nodes with a fixed DOF keep Q = I.
#include "device.hpp"

namespace fe {

namespace {

constexpr int kBlock = 256;

__constant__ double c_rot_sign[8][3] = {
    {-1, -1, -1}, {1, -1, -1}, {1, 1, -1}, {-1, 1, -1},
    {-1, -1, 1},  {1, -1, 1},  {1, 1, 1},  {-1, 1, 1}};

__device__ inline double det3d(const double *M) {
  return M[0] * (M[4] * M[8] - M[5] * M[7]) - M[1] * (M[3] * M[8] - M[5] * M[6]) +
         M[2] * (M[3] * M[7] - M[4] * M[6]);
}

// inverse transpose of a 3x3 row-major matrix with determinant d
__device__ inline void inv_t3(const double *M, double d, double *R) {
  const double id = 1.0 / d;
  R[0] = (M[4] * M[8] - M[5] * M[7]) * id;
  R[1] = (M[5] * M[6] - M[3] * M[8]) * id;
  R[2] = (M[3] * M[7] - M[4] * M[6]) * id;
  R[3] = (M[2] * M[7] - M[1] * M[8]) * id;
  R[4] = (M[0] * M[8] - M[2] * M[6]) * id;
  R[5] = (M[1] * M[6] - M[0] * M[7]) * id;
  R[6] = (M[1] * M[5] - M[2] * M[4]) * id;
  R[7] = (M[2] * M[3] - M[0] * M[5]) * id;
  R[8] = (M[0] * M[4] - M[1] * M[3]) * id;
}

// Deformation gradient at the element centre, F = sum_a x_a (x) g_a with g_a
// the rest-configuration gradient of N_a there, one element per thread,
// stored per element (Fe[9 e .. 9 e + 9), row-major).
template <int NEN>
__global__ __launch_bounds__(kBlock) void k_rot_elem(int64_t n_elems,
                                                     const int32_t *__restrict__ conn,
                                                     const double *__restrict__ X,
                                                     const double *__restrict__ q, double *Fe) {
  const int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (e >= n_elems) return;
  int nd[NEN];
#pragma unroll
  for (int a = 0; a < NEN; ++a) nd[a] = conn[e * NEN + a];
  // reference gradients dN_a/dxi at the centre
  double dN[NEN][3];
  if (NEN == 8) {
#pragma unroll
    for (int a = 0; a < 8; ++a)
#pragma unroll
      for (int i = 0; i < 3; ++i) dN[a][i] = 0.125 * c_rot_sign[a][i];
  } else {
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      dN[0][i] = -1.0;
#pragma unroll
      for (int a = 1; a < NEN; ++a) dN[a][i] = (a - 1 == i) ? 1.0 : 0.0;
    }
  }
  // rest Jacobian J = sum_a X_a (x) dN_a, current F~ = sum_a x_a (x) dN_a;
  // F = F~ J^{-1}
  double J[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0}, Fx[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
#pragma unroll
  for (int a = 0; a < NEN; ++a) {
    const int64_t o = 3 * (int64_t)nd[a];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      const double Xi = X[o + i], xi = q[o + i];
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        J[i * 3 + j] += Xi * dN[a][j];
        Fx[i * 3 + j] += xi * dN[a][j];
      }
    }
  }
  double Jit[9];
  inv_t3(J, det3d(J), Jit);  // J^{-T}
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j)
      Fe[9 * e + i * 3 + j] = Fx[i * 3] * Jit[j * 3] + Fx[i * 3 + 1] * Jit[j * 3 + 1] +
                              Fx[i * 3 + 2] * Jit[j * 3 + 2];  // (Fx J^{-1})_{ij}
}

// R_n = rotation factor of the polar decomposition of S_n, the sum of the
// centre deformation gradients of the elements around node n (in ascending
// element order, ne_idx[ne_ptr[n] .. ne_ptr[n + 1])), by the Newton
// iteration R <- (R + R^{-T}) / 2; the identity for nodes with a fixed DOF
// and for nodes whose S_n is singular or inverted.
__global__ __launch_bounds__(kBlock) void k_rot_node(int64_t n_nodes,
                                                     const int32_t *__restrict__ ne_ptr,
                                                     const int32_t *__restrict__ ne_idx,
                                                     const double *__restrict__ Fe,
                                                     const uint8_t *__restrict__ dof_fixed,
                                                     double *Rn) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= n_nodes) return;
  bool ok = !(dof_fixed[3 * i] | dof_fixed[3 * i + 1] | dof_fixed[3 * i + 2]);
  double R[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
  if (ok)
    for (int32_t k = ne_ptr[i]; k < ne_ptr[i + 1]; ++k) {
      const double *f = Fe + 9 * (int64_t)ne_idx[k];
#pragma unroll
      for (int u = 0; u < 9; ++u) R[u] += f[u];
    }
  for (int it = 0; ok && it < 40; ++it) {
    const double d = det3d(R);
    if (!(d > 0.0)) {
      ok = false;
      break;
    }
    double Rit[9];
    inv_t3(R, d, Rit);
    double diff = 0.0;
#pragma unroll
    for (int k = 0; k < 9; ++k) {
      const double rn = 0.5 * (R[k] + Rit[k]);
      diff = fmax(diff, fabs(rn - R[k]));
      R[k] = rn;
    }
    if (diff <= 1e-14) break;
  }
#pragma unroll
  for (int k = 0; k < 9; ++k) Rn[9 * i + k] = ok ? R[k] : ((k % 4 == 0) ? 1.0 : 0.0);
}

__global__ __launch_bounds__(kBlock) void k_rot_identity(int64_t n_nodes, double *R) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i < 9 * n_nodes) R[i] = (i % 9) % 4 == 0 ? 1.0 : 0.0;
}

// Q_n = R_n(t) R_n(t0)^T, stored in the context precision
template <typename T>
__global__ __launch_bounds__(kBlock) void k_rot_q(int64_t n_nodes, const double *__restrict__ Rt,
                                                  const double *__restrict__ R0, T *Q) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= n_nodes) return;
  const double *a = Rt + 9 * i, *b = R0 + 9 * i;
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int c = 0; c < 3; ++c)
      Q[9 * i + 3 * r + c] =
          (T)(a[3 * r] * b[3 * c] + a[3 * r + 1] * b[3 * c + 1] + a[3 * r + 2] * b[3 * c + 2]);
}

// sweep input w = Q^T r per node (the preparation pass has set y = 0 and the
// fixed DOFs, whose Q is the identity)
template <typename T>
__global__ __launch_bounds__(kBlock) void k_rot_in(int64_t n_nodes, const T *__restrict__ Q,
                                                   const double *__restrict__ r, T *w,
                                                   const PcgState *s) {
  if (s && s->done) return;
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= n_nodes) return;
  const T *q = Q + 9 * i;
  const double r0 = r[3 * i], r1 = r[3 * i + 1], r2 = r[3 * i + 2];
#pragma unroll
  for (int c = 0; c < 3; ++c)
    w[3 * i + c] = (T)((double)q[c] * r0 + (double)q[3 + c] * r1 + (double)q[6 + c] * r2);
}

// z = Q z per node, after the backward sweep
template <typename T>
__global__ __launch_bounds__(kBlock) void k_rot_out(int64_t n_nodes, const T *__restrict__ Q,
                                                    double *z, const PcgState *s) {
  if (s && s->done) return;
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= n_nodes) return;
  const T *q = Q + 9 * i;
  const double z0 = z[3 * i], z1 = z[3 * i + 1], z2 = z[3 * i + 2];
#pragma unroll
  for (int r = 0; r < 3; ++r)
    z[3 * i + r] = (double)q[3 * r] * z0 + (double)q[3 * r + 1] * z1 + (double)q[3 * r + 2] * z2;
}

unsigned grid_of(int64_t n) { return (unsigned)((n + kBlock - 1) / kBlock); }

}  // namespace

void launch_node_rotations(hipStream_t st, int elem_type, int64_t n_elems, const int32_t *conn,
                           const double *X, const double *q, int64_t n_nodes,
                           const uint8_t *dof_fixed, const int32_t *ne_ptr,
                           const int32_t *ne_idx, double *Fe, double *Rn) {
  if (n_elems > 0) {
    if (elem_type == 8)
      k_rot_elem<8><<<grid_of(n_elems), kBlock, 0, st>>>(n_elems, conn, X, q, Fe);
    else
      k_rot_elem<4><<<grid_of(n_elems), kBlock, 0, st>>>(n_elems, conn, X, q, Fe);
  }
  if (n_nodes > 0)
    k_rot_node<<<grid_of(n_nodes), kBlock, 0, st>>>(n_nodes, ne_ptr, ne_idx, Fe, dof_fixed, Rn);
}

void launch_rot_identity(hipStream_t st, int64_t n_nodes, double *R) {
  if (n_nodes > 0) k_rot_identity<<<grid_of(9 * n_nodes), kBlock, 0, st>>>(n_nodes, R);
}

template <typename T>
void launch_rot_q(hipStream_t st, int64_t n_nodes, const double *Rt, const double *R0, T *Q) {
  if (n_nodes > 0) k_rot_q<T><<<grid_of(n_nodes), kBlock, 0, st>>>(n_nodes, Rt, R0, Q);
}

template <typename T>
void launch_rot_in(hipStream_t st, int64_t n_nodes, const T *Q, const double *r, T *w,
                   const PcgState *s) {
  if (n_nodes > 0) k_rot_in<T><<<grid_of(n_nodes), kBlock, 0, st>>>(n_nodes, Q, r, w, s);
}

template <typename T>
void launch_rot_out(hipStream_t st, int64_t n_nodes, const T *Q, double *z, const PcgState *s) {
  if (n_nodes > 0) k_rot_out<T><<<grid_of(n_nodes), kBlock, 0, st>>>(n_nodes, Q, z, s);
}

#define FE_INST(T)                                                                           \
  template void launch_rot_q<T>(hipStream_t, int64_t, const double *, const double *, T *);  \
  template void launch_rot_in<T>(hipStream_t, int64_t, const T *, const double *, T *,       \
                                 const PcgState *);                                          \
  template void launch_rot_out<T>(hipStream_t, int64_t, const T *, double *, const PcgState *);
FE_INST(float)
FE_INST(double)
#undef FE_INST

}  // namespace fe
