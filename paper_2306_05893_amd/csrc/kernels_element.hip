// Element kernels: hyperelastic tangent, internal force and consistent mass
// per element, combined into A_e = (1 + h alpha) M_e + h (beta + h) K_e and
// b_e = M_e g - f_e - alpha M_e v_e - (beta + h) K_e v_e, and scattered into
// the CSR values of A and the FP64 vector b through the element map (paper
// Sec. 3.2 Eq. "dynamic equation2", Sec. 4.2 fast assembly with the LHS and
// RHS merged in one pass over the map).
//
// Mapping to the CDNA wavefront:
//   HEX8: one 64-lane wavefront per hexahedron; lane = (a, b) node pair holds
//         the 3x3 block K_ab.  Lanes 0..7 each set up one of the 8 Gauss
//         points (shape gradients, deformation, stress) into LDS; every lane
//         then accumulates its block over the Gauss points.  The force term
//         is spread over the lanes (lane (a, b) takes Gauss point b), and the
//         right-hand side of node a is reduced over its 8 lanes by shuffles.
//   TET4: 16 lanes per tetrahedron (4 per wavefront), lane = (a, b).
// Accuracy in FP32: the stress is formed from the displacement gradient
// H = grad u rather than from F = I + H, i.e. E = (H + H^T + H^T H)/2 and
// J - 1 = tr H + ((tr H)^2 - tr H^2)/2 + det H, ln J = log1p(J - 1), and the
// neo-Hookean P = F^{-T} (2 mu E + lambda ln J I), which equals
// mu (F - F^{-T}) + lambda ln J F^{-T} without the cancellation near rest.
#include "device.hpp"

namespace fe {

namespace {

__constant__ double c_hex_sign[8][3] = {
    {-1, -1, -1}, {1, -1, -1}, {1, 1, -1}, {-1, 1, -1},
    {-1, -1, 1},  {1, -1, 1},  {1, 1, 1},  {-1, 1, 1}};

template <typename T>
__device__ inline T det3(const T *M) {
  return M[0] * (M[4] * M[8] - M[5] * M[7]) - M[1] * (M[3] * M[8] - M[5] * M[6]) +
         M[2] * (M[3] * M[7] - M[4] * M[6]);
}

// inverse of a 3x3 row-major matrix with known determinant
template <typename T>
__device__ inline void inv3(const T *M, T det, T *R) {
  const T id = T(1) / det;
  R[0] = (M[4] * M[8] - M[5] * M[7]) * id;
  R[1] = (M[2] * M[7] - M[1] * M[8]) * id;
  R[2] = (M[1] * M[5] - M[2] * M[4]) * id;
  R[3] = (M[5] * M[6] - M[3] * M[8]) * id;
  R[4] = (M[0] * M[8] - M[2] * M[6]) * id;
  R[5] = (M[2] * M[3] - M[0] * M[5]) * id;
  R[6] = (M[3] * M[7] - M[4] * M[6]) * id;
  R[7] = (M[1] * M[6] - M[0] * M[7]) * id;
  R[8] = (M[0] * M[4] - M[1] * M[3]) * id;
}

template <typename T>
__device__ inline T log1p_t(T x);
template <>
__device__ inline float log1p_t<float>(float x) { return log1pf(x); }
template <>
__device__ inline double log1p_t<double>(double x) { return log1p(x); }

// Quantities of one quadrature point from H = grad u (row-major 3x3).
// Outputs (all pre-multiplied by the volume weight dV):
//   P[9]       first Piola stress * dV
//   NH:   vec = F^{-T} (left-multiplies g to give h), c[0] = mu dV,
//         c[1] = lambda dV, c[2] = (mu - lambda ln J) dV
//   StVK: vec = F, S[9] = S dV, FF[9] = mu dV F F^T, c[0] = lambda dV,
//         c[1] = mu dV
// Returns J (or <= 0 on inversion).
template <typename T, int MAT>
__device__ inline T material_point(const T *H, T mu, T lam, T dV, T *P, T *vec, T *S, T *FF,
                                   T *c) {
  T Eg[9];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      T hh = 0;
      for (int k = 0; k < 3; ++k) hh += H[k * 3 + i] * H[k * 3 + j];
      Eg[i * 3 + j] = T(0.5) * (H[i * 3 + j] + H[j * 3 + i] + hh);
    }
  const T trH = H[0] + H[4] + H[8];
  T trH2 = 0;
  for (int i = 0; i < 3; ++i)
    for (int k = 0; k < 3; ++k) trH2 += H[i * 3 + k] * H[k * 3 + i];
  const T Jm1 = trH + T(0.5) * (trH * trH - trH2) + det3(H);
  const T J = T(1) + Jm1;
  T F[9];
  for (int i = 0; i < 9; ++i) F[i] = H[i];
  F[0] += T(1);
  F[4] += T(1);
  F[8] += T(1);
  if (MAT == 0) {
    if (!(J > T(0))) return J;
    T Fi[9];
    inv3(F, J, Fi);
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) vec[i * 3 + j] = Fi[j * 3 + i];  // F^{-T}
    const T lnJ = log1p_t(Jm1);
    T Sm[9];  // 2 mu E + lambda ln J I
    for (int i = 0; i < 9; ++i) Sm[i] = T(2) * mu * Eg[i];
    Sm[0] += lam * lnJ;
    Sm[4] += lam * lnJ;
    Sm[8] += lam * lnJ;
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) {
        T acc = 0;
        for (int k = 0; k < 3; ++k) acc += vec[i * 3 + k] * Sm[k * 3 + j];
        P[i * 3 + j] = acc * dV;
      }
    c[0] = mu * dV;
    c[1] = lam * dV;
    c[2] = (mu - lam * lnJ) * dV;
  } else {
    const T trE = Eg[0] + Eg[4] + Eg[8];
    T Sm[9];
    for (int i = 0; i < 9; ++i) Sm[i] = T(2) * mu * Eg[i];
    Sm[0] += lam * trE;
    Sm[4] += lam * trE;
    Sm[8] += lam * trE;
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) {
        T acc = Sm[i * 3 + j];  // (I + H) S = S + H S
        for (int k = 0; k < 3; ++k) acc += H[i * 3 + k] * Sm[k * 3 + j];
        P[i * 3 + j] = acc * dV;
        S[i * 3 + j] = Sm[i * 3 + j] * dV;
        vec[i * 3 + j] = F[i * 3 + j];
      }
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) {
        T acc = 0;
        for (int k = 0; k < 3; ++k) acc += F[i * 3 + k] * F[j * 3 + k];
        FF[i * 3 + j] = mu * dV * acc;
      }
    c[0] = lam * dV;
    c[1] = mu * dV;
    c[2] = 0;
  }
  return J;
}

// K_ab contribution of one quadrature point (see oracle formulas):
//   NH:   mu (ga.gb) I + lam ha hb^T + (mu - lam lnJ) hb ha^T,  h = F^{-T} g
//   StVK: (ga^T S gb) I + lam (F ga)(F gb)^T + mu (F gb)(F ga)^T + mu (ga.gb) F F^T
template <typename T, int MAT>
__device__ inline void add_kab(T *K, const T *ga, const T *gb, const T *va, const T *vb,
                               const T *S, const T *FF, const T *c) {
  const T gg = ga[0] * gb[0] + ga[1] * gb[1] + ga[2] * gb[2];
  if (MAT == 0) {
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j)
        K[i * 3 + j] += c[1] * va[i] * vb[j] + c[2] * vb[i] * va[j];
    K[0] += c[0] * gg;
    K[4] += c[0] * gg;
    K[8] += c[0] * gg;
  } else {
    T Sg[3];
    for (int i = 0; i < 3; ++i) Sg[i] = S[i * 3] * gb[0] + S[i * 3 + 1] * gb[1] + S[i * 3 + 2] * gb[2];
    const T gSg = ga[0] * Sg[0] + ga[1] * Sg[1] + ga[2] * Sg[2];
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j)
        K[i * 3 + j] += c[0] * va[i] * vb[j] + c[1] * vb[i] * va[j] + gg * FF[i * 3 + j];
    K[0] += gSg;
    K[4] += gSg;
    K[8] += gSg;
  }
}

template <typename T>
__device__ inline void atomic_add_t(T *p, T v) {
  atomicAdd(p, v);
}

// Scatter the 3x3 block of lane (a, b) and reduce/scatter the RHS of node a.
template <typename T, bool COMPACT, int NEN>
__device__ inline void scatter(int64_t e, int a, int b, int ga, const T *Ablk, const T *rhs,
                               const uint8_t *slot, const int32_t *smap,
                               const int32_t *row_ptr, const uint8_t *dof_fixed, T *A,
                               double *bvec, T *ebuf, double *rbuf) {
  // RHS: sum over the NEN lanes that share node a (consecutive lanes)
  double r3[3] = {(double)rhs[0], (double)rhs[1], (double)rhs[2]};
  for (int off = 1; off < NEN; off <<= 1)
    for (int r = 0; r < 3; ++r) r3[r] += __shfl_xor(r3[r], off, NEN);
  if (COMPACT) {
    // contribution buffers, summed per node block by the gather kernel
    T *dst = ebuf + (e * (NEN * NEN) + a * NEN + b) * 9;
    for (int k = 0; k < 9; ++k) dst[k] = Ablk[k];
    if (b == 0)
      for (int r = 0; r < 3; ++r) rbuf[(e * NEN + a) * 3 + r] = r3[r];
  } else {
    if (b == 0)
      for (int r = 0; r < 3; ++r) {
        const int dof = 3 * ga + r;
        if (!dof_fixed[dof]) atomicAdd(bvec + dof, r3[r]);
      }
    const int ne = 3 * NEN;
    const int32_t *m = smap + e * (int64_t)(ne * ne);
    for (int r = 0; r < 3; ++r)
      for (int c = 0; c < 3; ++c) {
        const int32_t k = m[(3 * a + r) * ne + 3 * b + c];
        if (k >= 0) atomic_add_t(A + k, Ablk[r * 3 + c]);
      }
  }
}

// ------------------------------------------------------------------ HEX8
template <typename T, int MAT, bool COMPACT>
__global__ __launch_bounds__(256) void k_elem_hex(
    int64_t n_elems, const int32_t *__restrict__ conn, const uint8_t *__restrict__ slot,
    const int32_t *__restrict__ smap, const int32_t *__restrict__ row_ptr,
    const double *__restrict__ X, const double *__restrict__ q, const double *__restrict__ v,
    const double *__restrict__ Ev, const uint8_t *__restrict__ dof_fixed, ElemParams prm,
    T *__restrict__ A, double *__restrict__ bvec, T *__restrict__ ebuf,
    double *__restrict__ rbuf, PcgState *state) {
  constexpr int NW = 4;
  __shared__ T s_x[NW][8][3], s_u[NW][8][3], s_v[NW][8][3];
  __shared__ T s_g[NW][8][8][3], s_h[NW][8][8][3];
  __shared__ T s_P[NW][8][9], s_S[NW][8][9], s_FF[NW][8][9], s_c[NW][8][4];
  __shared__ int s_node[NW][8];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int64_t e = (int64_t)blockIdx.x * NW + w;
  const bool valid = e < n_elems;
  const int a = lane >> 3, b = lane & 7;

  if (valid && lane < 8) {
    const int nd = conn[e * 8 + lane];
    const int n0 = conn[e * 8];
    s_node[w][lane] = nd;
    for (int i = 0; i < 3; ++i) {
      s_x[w][lane][i] = (T)(X[3 * nd + i] - X[3 * n0 + i]);
      s_u[w][lane][i] = (T)(q[3 * nd + i] - X[3 * nd + i]);
      s_v[w][lane][i] = (T)v[3 * nd + i];
    }
  }
  __syncthreads();
  T Ee = valid ? (T)Ev[e] : T(0);
  const T nu = (T)prm.nu;
  const T mu = Ee / (T(2) * (T(1) + nu));
  const T lam = Ee * nu / ((T(1) + nu) * (T(1) - T(2) * nu));
  const T g1 = T(0.57735026918962576451);  // 1/sqrt(3)
  if (valid && lane < 8) {
    const int gp = lane;
    const T xi[3] = {(gp & 1) ? g1 : -g1, (gp & 2) ? g1 : -g1, (gp & 4) ? g1 : -g1};
    T dN[8][3];
    for (int n = 0; n < 8; ++n) {
      const T s0 = (T)c_hex_sign[n][0], s1 = (T)c_hex_sign[n][1], s2 = (T)c_hex_sign[n][2];
      const T t0 = T(1) + s0 * xi[0], t1 = T(1) + s1 * xi[1], t2 = T(1) + s2 * xi[2];
      dN[n][0] = T(0.125) * s0 * t1 * t2;
      dN[n][1] = T(0.125) * s1 * t0 * t2;
      dN[n][2] = T(0.125) * s2 * t0 * t1;
    }
    T J[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    for (int n = 0; n < 8; ++n)
      for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) J[i * 3 + j] += s_x[w][n][i] * dN[n][j];
    const T dJ = det3(J);
    T Ji[9];
    inv3(J, dJ, Ji);
    T H[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    for (int n = 0; n < 8; ++n) {
      T g[3];
      for (int i = 0; i < 3; ++i) g[i] = dN[n][0] * Ji[0 * 3 + i] + dN[n][1] * Ji[1 * 3 + i] + dN[n][2] * Ji[2 * 3 + i];
      for (int i = 0; i < 3; ++i) s_g[w][gp][n][i] = g[i];
      for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) H[i * 3 + j] += s_u[w][n][i] * g[j];
    }
    T P[9], vec[9], S[9], FF[9], c[3];
    const T Jf = material_point<T, MAT>(H, mu, lam, dJ, P, vec, S, FF, c);
    if (!(dJ > T(0)) || !(Jf > T(0))) atomicOr(&state->elem_status, 1);
    for (int i = 0; i < 9; ++i) {
      s_P[w][gp][i] = P[i];
      s_S[w][gp][i] = S[i];
      s_FF[w][gp][i] = FF[i];
    }
    s_c[w][gp][0] = c[0];
    s_c[w][gp][1] = c[1];
    s_c[w][gp][2] = c[2];
    s_c[w][gp][3] = dJ;
    for (int n = 0; n < 8; ++n)
      for (int i = 0; i < 3; ++i) {
        const T *gg = s_g[w][gp][n];
        s_h[w][gp][n][i] = vec[i * 3] * gg[0] + vec[i * 3 + 1] * gg[1] + vec[i * 3 + 2] * gg[2];
      }
  }
  __syncthreads();
  if (!valid) return;

  T K[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
  T Mab = 0;
  const T rho = (T)prm.rho;
  for (int gp = 0; gp < 8; ++gp) {
    add_kab<T, MAT>(K, s_g[w][gp][a], s_g[w][gp][b], s_h[w][gp][a], s_h[w][gp][b], s_S[w][gp],
                    s_FF[w][gp], s_c[w][gp]);
    const T xi0 = (gp & 1) ? g1 : -g1, xi1 = (gp & 2) ? g1 : -g1, xi2 = (gp & 4) ? g1 : -g1;
    const T Na = T(0.125) * (T(1) + (T)c_hex_sign[a][0] * xi0) * (T(1) + (T)c_hex_sign[a][1] * xi1) *
                 (T(1) + (T)c_hex_sign[a][2] * xi2);
    const T Nb = T(0.125) * (T(1) + (T)c_hex_sign[b][0] * xi0) * (T(1) + (T)c_hex_sign[b][1] * xi1) *
                 (T(1) + (T)c_hex_sign[b][2] * xi2);
    Mab += rho * Na * Nb * s_c[w][gp][3];
  }
  // force share: Gauss point b of node a
  T fa[3];
  {
    const T *P = s_P[w][b];
    const T *g = s_g[w][b][a];
    for (int i = 0; i < 3; ++i) fa[i] = P[i * 3] * g[0] + P[i * 3 + 1] * g[1] + P[i * 3 + 2] * g[2];
  }
  const T h = (T)prm.h, al = (T)prm.alpha, be = (T)prm.beta;
  const T cM = T(1) + h * al, cK = h * (be + h), cKv = be + h;
  const T *vb = s_v[w][b];
  const T grav[3] = {(T)prm.gx, (T)prm.gy, (T)prm.gz};
  T Ablk[9], rhs[3];
  for (int i = 0; i < 3; ++i) {
    T kv = 0;
    for (int j = 0; j < 3; ++j) {
      Ablk[i * 3 + j] = cK * K[i * 3 + j];
      kv += K[i * 3 + j] * vb[j];
    }
    Ablk[i * 4] += cM * Mab;
    rhs[i] = Mab * grav[i] - fa[i] - al * Mab * vb[i] - cKv * kv;
  }
  scatter<T, COMPACT, 8>(e, a, b, s_node[w][a], Ablk, rhs, slot, smap, row_ptr, dof_fixed, A,
                         bvec, ebuf, rbuf);
}

// ------------------------------------------------------------------ TET4
template <typename T, int MAT, bool COMPACT>
__global__ __launch_bounds__(256) void k_elem_tet(
    int64_t n_elems, const int32_t *__restrict__ conn, const uint8_t *__restrict__ slot,
    const int32_t *__restrict__ smap, const int32_t *__restrict__ row_ptr,
    const double *__restrict__ X, const double *__restrict__ q, const double *__restrict__ v,
    const double *__restrict__ Ev, const uint8_t *__restrict__ dof_fixed, ElemParams prm,
    T *__restrict__ A, double *__restrict__ bvec, T *__restrict__ ebuf,
    double *__restrict__ rbuf, PcgState *state) {
  constexpr int NT = 16;  // tets per block
  __shared__ T s_x[NT][4][3], s_u[NT][4][3], s_v[NT][4][3];
  __shared__ int s_node[NT][4];
  const int t = threadIdx.x >> 4, l16 = threadIdx.x & 15;
  const int64_t e = (int64_t)blockIdx.x * NT + t;
  const bool valid = e < n_elems;
  const int a = l16 >> 2, b = l16 & 3;
  if (valid && l16 < 4) {
    const int nd = conn[e * 4 + l16];
    const int n0 = conn[e * 4];
    s_node[t][l16] = nd;
    for (int i = 0; i < 3; ++i) {
      s_x[t][l16][i] = (T)(X[3 * nd + i] - X[3 * n0 + i]);
      s_u[t][l16][i] = (T)(q[3 * nd + i] - X[3 * nd + i]);
      s_v[t][l16][i] = (T)v[3 * nd + i];
    }
  }
  __syncthreads();
  if (!valid) return;
  const T Ee = (T)Ev[e];
  const T nu = (T)prm.nu;
  const T mu = Ee / (T(2) * (T(1) + nu));
  const T lam = Ee * nu / ((T(1) + nu) * (T(1) - T(2) * nu));
  T Dm[9];
  for (int i = 0; i < 3; ++i)
    for (int k = 0; k < 3; ++k) Dm[i * 3 + k] = s_x[t][k + 1][i];
  const T det = det3(Dm);
  T Di[9];
  inv3(Dm, det, Di);
  const T V = det / T(6);
  T g[4][3];
  for (int i = 0; i < 3; ++i) {
    g[1][i] = Di[0 * 3 + i];
    g[2][i] = Di[1 * 3 + i];
    g[3][i] = Di[2 * 3 + i];
    g[0][i] = -(g[1][i] + g[2][i] + g[3][i]);
  }
  T H[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
  for (int n = 0; n < 4; ++n)
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) H[i * 3 + j] += s_u[t][n][i] * g[n][j];
  T P[9], vec[9], S[9], FF[9], c[3];
  const T Jf = material_point<T, MAT>(H, mu, lam, V, P, vec, S, FF, c);
  if ((!(det > T(0)) || !(Jf > T(0))) && b == 0 && a == 0) atomicOr(&state->elem_status, 1);
  T va[3], vbv[3];
  for (int i = 0; i < 3; ++i) {
    va[i] = vec[i * 3] * g[a][0] + vec[i * 3 + 1] * g[a][1] + vec[i * 3 + 2] * g[a][2];
    vbv[i] = vec[i * 3] * g[b][0] + vec[i * 3 + 1] * g[b][1] + vec[i * 3 + 2] * g[b][2];
  }
  T K[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
  add_kab<T, MAT>(K, g[a], g[b], va, vbv, S, FF, c);
  const T Mab = (T)prm.rho * V * (a == b ? T(2) : T(1)) / T(20);
  T fa[3];
  for (int i = 0; i < 3; ++i)
    fa[i] = T(0.25) * (P[i * 3] * g[a][0] + P[i * 3 + 1] * g[a][1] + P[i * 3 + 2] * g[a][2]);
  const T h = (T)prm.h, al = (T)prm.alpha, be = (T)prm.beta;
  const T cM = T(1) + h * al, cK = h * (be + h), cKv = be + h;
  const T *vb = s_v[t][b];
  const T grav[3] = {(T)prm.gx, (T)prm.gy, (T)prm.gz};
  T Ablk[9], rhs[3];
  for (int i = 0; i < 3; ++i) {
    T kv = 0;
    for (int j = 0; j < 3; ++j) {
      Ablk[i * 3 + j] = cK * K[i * 3 + j];
      kv += K[i * 3 + j] * vb[j];
    }
    Ablk[i * 4] += cM * Mab;
    rhs[i] = Mab * grav[i] - fa[i] - al * Mab * vb[i] - cKv * kv;
  }
  scatter<T, COMPACT, 4>(e, a, b, s_node[t][a], Ablk, rhs, slot, smap, row_ptr, dof_fixed, A,
                         bvec, ebuf, rbuf);
}

template <typename T>
__global__ void k_assembly_init(int64_t nnz, T *A, int64_t n_fixed, const int32_t *fds,
                                int64_t n, double *b, const double *f_nodal,
                                const uint8_t *dof_fixed) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < nnz; k += stride) A[k] = T(0);
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += stride)
    b[k] = dof_fixed[k] ? 0.0 : (f_nodal ? f_nodal[k] : 0.0);
}

// One thread per node block: A entries (r, c) at blk_pos + r * L + c, L =
// the row length of the row node (its three rows share one column set).
template <typename T, int NEN>
__global__ void k_assembly_gather(int64_t n_blocks, const int32_t *__restrict__ blk_ptr,
                                  const int32_t *__restrict__ blk_src,
                                  const int32_t *__restrict__ blk_pos,
                                  const int32_t *__restrict__ blk_node,
                                  const int32_t *__restrict__ row_ptr, const T *__restrict__ ebuf,
                                  const double *__restrict__ rbuf,
                                  const double *__restrict__ f_nodal, T *__restrict__ A,
                                  double *__restrict__ b) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n_blocks) return;
  const int32_t info = blk_node[k];
  const int g = info & 0x7fffffff;
  const bool diag = info < 0;
  const int32_t pos = blk_pos[k];
  const int32_t L = row_ptr[3 * g + 1] - row_ptr[3 * g];
  double acc[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
  double br[3] = {0, 0, 0};
  for (int32_t j = blk_ptr[k]; j < blk_ptr[k + 1]; ++j) {
    const int32_t src = blk_src[j];
    const T *eb = ebuf + (int64_t)src * 9;
#pragma unroll
    for (int q = 0; q < 9; ++q) acc[q] += (double)eb[q];
    if (diag) {
      // src = e * NEN^2 + a * NEN + a: the RHS share of node a of element e
      const int64_t ea = (int64_t)(src / (NEN * NEN)) * NEN + (src % (NEN * NEN)) / NEN;
#pragma unroll
      for (int r = 0; r < 3; ++r) br[r] += rbuf[ea * 3 + r];
    }
  }
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int c = 0; c < 3; ++c) A[pos + r * L + c] = (T)acc[r * 3 + c];
  if (diag)
#pragma unroll
    for (int r = 0; r < 3; ++r) b[3 * g + r] = (f_nodal ? f_nodal[3 * g + r] : 0.0) + br[r];
}

template <typename T>
__global__ void k_set_fixed_diag(int64_t n_fixed, const int32_t *fds, T *A) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n_fixed) A[fds[k]] = T(1);
}

}  // namespace

template <typename T>
void launch_assembly_init(hipStream_t st, int64_t nnz, T *A, int64_t n_fixed,
                          const int32_t *fds, int64_t n, double *b, const double *f_nodal,
                          const uint8_t *dof_fixed, bool zero_A) {
  if (!zero_A) nnz = 0;  // every free-row entry is written by the gather
  const int64_t work = nnz > n ? nnz : n;
  int64_t blocks = (work + 255) / 256;
  if (blocks > 8192) blocks = 8192;
  k_assembly_init<T><<<(unsigned)blocks, 256, 0, st>>>(nnz, A, n_fixed, fds, n, b, f_nodal, dof_fixed);
  if (n_fixed > 0)
    k_set_fixed_diag<T><<<(unsigned)((n_fixed + 255) / 256), 256, 0, st>>>(n_fixed, fds, A);
}

template <typename T>
void launch_element(hipStream_t st, int elem_type, int64_t n_elems, const int32_t *conn,
                    const uint8_t *slot, const int32_t *smap, const int32_t *row_ptr,
                    const double *X, const double *q, const double *v, const double *E,
                    const uint8_t *dof_fixed, const ElemParams &prm, T *A, double *b,
                    T *ebuf, double *rbuf, PcgState *state) {
  if (n_elems <= 0) return;
  const bool compact = slot != nullptr;
  if (elem_type == 8) {
    const unsigned blocks = (unsigned)((n_elems + 3) / 4);
#define FE_HEX(MAT, CMP)                                                                    \
  k_elem_hex<T, MAT, CMP><<<blocks, 256, 0, st>>>(n_elems, conn, slot, smap, row_ptr, X, q, \
                                                   v, E, dof_fixed, prm, A, b, ebuf, rbuf, state)
    if (prm.material == 0) {
      if (compact) FE_HEX(0, true); else FE_HEX(0, false);
    } else {
      if (compact) FE_HEX(1, true); else FE_HEX(1, false);
    }
#undef FE_HEX
  } else {
    const unsigned blocks = (unsigned)((n_elems + 15) / 16);
#define FE_TET(MAT, CMP)                                                                    \
  k_elem_tet<T, MAT, CMP><<<blocks, 256, 0, st>>>(n_elems, conn, slot, smap, row_ptr, X, q, \
                                                   v, E, dof_fixed, prm, A, b, ebuf, rbuf, state)
    if (prm.material == 0) {
      if (compact) FE_TET(0, true); else FE_TET(0, false);
    } else {
      if (compact) FE_TET(1, true); else FE_TET(1, false);
    }
#undef FE_TET
  }
}

template <typename T>
void launch_assembly_gather(hipStream_t st, int nen, int64_t n_blocks, const int32_t *blk_ptr,
                            const int32_t *blk_src, const int32_t *blk_pos,
                            const int32_t *blk_node, const int32_t *row_ptr, const T *ebuf,
                            const double *rbuf, const double *f_nodal, T *A, double *b) {
  if (n_blocks <= 0) return;
  const unsigned blocks = (unsigned)((n_blocks + 255) / 256);
  if (nen == 8)
    k_assembly_gather<T, 8><<<blocks, 256, 0, st>>>(n_blocks, blk_ptr, blk_src, blk_pos, blk_node,
                                                    row_ptr, ebuf, rbuf, f_nodal, A, b);
  else
    k_assembly_gather<T, 4><<<blocks, 256, 0, st>>>(n_blocks, blk_ptr, blk_src, blk_pos, blk_node,
                                                    row_ptr, ebuf, rbuf, f_nodal, A, b);
}

template void launch_assembly_init<float>(hipStream_t, int64_t, float *, int64_t, const int32_t *,
                                          int64_t, double *, const double *, const uint8_t *,
                                          bool);
template void launch_assembly_init<double>(hipStream_t, int64_t, double *, int64_t,
                                           const int32_t *, int64_t, double *, const double *,
                                           const uint8_t *, bool);
template void launch_assembly_gather<float>(hipStream_t, int, int64_t, const int32_t *,
                                            const int32_t *, const int32_t *, const int32_t *,
                                            const int32_t *, const float *, const double *,
                                            const double *, float *, double *);
template void launch_assembly_gather<double>(hipStream_t, int, int64_t, const int32_t *,
                                             const int32_t *, const int32_t *, const int32_t *,
                                             const int32_t *, const double *, const double *,
                                             const double *, double *, double *);
template void launch_element<float>(hipStream_t, int, int64_t, const int32_t *, const uint8_t *,
                                    const int32_t *, const int32_t *, const double *,
                                    const double *, const double *, const double *,
                                    const uint8_t *, const ElemParams &, float *, double *,
                                    float *, double *, PcgState *);
template void launch_element<double>(hipStream_t, int, int64_t, const int32_t *, const uint8_t *,
                                     const int32_t *, const int32_t *, const double *,
                                     const double *, const double *, const double *,
                                     const uint8_t *, const ElemParams &, double *, double *,
                                     double *, double *, PcgState *);

}  // namespace fe
