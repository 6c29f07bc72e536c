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

// Index of block (a, b), a <= b, among the upper-triangle blocks of an
// element taken row by row.
template <int NEN>
__host__ __device__ constexpr int sym_block(int a, int b) {
  return a * NEN - a * (a - 1) / 2 + (b - a);
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
    // contribution buffers, summed per node block by the gather kernel.  A_e
    // is symmetric (block (b, a) is the transpose of block (a, b)), so only
    // the blocks a <= b are kept, in the row-major upper-triangle order of
    // sym_block
    if (a <= b) {
      T *dst = ebuf + (e * (NEN * (NEN + 1) / 2) + sym_block<NEN>(a, b)) * 9;
      for (int k = 0; k < 9; ++k) dst[k] = Ablk[k];
    }
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
// Cross-lane moves inside rows of 8 lanes (DPP; 64-bit values as two 32-bit
// moves).  CTRL: 0xB1 quad_perm [1,0,3,2], 0x4E quad_perm [2,3,0,1], 0x141
// row_half_mirror (lane i <- lane 7 - i within each group of 8).
template <int CTRL>
__device__ inline float dpp_mov(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, false));
}
template <int CTRL>
__device__ inline double dpp_mov(double v) {
  const long long x = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)x, CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(x >> 32), CTRL, 0xF, 0xF, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Sum over the 8 lanes of each aligned group of 8 (every lane of the group
// receives the sum): two quad exchanges, then the other half of the group.
template <typename T>
__device__ inline T sum8(T v) {
  v += dpp_mov<0xB1>(v);
  v += dpp_mov<0x4E>(v);
  v += dpp_mov<0x141>(v);
  return v;
}

// Trilinear shape function N_n at Gauss point gp (both 0..7, the corner and
// point sign patterns of c_hex_sign): 1/8 (1 + g)^k (1 - g)^(3-k) with
// g = 1/sqrt(3) and k the number of coordinates whose signs agree.
__constant__ double c_hex_N[4] = {
    0.125 * 0.42264973081037427 * 0.42264973081037427 * 0.42264973081037427,
    0.125 * 0.42264973081037427 * 0.42264973081037427 * 1.57735026918962573,
    0.125 * 0.42264973081037427 * 1.57735026918962573 * 1.57735026918962573,
    0.125 * 1.57735026918962573 * 1.57735026918962573 * 1.57735026918962573};

__device__ inline int hex_agree(int n, int gp) {
  // corner n and point gp share the bit pattern of their sign triples up to
  // the VTK ordering of the corners: c_hex_sign[n] in bits (x: bit 0 of
  // ((n ^ (n >> 1)) & 1), y: bit 1 of n, z: bit 2 of n)
  const int cx = (n ^ (n >> 1)) & 1, cy = (n >> 1) & 1, cz = (n >> 2) & 1;
  const int px = gp & 1, py = (gp >> 1) & 1, pz = (gp >> 2) & 1;
  return (cx == px) + (cy == py) + (cz == pz);
}

// One wavefront per hexahedron, 4 per workgroup.
//  set-up: lane (gp, n) = (lane / 8, lane % 8) takes node n at Gauss point
//    gp: its shape-function gradient dN_n, its share x_n (x) dN_n of the
//    Jacobian and u_n (x) g_n of H = grad u, both summed over the 8 lanes of
//    the point by DPP; the 8 lanes of a point then evaluate the material
//    point (the same values in each) and write g_n, h_n and the point's
//    stress data to LDS;
//  blocks: lane (a, b) accumulates the 3x3 block K_ab and M_ab over the 8
//    points, takes the force share of point b on node a, and forms its
//    blocks of A_e and b_e.  Node b's velocity is the one the lane loaded in
//    the set-up (same b).
template <typename T, int MAT, bool COMPACT>
__global__ __launch_bounds__(256) void k_elem_hex(
    int64_t n_elems, const int32_t *__restrict__ conn, const uint8_t *__restrict__ slot,
    const int32_t *__restrict__ smap, const int32_t *__restrict__ row_ptr,
    const double *__restrict__ X, const double *__restrict__ q, const double *__restrict__ v,
    const double *__restrict__ Ev, const uint8_t *__restrict__ dof_fixed, ElemParams prm,
    T *__restrict__ A, double *__restrict__ bvec, T *__restrict__ ebuf,
    double *__restrict__ rbuf, PcgState *state) {
  constexpr int NW = 4;
  __shared__ T s_g[NW][8][8][3], s_h[NW][8][8][3];
  __shared__ T s_P[NW][8][9], s_S[NW][8][9], s_FF[NW][8][9], s_c[NW][8][4];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int64_t e = (int64_t)blockIdx.x * NW + w;
  const bool valid = e < n_elems;
  const int a = lane >> 3, b = lane & 7;
  const int64_t ec = valid ? e : 0;  // clamped: every lane runs the set-up

  // node b of the element (lane (gp, n = b))
  const int nd = conn[ec * 8 + b];
  const int n0 = conn[ec * 8];
  T xr[3], u[3], vb[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    const double Xi = X[3 * nd + i];
    xr[i] = (T)(Xi - X[3 * n0 + i]);
    u[i] = (T)(q[3 * nd + i] - Xi);
    vb[i] = (T)v[3 * nd + i];
  }
  const T Ee = (T)Ev[ec];
  const T nu = (T)prm.nu;
  const T mu = Ee / (T(2) * (T(1) + nu));
  const T lam = Ee * nu / ((T(1) + nu) * (T(1) - T(2) * nu));
  const T g1 = T(0.57735026918962576451);  // 1/sqrt(3)
  {
    const int gp = a, n = b;
    const T xi[3] = {(gp & 1) ? g1 : -g1, (gp & 2) ? g1 : -g1, (gp & 4) ? g1 : -g1};
    const T s0 = (T)c_hex_sign[n][0], s1 = (T)c_hex_sign[n][1], s2 = (T)c_hex_sign[n][2];
    const T t0 = T(1) + s0 * xi[0], t1 = T(1) + s1 * xi[1], t2 = T(1) + s2 * xi[2];
    const T dN[3] = {T(0.125) * s0 * t1 * t2, T(0.125) * s1 * t0 * t2, T(0.125) * s2 * t0 * t1};
    T J[9];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j) J[i * 3 + j] = sum8(xr[i] * dN[j]);
    const T dJ = det3(J);
    T Ji[9];
    inv3(J, dJ, Ji);
    T g[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) g[i] = dN[0] * Ji[0 * 3 + i] + dN[1] * Ji[1 * 3 + i] + dN[2] * Ji[2 * 3 + i];
    T H[9];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j) H[i * 3 + j] = sum8(u[i] * g[j]);
    T P[9], vec[9], S[9], FF[9], c[3];
    const T Jf = material_point<T, MAT>(H, mu, lam, dJ, P, vec, S, FF, c);
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      s_g[w][gp][n][i] = g[i];
      s_h[w][gp][n][i] = vec[i * 3] * g[0] + vec[i * 3 + 1] * g[1] + vec[i * 3 + 2] * g[2];
    }
    if (n == 0) {
      if (valid && (!(dJ > T(0)) || !(Jf > T(0)))) atomicOr(&state->elem_status, 1);
#pragma unroll
      for (int i = 0; i < 9; ++i) {
        s_P[w][gp][i] = P[i];
        s_S[w][gp][i] = S[i];
        s_FF[w][gp][i] = FF[i];
      }
      s_c[w][gp][0] = c[0];
      s_c[w][gp][1] = c[1];
      s_c[w][gp][2] = c[2];
      s_c[w][gp][3] = dJ;
    }
  }
  __syncthreads();
  if (!valid) return;

  T K[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
  T Mab = 0;
  const T rho = (T)prm.rho;
#pragma unroll
  for (int gp = 0; gp < 8; ++gp) {
    add_kab<T, MAT>(K, s_g[w][gp][a], s_g[w][gp][b], s_h[w][gp][a], s_h[w][gp][b], s_S[w][gp],
                    s_FF[w][gp], s_c[w][gp]);
    const T Na = (T)c_hex_N[hex_agree(a, gp)], Nb = (T)c_hex_N[hex_agree(b, gp)];
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
  const int ga = COMPACT ? 0 : conn[e * 8 + a];
  scatter<T, COMPACT, 8>(e, a, b, ga, Ablk, rhs, slot, smap, row_ptr, dof_fixed, A, bvec, ebuf,
                         rbuf);
}

// ---------------------------------------------- Mooney-Rivlin, co-rotational
// Both are evaluated in FP64 whatever the context precision: the
// Mooney-Rivlin stress in the isochoric invariants and the polar factor R
// both lose every digit to cancellation in FP32 near rest (F = I + H with
// small H); the results are rounded to T once.

// Forward-mode dual number (value, derivative along one direction).
struct Dual {
  double v, d;
};
__device__ inline Dual operator+(Dual a, Dual b) { return {a.v + b.v, a.d + b.d}; }
__device__ inline Dual operator-(Dual a, Dual b) { return {a.v - b.v, a.d - b.d}; }
__device__ inline Dual operator*(Dual a, Dual b) { return {a.v * b.v, a.d * b.v + a.v * b.d}; }
__device__ inline Dual operator*(double s, Dual a) { return {s * a.v, s * a.d}; }
__device__ inline Dual operator/(Dual a, Dual b) {
  const double r = 1.0 / b.v;
  return {a.v * r, (a.d - a.v * r * b.d) * r};
}
__device__ inline Dual dlog(Dual a) { return {log(a.v), a.d / a.v}; }
__device__ inline Dual dexp(Dual a) {
  const double e = exp(a.v);
  return {e, e * a.d};
}

// Mooney-Rivlin first Piola stress, decoupled compressible form
//   Psi = C10 (J^{-2/3} I1 - 3) + C01 (J^{-4/3} I2 - 3) + kappa/2 (ln J)^2,
//   P = 2 C10 J^{-2/3} (F - I1/3 F^{-T})
//     + 2 C01 J^{-4/3} (I1 F - F C - 2/3 I2 F^{-T}) + kappa ln J F^{-T},
// with dI1/dF = 2F, dI2/dF = 2(I1 F - F C), dJ/dF = J F^{-T}.
__device__ inline void mr_piola(const Dual *F, double c10, double c01, double kappa, Dual *P) {
  Dual C[9];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j)
      C[i * 3 + j] = F[i] * F[j] + F[3 + i] * F[3 + j] + F[6 + i] * F[6 + j];
  const Dual I1 = C[0] + C[4] + C[8];
  Dual trCC = {0.0, 0.0};
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) trCC = trCC + C[i * 3 + j] * C[j * 3 + i];
  const Dual I2 = 0.5 * (I1 * I1 - trCC);
  // cofactors: F^{-T} = cof(F) / J
  Dual cof[9];
  cof[0] = F[4] * F[8] - F[5] * F[7];
  cof[1] = F[5] * F[6] - F[3] * F[8];
  cof[2] = F[3] * F[7] - F[4] * F[6];
  cof[3] = F[2] * F[7] - F[1] * F[8];
  cof[4] = F[0] * F[8] - F[2] * F[6];
  cof[5] = F[1] * F[6] - F[0] * F[7];
  cof[6] = F[1] * F[5] - F[2] * F[4];
  cof[7] = F[2] * F[3] - F[0] * F[5];
  cof[8] = F[0] * F[4] - F[1] * F[3];
  const Dual J = F[0] * cof[0] + F[1] * cof[1] + F[2] * cof[2];
  const Dual lnJ = dlog(J);
  const Dual j23 = dexp((-2.0 / 3.0) * lnJ), j43 = j23 * j23;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      const Dual FiT = cof[i * 3 + j] / J;
      const Dual FC = F[i * 3] * C[j] + F[i * 3 + 1] * C[3 + j] + F[i * 3 + 2] * C[6 + j];
      const Dual t1 = (2.0 * c10) * j23 * (F[i * 3 + j] - (1.0 / 3.0) * I1 * FiT);
      const Dual t2 =
          (2.0 * c01) * j43 * (I1 * F[i * 3 + j] - FC - (2.0 / 3.0) * I2 * FiT);
      P[i * 3 + j] = t1 + t2 + kappa * lnJ * FiT;
    }
}

// Column `dir` (F_kl, dir = 3k + l) of the elasticity tensor dP/dF and the
// stress itself at F = I + H, all scaled by dV.  Returns J.
__device__ inline double mr_column(const double *H, int dir, double c10, double c01, double kappa,
                                   double dV, double *Acol, double *P) {
  Dual F[9], Pd[9];
  for (int m = 0; m < 9; ++m) F[m] = {H[m] + ((m == 0 || m == 4 || m == 8) ? 1.0 : 0.0),
                                      m == dir ? 1.0 : 0.0};
  const double J = F[0].v * (F[4].v * F[8].v - F[5].v * F[7].v) -
                   F[1].v * (F[3].v * F[8].v - F[5].v * F[6].v) +
                   F[2].v * (F[3].v * F[7].v - F[4].v * F[6].v);
  if (!(J > 0.0)) return J;
  mr_piola(F, c10, c01, kappa, Pd);
  for (int m = 0; m < 9; ++m) {
    Acol[m] = Pd[m].d * dV;
    P[m] = Pd[m].v * dV;
  }
  return J;
}

// Rotation factor of the polar decomposition F = R U by the Newton iteration
// R <- (R + R^{-T}) / 2 (quadratic convergence, at most 30 steps).  Returns
// false if an iterate is singular or inverted.
__device__ inline bool polar_rotation(const double *F, double *R) {
  for (int m = 0; m < 9; ++m) R[m] = F[m];
  for (int it = 0; it < 30; ++it) {
    const double d = det3(R);
    if (!(d > 0.0)) return false;
    double Ri[9];
    inv3(R, d, Ri);
    double diff = 0.0;
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) {
        const double rn = 0.5 * (R[i * 3 + j] + Ri[j * 3 + i]);
        diff = fmax(diff, fabs(rn - R[i * 3 + j]));
        R[i * 3 + j] = rn;
      }
    if (diff <= 1e-15) break;
  }
  return true;
}

// Mooney-Rivlin constants from (mu, lambda) and the C01 share s:
// C10 = (1 - s) mu / 2, C01 = s mu / 2, kappa = lambda + 2 mu / 3 (so the
// small-strain limit is linear elasticity with the same mu and lambda).
__device__ inline void mr_constants(double mu, double lam, double share, double &c10,
                                    double &c01, double &kappa) {
  c10 = (1.0 - share) * 0.5 * mu;
  c01 = share * 0.5 * mu;
  kappa = lam + 2.0 * mu / 3.0;
}

// HEX8, Mooney-Rivlin (MAT 3) or co-rotational (MAT 2).  One wavefront per
// hexahedron, lane = (a, b) as in k_elem_hex.
//   MAT 3: lanes 0..7 set up the Gauss points; then the 72 (point, direction)
//     columns of dP/dF are spread over the 64 lanes (dual numbers, FP64);
//     lane (a, b) accumulates K_ab = sum_q g_a,j A_ijkl g_b,l; lane (a, b)
//     takes the force share of Gauss point b.
//   MAT 2: lanes 0..7 set up the Gauss points (gradients, weights), lane 0
//     the rotation R of F at the element centre; lanes 0..7 rotate their
//     node back, d_n = R^T (x_n - x_0) - (X_n - X_0); lane (a, b) forms the
//     linear-elastic block K0_ab, K_ab = R K0_ab R^T and the force share
//     R K0_ab d_b.
template <typename T, int MAT, bool COMPACT>
__global__ __launch_bounds__(256) void k_elem_hex_x(
    int64_t n_elems, const int32_t *__restrict__ conn, const uint8_t *__restrict__ slot,
    const int32_t *__restrict__ smap, const int32_t *__restrict__ row_ptr,
    const double *__restrict__ X, const double *__restrict__ q, const double *__restrict__ v,
    const double *__restrict__ Ev, const uint8_t *__restrict__ dof_fixed, ElemParams prm,
    T *__restrict__ A, double *__restrict__ bvec, T *__restrict__ ebuf,
    double *__restrict__ rbuf, PcgState *state) {
  constexpr int NW = 4;
  constexpr int NA = MAT == 3 ? 81 : 1;
  __shared__ T s_x[NW][8][3], s_u[NW][8][3], s_v[NW][8][3];
  __shared__ T s_g[NW][8][8][3], s_dv[NW][8];
  __shared__ double s_H[NW][8][9];
  __shared__ T s_A[NW][8][NA], s_P[NW][8][9];
  __shared__ double s_R[NW][9];
  __shared__ T s_Rt[NW][9], s_d[NW][8][3];
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
  const double Ee = valid ? Ev[e] : 0.0;
  const double nu = prm.nu;
  const double mu = Ee / (2.0 * (1.0 + nu));
  const double lam = Ee * nu / ((1.0 + nu) * (1.0 - 2.0 * nu));
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
    if (!(dJ > T(0))) atomicOr(&state->elem_status, 1);
    T Ji[9];
    inv3(J, dJ, Ji);
    double H[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    for (int n = 0; n < 8; ++n) {
      T g[3];
      for (int i = 0; i < 3; ++i)
        g[i] = dN[n][0] * Ji[0 * 3 + i] + dN[n][1] * Ji[1 * 3 + i] + dN[n][2] * Ji[2 * 3 + i];
      for (int i = 0; i < 3; ++i) s_g[w][gp][n][i] = g[i];
      for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) H[i * 3 + j] += (double)s_u[w][n][i] * (double)g[j];
    }
    for (int m = 0; m < 9; ++m) s_H[w][gp][m] = H[m];
    s_dv[w][gp] = dJ;
    if (MAT == 2 && gp == 0) {
      // deformation gradient at the centre: dN_n(0) = sign_n / 8
      T Jc[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
      for (int n = 0; n < 8; ++n)
        for (int i = 0; i < 3; ++i)
          for (int j = 0; j < 3; ++j) Jc[i * 3 + j] += s_x[w][n][i] * T(0.125) * (T)c_hex_sign[n][j];
      T Jci[9];
      inv3(Jc, det3(Jc), Jci);
      double Fc[9] = {1, 0, 0, 0, 1, 0, 0, 0, 1};
      for (int n = 0; n < 8; ++n)
        for (int j = 0; j < 3; ++j) {
          const double gc = 0.125 * (c_hex_sign[n][0] * (double)Jci[j] +
                                     c_hex_sign[n][1] * (double)Jci[3 + j] +
                                     c_hex_sign[n][2] * (double)Jci[6 + j]);
          for (int i = 0; i < 3; ++i) Fc[i * 3 + j] += (double)s_u[w][n][i] * gc;
        }
      double R[9];
      if (!polar_rotation(Fc, R)) atomicOr(&state->elem_status, 1);
      for (int m = 0; m < 9; ++m) s_R[w][m] = R[m];
    }
  }
  __syncthreads();
  if (MAT == 3) {
    double c10, c01, kappa;
    mr_constants(mu, lam, prm.mr_c01_share, c10, c01, kappa);
    for (int task = lane; task < 72; task += 64) {
      const int gp = task / 9, dir = task - 9 * (task / 9);
      if (!valid) break;
      double Acol[9], P[9];
      const double Jg = mr_column(s_H[w][gp], dir, c10, c01, kappa, (double)s_dv[w][gp], Acol, P);
      if (!(Jg > 0.0)) {
        if (dir == 0) atomicOr(&state->elem_status, 1);
        for (int m = 0; m < 9; ++m) Acol[m] = P[m] = 0.0;
      }
      for (int m = 0; m < 9; ++m) s_A[w][gp][m * 9 + dir] = (T)Acol[m];
      if (dir == 0)
        for (int m = 0; m < 9; ++m) s_P[w][gp][m] = (T)P[m];
    }
  } else {
    if (valid && lane < 8) {
      // node lane: d_n = R^T (x_n - x_0) - (X_n - X_0)
      //               = (R^T - I)(X_n - X_0) + R^T (u_n - u_0)
      const double *R = s_R[w];
      double dx[3], du[3];
      for (int i = 0; i < 3; ++i) {
        dx[i] = (double)s_x[w][lane][i];
        du[i] = (double)s_u[w][lane][i] - (double)s_u[w][0][i];
      }
      for (int i = 0; i < 3; ++i) {
        double r = 0.0;
        for (int j = 0; j < 3; ++j)
          r += (R[j * 3 + i] - (i == j ? 1.0 : 0.0)) * dx[j] + R[j * 3 + i] * du[j];
        s_d[w][lane][i] = (T)r;
      }
      if (lane == 0)
        for (int m = 0; m < 9; ++m) s_Rt[w][m] = (T)R[m];
    }
  }
  __syncthreads();
  if (!valid) return;

  T K[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
  T Mab = 0, fa[3] = {0, 0, 0};
  const T rho = (T)prm.rho;
  const T tmu = (T)mu, tlam = (T)lam;
  for (int gp = 0; gp < 8; ++gp) {
    const T *ga = s_g[w][gp][a], *gb = s_g[w][gp][b];
    if (MAT == 3) {
      const T *Ag = s_A[w][gp];
      for (int i = 0; i < 3; ++i)
        for (int k = 0; k < 3; ++k) {
          T acc = 0;
          for (int j = 0; j < 3; ++j) {
            const T *Ar = Ag + (i * 3 + j) * 9 + k * 3;
            acc += ga[j] * (Ar[0] * gb[0] + Ar[1] * gb[1] + Ar[2] * gb[2]);
          }
          K[i * 3 + k] += acc;
        }
    } else {
      // linear-elastic block: dV [lam g_a g_b^T + mu g_b g_a^T + mu (g_a.g_b) I]
      const T dv = s_dv[w][gp];
      const T gg = ga[0] * gb[0] + ga[1] * gb[1] + ga[2] * gb[2];
      for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j)
          K[i * 3 + j] += dv * (tlam * ga[i] * gb[j] + tmu * gb[i] * ga[j]);
      K[0] += dv * tmu * gg;
      K[4] += dv * tmu * gg;
      K[8] += dv * tmu * gg;
    }
    const T xi0 = (gp & 1) ? g1 : -g1, xi1 = (gp & 2) ? g1 : -g1, xi2 = (gp & 4) ? g1 : -g1;
    const T Na = T(0.125) * (T(1) + (T)c_hex_sign[a][0] * xi0) *
                 (T(1) + (T)c_hex_sign[a][1] * xi1) * (T(1) + (T)c_hex_sign[a][2] * xi2);
    const T Nb = T(0.125) * (T(1) + (T)c_hex_sign[b][0] * xi0) *
                 (T(1) + (T)c_hex_sign[b][1] * xi1) * (T(1) + (T)c_hex_sign[b][2] * xi2);
    Mab += rho * Na * Nb * s_dv[w][gp];
  }
  if (MAT == 3) {
    // force share: Gauss point b of node a
    const T *P = s_P[w][b];
    const T *g = s_g[w][b][a];
    for (int i = 0; i < 3; ++i) fa[i] = P[i * 3] * g[0] + P[i * 3 + 1] * g[1] + P[i * 3 + 2] * g[2];
  } else {
    // K0_ab d_b, rotated; then K_ab = R K0_ab R^T
    const T *R = s_Rt[w];
    const T *d = s_d[w][b];
    T kd[3];
    for (int i = 0; i < 3; ++i) kd[i] = K[i * 3] * d[0] + K[i * 3 + 1] * d[1] + K[i * 3 + 2] * d[2];
    for (int i = 0; i < 3; ++i) fa[i] = R[i * 3] * kd[0] + R[i * 3 + 1] * kd[1] + R[i * 3 + 2] * kd[2];
    T RK[9];
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j)
        RK[i * 3 + j] = R[i * 3] * K[j] + R[i * 3 + 1] * K[3 + j] + R[i * 3 + 2] * K[6 + j];
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j)
        K[i * 3 + j] = RK[i * 3] * R[j * 3] + RK[i * 3 + 1] * R[j * 3 + 1] + RK[i * 3 + 2] * R[j * 3 + 2];
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

// TET4, Mooney-Rivlin (MAT 3) or co-rotational (MAT 2): 16 lanes per
// tetrahedron, lane = (a, b), one quadrature point.  MAT 3: lanes 0..8 of the
// tetrahedron compute the nine columns of dP/dF; MAT 2: lane 0 computes R,
// lanes 0..3 rotate their node back.
template <typename T, int MAT, bool COMPACT>
__global__ __launch_bounds__(256) void k_elem_tet_x(
    int64_t n_elems, const int32_t *__restrict__ conn, const uint8_t *__restrict__ slot,
    const int32_t *__restrict__ smap, const int32_t *__restrict__ row_ptr,
    const double *__restrict__ X, const double *__restrict__ q, const double *__restrict__ v,
    const double *__restrict__ Ev, const uint8_t *__restrict__ dof_fixed, ElemParams prm,
    T *__restrict__ A, double *__restrict__ bvec, T *__restrict__ ebuf,
    double *__restrict__ rbuf, PcgState *state) {
  constexpr int NT = 16;  // tets per block
  constexpr int NA = MAT == 3 ? 81 : 1;
  __shared__ T s_x[NT][4][3], s_u[NT][4][3], s_v[NT][4][3];
  __shared__ T s_A[NT][NA], s_P[NT][9], s_Rt[NT][9], s_d[NT][4][3];
  __shared__ double s_R[NT][9];
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
  const double Ee = valid ? Ev[e] : 0.0;
  const double nu = prm.nu;
  const double mu = Ee / (2.0 * (1.0 + nu));
  const double lam = Ee * nu / ((1.0 + nu) * (1.0 - 2.0 * nu));
  T g[4][3], V = T(0);
  double H[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
  if (valid) {
    T Dm[9];
    for (int i = 0; i < 3; ++i)
      for (int k = 0; k < 3; ++k) Dm[i * 3 + k] = s_x[t][k + 1][i];
    const T det = det3(Dm);
    if (!(det > T(0)) && l16 == 0) atomicOr(&state->elem_status, 1);
    T Di[9];
    inv3(Dm, det, Di);
    V = det / T(6);
    for (int i = 0; i < 3; ++i) {
      g[1][i] = Di[0 * 3 + i];
      g[2][i] = Di[1 * 3 + i];
      g[3][i] = Di[2 * 3 + i];
      g[0][i] = -(g[1][i] + g[2][i] + g[3][i]);
    }
    for (int n = 0; n < 4; ++n)
      for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) H[i * 3 + j] += (double)s_u[t][n][i] * (double)g[n][j];
    if (MAT == 3 && l16 < 9) {
      double c10, c01, kappa, Acol[9], P[9];
      mr_constants(mu, lam, prm.mr_c01_share, c10, c01, kappa);
      const double Jg = mr_column(H, l16, c10, c01, kappa, (double)V, Acol, P);
      if (!(Jg > 0.0)) {
        if (l16 == 0) atomicOr(&state->elem_status, 1);
        for (int m = 0; m < 9; ++m) Acol[m] = P[m] = 0.0;
      }
      for (int m = 0; m < 9; ++m) s_A[t][m * 9 + l16] = (T)Acol[m];
      if (l16 == 0)
        for (int m = 0; m < 9; ++m) s_P[t][m] = (T)P[m];
    }
    if (MAT == 2 && l16 == 0) {
      double F[9], R[9];
      for (int m = 0; m < 9; ++m) F[m] = H[m] + ((m == 0 || m == 4 || m == 8) ? 1.0 : 0.0);
      if (!polar_rotation(F, R)) atomicOr(&state->elem_status, 1);
      for (int m = 0; m < 9; ++m) s_R[t][m] = R[m];
    }
  }
  __syncthreads();
  if (MAT == 2 && valid && l16 < 4) {
    const double *R = s_R[t];
    double dx[3], du[3];
    for (int i = 0; i < 3; ++i) {
      dx[i] = (double)s_x[t][l16][i];
      du[i] = (double)s_u[t][l16][i] - (double)s_u[t][0][i];
    }
    for (int i = 0; i < 3; ++i) {
      double r = 0.0;
      for (int j = 0; j < 3; ++j)
        r += (R[j * 3 + i] - (i == j ? 1.0 : 0.0)) * dx[j] + R[j * 3 + i] * du[j];
      s_d[t][l16][i] = (T)r;
    }
    if (l16 == 0)
      for (int m = 0; m < 9; ++m) s_Rt[t][m] = (T)R[m];
  }
  __syncthreads();
  if (!valid) return;
  T K[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0}, fa[3];
  if (MAT == 3) {
    for (int i = 0; i < 3; ++i)
      for (int k = 0; k < 3; ++k) {
        T acc = 0;
        for (int j = 0; j < 3; ++j) {
          const T *Ar = s_A[t] + (i * 3 + j) * 9 + k * 3;
          acc += g[a][j] * (Ar[0] * g[b][0] + Ar[1] * g[b][1] + Ar[2] * g[b][2]);
        }
        K[i * 3 + k] = acc;
      }
    const T *P = s_P[t];
    for (int i = 0; i < 3; ++i)
      fa[i] = T(0.25) * (P[i * 3] * g[a][0] + P[i * 3 + 1] * g[a][1] + P[i * 3 + 2] * g[a][2]);
  } else {
    const T tmu = (T)mu, tlam = (T)lam;
    const T gg = g[a][0] * g[b][0] + g[a][1] * g[b][1] + g[a][2] * g[b][2];
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) K[i * 3 + j] = V * (tlam * g[a][i] * g[b][j] + tmu * g[b][i] * g[a][j]);
    K[0] += V * tmu * gg;
    K[4] += V * tmu * gg;
    K[8] += V * tmu * gg;
    const T *R = s_Rt[t];
    const T *d = s_d[t][b];
    T kd[3];
    for (int i = 0; i < 3; ++i) kd[i] = K[i * 3] * d[0] + K[i * 3 + 1] * d[1] + K[i * 3 + 2] * d[2];
    for (int i = 0; i < 3; ++i) fa[i] = R[i * 3] * kd[0] + R[i * 3 + 1] * kd[1] + R[i * 3 + 2] * kd[2];
    T RK[9];
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j)
        RK[i * 3 + j] = R[i * 3] * K[j] + R[i * 3 + 1] * K[3 + j] + R[i * 3 + 2] * K[6 + j];
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j)
        K[i * 3 + j] = RK[i * 3] * R[j * 3] + RK[i * 3 + 1] * R[j * 3 + 1] + RK[i * 3 + 2] * R[j * 3 + 2];
  }
  const T Mab = (T)prm.rho * V * (a == b ? T(2) : T(1)) / T(20);
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
  // XCD-contiguous workgroups: the hardware hands workgroup b to XCD b % 8,
  // so XCD x takes the x-th contiguous eighth of the node blocks, and node
  // blocks that share elements (neighbours in the node order) read the
  // contribution buffer through the same L2
  const int64_t per = gridDim.x / 8;
  const int64_t wg = (int64_t)(blockIdx.x % 8) * per + blockIdx.x / 8;
  const int64_t k = wg * blockDim.x + threadIdx.x;
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
    // src = e * NEN^2 + a * NEN + b; block (a, b) of element e is stored as
    // such when a <= b, else as the transpose of block (b, a)
    const int32_t e = src / (NEN * NEN), ab = src % (NEN * NEN);
    const int a = ab / NEN, bb = ab % NEN;
    const bool tr = a > bb;
    const T *eb = ebuf + ((int64_t)e * (NEN * (NEN + 1) / 2) +
                          (tr ? sym_block<NEN>(bb, a) : sym_block<NEN>(a, bb))) * 9;
    T blk[9];
#pragma unroll
    for (int q = 0; q < 9; ++q) blk[q] = eb[q];
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
      for (int c = 0; c < 3; ++c) acc[r * 3 + c] += (double)(tr ? blk[c * 3 + r] : blk[r * 3 + c]);
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

// keepStruct test of the fill order: flag[0] = 1 if any entry differs.
template <typename U>
__global__ void k_struct_cmp(int64_t n, const U *__restrict__ a, const U *__restrict__ b,
                             int *flag) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
    if (a[i] != b[i]) *flag = 1;
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
#define FE_HEXX(MAT, CMP)                                                                   \
  k_elem_hex_x<T, MAT, CMP><<<blocks, 256, 0, st>>>(n_elems, conn, slot, smap, row_ptr, X, q, \
                                                     v, E, dof_fixed, prm, A, b, ebuf, rbuf,   \
                                                     state)
    if (prm.material == 0) {
      if (compact) FE_HEX(0, true); else FE_HEX(0, false);
    } else if (prm.material == 1) {
      if (compact) FE_HEX(1, true); else FE_HEX(1, false);
    } else if (prm.material == 2) {
      if (compact) FE_HEXX(2, true); else FE_HEXX(2, false);
    } else {
      if (compact) FE_HEXX(3, true); else FE_HEXX(3, false);
    }
#undef FE_HEX
#undef FE_HEXX
  } else {
    const unsigned blocks = (unsigned)((n_elems + 15) / 16);
#define FE_TET(MAT, CMP)                                                                    \
  k_elem_tet<T, MAT, CMP><<<blocks, 256, 0, st>>>(n_elems, conn, slot, smap, row_ptr, X, q, \
                                                   v, E, dof_fixed, prm, A, b, ebuf, rbuf, state)
#define FE_TETX(MAT, CMP)                                                                   \
  k_elem_tet_x<T, MAT, CMP><<<blocks, 256, 0, st>>>(n_elems, conn, slot, smap, row_ptr, X, q, \
                                                     v, E, dof_fixed, prm, A, b, ebuf, rbuf,   \
                                                     state)
    if (prm.material == 0) {
      if (compact) FE_TET(0, true); else FE_TET(0, false);
    } else if (prm.material == 1) {
      if (compact) FE_TET(1, true); else FE_TET(1, false);
    } else if (prm.material == 2) {
      if (compact) FE_TETX(2, true); else FE_TETX(2, false);
    } else {
      if (compact) FE_TETX(3, true); else FE_TETX(3, false);
    }
#undef FE_TET
#undef FE_TETX
  }
}

void launch_struct_cmp(hipStream_t st, int64_t n_conn, const int32_t *conn, const int32_t *ref_conn,
                       int64_t n_dofs, const uint8_t *fixed, const uint8_t *ref_fixed,
                       int *flag) {
  auto grid = [](int64_t n) { return (unsigned)std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, 4096)); };
  if (n_conn > 0) k_struct_cmp<int32_t><<<grid(n_conn), 256, 0, st>>>(n_conn, conn, ref_conn, flag);
  if (fixed && n_dofs > 0)
    k_struct_cmp<uint8_t><<<grid(n_dofs), 256, 0, st>>>(n_dofs, fixed, ref_fixed, flag);
}

template <typename T>
void launch_assembly_gather(hipStream_t st, int nen, int64_t n_blocks, const int32_t *blk_ptr,
                            const int32_t *blk_src, const int32_t *blk_pos,
                            const int32_t *blk_node, const int32_t *row_ptr, const T *ebuf,
                            const double *rbuf, const double *f_nodal, T *A, double *b) {
  if (n_blocks <= 0) return;
  // a multiple of 8 workgroups, see k_assembly_gather
  const unsigned blocks = (unsigned)(((n_blocks + 255) / 256 + 7) / 8 * 8);
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
