// Adjoint element pass (not in the paper): for the reverse step of the
// linearised backward-Euler update it needs, per element,
//   (K mu)_a   = sum_gp dV dP[Mu] g_a                  Mu = sum_b mu_b (x) g_b
//   (M mu)_a   = sum_gp rho N_a mu(gp) dV
//   T_a        = sum_gp dV d2P[Mu, V] g_a              V  = sum_b v+_b (x) g_b
//   mu.f       = sum_gp dV P : Mu
//   mu.K v+    = sum_gp dV dP[V] : Mu
// where dP[W] = d/de P(F + e W) and d2P[W, U] its derivative along U, i.e.
// T = d/de K(q + e mu) v+ is the third derivative of the stored energy.
// Closed forms (B = F^{-1}, W^ = B W, U^ = B U):
//  neo-Hookean  P = mu F + (lam lnJ - mu) F^{-T}
//    dP[W]    = mu W + lam tr(W^) B^T - (lam lnJ - mu) (W^ B)^T
//    d2P[W,U] = -lam tr(U^ W^) B^T - lam tr(W^) (U^ B)^T - lam tr(U^) (W^ B)^T
//               + (lam lnJ - mu) ((W^ U^ B)^T + (U^ W^ B)^T)
//  St Venant-Kirchhoff  P = F S(E),  S(X) = lam tr X I + 2 mu X
//    dP[W]    = W S + F S(sym(F^T W))
//    d2P[W,U] = W S(sym(F^T U)) + U S(sym(F^T W)) + F S(sym(U^T W))
// One thread per element; results are scattered with FP64 atomics.
// The element arithmetic is FP64 in both precision modes: the pass runs once
// per reverse step beside a whole CG solve, so its cost is small, and the
// third-derivative terms then carry no FP32 rounding into dL/dE.
#include "device.hpp"

namespace fe {

namespace {

__constant__ double c_sign[8][3] = {
    {-1, -1, -1}, {1, -1, -1}, {1, 1, -1}, {-1, 1, -1},
    {-1, -1, 1},  {1, -1, 1},  {1, 1, 1},  {-1, 1, 1}};

template <typename T>
struct Mat3 {
  T m[9];
  __device__ T &operator()(int i, int j) { return m[i * 3 + j]; }
  __device__ T operator()(int i, int j) const { return m[i * 3 + j]; }
};

template <typename T>
__device__ inline Mat3<T> mul(const Mat3<T> &A, const Mat3<T> &B) {
  Mat3<T> C;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      T s = 0;
      for (int k = 0; k < 3; ++k) s += A(i, k) * B(k, j);
      C(i, j) = s;
    }
  return C;
}
template <typename T>
__device__ inline Mat3<T> tr_(const Mat3<T> &A) {
  Mat3<T> C;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) C(i, j) = A(j, i);
  return C;
}
template <typename T>
__device__ inline T trace(const Mat3<T> &A) { return A(0, 0) + A(1, 1) + A(2, 2); }
template <typename T>
__device__ inline T ddot(const Mat3<T> &A, const Mat3<T> &B) {
  T s = 0;
  for (int i = 0; i < 9; ++i) s += A.m[i] * B.m[i];
  return s;
}
template <typename T>
__device__ inline T det3(const Mat3<T> &M) {
  return M(0, 0) * (M(1, 1) * M(2, 2) - M(1, 2) * M(2, 1)) -
         M(0, 1) * (M(1, 0) * M(2, 2) - M(1, 2) * M(2, 0)) +
         M(0, 2) * (M(1, 0) * M(2, 1) - M(1, 1) * M(2, 0));
}
template <typename T>
__device__ inline Mat3<T> inv3(const Mat3<T> &M, T d) {
  Mat3<T> R;
  const T id = T(1) / d;
  R(0, 0) = (M(1, 1) * M(2, 2) - M(1, 2) * M(2, 1)) * id;
  R(0, 1) = (M(0, 2) * M(2, 1) - M(0, 1) * M(2, 2)) * id;
  R(0, 2) = (M(0, 1) * M(1, 2) - M(0, 2) * M(1, 1)) * id;
  R(1, 0) = (M(1, 2) * M(2, 0) - M(1, 0) * M(2, 2)) * id;
  R(1, 1) = (M(0, 0) * M(2, 2) - M(0, 2) * M(2, 0)) * id;
  R(1, 2) = (M(0, 2) * M(1, 0) - M(0, 0) * M(1, 2)) * id;
  R(2, 0) = (M(1, 0) * M(2, 1) - M(1, 1) * M(2, 0)) * id;
  R(2, 1) = (M(0, 1) * M(2, 0) - M(0, 0) * M(2, 1)) * id;
  R(2, 2) = (M(0, 0) * M(1, 1) - M(0, 1) * M(1, 0)) * id;
  return R;
}
template <typename T>
__device__ inline Mat3<T> stvk_S(const Mat3<T> &X, T mu, T lam) {
  Mat3<T> S;
  const T t = trace(X);
  for (int i = 0; i < 9; ++i) S.m[i] = T(2) * mu * X.m[i];
  S(0, 0) += lam * t;
  S(1, 1) += lam * t;
  S(2, 2) += lam * t;
  return S;
}
template <typename T>
__device__ inline Mat3<T> sym_AtB(const Mat3<T> &A, const Mat3<T> &B) {
  // sym(A^T B) = (A^T B + B^T A) / 2
  Mat3<T> C = mul(tr_(A), B);
  Mat3<T> R;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) R(i, j) = T(0.5) * (C(i, j) + C(j, i));
  return R;
}

// Per quadrature point: P, dP[V], dP[Mu], d2P[Mu, V] from H = grad u.
template <typename T, int MAT>
__device__ inline void point_terms(const Mat3<T> &H, const Mat3<T> &Mu, const Mat3<T> &V, T mu,
                                   T lam, Mat3<T> &P, Mat3<T> &dPV, Mat3<T> &dPM,
                                   Mat3<T> &d2P) {
  Mat3<T> F = H;
  F(0, 0) += T(1);
  F(1, 1) += T(1);
  F(2, 2) += T(1);
  if (MAT == 0) {
    // J - 1 from the invariants of H (det(I + H) = 1 + tr H + (tr^2 H -
    // tr H^2) / 2 + det H) and P = F^{-T} (2 mu E + lam lnJ I) with
    // E = (H + H^T + H^T H) / 2: near rest neither cancels the O(1) parts
    // of F and F^{-T} against each other.
    const T trH = trace(H);
    const Mat3<T> HH = mul(H, H);
    const T Jm1 = trH + T(0.5) * (trH * trH - trace(HH)) + det3(H);
    const Mat3<T> B = inv3(F, T(1) + Jm1);
    const Mat3<T> BT = tr_(B);
    const T lnJ = log1p(Jm1);
    const T c = lam * lnJ - mu;
    {
      Mat3<T> S;
      const Mat3<T> HtH = mul(tr_(H), H);
      for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) S(i, j) = mu * (H(i, j) + H(j, i) + HtH(i, j));
      S(0, 0) += lam * lnJ;
      S(1, 1) += lam * lnJ;
      S(2, 2) += lam * lnJ;
      P = mul(BT, S);
    }
    const Mat3<T> Wh = mul(B, Mu), Uh = mul(B, V);
    const Mat3<T> WhB = tr_(mul(Wh, B)), UhB = tr_(mul(Uh, B));
    const T trW = trace(Wh), trU = trace(Uh);
    for (int i = 0; i < 9; ++i) {
      dPM.m[i] = mu * Mu.m[i] + lam * trW * BT.m[i] - c * WhB.m[i];
      dPV.m[i] = mu * V.m[i] + lam * trU * BT.m[i] - c * UhB.m[i];
    }
    const Mat3<T> WUB = tr_(mul(mul(Wh, Uh), B)), UWB = tr_(mul(mul(Uh, Wh), B));
    const T trUW = trace(mul(Uh, Wh));
    for (int i = 0; i < 9; ++i)
      d2P.m[i] = -lam * trUW * BT.m[i] - lam * trW * UhB.m[i] - lam * trU * WhB.m[i] +
                 c * (WUB.m[i] + UWB.m[i]);
  } else {
    Mat3<T> Eg;
    const Mat3<T> HtH = mul(tr_(H), H);
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) Eg(i, j) = T(0.5) * (H(i, j) + H(j, i) + HtH(i, j));
    const Mat3<T> S = stvk_S(Eg, mu, lam);
    P = mul(F, S);
    const Mat3<T> SW = stvk_S(sym_AtB(F, Mu), mu, lam);
    const Mat3<T> SU = stvk_S(sym_AtB(F, V), mu, lam);
    const Mat3<T> SWU = stvk_S(sym_AtB(V, Mu), mu, lam);
    const Mat3<T> a1 = mul(Mu, S), a2 = mul(F, SW), b1 = mul(V, S), b2 = mul(F, SU);
    const Mat3<T> c1 = mul(Mu, SU), c2 = mul(V, SW), c3 = mul(F, SWU);
    for (int i = 0; i < 9; ++i) {
      dPM.m[i] = a1.m[i] + a2.m[i];
      dPV.m[i] = b1.m[i] + b2.m[i];
      d2P.m[i] = c1.m[i] + c2.m[i] + c3.m[i];
    }
  }
}

template <typename T, int MAT, int NEN>
__global__ __launch_bounds__(128) void k_adjoint_elem(int64_t n_elems, const int32_t *conn,
                                                      const double *X, const double *q,
                                                      const double *mu_v, const double *vp,
                                                      const double *Ev, ElemParams prm,
                                                      double *Kmu, double *Mmu, double *Tmv,
                                                      double *dE) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n_elems) return;
  int nd[NEN];
  T x[NEN][3], u[NEN][3], m[NEN][3], w[NEN][3];
  for (int a = 0; a < NEN; ++a) {
    nd[a] = conn[e * NEN + a];
    for (int i = 0; i < 3; ++i) {
      x[a][i] = (T)(X[3 * nd[a] + i] - X[3 * conn[e * NEN] + i]);
      u[a][i] = (T)(q[3 * nd[a] + i] - X[3 * nd[a] + i]);
      m[a][i] = (T)mu_v[3 * nd[a] + i];
      w[a][i] = (T)vp[3 * nd[a] + i];
    }
  }
  const T Ee = (T)Ev[e], nu = (T)prm.nu;
  const T mu = Ee / (T(2) * (T(1) + nu));
  const T lam = Ee * nu / ((T(1) + nu) * (T(1) - T(2) * nu));
  const T rho = (T)prm.rho;
  T km[NEN][3], tm[NEN][3], mm[NEN][3];
  for (int a = 0; a < NEN; ++a)
    for (int i = 0; i < 3; ++i) km[a][i] = tm[a][i] = mm[a][i] = T(0);
  T muf = 0, muKv = 0;
  const int NGP = NEN == 8 ? 8 : 1;
  for (int gp = 0; gp < NGP; ++gp) {
    T g[NEN][3];
    T dV;
    T N[NEN];
    if (NEN == 8) {
      const T g1 = T(0.57735026918962576451);
      const T xi[3] = {(gp & 1) ? g1 : -g1, (gp & 2) ? g1 : -g1, (gp & 4) ? g1 : -g1};
      T dN[NEN][3];
      for (int n = 0; n < NEN; ++n) {
        const T s0 = (T)c_sign[n][0], s1 = (T)c_sign[n][1], s2 = (T)c_sign[n][2];
        const T t0 = T(1) + s0 * xi[0], t1 = T(1) + s1 * xi[1], t2 = T(1) + s2 * xi[2];
        dN[n][0] = T(0.125) * s0 * t1 * t2;
        dN[n][1] = T(0.125) * s1 * t0 * t2;
        dN[n][2] = T(0.125) * s2 * t0 * t1;
        N[n] = T(0.125) * t0 * t1 * t2;
      }
      Mat3<T> J;
      for (int i = 0; i < 9; ++i) J.m[i] = 0;
      for (int n = 0; n < NEN; ++n)
        for (int i = 0; i < 3; ++i)
          for (int j = 0; j < 3; ++j) J(i, j) += x[n][i] * dN[n][j];
      dV = det3(J);
      const Mat3<T> Ji = inv3(J, dV);
      for (int n = 0; n < NEN; ++n)
        for (int i = 0; i < 3; ++i)
          g[n][i] = dN[n][0] * Ji(0, i) + dN[n][1] * Ji(1, i) + dN[n][2] * Ji(2, i);
    } else {
      Mat3<T> Dm;
      for (int i = 0; i < 3; ++i)
        for (int k = 0; k < 3; ++k) Dm(i, k) = x[k + 1][i];
      const T d = det3(Dm);
      const Mat3<T> Di = inv3(Dm, d);
      for (int i = 0; i < 3; ++i) {
        g[1][i] = Di(0, i);
        g[2][i] = Di(1, i);
        g[3][i] = Di(2, i);
        g[0][i] = -(g[1][i] + g[2][i] + g[3][i]);
      }
      dV = d / T(6);
      for (int n = 0; n < NEN; ++n) N[n] = T(0.25);
    }
    Mat3<T> H, Mu, V;
    for (int i = 0; i < 9; ++i) H.m[i] = Mu.m[i] = V.m[i] = 0;
    for (int n = 0; n < NEN; ++n)
      for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
          H(i, j) += u[n][i] * g[n][j];
          Mu(i, j) += m[n][i] * g[n][j];
          V(i, j) += w[n][i] * g[n][j];
        }
    Mat3<T> P, dPV, dPM, d2P;
    point_terms<T, MAT>(H, Mu, V, mu, lam, P, dPV, dPM, d2P);
    muf += dV * ddot(P, Mu);
    muKv += dV * ddot(dPV, Mu);
    for (int a = 0; a < NEN; ++a)
      for (int i = 0; i < 3; ++i) {
        T s1 = 0, s2 = 0;
        for (int j = 0; j < 3; ++j) {
          s1 += dPM(i, j) * g[a][j];
          s2 += d2P(i, j) * g[a][j];
        }
        km[a][i] += dV * s1;
        tm[a][i] += dV * s2;
      }
    if (NEN == 8) {
      T mg[3] = {0, 0, 0};
      for (int n = 0; n < NEN; ++n)
        for (int i = 0; i < 3; ++i) mg[i] += N[n] * m[n][i];
      for (int a = 0; a < NEN; ++a)
        for (int i = 0; i < 3; ++i) mm[a][i] += rho * dV * N[a] * mg[i];
    } else {
      T ms[3] = {0, 0, 0};
      for (int n = 0; n < NEN; ++n)
        for (int i = 0; i < 3; ++i) ms[i] += m[n][i];
      for (int a = 0; a < NEN; ++a)
        for (int i = 0; i < 3; ++i) mm[a][i] = rho * dV / T(20) * (m[a][i] + ms[i]);
    }
  }
  for (int a = 0; a < NEN; ++a)
    for (int i = 0; i < 3; ++i) {
      atomicAdd(Kmu + 3 * nd[a] + i, (double)km[a][i]);
      atomicAdd(Tmv + 3 * nd[a] + i, (double)tm[a][i]);
      atomicAdd(Mmu + 3 * nd[a] + i, (double)mm[a][i]);
    }
  const double cKv = prm.beta + prm.h;
  dE[e] += -((double)muf + cKv * (double)muKv) / Ev[e];
}

__global__ void k_adjoint_combine(int64_t n, double h, double al, double be, const double *lq,
                                  const double *lv, const double *Kmu, const double *Mmu,
                                  const double *Tmv, double *lq_out, double *lv_out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double q = lq[i], v = lv[i];
  lv_out[i] = v + h * q - al * Mmu[i] - (be + h) * Kmu[i];
  lq_out[i] = q - Kmu[i] - (be + h) * Tmv[i];
}

__global__ void k_abar(int64_t n, double h, const double *lq, const double *lv,
                       const uint8_t *fixed, double *abar) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  abar[i] = fixed[i] ? 0.0 : h * lv[i] + h * h * lq[i];
}

}  // namespace

template <typename T>
void launch_adjoint_element(hipStream_t st, int elem_type, int64_t n_elems, const int32_t *conn,
                            const double *X, const double *q, const double *mu,
                            const double *vnp1, const double *E, const ElemParams &prm,
                            double *Kmu, double *Mmu, double *Tmv, double *dE) {
  if (n_elems <= 0) return;
  const unsigned blocks = (unsigned)((n_elems + 127) / 128);
#define FE_ADJ(MAT, NEN)                                                                   \
  k_adjoint_elem<double, MAT, NEN><<<blocks, 128, 0, st>>>(n_elems, conn, X, q, mu, vnp1, E, prm, \
                                                      Kmu, Mmu, Tmv, dE)
  if (elem_type == 8) {
    if (prm.material == 0) FE_ADJ(0, 8); else FE_ADJ(1, 8);
  } else {
    if (prm.material == 0) FE_ADJ(0, 4); else FE_ADJ(1, 4);
  }
#undef FE_ADJ
}

void launch_adjoint_combine(hipStream_t st, int64_t n, double h, double alpha, double beta,
                            const double *lq, const double *lv, const double *Kmu,
                            const double *Mmu, const double *Tmv, double *lq_out,
                            double *lv_out) {
  k_adjoint_combine<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(n, h, alpha, beta, lq, lv, Kmu,
                                                                 Mmu, Tmv, lq_out, lv_out);
}

void launch_abar(hipStream_t st, int64_t n, double h, const double *lq, const double *lv,
                 const uint8_t *fixed, double *abar) {
  k_abar<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(n, h, lq, lv, fixed, abar);
}

template void launch_adjoint_element<float>(hipStream_t, int, int64_t, const int32_t *,
                                            const double *, const double *, const double *,
                                            const double *, const double *, const ElemParams &,
                                            double *, double *, double *, double *);
template void launch_adjoint_element<double>(hipStream_t, int, int64_t, const int32_t *,
                                             const double *, const double *, const double *,
                                             const double *, const double *, const ElemParams &,
                                             double *, double *, double *, double *);

}  // namespace fe
