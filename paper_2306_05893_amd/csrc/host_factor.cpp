// FP64 numeric LDL^T factorisation on the host (paper Sec. 3.3: the factor of
// an earlier A is computed in a thread beside the simulation loop and used
// as the CG preconditioner some steps later).
//
// Multifrontal over the supernodal assembly tree: each supernode's frontal
// matrix gathers its columns of A (lower part) and its children's update
// matrices (extend-add), is partially factored (dense LDL^T of the own
// columns, right-looking, blocked), and leaves the Schur complement on its
// struct rows as the update matrix passed to the parent.
//
// Output is the explicit-inverse form used by the GPU sweeps: per supernode
//   G = [ L11^{-1} ; L21 L11^{-1} ]   (m x nc, column-major),
// so that the forward sweep of a block is y_s = L11^{-1} w_s with the
// ancestors' right-hand sides updated by w_anc -= (L21 L11^{-1}) w_s, and
// the backward sweep is x_s = L11^{-T} (D^{-1} y_s) - (L21 L11^{-1})^T x_anc;
// both are dense matrix-vector products whose input is known when the level
// starts.  This is algebraically the triangular solve of Eq. "lower STS".
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstring>
#include <thread>

#include "host.hpp"

namespace fe {

void parallel_for(int64_t n, int n_threads, const std::function<void(int64_t, int)> &fn) {
  if (n <= 0) return;
  const int T = (int)std::max<int64_t>(1, std::min<int64_t>(n_threads, n));
  if (T == 1) {
    for (int64_t i = 0; i < n; ++i) fn(i, 0);
    return;
  }
  std::atomic<int64_t> next{0};
  auto worker = [&](int tid) {
    for (;;) {
      const int64_t i = next.fetch_add(1);
      if (i >= n) break;
      fn(i, tid);
    }
  };
  std::vector<std::thread> th;
  th.reserve(T - 1);
  for (int t = 1; t < T; ++t) th.emplace_back(worker, t);
  worker(0);
  for (auto &t : th) t.join();
}

namespace {

constexpr int kPanel = 48;  // column block of the dense partial factorisation
constexpr int kRowBlk = 96; // row block of the trailing update

// C[i, j] -= sum_k A[i, k] * Bt[j, k] for i in [i0, i1), j in [j0, j1) with
// i >= j (lower part only); A and C column-major (ld), Bt row-major [j][kb].
inline void update_block(double *C, int64_t ldc, const double *Acol, int64_t lda,
                         const double *Bt, int kb, int64_t i0, int64_t i1, int64_t j0,
                         int64_t j1) {
  for (int64_t j = j0; j < j1; j += 4) {
    const int jn = (int)std::min<int64_t>(4, j1 - j);
    const int64_t is = std::max(i0, j);
    if (is >= i1) continue;
    double w[4][kPanel];
    for (int jj = 0; jj < 4; ++jj)
      for (int k = 0; k < kb; ++k) w[jj][k] = jj < jn ? Bt[(j - j0 + jj) * kb + k] : 0.0;
    double *c0 = C + (j + 0) * ldc;
    double *c1 = C + (j + (jn > 1 ? 1 : 0)) * ldc;
    double *c2 = C + (j + (jn > 2 ? 2 : 0)) * ldc;
    double *c3 = C + (j + (jn > 3 ? 3 : 0)) * ldc;
    // rows below the 4x4 corner: straight 4-column update
    for (int64_t ib = is; ib < i1; ib += 64) {
      const int64_t ie = std::min(i1, ib + 64);
      double acc0[64], acc1[64], acc2[64], acc3[64];
      for (int64_t i = ib; i < ie; ++i) acc0[i - ib] = acc1[i - ib] = acc2[i - ib] = acc3[i - ib] = 0.0;
      for (int k = 0; k < kb; ++k) {
        const double *a = Acol + k * lda;
        const double w0 = w[0][k], w1 = w[1][k], w2 = w[2][k], w3 = w[3][k];
        for (int64_t i = ib; i < ie; ++i) {
          const double av = a[i];
          acc0[i - ib] += av * w0;
          acc1[i - ib] += av * w1;
          acc2[i - ib] += av * w2;
          acc3[i - ib] += av * w3;
        }
      }
      for (int64_t i = ib; i < ie; ++i) {
        c0[i] -= acc0[i - ib];
        if (jn > 1 && i >= j + 1) c1[i] -= acc1[i - ib];
        if (jn > 2 && i >= j + 2) c2[i] -= acc2[i - ib];
        if (jn > 3 && i >= j + 3) c3[i] -= acc3[i - ib];
      }
    }
  }
}

// Partial LDL^T of the m x m front F (column-major, lower part used) over its
// first nc columns.  Afterwards F[k,k] = d_k, F[i,k] = L[i,k] (i > k, k < nc)
// and F[nc:, nc:] holds the update matrix.  Threads parallelise the trailing
// update of large fronts.
std::string partial_ldlt(double *F, int64_t m, int64_t nc, int n_threads) {
  std::vector<double> Wt;
  for (int64_t k0 = 0; k0 < nc; k0 += kPanel) {
    const int kb = (int)std::min<int64_t>(kPanel, nc - k0);
    // factor the panel columns (rows k0..m)
    for (int64_t k = k0; k < k0 + kb; ++k) {
      double *Fk = F + k * m;
      const double d = Fk[k];
      if (!(d > 0.0) || !std::isfinite(d)) return "non-positive pivot in LDL^T";
      const double inv = 1.0 / d;
      for (int64_t j = k + 1; j < k0 + kb; ++j) {
        const double s = Fk[j] * inv;
        double *Fj = F + j * m;
        for (int64_t i = j; i < m; ++i) Fj[i] -= Fk[i] * s;
      }
      for (int64_t i = k + 1; i < m; ++i) Fk[i] *= inv;
    }
    // trailing update F[i, j] -= sum_k L[i,k] d_k L[j,k] for j >= k0 + kb
    const int64_t j_beg = k0 + kb;
    if (j_beg >= m) continue;
    const int64_t nt = m - j_beg;
    Wt.assign(nt * kb, 0.0);
    for (int64_t j = 0; j < nt; ++j)
      for (int k = 0; k < kb; ++k) {
        const double *Fk = F + (k0 + k) * m;
        Wt[j * kb + k] = Fk[j_beg + j] * Fk[k0 + k];  // L[j,k] * d_k
      }
    const double *Acol = F + k0 * m;
    const int64_t nblk = (nt + 15) / 16;
    auto body = [&](int64_t b, int) {
      const int64_t j0 = j_beg + b * 16, j1 = std::min(m, j0 + 16);
      update_block(F, m, Acol, m, Wt.data() + (j0 - j_beg) * kb, kb, j0, m, j0, j1);
    };
    const double work = (double)nt * nt * kb;
    parallel_for(nblk, work > 4e6 ? n_threads : 1, body);
  }
  return "";
}

}  // namespace

template <typename TA>
std::string factorize(const Pattern &P, const Symbolic &S, const TA *A, int n_threads,
                      std::vector<double> &panels, std::vector<double> &dinv) {
  const int32_t ns = (int32_t)S.sn.size();
  if (n_threads <= 0) n_threads = std::max(1u, std::thread::hardware_concurrency());
  panels.assign(S.panel_entries, 0.0);
  dinv.assign(S.n, 1.0);
  std::vector<std::vector<double>> update(ns);
  std::vector<std::string> err(ns);

  std::vector<std::vector<int32_t>> by_level(S.n_levels);
  for (int32_t s = 0; s < ns; ++s) by_level[S.sn[s].level].push_back(s);

  // per-thread DOF -> front position scratch
  std::vector<std::vector<int32_t>> relpos(n_threads, std::vector<int32_t>(S.n, -1));

  auto do_front = [&](int32_t s, int tid, int inner_threads) {
    const Supernode &sn = S.sn[s];
    const int64_t m = sn.m, nc = sn.nc;
    const int32_t *rows = S.rows.data() + sn.rows_off;
    std::vector<int32_t> &rp = relpos[tid];
    for (int64_t i = 0; i < m; ++i) rp[rows[i]] = (int32_t)i;
    std::vector<double> F((size_t)(m * m), 0.0);
    // assemble the own columns of A (lower part)
    for (int64_t j = 0; j < nc; ++j) {
      const int32_t d = rows[j];
      for (int32_t k = P.row_ptr[d]; k < P.row_ptr[d + 1]; ++k) {
        const int32_t c = P.col_idx[k];
        const int32_t pos = rp[c];
        if (pos >= j) F[j * m + pos] += (double)A[k];
      }
    }
    // extend-add children's update matrices
    for (int32_t c : S.children[s]) {
      const Supernode &cs = S.sn[c];
      const int64_t cnr = cs.m - cs.nc;
      const int32_t *crows = S.rows.data() + cs.rows_off + cs.nc;
      const std::vector<double> &U = update[c];
      for (int64_t jj = 0; jj < cnr; ++jj) {
        const int64_t pj = rp[crows[jj]];
        for (int64_t ii = jj; ii < cnr; ++ii) {
          const int64_t pi = rp[crows[ii]];
          // lower part of the parent front
          if (pi >= pj) F[pj * m + pi] += U[jj * cnr + ii];
          else F[pi * m + pj] += U[jj * cnr + ii];
        }
      }
      std::vector<double>().swap(update[c]);
    }
    std::string e = partial_ldlt(F.data(), m, nc, inner_threads);
    if (!e.empty()) {
      err[s] = e + " (supernode " + std::to_string(s) + ")";
      for (int64_t i = 0; i < m; ++i) rp[rows[i]] = -1;
      return;
    }
    // update matrix for the parent (lower part, column-major nr x nr)
    const int64_t nr = m - nc;
    if (nr > 0 && sn.parent >= 0) {
      std::vector<double> U((size_t)(nr * nr), 0.0);
      for (int64_t j = 0; j < nr; ++j)
        for (int64_t i = j; i < nr; ++i) U[j * nr + i] = F[(nc + j) * m + nc + i];
      update[s] = std::move(U);
    }
    for (int64_t k = 0; k < nc; ++k) dinv[rows[k]] = 1.0 / F[k * m + k];
    // explicit inverse of the unit lower L11 (column by column)
    double *G = panels.data() + sn.panel_off;  // m x nc column-major
    for (int64_t j = 0; j < nc; ++j) {
      double *g = G + j * m;
      g[j] = 1.0;
      for (int64_t k = j; k < nc; ++k) {
        const double xk = g[k];
        if (xk == 0.0) continue;
        const double *Lk = F.data() + k * m;
        for (int64_t i = k + 1; i < nc; ++i) g[i] -= Lk[i] * xk;
      }
    }
    // W = L21 L11^{-1}: W[:, j] = sum_{k >= j} L21[:, k] Linv[k, j]
    if (nr > 0) {
      auto wcol = [&](int64_t j, int) {
        double *w = G + j * m + nc;
        const double *linv = G + j * m;
        for (int64_t k = j; k < nc; ++k) {
          const double lk = linv[k];
          if (lk == 0.0) continue;
          const double *L21k = F.data() + k * m + nc;
          for (int64_t i = 0; i < nr; ++i) w[i] += L21k[i] * lk;
        }
      };
      const double work = (double)nr * nc * nc;
      parallel_for(nc, work > 4e6 ? inner_threads : 1, wcol);
    }
    for (int64_t i = 0; i < m; ++i) rp[rows[i]] = -1;
  };

  for (int32_t L = 0; L < S.n_levels; ++L) {
    const auto &lv = by_level[L];
    if ((int)lv.size() >= 2 * n_threads) {
      parallel_for((int64_t)lv.size(), n_threads,
                   [&](int64_t i, int tid) { do_front(lv[i], tid, 1); });
    } else {
      for (int32_t s : lv) do_front(s, 0, n_threads);
    }
    for (int32_t s : lv)
      if (!err[s].empty()) return err[s];
  }
  return "";
}

template std::string factorize<float>(const Pattern &, const Symbolic &, const float *, int,
                                      std::vector<double> &, std::vector<double> &);
template std::string factorize<double>(const Pattern &, const Symbolic &, const double *, int,
                                       std::vector<double> &, std::vector<double> &);

}  // namespace fe
