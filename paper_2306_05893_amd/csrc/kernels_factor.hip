// GPU multifrontal LDL^T factorisation in FP64 (the refactorisation of the
// stale preconditioner, run on the device instead of a host thread).
//
// Per nested-dissection level (leaves first):
//   init     zero the level's fronts; augmented block X = [I; 0]
//   scatter  lower part of the own columns of A into the fronts
//   extend   children's update matrices (the Schur complements left in the
//            trailing part of their fronts) added into the parent fronts,
//            one launch per child rank
//   panels   for k0 = 0, 64, ...: one workgroup per front factors the
//            64 x 64 diagonal block in registers; then one launch applies
//            the block to the rows below it (one thread per row, panel
//            values in registers) and its row operations to the panel rows
//            of X (one thread per column); then 64 x 64 FP64 FMA tiles
//            update the rest of the panel's 256-column block of F and the
//            block's own rows of X
//   blocks   after the last panel of a 256-column block: the block applied
//            to the own columns and own rows of X past it, in one pass
//            (K = 256) on the matrix cores, so that the trailing own columns
//            are read and written once per block rather than once per panel
//   schur    once the own columns are done: the Schur complement
//            F22 -= L21 D L21^T and the struct rows of X, -L21 X_own, in one
//            pass over each 128 x 128 output tile (K = nc; 64 x 64 on the
//            levels with too few large tiles to fill the GPU), on the
//            matrix cores (FP64 MFMA 16x16x4)
//   emit     G = [X own rows; -X struct rows] -> panel (FP32 or FP64), and
//            1/d into dinv
// The row operations of the elimination applied to X = [I; 0] leave
// X = [L11^{-1}; -L21 L11^{-1}], the explicit-inverse panel the triangular
// sweeps use (the same numbers as the host factorisation).
#include "device.hpp"
#include "host.hpp"

namespace fe {

namespace {

constexpr int NB = kGfPanel;

// Start of a level: own columns and update block of F zeroed, X = [I; 0].
// Fronts of the level by blockIdx.y (stride gridDim.y), grid-stride over the
// entries of a front along x.
__global__ void k_gf_init(const GfFront *fr, const int32_t *sn, int nf, double *base) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t i0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (int q = blockIdx.y; q < nf; q += gridDim.y) {
    const GfFront f = fr[sn[q]];
    const int64_t nF = (int64_t)f.m * f.nc, r = f.m - f.nc, nU = r * r;
    for (int64_t i = i0; i < nF; i += stride) base[f.offF + i] = 0.0;
    for (int64_t i = i0; i < nU; i += stride) base[f.offU + i] = 0.0;
    // X = [I; 0] row-major: the unit entries are i = t (nc + 1), t < nc, all
    // inside the leading nc x nc block (32-bit arithmetic when it fits)
    const int64_t nc2 = (int64_t)f.nc * f.nc;
    const uint32_t step = (uint32_t)f.nc + 1u;
    const bool small = nc2 < ((int64_t)1 << 32);
    for (int64_t i = i0; i < nF; i += stride) {
      const bool unit =
          i < nc2 && (small ? (uint32_t)i % step == 0u : i % (int64_t)step == 0);
      base[f.offX + i] = unit ? 1.0 : 0.0;
    }
  }
}

template <typename TA>
__global__ void k_gf_scatter(int64_t n, const int32_t *a_csr, const int64_t *a_off, const TA *A,
                             double *base) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
    base[a_off[i]] = (double)A[a_csr[i]];
}

// extend-add: 32 x 32 tiles of the children's update matrices (tile per
// block, stride gridDim.x), one launch per child rank.  Within a launch every
// parent receives from one child and the child's rows map one to one into
// the parent's, so each target entry is added by one thread: plain
// read-add-write, coalesced along the rows, instead of atomics.  Thread
// (tx, ty) adds entries (i0 + tx, j0 + ty + 8q), q < 4, of the lower
// triangle; the four loads of each kind are clamped into the block and issued
// together before the adds.
__global__ __launch_bounds__(256) void k_gf_extend(const GfExt *__restrict__ ext, int64_t n_ext,
                                                   const GfFront *__restrict__ fr,
                                                   const int32_t *__restrict__ parent,
                                                   const int32_t *__restrict__ rel,
                                                   const int64_t *__restrict__ rel_off,
                                                   double *base) {
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  for (int64_t e = blockIdx.x; e < n_ext; e += gridDim.x) {
    const GfExt t = ext[e];
    const GfFront fc = fr[t.child];
    const GfFront fp = fr[parent[t.child]];
    const int nr = fc.m - fc.nc;
    const int32_t *rl = rel + rel_off[t.child];
    const int ii = t.i0 + tx;
    if (ii >= nr) continue;
    const int pi = rl[ii];
    const int rp = fp.m - fp.nc;
    double u[4];
    int pj[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int jj = min(t.j0 + ty + 8 * q, nr - 1);
      u[q] = base[fc.offU + (int64_t)jj * nr + ii];
      pj[q] = rl[jj];
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int jj = t.j0 + ty + 8 * q;
      if (jj >= min(t.j0 + 32, nr) || ii < jj) continue;
      const int hi = max(pi, pj[q]), lo = min(pi, pj[q]);
      // own columns of the parent, or its update block
      const int64_t o = lo < fp.nc ? fp.offF + (int64_t)lo * fp.m + hi
                                   : fp.offU + (int64_t)(lo - fp.nc) * rp + (hi - fp.nc);
      base[o] += u[q];
    }
  }
}

// Diagonal block of the panel (columns [k0, k1)) of one front, one workgroup:
// right-looking LDL^T of the kb x kb block in registers.  Thread (tx, ty)
// of the 16 x 16 grid holds entries (ty + 16a, tx + 16b), a, b < 4, of the
// lower triangle; at pivot k the owners of column k publish it through LDS
// (double-buffered, one barrier per pivot) and every thread applies
//   D[r][c] -= D[r][k] D[c][k] / d_k   (c, r > k, r >= c).
// Output: d on the diagonal, L = D[r][c] / d_c below it.
__device__ void gf_diag(const GfFront f, int k0, double *base, int *status) {
  static_assert(NB == 64, "thread layout assumes a 64-wide panel");
  const int m = f.m, nc = f.nc;
  const int k1 = min(k0 + NB, nc), kb = k1 - k0;
  double *F = base + f.offF + (int64_t)k0 * m + k0;
  __shared__ double col[2][NB];
  __shared__ double dg[NB];
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  double e[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const int r = ty + 16 * a, c = tx + 16 * b;
      e[a][b] = (r < kb && c < kb && r >= c) ? F[(int64_t)c * m + r] : 0.0;
    }
  for (int k = 0; k < kb; ++k) {
    double *ck = col[k & 1];
    if (tx == (k & 15)) {
      const int bk = k >> 4;
#pragma unroll
      for (int a = 0; a < 4; ++a) {
        double x = e[a][0];
#pragma unroll
        for (int b = 1; b < 4; ++b) x = bk == b ? e[a][b] : x;
        ck[ty + 16 * a] = x;
      }
    }
    __syncthreads();
    double d = ck[k];
    if (!(d > 0.0)) {
      if (threadIdx.x == 0) atomicOr(status, 1);
      d = 1.0;  // keep going; the host discards this factor
    }
    if (threadIdx.x == 0) dg[k] = d;
    const double inv = 1.0 / d;
    double lr[4], cc[4];
#pragma unroll
    for (int a = 0; a < 4; ++a) lr[a] = ck[ty + 16 * a] * inv;
#pragma unroll
    for (int b = 0; b < 4; ++b) cc[b] = ck[tx + 16 * b];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        const int r = ty + 16 * a, c = tx + 16 * b;
        if (c > k && r >= c) e[a][b] -= lr[a] * cc[b];
      }
  }
  __syncthreads();
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const int r = ty + 16 * a, c = tx + 16 * b;
      if (r < kb && c < kb && r >= c) F[(int64_t)c * m + r] = r == c ? dg[c] : e[a][b] / dg[c];
    }
}

// one front of the step per block (stride gridDim.x)
__global__ __launch_bounds__(256) void k_gf_diag(const GfFront *fr, const int32_t *sn, int np, int k0,
                                                 double *base, int *status) {
  for (int q = blockIdx.x; q < np; q += gridDim.x) {
    gf_diag(fr[sn[q]], k0, base, status);
    __syncthreads();
  }
}

// Row operations of one panel step (one launch, two roles; the kb x kb
// diagonal block, already factored, staged in LDS):
//  * blockIdx.x < nrb: rows below the block, one thread per row with the kb
//    panel values in registers:
//      f_k <- f_k - sum_{c<k} f_c L_d[k][c],  W[i, k] = f_k,  l_k = f_k / d_k;
//  * otherwise: columns c < k1 of the panel rows of X, one thread per
//    column, forward substitution with the unit lower factor of the block:
//      x_r <- x_r - sum_{k<r} L_d[r][k] x_k.
// blockIdx.y = front of the step; chunks of 256 rows / 256 columns.
//
// Both roles run the right-looking elimination order: for k, for c > k,
// v[c] -= v[k] L_d[c][k].  The strictly lower entries of the block are
// packed in LDS in exactly that order (pair (k, c) at kPairIdx(k, c)), so
// the entries the next few dozen updates need are read as whole 8-entry
// chunks, kRing - 1 chunks ahead of their use, into a register ring: the
// LDS latency overlaps the arithmetic instead of stalling every update.
constexpr int kPairs = NB * (NB - 1) / 2;
constexpr int kChunk = 8;
constexpr int kChunks = kPairs / kChunk;
constexpr int kRing = 4;
static_assert(kPairs % kChunk == 0, "the packed block splits into whole chunks");

__host__ __device__ constexpr int kPairIdx(int k, int c) { return k * (2 * NB - k - 1) / 2 + (c - k - 1); }

struct PairRing {
  double2 r[kRing][kChunk / 2];
  __device__ __forceinline__ void load(const double *P, int chunk) {
    const double2 *src = reinterpret_cast<const double2 *>(P) + chunk * (kChunk / 2);
#pragma unroll
    for (int q = 0; q < kChunk / 2; ++q) r[chunk % kRing][q] = src[q];
  }
  __device__ __forceinline__ double at(int p) const {
    const double2 w = r[(p / kChunk) % kRing][(p % kChunk) / 2];
    return (p & 1) ? w.y : w.x;
  }
};

// SCALE: the rows role (store f_k to W before l_k = f_k / d_k); otherwise
// the X role (unit lower substitution only).  v[k] is final after step k and
// goes out at once (out(k, v[k])), so the registers of the finished entries
// are free for the ring.
template <bool SCALE, typename Out>
__device__ __forceinline__ void gf_subst(double (&v)[NB], const double *P, const double *dinv,
                                         double *W, int64_t m, uint32_t i, Out out) {
  PairRing ring;
#pragma unroll
  for (int j = 0; j < kRing - 1; ++j) ring.load(P, j);
#pragma unroll
  for (int k = 0; k < NB; ++k) {
    if (SCALE) (W + (int64_t)k * m)[i] = v[k];
#pragma unroll
    for (int c = k + 1; c < NB; ++c) {
      const int p = kPairIdx(k, c);
      if (p % kChunk == 0 && p / kChunk + kRing - 1 < kChunks) ring.load(P, p / kChunk + kRing - 1);
      if (SCALE) v[c] -= v[k] * ring.at(p);
      else v[c] -= ring.at(p) * v[k];
    }
    if (SCALE) v[k] *= dinv[k];
    out(k, v[k]);
  }
}

__device__ void gf_rowops(const GfFront f, int k0, int bx, int nrb, double *base) {
  const int m = f.m, nc = f.nc;
  const int k1 = min(k0 + NB, nc), kb = k1 - k0;
  const bool rows_role = bx < nrb;
  const int first = rows_role ? k1 + bx * 256 : (bx - nrb) * 256;
  if (first >= (rows_role ? m : k1)) return;  // whole block past this front's work
  double *F = base + f.offF;
  // strictly lower entries of the block in elimination order; the padding
  // (k or c >= kb, last panel of a front) is the identity: zero entries and
  // unit pivots, so that the unrolled loops below need no bounds tests
  __shared__ __align__(16) double P[kPairs];
  __shared__ double dinv[NB];
  for (int idx = threadIdx.x; idx < NB * NB; idx += 256) {
    const int k = idx / NB, c = idx % NB;
    if (c > k) P[kPairIdx(k, c)] = c < kb ? F[(int64_t)(k0 + k) * m + k0 + c] : 0.0;
  }
  if (threadIdx.x < NB) {
    const int k = threadIdx.x;
    dinv[k] = k < kb ? 1.0 / F[(int64_t)(k0 + k) * m + k0 + k] : 1.0;
  }
  __syncthreads();
  // Branch-free: loads clamped to the block's columns, and the stores of
  // the padding columns c >= kb (last panel of a front) sent to the unused
  // columns of the W scratch (m x NB; rows-role threads use rows >= k1 of
  // it and X-role threads rows < k1, so the two never meet).
  const uint32_t i = (uint32_t)(first + (int)threadIdx.x);
  double *W = base + f.offW;
  double v[NB];
  if (rows_role) {
    if (i >= (uint32_t)m) return;
    double *Fk = F + (int64_t)k0 * m;
#pragma unroll
    for (int c = 0; c < NB; ++c) {
      const double x = (Fk + (int64_t)min(c, kb - 1) * m)[i];
      v[c] = c < kb ? x : 0.0;
    }
    gf_subst<true>(v, P, dinv, W, m, i,
                   [&](int c, double x) { ((c < kb ? Fk : W) + (int64_t)c * m)[i] = x; });
  } else {
    if (i >= (uint32_t)k1) return;
    double *Xk = base + f.offX + (int64_t)k0 * nc;
#pragma unroll
    for (int r = 0; r < NB; ++r) {
      const double x = (Xk + (int64_t)min(r, kb - 1) * nc)[i];
      v[r] = r < kb ? x : 0.0;
    }
    gf_subst<false>(v, P, dinv, W, m, i, [&](int r, double x) {
      double *dst = r < kb ? Xk + (int64_t)r * nc : W + (int64_t)r * m;
      dst[i] = x;
    });
  }
}

// blockIdx.x = role chunk, blockIdx.y = front of the step
__global__ __launch_bounds__(256) void k_gf_rowops(const GfFront *fr, const int32_t *sn, int k0,
                                                   int nrb, double *base) {
  gf_rowops(fr[sn[blockIdx.y]], k0, (int)blockIdx.x, nrb, base);
}

// One TL x TL output tile of an update (regions as in GfTile; TL/16 x TL/16
// outputs per thread, loaded into the accumulators before the first stage).
// The k range is staged through LDS 32 rows at a time: sA = L[i, k] (rows of
// the tile), sB = W[j, k], d_k L[j, k] or X[k, j] (columns of the tile).
template <int TL>
__device__ void gf_update(const GfTile t, const GfFront f, int k0, double *base) {
  constexpr int KC = 32;
  const int m = f.m, nc = f.nc;
  const int reg = t.region;
  int kbeg, kend, imax, jmax;
  if (reg == 0) {
    kbeg = k0, kend = min(k0 + NB, nc), imax = m, jmax = nc;
  } else if (reg == 1) {
    kbeg = k0, kend = min(k0 + NB, nc), imax = nc, jmax = kend;
  } else if (reg == 2) {
    kbeg = 0, kend = nc, imax = m, jmax = m;
  } else {
    kbeg = t.j0, kend = nc, imax = m, jmax = nc;  // X[k, j] = 0 for k < j
  }
  double *F = base + f.offF;
  double *X = base + f.offX;
  const double *W = base + f.offW;
  double *U = base + f.offU;  // region 2: entry (i, j) at (j - nc) * (m - nc) + i - nc
  const int64_t ru = m - nc;
  __shared__ double sA[KC][TL + 2];
  __shared__ double sB[KC][TL + 2];
  const int tid = threadIdx.x;
  const int tx = tid & 15, ty = tid >> 4;
  constexpr int R = TL / 16;
  // F outputs (column-major): thread rows tx + 16u, so consecutive threads
  // touch consecutive rows; X outputs (row-major): thread columns tx + 16v
  const bool fout = reg == 0 || reg == 2;
  const int ra = fout ? tx : ty, cb = fout ? ty : tx;
  // accumulators preloaded with the outputs' current values; the loads are
  // clamped into the region and unconditional (entries outside it are
  // computed on but never stored)
  double acc[R][R];
  int ii[R], jj[R];
#pragma unroll
  for (int u = 0; u < R; ++u) {
    ii[u] = min(t.i0 + ra + 16 * u, imax - 1);
    jj[u] = min(t.j0 + cb + 16 * u, jmax - 1);
  }
  if (reg == 0) {
#pragma unroll
    for (int u = 0; u < R; ++u)
#pragma unroll
      for (int v = 0; v < R; ++v) acc[u][v] = F[(int64_t)jj[v] * m + ii[u]];
  } else if (reg == 2) {
#pragma unroll
    for (int u = 0; u < R; ++u)
#pragma unroll
      for (int v = 0; v < R; ++v) acc[u][v] = U[(jj[v] - nc) * ru + (ii[u] - nc)];
  } else {
#pragma unroll
    for (int u = 0; u < R; ++u)
#pragma unroll
      for (int v = 0; v < R; ++v) acc[u][v] = X[(int64_t)ii[u] * nc + jj[v]];
  }
  // staging: thread (r, kq) fills column r of rows k = kq + KS q of both
  // operands; the loads are clamped into the front and unconditional, so a
  // batch of them is in flight at once, and the out-of-range entries are
  // zeroed when they are written to LDS
  constexpr int KS = 256 / TL;            // k rows staged per pass of the block
  constexpr int NPASS = 4;                // load batches per stage
  constexpr int QH = KC / KS / NPASS;     // entries per thread per batch
  const int sr = tid % TL, kq = tid / TL;
  const bool iok = t.i0 + sr < imax, jok = t.j0 + sr < jmax;
  const int si = min(t.i0 + sr, imax - 1), sj = min(t.j0 + sr, jmax - 1);
  for (int kc0 = kbeg; kc0 < kend; kc0 += KC) {
    const int kn = min(KC, kend - kc0);
    if (kc0 > kbeg) __syncthreads();
#pragma unroll
    for (int h = 0; h < NPASS; ++h) {
      double a[QH], b[QH];
      int kk[QH];
#pragma unroll
      for (int q = 0; q < QH; ++q) {
        kk[q] = kc0 + min(kq + KS * (q + QH * h), kn - 1);
        a[q] = F[(int64_t)kk[q] * m + si];
      }
      if (reg == 0) {
#pragma unroll
        for (int q = 0; q < QH; ++q) b[q] = W[(int64_t)(kk[q] - k0) * m + sj];
      } else if (reg == 2) {
        double dk[QH];
#pragma unroll
        for (int q = 0; q < QH; ++q) {
          b[q] = F[(int64_t)kk[q] * m + sj];
          dk[q] = F[(int64_t)kk[q] * m + kk[q]];
        }
#pragma unroll
        for (int q = 0; q < QH; ++q) b[q] *= dk[q];
      } else {
#pragma unroll
        for (int q = 0; q < QH; ++q) b[q] = X[(int64_t)kk[q] * nc + sj];
      }
#pragma unroll
      for (int q = 0; q < QH; ++q) {
        const int k = kq + KS * (q + QH * h);
        sA[k][sr] = (k < kn && iok) ? a[q] : 0.0;
        sB[k][sr] = (k < kn && jok) ? b[q] : 0.0;
      }
    }
    __syncthreads();
    for (int k = 0; k < kn; ++k) {
      double a[R], bb[R];
#pragma unroll
      for (int u = 0; u < R; ++u) {
        a[u] = sA[k][ra + 16 * u];
        bb[u] = sB[k][cb + 16 * u];
      }
#pragma unroll
      for (int u = 0; u < R; ++u)
#pragma unroll
        for (int v = 0; v < R; ++v) acc[u][v] = fma(-a[u], bb[v], acc[u][v]);
    }
  }
  // stores: in range, and on or below the diagonal for the F outputs
  if (reg == 0) {
#pragma unroll
    for (int u = 0; u < R; ++u)
#pragma unroll
      for (int v = 0; v < R; ++v) {
        const int i = t.i0 + ra + 16 * u, j = t.j0 + cb + 16 * v;
        if (i < imax && j < jmax && i >= j) F[(int64_t)j * m + i] = acc[u][v];
      }
  } else if (reg == 2) {
#pragma unroll
    for (int u = 0; u < R; ++u)
#pragma unroll
      for (int v = 0; v < R; ++v) {
        const int i = t.i0 + ra + 16 * u, j = t.j0 + cb + 16 * v;
        if (i < imax && j < jmax && i >= j) U[(j - nc) * ru + (i - nc)] = acc[u][v];
      }
  } else {
#pragma unroll
    for (int u = 0; u < R; ++u)
#pragma unroll
      for (int v = 0; v < R; ++v) {
        const int i = t.i0 + ra + 16 * u, j = t.j0 + cb + 16 * v;
        if (i < imax && j < jmax) X[(int64_t)i * nc + j] = acc[u][v];
      }
  }
}

// The same update on the matrix cores: FP64 MFMA 16x16x4.  The LDS stages
// are filled exactly as in gf_update; each of the four wavefronts owns a
// TL/2 x TL/2 quadrant of the output tile as (TL/32)^2 blocks of 16 x 16.
// An MFMA block's result holds, in register q of lane l, column l % 16 of
// row 4q + l / 16, so the instruction is oriented per region so that the 16
// lanes of a register run along the output's contiguous index: rows i for
// the column-major F and U outputs (regions 0, 2 and 4), columns j for the
// row-major X outputs (regions 1, 3 and 5).  "fast" below is that index,
// "slow" the other one; the slow operand is negated, so that each MFMA
// subtracts its product from the accumulators.
typedef double gf_d4 __attribute__((ext_vector_type(4)));

template <int TL>
__device__ void gf_update_mfma(const GfTile t, const GfFront f, int k0, double *base) {
  constexpr int KC = 16;
  constexpr int NBK = TL / 32;  // 16 x 16 blocks per wavefront quadrant edge
  const int m = f.m, nc = f.nc;
  const int reg = t.region;
  int kbeg, kend, imax, jmax;
  if (reg == 0) {
    kbeg = k0, kend = min(k0 + NB, nc), imax = m, jmax = nc;
  } else if (reg == 1) {
    kbeg = k0, kend = min(k0 + NB, nc), imax = nc, jmax = kend;
  } else if (reg == 2) {
    kbeg = 0, kend = nc, imax = m, jmax = m;
  } else if (reg == 3) {
    kbeg = t.j0, kend = nc, imax = m, jmax = nc;  // X[k, j] = 0 for k < j
  } else if (reg == 4) {
    kbeg = k0, kend = min(k0 + kGfBlock, nc), imax = m, jmax = nc;  // k0: the block start
  } else {
    kbeg = max(k0, t.j0), kend = min(k0 + kGfBlock, nc), imax = nc, jmax = nc;
  }
  double *F = base + f.offF;
  double *X = base + f.offX;
  const double *W = base + f.offW;
  double *U = base + f.offU;
  const int64_t ru = m - nc;
  __shared__ double sA[KC][TL + 2];
  __shared__ double sB[KC][TL + 2];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const bool fout = reg == 0 || reg == 2 || reg == 4;  // column-major F or U output
  const bool fl = reg == 0 || reg == 4;                // F output
  // quadrant of this wavefront and the output index of each accumulator
  const int wf = (wv & 1) * (TL / 2), ws = (wv >> 1) * (TL / 2);
  const int fbase = fout ? t.i0 : t.j0, sbase = fout ? t.j0 : t.i0;
  const int fmax = fout ? imax : jmax, smax = fout ? jmax : imax;
  const int lf = lane & 15, ls = lane >> 4;
  gf_d4 acc[NBK][NBK];
#pragma unroll
  for (int sb = 0; sb < NBK; ++sb)
#pragma unroll
    for (int fb = 0; fb < NBK; ++fb)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int fi = min(fbase + wf + 16 * fb + lf, fmax - 1);
        const int si = min(sbase + ws + 16 * sb + 4 * q + ls, smax - 1);
        double v;
        if (fl) v = F[(int64_t)si * m + fi];
        else if (reg == 2) v = U[(si - nc) * ru + (fi - nc)];
        else v = X[(int64_t)si * nc + fi];
        acc[sb][fb][q] = v;
      }
  // Staging: thread (sr, kq) holds column sr of the rows k = kq + KS q of
  // both operands.  The whole next chunk is fetched into registers while
  // the current one is multiplied out of LDS (the loads are clamped into the
  // range and unconditional; the rows past the range are zeroed when written
  // to LDS), so a chunk's loads are in flight for a chunk's worth of matrix
  // work.  For the L D L^T products (regions 2 and 4) the pivots d_k of the
  // chunk go to sD and scale the slow operand as it is read.
  constexpr int KS = 256 / TL;  // k rows per pass of the block
  constexpr int QN = KC / KS;   // staged entries per thread and operand
  const int sr = tid % TL, kq = tid / TL;
  const bool iok = t.i0 + sr < imax, jok = t.j0 + sr < jmax;
  const int si_ = min(t.i0 + sr, imax - 1), sj_ = min(t.j0 + sr, jmax - 1);
  const bool scale = reg == 2 || reg == 4;
  __shared__ double sD[KC];
  double(*fast)[TL + 2] = fout ? sA : sB;
  double(*slow)[TL + 2] = fout ? sB : sA;
  double pa[QN], pb[QN], pd = 0.0;
  auto fetch = [&](int kc0) {
    const int kn = min(KC, kend - kc0);
#pragma unroll
    for (int q = 0; q < QN; ++q) pa[q] = F[(int64_t)(kc0 + min(kq + KS * q, kn - 1)) * m + si_];
    // a pivot per thread, in every region (a load only some threads or some
    // regions make would leave the compiler waiting for the whole fetch
    // before the products)
    const int kd = kc0 + min(tid, kn - 1);
    pd = F[(int64_t)kd * m + kd];
    if (reg == 0) {
#pragma unroll
      for (int q = 0; q < QN; ++q)
        pb[q] = W[(int64_t)(kc0 + min(kq + KS * q, kn - 1) - k0) * m + sj_];
    } else if (scale) {
#pragma unroll
      for (int q = 0; q < QN; ++q) pb[q] = F[(int64_t)(kc0 + min(kq + KS * q, kn - 1)) * m + sj_];
    } else {
#pragma unroll
      for (int q = 0; q < QN; ++q)
        pb[q] = X[(int64_t)(kc0 + min(kq + KS * q, kn - 1)) * nc + sj_];
    }
  };
  if (kbeg < kend) fetch(kbeg);
  for (int kc0 = kbeg; kc0 < kend; kc0 += KC) {
    const int kn = min(KC, kend - kc0);
    if (kc0 > kbeg) __syncthreads();  // the previous chunk's products are done with LDS
#pragma unroll
    for (int q = 0; q < QN; ++q) {
      const int k = kq + KS * q;
      sA[k][sr] = (k < kn && iok) ? pa[q] : 0.0;
      sB[k][sr] = (k < kn && jok) ? pb[q] : 0.0;
    }
    if (scale && tid < KC) sD[tid] = pd;
    __syncthreads();
    if (kc0 + KC < kend) fetch(kc0 + KC);
    // the staged rows k >= kn are zero, so whole steps of 4 are taken
    for (int k = 0; k < kn; k += 4) {
      double av[NBK], bv[NBK];
      const double dk = scale ? sD[k + ls] : 1.0;
#pragma unroll
      for (int sb = 0; sb < NBK; ++sb) av[sb] = -(slow[k + ls][ws + 16 * sb + lf] * dk);
#pragma unroll
      for (int fb = 0; fb < NBK; ++fb) bv[fb] = fast[k + ls][wf + 16 * fb + lf];
#pragma unroll
      for (int sb = 0; sb < NBK; ++sb)
#pragma unroll
        for (int fb = 0; fb < NBK; ++fb)
          acc[sb][fb] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[sb], bv[fb], acc[sb][fb], 0, 0, 0);
    }
  }
  // stores: in range, and on or below the diagonal for the F outputs
#pragma unroll
  for (int sb = 0; sb < NBK; ++sb)
#pragma unroll
    for (int fb = 0; fb < NBK; ++fb)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int fi = fbase + wf + 16 * fb + lf;
        const int si = sbase + ws + 16 * sb + 4 * q + ls;
        const int i = fout ? fi : si, j = fout ? si : fi;
        if (i >= imax || j >= jmax) continue;
        const double v = acc[sb][fb][q];
        if (fl) {
          if (i >= j) F[(int64_t)j * m + i] = v;
        } else if (reg == 2) {
          if (i >= j) U[(j - nc) * ru + (i - nc)] = v;
        } else {
          X[(int64_t)i * nc + j] = v;
        }
      }
}

// Tile of workgroup blockIdx.x in the round of gridDim.x tiles starting at
// r0.  The hardware hands workgroup b to XCD b % 8, the XCD's k-th being
// b = 8 k + x; in a full round of 512-tile spans, XCD x takes tiles
// 64 x .. 64 x + 63 of each span in turn, so the tiles in flight on one XCD
// (two per CU) are 64 consecutive tiles of the list, which the plan orders
// in 8 x 8 super-blocks of a front.  The rest of the round keeps the plain
// order.
__device__ inline int64_t gf_tile_of(int64_t r0, int64_t n_tiles) {
  const int64_t g = gridDim.x / 512 * 512, b = blockIdx.x;
  if (b < g && r0 + g <= n_tiles) {
    const int64_t k = b / 8;
    return r0 + (k / 64) * 512 + (b % 8) * 64 + k % 64;
  }
  return r0 + b;
}

// The next chunk's loads overlap the current chunk's matrix work inside the
// workgroup (the 128-wide tiles hold their accumulators and the fetched
// chunk in the full register file, one workgroup per CU).
template <int TL>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void k_gf_update_mfma(
    const GfTile *tiles, int64_t n_tiles, const GfFront *fr, int k0, double *base) {
  for (int64_t r0 = 0; r0 + blockIdx.x < n_tiles; r0 += gridDim.x) {
    const GfTile t = tiles[gf_tile_of(r0, n_tiles)];
    gf_update_mfma<TL>(t, fr[t.s], k0, base);
    __syncthreads();
  }
}

// one tile per block (stride gridDim.x)
template <int TL>
__global__ __launch_bounds__(256) void k_gf_update(const GfTile *tiles, int64_t n_tiles,
                                                   const GfFront *fr, int k0, double *base) {
  for (int64_t q = blockIdx.x; q < n_tiles; q += gridDim.x) {
    const GfTile t = tiles[q];
    gf_update<TL>(t, fr[t.s], k0, base);
    __syncthreads();
  }
}

// panel G (m x nc column-major) from X (row-major) and 1/d: 64 x 64 tiles
// transposed through LDS, so that both the reads of X and the writes of G
// are coalesced; fronts of the level by blockIdx.y (stride gridDim.y), tiles
// of a front by blockIdx.x (stride gridDim.x)
constexpr int kEmitTile = 64;

template <typename T>
__global__ __launch_bounds__(256) void k_gf_emit(const GfFront *fr, const int32_t *sn, int nf,
                                                 const double *base, const int32_t *rows,
                                                 T *panels, T *dinv) {
  constexpr int E = kEmitTile, RP = 256 / E;  // rows (columns) per pass
  __shared__ double tile[E][E + 1];
  const int c = threadIdx.x % E, rq = threadIdx.x / E;
  for (int q = blockIdx.y; q < nf; q += gridDim.y) {
    const GfFront f = fr[sn[q]];
    const int m = f.m, nc = f.nc;
    const int ti = (m + E - 1) / E, tj = (nc + E - 1) / E;
    const double *X = base + f.offX;
    T *G = panels + f.panel_off;
    for (int t = blockIdx.x; t < ti * tj; t += gridDim.x) {
      const int i0 = (t % ti) * E, j0 = (t / ti) * E;
      const int jc = min(j0 + c, nc - 1);
      double v[E / RP];
#pragma unroll
      for (int u = 0; u < E / RP; ++u) v[u] = X[(int64_t)min(i0 + rq + RP * u, m - 1) * nc + jc];
      __syncthreads();  // the previous tile's reads of LDS are done
#pragma unroll
      for (int u = 0; u < E / RP; ++u) tile[rq + RP * u][c] = v[u];
      __syncthreads();
      const int i = i0 + c;
#pragma unroll
      for (int u = 0; u < E / RP; ++u) {
        const int j = j0 + rq + RP * u;
        const double x = tile[c][rq + RP * u];
        if (i < m && j < nc) G[(int64_t)j * f.ld + i] = (T)(i < nc ? x : -x);
      }
    }
    if (blockIdx.x == 0) {
      const int32_t *rw = rows + f.rows_off;
      const double *F = base + f.offF;
      for (int k = threadIdx.x; k < f.nc; k += blockDim.x)
        dinv[rw[k]] = (T)(1.0 / F[(int64_t)k * f.m + k]);
    }
  }
}

}  // namespace

constexpr int64_t kLevelBlocks = 16384;  // workgroups of the init, extend-add and emit launches

template <typename TA, typename T>
void launch_gpu_factor(hipStream_t st, const GfPlan &P, const GfDev &d, const TA *A, T *panels,
                       T *dinv) {
  // grid of (gx x gy) workgroups for gx x gy work items, within the bound
  const int64_t cap = d.max_blocks > 0 ? d.max_blocks : INT64_MAX;
  auto grid1 = [&](int64_t n) { return (unsigned)std::max<int64_t>(1, std::min(n, cap)); };
  auto grid2 = [&](int64_t gx, int64_t gy) {
    gx = std::max<int64_t>(1, std::min(gx, cap));
    gy = std::max<int64_t>(1, std::min(gy, std::max<int64_t>(1, cap / gx)));
    return dim3((unsigned)gx, (unsigned)std::min<int64_t>(gy, 65535));
  };
  const int nl = (int)P.lvl_ptr.size() - 1;
  for (int L = 0; L < nl; ++L) {
    const int f0 = P.lvl_ptr[L], nf = P.lvl_ptr[L + 1] - f0;
    if (nf == 0) continue;
    int64_t maxz = 0;
    for (int k = f0; k < f0 + nf; ++k) {
      const GfFront &g = P.fr[P.lvl_sn[k]];
      maxz = std::max<int64_t>(maxz, std::max<int64_t>((int64_t)g.m * g.nc,
                                                       (int64_t)(g.m - g.nc) * (g.m - g.nc)));
    }
    // about kLevelBlocks workgroups per level whatever the number of fronts
    // (the kernel strides over fronts and entries): one row of workgroups
    // per front sized for the largest would launch millions of idle ones on
    // the leaf levels and too few for a lone top front
    const int64_t gy = std::min<int64_t>(nf, 65535);
    const int64_t zx = std::max<int64_t>(
        1, std::min<int64_t>((maxz + 255) / 256, kLevelBlocks / gy));
    k_gf_init<<<grid2(zx, gy), 256, 0, st>>>(d.fr, d.lvl_sn + f0, nf, d.fronts);
    const int64_t a0 = P.a_ptr[L], na = P.a_ptr[L + 1] - a0;
    if (na > 0)
      k_gf_scatter<TA><<<grid1((na + 255) / 256), 256, 0, st>>>(na, d.a_csr + a0, d.a_off + a0, A,
                                                                 d.fronts);
    const int p_end = L + 1 < nl ? P.ext_lvl_pass[L + 1] : (int)P.ext_pass.size() - 1;
    for (int pass = P.ext_lvl_pass[L]; pass < p_end; ++pass) {
      const int64_t e0 = P.ext_pass[pass], ne = P.ext_pass[pass + 1] - e0;
      if (ne > 0)
        k_gf_extend<<<grid1(std::min<int64_t>(ne, kLevelBlocks)), 256, 0, st>>>(
            d.ext + e0, ne, d.fr, d.parent, d.rel, d.rel_off, d.fronts);
    }
    for (int s = P.lvl_step_ptr[L]; s < P.lvl_step_ptr[L + 1]; ++s) {
      const int k0 = P.step_k0[s];
      const int64_t p0 = P.panel_ptr[s], np = P.panel_ptr[s + 1] - p0;
      if (np > 0) {
        k_gf_diag<<<grid1(np), 256, 0, st>>>(d.fr, d.panel_sn + p0, (int)np, k0, d.fronts,
                                             d.status);
        int maxrows = 0;
        for (int64_t q = p0; q < p0 + np; ++q) {
          const GfFront &g = P.fr[P.panel_sn[q]];
          maxrows = std::max(maxrows, g.m - std::min(k0 + NB, g.nc));
        }
        const int nrb = (maxrows + 255) / 256;
        const int ncb = (k0 + NB + 255) / 256;  // columns [0, k1) of X, k1 <= k0 + NB
        // fronts in launches of at most the bound (the role chunks of a front
        // stay in one launch)
        const int64_t fy = std::max<int64_t>(1, std::min<int64_t>(65535, cap / (nrb + ncb)));
        for (int64_t q0 = 0; q0 < np; q0 += fy)
          k_gf_rowops<<<dim3((unsigned)(nrb + ncb), (unsigned)std::min(fy, np - q0)), 256, 0,
                        st>>>(d.fr, d.panel_sn + p0 + q0, k0, nrb, d.fronts);
      }
      const int64_t u0 = P.upd_lo[s], nu = P.upd_hi[s] - u0;
      if (nu > 0)
        k_gf_update<kGfStepTile><<<grid1(nu), 256, 0, st>>>(d.upd + u0, nu, d.fr, k0, d.fronts);
      const int64_t b0 = P.blk_lo[s], nb = P.blk_hi[s] - b0;
      if (nb > 0 && P.blk_tile[s] == kGfTile)
        k_gf_update_mfma<kGfTile><<<grid1(nb), 256, 0, st>>>(d.upd + b0, nb, d.fr, P.blk_k0[s],
                                                             d.fronts);
      else if (nb > 0)
        k_gf_update_mfma<kGfStepTile><<<grid1(nb), 256, 0, st>>>(d.upd + b0, nb, d.fr,
                                                                 P.blk_k0[s], d.fronts);
    }
    const int64_t h0 = P.schur_lo[L], nh = P.schur_hi[L] - h0;
    if (nh > 0 && P.schur_tile[L] == kGfTile)
      k_gf_update_mfma<kGfTile><<<grid1(nh), 256, 0, st>>>(d.upd + h0, nh, d.fr, 0, d.fronts);
    else if (nh > 0)
      k_gf_update_mfma<kGfStepTile><<<grid1(nh), 256, 0, st>>>(d.upd + h0, nh, d.fr, 0,
                                                               d.fronts);
    int64_t maxt = 0;
    for (int k = f0; k < f0 + nf; ++k) {
      const GfFront &g = P.fr[P.lvl_sn[k]];
      maxt = std::max<int64_t>(maxt, (int64_t)((g.m + kEmitTile - 1) / kEmitTile) *
                                         ((g.nc + kEmitTile - 1) / kEmitTile));
    }
    const int64_t ey = std::min<int64_t>(nf, 65535);
    const int64_t gx = std::max<int64_t>(1, std::min<int64_t>(maxt, kLevelBlocks / ey));
    k_gf_emit<T><<<grid2(gx, ey), 256, 0, st>>>(d.fr, d.lvl_sn + f0, nf, d.fronts, d.rows, panels,
                                                dinv);
  }
}

template void launch_gpu_factor<float, float>(hipStream_t, const GfPlan &, const GfDev &,
                                              const float *, float *, float *);
template void launch_gpu_factor<double, double>(hipStream_t, const GfPlan &, const GfDev &,
                                                const double *, double *, double *);

}  // namespace fe
