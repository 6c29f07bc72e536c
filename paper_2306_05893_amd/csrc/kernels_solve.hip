// Solve kernels: CSR SpMV, the CG vector operations and control scalars, the
// Jacobi fallback, the level-scheduled triangular sweeps of the LDL^T
// preconditioner, and the backward-Euler update (paper Sec. 5 and Fig.
// "DataTransfer": the whole preconditioned CG runs on the GPU and only a
// small status word is read back).
//
// Determinism: dot products are reduced per block into a partial array and
// summed by a one-block control kernel in a fixed order.  The triangular
// sweeps accumulate with atomics (as the paper's column-major lower solve
// does), so the preconditioner output is correct to rounding but its
// summation order is not fixed.
#include "device.hpp"

namespace fe {

namespace {

constexpr int kBlock = 256;

__device__ inline double wave_sum(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// block-wide sum; result valid in thread 0
__device__ inline double block_sum(double v) {
  __shared__ double s_part[kBlock / 64];
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0) s_part[w] = v;
  __syncthreads();
  double r = 0.0;
  if (threadIdx.x == 0)
    for (int i = 0; i < (int)(blockDim.x >> 6); ++i) r += s_part[i];
  __syncthreads();
  return r;
}

// ------------------------------------------------------------------- SpMV
// G lanes per row, FP64 products and row sums of T-valued entries.  Each lane
// issues the index and value loads of its first U entries at once (clamped
// to the row, so without branches), then the U gathers of x, so that a row
// costs three memory latencies; longer rows finish in a loop.
template <typename T, int G>
__global__ __launch_bounds__(kBlock) void k_spmv(int64_t n, const int32_t *__restrict__ row_ptr,
                                                 const int32_t *__restrict__ col,
                                                 const T *__restrict__ val,
                                                 const double *__restrict__ x, double *__restrict__ y,
                                                 const double *__restrict__ w, double *part,
                                                 const PcgState *state) {
  if (state && state->done) return;
  constexpr int U = 6;
  const int64_t row = ((int64_t)blockIdx.x * kBlock + threadIdx.x) / G;
  const int sub = threadIdx.x & (G - 1);
  double sum = 0.0;
  if (row < n) {
    const int32_t k0 = row_ptr[row], k1 = row_ptr[row + 1];
    int32_t c[U];
    T v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int32_t k = min(k0 + sub + u * G, k1 - 1);
      c[u] = col[k];
      v[u] = val[k];
    }
    double xv[U];
#pragma unroll
    for (int u = 0; u < U; ++u) xv[u] = x[c[u]];
#pragma unroll
    for (int u = 0; u < U; ++u)
      if (k0 + sub + u * G < k1) sum += (double)v[u] * xv[u];
    for (int32_t k = k0 + sub + U * G; k < k1; k += G) sum += (double)val[k] * x[col[k]];
  }
  for (int off = G / 2; off > 0; off >>= 1) sum += __shfl_xor(sum, off, G);
  double d = 0.0;
  if (row < n && sub == 0) {
    y[row] = sum;
    if (w) d = w[row] * sum;
  }
  if (part) {
    d = block_sum(d);
    if (threadIdx.x == 0) part[blockIdx.x] = d;
  }
}

// ---------------------------------------------------------------- CG ops
__global__ __launch_bounds__(kBlock) void k_residual(int64_t n, const double *b, const double *Ax,
                                                     double *r, double *part_rr, double *part_bb) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  double rr = 0.0, bb = 0.0;
  if (i < n) {
    const double ri = b[i] - Ax[i];
    r[i] = ri;
    rr = ri * ri;
    bb = b[i] * b[i];
  }
  rr = block_sum(rr);
  bb = block_sum(bb);
  if (threadIdx.x == 0) {
    part_rr[blockIdx.x] = rr;
    if (part_bb) part_bb[blockIdx.x] = bb;
  }
}

__device__ inline double sum_parts(const double *p, int np) {
  // one block: fixed-order strided sums (8 independent accumulators, so that
  // 8 loads are in flight per thread) then a fixed tree
  double a[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  int i = threadIdx.x;
  for (; i + 7 * kBlock < np; i += 8 * kBlock)
#pragma unroll
    for (int u = 0; u < 8; ++u) a[u] += p[i + u * kBlock];
  for (; i < np; i += kBlock) a[0] += p[i];
  const double v = ((a[0] + a[1]) + (a[2] + a[3])) + ((a[4] + a[5]) + (a[6] + a[7]));
  return block_sum(v);
}

__global__ __launch_bounds__(kBlock) void k_ctl_init(PcgState *s, const double *prr,
                                                     const double *pbb, int np, double rel_tol) {
  const double rr = sum_parts(prr, np);
  const double bb = sum_parts(pbb, np);
  if (threadIdx.x == 0) {
    s->rr = rr;
    s->bb = bb;
    s->tol2 = rel_tol * rel_tol * bb;
    s->it = 0;
    s->status = 0;
    s->done = (bb == 0.0 || rr <= s->tol2) ? 1 : 0;
    s->rr_true = rr;
  }
}

__global__ __launch_bounds__(kBlock) void k_dot(int64_t n, const double *a, const double *b,
                                                double *part, const PcgState *state) {
  if (state && state->done) return;
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  double v = i < n ? a[i] * b[i] : 0.0;
  v = block_sum(v);
  if (threadIdx.x == 0) part[blockIdx.x] = v;
}

// rz <- r.z; beta = rz_new / rz_old (first: no beta)
__global__ __launch_bounds__(kBlock) void k_ctl_rz(PcgState *s, const double *part, int np,
                                                   int first) {
  if (s->done) return;
  const double rz = sum_parts(part, np);
  if (threadIdx.x == 0) {
    s->beta = first ? 0.0 : rz / s->rz;
    s->rz = rz;
  }
}

// First stage of a long partial sum: block b adds in[b * kPartChunk ..) in a
// fixed order (each thread a strided run, then the block's tree) into
// out[b], so that the one-block control kernel after it sums a few dozen
// values instead of one per SpMV block (87 k on the largest mesh).
constexpr int kPartChunk = 2048;

__global__ __launch_bounds__(kBlock) void k_part_reduce(const double *in, int n, double *out,
                                                        const PcgState *s) {
  if (s->done) return;
  const int64_t lo = (int64_t)blockIdx.x * kPartChunk, hi = min((int64_t)n, lo + kPartChunk);
  double t = 0.0;
  for (int64_t i = lo + threadIdx.x; i < hi; i += kBlock) t += in[i];
  t = block_sum(t);
  if (threadIdx.x == 0) out[blockIdx.x] = t;
}

__global__ __launch_bounds__(kBlock) void k_ctl_alpha(PcgState *s, const double *part, int np) {
  if (s->done) return;
  const double pAp = sum_parts(part, np);
  if (threadIdx.x == 0) {
    s->pAp = pAp;
    if (!(pAp > 0.0)) {
      s->status = 4;
      s->done = 1;
      s->alpha = 0.0;
    } else {
      s->alpha = s->rz / pAp;
    }
  }
}

__global__ __launch_bounds__(kBlock) void k_ctl_rr(PcgState *s, const double *part, int np) {
  if (s->done) return;
  const double rr = sum_parts(part, np);
  if (threadIdx.x == 0) {
    s->rr = rr;
    s->it += 1;
    if (rr <= s->tol2) s->done = 1;
  }
}

__global__ __launch_bounds__(kBlock) void k_ctl_true(PcgState *s, const double *part, int np) {
  const double rr = sum_parts(part, np);
  if (threadIdx.x == 0) {
    s->rr_true = rr;
    s->rr = rr;
  }
}

__global__ __launch_bounds__(kBlock) void k_update_p(int64_t n, double *p, const double *z,
                                                     const PcgState *s, int first) {
  if (s->done) return;
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i < n) p[i] = first ? z[i] : z[i] + s->beta * p[i];
}

// x += alpha p, r -= alpha q with per-block ||r||^2 partials; when w is
// given it also writes the sweep inputs (w = r, y = 0, z = 0 or r on fixed
// DOFs), saving the separate preparation pass.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_update_xr_prep(int64_t n, double *x, double *r,
                                                           const double *p, const double *q,
                                                           double *part, const PcgState *s,
                                                           T *w, T *y, double *z,
                                                           const uint8_t *fixed) {
  if (s->done) return;
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  const double al = s->alpha;
  double rr = 0.0;
  if (i < n) {
    x[i] += al * p[i];
    const double ri = r[i] - al * q[i];
    r[i] = ri;
    rr = ri * ri;
    if (w) {
      w[i] = (T)ri;
      y[i] = T(0);
      z[i] = fixed[i] ? ri : 0.0;
    }
  }
  rr = block_sum(rr);
  if (threadIdx.x == 0) part[blockIdx.x] = rr;
}

__global__ void k_zero(int64_t n, double *x) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i < n) x[i] = 0.0;
}

__global__ void k_integrate(int64_t n, double h, const double *a, double *q, double *v) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i < n) {
    const double vn = v[i] + h * a[i];
    v[i] = vn;
    q[i] += h * vn;
  }
}

// ---------------------------------------------------------------- Jacobi
template <typename T>
__global__ void k_diag_inv(int64_t n, const int32_t *row_ptr, const int32_t *col, const T *val,
                           double *dinv) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  double d = 0.0;
  for (int32_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k)
    if (col[k] == i) d += (double)val[k];
  dinv[i] = d != 0.0 ? 1.0 / d : 1.0;
}

__global__ void k_jacobi(int64_t n, const double *dinv, const double *r, double *z,
                         const PcgState *s) {
  if (s && s->done) return;
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i < n) z[i] = dinv[i] * r[i];
}

// ------------------------------------------------------ triangular sweeps
// prep: w = r (free DOFs), y = 0, z = 0 (free) / r (fixed: identity rows)
template <typename T>
__global__ void k_tri_prep(int64_t n, const double *r, T *w, T *y, double *z,
                           const uint8_t *fixed, const PcgState *s) {
  if (s && s->done) return;
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  const double ri = r[i];
  w[i] = (T)ri;
  y[i] = T(0);
  z[i] = fixed[i] ? ri : 0.0;
}

constexpr int kFR = 256;  // forward tile: 256 rows x NG groups of TC columns (TC: 16..128)
// backward tile: 4 NW columns x BR rows (BR: 256..1024), NW wavefronts of 4 columns

// Forward tile: t[i] = sum_{j in tile cols} G[i, j] w[rows[j]] for the tile's
// rows (one row per thread of each group of 4 wavefronts, consecutive rows =
// consecutive addresses of the column-major panel; NG groups take NG runs of
// TC columns and meet in one sum per row); own rows (i < nc) accumulate into
// y, struct rows subtract from w.  Entries above the diagonal of L11^{-1}
// are skipped.
// All TC panel loads of a row are issued before the gather of the inputs
// w[rows[j]] (an index load and a dependent load), so one tile costs about
// three memory latencies instead of one per group of columns.  With NT the
// panels are read non-temporally, for factors larger than the last-level
// cache (each entry is read once per application, 11.6 GB on the largest
// mesh): the stream then does not evict the vectors, row indices and
// descriptors that the gathers and atomics reuse (forward 151.6 -> 138.9 us,
// backward 155.1 -> 148.6 us per launch on the 1.39 M-DOF block).  A factor
// that fits in that cache is read with ordinary loads and stays there from
// one application to the next.
template <bool NT, typename T>
__device__ inline T panel_load(const T *p) {
  if constexpr (NT) return __builtin_nontemporal_load(p);
  else return *p;
}

template <typename T, int TC, bool NT, int NG>
__global__ __launch_bounds__(kFR * NG) void k_tri_fwd(const TileDev *__restrict__ tiles,
                                                      const int32_t *__restrict__ rows,
                                                      const T *__restrict__ panels, T *w, T *y,
                                                      const PcgState *s) {
  // the descriptor, the control word and the kernel arguments are loaded
  // together, one latency before the index and panel loads (the empty asm
  // takes the values the tile needs, so that the compiler does not sink
  // their loads below the exit branch)
  const TileDev d = tiles[blockIdx.x];
  const int done = s ? s->done : 0;
  asm volatile("" ::"s"(d.panel_off), "s"(d.rows_off), "s"(d.nc), "s"(d.m), "s"(rows),
               "s"(panels));
  if (done) return;
  __shared__ T s_in[NG][TC];
  __shared__ T s_part[NG > 1 ? NG - 1 : 1][kFR];
  const TileDev &t = d;
  const int32_t *rw = rows + d.rows_off;
  const int tid = (int)threadIdx.x, r = tid % kFR, grp = tid / kFR;
  // group grp (4 wavefronts) takes columns c0 .. c0 + TC - 1 of the tile;
  // a group past the supernode's last column has ncol <= 0 and loads nothing
  const int c0 = t.c0 + grp * TC, ncol = min(d.nc - c0, TC);
  const int i = t.r0 + r;
  const bool valid = i < d.m;
  // index loads first, unconditional (clamped: c0 + min(r, ncol - 1) is at
  // most nc - 1, also when ncol <= 0), so that no wait separates them from
  // the panel loads issued next
  const int32_t din = rw[c0 + min(r, ncol - 1)];
  const int32_t dout = rw[min(i, d.m - 1)];
  // columns of this row inside the group (own rows stop at the diagonal)
  const int lim = !valid ? 0 : (i < d.nc ? min(ncol, i + 1 - c0) : ncol);
  const int64_t m = d.ld;  // column stride
  const T *G = panels + d.panel_off + (int64_t)min(c0, d.nc - 1) * m + (valid ? i : 0);
  const bool full = ncol == TC && t.r0 + kFR <= d.m && (t.r0 >= d.nc || t.r0 + 1 >= c0 + TC);
  // a row's TC panel values are held in registers at once, except for FP64
  // panels in grouped tiles (larger workgroups leave a thread fewer
  // registers: 128 with 16 wavefronts): there the row is taken in chunks of
  // TC / 2 (2 groups) or TC / 4 columns (4 groups), each loaded after the
  // previous one's products
  constexpr int TH = sizeof(T) == 8 && NG > 2 ? TC / 4 : sizeof(T) == 8 && NG > 1 ? TC / 2 : TC;
  T g[TH];
  auto load_chunk = [&](int j0) {
    if (full) {
#pragma unroll
      for (int j = 0; j < TH; ++j) g[j] = panel_load<NT>(G + (j0 + j) * m);
    } else {
#pragma unroll
      for (int j = 0; j < TH; ++j) g[j] = j0 + j < lim ? panel_load<NT>(G + (j0 + j) * m) : T(0);
    }
  };
  load_chunk(0);
  if (r < TC) s_in[grp][r] = r < ncol ? w[din] : T(0);
  __syncthreads();
  T acc = T(0);
#pragma unroll 1
  for (int h = 0; h < TC / TH; ++h) {
    if (h > 0) load_chunk(h * TH);
    if (lim > h * TH) {
      const T *x = s_in[grp] + h * TH;
      T a0 = T(0), a1 = T(0), a2 = T(0), a3 = T(0);
#pragma unroll
      for (int j = 0; j < TH; j += 4) {
        a0 += g[j] * x[j];
        a1 += g[j + 1] * x[j + 1];
        a2 += g[j + 2] * x[j + 2];
        a3 += g[j + 3] * x[j + 3];
      }
      acc += (a0 + a1) + (a2 + a3);
    }
  }
  if constexpr (NG > 1) {
    // the groups' partial sums of a row meet in group 0 (fixed order), so a
    // row takes one atomic per NG TC columns
    if (grp > 0) s_part[grp - 1][r] = acc;
    __syncthreads();
    if (grp > 0) return;
#pragma unroll
    for (int q = 0; q < NG - 1; ++q) acc += s_part[q][r];
  }
  // a row has entries in the tile unless it is an own row above the tile's
  // first column
  if (!valid || (i < d.nc && i < t.c0)) return;
  if (i < d.nc) atomicAdd(y + dout, acc);
  else atomicAdd(w + dout, -acc);
}

// Backward tile: x[rows[j]] += sum_{i in tile rows} G[i, j] v_i with
// v_i = dinv y (own rows) or -x[rows[i]] (struct rows, already final).
// Each of the NW wavefronts handles CPW = 4 consecutive columns (lanes stride
// over rows) and issues all BR/64 x CPW of its panel loads before the inputs
// v are gathered; the workgroup gathers the BR inputs once for its 4 NW
// columns.  Rows above a column's diagonal (zeros of L11^{-1}) are not read.
template <typename T, int BR, bool NT, int NW>
__global__ __launch_bounds__(64 * NW) void k_tri_bwd(const TileDev *__restrict__ tiles,
                                                 const int32_t *__restrict__ rows,
                                                 const T *__restrict__ panels,
                                                 const T *__restrict__ dinv,
                                                 const T *__restrict__ y, double *z,
                                                 const PcgState *s) {
  const TileDev d = tiles[blockIdx.x];  // loaded with the control word, as in k_tri_fwd
  const int done = s ? s->done : 0;
  asm volatile("" ::"s"(d.panel_off), "s"(d.rows_off), "s"(d.nc), "s"(d.m), "s"(rows),
               "s"(panels));
  if (done) return;
  constexpr int NI = BR / 64, CPW = kBwdColsPerWave, NTH = 64 * NW;
  __shared__ T s_v[BR];
  const TileDev &t = d;
  const int32_t *rw = rows + d.rows_off;
  const int r0 = t.r0, r1 = min(d.m, r0 + BR);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int j0 = t.c0 + CPW * wv;
  const int nj = max(0, min(CPW, d.nc - j0));
  const int ibeg = max(r0, j0);
  const int64_t m = d.ld;  // column stride
  const T *G = panels + d.panel_off + (int64_t)min(j0, d.nc - 1) * m;
  // index loads of the inputs first (clamped, unconditional), then the panel
  // loads, then the input values
  constexpr int NV = (BR + NTH - 1) / NTH;
  int32_t dof[NV];
#pragma unroll
  for (int u = 0; u < NV; ++u) dof[u] = rw[min(r0 + (int)threadIdx.x + NTH * u, r1 - 1)];
  T g[NI][CPW];
  if (nj == CPW && ibeg == r0 && r1 == r0 + BR) {
#pragma unroll
    for (int q = 0; q < NI; ++q) {
      const int i = r0 + lane + 64 * q;
#pragma unroll
      for (int c = 0; c < CPW; ++c) g[q][c] = panel_load<NT>(G + c * m + i);
    }
  } else {
#pragma unroll
    for (int q = 0; q < NI; ++q) {
      const int i = r0 + lane + 64 * q;
      const bool ok = i >= ibeg && i < r1;
#pragma unroll
      for (int c = 0; c < CPW; ++c)
        g[q][c] = (ok && c < nj) ? panel_load<NT>(G + c * m + i) : T(0);
    }
  }
  // inputs: own rows need dinv y, struct rows -x; a tile that lies in one
  // kind only loads that one (uniform test), a mixed tile loads both
  const int mode = r0 >= d.nc ? 1 : (r1 <= d.nc ? 0 : 2);
#pragma unroll
  for (int u = 0; u < NV; ++u) {
    const int k = (int)threadIdx.x + NTH * u, i = r0 + k;
    if (NTH * (u + 1) > BR && k >= BR) break;  // (compile-time false unless NTH > BR)
    T v;
    if (mode == 0) {
      v = dinv[dof[u]] * y[dof[u]];
    } else if (mode == 1) {
      v = (T)(-z[dof[u]]);
    } else {
      const T own = dinv[dof[u]] * y[dof[u]];
      const T st = (T)(-z[dof[u]]);
      v = i < d.nc ? own : st;
    }
    s_v[k] = i < r1 ? v : T(0);
  }
  __syncthreads();
  if (nj == 0 || ibeg >= r1) return;
  T p[CPW];
#pragma unroll
  for (int c = 0; c < CPW; ++c) p[c] = T(0);
#pragma unroll
  for (int q = 0; q < NI; ++q) {
    const T v = s_v[lane + 64 * q];
#pragma unroll
    for (int c = 0; c < CPW; ++c) p[c] += g[q][c] * v;
  }
  // transpose-reduce of the 4 column partials (fixed order): lanes trade
  // halves of their columns with lane^1, then lane^2, so that each lane
  // holds one column summed over 4 lanes, then a butterfly over the rest;
  // lanes 0..3 end with the totals of columns 2(l&1) + (l>>1&1)
  static_assert(CPW == 4, "the exchange pattern is for 4 columns per wavefront");
  const bool odd = lane & 1, b1 = lane & 2;
  T k0 = odd ? p[2] : p[0], k1 = odd ? p[3] : p[1];
  k0 += __shfl_xor(odd ? p[0] : p[2], 1);
  k1 += __shfl_xor(odd ? p[1] : p[3], 1);
  T tot = b1 ? k1 : k0;
  tot += __shfl_xor(b1 ? k0 : k1, 2);
#pragma unroll
  for (int off = 4; off < 64; off <<= 1) tot += __shfl_xor(tot, off);
  const int c = (odd ? 2 : 0) + (b1 ? 1 : 0);
  if (lane < 4 && c < nj) atomicAdd(z + rw[j0 + c], (double)tot);
}

}  // namespace

int spmv_lanes_for(double avg) {
  if (avg > 48) return 16;
  if (avg > 24) return 8;
  if (avg > 12) return 4;
  return 2;
}

template <typename T>
void launch_spmv(hipStream_t st, int64_t n, int G, const int32_t *row_ptr, const int32_t *col,
                 const T *val, const double *x, double *y, const double *w, double *part,
                 int *n_part, const PcgState *state) {
  const int64_t rows_per_block = kBlock / G;
  const unsigned blocks = (unsigned)((n + rows_per_block - 1) / rows_per_block);
  if (n_part) *n_part = (int)blocks;
  switch (G) {
    case 16: k_spmv<T, 16><<<blocks, kBlock, 0, st>>>(n, row_ptr, col, val, x, y, w, part, state); break;
    case 8: k_spmv<T, 8><<<blocks, kBlock, 0, st>>>(n, row_ptr, col, val, x, y, w, part, state); break;
    case 4: k_spmv<T, 4><<<blocks, kBlock, 0, st>>>(n, row_ptr, col, val, x, y, w, part, state); break;
    default: k_spmv<T, 2><<<blocks, kBlock, 0, st>>>(n, row_ptr, col, val, x, y, w, part, state); break;
  }
}

int cg_blocks(int64_t n) { return (int)((n + kBlock - 1) / kBlock); }

template <typename T>
void launch_update_xr_prep(hipStream_t st, int64_t n, double *x, double *r, const double *p,
                           const double *q, double *part, const PcgState *s, T *w, T *y, double *z,
                           const uint8_t *fixed) {
  k_update_xr_prep<T><<<cg_blocks(n), kBlock, 0, st>>>(n, x, r, p, q, part, s, w, y, z, fixed);
}


void launch_residual(hipStream_t st, int64_t n, const double *b, const double *Ax, double *r,
                     double *prr, double *pbb) {
  k_residual<<<cg_blocks(n), kBlock, 0, st>>>(n, b, Ax, r, prr, pbb);
}
void launch_ctl_init(hipStream_t st, PcgState *s, const double *prr, const double *pbb, int np,
                     double rel_tol) {
  k_ctl_init<<<1, kBlock, 0, st>>>(s, prr, pbb, np, rel_tol);
}
void launch_dot(hipStream_t st, int64_t n, const double *a, const double *b, double *part,
                const PcgState *state) {
  k_dot<<<cg_blocks(n), kBlock, 0, st>>>(n, a, b, part, state);
}
void launch_ctl_rz(hipStream_t st, PcgState *s, const double *part, int np, int first) {
  k_ctl_rz<<<1, kBlock, 0, st>>>(s, part, np, first);
}
void launch_ctl_alpha(hipStream_t st, PcgState *s, const double *part, int np, double *stage) {
  if (stage && np > 4 * kPartChunk) {
    const int nb = (np + kPartChunk - 1) / kPartChunk;
    k_part_reduce<<<nb, kBlock, 0, st>>>(part, np, stage, s);
    k_ctl_alpha<<<1, kBlock, 0, st>>>(s, stage, nb);
  } else {
    k_ctl_alpha<<<1, kBlock, 0, st>>>(s, part, np);
  }
}
void launch_ctl_rr(hipStream_t st, PcgState *s, const double *part, int np) {
  k_ctl_rr<<<1, kBlock, 0, st>>>(s, part, np);
}
void launch_ctl_true(hipStream_t st, PcgState *s, const double *part, int np) {
  k_ctl_true<<<1, kBlock, 0, st>>>(s, part, np);
}
void launch_update_p(hipStream_t st, int64_t n, double *p, const double *z, const PcgState *state,
                     int first) {
  k_update_p<<<cg_blocks(n), kBlock, 0, st>>>(n, p, z, state, first);
}
void launch_zero(hipStream_t st, int64_t n, double *x) {
  if (n > 0) k_zero<<<cg_blocks(n), kBlock, 0, st>>>(n, x);
}
void launch_integrate(hipStream_t st, int64_t n, double h, const double *a, double *q,
                      double *v) {
  k_integrate<<<cg_blocks(n), kBlock, 0, st>>>(n, h, a, q, v);
}

template <typename T>
void launch_diag_inv(hipStream_t st, int64_t n, const int32_t *row_ptr, const int32_t *col,
                     const T *val, double *dinv) {
  k_diag_inv<T><<<cg_blocks(n), kBlock, 0, st>>>(n, row_ptr, col, val, dinv);
}
void launch_jacobi(hipStream_t st, int64_t n, const double *dinv, const double *r, double *z,
                   const PcgState *state) {
  k_jacobi<<<cg_blocks(n), kBlock, 0, st>>>(n, dinv, r, z, state);
}

template <typename T>
void launch_tri_prep(hipStream_t st, int64_t n, const double *r, T *w, T *y, double *z,
                     const uint8_t *fixed, const PcgState *state) {
  k_tri_prep<T><<<cg_blocks(n), kBlock, 0, st>>>(n, r, w, y, z, fixed, state);
}
template <typename T>
void launch_tri_fwd(hipStream_t st, const TileDev *tiles, int n_tiles,
                    const int32_t *rows, const T *panels, T *w, T *y, const PcgState *state,
                    int tile_cols, int groups, bool stream) {
  if (n_tiles <= 0) return;
#define FE_FWD(TC, NG)                                                                       \
  (stream ? k_tri_fwd<T, TC, true, NG><<<n_tiles, kFR * NG, 0, st>>>(tiles, rows, panels, w, \
                                                                     y, state)             \
          : k_tri_fwd<T, TC, false, NG><<<n_tiles, kFR * NG, 0, st>>>(tiles, rows, panels,  \
                                                                      w, y, state))
  if (groups == 1) {
    switch (tile_cols) {
      case 16: FE_FWD(16, 1); break;
      case 32: FE_FWD(32, 1); break;
      case 64: FE_FWD(64, 1); break;
      case 128: FE_FWD(128, 1); break;
      default: throw std::runtime_error("forward tile width must be 16, 32, 64 or 128");
    }
  } else if (tile_cols == 64 && groups == 2) {
    FE_FWD(64, 2);
  } else if (tile_cols == 64 && groups == 4) {
    FE_FWD(64, 4);
  } else {
    throw std::runtime_error("forward column groups: 2 or 4 groups of 64 columns");
  }
#undef FE_FWD
}
template <typename T>
void launch_tri_bwd(hipStream_t st, const TileDev *tiles, int n_tiles,
                    const int32_t *rows, const T *panels, const T *dinv, const T *y, double *z,
                    const PcgState *state, int tile_rows, int tile_cols, bool stream) {
  if (n_tiles <= 0) return;
#define FE_BWD(BR, NW)                                                                       \
  (stream ? k_tri_bwd<T, BR, true, NW><<<n_tiles, 64 * NW, 0, st>>>(tiles, rows, panels,    \
                                                                   dinv, y, z, state)       \
          : k_tri_bwd<T, BR, false, NW><<<n_tiles, 64 * NW, 0, st>>>(tiles, rows, panels,   \
                                                                    dinv, y, z, state))
#define FE_BWD_ROWS(NW)                                                                     \
  switch (tile_rows) {                                                                      \
    case 256: FE_BWD(256, NW); break;                                                       \
    case 512: FE_BWD(512, NW); break;                                                       \
    case 1024: FE_BWD(1024, NW); break;                                                     \
    default: throw std::runtime_error("backward tile height must be 256, 512 or 1024");     \
  }
  if (tile_cols == 4 * kBwdColsPerWave) {
    FE_BWD_ROWS(4)
  } else if (tile_cols == 8 * kBwdColsPerWave) {
    FE_BWD_ROWS(8)
  } else if (tile_cols == 16 * kBwdColsPerWave) {
    FE_BWD_ROWS(16)
  } else {
    throw std::runtime_error("backward tile width must be 16, 32 or 64");
  }
#undef FE_BWD_ROWS
#undef FE_BWD
}

#define FE_INST(T)                                                                             \
  template void launch_spmv<T>(hipStream_t, int64_t, int, const int32_t *, const int32_t *,    \
                               const T *, const double *, double *, const double *, double *,  \
                               int *, const PcgState *);                                       \
  template void launch_update_xr_prep<T>(hipStream_t, int64_t, double *, double *,             \
                                         const double *, const double *, double *,             \
                                         const PcgState *,                                     \
                                         T *, T *, double *, const uint8_t *);                 \
  template void launch_diag_inv<T>(hipStream_t, int64_t, const int32_t *, const int32_t *,     \
                                   const T *, double *);                                       \
  template void launch_tri_prep<T>(hipStream_t, int64_t, const double *, T *, T *, double *,   \
                                   const uint8_t *, const PcgState *);                         \
  template void launch_tri_fwd<T>(hipStream_t, const TileDev *, int,            \
                                  const int32_t *, const T *, T *, T *, const PcgState *, int,  \
                                  int, bool);                                                       \
  template void launch_tri_bwd<T>(hipStream_t, const TileDev *, int,            \
                                  const int32_t *, const T *, const T *, const T *, double *,  \
                                  const PcgState *, int, int, bool);
FE_INST(float)
FE_INST(double)
#undef FE_INST

}  // namespace fe
