// Many-right-hand-side application of the LDL^T preconditioner, and the
// contact kernels built on it (paper Sec. 6.2: the compliance matrix
// W = H P^{-1} H^T from the asynchronous factor and a solver for many
// right-hand sides, projected Gauss-Seidel on its complementarity problem,
// and the constraint products H x and H^T lambda of the motion correction).
//
// With k right-hand sides the triangular sweeps become dense products: a
// block of 64 panel rows (forward) or 64 own columns (backward) multiplies a
// k-wide block of gathered inputs, so every panel entry is read once for all
// right-hand sides and the arithmetic runs on the matrix cores (MFMA
// 16x16x4 in FP32 or FP64).  Right-hand sides are stored DOF-major: the
// values of one DOF are contiguous, with a leading dimension ld = k rounded
// up to the tile width, so each gathered input row is one contiguous load.
#include "device.hpp"

namespace fe {

namespace {

typedef float f4v __attribute__((ext_vector_type(4)));
typedef double d4v __attribute__((ext_vector_type(4)));

template <typename T>
struct Mma;
// A operand: lane i + 16 k holds A[i][k]; B operand: lane j + 16 k holds
// B[k][j]; the 16 x 16 result: register q of lane l holds column l % 16 of
// the row given by row(l, q) (different for the FP32 and FP64 instructions).
template <>
struct Mma<float> {
  typedef f4v acc;
  __device__ static acc step(float a, float b, acc c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  __device__ static int row(int l, int q) { return 4 * (l >> 4) + q; }
};
template <>
struct Mma<double> {
  typedef d4v acc;
  __device__ static acc step(double a, double b, acc c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  __device__ static int row(int l, int q) { return 4 * q + (l >> 4); }
};

constexpr int kMR = kMultiRows;  // output rows (forward) / columns (backward) per tile
constexpr int kKC = 16;          // contraction chunk staged in LDS
constexpr int kPad = 16;         // LDS row padding: the four 16-lane groups of
                                 // a fragment read hit different banks

// BV contiguous values of a DOF-major row (16-byte aligned)
template <typename T, int BV>
__device__ inline void load_row(const T *src, T (&v)[BV]) {
  if constexpr (sizeof(T) == 4) {
#pragma unroll
    for (int u = 0; u < BV / 4; ++u) {
      const float4 x = reinterpret_cast<const float4 *>(src)[u];
      v[4 * u] = x.x;
      v[4 * u + 1] = x.y;
      v[4 * u + 2] = x.z;
      v[4 * u + 3] = x.w;
    }
  } else {
#pragma unroll
    for (int u = 0; u < BV / 2; ++u) {
      const double2 x = reinterpret_cast<const double2 *>(src)[u];
      v[2 * u] = x.x;
      v[2 * u + 1] = x.y;
    }
  }
}

// One staged chunk: four MFMA k-steps over the 16 entries of the chunk.  The
// wave owns rows wr..wr+31 and columns wc..wc+BN/2-1 of the block's result.
template <typename T, int BN>
__device__ inline void mma_chunk(const T (*sA)[kMR + kPad], const T (*sB)[BN + kPad], int wr,
                                 int wc, int lane, typename Mma<T>::acc (&acc)[2][BN / 32]) {
  constexpr int NCB = BN / 32;
  const int kk = lane >> 4, ii = lane & 15;
#pragma unroll
  for (int kq = 0; kq < kKC; kq += 4) {
    T a[2], b[NCB];
#pragma unroll
    for (int r = 0; r < 2; ++r) a[r] = sA[kq + kk][wr + 16 * r + ii];
#pragma unroll
    for (int c = 0; c < NCB; ++c) b[c] = sB[kq + kk][wc + 16 * c + ii];
#pragma unroll
    for (int r = 0; r < 2; ++r)
#pragma unroll
      for (int c = 0; c < NCB; ++c) acc[r][c] = Mma<T>::step(a[r], b[c], acc[r][c]);
  }
}

// Forward tile: T = G[r0:r0+64, lo:hi] * w[rows[lo:hi], k0:k0+BN] for
// supernode s; own rows (i < nc) add T into y, update rows subtract it from
// w (their DOFs belong to ancestors, finished at a later level).  Entries of
// L11^{-1} above its diagonal are read as zero.  blockIdx.y picks the
// right-hand-side block.  The global loads of the next chunk are issued
// before the MFMAs of the current one.
template <typename T, int BN>
__global__ __launch_bounds__(256) void k_mfwd(const MTile *__restrict__ tiles,
                                              const SnDev *__restrict__ sn,
                                              const int32_t *__restrict__ rows,
                                              const T *__restrict__ panels, T *w, T *y, int ld) {
  constexpr int NCB = BN / 32, BV = BN / 16;
  __shared__ T sA[kKC][kMR + kPad];  // sA[k][i] = G[r0 + i][c + k]
  __shared__ T sB[kKC][BN + kPad];   // sB[k][j] = w[rows[c + k]][k0 + j]
  const MTile t = tiles[blockIdx.x];
  const SnDev d = sn[t.s];
  const int32_t *rw = rows + d.rows_off;
  const int m = d.m, nc = d.nc, r0 = t.b0;
  const int64_t k0 = (int64_t)blockIdx.y * BN;
  const int tid = (int)threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int wr = (wv & 1) * 32, wc = (wv >> 1) * (BN / 2);
  const T *G = panels + d.panel_off;
  const int ak = tid >> 4, ai = (tid & 15) * 4;  // staging: panel column, 4 rows
  const int bk = tid >> 4, bj = (tid & 15) * BV; // staging: input row, BV values
  T ra[4], rb[BV];
  auto load = [&](int c) {
    const int j = c + ak;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int i = r0 + ai + q;
      const bool ok = i < m && j < t.hi && (i >= nc || j <= i);
      ra[q] = ok ? G[(int64_t)j * m + i] : T(0);
    }
    const int jb = c + bk;
    if (jb < t.hi) {
      load_row<T, BV>(w + (int64_t)rw[jb] * ld + k0 + bj, rb);
    } else {
#pragma unroll
      for (int v = 0; v < BV; ++v) rb[v] = T(0);
    }
  };
  typename Mma<T>::acc acc[2][NCB];
#pragma unroll
  for (int r = 0; r < 2; ++r)
#pragma unroll
    for (int c = 0; c < NCB; ++c) acc[r][c] = typename Mma<T>::acc{0, 0, 0, 0};
  load(t.lo);
  for (int c = t.lo; c < t.hi; c += kKC) {
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 4; ++q) sA[ak][ai + q] = ra[q];
#pragma unroll
    for (int v = 0; v < BV; ++v) sB[bk][bj + v] = rb[v];
    __syncthreads();
    if (c + kKC < t.hi) load(c + kKC);
    mma_chunk<T, BN>(sA, sB, wr, wc, lane, acc);
  }
#pragma unroll
  for (int r = 0; r < 2; ++r)
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int i = r0 + wr + 16 * r + Mma<T>::row(lane, q);
      if (i >= m) continue;
      const int64_t o = (int64_t)rw[i] * ld + k0 + wc + (lane & 15);
#pragma unroll
      for (int c = 0; c < NCB; ++c) {
        const T v = acc[r][c][q];
        if (i < nc) atomicAdd(y + o + 16 * c, v);
        else atomicAdd(w + o + 16 * c, -v);
      }
    }
}

// Backward tile: x[rows[j0:j0+64], k0:k0+BN] += G[lo:hi, j0:j0+64]^T v with
// v_i = dinv y (own rows, i < nc) or -z (update rows: ancestor DOFs, final
// before this level).  Entries of L11^{-1} above its diagonal read as zero.
template <typename T, int BN>
__global__ __launch_bounds__(256) void k_mbwd(const MTile *__restrict__ tiles,
                                              const SnDev *__restrict__ sn,
                                              const int32_t *__restrict__ rows,
                                              const T *__restrict__ panels,
                                              const T *__restrict__ dinv,
                                              const T *__restrict__ y, double *z, int ld) {
  constexpr int NCB = BN / 32, BV = BN / 16;
  __shared__ T sA[kKC][kMR + kPad];  // sA[k][j] = G[c + k][j0 + j]
  __shared__ T sB[kKC][BN + kPad];   // sB[k][j] = v[c + k][k0 + j]
  const MTile t = tiles[blockIdx.x];
  const SnDev d = sn[t.s];
  const int32_t *rw = rows + d.rows_off;
  const int m = d.m, nc = d.nc, j0 = t.b0;
  const int64_t k0 = (int64_t)blockIdx.y * BN;
  const int tid = (int)threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int wr = (wv & 1) * 32, wc = (wv >> 1) * (BN / 2);
  const T *G = panels + d.panel_off;
  const int aj = tid >> 2, ak = (tid & 3) * 4;   // staging: own column, 4 panel rows
  const int bk = tid >> 4, bj = (tid & 15) * BV; // staging: input row, BV values
  T ra[4], rb[BV];
  auto load = [&](int c) {
    const int j = j0 + aj;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int i = c + ak + q;
      const bool ok = i < t.hi && j < nc && (i >= nc || i >= j);
      ra[q] = ok ? G[(int64_t)j * m + i] : T(0);
    }
    const int ib = c + bk;
    if (ib < t.hi) {
      const int64_t dof = rw[ib];
      if (ib < nc) {
        const T s = dinv[dof];
        load_row<T, BV>(y + dof * ld + k0 + bj, rb);
#pragma unroll
        for (int v = 0; v < BV; ++v) rb[v] *= s;
      } else {
        double zz[BV];
        load_row<double, BV>(z + dof * ld + k0 + bj, zz);
#pragma unroll
        for (int v = 0; v < BV; ++v) rb[v] = (T)(-zz[v]);
      }
    } else {
#pragma unroll
      for (int v = 0; v < BV; ++v) rb[v] = T(0);
    }
  };
  typename Mma<T>::acc acc[2][NCB];
#pragma unroll
  for (int r = 0; r < 2; ++r)
#pragma unroll
    for (int c = 0; c < NCB; ++c) acc[r][c] = typename Mma<T>::acc{0, 0, 0, 0};
  load(t.lo);
  for (int c = t.lo; c < t.hi; c += kKC) {
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 4; ++q) sA[ak + q][aj] = ra[q];
#pragma unroll
    for (int v = 0; v < BV; ++v) sB[bk][bj + v] = rb[v];
    __syncthreads();
    if (c + kKC < t.hi) load(c + kKC);
    mma_chunk<T, BN>(sA, sB, wr, wc, lane, acc);
  }
#pragma unroll
  for (int r = 0; r < 2; ++r)
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int j = j0 + wr + 16 * r + Mma<T>::row(lane, q);
      if (j >= nc) continue;
      const int64_t o = (int64_t)rw[j] * ld + k0 + wc + (lane & 15);
#pragma unroll
      for (int c = 0; c < NCB; ++c) atomicAdd(z + o + 16 * c, (double)acc[r][c][q]);
    }
}

// w = r, y = 0, z = r on fixed DOFs (their rows of A are the identity) and 0
// elsewhere, for the DOF-major n x ld blocks; columns >= k are zero padding.
template <typename T>
__global__ void k_mprep(int64_t n, int k, int ld, const double *__restrict__ R, T *w, T *y,
                        double *z, const uint8_t *__restrict__ fixed) {
  const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (idx >= n * ld) return;
  const int64_t dof = idx / ld;
  const int c = (int)(idx - dof * ld);
  const double r = c < k ? R[dof * k + c] : 0.0;
  w[idx] = (T)r;
  y[idx] = T(0);
  z[idx] = fixed[dof] ? r : 0.0;
}

template <typename T>
__global__ void k_mzero(int64_t total, T *w, T *y, double *z) {
  const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (idx >= total) return;
  w[idx] = T(0);
  y[idx] = T(0);
  z[idx] = 0.0;
}

__global__ void k_mout(int64_t n, int k, int ld, const double *__restrict__ z,
                       double *__restrict__ Z) {
  const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (idx >= n * k) return;
  const int64_t dof = idx / k;
  Z[idx] = z[dof * ld + (idx - dof * k)];
}

// Row range of constraint a, or false (and the error flag) if it is invalid.
__device__ inline bool h_row(int a, int64_t nnz_h, const int32_t *hrp, int32_t &p0, int32_t &p1,
                             int *err) {
  p0 = hrp[a];
  p1 = hrp[a + 1];
  if (p0 < 0 || p1 < p0 || (int64_t)p1 > nnz_h) {
    if (err) *err = 1;
    return false;
  }
  return true;
}

// Right-hand sides H^T: column a of the n x ld block holds row a of H.  One
// thread per constraint, so each (DOF, a) entry has a single writer.
template <typename T>
__global__ void k_hscatter(int kc, int64_t n, int64_t nnz_h, const int32_t *__restrict__ hrp,
                           const int32_t *__restrict__ hcol, const double *__restrict__ hval,
                           int ld, T *w, double *z, const uint8_t *__restrict__ fixed, int *err) {
  const int a = (int)(blockIdx.x * 256 + threadIdx.x);
  if (a >= kc) return;
  int32_t p0, p1;
  if (!h_row(a, nnz_h, hrp, p0, p1, err)) return;
  for (int32_t p = p0; p < p1; ++p) {
    const int32_t col = hcol[p];
    if (col < 0 || (int64_t)col >= n) {
      *err = 1;
      continue;
    }
    const int64_t o = (int64_t)col * ld + a;
    w[o] += (T)hval[p];
    if (fixed[col]) z[o] += hval[p];
  }
}

// W[a][b] = sum_p H[a][p] Z[p][b]: one block per constraint row a.
__global__ void k_hz(int kc, int64_t n, int64_t nnz_h, const int32_t *__restrict__ hrp,
                     const int32_t *__restrict__ hcol, const double *__restrict__ hval, int ld,
                     const double *__restrict__ z, double *__restrict__ W) {
  const int a = (int)blockIdx.x;
  int32_t p0, p1;
  if (!h_row(a, nnz_h, hrp, p0, p1, nullptr)) return;
  for (int b = (int)threadIdx.x; b < kc; b += 256) {
    double s = 0.0;
    for (int32_t p = p0; p < p1; ++p) {
      const int32_t col = hcol[p];
      if (col >= 0 && (int64_t)col < n) s += hval[p] * z[(int64_t)col * ld + b];
    }
    W[(int64_t)a * kc + b] = s;
  }
}

// y = s_h H x + s_y y_in (k values; y_in NULL counts as 0; y may alias
// y_in), one thread per constraint.
__global__ void k_hx(int kc, int64_t n, int64_t nnz_h, const int32_t *__restrict__ hrp,
                     const int32_t *__restrict__ hcol, const double *__restrict__ hval,
                     double s_h, const double *__restrict__ x, double s_y, const double *y_in,
                     double *y, int *err) {
  const int a = (int)(blockIdx.x * 256 + threadIdx.x);
  if (a >= kc) return;
  int32_t p0, p1;
  double s = 0.0;
  if (h_row(a, nnz_h, hrp, p0, p1, err))
    for (int32_t p = p0; p < p1; ++p) {
      const int32_t col = hcol[p];
      if (col < 0 || (int64_t)col >= n) {
        *err = 1;
        continue;
      }
      s += hval[p] * x[col];
    }
  y[a] = s_h * s + (y_in ? s_y * y_in[a] : 0.0);
}

// y = s_y y_in (0 if y_in is NULL; y may alias y_in), before k_htx.
__global__ void k_scale_copy(int64_t n, double s_y, const double *y_in, double *y) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) y[i] = y_in ? s_y * y_in[i] : 0.0;
}

// y += s_h H^T lam, one thread per constraint.
__global__ void k_htx(int kc, int64_t n, int64_t nnz_h, const int32_t *__restrict__ hrp,
                      const int32_t *__restrict__ hcol, const double *__restrict__ hval,
                      double s_h, const double *__restrict__ lam, double *y, int *err) {
  const int a = (int)(blockIdx.x * 256 + threadIdx.x);
  if (a >= kc) return;
  int32_t p0, p1;
  if (!h_row(a, nnz_h, hrp, p0, p1, err)) return;
  const double l = s_h * lam[a];
  for (int32_t p = p0; p < p1; ++p) {
    const int32_t col = hcol[p];
    if (col < 0 || (int64_t)col >= n) {
      *err = 1;
      continue;
    }
    atomicAdd(y + col, hval[p] * l);
  }
}

__device__ inline double wave_sum64(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Projected Gauss-Seidel on lambda >= 0, W lambda - c >= 0, complementary:
// one wavefront; lambda lives in LDS, each lane holds NR entries of the
// current row of W and has the next row's loads in flight while the current
// row is reduced.  The butterfly sum leaves the same total in every lane, so
// all lanes take the same update and the same exit decision.  A sweep whose
// largest change is <= tol * max(lambda) ends the iteration.  A row whose
// diagonal is not positive leaves its multiplier unchanged.
template <int NR>
__global__ __launch_bounds__(64) void k_pgs(int kc, const double *__restrict__ W,
                                            const double *__restrict__ c, double *lam,
                                            int max_sweeps, double tol, double *info) {
  __shared__ double s_lam[64 * NR];
  const int lane = (int)threadIdx.x;
#pragma unroll
  for (int q = 0; q < NR; ++q) {
    const int j = lane + 64 * q;
    s_lam[j] = j < kc ? lam[j] : 0.0;
  }
  __syncthreads();
  double wr[NR];
#pragma unroll
  for (int q = 0; q < NR; ++q) {
    const int j = lane + 64 * q;
    wr[q] = j < kc ? W[j] : 0.0;
  }
  int sweeps = 0;
  double dmax = 0.0;
  while (sweeps < max_sweeps) {
    dmax = 0.0;
    double lmax = 0.0;
    for (int i = 0; i < kc; ++i) {
      const int64_t nxt = (int64_t)(i + 1 < kc ? i + 1 : 0) * kc;
      double wn[NR];
#pragma unroll
      for (int q = 0; q < NR; ++q) {
        const int j = lane + 64 * q;
        wn[q] = j < kc ? W[nxt + j] : 0.0;
      }
      double p = 0.0;
#pragma unroll
      for (int q = 0; q < NR; ++q) p += wr[q] * s_lam[lane + 64 * q];
      p = wave_sum64(p);
      const double li = s_lam[i];
      const double wii = W[(int64_t)i * kc + i];
      const double nl = wii > 0.0 ? fmax(0.0, li - (p - c[i]) / wii) : li;
      dmax = fmax(dmax, fabs(nl - li));
      lmax = fmax(lmax, nl);
      __syncthreads();
      if (lane == 0) s_lam[i] = nl;
      __syncthreads();
#pragma unroll
      for (int q = 0; q < NR; ++q) wr[q] = wn[q];
    }
    ++sweeps;
    if (dmax <= tol * lmax) break;
  }
#pragma unroll
  for (int q = 0; q < NR; ++q) {
    const int j = lane + 64 * q;
    if (j < kc) lam[j] = s_lam[j];
  }
  if (lane == 0 && info) {
    info[0] = (double)sweeps;
    info[1] = dmax;
  }
}

unsigned grid_for(int64_t n) { return (unsigned)((n + 255) / 256); }

}  // namespace

template <typename T>
void launch_multi_prep(hipStream_t st, int64_t n, int k, int ld, const double *R, T *w, T *y,
                       double *z, const uint8_t *fixed) {
  if (n * ld > 0) k_mprep<T><<<grid_for(n * ld), 256, 0, st>>>(n, k, ld, R, w, y, z, fixed);
}

template <typename T>
void launch_multi_zero(hipStream_t st, int64_t total, T *w, T *y, double *z) {
  if (total > 0) k_mzero<T><<<grid_for(total), 256, 0, st>>>(total, w, y, z);
}

void launch_multi_out(hipStream_t st, int64_t n, int k, int ld, const double *z, double *Z) {
  if (n * k > 0) k_mout<<<grid_for(n * k), 256, 0, st>>>(n, k, ld, z, Z);
}

template <typename T>
void launch_multi_fwd(hipStream_t st, const MTile *tiles, int n_tiles, int n_kb, int bn,
                      const SnDev *sn, const int32_t *rows, const T *panels, T *w, T *y, int ld) {
  if (n_tiles <= 0 || n_kb <= 0) return;
  const dim3 grid((unsigned)n_tiles, (unsigned)n_kb);
  if (bn == 128) k_mfwd<T, 128><<<grid, 256, 0, st>>>(tiles, sn, rows, panels, w, y, ld);
  else k_mfwd<T, 64><<<grid, 256, 0, st>>>(tiles, sn, rows, panels, w, y, ld);
}

template <typename T>
void launch_multi_bwd(hipStream_t st, const MTile *tiles, int n_tiles, int n_kb, int bn,
                      const SnDev *sn, const int32_t *rows, const T *panels, const T *dinv,
                      const T *y, double *z, int ld) {
  if (n_tiles <= 0 || n_kb <= 0) return;
  const dim3 grid((unsigned)n_tiles, (unsigned)n_kb);
  if (bn == 128) k_mbwd<T, 128><<<grid, 256, 0, st>>>(tiles, sn, rows, panels, dinv, y, z, ld);
  else k_mbwd<T, 64><<<grid, 256, 0, st>>>(tiles, sn, rows, panels, dinv, y, z, ld);
}

template <typename T>
void launch_h_scatter(hipStream_t st, int kc, int64_t n, int64_t nnz_h, const int32_t *hrp,
                      const int32_t *hcol, const double *hval, int ld, T *w, double *z,
                      const uint8_t *fixed, int *err) {
  if (kc > 0)
    k_hscatter<T><<<grid_for(kc), 256, 0, st>>>(kc, n, nnz_h, hrp, hcol, hval, ld, w, z, fixed,
                                                 err);
}

void launch_hz(hipStream_t st, int kc, int64_t n, int64_t nnz_h, const int32_t *hrp,
               const int32_t *hcol, const double *hval, int ld, const double *z, double *W) {
  if (kc > 0) k_hz<<<(unsigned)kc, 256, 0, st>>>(kc, n, nnz_h, hrp, hcol, hval, ld, z, W);
}

void launch_h_apply(hipStream_t st, int kc, int64_t n, int64_t nnz_h, const int32_t *hrp,
                    const int32_t *hcol, const double *hval, bool transpose, double s_h,
                    const double *x, double s_y, const double *y_in, double *y, int *err) {
  if (transpose) {
    if (n > 0) k_scale_copy<<<grid_for(n), 256, 0, st>>>(n, s_y, y_in, y);
    if (kc > 0)
      k_htx<<<grid_for(kc), 256, 0, st>>>(kc, n, nnz_h, hrp, hcol, hval, s_h, x, y, err);
  } else if (kc > 0) {
    k_hx<<<grid_for(kc), 256, 0, st>>>(kc, n, nnz_h, hrp, hcol, hval, s_h, x, s_y, y_in, y, err);
  }
}

int pgs_max_constraints() { return 64 * 64; }

void launch_pgs(hipStream_t st, int kc, const double *W, const double *c, double *lam,
                int max_sweeps, double tol, double *info) {
  if (kc <= 64) k_pgs<1><<<1, 64, 0, st>>>(kc, W, c, lam, max_sweeps, tol, info);
  else if (kc <= 128) k_pgs<2><<<1, 64, 0, st>>>(kc, W, c, lam, max_sweeps, tol, info);
  else if (kc <= 256) k_pgs<4><<<1, 64, 0, st>>>(kc, W, c, lam, max_sweeps, tol, info);
  else if (kc <= 512) k_pgs<8><<<1, 64, 0, st>>>(kc, W, c, lam, max_sweeps, tol, info);
  else if (kc <= 1024) k_pgs<16><<<1, 64, 0, st>>>(kc, W, c, lam, max_sweeps, tol, info);
  else if (kc <= 2048) k_pgs<32><<<1, 64, 0, st>>>(kc, W, c, lam, max_sweeps, tol, info);
  else k_pgs<64><<<1, 64, 0, st>>>(kc, W, c, lam, max_sweeps, tol, info);
}

#define FE_INST(T)                                                                             \
  template void launch_multi_prep<T>(hipStream_t, int64_t, int, int, const double *, T *, T *, \
                                     double *, const uint8_t *);                               \
  template void launch_multi_zero<T>(hipStream_t, int64_t, T *, T *, double *);                \
  template void launch_multi_fwd<T>(hipStream_t, const MTile *, int, int, int, const SnDev *,  \
                                    const int32_t *, const T *, T *, T *, int);                \
  template void launch_multi_bwd<T>(hipStream_t, const MTile *, int, int, int, const SnDev *,  \
                                    const int32_t *, const T *, const T *, const T *,          \
                                    double *, int);                                            \
  template void launch_h_scatter<T>(hipStream_t, int, int64_t, int64_t, const int32_t *,       \
                                    const int32_t *, const double *, int, T *, double *,       \
                                    const uint8_t *, int *);
FE_INST(float)
FE_INST(double)
#undef FE_INST

}  // namespace fe
