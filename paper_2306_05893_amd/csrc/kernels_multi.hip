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
// contraction chunk staged in LDS: 32 for FP32; 16 for FP64, whose larger
// registers and LDS tiles would otherwise leave too few waves per SIMD
template <typename T>
constexpr int chunk_of() { return sizeof(T) == 8 ? 16 : 32; }
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

// One staged chunk: KC / 4 MFMA k-steps.  The wave owns rows wr..wr+31 and
// columns wc..wc+BN/2-1 of the block's result.
template <typename T, int BN, int KC>
__device__ inline void mma_chunk(const T (*sA)[kMR + kPad], const T (*sB)[BN + kPad], int wr,
                                 int wc, int lane, typename Mma<T>::acc (&acc)[2][BN / 32]) {
  constexpr int NCB = BN / 32;
  const int kk = lane >> 4, ii = lane & 15;
#pragma unroll
  for (int kq = 0; kq < KC; kq += 4) {
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

// Work units are (tile, right-hand-side block) pairs, the block index
// fastest.  The hardware hands workgroup b of a launch to XCD b % 8; a launch
// has 8 * per workgroups and workgroup b takes unit (b % 8) * per + b / 8,
// so every XCD runs a contiguous range of units: the row blocks of one
// supernode (which gather the same inputs) and the right-hand-side blocks of
// one tile (which read the same panel entries) meet in the same L2.
constexpr int kXcds = 8;
__device__ inline int xcd_unit(int per) {
  const int b = (int)blockIdx.x;
  return (b % kXcds) * per + b / kXcds;
}

// One sweep tile, forward (FWD) or backward.
//   forward:  T = G[r0:r0+64, lo:hi] * src[rows[lo:hi], k0:k0+BN]; own rows
//             (i < nc) add T into y, update rows subtract it from src = w
//             (their DOFs belong to ancestors, finished at a later level);
//   backward: x = G[lo:hi, j0:j0+64]^T v added into z for the own columns,
//             v = dinv src on the own rows and src on the update rows, with
//             src = y holding y on the own rows and -z on the update rows
//             (ancestor DOFs, final before this level).
// A tile that covers its whole contraction writes its own-row results with
// plain stores (no other tile writes them); split tiles and the update rows
// of the forward sweep add with atomics.  Padding columns (>= kreal) are not
// written.
// Entries of L11^{-1} above its diagonal read as zero.  Staging: every global
// load is unconditional with its index clamped into the tile, the masks are
// applied when the values go to LDS, and the gather index of the next chunk
// is loaded one chunk ahead, so no load waits behind a branch or a dependent
// index load and the loads of chunk c + 1 are in flight during the MFMAs of
// chunk c.
template <typename T, int BN, bool FWD>
__global__ __launch_bounds__(256) void k_msweep(const MTile *__restrict__ tiles, int n_units,
                                                int n_kb, int per, const SnDev *__restrict__ sn,
                                                const int32_t *__restrict__ rows,
                                                const T *__restrict__ panels,
                                                const T *__restrict__ dinv, T *src, T *y,
                                                double *z, int ld, int kreal) {
  constexpr int KC = chunk_of<T>();
  constexpr int NA = KC / 4;          // panel values staged per thread
  constexpr int TPC = kMR / NA;       // forward: threads per staged panel column
  constexpr int TPR = 256 / KC;       // threads per staged input row
  constexpr int NCB = BN / 32, BV = BN / TPR;
  __shared__ T sA[KC][kMR + kPad];  // forward: G[r0 + i][c + k]; backward: G[c + k][j0 + j]
  __shared__ T sB[KC][BN + kPad];   // src[rows[c + k]][k0 + j]
  const int u = xcd_unit(per);
  if (u >= n_units) return;
  const MTile t = tiles[u / n_kb];
  const SnDev d = sn[t.s];
  const int32_t *rw = rows + d.rows_off;
  const int m = d.m, nc = d.nc, b0 = t.b0, hi = t.hi;
  const int64_t k0 = (int64_t)(u % n_kb) * BN;
  const int tid = (int)threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int wr = (wv & 1) * 32, wc = (wv >> 1) * (BN / 2);
  const T *G = panels + d.panel_off;
  // staging roles.  A, forward: panel column fa_k of the chunk, NA rows from
  // fa_i; backward: own column ba_j, NA panel rows from ba_k.  B: input row
  // bk of the chunk, BV values from bj.
  const int fa_k = tid / TPC, fa_i = (tid % TPC) * NA;
  const int ba_j = tid >> 2, ba_k = (tid & 3) * NA;
  const int bk = tid / TPR, bj = (tid % TPR) * BV;
  const int64_t pld = d.ld;  // column stride of the panel
  const T *Gb = G + (int64_t)min(b0 + ba_j, nc - 1) * pld;  // backward: this thread's column
  T ra[NA], rb[BV], sc = T(1);
  unsigned amask = 0;
  bool bok = false;
  auto load = [&](int c, int32_t dof) {
    amask = 0;
    if constexpr (FWD) {
      const int j = c + fa_k, jc = min(j, hi - 1);
#pragma unroll
      for (int q = 0; q < NA; ++q) {
        const int i = b0 + fa_i + q;
        ra[q] = G[(int64_t)jc * pld + min(i, m - 1)];
        amask |= (i < m && j < hi && (i >= nc || j <= i)) ? (1u << q) : 0u;
      }
    } else {
      const int j = b0 + ba_j;
#pragma unroll
      for (int q = 0; q < NA; ++q) {
        const int i = c + ba_k + q;
        ra[q] = Gb[min(i, hi - 1)];
        amask |= (i < hi && j < nc && (i >= nc || i >= j)) ? (1u << q) : 0u;
      }
    }
    bok = c + bk < hi;
    if constexpr (!FWD) {
      const T di = dinv[dof];
      sc = c + bk < nc ? di : T(1);
    }
    load_row<T, BV>(src + (int64_t)dof * ld + k0 + bj, rb);
  };
  typename Mma<T>::acc acc[2][NCB];
#pragma unroll
  for (int r = 0; r < 2; ++r)
#pragma unroll
    for (int c = 0; c < NCB; ++c) acc[r][c] = typename Mma<T>::acc{0, 0, 0, 0};
  load(t.lo, rw[min(t.lo + bk, hi - 1)]);
  int32_t gnext = rw[min(t.lo + KC + bk, hi - 1)];
  for (int c = t.lo; c < hi; c += KC) {
    __syncthreads();
#pragma unroll
    for (int q = 0; q < NA; ++q) {
      const T v = (amask >> q) & 1u ? ra[q] : T(0);
      if constexpr (FWD) sA[fa_k][fa_i + q] = v;
      else sA[ba_k + q][ba_j] = v;
    }
#pragma unroll
    for (int v = 0; v < BV; ++v) {
      if constexpr (FWD) sB[bk][bj + v] = bok ? rb[v] : T(0);
      else sB[bk][bj + v] = bok ? sc * rb[v] : T(0);
    }
    __syncthreads();
    if (c + KC < hi) {
      load(c + KC, gnext);
      gnext = rw[min(c + 2 * KC + bk, hi - 1)];
    }
    mma_chunk<T, BN, KC>(sA, sB, wr, wc, lane, acc);
  }
  // whole contraction in this tile: forward [0, min(nc, r0 + 64)) for a
  // block with own rows, backward [j0, m)
  const bool whole = FWD ? (t.lo == 0 && hi == (b0 < nc ? min(nc, b0 + kMR) : nc))
                         : (t.lo == b0 && hi == m);
  const int col0 = (int)k0 + wc + (lane & 15);
#pragma unroll
  for (int r = 0; r < 2; ++r)
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int i = b0 + wr + 16 * r + Mma<T>::row(lane, q);
      if (i >= (FWD ? m : nc)) continue;
      const int64_t o = (int64_t)rw[i] * ld + col0;
#pragma unroll
      for (int c = 0; c < NCB; ++c) {
        if (col0 + 16 * c >= kreal) continue;
        const T v = acc[r][c][q];
        if constexpr (FWD) {
          if (i >= nc) atomicAdd(src + o + 16 * c, -v);
          else if (whole) y[o + 16 * c] = v;
          else atomicAdd(y + o + 16 * c, v);
        } else {
          if (whole) z[o + 16 * c] = (double)v;
          else atomicAdd(z + o + 16 * c, (double)v);
        }
      }
    }
}

// y <- -z on the DOFs of one backward level once they are final: later
// (lower) levels read them as update-row inputs.
template <typename T>
__global__ void k_mconv(const int32_t *__restrict__ dofs, int64_t cnt, int ld,
                        const double *__restrict__ z, T *y) {
  const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (idx >= cnt * ld) return;
  const int64_t e = idx / ld;
  const int64_t o = (int64_t)dofs[e] * ld + (idx - e * ld);
  y[o] = (T)(-z[o]);
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

// ---------------------------------------------------- projected Gauss-Seidel
// Lane-crossing helpers on the two 32-bit halves of a double.
template <int CTRL>
__device__ inline double dpp_mov(double v) {
  const long long x = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)x, CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(x >> 32), CTRL, 0xF, 0xF, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

__device__ inline double readlane_d(double v, int l) {
  const long long x = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)x, l);
  const int hi = __builtin_amdgcn_readlane((int)(x >> 32), l);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// Sum over the wavefront, the same value in every lane: within each row of 16
// lanes pairwise exchanges (lane ^ 1, lane ^ 2, then the mirrors that pair
// the two quads of each half and the two halves of the row), each pairing two
// lanes that then hold the same sum; then the four row sums read as scalars.
__device__ inline double wave_total(double v) {
  v += dpp_mov<0xB1>(v);   // quad_perm [1,0,3,2]
  v += dpp_mov<0x4E>(v);   // quad_perm [2,3,0,1]
  v += dpp_mov<0x141>(v);  // row_half_mirror
  v += dpp_mov<0x140>(v);  // row_mirror
  return (readlane_d(v, 0) + readlane_d(v, 16)) + (readlane_d(v, 32) + readlane_d(v, 48));
}

// Projected Gauss-Seidel on lambda >= 0, W lambda - c >= 0, complementary,
// by one wavefront.  Lane l holds the multipliers l + 64 q (q < NR) in
// registers; c, 1 / W_ii and W_{i,i-1} are broadcast reads from LDS.  The rows
// of W stream through a ring of D register buffers, each refilled with the
// row D positions ahead (wrapping into the next sweep) as soon as it has been
// used.  Row products are computed one row ahead: while row i is updated,
// the product of row i + 1 with the multipliers as they stand before that
// update is reduced, and the update of row i + 1 adds W_{i+1,i} times the
// change of lambda_i.  So the reduction of one row overlaps the scalar update
// of the previous one.  Every lane computes the same update; the owner lane
// of lambda_i keeps it (the selects are written so that the compiler keeps
// the multipliers in registers).  A sweep whose largest change is <= tol *
// max(lambda) ends the iteration.  A row whose diagonal is not positive keeps
// its multiplier.
template <int NR, int D>
__global__ __launch_bounds__(64) void k_pgs(int kc, const double *__restrict__ W,
                                            const double *__restrict__ c, double *lam,
                                            int max_sweeps, double tol, double *info) {
  __shared__ double s_c[64 * NR], s_inv[64 * NR], s_sub[64 * NR];
  const int lane = (int)threadIdx.x;
  for (int j = lane; j < 64 * NR; j += 64) {
    const bool ok = j < kc;
    s_c[j] = ok ? c[j] : 0.0;
    const double wii = ok ? W[(int64_t)j * kc + j] : 0.0;
    s_inv[j] = wii > 0.0 ? 1.0 / wii : 0.0;
    s_sub[j] = ok ? W[(int64_t)j * kc + (j + kc - 1) % kc] : 0.0;
  }
  double lr[NR];
#pragma unroll
  for (int q = 0; q < NR; ++q) {
    const int j = lane + 64 * q;
    lr[q] = j < kc ? lam[j] : 0.0;
  }
  double buf[D][NR];
#pragma unroll
  for (int d = 0; d < D; ++d) {
    const int64_t r = (int64_t)(d % kc) * kc;
#pragma unroll
    for (int q = 0; q < NR; ++q) buf[d][q] = W[r + min(lane + 64 * q, kc - 1)];
  }
  __syncthreads();
  // product of row 0 with the starting multipliers; slot 0 then takes row D
  double pre = 0.0;
#pragma unroll
  for (int q = 0; q < NR; ++q) pre += buf[0][q] * lr[q];
  pre = wave_total(pre);
  {
    const int64_t nr = (int64_t)(D % kc) * kc;
#pragma unroll
    for (int q = 0; q < NR; ++q) buf[0][q] = W[nr + min(lane + 64 * q, kc - 1)];
  }
  int row = 0, sweeps = 0;
  int lrow = (D + 1) % kc;  // row the next refill loads: row + 1 + D (mod kc)
  double dprev = 0.0, dmax = 0.0, lmax = 0.0, last = 0.0;
  bool done = max_sweeps <= 0;
  // rows run in groups of D with no branch around the loads (a group may run
  // past the end of the last sweep: those rows are computed but not kept),
  // so the wait for each ring slot counts only the loads issued before it
  while (!done) {
#pragma unroll
    for (int d = 0; d < D; ++d) {
      const int nxt = (d + 1) % D;  // ring slot of row + 1
      const int own = row & 63, qi = row >> 6;
      const double ci = s_c[row], inv = s_inv[row], sub = s_sub[row];
      double li = lr[0];
#pragma unroll
      for (int q = 1; q < NR; ++q) {
        li = q == qi ? lr[q] : li;
        asm volatile("" : "+v"(li));
      }
      li = readlane_d(li, own);
      // product of row + 1 with the multipliers before the update of row
      double pn = 0.0;
#pragma unroll
      for (int q = 0; q < NR; ++q) pn += buf[nxt][q] * lr[q];
      const double p = pre + sub * dprev;
      const double nl = inv > 0.0 ? fmax(0.0, li - (p - ci) * inv) : li;
      const bool keep = lane == own && !done;
#pragma unroll
      for (int q = 0; q < NR; ++q) {
        lr[q] = keep && q == qi ? nl : lr[q];
        asm volatile("" : "+v"(lr[q]));
      }
      pn = wave_total(pn);
      dprev = nl - li;
      dmax = fmax(dmax, fabs(dprev));
      lmax = fmax(lmax, nl);
      pre = pn;
      // unconditional loads, clamped to the row: the entries of lanes past
      // the end meet lambda = 0 in the product, so they need no masking (a
      // select here would wait for the load at once)
      const int64_t nr = (int64_t)lrow * kc;
#pragma unroll
      for (int q = 0; q < NR; ++q) buf[nxt][q] = W[nr + min(lane + 64 * q, kc - 1)];
      lrow = lrow + 1 == kc ? 0 : lrow + 1;
      if (++row == kc) {
        row = 0;
        if (!done) {
          ++sweeps;
          last = dmax;
          done = sweeps >= max_sweeps || dmax <= tol * lmax;
        }
        dmax = 0.0;
        lmax = 0.0;
      }
    }
  }
#pragma unroll
  for (int q = 0; q < NR; ++q) {
    const int j = lane + 64 * q;
    if (j < kc) lam[j] = lr[q];
  }
  if (lane == 0 && info) {
    info[0] = (double)sweeps;
    info[1] = last;
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
                      const SnDev *sn, const int32_t *rows, const T *panels, T *w, T *y, int ld,
                      int k) {
  if (n_tiles <= 0 || n_kb <= 0) return;
  const int units = n_tiles * n_kb, per = (units + kXcds - 1) / kXcds;
  const unsigned grid = (unsigned)(per * kXcds);
  if (bn == 128)
    k_msweep<T, 128, true><<<grid, 256, 0, st>>>(tiles, units, n_kb, per, sn, rows, panels,
                                                  nullptr, w, y, nullptr, ld, k);
  else
    k_msweep<T, 64, true><<<grid, 256, 0, st>>>(tiles, units, n_kb, per, sn, rows, panels,
                                                 nullptr, w, y, nullptr, ld, k);
}

template <typename T>
void launch_multi_bwd(hipStream_t st, const MTile *tiles, int n_tiles, int n_kb, int bn,
                      const SnDev *sn, const int32_t *rows, const T *panels, const T *dinv, T *y,
                      double *z, int ld, int k) {
  if (n_tiles <= 0 || n_kb <= 0) return;
  const int units = n_tiles * n_kb, per = (units + kXcds - 1) / kXcds;
  const unsigned grid = (unsigned)(per * kXcds);
  if (bn == 128)
    k_msweep<T, 128, false><<<grid, 256, 0, st>>>(tiles, units, n_kb, per, sn, rows, panels,
                                                   dinv, y, nullptr, z, ld, k);
  else
    k_msweep<T, 64, false><<<grid, 256, 0, st>>>(tiles, units, n_kb, per, sn, rows, panels,
                                                  dinv, y, nullptr, z, ld, k);
}

template <typename T>
void launch_multi_conv(hipStream_t st, const int32_t *dofs, int64_t cnt, int ld, const double *z,
                       T *y) {
  if (cnt * ld > 0) k_mconv<T><<<grid_for(cnt * ld), 256, 0, st>>>(dofs, cnt, ld, z, y);
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
  // register ring depth D shrinks as the rows get longer (D * NR <= 64)
  if (kc <= 64) k_pgs<1, 8><<<1, 64, 0, st>>>(kc, W, c, lam, max_sweeps, tol, info);
  else if (kc <= 128) k_pgs<2, 8><<<1, 64, 0, st>>>(kc, W, c, lam, max_sweeps, tol, info);
  else if (kc <= 256) k_pgs<4, 8><<<1, 64, 0, st>>>(kc, W, c, lam, max_sweeps, tol, info);
  else if (kc <= 512) k_pgs<8, 8><<<1, 64, 0, st>>>(kc, W, c, lam, max_sweeps, tol, info);
  else if (kc <= 1024) k_pgs<16, 4><<<1, 64, 0, st>>>(kc, W, c, lam, max_sweeps, tol, info);
  else if (kc <= 2048) k_pgs<32, 2><<<1, 64, 0, st>>>(kc, W, c, lam, max_sweeps, tol, info);
  else k_pgs<64, 1><<<1, 64, 0, st>>>(kc, W, c, lam, max_sweeps, tol, info);
}

#define FE_INST(T)                                                                             \
  template void launch_multi_prep<T>(hipStream_t, int64_t, int, int, const double *, T *, T *, \
                                     double *, const uint8_t *);                               \
  template void launch_multi_zero<T>(hipStream_t, int64_t, T *, T *, double *);                \
  template void launch_multi_fwd<T>(hipStream_t, const MTile *, int, int, int, const SnDev *,  \
                                    const int32_t *, const T *, T *, T *, int, int);           \
  template void launch_multi_bwd<T>(hipStream_t, const MTile *, int, int, int, const SnDev *,  \
                                    const int32_t *, const T *, const T *, T *, double *, int, \
                                    int);                                                      \
  template void launch_multi_conv<T>(hipStream_t, const int32_t *, int64_t, int,               \
                                     const double *, T *);                                     \
  template void launch_h_scatter<T>(hipStream_t, int, int64_t, int64_t, const int32_t *,       \
                                    const int32_t *, const double *, int, T *, double *,       \
                                    const uint8_t *, int *);
FE_INST(float)
FE_INST(double)
#undef FE_INST

}  // namespace fe
