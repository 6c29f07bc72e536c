// Initial guess of a step's CG from the solutions of earlier steps (the
// paper leaves x0 open): the A-norm projection of the new solution onto the
// span of the last m solutions, x0 = V c with (V^T A V) c = V^T b (Fischer,
// "Projection techniques for iterative solution of Ax = b with successive
// right-hand sides", 1998).  Per step: one pass over A with the m vectors at
// once, the m(m+1)/2 + m dot products, an m x m Cholesky with the newest
// vectors first (a vector that is nearly a combination of newer ones is
// dropped), and x0 = V c.
#include "device.hpp"

namespace fe {

namespace {

constexpr int kBlock = 256;

__device__ inline double wave_sum(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// V holds the m vectors interleaved, DOF k's values at
// V[k * kHist .. k * kHist + m).
constexpr int kHistDots = kHist * (kHist + 1) / 2 + kHist;  // G (upper) and V^T b
constexpr int kHistBlocks = 256;

// W = A V for every slot of the ring (the m newest vectors may sit in any
// of them): G lanes per row as in k_spmv; each entry of the row is used with
// the kHist interleaved values of its column (one row of V), the row sums
// reduced over the G lanes, lane sub writes column sub.  Slots never filled
// give columns that the solve does not read.
template <typename T, int G>
__global__ __launch_bounds__(kBlock) void k_hist_spmv(int64_t n,
                                                      const int32_t *__restrict__ row_ptr,
                                                      const int32_t *__restrict__ col,
                                                      const T *__restrict__ val,
                                                      const double *__restrict__ V,
                                                      double *__restrict__ W) {
  static_assert(G == kHist, "one lane per history column at the write");
  const int64_t row = ((int64_t)blockIdx.x * kBlock + threadIdx.x) / G;
  const int sub = threadIdx.x & (G - 1);
  double acc[kHist];
#pragma unroll
  for (int j = 0; j < kHist; ++j) acc[j] = 0.0;
  if (row < n) {
    const int32_t k0 = row_ptr[row], k1 = row_ptr[row + 1];
    for (int32_t k = k0 + sub; k < k1; k += G) {
      const double a = (double)val[k];
      const double2 *vr = reinterpret_cast<const double2 *>(V + (int64_t)col[k] * kHist);
#pragma unroll
      for (int j = 0; j < kHist / 2; ++j) {
        const double2 x = vr[j];
        acc[2 * j] += a * x.x;
        acc[2 * j + 1] += a * x.y;
      }
    }
  }
#pragma unroll
  for (int j = 0; j < kHist; ++j)
    for (int off = G / 2; off > 0; off >>= 1) acc[j] += __shfl_xor(acc[j], off, G);
  double mine = acc[0];
#pragma unroll
  for (int j = 1; j < kHist; ++j) mine = sub == j ? acc[j] : mine;
  if (row < n) W[row * kHist + sub] = mine;
}

// Per-block partials of G_ij = V_i . W_j (i <= j) and r_i = V_i . b, stored
// value-major: part[q * kHistBlocks + block].  blockIdx.y takes rows
// [kHistRG y, kHistRG (y + 1)) of G (all kHist columns are accumulated, the
// ones below the diagonal are not written), so that a thread holds
// kHistRG (kHist + 1) sums.
constexpr int kHistRG = 4;
constexpr int kHistAcc = kHistRG * (kHist + 1);
static_assert(kHist % kHistRG == 0, "whole row groups");

__device__ inline int hist_gidx(int i, int j) {  // upper-triangle index of (i, j), i <= j
  return i * kHist - i * (i - 1) / 2 + (j - i);
}

__global__ __launch_bounds__(kBlock) void k_hist_dots(int64_t n, const double *__restrict__ V,
                                                      const double *__restrict__ W,
                                                      const double *__restrict__ b,
                                                      double *part) {
  __shared__ double s_red[kBlock / 64][kHistAcc];
  const int i0 = blockIdx.y * kHistRG;
  double acc[kHistAcc];
#pragma unroll
  for (int q = 0; q < kHistAcc; ++q) acc[q] = 0.0;
  const int64_t stride = (int64_t)gridDim.x * kBlock;
  for (int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x; k < n; k += stride) {
    double v[kHistRG], w[kHist];
    const double2 *vr = reinterpret_cast<const double2 *>(V + k * kHist + i0);
    const double2 *wr = reinterpret_cast<const double2 *>(W + k * kHist);
#pragma unroll
    for (int j = 0; j < kHistRG / 2; ++j) {
      const double2 a = vr[j];
      v[2 * j] = a.x;
      v[2 * j + 1] = a.y;
    }
#pragma unroll
    for (int j = 0; j < kHist / 2; ++j) {
      const double2 c = wr[j];
      w[2 * j] = c.x;
      w[2 * j + 1] = c.y;
    }
    const double bk = b[k];
#pragma unroll
    for (int r = 0; r < kHistRG; ++r) {
#pragma unroll
      for (int j = 0; j < kHist; ++j) acc[r * (kHist + 1) + j] += v[r] * w[j];
      acc[r * (kHist + 1) + kHist] += v[r] * bk;
    }
  }
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int q = 0; q < kHistAcc; ++q) {
    const double t = wave_sum(acc[q]);
    if (lane == 0) s_red[wv][q] = t;
  }
  __syncthreads();
  if (threadIdx.x < kHistAcc) {
    const int r = threadIdx.x / (kHist + 1), j = threadIdx.x % (kHist + 1), i = i0 + r;
    double t = 0.0;
    for (int u = 0; u < kBlock / 64; ++u) t += s_red[u][threadIdx.x];
    // column kHist holds V_i . b, stored after the upper triangle of G
    const int q = j == kHist ? kHist * (kHist + 1) / 2 + i : (j >= i ? hist_gidx(i, j) : -1);
    if (q >= 0) part[q * kHistBlocks + blockIdx.x] = t;
  }
}

// One block: sum the partials in a fixed order, then (thread 0) the
// Cholesky factorisation of G over the history vectors taken newest first,
// dropping a vector whose pivot is below kHistDrop of its diagonal (nearly a
// combination of the newer ones), and the solve for the coefficients.
__global__ __launch_bounds__(kBlock) void k_hist_solve(int m, int newest, const double *part,
                                                       int nparts, double *coef) {
  __shared__ double s_val[kHistDots];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  for (int q = wv; q < kHistDots; q += kBlock / 64) {
    double t = 0.0;
    for (int i = lane; i < nparts; i += 64) t += part[q * kHistBlocks + i];
    t = wave_sum(t);
    if (lane == 0) s_val[q] = t;
  }
  // the factor and the triangular solves in LDS (one thread works on them)
  __shared__ double L[kHist][kHist];
  __shared__ double y[kHist], c[kHist];
  __shared__ int ord[kHist];
  __shared__ bool keep[kHist];
  __syncthreads();
  if (threadIdx.x != 0) return;
  constexpr double kHistDrop = 1e-13;
  auto gidx = [](int i, int j) { return i < j ? hist_gidx(i, j) : hist_gidx(j, i); };
  for (int t = 0; t < m; ++t) ord[t] = (newest - t + kHist) % kHist;
  for (int t = 0; t < m; ++t) {
    const int i = ord[t];
    const double gii = s_val[gidx(i, i)];
    double d = gii;
    for (int u = 0; u < t; ++u)
      if (keep[u]) d -= L[t][u] * L[t][u];
    keep[t] = gii > 0.0 && d > kHistDrop * gii;
    if (!keep[t]) continue;
    L[t][t] = sqrt(d);
    for (int s = t + 1; s < m; ++s) {
      double x = s_val[gidx(ord[s], i)];
      for (int u = 0; u < t; ++u)
        if (keep[u]) x -= L[s][u] * L[t][u];
      L[s][t] = x / L[t][t];
    }
  }
  const int rb = kHist * (kHist + 1) / 2;
  for (int t = 0; t < m; ++t) {
    if (!keep[t]) { y[t] = 0.0; continue; }
    double x = s_val[rb + ord[t]];
    for (int u = 0; u < t; ++u)
      if (keep[u]) x -= L[t][u] * y[u];
    y[t] = x / L[t][t];
  }
  for (int t = m - 1; t >= 0; --t) {
    if (!keep[t]) { c[t] = 0.0; continue; }
    double x = y[t];
    for (int s = t + 1; s < m; ++s)
      if (keep[s]) x -= L[s][t] * c[s];
    c[t] = x / L[t][t];
  }
  for (int j = 0; j < kHist; ++j) coef[j] = 0.0;
  for (int t = 0; t < m; ++t) coef[ord[t]] = c[t];
}

// x = V coef over the slots with a coefficient (the others may never have
// been filled: their contents are not read)
__global__ __launch_bounds__(kBlock) void k_hist_combine(int64_t n, const double *__restrict__ V,
                                                         const double *__restrict__ coef,
                                                         double *__restrict__ x) {
  const int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (k >= n) return;
  const double *vr = V + k * kHist;
  double s = 0.0;
#pragma unroll
  for (int j = 0; j < kHist; ++j)
    if (coef[j] != 0.0) s += coef[j] * vr[j];
  x[k] = s;
}

// V[:, slot] = x
__global__ __launch_bounds__(kBlock) void k_hist_push(int64_t n, int slot, const double *x,
                                                      double *V) {
  const int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (k < n) V[k * kHist + slot] = x[k];
}

}  // namespace

template <typename T>
void launch_hist_guess(hipStream_t st, int64_t n, int m, int newest, const int32_t *row_ptr,
                       const int32_t *col, const T *val, const double *V, double *W,
                       const double *b, double *part, double *coef, double *x) {
  const unsigned rb = (unsigned)((n * kHist + kBlock - 1) / kBlock);
  k_hist_spmv<T, kHist><<<rb, kBlock, 0, st>>>(n, row_ptr, col, val, V, W);
  k_hist_dots<<<dim3(kHistBlocks, kHist / kHistRG), kBlock, 0, st>>>(n, V, W, b, part);
  k_hist_solve<<<1, kBlock, 0, st>>>(m, newest, part, kHistBlocks, coef);
  k_hist_combine<<<(unsigned)((n + kBlock - 1) / kBlock), kBlock, 0, st>>>(n, V, coef, x);
}

void launch_hist_push(hipStream_t st, int64_t n, int slot, const double *x, double *V) {
  k_hist_push<<<(unsigned)((n + kBlock - 1) / kBlock), kBlock, 0, st>>>(n, slot, x, V);
}

int64_t hist_part_doubles() { return (int64_t)kHistDots * kHistBlocks + kHist; }

#define FE_INST(T)                                                                          \
  template void launch_hist_guess<T>(hipStream_t, int64_t, int, int, const int32_t *,       \
                                     const int32_t *, const T *, const double *, double *,  \
                                     const double *, double *, double *, double *);
FE_INST(float)
FE_INST(double)
#undef FE_INST

}  // namespace fe
