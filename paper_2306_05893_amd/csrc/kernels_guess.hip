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

// W = A V for the m history vectors: G lanes per row as in k_spmv; each entry
// of the row is used with the m interleaved values of its column (one 64-byte
// row of V), the row sums reduced over the G lanes, lane sub writes column sub.
template <typename T, int G>
__global__ __launch_bounds__(kBlock) void k_hist_spmv(int64_t n, int m,
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
  if (row < n) W[row * kHist + sub] = sub < m ? mine : 0.0;
}

// Per-block partials of G_ij = V_i . W_j (i <= j) and r_i = V_i . b, stored
// value-major: part[q * kHistBlocks + block].
__global__ __launch_bounds__(kBlock) void k_hist_dots(int64_t n, const double *__restrict__ V,
                                                      const double *__restrict__ W,
                                                      const double *__restrict__ b,
                                                      double *part) {
  __shared__ double s_red[kBlock / 64][kHistDots];
  double acc[kHistDots];
#pragma unroll
  for (int q = 0; q < kHistDots; ++q) acc[q] = 0.0;
  const int64_t stride = (int64_t)gridDim.x * kBlock;
  for (int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x; k < n; k += stride) {
    double v[kHist], w[kHist];
    const double2 *vr = reinterpret_cast<const double2 *>(V + k * kHist);
    const double2 *wr = reinterpret_cast<const double2 *>(W + k * kHist);
#pragma unroll
    for (int j = 0; j < kHist / 2; ++j) {
      const double2 a = vr[j], c = wr[j];
      v[2 * j] = a.x;
      v[2 * j + 1] = a.y;
      w[2 * j] = c.x;
      w[2 * j + 1] = c.y;
    }
    const double bk = b[k];
    int q = 0;
#pragma unroll
    for (int i = 0; i < kHist; ++i)
#pragma unroll
      for (int j = i; j < kHist; ++j) acc[q++] += v[i] * w[j];
#pragma unroll
    for (int i = 0; i < kHist; ++i) acc[q++] += v[i] * bk;
  }
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int q = 0; q < kHistDots; ++q) {
    const double t = wave_sum(acc[q]);
    if (lane == 0) s_red[wv][q] = t;
  }
  __syncthreads();
  if (threadIdx.x < kHistDots) {
    double t = 0.0;
    for (int i = 0; i < kBlock / 64; ++i) t += s_red[i][threadIdx.x];
    part[threadIdx.x * kHistBlocks + blockIdx.x] = t;
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
  __syncthreads();
  if (threadIdx.x != 0) return;
  constexpr double kHistDrop = 1e-13;
  auto gidx = [](int i, int j) {  // upper-triangle index of (min, max)
    const int a = i < j ? i : j, b = i < j ? j : i;
    return a * kHist - a * (a - 1) / 2 + (b - a);
  };
  int ord[kHist];
  bool keep[kHist];
  double L[kHist][kHist], y[kHist], c[kHist];
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

// x = V coef
__global__ __launch_bounds__(kBlock) void k_hist_combine(int64_t n, const double *__restrict__ V,
                                                         const double *__restrict__ coef,
                                                         double *__restrict__ x) {
  const int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (k >= n) return;
  const double2 *vr = reinterpret_cast<const double2 *>(V + k * kHist);
  double s = 0.0;
#pragma unroll
  for (int j = 0; j < kHist / 2; ++j) {
    const double2 a = vr[j];
    s += coef[2 * j] * a.x + coef[2 * j + 1] * a.y;
  }
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
  k_hist_spmv<T, kHist><<<rb, kBlock, 0, st>>>(n, m, row_ptr, col, val, V, W);
  k_hist_dots<<<kHistBlocks, kBlock, 0, st>>>(n, V, W, b, part);
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
