// Element-wise kernels and deterministic reductions (HBM-bound): Frobenius norms, the scaled
// Newton update A_k = (mu A + mu^-1 A^-1)/2 (eq 3.1a) fused with ||A_k - A_{k-1}||_F,
// ||A_k||_F and ||A_k + I||_1, casts to the solver precision, fills and block copies.
// Reductions are two-stage with a fixed combination order (no floating-point atomics), so
// results are bit-reproducible.
#include <algorithm>
#include <cmath>

#include "common.hpp"
#include "internal.hpp"

namespace lyap {
namespace {

constexpr int RB = 256;      // threads per reduction block
constexpr int RPARTS = 256;  // reduction blocks

__global__ void k_fill_int(int* p, int count, int value) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) p[i] = value;
}

__global__ void k_fill_f64(double* p, long count, double value) {
  long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) p[i] = value;
}

__global__ void k_copy_block(int rows, int cols, const double* __restrict__ src, long lds,
                             double* __restrict__ dst, long ldd, const double* __restrict__ cs,
                             double scale) {
  long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
  long total = (long)rows * cols;
  if (idx >= total) return;
  int i = (int)(idx / cols), j = (int)(idx % cols);
  double v = src[(long)i * lds + j] * scale;
  if (cs) v *= cs[j];
  dst[(long)i * ldd + j] = v;
}

template <class T>
__global__ void k_cast(int rows, int cols, const double* __restrict__ src, long lds,
                       T* __restrict__ dst) {
  long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
  long total = (long)rows * cols;
  if (idx >= total) return;
  int i = (int)(idx / cols), j = (int)(idx % cols);
  dst[idx] = (T)(float)src[(long)i * lds + j];
}
template <>
__global__ void k_cast<double>(int rows, int cols, const double* __restrict__ src, long lds,
                               double* __restrict__ dst) {
  long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
  long total = (long)rows * cols;
  if (idx >= total) return;
  int i = (int)(idx / cols), j = (int)(idx % cols);
  dst[idx] = src[(long)i * lds + j];
}
template <>
__global__ void k_cast<float>(int rows, int cols, const double* __restrict__ src, long lds,
                              float* __restrict__ dst) {
  long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
  long total = (long)rows * cols;
  if (idx >= total) return;
  int i = (int)(idx / cols), j = (int)(idx % cols);
  dst[idx] = (float)src[(long)i * lds + j];
}

__device__ inline double block_sum(double v, double* red) {
  red[threadIdx.x] = v;
  __syncthreads();
  for (int s = RB / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  double r = red[0];
  __syncthreads();
  return r;
}

__global__ void k_sumsq_partial(int rows, int cols, const double* __restrict__ A, long lda,
                                double* __restrict__ part) {
  __shared__ double red[RB];
  double acc = 0.0;
  if (cols >= RB / 4) {
    // rows strided over blocks, columns over threads (coalesced, no index division); four
    // independent accumulators keep several loads in flight per thread
    double acc4[4] = {0.0, 0.0, 0.0, 0.0};
    for (int i = blockIdx.x; i < rows; i += gridDim.x) {
      const double* a = A + (long)i * lda;
      int j = threadIdx.x;
      for (; j + 3 * RB < cols; j += 4 * RB) {
#pragma unroll
        for (int u = 0; u < 4; ++u) acc4[u] += a[j + u * RB] * a[j + u * RB];
      }
      for (; j < cols; j += RB) acc4[0] += a[j] * a[j];
    }
    acc = (acc4[0] + acc4[1]) + (acc4[2] + acc4[3]);
  } else {
    long total = (long)rows * cols;
    for (long e = (long)blockIdx.x * RB + threadIdx.x; e < total; e += (long)gridDim.x * RB) {
      int i = (int)(e / cols), j = (int)(e % cols);
      double v = A[(long)i * lda + j];
      acc += v * v;
    }
  }
  double s = block_sum(acc, red);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

__global__ void k_sum_parts(int nparts, const double* __restrict__ part, double* __restrict__ out) {
  __shared__ double red[RB];
  double acc = 0.0;
  for (int i = threadIdx.x; i < nparts; i += RB) acc += part[i];
  double s = block_sum(acc, red);
  if (threadIdx.x == 0) *out = s;
}

// Newton update, tiled: block (x, y) handles the row range x of height ``rows_per`` and the
// column chunk y of RB columns (one column per thread).  It writes the column partial sums of
// |Anew + I| over its rows to colpart[x][j] and its partial sums of squares to part; all
// partials are combined afterwards in a fixed order.
__global__ void k_newton(int n, const double* __restrict__ A, long lda,
                         const double* __restrict__ Ai, long ldi, const double* __restrict__ mu_dev,
                         double* __restrict__ An, long ldn, int rows_per, double* __restrict__ part,
                         double* __restrict__ colpart) {
  __shared__ double red[RB];
  const double mu = *mu_dev;
  const double hm = 0.5 * mu, hi = 0.5 / mu;
  const int r0 = blockIdx.x * rows_per, r1 = min(n, r0 + rows_per);
  const int j = blockIdx.y * RB + threadIdx.x;
  double sd = 0.0, sa = 0.0, cs = 0.0;
  if (j < n) {
#pragma unroll 4
    for (int i = r0; i < r1; ++i) {
      const double a = A[(long)i * lda + j];
      const double x = hm * a + hi * Ai[(long)i * ldi + j];
      An[(long)i * ldn + j] = x;
      const double d = x - a;
      sd += d * d;
      sa += x * x;
      cs += fabs(x + (i == j ? 1.0 : 0.0));
    }
    colpart[(long)blockIdx.x * n + j] = cs;
  }
  const double s1 = block_sum(sd, red);
  const double s2 = block_sum(sa, red);
  if (threadIdx.x == 0) {
    const int b = blockIdx.y * gridDim.x + blockIdx.x, nb = gridDim.x * gridDim.y;
    part[b] = s1;
    part[nb + b] = s2;
  }
}

// colsum[j] = sum_x colpart[x][j] in order of x; colmax[block] = max over the block's columns.
__global__ void k_colsum(int n, int nparts, const double* __restrict__ colpart,
                         double* __restrict__ colsum, double* __restrict__ colmax) {
  __shared__ double red[RB];
  const int j = blockIdx.x * RB + threadIdx.x;
  double s = 0.0;
  if (j < n) {
    for (int b = 0; b < nparts; ++b) s += colpart[(long)b * n + j];
    colsum[j] = s;
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int h = RB / 2; h > 0; h >>= 1) {
    if (threadIdx.x < h) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + h]);
    __syncthreads();
  }
  if (threadIdx.x == 0) colmax[blockIdx.x] = red[0];
}

__global__ void k_newton_finish(int nb, const double* __restrict__ part, int nchunks,
                                const double* __restrict__ colmax, double* __restrict__ out4) {
  __shared__ double red[RB];
  double m = 0.0;
  for (int i = threadIdx.x; i < nchunks; i += RB) m = fmax(m, colmax[i]);
  red[threadIdx.x] = m;
  __syncthreads();
  for (int h = RB / 2; h > 0; h >>= 1) {
    if (threadIdx.x < h) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + h]);
    __syncthreads();
  }
  const double onenorm = red[0];
  __syncthreads();
  double a = 0.0, b = 0.0;
  for (int i = threadIdx.x; i < nb; i += RB) {
    a += part[i];
    b += part[nb + i];
  }
  const double sa = block_sum(a, red);
  const double sb = block_sum(b, red);
  if (threadIdx.x == 0) {
    out4[0] = sa;
    out4[1] = sb;
    out4[2] = onenorm;
  }
}

__global__ void k_mu(const double* inv_ss, const double* a_ss, int scaling, double* mu) {
  if (scaling) *mu = sqrt(sqrt(*inv_ss) / sqrt(*a_ss));
  else *mu = 1.0;
}

// out[0] = sum_ij w[j] X_ij^2 (one block, fixed order).
__global__ void k_colw_sumsq(int rows, int cols, const double* __restrict__ X, long ldx,
                             const double* __restrict__ w, double* __restrict__ out) {
  __shared__ double red[RB];
  double acc = 0.0;
  for (long e = threadIdx.x; e < (long)rows * cols; e += RB) {
    const int i = (int)(e / cols), j = (int)(e % cols);
    const double x = X[(long)i * ldx + j];
    acc += w[j] * x * x;
  }
  const double t = block_sum(acc, red);
  if (threadIdx.x == 0) out[0] = t;
}

// out[c] = sum_i w[i] X_ic^2, one thread per column.
__global__ void k_roww_colsumsq(int rows, int cols, const double* __restrict__ X, long ldx,
                                const double* __restrict__ w, double* __restrict__ out) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= cols) return;
  double acc = 0.0;
  for (int i = 0; i < rows; ++i) {
    const double x = X[(long)i * ldx + c];
    acc += w[i] * x * x;
  }
  out[c] = acc;
}

inline unsigned nblk(long total, int bs = 256) { return (unsigned)((total + bs - 1) / bs); }

}  // namespace

int fill_int(hipStream_t s, int* p, int count, int value) {
  if (count <= 0) return LYAP_OK;
  hipLaunchKernelGGL(k_fill_int, dim3(nblk(count)), dim3(256), 0, s, p, count, value);
  LYAP_HIP(hipGetLastError());
  return LYAP_OK;
}

int fill_f64(hipStream_t s, double* p, long count, double value) {
  if (count <= 0) return LYAP_OK;
  hipLaunchKernelGGL(k_fill_f64, dim3(nblk(count)), dim3(256), 0, s, p, count, value);
  LYAP_HIP(hipGetLastError());
  return LYAP_OK;
}

int copy_block(hipStream_t s, int rows, int cols, const double* src, long lds, double* dst,
               long ldd, const double* colscale, double scale) {
  long total = (long)rows * cols;
  if (total <= 0) return LYAP_OK;
  hipLaunchKernelGGL(k_copy_block, dim3(nblk(total)), dim3(256), 0, s, rows, cols, src, lds, dst,
                     ldd, colscale, scale);
  LYAP_HIP(hipGetLastError());
  return LYAP_OK;
}

int cast_store(hipStream_t s, Store st, int rows, int cols, const double* src, long lds,
               void* dst) {
  long total = (long)rows * cols;
  if (total <= 0) return LYAP_OK;
  dim3 g(nblk(total)), b(256);
  switch (st) {
    case Store::F64:
      hipLaunchKernelGGL(k_cast<double>, g, b, 0, s, rows, cols, src, lds, (double*)dst);
      break;
    case Store::F32:
      hipLaunchKernelGGL(k_cast<float>, g, b, 0, s, rows, cols, src, lds, (float*)dst);
      break;
    case Store::F16:
      hipLaunchKernelGGL(k_cast<_Float16>, g, b, 0, s, rows, cols, src, lds, (_Float16*)dst);
      break;
    case Store::BF16:
      hipLaunchKernelGGL(k_cast<__bf16>, g, b, 0, s, rows, cols, src, lds, (__bf16*)dst);
      break;
  }
  LYAP_HIP(hipGetLastError());
  return LYAP_OK;
}

int sumsq(hipStream_t s, int rows, int cols, const double* A, long lda, double* out,
          double* partial) {
  // a large matrix takes four workgroups per CU so that enough loads are in flight
  const int nparts = rows >= 4 * RPARTS ? 4 * RPARTS : RPARTS;
  hipLaunchKernelGGL(k_sumsq_partial, dim3(nparts), dim3(RB), 0, s, rows, cols, A, lda, partial);
  hipLaunchKernelGGL(k_sum_parts, dim3(1), dim3(RB), 0, s, nparts, partial, out);
  LYAP_HIP(hipGetLastError());
  return LYAP_OK;
}

int newton_update(hipStream_t s, int n, const double* A, long lda, const double* Ainv, long ldi,
                  const double* mu_dev, double* Anew, long ldn, double* out4, double* colsum,
                  double* partial) {
  // partial layout: 2*nb block sums, then nparts*n column partial sums, then nchunks maxima
  // (at most 2*RPARTS + RPARTS*n doubles for n >= 1)
  const int nparts = std::min(64, n);
  const int rows_per = (n + nparts - 1) / nparts;
  const int nrows = (n + rows_per - 1) / rows_per;
  const int nchunks = (n + RB - 1) / RB;
  const int nb = nrows * nchunks;
  double* colpart = partial + 2 * nb;
  double* colmax = colpart + (long)nrows * n;
  hipLaunchKernelGGL(k_newton, dim3(nrows, nchunks), dim3(RB), 0, s, n, A, lda, Ainv, ldi, mu_dev,
                     Anew, ldn, rows_per, partial, colpart);
  hipLaunchKernelGGL(k_colsum, dim3(nchunks), dim3(RB), 0, s, n, nrows, colpart, colsum, colmax);
  hipLaunchKernelGGL(k_newton_finish, dim3(1), dim3(RB), 0, s, nb, partial, nchunks, colmax, out4);
  LYAP_HIP(hipGetLastError());
  return LYAP_OK;
}

int newton_mu(hipStream_t s, const double* inv_sumsq, const double* a_sumsq, int scaling,
              double* mu_dev) {
  hipLaunchKernelGGL(k_mu, dim3(1), dim3(1), 0, s, inv_sumsq, a_sumsq, scaling, mu_dev);
  LYAP_HIP(hipGetLastError());
  return LYAP_OK;
}

}  // namespace lyap

namespace lyap {
namespace {

// sum_ij d_i d_j G_ij^2 (G symmetric c x c): ||Z diag(d) Z^T||_F^2 with G = Z^T Z.
__global__ void k_wsumsq_partial(int c, const double* __restrict__ G, long ldg,
                                 const double* __restrict__ d, double* __restrict__ part) {
  __shared__ double red[RB];
  double acc = 0.0;
  long total = (long)c * c;
  for (long e = (long)blockIdx.x * RB + threadIdx.x; e < total; e += (long)gridDim.x * RB) {
    int i = (int)(e / c), j = (int)(e % c);
    double g = G[(long)i * ldg + j];
    acc += d[i] * d[j] * g * g;
  }
  double s = block_sum(acc, red);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// dst[:, k] = src[:, idx[k]] for k < count, rows rows.
__global__ void k_gather_cols(int rows, int count, const double* __restrict__ src, long lds,
                              const int* __restrict__ idx, double* __restrict__ dst, long ldd) {
  long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (long)rows * count) return;
  int i = (int)(e / count), k = (int)(e % count);
  dst[(long)i * ldd + k] = src[(long)i * lds + idx[k]];
}

__global__ void k_trace(int n, const double* __restrict__ A, long lda, double* __restrict__ out) {
  __shared__ double red[RB];
  double acc = 0.0;
  for (int i = threadIdx.x; i < n; i += RB) acc += A[(long)i * lda + i];
  double s = block_sum(acc, red);
  if (threadIdx.x == 0) *out = s;
}

}  // namespace

int wsumsq(hipStream_t s, int c, const double* G, long ldg, const double* d, double* out,
           double* partial) {
  hipLaunchKernelGGL(k_wsumsq_partial, dim3(RPARTS), dim3(RB), 0, s, c, G, ldg, d, partial);
  hipLaunchKernelGGL(k_sum_parts, dim3(1), dim3(RB), 0, s, RPARTS, partial, out);
  LYAP_HIP(hipGetLastError());
  return LYAP_OK;
}

int gather_cols(hipStream_t s, int rows, int count, const double* src, long lds, const int* idx,
                double* dst, long ldd) {
  long total = (long)rows * count;
  if (total <= 0) return LYAP_OK;
  hipLaunchKernelGGL(k_gather_cols, dim3(nblk(total)), dim3(256), 0, s, rows, count, src, lds, idx,
                     dst, ldd);
  LYAP_HIP(hipGetLastError());
  return LYAP_OK;
}

int colw_sumsq(hipStream_t s, int rows, int cols, const double* X, long ldx, const double* w,
               double* out) {
  hipLaunchKernelGGL(k_colw_sumsq, dim3(1), dim3(RB), 0, s, rows, cols, X, ldx, w, out);
  LYAP_HIP(hipGetLastError());
  return LYAP_OK;
}

int roww_colsumsq(hipStream_t s, int rows, int cols, const double* X, long ldx, const double* w,
                  double* out) {
  if (cols <= 0) return LYAP_OK;
  hipLaunchKernelGGL(k_roww_colsumsq, dim3(nblk(cols)), dim3(256), 0, s, rows, cols, X, ldx, w,
                     out);
  LYAP_HIP(hipGetLastError());
  return LYAP_OK;
}

int trace(hipStream_t s, int n, const double* A, long lda, double* out) {
  hipLaunchKernelGGL(k_trace, dim3(1), dim3(RB), 0, s, n, A, lda, out);
  LYAP_HIP(hipGetLastError());
  return LYAP_OK;
}

}  // namespace lyap
