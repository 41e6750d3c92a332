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

__global__ void k_fill_u64(unsigned long long* p, long count) {
  long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) p[i] = 0ull;
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

// dst += alpha src (rows x cols blocks).
__global__ void k_add_block(int rows, int cols, double alpha, const double* __restrict__ src,
                            long lds, double* __restrict__ dst, long ldd) {
  long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
  long total = (long)rows * cols;
  if (idx >= total) return;
  int i = (int)(idx / cols), j = (int)(idx % cols);
  dst[(long)i * ldd + j] += alpha * src[(long)i * lds + j];
}

// M_ii += p.
__global__ void k_add_diag(int n, double* __restrict__ M, long ld, double p) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) M[(long)i * ld + i] += p;
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

// Scaling parameter of the Newton step (Section 3): mode 0 Frobenius sqrt(sqrt(x) / sqrt(y))
// with x, y the squared Frobenius norms of A^-1 and A; mode 1 determinantal exp(-x / n) with
// x = log|det A|; mode 2 sqrt(x / y) with x, y norm (or spectral radius) estimates of A^-1
// and A.  mu = 1 when scaling is off.
__global__ void k_mu(int mode, const double* x, const double* y, int n, int scaling, double* mu) {
  if (!scaling) { *mu = 1.0; return; }
  if (mode == 1) *mu = exp(-(*x) / (double)n);
  else if (mode == 2) *mu = sqrt(*x / *y);
  else *mu = sqrt(sqrt(*x) / sqrt(*y));
}

// ---- power iterations for the optional 2-norm and spectral scalings
__global__ void k_vec_init(int n, double* __restrict__ x) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) x[i] = 1.0 / sqrt((double)n);
}
// y = M x, one wave per row (fixed-order lane sums, then a fixed butterfly).
__global__ void k_gemv_n(int n, const double* __restrict__ M, long ld, const double* __restrict__ x,
                         double* __restrict__ y) {
  const int lane = threadIdx.x & 63;
  const int row = blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6);
  if (row >= n) return;
  const double* m = M + (long)row * ld;
  double acc = 0.0;
  for (int j = lane; j < n; j += 64) acc += m[j] * x[j];
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
  if (lane == 0) y[row] = acc;
}
// part[r][j] = sum over rows of chunk r of M_ij x_i (columns over threads, coalesced).
__global__ void k_gemv_t_part(int n, const double* __restrict__ M, long ld,
                              const double* __restrict__ x, int rows_per,
                              double* __restrict__ part) {
  const int j = blockIdx.x * RB + threadIdx.x;
  if (j >= n) return;
  const int r0 = blockIdx.y * rows_per, r1 = min(n, r0 + rows_per);
  double acc = 0.0;
  for (int i = r0; i < r1; ++i) acc += M[(long)i * ld + j] * x[i];
  part[(long)blockIdx.y * n + j] = acc;
}
__global__ void k_gemv_t_fin(int n, int nparts, const double* __restrict__ part,
                             double* __restrict__ y) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  double acc = 0.0;
  for (int r = 0; r < nparts; ++r) acc += part[(long)r * n + j];
  y[j] = acc;
}
// x = y / ||y||_2 (one block); *nrm = ||y||_2; with logacc, *logacc += log ||y||_2.
__global__ void k_normalize(int n, const double* __restrict__ y, double* __restrict__ x,
                            double* __restrict__ nrm, double* __restrict__ logacc) {
  __shared__ double red[RB];
  double acc = 0.0;
  for (int i = threadIdx.x; i < n; i += RB) acc += y[i] * y[i];
  const double ss = block_sum(acc, red);
  const double nr = sqrt(ss);
  const double inv = nr > 0.0 ? 1.0 / nr : 0.0;
  for (int i = threadIdx.x; i < n; i += RB) x[i] = y[i] * inv;
  if (threadIdx.x == 0) {
    *nrm = nr;
    if (logacc) *logacc += log(nr);
  }
}
__global__ void k_set_scalar(double* p, double v) { *p = v; }
__global__ void k_norm_finish(const double* __restrict__ v, int mode, int count,
                              double* __restrict__ out) {
  if (mode == 0) *out = sqrt(*v);
  else *out = exp(*v / (double)count);
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

// Largest |A_ij| of a rows x cols block: per-block partial maxima (NaN poisons the partial).
__global__ void k_absmax_partial(int rows, int cols, const double* __restrict__ A, long lda,
                                 double* __restrict__ part) {
  __shared__ double red[RB];
  __shared__ int rnan[RB];
  double m = 0.0;
  int nan = 0;
  for (int i = blockIdx.x; i < rows; i += gridDim.x) {
    const double* a = A + (long)i * lda;
    for (int j = threadIdx.x; j < cols; j += RB) {
      const double v = fabs(a[j]);
      if (v != v) nan = 1;
      else m = fmax(m, v);
    }
  }
  red[threadIdx.x] = m;
  rnan[threadIdx.x] = nan;
  __syncthreads();
  for (int h = RB / 2; h > 0; h >>= 1) {
    if (threadIdx.x < h) {
      red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + h]);
      rnan[threadIdx.x] |= rnan[threadIdx.x + h];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = rnan[0] ? NAN : red[0];
}

// e with 2^(e-1) <= max < 2^e (0 for max == 0); *bad <- 1 for a NaN or infinite maximum.
__global__ void k_absmax_exp(int nparts, const double* __restrict__ part, int* __restrict__ e,
                             int* __restrict__ bad) {
  __shared__ double red[RB];
  __shared__ int rnan[RB];
  double m = 0.0;
  int nan = 0;
  for (int i = threadIdx.x; i < nparts; i += RB) {
    const double v = part[i];
    if (v != v) nan = 1;
    else m = fmax(m, v);
  }
  red[threadIdx.x] = m;
  rnan[threadIdx.x] = nan;
  __syncthreads();
  for (int h = RB / 2; h > 0; h >>= 1) {
    if (threadIdx.x < h) {
      red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + h]);
      rnan[threadIdx.x] |= rnan[threadIdx.x + h];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double mx = red[0];
    int ex = 0;
    if (mx > 0.0 && !isinf(mx)) frexp(mx, &ex);
    *e = ex;
    if (bad && (rnan[0] || isinf(mx))) *bad = 1;
  }
}

// dst = RNE(2^-e src) in storage T (row-major, ld = cols): the power-of-two scaled cast.
template <class T>
__global__ void k_cast_scaled(int rows, int cols, const double* __restrict__ src, long lds,
                              T* __restrict__ dst, const int* __restrict__ e) {
  long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
  long total = (long)rows * cols;
  if (idx >= total) return;
  const int ex = e ? *e : 0;
  int i = (int)(idx / cols), j = (int)(idx % cols);
  dst[idx] = rne_from_f64<T>(ldexp(src[(long)i * lds + j], -ex));
}

// X <- RNE_T(X) in place (values of the FP64 block rounded to the storage format T).
template <class T>
__global__ void k_round_block(int rows, int cols, double* __restrict__ X, long ldx) {
  long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
  long total = (long)rows * cols;
  if (idx >= total) return;
  int i = (int)(idx / cols), j = (int)(idx % cols);
  double* p = X + (long)i * ldx + j;
  *p = (double)rne_from_f64<T>(*p);
}

// Column maxima of |X| (rows x cols) as bit patterns: for non-negative binary64 values the
// bit patterns order as the values do (NaN above +inf), so an integer maximum is exact and
// independent of the order of the updates.  Block (x, y): rows strided by gridDim.x, columns
// y*RB + thread.
__global__ void k_colmax_bits(int rows, int cols, const double* __restrict__ X, long ldx,
                              unsigned long long* __restrict__ bits) {
  const int j = blockIdx.y * RB + threadIdx.x;
  if (j >= cols) return;
  unsigned long long m = 0ull;
  for (int i = blockIdx.x; i < rows; i += gridDim.x) {
    const unsigned long long b =
        (unsigned long long)__double_as_longlong(X[(long)i * ldx + j]) & 0x7fffffffffffffffull;
    m = b > m ? b : m;
  }
  atomicMax(bits + j, m);
}

// e_j with 2^(e_j - 1) <= max_i |X_ij| < 2^e_j (0 for a zero column); *bad <- 1 when a column
// holds a NaN or an infinity.
__global__ void k_colexp_finish(int cols, const unsigned long long* __restrict__ bits,
                                int* __restrict__ e, int* __restrict__ bad) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= cols) return;
  const double mx = __longlong_as_double((long long)bits[j]);
  int ex = 0;
  if (mx > 0.0 && isfinite(mx)) frexp(mx, &ex);
  else if (!(mx == 0.0) && bad) *bad = 1;
  e[j] = ex;
}

// 64-bit fingerprint of the contents of an n x n matrix: the wrapping sum over entries of a
// mixed (bit pattern, position) word.  Integer addition modulo 2^64 is associative, so the
// result does not depend on the order of the atomic updates.
__device__ inline unsigned long long fp_mix(unsigned long long x) {
  x ^= x >> 30;
  x *= 0xbf58476d1ce4e5b9ull;
  x ^= x >> 27;
  x *= 0x94d049bb133111ebull;
  x ^= x >> 31;
  return x;
}
__global__ void k_fingerprint(int rows, int cols, const double* __restrict__ A, long lda,
                              unsigned long long* __restrict__ out) {
  __shared__ unsigned long long red[RB];
  unsigned long long acc = 0ull;
  for (int i = blockIdx.x; i < rows; i += gridDim.x) {
    for (int j = threadIdx.x; j < cols; j += RB) {
      const unsigned long long b = (unsigned long long)__double_as_longlong(A[(long)i * lda + j]);
      const unsigned long long pos = (unsigned long long)i * (unsigned long long)cols + j;
      acc += fp_mix(b ^ fp_mix(pos + 0x9e3779b97f4a7c15ull));
    }
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int h = RB / 2; h > 0; h >>= 1) {
    if (threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) atomicAdd(out, red[0]);
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

int add_block(hipStream_t s, int rows, int cols, double alpha, const double* src, long lds,
              double* dst, long ldd) {
  long total = (long)rows * cols;
  if (total <= 0) return LYAP_OK;
  hipLaunchKernelGGL(k_add_block, dim3(nblk(total)), dim3(256), 0, s, rows, cols, alpha, src, lds,
                     dst, ldd);
  LYAP_HIP(hipGetLastError());
  return LYAP_OK;
}

int add_diag(hipStream_t s, int n, double* M, long ld, double p) {
  if (n <= 0) return LYAP_OK;
  hipLaunchKernelGGL(k_add_diag, dim3(nblk(n)), dim3(256), 0, s, n, M, ld, p);
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

int absmax_exp(hipStream_t s, int rows, int cols, const double* A, long lda, int* e_dev,
               int* bad_dev, double* partial) {
  if (rows <= 0 || cols <= 0) return fill_int(s, e_dev, 1, 0);
  const int nparts = rows >= 4 * RPARTS ? 4 * RPARTS : std::max(1, std::min(RPARTS, rows));
  hipLaunchKernelGGL(k_absmax_partial, dim3(nparts), dim3(RB), 0, s, rows, cols, A, lda, partial);
  hipLaunchKernelGGL(k_absmax_exp, dim3(1), dim3(RB), 0, s, nparts, partial, e_dev, bad_dev);
  LYAP_HIP(hipGetLastError());
  return LYAP_OK;
}

int cast_scaled(hipStream_t s, Store st, int rows, int cols, const double* src, long lds,
                void* dst, const int* e_dev) {
  long total = (long)rows * cols;
  if (total <= 0) return LYAP_OK;
  dim3 g(nblk(total)), b(256);
  switch (st) {
    case Store::F64:
      hipLaunchKernelGGL(k_cast_scaled<double>, g, b, 0, s, rows, cols, src, lds, (double*)dst,
                         e_dev);
      break;
    case Store::F32:
      hipLaunchKernelGGL(k_cast_scaled<float>, g, b, 0, s, rows, cols, src, lds, (float*)dst,
                         e_dev);
      break;
    case Store::F16:
      hipLaunchKernelGGL(k_cast_scaled<_Float16>, g, b, 0, s, rows, cols, src, lds,
                         (_Float16*)dst, e_dev);
      break;
    case Store::BF16:
      hipLaunchKernelGGL(k_cast_scaled<__bf16>, g, b, 0, s, rows, cols, src, lds, (__bf16*)dst,
                         e_dev);
      break;
  }
  LYAP_HIP(hipGetLastError());
  return LYAP_OK;
}

int round_block(hipStream_t s, Store st, int rows, int cols, double* X, long ldx) {
  long total = (long)rows * cols;
  if (total <= 0 || st == Store::F64) return LYAP_OK;
  dim3 g(nblk(total)), b(256);
  switch (st) {
    case Store::F32:
      hipLaunchKernelGGL(k_round_block<float>, g, b, 0, s, rows, cols, X, ldx);
      break;
    case Store::F16:
      hipLaunchKernelGGL(k_round_block<_Float16>, g, b, 0, s, rows, cols, X, ldx);
      break;
    case Store::BF16:
      hipLaunchKernelGGL(k_round_block<__bf16>, g, b, 0, s, rows, cols, X, ldx);
      break;
    default: break;
  }
  LYAP_HIP(hipGetLastError());
  return LYAP_OK;
}

int col_exponents(hipStream_t s, int rows, int cols, const double* X, long ldx, int* e_dev,
                  int* bad_dev, unsigned long long* bits) {
  if (cols <= 0) return LYAP_OK;
  hipLaunchKernelGGL(k_fill_u64, dim3(nblk(cols)), dim3(256), 0, s, bits, (long)cols);
  const int ry = ceil_div(cols, RB);
  const int rx = std::max(1, std::min(rows, std::max(1, 1024 / ry)));
  if (rows > 0)
    hipLaunchKernelGGL(k_colmax_bits, dim3(rx, ry), dim3(RB), 0, s, rows, cols, X, ldx, bits);
  hipLaunchKernelGGL(k_colexp_finish, dim3(nblk(cols)), dim3(256), 0, s, cols, bits, e_dev,
                     bad_dev);
  LYAP_HIP(hipGetLastError());
  return LYAP_OK;
}

int fingerprint(hipStream_t s, int rows, int cols, const double* A, long lda,
                unsigned long long* out) {
  hipLaunchKernelGGL(k_fill_u64, dim3(1), dim3(256), 0, s, out, 1l);
  LYAP_HIP(hipGetLastError());
  if (rows <= 0 || cols <= 0) return LYAP_OK;
  const int nb = std::min(rows, 1024);
  hipLaunchKernelGGL(k_fingerprint, dim3(nb), dim3(RB), 0, s, rows, cols, A, lda, out);
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

int newton_mu(hipStream_t s, int mode, const double* x, const double* y, int n, int scaling,
              double* mu_dev) {
  hipLaunchKernelGGL(k_mu, dim3(1), dim3(1), 0, s, mode, x, y, n, scaling, mu_dev);
  LYAP_HIP(hipGetLastError());
  return LYAP_OK;
}

namespace {
// y = M x (op 0) or y = M^T x (op 1) for an n x n row-major M; part: 16 n doubles.
int gemv_sq(hipStream_t s, int op, int n, const double* M, long ld, const double* x, double* y,
            double* part) {
  if (op == 0) {
    hipLaunchKernelGGL(k_gemv_n, dim3((unsigned)ceil_div(n, 4)), dim3(256), 0, s, n, M, ld, x, y);
  } else {
    const int R = std::min(16, n);
    const int rows_per = ceil_div(n, R);
    const int nparts = ceil_div(n, rows_per);
    hipLaunchKernelGGL(k_gemv_t_part, dim3((unsigned)ceil_div(n, RB), (unsigned)nparts),
                       dim3(RB), 0, s, n, M, ld, x, rows_per, part);
    hipLaunchKernelGGL(k_gemv_t_fin, dim3(nblk(n)), dim3(256), 0, s, n, nparts, part, y);
  }
  LYAP_HIP(hipGetLastError());
  return LYAP_OK;
}
}  // namespace

int norm2_est(hipStream_t s, int n, const double* M, long ld, int iters, double* out,
              double* work) {
  double* x = work;
  double* y = work + n;
  double* z = work + 2 * n;
  double* part = work + 3 * n;
  hipLaunchKernelGGL(k_vec_init, dim3(nblk(n)), dim3(256), 0, s, n, x);
  for (int it = 0; it < iters; ++it) {
    LYAP_TRY(gemv_sq(s, 0, n, M, ld, x, y, part));
    LYAP_TRY(gemv_sq(s, 1, n, M, ld, y, z, part));
    // ||M^T M x||_2 -> sigma_max^2 as x converges to the top right singular vector
    hipLaunchKernelGGL(k_normalize, dim3(1), dim3(RB), 0, s, n, z, x, out, (double*)nullptr);
  }
  hipLaunchKernelGGL(k_norm_finish, dim3(1), dim3(1), 0, s, out, 0, 0, out);
  LYAP_HIP(hipGetLastError());
  return LYAP_OK;
}

int specrad_est(hipStream_t s, int n, const double* M, long ld, int iters, double* out,
                double* work) {
  double* x = work;
  double* y = work + n;
  double* nrm = work + 2 * n;
  double* part = work + 3 * n;
  hipLaunchKernelGGL(k_vec_init, dim3(nblk(n)), dim3(256), 0, s, n, x);
  hipLaunchKernelGGL(k_set_scalar, dim3(1), dim3(1), 0, s, out, 0.0);
  // rho(M) = lim ||M^k x||^(1/k): the mean growth rate of the last half of the steps
  const int half = iters / 2;
  for (int it = 0; it < iters; ++it) {
    LYAP_TRY(gemv_sq(s, 0, n, M, ld, x, y, part));
    hipLaunchKernelGGL(k_normalize, dim3(1), dim3(RB), 0, s, n, y, x, nrm,
                       it >= half ? out : (double*)nullptr);
  }
  hipLaunchKernelGGL(k_norm_finish, dim3(1), dim3(1), 0, s, out, 1, iters - half, out);
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
