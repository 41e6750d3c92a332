// Inversion through a random butterfly transformation (Parker 1995; Baboulin, Dongarra,
// Herrmann and Tomov 2013): with U, V random recursive butterflies of depth 2,
//     A_r = U^T A V,   A^{-1} = V A_r^{-1} U^T,
// and Gauss-Jordan elimination of A_r needs no pivoting with high probability.  The pivot
// search is what makes the pivoted inversion latency-bound (one column at a time over all n
// rows), so the transformed inversion is about twice as fast; a residual probe
// ||A (A^{-1} x) - x|| with a seeded random x tells the caller whether to redo the step
// with partial pivoting.
//
// A butterfly of size N is B = 2^{-1/2} [[R0, R1], [R0, -R1]] with R0, R1 diagonal of size
// N / 2 and entries exp(r / 10), r uniform in [-1/2, 1/2); the depth-2 recursive butterfly is
// U = diag(B1, B2) B0 (B0 of size n, B1 and B2 of size n / 2).  Applying U, U^T, V or V^T to
// every column (or row) of an n x n matrix touches each entry once: index q < n / 4 mixes
// the four entries q, q + n/4, q + n/2, q + 3n/4.  The random entries come from a
// counter-based generator (SplitMix64 finaliser on seed and index), so every run draws the
// same transformation.  |det U| is the product of its diagonal entries, which gives
// log|det A| from log|det A_r|.
#include <cmath>

#include "common.hpp"
#include "internal.hpp"

namespace lyap {
namespace {

constexpr double INV_SQRT2 = 0.70710678118654752440;

__device__ inline unsigned long long rbt_mix(unsigned long long x) {
  x += 0x9e3779b97f4a7c15ull;
  x = (x ^ (x >> 30)) * 0xbf58476d1ce4e5b9ull;
  x = (x ^ (x >> 27)) * 0x94d049bb133111ebull;
  return x ^ (x >> 31);
}

// r[i] = exp(rho_i / 10), rho_i = u_i - 1/2 with u_i = (top 53 bits of mix(seed, i)) / 2^53;
// one butterfly set (2 n entries: R0, R1 of B0, then R0, R1 of B1 and of B2) for U and one
// for V.  logr[0] receives sum(rho_i) / 10 over both sets (fixed order, one workgroup).
__global__ __launch_bounds__(256) void k_rbt_init(int n, unsigned long long seed,
                                                  double* __restrict__ r,
                                                  double* __restrict__ logr) {
  __shared__ double red[256];
  double acc = 0.0;
  for (int i = threadIdx.x; i < 4 * n; i += 256) {
    const unsigned long long h = rbt_mix(seed ^ rbt_mix((unsigned long long)i));
    const double rho = (double)(h >> 11) * (1.0 / 9007199254740992.0) - 0.5;
    r[i] = exp(rho / 10.0);
    acc += rho / 10.0;
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) *logr = red[0];
}

// In place on X (n x n, leading dimension ld): along_rows mixes the row indices of every
// column (X <- U X or U^T X), otherwise the column indices of every row (X <- X U^T or X U).
// fwd applies U, otherwise U^T; r is U's set of 2 n diagonal entries.
template <bool ALONG_ROWS, bool FWD>
__global__ void k_butterfly(int n, double* __restrict__ X, long ld, const double* __restrict__ r) {
  const int n4 = n / 4;
  const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (long)n4 * n) return;
  int q, j;
  if (ALONG_ROWS) { j = (int)(idx % n); q = (int)(idx / n); }
  else { q = (int)(idx % n4); j = (int)(idx / n4); }
  double* p[4];
#pragma unroll
  for (int k = 0; k < 4; ++k)
    p[k] = ALONG_ROWS ? X + (long)(q + k * n4) * ld + j : X + (long)j * ld + q + k * n4;
  const double xa = *p[0], xb = *p[1], xc = *p[2], xd = *p[3];
  const double* r0 = r;           // R0 of B0 (n / 2)
  const double* r1 = r + n / 2;   // R1 of B0
  const double* s0 = r + n;       // R0 of B1 (n / 4)
  const double* s1 = s0 + n4;     // R1 of B1
  const double* t0 = s1 + n4;     // R0 of B2
  const double* t1 = t0 + n4;     // R1 of B2
  const double c = INV_SQRT2;
  double za, zb, zc, zd;
  if (FWD) {
    // B0 first (pairs t, t + n/2), then diag(B1, B2)
    const double wa = c * (r0[q] * xa + r1[q] * xc), wc = c * (r0[q] * xa - r1[q] * xc);
    const double wb = c * (r0[q + n4] * xb + r1[q + n4] * xd);
    const double wd = c * (r0[q + n4] * xb - r1[q + n4] * xd);
    za = c * (s0[q] * wa + s1[q] * wb);
    zb = c * (s0[q] * wa - s1[q] * wb);
    zc = c * (t0[q] * wc + t1[q] * wd);
    zd = c * (t0[q] * wc - t1[q] * wd);
  } else {
    // U^T = B0^T diag(B1^T, B2^T), with B^T = 2^{-1/2} [[R0, R0], [R1, -R1]]
    const double ya = c * s0[q] * (xa + xb), yb = c * s1[q] * (xa - xb);
    const double yc = c * t0[q] * (xc + xd), yd = c * t1[q] * (xc - xd);
    za = c * r0[q] * (ya + yc);
    zc = c * r1[q] * (ya - yc);
    zb = c * r0[q + n4] * (yb + yd);
    zd = c * r1[q + n4] * (yb - yd);
  }
  *p[0] = za;
  *p[1] = zb;
  *p[2] = zc;
  *p[3] = zd;
}

// ---- the residual probe ||A (Ainv x) - x||_2 / ||x||_2
__global__ void k_probe_vec(int n, unsigned long long seed, double* __restrict__ x) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const unsigned long long h = rbt_mix(seed ^ rbt_mix(0x5eedull + (unsigned long long)i));
  x[i] = (double)(h >> 11) * (1.0 / 9007199254740992.0) - 0.5;
}
// y = M x - w (w may be NULL), one wave per row, fixed-order lane sums and butterfly.
__global__ void k_rowdot(int n, const double* __restrict__ M, long ld, const double* __restrict__ x,
                         double* __restrict__ y, const double* __restrict__ w) {
  const int lane = threadIdx.x & 63;
  const int row = blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6);
  if (row >= n) return;
  const double* m = M + (long)row * ld;
  double acc = 0.0;
  for (int j = lane; j < n; j += 64) acc += m[j] * x[j];
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
  if (lane == 0) y[row] = w ? acc - w[row] : acc;
}
__global__ __launch_bounds__(256) void k_probe_ratio(int n, const double* __restrict__ z,
                                                     const double* __restrict__ x,
                                                     double* __restrict__ out) {
  __shared__ double rz[256], rx[256];
  double az = 0.0, ax = 0.0;
  for (int i = threadIdx.x; i < n; i += 256) {
    az += z[i] * z[i];
    ax += x[i] * x[i];
  }
  rz[threadIdx.x] = az;
  rx[threadIdx.x] = ax;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (threadIdx.x < h) {
      rz[threadIdx.x] += rz[threadIdx.x + h];
      rx[threadIdx.x] += rx[threadIdx.x + h];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double v = sqrt(rz[0] / rx[0]);
    *out = (v == v) ? v : INFINITY;
  }
}
__global__ void k_sub_scalar(double* __restrict__ a, const double* __restrict__ b) { *a -= *b; }

inline unsigned nb(long total) { return (unsigned)((total + 255) / 256); }

template <bool ALONG_ROWS, bool FWD>
int butterfly(hipStream_t s, int n, double* X, long ld, const double* r) {
  const long total = (long)(n / 4) * n;
  hipLaunchKernelGGL((k_butterfly<ALONG_ROWS, FWD>), dim3(nb(total)), dim3(256), 0, s, n, X, ld,
                     r);
  LYAP_HIP(hipGetLastError());
  return LYAP_OK;
}

}  // namespace

size_t rbt_workspace_bytes(int n) { return ((size_t)4 * n + 3 * (size_t)n + 16) * 8 + 1024; }

int rbt_invert(hipStream_t s, Prec op, int n, const double* A, long lda, double* out, long ldo,
               Arena& ws, int* flags_dev, KernTimer* kt, double* logdet,
               unsigned long long seed, double* probe) {
  if (n <= 0) return LYAP_OK;
  if (n % 4 != 0 || n > 4096) return LYAP_BADARG;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (kt) LYAP_TRY(kt->mark(s, &e0));
  double* r = ws.take<double>((size_t)4 * n);
  double* x = ws.take<double>(n);
  double* y = ws.take<double>(n);
  double* z = ws.take<double>(n);
  double* logr = ws.take<double>(2);
  if (!r || !x || !y || !z || !logr) return LYAP_NO_MEMORY;
  const double* rU = r;
  const double* rV = r + 2 * n;
  hipLaunchKernelGGL(k_rbt_init, dim3(1), dim3(256), 0, s, n, seed, r, logr);
  LYAP_HIP(hipGetLastError());
  // A_r = U^T A V in out
  LYAP_TRY(copy_block(s, n, n, A, lda, out, ldo));
  LYAP_TRY((butterfly<true, false>(s, n, out, ldo, rU)));   // U^T A
  LYAP_TRY((butterfly<false, false>(s, n, out, ldo, rV)));  // (U^T A) V: rows r -> (V^T r^T)^T
  // A_r^{-1} by Gauss-Jordan without pivoting (in place: the working copy is read first)
  LYAP_TRY(invert(s, op, n, out, ldo, out, ldo, ws, flags_dev, false, nullptr, logdet));
  // A^{-1} = V A_r^{-1} U^T
  LYAP_TRY((butterfly<true, true>(s, n, out, ldo, rV)));    // V M
  LYAP_TRY((butterfly<false, true>(s, n, out, ldo, rU)));   // M U^T: rows r -> (U r^T)^T
  if (logdet) {
    // log|det A| = log|det A_r| - log|det U| - log|det V|
    hipLaunchKernelGGL(k_sub_scalar, dim3(1), dim3(1), 0, s, logdet, logr);
  }
  if (probe) {
    hipLaunchKernelGGL(k_probe_vec, dim3(nb(n)), dim3(256), 0, s, n, seed, x);
    hipLaunchKernelGGL(k_rowdot, dim3((unsigned)ceil_div(n, 4)), dim3(256), 0, s, n, out, ldo, x,
                       y, (const double*)nullptr);
    // z = A y - x
    hipLaunchKernelGGL(k_rowdot, dim3((unsigned)ceil_div(n, 4)), dim3(256), 0, s, n, A, lda, y, z,
                       x);
    hipLaunchKernelGGL(k_probe_ratio, dim3(1), dim3(256), 0, s, n, z, x, probe);
  }
  LYAP_HIP(hipGetLastError());
  if (kt) {
    LYAP_TRY(kt->mark(s, &e1));
    kt->add(e0, e1, 0, 2.0 * (double)n * n * n, 1);
  }
  return LYAP_OK;
}

int probe_inverse(hipStream_t s, int n, const double* A, long lda, const double* Ainv, long ldi,
                  Arena& ws, unsigned long long seed, double* probe) {
  double* x = ws.take<double>(n);
  double* y = ws.take<double>(n);
  double* z = ws.take<double>(n);
  if (!x || !y || !z) return LYAP_NO_MEMORY;
  hipLaunchKernelGGL(k_probe_vec, dim3(nb(n)), dim3(256), 0, s, n, seed, x);
  hipLaunchKernelGGL(k_rowdot, dim3((unsigned)ceil_div(n, 4)), dim3(256), 0, s, n, Ainv, ldi, x, y,
                     (const double*)nullptr);
  hipLaunchKernelGGL(k_rowdot, dim3((unsigned)ceil_div(n, 4)), dim3(256), 0, s, n, A, lda, y, z, x);
  hipLaunchKernelGGL(k_probe_ratio, dim3(1), dim3(256), 0, s, n, z, x, probe);
  LYAP_HIP(hipGetLastError());
  return LYAP_OK;
}

}  // namespace lyap
