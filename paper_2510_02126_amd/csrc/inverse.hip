// Matrix inversion by Gauss-Jordan elimination with partial pivoting (the inversion in the
// first line of the Newton loop of Alg 3.1/3.2), recursive-blocked for gfx950.
//
// Data: a working copy Wk (n x n, row-major) in binary64 (FP64 solver) or binary32 (reduced
// solver precisions, prescaled by a power of two so the largest entry lies in [1/2, 1)).
// Rows are never swapped physically: the pivot for column j is the unused row r_j with the
// largest |Wk[r][j]| (ties to the lowest row index).  Gauss-Jordan eliminates column j from
// every other row, so after all n steps Wk[r_i][j] = (PA)^{-1}[i][j] and the inverse is
// A^{-1}[i][r_j] = Wk[r_i][j].
//
// Blocking: columns [c0, c1) are processed recursively.  A leaf of at most WC columns is
// handled by one workgroup that keeps the n x WC panel in registers and takes the pivot
// decisions one column at a time.  An internal node processes its left half, then applies
// the left half's transformation to its right-half columns, processes the right half, and
// finally applies the right half's transformation to the left-half columns.  Applying the
// transformation of pivots [a, b) to columns [c, d) is
//     R = Wk[r_a..r_{b-1}, c:d];  Wk[r_a..r_{b-1}, c:d] = 0;  Wk[:, c:d] += Wk[:, a:b] R,
// a matrix-core product whose operands are rounded to the solver precision (binary32
// accumulation for the reduced precisions).
#include <cmath>
#include <type_traits>

#include "common.hpp"
#include "internal.hpp"

namespace lyap {
namespace {

constexpr int LEAF_THREADS = 1024;

template <class T> struct LeafWidth;
template <> struct LeafWidth<double> { static constexpr int v = 8; };
template <> struct LeafWidth<float> { static constexpr int v = 16; };

// ---------------------------------------------------------------- prescale and copy
__global__ void absmax_partial(int n, const double* __restrict__ A, long lda,
                               double* __restrict__ part) {
  __shared__ double red[256];
  __shared__ int rnan[256];
  double m = 0.0;
  int nan = 0;
  long total = (long)n * n;
  for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (long)gridDim.x * blockDim.x) {
    long i = e / n, j = e % n;
    double v = fabs(A[i * lda + j]);
    if (v != v) nan = 1;
    else m = fmax(m, v);
  }
  red[threadIdx.x] = m;
  rnan[threadIdx.x] = nan;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) {
      red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + s]);
      rnan[threadIdx.x] |= rnan[threadIdx.x + s];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = rnan[0] ? NAN : red[0];
}

// Reduce the partial maxima and derive e with 2^(e-1) <= max < 2^e (0 when max == 0).
__global__ void absmax_exponent(int nparts, const double* __restrict__ part, int* __restrict__ e,
                                int* __restrict__ bad) {
  double m = 0.0;
  bool nan = false;
  for (int i = 0; i < nparts; ++i) {
    double v = part[i];
    if (v != v) nan = true;
    else m = fmax(m, v);
  }
  int ex = 0;
  if (m > 0.0 && !isinf(m)) frexp(m, &ex);
  *e = ex;
  if (nan || isinf(m)) *bad = 1;
}

template <class T>
__global__ void load_scaled(int n, const double* __restrict__ A, long lda, const int* __restrict__ e,
                            bool scale, T* __restrict__ Wk, int* __restrict__ used) {
  long total = (long)n * n;
  long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx < n) used[idx] = 0;
  if (idx >= total) return;
  long i = idx / n, j = idx % n;
  double v = A[i * lda + j];
  if (scale) v = ldexp(v, -*e);
  Wk[idx] = (T)v;
}

// ------------------------------------------------------------------------- leaf kernel
// One workgroup of 1024 threads; thread t owns rows t, t + 1024, ..., t + 1024 (RPT - 1).
template <class T, int RPT, int WC>
__global__ __launch_bounds__(LEAF_THREADS) void gj_leaf(int n, T* __restrict__ Wk, int c0, int wc,
                                                         int* __restrict__ used,
                                                         int* __restrict__ piv,
                                                         int* __restrict__ sing) {
  __shared__ T prow[2][WC];
  __shared__ T redv[LEAF_THREADS / 64];
  __shared__ int redr[LEAF_THREADS / 64];
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  T v[RPT][WC];
  bool u[RPT];
#pragma unroll
  for (int r = 0; r < RPT; ++r) {
    int row = t + LEAF_THREADS * r;
    u[r] = true;
#pragma unroll
    for (int c = 0; c < WC; ++c) v[r][c] = (T)0;
    if (row < n) {
      u[r] = used[row] != 0;
      const T* src = Wk + (long)row * n + c0;
#pragma unroll
      for (int c = 0; c < WC; ++c)
        if (c < wc) v[r][c] = src[c];
    }
  }
#pragma unroll
  for (int j = 0; j < WC; ++j) {
    if (j >= wc) continue;  // wc is uniform across the block
    // local arg-max over unused rows
    T best = (T)-1;
    int brow = 0x7fffffff;
#pragma unroll
    for (int r = 0; r < RPT; ++r) {
      int row = t + LEAF_THREADS * r;
      T a = fabs(v[r][j]);
      if (!u[r] && (a > best || (a == best && row < brow))) { best = a; brow = row; }
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      T ob = __shfl_xor(best, off);
      int orow = __shfl_xor(brow, off);
      if (ob > best || (ob == best && orow < brow)) { best = ob; brow = orow; }
    }
    if (lane == 0) { redv[wave] = best; redr[wave] = brow; }
    __syncthreads();
    best = redv[0];
    brow = redr[0];
#pragma unroll
    for (int w = 1; w < LEAF_THREADS / 64; ++w) {
      T ob = redv[w];
      int orow = redr[w];
      if (ob > best || (ob == best && orow < brow)) { best = ob; brow = orow; }
    }
    const int rp = brow;  // every thread holds the same winner
    const int buf = j & 1;
    if (rp != 0x7fffffff && (rp % LEAF_THREADS) == t) {
      const int rr = rp / LEAF_THREADS;
#pragma unroll
      for (int r = 0; r < RPT; ++r)
        if (r == rr) {
#pragma unroll
          for (int c = 0; c < WC; ++c) prow[buf][c] = v[r][c];
          u[r] = true;
        }
      used[rp] = 1;
      piv[c0 + j] = rp;
    }
    if (t == 0 && (rp == 0x7fffffff || !(best > (T)0))) *sing = 1;
    __syncthreads();
    T p = prow[buf][j];
    if (rp == 0x7fffffff || !(fabs(p) > (T)0)) p = (T)1;  // singular: keep going, flagged
    const T inv = (T)1 / p;
#pragma unroll
    for (int r = 0; r < RPT; ++r) {
      int row = t + LEAF_THREADS * r;
      if (row == rp) {
#pragma unroll
        for (int c = 0; c < WC; ++c) v[r][c] = (c == j) ? inv : v[r][c] * inv;
      } else {
        const T f = v[r][j] * inv;
#pragma unroll
        for (int c = 0; c < WC; ++c) v[r][c] = (c == j) ? -f : v[r][c] - f * prow[buf][c];
      }
    }
  }
#pragma unroll
  for (int r = 0; r < RPT; ++r) {
    int row = t + LEAF_THREADS * r;
    if (row < n) {
      T* dst = Wk + (long)row * n + c0;
#pragma unroll
      for (int c = 0; c < WC; ++c)
        if (c < wc) dst[c] = v[r][c];
    }
  }
}

// R[k][j] = Wk[piv[a+k]][c+j]; Wk[piv[a+k]][c+j] = 0.
template <class T>
__global__ void gather_zero(int n, T* __restrict__ Wk, const int* __restrict__ piv, int a, int w,
                            int c, int v, T* __restrict__ R) {
  long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
  long total = (long)w * v;
  if (idx >= total) return;
  int k = (int)(idx / v), j = (int)(idx % v);
  long src = (long)piv[a + k] * n + c + j;
  R[idx] = Wk[src];
  Wk[src] = (T)0;
}

// A^{-1}[i][r_j] = 2^-e * Wk[r_i][j]
template <class T>
__global__ void unpermute(int n, const T* __restrict__ Wk, const int* __restrict__ piv,
                          const int* __restrict__ e, bool scale, double* __restrict__ out,
                          long ldo, int* __restrict__ bad) {
  long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
  long total = (long)n * n;
  if (idx >= total) return;
  int i = (int)(idx / n), j = (int)(idx % n);
  double x = (double)Wk[(long)piv[i] * n + j];
  if (scale) x = ldexp(x, -*e);
  if (!isfinite(x)) *bad = 1;
  out[(long)i * ldo + piv[j]] = x;
}

template <class T> struct Inv {
  hipStream_t s;
  int n;
  T* Wk;
  T* R;
  int* used;
  int* piv;
  int* sing;
  Prec op;

  int leaf(int c0, int wc) {
    constexpr int WC = LeafWidth<T>::v;
    int rpt = ceil_div(n, LEAF_THREADS);
#define LEAF(RPT)                                                                           \
  hipLaunchKernelGGL((gj_leaf<T, RPT, WC>), dim3(1), dim3(LEAF_THREADS), 0, s, n, Wk, c0, wc, \
                     used, piv, sing)
    if (rpt <= 1) LEAF(1);
    else if (rpt <= 2) LEAF(2);
    else if (rpt <= 4) LEAF(4);
    else return LYAP_BADARG;
#undef LEAF
    LYAP_HIP(hipGetLastError());
    return LYAP_OK;
  }

  int update(int a, int b, int c, int d) {
    int w = b - a, v = d - c;
    long total = (long)w * v;
    hipLaunchKernelGGL((gather_zero<T>), dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s,
                       n, Wk, piv, a, w, c, v, R);
    LYAP_HIP(hipGetLastError());
    GemmDesc g;
    g.M = n; g.N = v; g.K = w;
    g.alpha = 1.0; g.beta = 1.0;
    g.A = Wk + a; g.sar = n; g.sac = 1;
    g.B = R; g.sbr = v; g.sbc = 1;
    g.C = Wk + c; g.ldc = n;
    if (std::is_same<T, double>::value) return gemm_f64(s, g);
    return gemm_lp(s, op, Store::F32, Store::F32, Store::F32, g);
  }

  int rec(int c0, int c1) {
    constexpr int WC = LeafWidth<T>::v;
    int w = c1 - c0;
    if (w <= WC) return leaf(c0, w);
    int half = ceil_div(ceil_div(w, 2), WC) * WC;
    int mid = c0 + half;
    if (mid >= c1) mid = c1 - WC;
    LYAP_TRY(rec(c0, mid));
    LYAP_TRY(update(c0, mid, mid, c1));
    LYAP_TRY(rec(mid, c1));
    LYAP_TRY(update(mid, c1, c0, mid));
    return LYAP_OK;
  }
};

template <class T>
int invert_t(hipStream_t s, Prec op, int n, const double* A, long lda, double* out, long ldo,
             Arena& ws, int* flags_dev) {
  size_t nn = (size_t)n * n;
  T* Wk = ws.take<T>(nn);
  T* R = ws.take<T>((size_t)((n + 1) / 2 + LeafWidth<T>::v) * ((n + 1) / 2 + LeafWidth<T>::v));
  int* used = ws.take<int>(n);
  int* piv = ws.take<int>(n);
  int* ex = ws.take<int>(1);
  int nparts = 256;
  double* part = ws.take<double>(nparts);
  if (!Wk || !R || !used || !piv || !ex || !part) return LYAP_NO_MEMORY;
  const bool scale = !std::is_same<T, double>::value;
  hipLaunchKernelGGL(absmax_partial, dim3(nparts), dim3(256), 0, s, n, A, lda, part);
  hipLaunchKernelGGL(absmax_exponent, dim3(1), dim3(1), 0, s, nparts, part, ex, flags_dev + 1);
  hipLaunchKernelGGL((load_scaled<T>), dim3((unsigned)((nn + 255) / 256)), dim3(256), 0, s, n, A,
                     lda, ex, scale, Wk, used);
  LYAP_HIP(hipGetLastError());
  Inv<T> inv{s, n, Wk, R, used, piv, flags_dev + 0, op};
  LYAP_TRY(inv.rec(0, n));
  hipLaunchKernelGGL((unpermute<T>), dim3((unsigned)((nn + 255) / 256)), dim3(256), 0, s, n, Wk,
                     piv, ex, scale, out, ldo, flags_dev + 1);
  LYAP_HIP(hipGetLastError());
  return LYAP_OK;
}

}  // namespace

size_t inverse_workspace_bytes(Prec op, int n) {
  size_t el = op == Prec::F64 ? 8 : 4;
  size_t half = (size_t)((n + 1) / 2 + 16);
  return (size_t)n * n * el + half * half * el + 4 * (size_t)n * 4 + 256 * 8 + 8 * 256;
}

// flags_dev[0] = singular pivot seen, flags_dev[1] = non-finite input/output (device ints,
// zeroed by the caller).
int invert(hipStream_t s, Prec op, int n, const double* A, long lda, double* out, long ldo,
           Arena& ws, int* flags_dev) {
  if (n <= 0) return LYAP_OK;
  if (n > 4 * LEAF_THREADS) return LYAP_BADARG;
  if (op == Prec::F64) return invert_t<double>(s, op, n, A, lda, out, ldo, ws, flags_dev);
  return invert_t<float>(s, op, n, A, lda, out, ldo, ws, flags_dev);
}

}  // namespace lyap
