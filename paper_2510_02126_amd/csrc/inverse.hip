// Matrix inversion by Gauss-Jordan elimination (the inversion in the first line of the Newton
// loop of Alg 3.1/3.2), recursive-blocked for gfx950.
//
// Data: a working copy W (n x n) in binary64 (FP64 solver) or binary32 (reduced solver
// precisions, prescaled by a power of two so the largest entry lies in [1/2, 1)).  W is held
// TRANSPOSED in memory, WT[j][i] = W[i][j]: a column of W is contiguous, so the n x w column
// panels that the leaves work on are w contiguous vectors of length n.
//
// Rows are never swapped physically: the pivot for column j is the unused row r_j with the
// largest |W[r][j]| (ties to the lowest row index).  Gauss-Jordan eliminates column j from
// every other row, so after all n steps W[r_i][j] = (PA)^{-1}[i][j] and the inverse is
// A^{-1}[i][r_j] = W[r_i][j].
//
// Blocking: columns [c0, c1) are processed recursively.  An internal node processes its left
// half, applies the left half's transformation to its right-half columns, processes the right
// half, and finally applies the right half's transformation to the left-half columns.
// Applying the transformation of pivots [a, b) to columns [c, d) is
//     R = W[r_a..r_{b-1}, c:d];  W[r_a..r_{b-1}, c:d] = 0;  W[:, c:d] += W[:, a:b] R,
// i.e. WT[c:d, :] += R^T WT[a:b, :], a matrix-core product whose operands are rounded to the
// solver precision (binary32 accumulation for the reduced precisions).
//
// Leaves:
//  * with pivoting, one workgroup keeps the n x WC panel in registers and takes the pivot
//    decisions one column at a time (DPP wave reductions + one LDS exchange per column);
//  * without pivoting (used only when the matrix is strictly column diagonally dominant, where
//    partial pivoting selects the diagonal anyway), a WN-column leaf inverts its WN x WN
//    diagonal block D and sets the other rows of the panel to -W_other D^{-1}, which is
//    exactly the Gauss-Jordan result for those pivots.
#include <cmath>
#include <type_traits>

#include "common.hpp"
#include "internal.hpp"

namespace lyap {
namespace {

constexpr int LEAF_THREADS = 512;  // pivoted leaf: 8 waves
constexpr int WN = 64;             // non-pivoted leaf width
constexpr int TT = 64;             // transpose tile

template <class T> struct LeafWidth;
template <> struct LeafWidth<double> { static constexpr int v = 8; };
template <> struct LeafWidth<float> { static constexpr int v = 8; };

// ---------------------------------------------------------------- prescale and copy
// Block b scans rows b, b + gridDim.x, ...; NaN anywhere poisons the partial.  Four
// independent maxima keep several loads in flight per thread.
__global__ void absmax_partial(int n, const double* __restrict__ A, long lda,
                               double* __restrict__ part) {
  __shared__ double red[256];
  __shared__ int rnan[256];
  double m4[4] = {0.0, 0.0, 0.0, 0.0};
  int nan = 0;
  for (int i = blockIdx.x; i < n; i += gridDim.x) {
    const double* a = A + (long)i * lda;
    int j = threadIdx.x;
    for (; j + 3 * 256 < n; j += 4 * 256) {
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const double v = fabs(a[j + u * 256]);
        if (v != v) nan = 1;
        else m4[u] = fmax(m4[u], v);
      }
    }
    for (; j < n; j += 256) {
      const double v = fabs(a[j]);
      if (v != v) nan = 1;
      else m4[0] = fmax(m4[0], v);
    }
  }
  const double m = fmax(fmax(m4[0], m4[1]), fmax(m4[2], m4[3]));
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

// Reduce the partial maxima (one workgroup of 256) and derive e with 2^(e-1) <= max < 2^e
// (0 when max == 0).
__global__ __launch_bounds__(256) void absmax_exponent(int nparts, const double* __restrict__ part,
                                                       int* __restrict__ e,
                                                       int* __restrict__ bad) {
  __shared__ double red[256];
  __shared__ int rnan[256];
  double m = 0.0;
  int nan = 0;
  for (int i = threadIdx.x; i < nparts; i += 256) {
    const double v = part[i];
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
  if (threadIdx.x == 0) {
    const double mx = red[0];
    int ex = 0;
    if (mx > 0.0 && !isinf(mx)) frexp(mx, &ex);
    *e = ex;
    if (rnan[0] || isinf(mx)) *bad = 1;
  }
}

// WT[j][i] = (T)(2^-e A[i][j]) through a TT x TT LDS tile; blocks of the first tile row also
// clear ``used``.
template <class T>
__global__ __launch_bounds__(256) void load_transposed(int n, const double* __restrict__ A,
                                                       long lda, const int* __restrict__ e,
                                                       bool scale, T* __restrict__ WT,
                                                       int* __restrict__ used) {
  __shared__ double tile[TT][TT + 1];
  const int t = threadIdx.x;
  const int i0 = blockIdx.y * TT, j0 = blockIdx.x * TT;
  if (blockIdx.y == 0 && t < TT && j0 + t < n) used[j0 + t] = 0;
  for (int q = t; q < TT * TT; q += 256) {
    const int r = q / TT, c = q % TT;
    const int i = i0 + r, j = j0 + c;
    tile[r][c] = (i < n && j < n) ? A[(long)i * lda + j] : 0.0;
  }
  __syncthreads();
  const int ex = scale ? *e : 0;
  for (int q = t; q < TT * TT; q += 256) {
    const int r = q / TT, c = q % TT;  // r: column offset, c: row offset
    const int j = j0 + r, i = i0 + c;
    if (i < n && j < n) {
      double v = tile[c][r];
      if (scale) v = ldexp(v, -ex);
      WT[(long)j * n + i] = (T)v;
    }
  }
}

// ------------------------------------------------------------------ pivoted leaf kernel
// One workgroup of LEAF_THREADS; thread t owns rows t + LEAF_THREADS * r, r < RPT, of the
// n x WC panel in registers (coalesced loads: the panel columns are contiguous).
//
// Pivot search per column: each thread scans its rows, each wave combines its 64 candidates
// with DPP moves (quad permutations and row mirrors) and lane reads, and the wave's winning
// lane publishes its candidate value, row index and row contents in LDS.  After a single
// barrier every thread combines the NW wave candidates in the same fixed order, so all
// threads agree on the pivot.  The candidate order (larger |value|, then lower row index,
// NaN counted as +inf) is a total order, hence the combine is associative and commutative.
constexpr int NO_ROW = 0x7fffffff;

template <int CTRL>
__device__ inline int dpp_i(int x) {
  return __builtin_amdgcn_update_dpp(x, x, CTRL, 0xf, 0xf, false);
}
template <int CTRL>
__device__ inline float dpp_t(float x) {
  return __int_as_float(dpp_i<CTRL>(__float_as_int(x)));
}
template <int CTRL>
__device__ inline double dpp_t(double x) {
  const long long b = __double_as_longlong(x);
  const int lo = dpp_i<CTRL>((int)(b & 0xffffffffll));
  const int hi = dpp_i<CTRL>((int)(b >> 32));
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}
__device__ inline float readlane_t(float x, int l) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), l));
}
__device__ inline double readlane_t(double x, int l) {
  const long long b = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), l);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

template <class T>
__device__ inline void take_better(T& best, int& brow, T ob, int orow) {
  if (ob > best || (ob == best && orow < brow)) { best = ob; brow = orow; }
}
template <int CTRL, class T>
__device__ inline void dpp_step(T& best, int& brow) {
  const T ob = dpp_t<CTRL>(best);
  const int orow = dpp_i<CTRL>(brow);
  take_better(best, brow, ob, orow);
}
// All lanes of the wave end with the wave's best candidate.
template <class T>
__device__ inline void wave_argmax(T& best, int& brow) {
  dpp_step<0xB1>(best, brow);   // quad_perm [1,0,3,2]
  dpp_step<0x4E>(best, brow);   // quad_perm [2,3,0,1]
  dpp_step<0x141>(best, brow);  // row_half_mirror: combines the two quads of each 8 lanes
  dpp_step<0x140>(best, brow);  // row_mirror: combines the two halves of each 16 lanes
  T b = readlane_t(best, 0);
  int r = __builtin_amdgcn_readlane(brow, 0);
  take_better(b, r, readlane_t(best, 16), __builtin_amdgcn_readlane(brow, 16));
  take_better(b, r, readlane_t(best, 32), __builtin_amdgcn_readlane(brow, 32));
  take_better(b, r, readlane_t(best, 48), __builtin_amdgcn_readlane(brow, 48));
  best = b;
  brow = r;
}

// With gv > 0 the leaf also does the gather of the block update that follows it,
// W[piv[c0..c0+wc), gc..gc+gv) -> RT (gv x wc) with those entries of W set to zero: they lie
// in columns the leaf does not touch, at rows it has just chosen as pivots.
template <class T, int RPT, int WC>
__global__ __launch_bounds__(LEAF_THREADS) void gj_leaf(int n, T* __restrict__ WT, int c0, int wc,
                                                         int* __restrict__ used,
                                                         int* __restrict__ piv,
                                                         int* __restrict__ sing, int gc, int gv,
                                                         T* __restrict__ RT,
                                                         T* __restrict__ pv) {
  constexpr int NW = LEAF_THREADS / 64;
  __shared__ T crow[2][NW][WC];  // per-wave candidate rows, double-buffered by column parity
  __shared__ T cval[2][NW];
  __shared__ int cidx[2][NW];
  __shared__ int lpiv[WC];
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  T v[RPT][WC];
  bool u[RPT];
  unsigned taken = 0;  // rows of this thread chosen as pivots in this leaf (bit r)
#pragma unroll
  for (int r = 0; r < RPT; ++r) {
    const int row = t + LEAF_THREADS * r;
    u[r] = true;
#pragma unroll
    for (int c = 0; c < WC; ++c) v[r][c] = (T)0;
    if (row < n) {
      u[r] = used[row] != 0;
#pragma unroll
      for (int c = 0; c < WC; ++c)
        if (c < wc) v[r][c] = WT[(long)(c0 + c) * n + row];
    }
  }
#pragma unroll
  for (int j = 0; j < WC; ++j) {
    if (j >= wc) continue;  // wc is uniform across the block
    const int buf = j & 1;
    T best = (T)-1;
    int brow = NO_ROW;
#pragma unroll
    for (int r = 0; r < RPT; ++r) {
      T a = fabs(v[r][j]);
      if (a != a) a = (T)INFINITY;
      if (!u[r] && a > best) { best = a; brow = t + LEAF_THREADS * r; }
    }
    wave_argmax(best, brow);
    if (brow != NO_ROW && (brow % LEAF_THREADS) == t) {  // the wave's winning lane
      const int rr = brow / LEAF_THREADS;
#pragma unroll
      for (int r = 0; r < RPT; ++r)
        if (r == rr) {
#pragma unroll
          for (int c = 0; c < WC; ++c) crow[buf][wave][c] = v[r][c];
        }
    }
    if (lane == 0) { cval[buf][wave] = best; cidx[buf][wave] = brow; }
    __syncthreads();
    best = cval[buf][0];
    brow = cidx[buf][0];
    int gw = 0;
#pragma unroll
    for (int w = 1; w < NW; ++w) {
      const T ob = cval[buf][w];
      const int orow = cidx[buf][w];
      if (ob > best || (ob == best && orow < brow)) { best = ob; brow = orow; gw = w; }
    }
    const int rp = brow;  // every thread holds the same winner
    T pr[WC];
#pragma unroll
    for (int c = 0; c < WC; ++c) pr[c] = crow[buf][gw][c];
    if (t == 0) lpiv[j] = rp == NO_ROW ? 0 : rp;
    T p = pr[j];
    if (t == 0) pv[c0 + j] = rp == NO_ROW ? (T)0 : p;
    const bool zero = rp == NO_ROW || !(best > (T)0) || !(fabs(p) > (T)0);
    if (t == 0 && zero) *sing = 1;
    if (zero) p = (T)1;  // singular: keep going, flagged
    const T inv = (T)1 / p;
#pragma unroll
    for (int r = 0; r < RPT; ++r) {
      const int row = t + LEAF_THREADS * r;
      if (row == rp) {
        u[r] = true;
        taken |= 1u << r;
#pragma unroll
        for (int c = 0; c < WC; ++c) v[r][c] = (c == j) ? inv : v[r][c] * inv;
      } else {
        const T f = v[r][j] * inv;
#pragma unroll
        for (int c = 0; c < WC; ++c) v[r][c] = (c == j) ? -f : v[r][c] - f * pr[c];
      }
    }
  }
  __syncthreads();  // lpiv complete
  if (t < wc) piv[c0 + t] = lpiv[t];
  if (t < gv * wc) {
    const int j = t / wc, k = t % wc;
    T* src = WT + (long)(gc + j) * n + lpiv[k];
    RT[t] = *src;
    *src = (T)0;
  }
#pragma unroll
  for (int r = 0; r < RPT; ++r) {
    const int row = t + LEAF_THREADS * r;
    if (taken & (1u << r)) used[row] = 1;
    if (row < n) {
#pragma unroll
      for (int c = 0; c < WC; ++c)
        if (c < wc) WT[(long)(c0 + c) * n + row] = v[r][c];
    }
  }
}

// -------------------------------------------------------------- non-pivoted leaf kernels
// Invert the w x w diagonal block D = W[c0.., c0..] (w <= WN) by Gauss-Jordan without
// pivoting; Dinv (w x w, row-major) to global; the pivots are the diagonal rows.  Thread t
// holds row i = t % 64 of D at the ND contiguous columns ND g + q (g = t / 64, q < ND) in
// registers, so the loads from WT are coalesced and the pivot row comes back from LDS as
// contiguous vectors; two waves per SIMD let one wave's barrier and LDS latency overlap the
// other's arithmetic, and the step loop is fully unrolled so that every register index is a
// constant.  Step k publishes the pivot row and the multiplier column in LDS
// (double-buffered, one barrier per step); a non-pivot row takes one FMA per entry,
// d <- d - (f / p) r.
constexpr int ND_THREADS = 512;
template <class T>
__global__ __launch_bounds__(ND_THREADS) void nop_diag(int n, const T* __restrict__ WT, int c0,
                                                       int w, T* __restrict__ Dinv,
                                                       int* __restrict__ used,
                                                       int* __restrict__ piv,
                                                       int* __restrict__ sing,
                                                       T* __restrict__ pv) {
  constexpr int NG = ND_THREADS / 64, ND = WN / NG;
  static_assert(WN == 64 && ND * NG == WN, "groups of ND columns");
  __shared__ __align__(16) T rowk[2][WN];
  __shared__ T colk[2][WN];
  const int t = threadIdx.x, i = t & 63, g = t >> 6;
  T d[ND];
#pragma unroll
  for (int q = 0; q < ND; ++q) {
    const int j = ND * g + q;
    d[q] = (i < w && j < w) ? WT[(long)(c0 + j) * n + c0 + i] : (T)(i == j ? 1 : 0);
  }
  if (t < w) {
    used[c0 + t] = 1;
    piv[c0 + t] = c0 + t;
  }
  // all WN steps run: past w the block is padded with the identity (block diagonal), whose
  // steps change nothing in the leading w x w block
#pragma unroll
  for (int k = 0; k < WN; ++k) {
    const int buf = k & 1;
    if (i == k) {
#pragma unroll
      for (int q = 0; q < ND; ++q) rowk[buf][ND * g + q] = d[q];
    }
    if (g == k / ND) colk[buf][i] = d[k % ND];
    __syncthreads();
    T r[ND];
#pragma unroll
    for (int q = 0; q < ND; ++q) r[q] = rowk[buf][ND * g + q];
    T p = rowk[buf][k];
    const T f = colk[buf][i];
    if (t == 0 && k < w) pv[c0 + k] = p;
    if (!(fabs(p) > (T)0)) {
      if (t == 0) *sing = 1;
      p = (T)1;
    }
    const T inv = (T)1 / p;
    const T fi = f * inv;
    if (i == k) {
#pragma unroll
      for (int q = 0; q < ND; ++q) d[q] = r[q] * inv;
    } else {
#pragma unroll
      for (int q = 0; q < ND; ++q) d[q] = fma(-fi, r[q], d[q]);
    }
    if (g == k / ND) d[k % ND] = (i == k) ? inv : -fi;
  }
#pragma unroll
  for (int q = 0; q < ND; ++q) {
    const int j = ND * g + q;
    if (i < w && j < w) Dinv[i * w + j] = d[q];
  }
}

// Panel rows: rows in [c0, c0+w) take Dinv, the others become -row * Dinv.  Block x owns
// rows [AR x, AR x + AR) at every panel column, so the panel entries it reads are the ones it
// overwrites (no other block touches them); thread t computes row AR x + t % AR at columns
// 8 (t / AR) + s, s < 8 (coalesced along rows in WT).
constexpr int AR = 32;
template <class T>
__global__ __launch_bounds__(256) void nop_apply(int n, T* __restrict__ WT, int c0, int w,
                                                 const T* __restrict__ Dinv) {
  static_assert(WN == 8 * (256 / AR), "one thread per row and 8 panel columns");
  __shared__ T Di[WN][WN];
  __shared__ T X[WN][AR];
  const int t = threadIdx.x, il = t % AR, jg = t / AR;
  const int i0 = blockIdx.x * AR;
  for (int q = t; q < WN * WN; q += 256) {
    const int k = q / WN, j = q % WN;
    Di[k][j] = (k < w && j < w) ? Dinv[k * w + j] : (T)0;
  }
  for (int q = t; q < WN * AR; q += 256) {
    const int k = q / AR, i = q % AR;
    X[k][i] = (k < w && i0 + i < n) ? WT[(long)(c0 + k) * n + i0 + i] : (T)0;
  }
  __syncthreads();
  const int gi = i0 + il;
  if (gi >= n) return;
  T acc[8] = {};
  for (int k = 0; k < w; ++k) {
    const T x = X[k][il];
#pragma unroll
    for (int s = 0; s < 8; ++s) acc[s] += x * Di[k][8 * jg + s];
  }
  const bool diag = gi >= c0 && gi < c0 + w;
#pragma unroll
  for (int s = 0; s < 8; ++s) {
    const int j = 8 * jg + s;
    if (j < w) WT[(long)(c0 + j) * n + gi] = diag ? Di[gi - c0][j] : -acc[s];
  }
}

// RT[j][k] = W[piv[a+k]][c+j] = WT[c+j][piv[a+k]]; that entry of W becomes 0.
template <class T>
__global__ void gather_zero(int n, T* __restrict__ WT, const int* __restrict__ piv, int a, int w,
                            int c, int v, T* __restrict__ RT) {
  long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
  long total = (long)w * v;
  if (idx >= total) return;
  int j = (int)(idx / w), k = (int)(idx % w);
  long src = (long)(c + j) * n + piv[a + k];
  RT[idx] = WT[src];
  WT[src] = (T)0;
}

// A^{-1}[i][r_j] = 2^-e W[r_i][j] = 2^-e WT[j][r_i], through a TT x TT LDS tile: rows of WT
// are gathered along r_i, rows of the output scattered along r_j.
template <class T>
__global__ __launch_bounds__(256) void unpermute(int n, const T* __restrict__ WT,
                                                 const int* __restrict__ piv,
                                                 const int* __restrict__ e, bool scale,
                                                 double* __restrict__ out, long ldo,
                                                 int* __restrict__ bad) {
  __shared__ double tile[TT][TT + 1];
  const int t = threadIdx.x;
  const int i0 = blockIdx.y * TT, j0 = blockIdx.x * TT;
  const int ex = scale ? *e : 0;
  for (int q = t; q < TT * TT; q += 256) {
    const int r = q / TT, c = q % TT;  // r: j offset, c: i offset
    const int j = j0 + r, i = i0 + c;
    tile[r][c] = (i < n && j < n) ? (double)WT[(long)j * n + piv[i]] : 0.0;
  }
  __syncthreads();
  int nonfinite = 0;
  for (int q = t; q < TT * TT; q += 256) {
    const int r = q / TT, c = q % TT;  // r: i offset, c: j offset
    const int i = i0 + r, j = j0 + c;
    if (i < n && j < n) {
      double x = tile[c][r];
      if (scale) x = ldexp(x, -ex);
      if (!isfinite(x)) nonfinite = 1;
      out[(long)i * ldo + piv[j]] = x;
    }
  }
  if (nonfinite) *bad = 1;
}

// log|det A| = sum_j log|p_j| + n e log 2 from the Gauss-Jordan pivots p_j of the working
// copy 2^-e A (the pivots of Gauss-Jordan elimination are those of LU with the same row
// order); one workgroup, fixed summation order.
template <class T>
__global__ __launch_bounds__(256) void logdet_pivots(int n, const T* __restrict__ pv,
                                                     const int* __restrict__ e, bool scale,
                                                     double* __restrict__ out) {
  __shared__ double red[256];
  double acc = 0.0;
  for (int j = threadIdx.x; j < n; j += 256) acc += log(fabs((double)pv[j]));
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double ex = scale ? (double)(*e) : 0.0;
    *out = red[0] + (double)n * ex * 0.69314718055994530942;
  }
}

template <class T> struct Inv {
  hipStream_t s;
  int n;
  T* WT;
  T* RT;
  T* Dinv;
  int* used;
  int* piv;
  int* sing;
  T* pv;
  Prec op;
  bool pivot;

  int leaf_width() const { return pivot ? LeafWidth<T>::v : WN; }

  // gc / gv: columns of the update that follows, whose gather the pivoted leaf does itself
  int leaf(int c0, int wc, int gc = 0, int gv = 0) {
    if (!pivot) {
      hipLaunchKernelGGL((nop_diag<T>), dim3(1), dim3(ND_THREADS), 0, s, n, WT, c0, wc, Dinv, used, piv,
                         sing, pv);
      hipLaunchKernelGGL((nop_apply<T>), dim3((unsigned)ceil_div(n, AR)), dim3(256), 0, s, n, WT,
                         c0, wc, Dinv);
      LYAP_HIP(hipGetLastError());
      return LYAP_OK;
    }
    constexpr int WC = LeafWidth<T>::v;
    const int rpt = ceil_div(n, LEAF_THREADS);
#define LEAF(RPT)                                                                          \
  hipLaunchKernelGGL((gj_leaf<T, RPT, WC>), dim3(1), dim3(LEAF_THREADS), 0, s, n, WT, c0, wc, \
                     used, piv, sing, gc, gv, RT, pv)
    if (rpt <= 1) LEAF(1);
    else if (rpt <= 2) LEAF(2);
    else if (rpt <= 4) LEAF(4);
    else if (rpt <= 8) LEAF(8);
    else return LYAP_BADARG;
#undef LEAF
    LYAP_HIP(hipGetLastError());
    return LYAP_OK;
  }

  // WT[c:d, :] += RT WT[a:b, :] with RT (d-c) x (b-a) gathered from the pivot rows (here, or
  // by the leaf just before when ``gathered``).
  int update(int a, int b, int c, int d, bool gathered = false) {
    int w = b - a, v = d - c;
    long total = (long)w * v;
    if (!gathered) {
      hipLaunchKernelGGL((gather_zero<T>), dim3((unsigned)((total + 255) / 256)), dim3(256), 0,
                         s, n, WT, piv, a, w, c, v, RT);
      LYAP_HIP(hipGetLastError());
    }
    GemmDesc g;
    g.M = v; g.N = n; g.K = w;
    g.alpha = 1.0; g.beta = 1.0;
    g.A = RT; g.sar = w; g.sac = 1;
    g.B = WT + (long)a * n; g.sbr = n; g.sbc = 1;
    g.C = WT + (long)c * n; g.ldc = n;
    if (std::is_same<T, double>::value) return gemm_f64(s, g);
    return gemm_lp(s, op, Store::F32, Store::F32, Store::F32, g);
  }

  int rec(int c0, int c1) {
    const int lw = leaf_width();
    int w = c1 - c0;
    if (w <= lw) return leaf(c0, w);
    int half = ceil_div(ceil_div(w, 2), lw) * lw;
    int mid = c0 + half;
    if (mid >= c1) mid = c1 - lw;
    if (pivot && mid - c0 <= lw && c1 - mid <= lw) {
      // two pivoted leaves: each does the gather of the update after it
      LYAP_TRY(leaf(c0, mid - c0, mid, c1 - mid));
      LYAP_TRY(update(c0, mid, mid, c1, true));
      LYAP_TRY(leaf(mid, c1 - mid, c0, mid - c0));
      LYAP_TRY(update(mid, c1, c0, mid, true));
      return LYAP_OK;
    }
    LYAP_TRY(rec(c0, mid));
    LYAP_TRY(update(c0, mid, mid, c1));
    LYAP_TRY(rec(mid, c1));
    LYAP_TRY(update(mid, c1, c0, mid));
    return LYAP_OK;
  }
};

template <class T>
int invert_t(hipStream_t s, Prec op, int n, const double* A, long lda, double* out, long ldo,
             Arena& ws, int* flags_dev, bool pivot, double* logdet) {
  size_t nn = (size_t)n * n;
  const size_t half = (size_t)((n + 1) / 2 + WN);
  T* WT = ws.take<T>(nn);
  T* RT = ws.take<T>(half * half);
  T* Dinv = ws.take<T>((size_t)WN * WN);
  int* used = ws.take<int>(n);
  int* piv = ws.take<int>(n);
  int* ex = ws.take<int>(1);
  T* pv = ws.take<T>(n);
  const int nparts = n >= 1024 ? 1024 : 256;  // four workgroups per CU for a large matrix
  double* part = ws.take<double>(nparts);
  if (!WT || !RT || !Dinv || !used || !piv || !ex || !part || !pv) return LYAP_NO_MEMORY;
  const bool scale = !std::is_same<T, double>::value;
  const dim3 tiles((unsigned)ceil_div(n, TT), (unsigned)ceil_div(n, TT));
  hipLaunchKernelGGL(absmax_partial, dim3(nparts), dim3(256), 0, s, n, A, lda, part);
  hipLaunchKernelGGL(absmax_exponent, dim3(1), dim3(256), 0, s, nparts, part, ex, flags_dev + 1);
  hipLaunchKernelGGL((load_transposed<T>), tiles, dim3(256), 0, s, n, A, lda, ex, scale, WT, used);
  LYAP_HIP(hipGetLastError());
  Inv<T> inv{s, n, WT, RT, Dinv, used, piv, flags_dev + 0, pv, op, pivot};
  LYAP_TRY(inv.rec(0, n));
  if (logdet)
    hipLaunchKernelGGL((logdet_pivots<T>), dim3(1), dim3(256), 0, s, n, pv, ex, scale, logdet);
  hipLaunchKernelGGL((unpermute<T>), tiles, dim3(256), 0, s, n, WT, piv, ex, scale, out, ldo,
                     flags_dev + 1);
  LYAP_HIP(hipGetLastError());
  return LYAP_OK;
}

}  // namespace

size_t inverse_workspace_bytes(Prec op, int n) {
  size_t el = op == Prec::F64 ? 8 : 4;
  size_t half = (size_t)((n + 1) / 2 + WN);
  return (size_t)n * n * el + half * half * el + (size_t)WN * WN * el + 4 * (size_t)n * 4 +
         (size_t)n * el + 1024 * 8 + 12 * 256;
}

// flags_dev[0] = singular pivot seen, flags_dev[1] = non-finite input/output (device ints,
// zeroed by the caller).
int invert(hipStream_t s, Prec op, int n, const double* A, long lda, double* out, long ldo,
           Arena& ws, int* flags_dev, bool pivot, KernTimer* kt, double* logdet) {
  if (n <= 0) return LYAP_OK;
  if (n > 8 * LEAF_THREADS) return LYAP_BADARG;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (kt) LYAP_TRY(kt->mark(s, &e0));
  if (op == Prec::F64)
    LYAP_TRY(invert_t<double>(s, op, n, A, lda, out, ldo, ws, flags_dev, pivot, logdet));
  else LYAP_TRY(invert_t<float>(s, op, n, A, lda, out, ldo, ws, flags_dev, pivot, logdet));
  if (kt) {
    LYAP_TRY(kt->mark(s, &e1));
    kt->add(e0, e1, 0, 2.0 * (double)n * n * n, 1);
  }
  return LYAP_OK;
}

}  // namespace lyap
