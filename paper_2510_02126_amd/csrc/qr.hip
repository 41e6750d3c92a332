// Thin QR F = U T of an n x p FP64 matrix (U n x min(n,p) orthonormal, T upper trapezoidal)
// (the "thin QR decomposition" of Fragments 2.1-2.4 and of RankTruncLdlt in Alg 3.2), by
// Householder reflections only.
//
// Right-looking, panel by panel (32 columns).  Panel j covers columns [c, c+w) and rows
// [c, n) of the working copy.  Its orthogonal factor is a two-level tree of Householder
// reflectors (tall-skinny QR):
//   level 1  each 256-row chunk is factored by one workgroup,
//   level 2  the stacked chunk R factors (<= 16 x 32 rows) are factored by one workgroup.
// Each set of (at most 32) reflectors is kept in compact WY form H_0 H_1 ... H_{k-1} =
// I - V Tw V^T (V unit lower trapezoidal, Tw upper triangular), so the panel's transformation
// Q_j^T is applied to the trailing columns as X <- X - V Tw^T (V^T X): three products on the
// FP64 matrix cores per 32-column tile (level 1 per chunk, then level 2 on the stacked rows),
// which leaves the R rows of the panel in rows [c, c+w).  After the last panel,
// U = Q_1 ... Q_k [I_p; 0] is formed by applying the block reflectors in reverse.  Because
// only reflectors are used, U is orthonormal to working precision even for numerically
// rank-deficient F (such as F = [Z, AZ, L] near convergence, where AZ lies almost in the span
// of Z and L).
//
// Panel factorisation: the r x 32 block is held in registers, 4 (or 8) rows x 8 columns per
// thread, and the 32 steps are unrolled.  Step k forms, in one reduction over rows below k, the
// sums s_c = sum_i A[i][c] A[i][k] for all 32 columns: s_k is the squared norm below the
// diagonal, s_j (j > k) gives the reflector's action on the trailing columns and s_c (c < k)
// gives v_c^T v_k.  Those inner products and the tau_k make up the inverse of Tw
// (diag(1 / tau) plus the strict upper triangle of V^T V), which is inverted after the loop.
#include <algorithm>
#include <cmath>

#include "common.hpp"
#include "internal.hpp"

namespace lyap {
namespace {

constexpr int PB = 32;     // panel width
constexpr int CH = 256;    // chunk rows at level 1
constexpr int NTH = 256;   // threads per workgroup
constexpr int MAXCH = 16;  // chunks per panel (n <= 4096)

constexpr int CPT = 8;         // panel columns per thread
constexpr int NCG = PB / CPT;  // column groups: thread t owns column group t % NCG

template <int NT>
struct PanelLds {
  double part[NT / 16][PB];  // partial sums per 16-lane row of each wave
  double prow[PB];            // row k
  double dvec[PB];            // tau (A[k][j] + v_k^T A[k+1:, j]) for j > k, else 0
  double sc[2];               // beta, scale
  double tau[PB];
  double Zs[PB][PB + 1];      // Zs[k][c] = (V^T v_k)[c] for c < k
  double Tw[PB][PB + 1];
};

template <int CTRL>
__device__ inline double dpp_d(double x) {
  const long long b = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_update_dpp((int)(b & 0xffffffffll), (int)(b & 0xffffffffll),
                                             CTRL, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp((int)(b >> 32), (int)(b >> 32), CTRL, 0xf, 0xf,
                                             false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// Householder QR of an r x w block (r <= NT RPR / 4, w <= PB).  Thread t = NCG g + cg holds rows
// g RPR + i (i < RPR) at columns CPT cg + jj (jj < CPT) in a[i][jj].  On return the rows hold
// R on and above the diagonal and the reflectors v below it (unit diagonal implied); L.Tw holds
// Tw (zero outside the kmax x kmax upper triangle).
//
// Step k: the pivot column reaches the other threads of a row group by quad broadcasts; the
// sums s_c = sum_{i>k} A[i][c] A[i][k] are reduced inside each 16-lane row by DPP rotations
// and across rows and waves in LDS by 32 threads, which then form the reflector (s_k is the
// squared norm below the diagonal), the update coefficients of the trailing columns and
// z = V^T v_k for the Tw recurrence.
template <int RPR, int NT>
__device__ void panel_factor(double (&a)[RPR][CPT], int r, int w, PanelLds<NT>& L) {
  const int t = threadIdx.x, cg = t % NCG, g = t / NCG;
  const int lane = t & 63, wave = t >> 6;
  const int kmax = min(r, w);
  for (int e = t; e < PB * PB; e += NT) L.Tw[e / PB][e % PB] = 0.0;
  // fully unrolled, so the pivot column's group and slot are constants of each step
#pragma unroll
  for (int k = 0; k < PB; ++k) {
    if (k < kmax) {
    const int cgk = k / CPT, jk = k % CPT;
    double x[RPR];
#pragma unroll
    for (int i = 0; i < RPR; ++i) {
      const int row = g * RPR + i;
      double mine = 0.0;
#pragma unroll
      for (int jj = 0; jj < CPT; ++jj)
        if (jj == jk) mine = a[i][jj];
      if (row == k) {
#pragma unroll
        for (int jj = 0; jj < CPT; ++jj) L.prow[CPT * cg + jj] = a[i][jj];
      }
      const double b0 = dpp_d<0x00>(mine), b1 = dpp_d<0x55>(mine);  // quad lanes 0, 1
      const double b2 = dpp_d<0xAA>(mine), b3 = dpp_d<0xFF>(mine);  // quad lanes 2, 3
      x[i] = cgk == 0 ? b0 : (cgk == 1 ? b1 : (cgk == 2 ? b2 : b3));
    }
    double pr[CPT];
#pragma unroll
    for (int jj = 0; jj < CPT; ++jj) pr[jj] = 0.0;
#pragma unroll
    for (int i = 0; i < RPR; ++i) {
      const int row = g * RPR + i;
      if (row > k && row < r) {
#pragma unroll
        for (int jj = 0; jj < CPT; ++jj) pr[jj] += a[i][jj] * x[i];
      }
    }
    // lanes cg, cg + 4, cg + 8, cg + 12 of each 16-lane row share a column group
#pragma unroll
    for (int jj = 0; jj < CPT; ++jj) {
      pr[jj] += dpp_d<0x124>(pr[jj]);  // row_ror:4
      pr[jj] += dpp_d<0x128>(pr[jj]);  // row_ror:8
    }
    if ((lane & 15) < NCG) {
#pragma unroll
      for (int jj = 0; jj < CPT; ++jj) L.part[wave * 4 + (lane >> 4)][CPT * cg + jj] = pr[jj];
    }
    __syncthreads();
    if (t < PB) {
      double sc = 0.0;
#pragma unroll
      for (int q = 0; q < NT / 16; ++q) sc += L.part[q][t];
      const double sigma = __shfl(sc, k, PB);
      const double alpha = L.prow[k];
      double beta, tau, scale;
      if (sigma == 0.0) {
        beta = alpha;
        tau = 0.0;
        scale = 0.0;
      } else {
        const double nrm = sqrt(alpha * alpha + sigma);
        beta = alpha <= 0.0 ? nrm : -nrm;
        tau = (beta - alpha) / beta;
        scale = 1.0 / (alpha - beta);
      }
      const double z = L.prow[t] + scale * sc;  // A[k][t] + v_k^T A[k+1:, t]
      L.dvec[t] = t > k ? tau * z : 0.0;
      if (t < k) L.Zs[k][t] = z;
      if (t == 0) {
        L.sc[0] = beta;
        L.sc[1] = scale;
        L.tau[k] = tau;
      }
    }
    __syncthreads();
    const double beta = L.sc[0], scale = L.sc[1];
    double d[CPT];
#pragma unroll
    for (int jj = 0; jj < CPT; ++jj) d[jj] = L.dvec[CPT * cg + jj];
#pragma unroll
    for (int i = 0; i < RPR; ++i) {
      const int row = g * RPR + i;
      if (row == k) {
#pragma unroll
        for (int jj = 0; jj < CPT; ++jj)
          a[i][jj] = (cg == cgk && jj == jk) ? beta : a[i][jj] - d[jj];
      } else if (row > k && row < r) {
        const double v = scale * x[i];
#pragma unroll
        for (int jj = 0; jj < CPT; ++jj)
          a[i][jj] = (cg == cgk && jj == jk) ? v : a[i][jj] - d[jj] * v;
      }
    }
    }
  }
  __syncthreads();
  // Tw is the inverse of the upper triangular U with U[c][c] = 1 / tau_c and U[c][k] = v_c^T v_k
  // = Zs[k][c] (c < k): the recurrence Tw_k = [[Tw_{k-1}, -tau_k Tw_{k-1} V^T v_k], [0, tau_k]]
  // inverts to [[U_{k-1}, V^T v_k], [0, 1 / tau_k]].  It is inverted by doubling: with the
  // diagonal blocks Tw11, Tw22 (s x s) of a 2s x 2s diagonal block known, its upper right block
  // is -Tw11 U12 Tw22.  Diagonal entries are set to tau_c directly, so a reflector with tau = 0
  // (an identity factor) gets a zero row and column, as in the recurrence; indices >= kmax
  // stay zero.
  if (t < kmax) L.Tw[t][t] = L.tau[t];
  double* X = &L.part[0][0];  // s x s products of the current level, 16 s entries
  for (int s = 1; s < PB; s *= 2) {
    __syncthreads();
    const int b = t / (s * s), i = (t / s) % s, j = t % s;
    const int r0 = 2 * s * b, c0 = r0 + s;
    const bool act = t < 16 * s;  // PB / (2 s) block pairs of s x s entries
    if (act) {
      double x = 0.0;  // (U12 Tw22)[i][j], Tw22 upper triangular
      for (int k = 0; k <= j; ++k) {
        const int c = r0 + i, kk = c0 + k;
        const double u = (kk < kmax) ? L.Zs[kk][c] : 0.0;
        x += u * L.Tw[kk][c0 + j];
      }
      X[t] = x;
    }
    __syncthreads();
    if (act) {
      double y = 0.0;  // (Tw11 X)[i][j], Tw11 upper triangular
      for (int k = i; k < s; ++k) y += L.Tw[r0 + i][r0 + k] * X[b * s * s + k * s + j];
      L.Tw[r0 + i][c0 + j] = -y;
    }
  }
  __syncthreads();
}

template <int RPR>
__device__ void panel_load(double (&a)[RPR][CPT], const double* __restrict__ src, long ld, int r,
                           int w) {
  const int t = threadIdx.x, cg = t % NCG, g = t / NCG;
#pragma unroll
  for (int i = 0; i < RPR; ++i) {
    const int row = g * RPR + i;
#pragma unroll
    for (int jj = 0; jj < CPT; ++jj) {
      const int c = CPT * cg + jj;
      a[i][jj] = (row < r && c < w) ? src[(long)row * ld + c] : 0.0;
    }
  }
}

// The reflectors below the diagonal (kmax of them) as a unit lower trapezoidal r x PB matrix
// (zero above the diagonal and beyond kmax).
template <int RPR>
__device__ void panel_store_v(const double (&a)[RPR][CPT], double* __restrict__ dst, int r,
                              int kmax) {
  const int t = threadIdx.x, cg = t % NCG, g = t / NCG;
#pragma unroll
  for (int i = 0; i < RPR; ++i) {
    const int row = g * RPR + i;
    if (row < r) {
#pragma unroll
      for (int jj = 0; jj < CPT; ++jj) {
        const int c = CPT * cg + jj;
        dst[(long)row * PB + c] = c < kmax ? (row > c ? a[i][jj] : (row == c ? 1.0 : 0.0)) : 0.0;
      }
    }
  }
}

// Rows < PB of R (upper triangle of the first kmax rows, columns < w) with row stride ldr;
// ``full`` writes zeros for the other entries of the PB x PB block, otherwise only columns < w.
template <int RPR>
__device__ void panel_store_r(const double (&a)[RPR][CPT], double* __restrict__ dst, long ldr,
                              int kmax, int w, bool full) {
  const int t = threadIdx.x, cg = t % NCG, g = t / NCG;
#pragma unroll
  for (int i = 0; i < RPR; ++i) {
    const int row = g * RPR + i;
    if (row < (full ? PB : w)) {
#pragma unroll
      for (int jj = 0; jj < CPT; ++jj) {
        const int c = CPT * cg + jj;
        const double v = (row < kmax && c >= row && c < w) ? a[i][jj] : 0.0;
        if (full || c < w) dst[(long)row * ldr + c] = v;
      }
    }
  }
}

// Level 1: chunk b of the panel (rows [b*CH, b*CH + rows) of P, w columns).  Writes the
// reflectors (unit lower trapezoidal, zero above) to Vg rows, Tw to Twg[b] and the chunk's R
// (PB x PB, zero below the diagonal and beyond kmax) to Rstack[b].
__global__ __launch_bounds__(NTH) void tsqr_local(int nr, int w, const double* __restrict__ P,
                                                  long ldp, double* __restrict__ Vg,
                                                  double* __restrict__ Twg,
                                                  double* __restrict__ Rstack) {
  __shared__ PanelLds<NTH> L;
  constexpr int RPR = CH / (NTH / NCG);
  const int b = blockIdx.x, r0 = b * CH, rows = min(CH, nr - r0), t = threadIdx.x;
  double a[RPR][CPT];
  panel_load<RPR>(a, P + (long)r0 * ldp, ldp, rows, w);
  panel_factor<RPR, NTH>(a, rows, w, L);
  const int kmax = min(rows, w);
  panel_store_r<RPR>(a, Rstack + (long)b * PB * PB, PB, kmax, w, true);
  double* Tw = Twg + (long)b * PB * PB;
  for (int e = t; e < PB * PB; e += NTH) Tw[e] = L.Tw[e / PB][e % PB];
  panel_store_v<RPR>(a, Vg + (long)r0 * PB, rows, kmax);
}

// Level 2: QR of the stacked R factors (nch*PB x w) by one workgroup of NTS threads (4 rows
// per thread, as at level 1); R (w x w) goes to T, the reflectors to V2 (nch*PB x PB) and the
// WY factor to Tw2.
constexpr int NTS = 512;
__global__ __launch_bounds__(NTS) void tsqr_stack(int nch, int w, const double* __restrict__ Rstack,
                                                  double* __restrict__ T, long ldt,
                                                  double* __restrict__ V2,
                                                  double* __restrict__ Tw2) {
  __shared__ PanelLds<NTS> L;
  constexpr int RPR = MAXCH * PB / (NTS / NCG);
  const int r = nch * PB, t = threadIdx.x;
  double a[RPR][CPT];
  panel_load<RPR>(a, Rstack, PB, r, w);
  panel_factor<RPR, NTS>(a, r, w, L);
  const int kmax = min(r, w);
  panel_store_r<RPR>(a, T, ldt, kmax, w, false);
  for (int e = t; e < PB * PB; e += NTS) Tw2[e] = L.Tw[e / PB][e % PB];
  panel_store_v<RPR>(a, V2, r, kmax);
}

__device__ inline f64x4 mfma_f64(double a, double b, f64x4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// X <- (I - V Tw V^T)^T X (trans) or (I - V Tw V^T) X on a set of rows of X and 32 columns
// [32 blockIdx.y, ...).  STACK = false: the rows of chunk blockIdx.x (panel rows
// [b*CH, b*CH + CH) clipped to nr), V = Vg rows of that chunk, Tw = Twg[b].  STACK = true:
// the stacked rows i < nch*PB, i.e. panel row (i / PB) * CH + i % PB, V = V2, Tw = Tw2.
// Y = V^T X, Y <- op(Tw) Y, X <- X - V Y, all on the FP64 matrix cores with the operands of
// V and X loaded from memory straight into the matrix-core lanes.  For Y each wave sums all
// four 16 x 16 tiles over a quarter of the rows and the four partial sums are added in a
// fixed order in LDS; the update then covers the same quarter of the rows, whose X entries
// each lane still holds in registers from the first product (lane (r, k) of step m loaded row
// 4 m + k of the quarter, which is where the update's result lands), so X is read once.
template <bool STACK>
__global__ __launch_bounds__(NTH) void apply_wy(int nr, int nch, bool trans,
                                                const double* __restrict__ Vsrc,
                                                const double* __restrict__ Twsrc,
                                                double* __restrict__ X, long ldx, int ncols) {
  __shared__ double Yp[4][PB][PB + 1];
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int lr = lane & 15, lk = lane >> 4;
  const int b = STACK ? 0 : blockIdx.x;
  const int rows = STACK ? nch * PB : min(CH, nr - b * CH);
  const int c0 = blockIdx.y * PB;
  const double* V = STACK ? Vsrc : Vsrc + (long)b * CH * PB;
  const double* Tw = STACK ? Twsrc : Twsrc + (long)b * PB * PB;
  auto xrow = [&](int i) -> int {  // panel row of block row i, or -1
    if (i >= rows) return -1;
    const int g = STACK ? (i / PB) * CH + (i % PB) : b * CH + i;
    return g < nr ? g : -1;
  };
  const bool col0 = c0 + lr < ncols, col1 = c0 + 16 + lr < ncols;
  // Y partial over rows [i0, i1) of this wave
  constexpr int MX = (STACK ? MAXCH * PB : CH) / 16;  // most 4-row steps of a quarter
  const int rpw = (((rows + 3) / 4 + 3) / 4) * 4;  // a quarter of the rows, a multiple of 4
  const int i0 = wave * rpw, i1 = min(rows, i0 + rpw);
  f64x4 y00 = {0.0, 0.0, 0.0, 0.0}, y01 = y00, y10 = y00, y11 = y00;
  double xs0[MX], xs1[MX];  // X entries of this lane's rows, kept for the update
#pragma unroll
  for (int m = 0; m < MX; ++m) {
    const int k0 = i0 + 4 * m;
    xs0[m] = 0.0;
    xs1[m] = 0.0;
    if (k0 < i1) {  // uniform across the wave
      const int i = k0 + lk;
      const int g = i < i1 ? xrow(i) : -1;
      const double v0 = i < i1 ? V[(long)i * PB + lr] : 0.0;
      const double v1 = i < i1 ? V[(long)i * PB + 16 + lr] : 0.0;
      xs0[m] = (g >= 0 && col0) ? X[(long)g * ldx + c0 + lr] : 0.0;
      xs1[m] = (g >= 0 && col1) ? X[(long)g * ldx + c0 + 16 + lr] : 0.0;
      y00 = mfma_f64(v0, xs0[m], y00);
      y01 = mfma_f64(v0, xs1[m], y01);
      y10 = mfma_f64(v1, xs0[m], y10);
      y11 = mfma_f64(v1, xs1[m], y11);
    }
  }
  // D layout (FP64 16x16x4): lane l, register i -> row 4 i + l / 16, column l % 16
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    Yp[wave][4 * i + lk][lr] = y00[i];
    Yp[wave][4 * i + lk][16 + lr] = y01[i];
    Yp[wave][16 + 4 * i + lk][lr] = y10[i];
    Yp[wave][16 + 4 * i + lk][16 + lr] = y11[i];
  }
  __syncthreads();
  for (int e = t; e < PB * PB; e += NTH) {
    const int i = e / PB, c = e % PB;
    Yp[0][i][c] = ((Yp[0][i][c] + Yp[1][i][c]) + Yp[2][i][c]) + Yp[3][i][c];
  }
  __syncthreads();
  // Y2 = op(Tw) Y into Yp[1]: wave w owns the 16 x 16 tile (w / 2, w % 2)
  const int ti = wave >> 1, tj = wave & 1;
  f64x4 y2 = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int k = 0; k < PB; k += 4) {
    const double aop = trans ? Tw[(k + lk) * PB + 16 * ti + lr] : Tw[(16 * ti + lr) * PB + k + lk];
    y2 = mfma_f64(aop, Yp[0][k + lk][16 * tj + lr], y2);
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) Yp[1][16 * ti + 4 * i + lk][16 * tj + lr] = y2[i];
  __syncthreads();
  // X <- X - V Y2 on this wave's rows [i0, i1), 16-row tiles; result row r0 + 4 i + k of
  // lane (r, k) is row 4 (4 t + i) + k of the quarter, held in xs*[4 t + i]
#pragma unroll
  for (int tt = 0; tt < MX / 4; ++tt) {
    const int r0 = i0 + 16 * tt;
    if (r0 < i1) {  // uniform across the wave
      double vt[PB / 4];
#pragma unroll
      for (int q = 0; q < PB / 4; ++q)
        vt[q] = r0 + lr < rows ? V[(long)(r0 + lr) * PB + 4 * q + lk] : 0.0;
#pragma unroll
      for (int cj = 0; cj < 2; ++cj) {
        f64x4 u = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int q = 0; q < PB / 4; ++q)
          u = mfma_f64(vt[q], Yp[1][4 * q + lk][16 * cj + lr], u);
        const bool cok = cj == 0 ? col0 : col1;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int row = r0 + 4 * i + lk;
          const int g = row < i1 ? xrow(row) : -1;
          if (g >= 0 && cok)
            X[(long)g * ldx + c0 + 16 * cj + lr] = (cj == 0 ? xs0[4 * tt + i] : xs1[4 * tt + i]) - u[i];
        }
      }
    }
  }
}

__global__ void copy_rows(int rows, int cols, const double* __restrict__ src, long lds,
                          double* __restrict__ dst, long ldd) {
  long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (long)rows * cols) return;
  int i = (int)(idx / cols), j = (int)(idx % cols);
  dst[(long)i * ldd + j] = src[(long)i * lds + j];
}

__global__ void zero_block(int rows, int cols, double* __restrict__ dst, long ldd) {
  long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (long)rows * cols) return;
  int i = (int)(idx / cols), j = (int)(idx % cols);
  dst[(long)i * ldd + j] = 0.0;
}

__global__ void eye_block(int rows, int cols, double* __restrict__ dst, long ldd) {
  long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (long)rows * cols) return;
  int i = (int)(idx / cols), j = (int)(idx % cols);
  dst[(long)i * ldd + j] = i == j ? 1.0 : 0.0;
}

__global__ void add_block(int rows, int cols, const double* __restrict__ src, long lds,
                          double* __restrict__ dst, long ldd) {
  long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (long)rows * cols) return;
  int i = (int)(idx / cols), j = (int)(idx % cols);
  dst[(long)i * ldd + j] += src[(long)i * lds + j];
}

inline unsigned nb256(long total) { return (unsigned)((total + 255) / 256); }

// X (rows x cols, leading dimension ldx) <- uniform values in [-1, 1) from a counter-based
// generator (the SplitMix64 finaliser of seed + linear index), the same on every run.
__global__ void fill_uniform(int rows, int cols, double* __restrict__ X, long ldx,
                             unsigned long long seed) {
  long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (long)rows * cols) return;
  unsigned long long x = seed + (unsigned long long)idx + 0x9e3779b97f4a7c15ull;
  x = (x ^ (x >> 30)) * 0xbf58476d1ce4e5b9ull;
  x = (x ^ (x >> 27)) * 0x94d049bb133111ebull;
  x ^= x >> 31;
  const int i = (int)(idx / cols), j = (int)(idx % cols);
  X[(long)i * ldx + j] = (double)(x >> 11) * 0x1.0p-52 - 1.0;
}

}  // namespace

size_t qr_workspace_bytes(int n, int p) {
  size_t npan = (size_t)ceil_div(std::min(n, p), PB);
  size_t s = 0;
  s += align_up((size_t)n * p * 8, 256);                       // working copy
  s += npan * align_up((size_t)n * PB * 8, 256);               // level-1 reflectors per panel
  s += npan * align_up((size_t)MAXCH * PB * PB * 8, 256);      // level-1 WY factors
  s += npan * align_up((size_t)MAXCH * PB * PB * 8, 256);      // level-2 reflectors
  s += npan * align_up((size_t)PB * PB * 8, 256);              // level-2 WY factor
  s += align_up((size_t)MAXCH * PB * PB * 8, 256);             // stacked R factors
  return s + 4096;
}

int qr(hipStream_t s, int n, int p, const double* F, long ldf, double* U, long ldu, double* T,
       long ldt, Arena& ws, KernTimer* kt) {
  if (p <= 0 || n <= 0) return LYAP_OK;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (kt) LYAP_TRY(kt->mark(s, &e0));
  if (n > MAXCH * CH) return LYAP_BADARG;
  const int kk = std::min(n, p);  // U is n x kk, T is kk x p (upper trapezoidal)
  const int npan = ceil_div(kk, PB);
  double* W = ws.take<double>((size_t)n * p);
  double* Rstack = ws.take<double>((size_t)MAXCH * PB * PB);
  if (!W || !Rstack) return LYAP_NO_MEMORY;
  struct Pan { double *Vg, *Twg, *V2, *Tw2; };
  Pan pans[4096 / PB];
  for (int j = 0; j < npan; ++j) {
    pans[j].Vg = ws.take<double>((size_t)n * PB);
    pans[j].Twg = ws.take<double>((size_t)MAXCH * PB * PB);
    pans[j].V2 = ws.take<double>((size_t)MAXCH * PB * PB);
    pans[j].Tw2 = ws.take<double>((size_t)PB * PB);
    if (!pans[j].Vg || !pans[j].Twg || !pans[j].V2 || !pans[j].Tw2) return LYAP_NO_MEMORY;
  }
  LYAP_TRY(copy_block(s, n, p, F, ldf, W, p));
  hipLaunchKernelGGL(zero_block, dim3(nb256((long)kk * p)), dim3(256), 0, s, kk, p, T, ldt);
  for (int j = 0; j < npan; ++j) {
    const int c = j * PB, w = std::min(PB, kk - c), nr = n - c, nch = ceil_div(nr, CH);
    double* P = W + (long)c * p + c;  // rows [c, n), columns [c, c+w)
    hipLaunchKernelGGL(tsqr_local, dim3(nch), dim3(NTH), 0, s, nr, w, P, (long)p, pans[j].Vg,
                       pans[j].Twg, Rstack);
    hipLaunchKernelGGL(tsqr_stack, dim3(1), dim3(NTS), 0, s, nch, w, Rstack,
                       T + (long)c * ldt + c, ldt, pans[j].V2, pans[j].Tw2);
    const int rest = p - c - w;
    if (rest > 0) {
      double* X = P + w;  // rows [c, n), columns [c+w, p)
      const unsigned ct = (unsigned)ceil_div(rest, PB);
      hipLaunchKernelGGL((apply_wy<false>), dim3(nch, ct), dim3(NTH), 0, s, nr, nch, true,
                         pans[j].Vg, pans[j].Twg, X, (long)p, rest);
      hipLaunchKernelGGL((apply_wy<true>), dim3(1, ct), dim3(NTH), 0, s, nr, nch, true,
                         pans[j].V2, pans[j].Tw2, X, (long)p, rest);
      hipLaunchKernelGGL(copy_rows, dim3(nb256((long)w * rest)), dim3(256), 0, s, w, rest, X,
                         (long)p, T + (long)c * ldt + c + w, ldt);
    }
    LYAP_HIP(hipGetLastError());
  }
  // U = Q_1 ... Q_k [I_kk; 0]
  hipLaunchKernelGGL(eye_block, dim3(nb256((long)n * kk)), dim3(256), 0, s, n, kk, U, ldu);
  for (int j = npan - 1; j >= 0; --j) {
    const int c = j * PB, nr = n - c, nch = ceil_div(nr, CH);
    const int cols = kk - c;
    const unsigned ct = (unsigned)ceil_div(cols, PB);
    double* X = U + (long)c * ldu + c;
    hipLaunchKernelGGL((apply_wy<true>), dim3(1, ct), dim3(NTH), 0, s, nr, nch, false,
                       pans[j].V2, pans[j].Tw2, X, ldu, cols);
    hipLaunchKernelGGL((apply_wy<false>), dim3(nch, ct), dim3(NTH), 0, s, nr, nch, false,
                       pans[j].Vg, pans[j].Twg, X, ldu, cols);
    LYAP_HIP(hipGetLastError());
  }
  if (kt) {
    // Householder factorisation 2 n k^2 - 2 k^3 / 3 and the same again to form U (k = kk)
    LYAP_TRY(kt->mark(s, &e1));
    const double k = kk;
    kt->add(e0, e1, 2, 4.0 * n * k * k - 4.0 * k * k * k / 3.0, 1);
  }
  return LYAP_OK;
}

namespace {

// G <- G - Z (Z^T G) for the n x c orthonormal Z and the n x g block G (leading dimension g),
// with the c x g coefficients in CG (split-K partial products in part).
int project_off(hipStream_t s, int n, int c, int g, const double* Z, long ldz, double* G,
                double* CG, double* part, size_t kws) {
  GemmDesc a;  // CG = Z^T G
  a.M = c; a.N = g; a.K = n;
  a.A = Z; a.sar = 1; a.sac = ldz;
  a.B = G; a.sbr = g; a.sbc = 1;
  a.C = CG; a.ldc = g;
  GemmDesc b;  // G -= Z CG
  b.M = n; b.N = g; b.K = c;
  b.alpha = -1.0; b.beta = 1.0;
  b.A = Z; b.sar = ldz; b.sac = 1;
  b.B = CG; b.sbr = g; b.sbc = 1;
  b.C = G; b.ldc = g;
  LYAP_TRY(gemm_f64(s, a, part, kws));
  return gemm_f64(s, b);
}

// F = [Z, Y] with more columns than rows (p > n) whose first c columns Z are orthonormal:
// the columns span the whole space, so any orthonormal basis U of it gives F = U T with
// T = U^T F.  U = [Z, Q2] completes Z with Q2, the orthonormal factor of a seeded random
// n x (n - c) block projected off range(Z) (two Gram-Schmidt passes, a Householder QR, then
// one more projection and QR so that Q2 is orthogonal to Z to working precision whatever the
// conditioning of the random block), and T = [[I, Z^T Y], [0, Q2^T Y]].  Keeping Z as the
// leading block keeps T's leading block the identity (the Jacobi iterations that follow start
// from a nearly diagonal leading block), and the Householder work is that of n - c columns
// instead of an n x p QR.  T is n x p (not triangular; the callers only form products with
// it).
int qr_complete(hipStream_t s, int n, int p, int c, const double* F, long ldf, double* U,
                long ldu, double* T, long ldt, Arena& ws, KernTimer* kt) {
  const int g = n - c, q = p - c;
  if (g > 0) {
    double* G = ws.take<double>((size_t)n * g);
    double* CG = ws.take<double>((size_t)c * g);
    const size_t kws = std::min((size_t)8 * c * g, (size_t)4 << 20);
    double* part = ws.take<double>(kws);
    if (!G || !CG || !part) return LYAP_NO_MEMORY;
    // the R factors of the two QRs go to T's columns c .. c + g - 1 (g < q), which the last
    // product overwrites; the second QR reuses the first one's scratch
    double* Rg = T + c;
    hipLaunchKernelGGL(fill_uniform, dim3(nb256((long)n * g)), dim3(256), 0, s, n, g, G,
                       (long)g, 0x51a3c0d2e4f6b789ull + (unsigned long long)n);
    LYAP_HIP(hipGetLastError());
    LYAP_TRY(project_off(s, n, c, g, F, ldf, G, CG, part, kws));
    LYAP_TRY(project_off(s, n, c, g, F, ldf, G, CG, part, kws));
    const size_t mark = ws.top;
    LYAP_TRY(qr(s, n, g, G, g, U + c, ldu, Rg, ldt, ws, kt));
    ws.top = mark;
    hipLaunchKernelGGL(copy_rows, dim3(nb256((long)n * g)), dim3(256), 0, s, n, g, U + c, ldu,
                       G, (long)g);
    LYAP_HIP(hipGetLastError());
    LYAP_TRY(project_off(s, n, c, g, F, ldf, G, CG, part, kws));
    LYAP_TRY(qr(s, n, g, G, g, U + c, ldu, Rg, ldt, ws, kt));
  }
  LYAP_TRY(copy_block(s, n, c, F, ldf, U, ldu));
  GemmDesc t;  // T[:, c:p] = U^T Y
  t.M = n; t.N = q; t.K = n;
  t.A = U; t.sar = 1; t.sac = ldu;
  t.B = F + c; t.sbr = ldf; t.sbc = 1;
  t.C = T + c; t.ldc = ldt;
  LYAP_TRY(gemm_f64(s, t));
  hipLaunchKernelGGL(eye_block, dim3(nb256((long)n * c)), dim3(256), 0, s, n, c, T, ldt);
  LYAP_HIP(hipGetLastError());
  return LYAP_OK;
}

// Scratch qr_complete takes from the arena.
size_t complete_bytes(int n, int c) {
  const size_t g = (size_t)(n - c);
  return (n * g + c * g + std::min((size_t)8 * c * g, (size_t)4 << 20)) * 8 + 3 * 256 +
         qr_workspace_bytes(n, (int)g);
}

}  // namespace

// Thin QR of F = [Z, Y] whose first c columns Z are orthonormal: U = [Z, Q2] and
// T = [[I, C], [0, R2]] with C = Z^T Y from two block Gram-Schmidt passes (the second removes
// what rounding left of range(Z) in Y) and Q2 R2 the Householder QR above of Y - Z C.  The
// same factorisation F = U T as ``qr`` (U orthonormal, T upper triangular) with half the
// Householder work when c = p / 2.  Y (columns c.. of F) is overwritten.
int qr_lead(hipStream_t s, int n, int p, int c, double* F, long ldf, double* U, long ldu,
            double* T, long ldt, Arena& ws, KernTimer* kt, bool complete) {
  if (complete && p > n && c >= PB && c <= n && complete_bytes(n, c) + ws.top <= ws.cap)
    return qr_complete(s, n, p, c, F, ldf, U, ldu, T, ldt, ws, kt);
  if (c < PB || c >= p || p > n) return qr(s, n, p, F, ldf, U, ldu, T, ldt, ws, kt);
  const int q = p - c;
  double* Y = F + c;
  double* C = T + c;  // T[0:c, c:p]
  double* C2 = ws.take<double>((size_t)c * q);
  const size_t kws = std::min((size_t)8 * c * q, (size_t)4 << 20);
  double* part = ws.take<double>(kws);
  if (!C2 || !part) return LYAP_NO_MEMORY;
  GemmDesc g;  // C <- Z^T Y
  g.M = c; g.N = q; g.K = n;
  g.A = F; g.sar = 1; g.sac = ldf;
  g.B = Y; g.sbr = ldf; g.sbc = 1;
  g.C = C; g.ldc = ldt;
  GemmDesc u;  // Y <- Y - Z C
  u.M = n; u.N = q; u.K = c;
  u.alpha = -1.0; u.beta = 1.0;
  u.A = F; u.sar = ldf; u.sac = 1;
  u.B = C; u.sbr = ldt; u.sbc = 1;
  u.C = Y; u.ldc = ldf;
  LYAP_TRY(gemm_f64(s, g, part, kws));
  LYAP_TRY(gemm_f64(s, u));
  g.C = C2; g.ldc = q;
  u.B = C2; u.sbr = q;
  LYAP_TRY(gemm_f64(s, g, part, kws));
  LYAP_TRY(gemm_f64(s, u));
  hipLaunchKernelGGL(add_block, dim3(nb256((long)c * q)), dim3(256), 0, s, c, q, C2, (long)q, C,
                     ldt);
  LYAP_HIP(hipGetLastError());
  LYAP_TRY(qr(s, n, q, Y, ldf, U + c, ldu, T + (long)c * ldt + c, ldt, ws, kt));
  LYAP_TRY(copy_block(s, n, c, F, ldf, U, ldu));
  hipLaunchKernelGGL(eye_block, dim3(nb256((long)c * c)), dim3(256), 0, s, c, c, T, ldt);
  hipLaunchKernelGGL(zero_block, dim3(nb256((long)q * c)), dim3(256), 0, s, q, c,
                     T + (long)c * ldt, ldt);
  LYAP_HIP(hipGetLastError());
  return LYAP_OK;
}

}  // namespace lyap
