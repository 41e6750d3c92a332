// Thin QR F = U T of an n x p FP64 matrix (U n x min(n,p) orthonormal, T upper trapezoidal) (the "thin QR decomposition" of
// Fragments 2.1-2.4 and of RankTruncLdlt in Alg 3.2), by Householder reflections only.
//
// Right-looking, panel by panel (32 columns).  Panel j covers columns [c, c+w) and rows
// [c, n) of the working copy.  Its orthogonal factor is a two-level tree of Householder
// reflectors (tall-skinny QR):
//   level 1  each 256-row chunk is factored in LDS (reflectors kept in global memory),
//   level 2  the stacked chunk R factors (<= 16 x 32 rows) are factored by one workgroup.
// The panel's transformation Q_j^T is then applied to the trailing columns (level-1
// reflectors per chunk, then level-2 reflectors on the stacked rows), which leaves the R
// rows of the panel in rows [c, c+w).  After the last panel, U = Q_1 ... Q_k [I_p; 0] is
// formed by applying the stored reflectors in reverse.  Because only reflectors are used,
// U is orthonormal to working precision even for numerically rank-deficient F (such as
// F = [Z, AZ, L] near convergence, where AZ lies almost in the span of Z and L).
#include <algorithm>
#include <cmath>

#include "common.hpp"
#include "internal.hpp"

namespace lyap {
namespace {

constexpr int PB = 32;     // panel width
constexpr int CH = 256;    // chunk rows at level 1
constexpr int NG = 8;      // row groups per workgroup (threads = NG * PB = 256)
constexpr int NTH = NG * PB;
constexpr int MAXCH = 16;  // chunks per panel (n <= 4096)

__device__ inline int first_row(int k0, int g) {  // smallest i >= k0 with i = g (mod NG)
  return k0 + ((g - k0) % NG + NG) % NG;
}

// Householder QR of an r x w block held in LDS (A[i * lda + j]), r <= 512, w <= 32.
// Reflector k: v = (1, A[k+1..r-1][k]) stored below the diagonal, tau[k]; R on and above.
// Thread (g, j) = (tid / PB, tid % PB) works on rows i = g (mod NG) of column j.
__device__ void lds_householder(double* A, int lda, int r, int w, double* tau, double* red) {
  const int tid = threadIdx.x, g = tid / PB, j = tid % PB;
  const int kmax = min(r, w);
  for (int k = 0; k < kmax; ++k) {
    double part = 0.0;
    if (j == 0)
      for (int i = first_row(k + 1, g); i < r; i += NG) {
        double x = A[i * lda + k];
        part += x * x;
      }
    if (j == 0) red[g] = part;
    __syncthreads();
    double sigma = 0.0;
    for (int q = 0; q < NG; ++q) sigma += red[q];
    const double alpha = A[k * lda + k];
    double beta, t, scale;
    if (sigma == 0.0) {
      beta = alpha;
      t = 0.0;
      scale = 0.0;
    } else {
      double nrm = sqrt(alpha * alpha + sigma);
      beta = alpha <= 0.0 ? nrm : -nrm;
      t = (beta - alpha) / beta;
      scale = 1.0 / (alpha - beta);
    }
    __syncthreads();
    for (int i = k + 1 + tid; i < r; i += NTH) A[i * lda + k] *= scale;
    if (tid == 0) {
      A[k * lda + k] = beta;
      tau[k] = t;
    }
    __syncthreads();
    double s = 0.0;
    if (j > k && j < w) {
      if (g == 0) s = A[k * lda + j];
      for (int i = first_row(k + 1, g); i < r; i += NG) s += A[i * lda + k] * A[i * lda + j];
    }
    red[NG + g * PB + j] = s;
    __syncthreads();
    if (j > k && j < w && t != 0.0) {
      double tot = 0.0;
      for (int q = 0; q < NG; ++q) tot += red[NG + q * PB + j];
      tot *= t;
      if (g == 0) A[k * lda + j] -= tot;
      for (int i = first_row(k + 1, g); i < r; i += NG) A[i * lda + j] -= tot * A[i * lda + k];
    }
    __syncthreads();
  }
}

// Apply the reflectors (V below the diagonal of an LDS block with leading dimension ldv,
// taus in LDS) to E (r x 32, thread (g, j) holds rows g + NG*q in registers).
// transpose = true: E <- H_{k-1} ... H_0 E (= Q^T E); false: E <- H_0 ... H_{k-1} E (= Q E).
template <int RPT>
__device__ void lds_apply(const double* V, int ldv, const double* tau, int r, int kmax,
                          bool transpose, double (&E)[RPT], double* red) {
  const int tid = threadIdx.x, g = tid / PB, j = tid % PB;
  for (int step = 0; step < kmax; ++step) {
    const int k = transpose ? step : kmax - 1 - step;
    const double t = tau[k];
    double s = 0.0;
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
      int i = g + NG * q;
      if (i < r && i >= k) s += (i == k ? 1.0 : V[i * ldv + k]) * E[q];
    }
    red[g * PB + j] = s;
    __syncthreads();
    double tot = 0.0;
    for (int q = 0; q < NG; ++q) tot += red[q * PB + j];
    tot *= t;
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
      int i = g + NG * q;
      if (i < r && i >= k) E[q] -= tot * (i == k ? 1.0 : V[i * ldv + k]);
    }
    __syncthreads();
  }
}

// Level 1: chunk b of the panel (rows [b*CH, b*CH + rows) of P, w columns).
__global__ __launch_bounds__(NTH) void tsqr_local(int n, int w, const double* __restrict__ P,
                                                  long ldp, double* __restrict__ Vg,
                                                  double* __restrict__ taug,
                                                  double* __restrict__ Rstack) {
  __shared__ double A[CH * (PB + 1)];
  __shared__ double tau[PB];
  __shared__ double red[NG + NG * PB];
  const int b = blockIdx.x, r0 = b * CH, rows = min(CH, n - r0);
  const int lda = PB + 1;
  for (int e = threadIdx.x; e < CH * PB; e += NTH) {
    int i = e / PB, j = e % PB;
    A[i * lda + j] = (i < rows && j < w) ? P[(long)(r0 + i) * ldp + j] : 0.0;
  }
  __syncthreads();
  lds_householder(A, lda, rows, w, tau, red);
  const int kmax = min(rows, w);
  for (int e = threadIdx.x; e < rows * PB; e += NTH) {
    int i = e / PB, j = e % PB;
    Vg[(long)(r0 + i) * PB + j] = (j < kmax && i > j) ? A[i * lda + j] : 0.0;
  }
  if (threadIdx.x < PB) taug[b * PB + threadIdx.x] = threadIdx.x < kmax ? tau[threadIdx.x] : 0.0;
  for (int e = threadIdx.x; e < PB * PB; e += NTH) {
    int i = e / PB, j = e % PB;
    Rstack[(long)(b * PB + i) * PB + j] = (i < rows && j >= i && j < w) ? A[i * lda + j] : 0.0;
  }
}

// Level 2: QR of the stacked R factors (nch*PB x w) by one workgroup; R (w x w) goes to T,
// the reflectors to V2 (nch*PB x PB) and tau2.
__global__ __launch_bounds__(NTH) void tsqr_stack(int nch, int w, const double* __restrict__ Rstack,
                                                  double* __restrict__ T, long ldt,
                                                  double* __restrict__ V2,
                                                  double* __restrict__ tau2) {
  __shared__ double A[MAXCH * PB * (PB + 1)];
  __shared__ double tau[PB];
  __shared__ double red[NG + NG * PB];
  const int r = nch * PB, lda = PB + 1;
  for (int e = threadIdx.x; e < r * PB; e += NTH) {
    int i = e / PB, j = e % PB;
    A[i * lda + j] = j < w ? Rstack[(long)i * PB + j] : 0.0;
  }
  __syncthreads();
  lds_householder(A, lda, r, w, tau, red);
  const int kmax = min(r, w);
  for (int e = threadIdx.x; e < w * w; e += NTH) {
    int i = e / w, j = e % w;
    T[(long)i * ldt + j] = j >= i ? A[i * lda + j] : 0.0;
  }
  for (int e = threadIdx.x; e < r * PB; e += NTH) {
    int i = e / PB, j = e % PB;
    V2[(long)i * PB + j] = (j < kmax && i > j) ? A[i * lda + j] : 0.0;
  }
  if (threadIdx.x < PB) tau2[threadIdx.x] = threadIdx.x < kmax ? tau[threadIdx.x] : 0.0;
}

// Apply the level-1 reflectors of every chunk to X (rows [0, n) of the panel's row range,
// ncols columns starting at X): grid (nch, ceil(ncols/32)).
__global__ __launch_bounds__(NTH) void apply_local(int n, int w, bool transpose,
                                                   const double* __restrict__ Vg,
                                                   const double* __restrict__ taug,
                                                   double* __restrict__ X, long ldx, int ncols) {
  __shared__ double V[CH * (PB + 1)];
  __shared__ double tau[PB];
  __shared__ double red[NG * PB];
  const int b = blockIdx.x, r0 = b * CH, rows = min(CH, n - r0), ldv = PB + 1;
  const int kmax = min(rows, w);
  const int c0 = blockIdx.y * PB;
  for (int e = threadIdx.x; e < CH * PB; e += NTH) {
    int i = e / PB, j = e % PB;
    V[i * ldv + j] = i < rows ? Vg[(long)(r0 + i) * PB + j] : 0.0;
  }
  if (threadIdx.x < PB) tau[threadIdx.x] = taug[b * PB + threadIdx.x];
  constexpr int RPT = CH / NG;
  double E[RPT];
  const int g = threadIdx.x / PB, j = threadIdx.x % PB;
  const bool colok = c0 + j < ncols;
#pragma unroll
  for (int q = 0; q < RPT; ++q) {
    int i = g + NG * q;
    E[q] = (i < rows && colok) ? X[(long)(r0 + i) * ldx + c0 + j] : 0.0;
  }
  __syncthreads();
  lds_apply<RPT>(V, ldv, tau, rows, kmax, transpose, E, red);
#pragma unroll
  for (int q = 0; q < RPT; ++q) {
    int i = g + NG * q;
    if (i < rows && colok) X[(long)(r0 + i) * ldx + c0 + j] = E[q];
  }
}

// Apply the level-2 reflectors to the stacked rows (top PB rows of each chunk) of X:
// grid ceil(ncols/32).
__global__ __launch_bounds__(NTH) void apply_stack(int n, int nch, int w, bool transpose,
                                                   const double* __restrict__ V2,
                                                   const double* __restrict__ tau2,
                                                   double* __restrict__ X, long ldx, int ncols) {
  __shared__ double V[MAXCH * PB * (PB + 1)];
  __shared__ double tau[PB];
  __shared__ double red[NG * PB];
  const int r = nch * PB, ldv = PB + 1;
  const int kmax = min(r, w);
  const int c0 = blockIdx.x * PB;
  for (int e = threadIdx.x; e < r * PB; e += NTH) {
    int i = e / PB, j = e % PB;
    V[i * ldv + j] = V2[(long)i * PB + j];
  }
  if (threadIdx.x < PB) tau[threadIdx.x] = tau2[threadIdx.x];
  constexpr int RPT = MAXCH * PB / NG;
  double E[RPT];
  const int g = threadIdx.x / PB, j = threadIdx.x % PB;
  const bool colok = c0 + j < ncols;
#pragma unroll
  for (int q = 0; q < RPT; ++q) {
    int i = g + NG * q;  // stack row: chunk i / PB, row i % PB of that chunk
    int row = (i / PB) * CH + (i % PB);
    E[q] = (i < r && row < n && colok) ? X[(long)row * ldx + c0 + j] : 0.0;
  }
  __syncthreads();
  lds_apply<RPT>(V, ldv, tau, r, kmax, transpose, E, red);
#pragma unroll
  for (int q = 0; q < RPT; ++q) {
    int i = g + NG * q;
    int row = (i / PB) * CH + (i % PB);
    if (i < r && row < n && colok) X[(long)row * ldx + c0 + j] = E[q];
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

inline unsigned nb256(long total) { return (unsigned)((total + 255) / 256); }

}  // namespace

size_t qr_workspace_bytes(int n, int p) {
  size_t npan = (size_t)ceil_div(std::min(n, p), PB);
  size_t s = 0;
  s += align_up((size_t)n * p * 8, 256);                       // working copy
  s += npan * align_up((size_t)n * PB * 8, 256);               // level-1 reflectors per panel
  s += npan * align_up((size_t)MAXCH * PB * 8, 256);           // level-1 taus
  s += npan * align_up((size_t)MAXCH * PB * PB * 8, 256);      // level-2 reflectors
  s += npan * align_up((size_t)PB * 8, 256);                   // level-2 taus
  s += align_up((size_t)MAXCH * PB * PB * 8, 256);             // stacked R factors
  return s + 4096;
}

int qr(hipStream_t s, int n, int p, const double* F, long ldf, double* U, long ldu, double* T,
       long ldt, Arena& ws) {
  if (p <= 0 || n <= 0) return LYAP_OK;
  if (n > MAXCH * CH) return LYAP_BADARG;
  const int kk = std::min(n, p);  // U is n x kk, T is kk x p (upper trapezoidal)
  const int npan = ceil_div(kk, PB);
  double* W = ws.take<double>((size_t)n * p);
  double* Rstack = ws.take<double>((size_t)MAXCH * PB * PB);
  if (!W || !Rstack) return LYAP_NO_MEMORY;
  struct Pan { double *Vg, *taug, *V2, *tau2; };
  Pan pans[4096 / PB];
  for (int j = 0; j < npan; ++j) {
    pans[j].Vg = ws.take<double>((size_t)n * PB);
    pans[j].taug = ws.take<double>((size_t)MAXCH * PB);
    pans[j].V2 = ws.take<double>((size_t)MAXCH * PB * PB);
    pans[j].tau2 = ws.take<double>(PB);
    if (!pans[j].Vg || !pans[j].taug || !pans[j].V2 || !pans[j].tau2) return LYAP_NO_MEMORY;
  }
  LYAP_TRY(copy_block(s, n, p, F, ldf, W, p));
  hipLaunchKernelGGL(zero_block, dim3(nb256((long)kk * p)), dim3(256), 0, s, kk, p, T, ldt);
  for (int j = 0; j < npan; ++j) {
    const int c = j * PB, w = std::min(PB, kk - c), nr = n - c, nch = ceil_div(nr, CH);
    double* P = W + (long)c * p + c;  // rows [c, n), columns [c, c+w)
    hipLaunchKernelGGL(tsqr_local, dim3(nch), dim3(NTH), 0, s, nr, w, P, (long)p, pans[j].Vg,
                       pans[j].taug, Rstack);
    hipLaunchKernelGGL(tsqr_stack, dim3(1), dim3(NTH), 0, s, nch, w, Rstack,
                       T + (long)c * ldt + c, ldt, pans[j].V2, pans[j].tau2);
    const int rest = p - c - w;
    if (rest > 0) {
      double* X = P + w;  // rows [c, n), columns [c+w, p)
      hipLaunchKernelGGL(apply_local, dim3(nch, ceil_div(rest, PB)), dim3(NTH), 0, s, nr, w, true,
                         pans[j].Vg, pans[j].taug, X, (long)p, rest);
      hipLaunchKernelGGL(apply_stack, dim3(ceil_div(rest, PB)), dim3(NTH), 0, s, nr, nch, w, true,
                         pans[j].V2, pans[j].tau2, X, (long)p, rest);
      hipLaunchKernelGGL(copy_rows, dim3(nb256((long)w * rest)), dim3(256), 0, s, w, rest, X,
                         (long)p, T + (long)c * ldt + c + w, ldt);
    }
    LYAP_HIP(hipGetLastError());
  }
  // U = Q_1 ... Q_k [I_kk; 0]
  hipLaunchKernelGGL(eye_block, dim3(nb256((long)n * kk)), dim3(256), 0, s, n, kk, U, ldu);
  for (int j = npan - 1; j >= 0; --j) {
    const int c = j * PB, w = std::min(PB, kk - c), nr = n - c, nch = ceil_div(nr, CH);
    const int cols = kk - c;
    double* X = U + (long)c * ldu + c;
    hipLaunchKernelGGL(apply_stack, dim3(ceil_div(cols, PB)), dim3(NTH), 0, s, nr, nch, w, false,
                       pans[j].V2, pans[j].tau2, X, ldu, cols);
    hipLaunchKernelGGL(apply_local, dim3(nch, ceil_div(cols, PB)), dim3(NTH), 0, s, nr, w, false,
                       pans[j].Vg, pans[j].taug, X, ldu, cols);
    LYAP_HIP(hipGetLastError());
  }
  return LYAP_OK;
}

}  // namespace lyap
