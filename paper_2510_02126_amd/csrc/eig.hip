// Symmetric spectral decomposition H = V diag(w) V^T in FP64 (the spectral decompositions of
// Fragments 2.1-2.4 and of RankTruncLdlt in Alg 3.2): two-sided cyclic block Jacobi.
//
// The matrix (padded to a multiple of 32 with zero rows/columns, which stay decoupled) is cut
// into blocks of 16 indices.  A sweep visits every pair of blocks once in a round-robin
// tournament (nb - 1 rounds of nb / 2 disjoint pairs).  Per round:
//   jac_solve : one workgroup per pair runs cyclic Jacobi sweeps on its 32 x 32 diagonal
//               subproblem in LDS (16 disjoint rotations per inner step) and stores the
//               accumulated 32 x 32 rotation R_p;
//   jac_apply : A <- G^T A G and V <- V G, with G the block-diagonal (in pair order) of the
//               R_p; block (p, q) of A becomes R_p^T A_pq R_q, computed independently per
//               block by one workgroup, and each 32 x 32 tile of V is multiplied by R_q.
// Sweeps repeat until ||offdiag(A)||_F <= tol ||A||_F.  Eigenvalues are then sorted by
// descending magnitude (ties by index) and the eigenvectors gathered accordingly.
#include <algorithm>
#include <cmath>
#include <vector>

#include "common.hpp"
#include "internal.hpp"

namespace lyap {
namespace {

constexpr int HB = 16;        // block size (indices per block)
constexpr int SB = 2 * HB;    // subproblem size
constexpr int LDS_PAD = SB + 1;

__device__ inline void rot_params(double app, double aqq, double apq, double thr, double& c,
                                  double& s) {
  if (fabs(apq) <= thr) {
    c = 1.0;
    s = 0.0;
    return;
  }
  double theta = (aqq - app) / (2.0 * apq);
  double t;
  if (fabs(theta) > 1e150) t = 0.5 / theta;
  else t = (theta >= 0.0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(1.0 + theta * theta));
  c = 1.0 / sqrt(1.0 + t * t);
  s = t * c;
}

// Index of the partner of position k in round r of a circle-method tournament on m slots
// (m even): slot 0 fixed, the others rotate.  Returns the element at slot k.
__device__ inline int circle_elem(int slot, int r, int m) {
  if (slot == 0) return 0;
  return 1 + (slot - 1 + r) % (m - 1);
}

// One workgroup (256 threads) per pair: cyclic Jacobi on the 32 x 32 subproblem.
__global__ __launch_bounds__(256) void jac_solve(int pp, const double* __restrict__ A,
                                                 const int* __restrict__ pairs, int inner_sweeps,
                                                 const double* __restrict__ thr_dev,
                                                 double* __restrict__ Rout) {
  __shared__ double S[SB][LDS_PAD];
  __shared__ double R[SB][LDS_PAD];
  __shared__ double cs[SB / 2][2];
  __shared__ int idx[SB / 2][2];
  const int pair = blockIdx.x;
  const int bI = pairs[2 * pair], bJ = pairs[2 * pair + 1];
  const double thr = *thr_dev;
  for (int e = threadIdx.x; e < SB * SB; e += 256) {
    int i = e / SB, j = e % SB;
    int gi = (i < HB ? bI * HB + i : bJ * HB + (i - HB));
    int gj = (j < HB ? bI * HB + j : bJ * HB + (j - HB));
    S[i][j] = A[(long)gi * pp + gj];
    R[i][j] = (i == j) ? 1.0 : 0.0;
  }
  __syncthreads();
  const int a = threadIdx.x / (SB / 2), b = threadIdx.x % (SB / 2);  // 16 x 16 grid of 2x2 blocks
  for (int sw = 0; sw < inner_sweeps; ++sw) {
    for (int r = 0; r < SB - 1; ++r) {
      if (threadIdx.x < SB / 2) {
        int k = threadIdx.x;
        int p = circle_elem(k, r, SB), q = circle_elem(SB - 1 - k, r, SB);
        if (p > q) { int t = p; p = q; q = t; }
        double c, s;
        rot_params(S[p][p], S[q][q], S[p][q], thr, c, s);
        cs[k][0] = c;
        cs[k][1] = s;
        idx[k][0] = p;
        idx[k][1] = q;
      }
      __syncthreads();
      {
        const int p0 = idx[a][0], q0 = idx[a][1], p1 = idx[b][0], q1 = idx[b][1];
        const double ca = cs[a][0], sa = cs[a][1], cb = cs[b][0], sb = cs[b][1];
        double m00 = S[p0][p1], m01 = S[p0][q1], m10 = S[q0][p1], m11 = S[q0][q1];
        // G_a^T M
        double x00 = ca * m00 - sa * m10, x01 = ca * m01 - sa * m11;
        double x10 = sa * m00 + ca * m10, x11 = sa * m01 + ca * m11;
        // (G_a^T M) G_b
        double y00 = x00 * cb - x01 * sb, y01 = x00 * sb + x01 * cb;
        double y10 = x10 * cb - x11 * sb, y11 = x10 * sb + x11 * cb;
        // R <- R G_b on rows p0, q0 (thread a covers rows of pair a, columns of pair b)
        double r00 = R[p0][p1], r01 = R[p0][q1], r10 = R[q0][p1], r11 = R[q0][q1];
        __syncthreads();
        S[p0][p1] = y00; S[p0][q1] = y01; S[q0][p1] = y10; S[q0][q1] = y11;
        R[p0][p1] = r00 * cb - r01 * sb;
        R[p0][q1] = r00 * sb + r01 * cb;
        R[q0][p1] = r10 * cb - r11 * sb;
        R[q0][q1] = r10 * sb + r11 * cb;
      }
      __syncthreads();
    }
  }
  double* Ro = Rout + (long)pair * SB * SB;
  for (int e = threadIdx.x; e < SB * SB; e += 256) Ro[e] = R[e / SB][e % SB];
}

// Blocks [0, np*np): A block (pair P rows, pair Q cols) <- R_P^T A_PQ R_Q.
// Blocks [np*np, np*np + np*(pp/SB)): V tile (rows 32*t .., cols of pair Q) <- V_tile R_Q.
__global__ __launch_bounds__(256) void jac_apply(int pp, int np, double* __restrict__ A,
                                                 double* __restrict__ V,
                                                 const int* __restrict__ pairs,
                                                 const double* __restrict__ Rall) {
  __shared__ double M[SB][LDS_PAD];
  __shared__ double RQ[SB][LDS_PAD];
  __shared__ double RP[SB][LDS_PAD];
  __shared__ double T1[SB][LDS_PAD];
  const int blk = blockIdx.x;
  const bool isA = blk < np * np;
  int P, Q, tile = 0;
  if (isA) { P = blk / np; Q = blk % np; }
  else { int b2 = blk - np * np; Q = b2 % np; tile = b2 / np; P = 0; }
  const int qI = pairs[2 * Q], qJ = pairs[2 * Q + 1];
  const int pI = pairs[2 * P], pJ = pairs[2 * P + 1];
  auto gidx = [](int i, int bi, int bj) { return i < HB ? bi * HB + i : bj * HB + (i - HB); };
  const double* RQg = Rall + (long)Q * SB * SB;
  const double* RPg = Rall + (long)P * SB * SB;
  for (int e = threadIdx.x; e < SB * SB; e += 256) {
    int i = e / SB, j = e % SB;
    RQ[i][j] = RQg[e];
    if (isA) {
      RP[i][j] = RPg[e];
      M[i][j] = A[(long)gidx(i, pI, pJ) * pp + gidx(j, qI, qJ)];
    } else {
      M[i][j] = V[(long)(tile * SB + i) * pp + gidx(j, qI, qJ)];
    }
  }
  __syncthreads();
  // T1 = M R_Q
  for (int e = threadIdx.x; e < SB * SB; e += 256) {
    int i = e / SB, j = e % SB;
    double s = 0.0;
#pragma unroll 8
    for (int k = 0; k < SB; ++k) s += M[i][k] * RQ[k][j];
    T1[i][j] = s;
  }
  __syncthreads();
  if (isA) {
    for (int e = threadIdx.x; e < SB * SB; e += 256) {
      int i = e / SB, j = e % SB;
      double s = 0.0;
#pragma unroll 8
      for (int k = 0; k < SB; ++k) s += RP[k][i] * T1[k][j];
      A[(long)gidx(i, pI, pJ) * pp + gidx(j, qI, qJ)] = s;
    }
  } else {
    for (int e = threadIdx.x; e < SB * SB; e += 256) {
      int i = e / SB, j = e % SB;
      V[(long)(tile * SB + i) * pp + gidx(j, qI, qJ)] = T1[i][j];
    }
  }
}

__global__ void jac_load(int p, int pp, const double* __restrict__ H, long ldh,
                         double* __restrict__ A, double* __restrict__ V) {
  long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (long)pp * pp) return;
  int i = (int)(idx / pp), j = (int)(idx % pp);
  double v = 0.0;
  if (i < p && j < p) v = 0.5 * (H[(long)i * ldh + j] + H[(long)j * ldh + i]);
  A[idx] = v;
  V[idx] = (i == j) ? 1.0 : 0.0;
}

// partial sums: [0] off-diagonal squares, [1] all squares
__global__ void jac_norms(int pp, const double* __restrict__ A, double* __restrict__ part) {
  __shared__ double r0[256], r1[256];
  double off = 0.0, all = 0.0;
  long total = (long)pp * pp;
  for (long e = (long)blockIdx.x * 256 + threadIdx.x; e < total; e += (long)gridDim.x * 256) {
    int i = (int)(e / pp), j = (int)(e % pp);
    double v = A[e];
    double v2 = v * v;
    all += v2;
    if (i != j) off += v2;
  }
  r0[threadIdx.x] = off;
  r1[threadIdx.x] = all;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) {
      r0[threadIdx.x] += r0[threadIdx.x + s];
      r1[threadIdx.x] += r1[threadIdx.x + s];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = r0[0];
    part[2 * blockIdx.x + 1] = r1[0];
  }
}

__global__ void jac_norms_finish(int nparts, const double* __restrict__ part,
                                 double* __restrict__ out, double thr_rel,
                                 double* __restrict__ thr_dev) {
  double off = 0.0, all = 0.0;
  for (int i = 0; i < nparts; ++i) {
    off += part[2 * i];
    all += part[2 * i + 1];
  }
  out[0] = off;
  out[1] = all;
  *thr_dev = thr_rel * sqrt(all);
}

// Sort the first p diagonal entries by descending |value| (ties by index) and gather the
// eigenvectors: one workgroup, rank computed by counting.
__global__ __launch_bounds__(1024) void jac_sort(int p, int pp, const double* __restrict__ A,
                                                 int* __restrict__ perm, double* __restrict__ w) {
  __shared__ double dg[4096];
  for (int i = threadIdx.x; i < p; i += 1024) dg[i] = A[(long)i * pp + i];
  __syncthreads();
  for (int i = threadIdx.x; i < p; i += 1024) {
    double ai = dg[i], ki = fabs(ai);
    int rank = 0;
    for (int j = 0; j < p; ++j) {
      double kj = fabs(dg[j]);
      if (kj > ki || (kj == ki && j < i)) ++rank;
    }
    w[rank] = ai;
    perm[rank] = i;
  }
}

__global__ void jac_gather(int p, int pp, const double* __restrict__ Vw, const int* __restrict__ perm,
                           double* __restrict__ V, long ldv) {
  long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (long)p * p) return;
  int i = (int)(idx / p), k = (int)(idx % p);
  V[(long)i * ldv + k] = Vw[(long)i * pp + perm[k]];
}

}  // namespace

size_t syev_workspace_bytes(int p) {
  size_t pp = (size_t)ceil_div(p, SB) * SB;
  size_t nb = pp / HB, np = nb / 2;
  size_t s = 0;
  s += 2 * align_up(pp * pp * 8, 256);
  s += align_up(np * SB * SB * 8, 256);
  s += align_up((nb - 1) * np * 2 * 4 + 8, 256);
  s += align_up(2 * 256 * 8, 256) + align_up(4 * 8, 256) + align_up(pp * 4, 256);
  return s + 4096;
}

int syev(hipStream_t s, int p, const double* H, long ldh, double* w, double* V, long ldv,
         Arena& ws, double tol_rel, int* sweeps_out) {
  if (p <= 0) return LYAP_OK;
  if (p > 4096) return LYAP_BADARG;
  const int pp = ceil_div(p, SB) * SB;
  const int nb = pp / HB, np = nb / 2, rounds = nb - 1;
  double* Aw = ws.take<double>((size_t)pp * pp);
  double* Vw = ws.take<double>((size_t)pp * pp);
  double* Rall = ws.take<double>((size_t)np * SB * SB);
  int* pairs = ws.take<int>((size_t)rounds * np * 2 + 2);
  double* part = ws.take<double>(2 * 256);
  double* scal = ws.take<double>(4);
  int* perm = ws.take<int>(pp);
  if (!Aw || !Vw || !Rall || !pairs || !part || !scal || !perm) return LYAP_NO_MEMORY;
  if (tol_rel <= 0.0) tol_rel = 1e-15;
  // round-robin schedule of block pairs (host-computed, uploaded once)
  std::vector<int> sched((size_t)rounds * np * 2);
  for (int r = 0; r < rounds; ++r)
    for (int k = 0; k < np; ++k) {
      int a = (k == 0) ? 0 : 1 + (k - 1 + r) % (nb - 1);
      int kb = nb - 1 - k;
      int b = (kb == 0) ? 0 : 1 + (kb - 1 + r) % (nb - 1);
      sched[((size_t)r * np + k) * 2] = std::min(a, b);
      sched[((size_t)r * np + k) * 2 + 1] = std::max(a, b);
    }
  LYAP_HIP(hipMemcpyAsync(pairs, sched.data(), sched.size() * sizeof(int), hipMemcpyHostToDevice,
                          s));
  hipLaunchKernelGGL(jac_load, dim3((unsigned)ceil_div(pp * pp, 256)), dim3(256), 0, s, p, pp, H,
                     ldh, Aw, Vw);
  const int nparts = 64;
  double* thr = scal + 2;
  // rotations are skipped when the entry is below tol / (4 pp) * ||A||_F
  hipLaunchKernelGGL(jac_norms, dim3(nparts), dim3(256), 0, s, pp, Aw, part);
  const double thr_rel = 0.25 * tol_rel / pp;
  hipLaunchKernelGGL(jac_norms_finish, dim3(1), dim3(1), 0, s, nparts, part, scal, thr_rel, thr);
  LYAP_HIP(hipGetLastError());
  double host[2] = {0, 0};
  int sweep = 0;
  const int max_sweeps = 40;
  LYAP_HIP(hipMemcpyAsync(host, scal, 2 * sizeof(double), hipMemcpyDeviceToHost, s));
  LYAP_HIP(hipStreamSynchronize(s));
  const double total = host[1];
  double off = host[0];
  while (sweep < max_sweeps && off > tol_rel * tol_rel * total && np > 0) {
    for (int r = 0; r < rounds; ++r) {
      const int* pr = pairs + (size_t)r * np * 2;
      hipLaunchKernelGGL(jac_solve, dim3(np), dim3(256), 0, s, pp, Aw, pr, 1, thr, Rall);
      hipLaunchKernelGGL(jac_apply, dim3(np * np + np * (pp / SB)), dim3(256), 0, s, pp, np, Aw,
                         Vw, pr, Rall);
    }
    hipLaunchKernelGGL(jac_norms, dim3(nparts), dim3(256), 0, s, pp, Aw, part);
    hipLaunchKernelGGL(jac_norms_finish, dim3(1), dim3(1), 0, s, nparts, part, scal, thr_rel, thr);
    LYAP_HIP(hipGetLastError());
    LYAP_HIP(hipMemcpyAsync(host, scal, 2 * sizeof(double), hipMemcpyDeviceToHost, s));
    LYAP_HIP(hipStreamSynchronize(s));
    off = host[0];
    ++sweep;
  }
  if (sweeps_out) *sweeps_out = sweep;
  hipLaunchKernelGGL(jac_sort, dim3(1), dim3(1024), 0, s, p, pp, Aw, perm, w);
  hipLaunchKernelGGL(jac_gather, dim3((unsigned)ceil_div(p * p, 256)), dim3(256), 0, s, p, pp, Vw,
                     perm, V, ldv);
  LYAP_HIP(hipGetLastError());
  return LYAP_OK;
}

}  // namespace lyap
