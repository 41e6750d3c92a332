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

// Rotation zeroing a_pq of the 2 x 2 block [[app, apq], [apq, aqq]].  The rotation is skipped
// (c = 1, s = 0) when |a_pq| <= thr (absolute floor) or |a_pq| <= eps sqrt(|a_pp a_qq|)
// (relative to the coupled diagonal entries); returns whether it is applied.
__device__ inline bool rot_params(double app, double aqq, double apq, double thr, double eps,
                                  double& c, double& s) {
  const double a = fabs(apq);
  if (a <= thr || a <= eps * sqrt(fabs(app) * fabs(aqq))) {
    c = 1.0;
    s = 0.0;
    return false;
  }
  double theta = (aqq - app) / (2.0 * apq);
  double t;
  if (fabs(theta) > 1e150) t = 0.5 / theta;
  else t = (theta >= 0.0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(1.0 + theta * theta));
  c = 1.0 / sqrt(1.0 + t * t);
  s = t * c;
  return true;
}

// Index of the partner of position k in round r of a circle-method tournament on m slots
// (m even): slot 0 fixed, the others rotate.  Returns the element at slot k.
__device__ inline int circle_elem(int slot, int r, int m) {
  if (slot == 0) return 0;
  return 1 + (slot - 1 + r) % (m - 1);
}

// One workgroup per pair: cyclic Jacobi on the 32 x 32 subproblem in LDS.  Each inner step
// applies 16 disjoint rotations G_a; thread t owns the 2 x 2 blocks (pair a = t / 16 rows,
// pair b = t % 16 columns) of S and R, which the step rewrites as G_a^T S_ab G_b and R_ab G_b.
// Each thread computes the parameters of G_a and G_b itself from the diagonal blocks, reads
// everything it needs, and writes only after a barrier (the diagonal blocks are owned by
// other threads).
__global__ __launch_bounds__(256) void jac_solve(int pp, const double* __restrict__ A,
                                                 const int* __restrict__ pairs, int inner_sweeps,
                                                 const double* __restrict__ thr_dev, double eps,
                                                 double* __restrict__ Rout,
                                                 int* __restrict__ applied) {
  __shared__ double S[SB][LDS_PAD];
  __shared__ double R[SB][LDS_PAD];
  __shared__ int any;
  const int pair = blockIdx.x, t = threadIdx.x;
  if (t == 0) any = 0;
  const int bI = pairs[2 * pair], bJ = pairs[2 * pair + 1];
  const double thr = *thr_dev;
  for (int e = t; e < SB * SB; e += 256) {
    const int i = e / SB, j = e % SB;
    const int gi = (i < HB ? bI * HB + i : bJ * HB + (i - HB));
    const int gj = (j < HB ? bI * HB + j : bJ * HB + (j - HB));
    S[i][j] = A[(long)gi * pp + gj];
    R[i][j] = (i == j) ? 1.0 : 0.0;
  }
  __syncthreads();
  const int a = t / (SB / 2), b = t % (SB / 2);
  for (int sw = 0; sw < inner_sweeps; ++sw) {
    for (int r = 0; r < SB - 1; ++r) {
      int p0 = circle_elem(a, r, SB), q0 = circle_elem(SB - 1 - a, r, SB);
      if (p0 > q0) { const int x = p0; p0 = q0; q0 = x; }
      int p1 = circle_elem(b, r, SB), q1 = circle_elem(SB - 1 - b, r, SB);
      if (p1 > q1) { const int x = p1; p1 = q1; q1 = x; }
      const double app = S[p0][p0], aqq = S[q0][q0], apq = S[p0][q0];
      const double bpp = S[p1][p1], bqq = S[q1][q1], bpq = S[p1][q1];
      const double m00 = S[p0][p1], m01 = S[p0][q1], m10 = S[q0][p1], m11 = S[q0][q1];
      const double r00 = R[p0][p1], r01 = R[p0][q1], r10 = R[q0][p1], r11 = R[q0][q1];
      double ca, sa, cb, sb;
      if (rot_params(app, aqq, apq, thr, eps, ca, sa) && b == 0) any = 1;
      rot_params(bpp, bqq, bpq, thr, eps, cb, sb);
      // G_a^T M, then (G_a^T M) G_b
      const double x00 = ca * m00 - sa * m10, x01 = ca * m01 - sa * m11;
      const double x10 = sa * m00 + ca * m10, x11 = sa * m01 + ca * m11;
      __syncthreads();
      S[p0][p1] = x00 * cb - x01 * sb;
      S[p0][q1] = x00 * sb + x01 * cb;
      S[q0][p1] = x10 * cb - x11 * sb;
      S[q0][q1] = x10 * sb + x11 * cb;
      R[p0][p1] = r00 * cb - r01 * sb;
      R[p0][q1] = r00 * sb + r01 * cb;
      R[q0][p1] = r10 * cb - r11 * sb;
      R[q0][q1] = r10 * sb + r11 * cb;
      __syncthreads();
    }
  }
  double* Ro = Rout + (long)pair * SB * SB;
  for (int e = t; e < SB * SB; e += 256) Ro[e] = R[e / SB][e % SB];
  if (t == 0 && any) atomicAdd(applied, 1);
}

// Blocks [0, np*np): A block (pair P rows, pair Q cols) <- R_P^T A_PQ R_Q.
// Blocks [np*np, np*np + np*(pp/SB)): V tile (rows 32*t .., cols of pair Q) <- V_tile R_Q.
// The 32 x 32 products run on the FP64 matrix cores (v_mfma_f64_16x16x4f64): wave w owns the
// 16 x 16 output tile (w / 2, w % 2); operands are staged in LDS.
__device__ inline f64x4 mfma_f64(double a, double b, f64x4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

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
    const int i = e / SB, j = e % SB;
    RQ[i][j] = RQg[e];
    if (isA) {
      RP[i][j] = RPg[e];
      M[i][j] = A[(long)gidx(i, pI, pJ) * pp + gidx(j, qI, qJ)];
    } else {
      M[i][j] = V[(long)(tile * SB + i) * pp + gidx(j, qI, qJ)];
    }
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int ti = wave >> 1, tj = wave & 1;
  const int lr = lane & 15, lk = lane >> 4;
  // T1 = M R_Q
  f64x4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int k0 = 0; k0 < SB; k0 += 4)
    acc = mfma_f64(M[16 * ti + lr][k0 + lk], RQ[k0 + lk][16 * tj + lr], acc);
  // D layout (FP64 16x16x4): lane l, register i -> row 4 i + l / 16, column l % 16
  if (!isA) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int r = 16 * ti + 4 * i + lk, c = 16 * tj + lr;
      V[(long)(tile * SB + r) * pp + gidx(c, qI, qJ)] = acc[i];
    }
    return;
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) T1[16 * ti + 4 * i + lk][16 * tj + lr] = acc[i];
  __syncthreads();
  // out = R_P^T T1
  f64x4 out = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int k0 = 0; k0 < SB; k0 += 4)
    out = mfma_f64(RP[k0 + lk][16 * ti + lr], T1[k0 + lk][16 * tj + lr], out);
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int r = 16 * ti + 4 * i + lk, c = 16 * tj + lr;
    A[(long)gidx(r, pI, pJ) * pp + gidx(c, qI, qJ)] = out[i];
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

// out[0] = ||offdiag||_F^2, out[1] = ||A||_F^2, out[2] = number of subproblems that applied a
// rotation since the last call (the counter is reset).
__global__ void jac_norms_finish(int nparts, const double* __restrict__ part,
                                 double* __restrict__ out, double thr_rel,
                                 double* __restrict__ thr_dev, int* __restrict__ applied) {
  double off = 0.0, all = 0.0;
  for (int i = 0; i < nparts; ++i) {
    off += part[2 * i];
    all += part[2 * i + 1];
  }
  out[0] = off;
  out[1] = all;
  out[2] = (double)*applied;
  *applied = 0;
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
  int* applied = ws.take<int>(1);
  if (!Aw || !Vw || !Rall || !pairs || !part || !scal || !perm || !applied) return LYAP_NO_MEMORY;
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
  double* thr = scal + 3;
  // rotations are skipped when the entry is below tol / (4 pp) * ||A||_F, or below
  // tol sqrt(|a_pp a_qq|)
  hipLaunchKernelGGL(jac_norms, dim3(nparts), dim3(256), 0, s, pp, Aw, part);
  const double thr_rel = 0.25 * tol_rel / pp;
  hipLaunchKernelGGL(jac_norms_finish, dim3(1), dim3(1), 0, s, nparts, part, scal, thr_rel, thr,
                     applied);
  LYAP_HIP(hipGetLastError());
  double host[3] = {0, 0, 0};
  int sweep = 0;
  const int max_sweeps = 40;
  LYAP_HIP(hipMemcpyAsync(host, scal, 3 * sizeof(double), hipMemcpyDeviceToHost, s));
  LYAP_HIP(hipStreamSynchronize(s));
  const double total = host[1];
  // Stop when ||offdiag||_F <= tol ||A||_F, or when a whole sweep found no entry worth a
  // rotation (every |a_pq| below both skip thresholds).
  while (sweep < max_sweeps && np > 0) {
    if (host[0] <= tol_rel * tol_rel * total) break;
    if (sweep > 0 && host[2] == 0.0) break;
    for (int r = 0; r < rounds; ++r) {
      const int* pr = pairs + (size_t)r * np * 2;
      hipLaunchKernelGGL(jac_solve, dim3(np), dim3(256), 0, s, pp, Aw, pr, 1, thr, tol_rel, Rall,
                         applied);
      hipLaunchKernelGGL(jac_apply, dim3(np * np + np * (pp / SB)), dim3(256), 0, s, pp, np, Aw,
                         Vw, pr, Rall);
    }
    hipLaunchKernelGGL(jac_norms, dim3(nparts), dim3(256), 0, s, pp, Aw, part);
    hipLaunchKernelGGL(jac_norms_finish, dim3(1), dim3(1), 0, s, nparts, part, scal, thr_rel, thr,
                       applied);
    LYAP_HIP(hipGetLastError());
    LYAP_HIP(hipMemcpyAsync(host, scal, 3 * sizeof(double), hipMemcpyDeviceToHost, s));
    LYAP_HIP(hipStreamSynchronize(s));
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
