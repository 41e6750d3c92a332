// Symmetric spectral decomposition H = V diag(w) V^T (the spectral decompositions of
// Fragments 2.1-2.4 and of RankTruncLdlt in Alg 3.2): two-sided cyclic block Jacobi, in FP64
// (or FP32 rotations on request; H, w and V stay FP64).
//
// The matrix (padded to a multiple of 32 with zero rows/columns, which stay decoupled) is cut
// into nb blocks of 16 indices.  A sweep visits every pair of blocks once in nb rounds of
// nb / 2 disjoint pairs, in the modulus ordering: round t takes the pairs (i, j), i < j, with
// i + j = t mod nb.  That sequence is the row-cyclic ordering of the block pairs with only
// disjoint pairs exchanged, so it performs the same rotations as row-cyclic Jacobi, which on
// the graded matrices met here needs far fewer sweeps than a round-robin tournament.  Round t
// computes, for each of its pairs, a 32 x 32 orthogonal R_p from Jacobi rotations of the
// pair's subproblem in LDS, and then A <- G^T A G, V <- V G with G the block-diagonal (in pair
// order) of the R_p: block (p, q) of A becomes R_p^T A_pq R_q (FP64 matrix cores).  In the
// first two rounds of a sweep (between them every block takes part) the subproblems get a
// full cyclic sweep (every pair of their 32 indices, including the pairs inside a block);
// later rounds rotate only the 16 x 16 pairs across the two blocks (16 steps instead of 31).
//
// One kernel per round, with A ping-ponged between two buffers: its first workgroups solve the
// subproblems of round r + 1 while the others (persistent workers) apply round r.  The
// subproblem of a round-(r+1) pair is formed directly from the matrix before round r and round
// r's rotations (each of its four 16 x 16 blocks is a slice of R_P^T A_PQ R_Q), so the solves
// do not wait for the update.  A is kept as its upper triangle of 16 x 16 blocks (a block
// below the diagonal is read as the transpose of its mirror), so a round updates the pair
// blocks P <= Q only.
//
// Rotations are skipped when |a_pq| is below an absolute floor (tol ||A||_F / (4 pp)) or, when
// the caller asks for eigenvalues accurate relative to their own size, below
// tol sqrt(|a_pp a_qq|).  Sweeps stop when ||offdiag(A)||_F <= tol ||A||_F or when the solves
// of a whole sweep applied no rotation.  Eigenvalues are then sorted by descending magnitude
// (ties by index) and the eigenvectors gathered accordingly.
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

// Reciprocal and reciprocal square root from the hardware estimates refined by Newton steps
// (each step roughly doubles the number of correct bits of the estimate; the FP64 estimates
// are good to about 2^-24, one step to about 2e-15, two to full precision).
__device__ inline double recip(double x) {
  double r = __builtin_amdgcn_rcp(x);
  double e = fma(-x, r, 1.0);
  r = fma(r, e, r);
  e = fma(-x, r, 1.0);
  return fma(r, e, r);
}
__device__ inline double recip1(double x) {  // one step
  const double r = __builtin_amdgcn_rcp(x);
  return fma(r, fma(-x, r, 1.0), r);
}
__device__ inline double rsqrt1(double x) {
  const double y = __builtin_amdgcn_rsq(x);
  const double h = 0.5 * x * y;
  return fma(y, fma(-h, y, 0.5), y);
}
__device__ inline double rsqrt_nr(double x) {
  double y = __builtin_amdgcn_rsq(x);
  double h = 0.5 * x * y;  // Newton step y <- y (3 - x y^2) / 2, twice
  y = fma(y, fma(-h, y, 0.5), y);
  h = 0.5 * x * y;
  return fma(y, fma(-h, y, 0.5), y);
}
// FP32: one Newton step on the hardware estimate
__device__ inline float recip(float x) {
  const float r = __builtin_amdgcn_rcpf(x);
  return fmaf(r, fmaf(-x, r, 1.0f), r);
}
__device__ inline float rsqrt_nr(float x) {
  const float y = __builtin_amdgcn_rsqf(x);
  const float h = 0.5f * x * y;
  return fmaf(y, fmaf(-h, y, 0.5f), y);
}
__device__ inline float recip1(float x) { return recip(x); }
__device__ inline float rsqrt1(float x) { return rsqrt_nr(x); }

// Rotation zeroing a_pq of the 2 x 2 block [[app, apq], [apq, aqq]], or none (c = 1, s = 0)
// when |a_pq| <= thr or |a_pq| <= eps sqrt(|a_pp a_qq|); returns whether it is applied.
// t = tan(angle) is the smaller root of t^2 + 2 theta t - 1 = 0, c = 1 / sqrt(1 + t^2).
// An error in t only leaves a slightly larger remainder of a_pq, so t takes one refinement
// step; c and s = t c must satisfy c^2 + s^2 = 1 to working precision, so c takes two.
template <class T>
__device__ inline bool rot_params(T app, T aqq, T apq, T thr, T eps, T& c, T& s) {
  const T a = fabs(apq);
  if (a <= thr || a * a <= eps * eps * fabs(app * aqq)) {
    c = T(1);
    s = T(0);
    return false;
  }
  const T theta = (aqq - app) * recip1(T(2) * apq);
  const T at = fabs(theta);
  const T big = sizeof(T) == 8 ? T(1e150) : T(1e18);  // theta^2 would overflow
  T t;
  if (at > big) {
    t = T(0.5) * recip1(theta);
  } else {
    const T q = T(1) + theta * theta;
    const T h = q * rsqrt1(q);  // sqrt(1 + theta^2)
    t = copysign(recip1(at + h), theta);
  }
  c = rsqrt_nr(T(1) + t * t);
  s = t * c;
  return true;
}

// Element at slot k in round r of a circle-method tournament on m slots (m even): slot 0
// fixed, the others rotate.
__device__ inline int circle_elem(int slot, int r, int m) {
  if (slot == 0) return 0;
  return 1 + (slot - 1 + r) % (m - 1);
}

// 16 x 16 x 4 matrix-core products.  A operand: lane l holds A[l % 16][l / 16]; B operand:
// B[l / 16][l % 16]; result register i of lane l is row row(i, l / 16), column l % 16, which
// differs between the FP64 and FP32 instructions.
template <class T> struct Mf;
template <> struct Mf<double> {
  using V4 = f64x4;
  static __device__ V4 mma(double a, double b, V4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ int row(int i, int lk) { return 4 * i + lk; }
};
template <> struct Mf<float> {
  using V4 = f32x4;
  static __device__ V4 mma(float a, float b, V4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ int row(int i, int lk) { return 4 * lk + i; }
};

__device__ inline int gidx(int i, int bi, int bj) { return i < HB ? bi * HB + i : bj * HB + (i - HB); }

// A is kept as its upper triangle of 16 x 16 blocks (both triangles inside diagonal blocks):
// entry (r, c) lives at (r, c) when block(r) <= block(c), otherwise at (c, r).
__device__ inline long sidx(int r, int c, int pp) {
  return (r / HB <= c / HB) ? (long)r * pp + c : (long)c * pp + r;
}

// LDS of a round workgroup: 32 x 32 buffers, three in FP64 (six workgroups fit on a CU) and
// four in binary32.  A solve uses S[0..1] and R[0] for the sweep and, while it forms a binary32
// subproblem, S[1] / R[1] / R[0] as staging (X / RA / RB); an update workgroup uses S[1],
// S[0] and R[0] for its operands (M, RQ, RP).
template <class T>
struct SolveLds {
  T S[2][SB][LDS_PAD];  // subproblem, double-buffered by step parity
  // accumulated rotation, updated in place (a sweep step rotates its columns only, and each
  // entry belongs to one thread); binary32 subproblem formation stages a rotation in R[1].
  // Three FP64 buffers (25 KB) let six round workgroups share a CU.
  T R[sizeof(T) == 8 ? 1 : 2][SB][LDS_PAD];
  int any;
};

// Round and first-solve workgroups: 4 waves (the 2 x 2 block updates of a sweep step, the
// matrix-core tiles of the A and V update).
constexpr int NTJ = 256;

// Index pair k of step r of a subproblem sweep (p < q).  A full sweep (SB - 1 steps of the
// circle tournament on SB indices) rotates every pair of the subproblem once; a cross sweep
// (HB steps, pair k of step r = (k, HB + (k + r) mod HB)) rotates only the pairs with one
// index in each block.
__device__ inline void step_pair(bool full, int k, int r, int& p, int& q) {
  if (full) {
    p = circle_elem(k, r, SB);
    q = circle_elem(SB - 1 - k, r, SB);
    if (p > q) { const int x = p; p = q; q = x; }
  } else {
    p = k;
    q = HB + (k + r) % HB;
  }
}

// One sweep on L.S[0] (R starts as I in L.R[0]); returns the buffer of S holding the result
// (the parity of the step count; R ends in L.R[0]).  Thread t owns the 2 x 2 blocks (pair
// a = t / 16 rows, pair b = t % 16 columns) and computes the two rotations it applies itself
// (the same arithmetic on the same entries as any other thread that needs them, so no lane
// exchange); every thread reads the current S buffer and writes its block of the other one,
// and rotates its block of R in place, so a step needs a single barrier.
template <class T>
__device__ int subproblem_sweep(SolveLds<T>& L, T thr, T eps, bool full) {
  const int t = threadIdx.x;
  const int a = t / (SB / 2), b = t % (SB / 2);
  const int steps = full ? SB - 1 : HB;
  for (int r = 0; r < steps; ++r) {
    const int cur = r & 1, nxt = cur ^ 1;
    int p0, q0, p1, q1;
    step_pair(full, a, r, p0, q0);
    step_pair(full, b, r, p1, q1);
    T ca, sa, cb, sb;
    if (rot_params(L.S[cur][p0][p0], L.S[cur][q0][q0], L.S[cur][p0][q0], thr, eps, ca, sa) &&
        b == 0)
      L.any = 1;
    rot_params(L.S[cur][p1][p1], L.S[cur][q1][q1], L.S[cur][p1][q1], thr, eps, cb, sb);
    const T m00 = L.S[cur][p0][p1], m01 = L.S[cur][p0][q1];
    const T m10 = L.S[cur][q0][p1], m11 = L.S[cur][q0][q1];
    const T r00 = L.R[0][p0][p1], r01 = L.R[0][p0][q1];
    const T r10 = L.R[0][q0][p1], r11 = L.R[0][q0][q1];
    // G_a^T M G_b and R G_b
    const T x00 = ca * m00 - sa * m10, x01 = ca * m01 - sa * m11;
    const T x10 = sa * m00 + ca * m10, x11 = sa * m01 + ca * m11;
    L.S[nxt][p0][p1] = x00 * cb - x01 * sb;
    L.S[nxt][p0][q1] = x00 * sb + x01 * cb;
    L.S[nxt][q0][p1] = x10 * cb - x11 * sb;
    L.S[nxt][q0][q1] = x10 * sb + x11 * cb;
    L.R[0][p0][p1] = r00 * cb - r01 * sb;
    L.R[0][p0][q1] = r00 * sb + r01 * cb;
    L.R[0][q0][p1] = r10 * cb - r11 * sb;
    L.R[0][q0][q1] = r10 * sb + r11 * cb;
    __syncthreads();
  }
  return steps & 1;
}

// Solve workgroup for pair j = (bI, bJ) of ``pn``: form its subproblem, run one sweep, store
// the rotation to Rn[j].  With Rc == nullptr the subproblem is read from A directly; otherwise
// A is the matrix before the round whose pairs ``pc``, block map ``mc`` (block b sits in pair
// mc[b] / 2 at half mc[b] % 2) and rotations Rc are given.  The pair j == pseudo (the two
// blocks idle in a round) gets the identity.
template <class T>
__device__ void solve_pair(SolveLds<T>& L, int pp, int np, const T* __restrict__ A,
                           const int* __restrict__ pc, const int* __restrict__ mc,
                           const T* __restrict__ Rc, const int* __restrict__ pn, int j,
                           int pseudo, bool full, T thr, T eps, T* __restrict__ Rn,
                           int* __restrict__ applied) {
  const int t = threadIdx.x;
  if (j == pseudo) {
    T* Ro = Rn + (long)j * SB * SB;
    for (int e = t; e < SB * SB; e += NTJ) Ro[e] = (e / SB == e % SB) ? T(1) : T(0);
    return;
  }
  const int nI = pn[2 * j], nJ = pn[2 * j + 1];
  if (t == 0) L.any = 0;
  if (!Rc) {
    for (int e = t; e < SB * SB; e += NTJ) {
      const int i = e / SB, k = e % SB;
      L.S[0][i][k] = A[sidx(gidx(i, nI, nJ), gidx(k, nI, nJ), pp)];
    }
  } else {
    // block b of the new pair sits in current pair P(b) at half H(b)
    int P[2], H[2];
    for (int h = 0; h < 2; ++h) {
      const int e = mc[h == 0 ? nI : nJ];
      P[h] = e >> 1;
      H[h] = e & 1;
    }
    int bi[2], bj[2];
    for (int h = 0; h < 2; ++h) {
      bi[h] = pc[2 * P[h]];
      bj[h] = pc[2 * P[h] + 1];
    }
    if constexpr (sizeof(T) == 8) {
      // FP64: wave w forms block (h1, h2) = (w / 2, w % 2) on the matrix cores,
      // S_h1h2 = R_P[h1][:, half H[h1]]^T (X R_P[h2][:, half H[h2]]) with X the 32 x 32
      // block of A; the operands come straight from memory and Y = X R stays in registers
      // (the FP64 result layout, row 4 i + l / 16, is the next product's B-operand layout).
      const int lane = t & 63, wave = t >> 6, lr = lane & 15, lk = lane >> 4;
      const int h1 = wave >> 1, h2 = wave & 1;
      const T* R1 = Rc + (long)P[h1] * SB * SB + HB * H[h1];
      const T* R2 = Rc + (long)P[h2] * SB * SB + HB * H[h2];
      typename Mf<T>::V4 y0 = {T(0), T(0), T(0), T(0)}, y1 = y0, sb = y0;
      const int r0 = gidx(lr, bi[h1], bj[h1]);       // X row lr
      const int r1 = gidx(HB + lr, bi[h1], bj[h1]);  // X row 16 + lr
#pragma unroll
      for (int k0 = 0; k0 < SB; k0 += 4) {
        const int col = gidx(k0 + lk, bi[h2], bj[h2]);
        const T rk = R2[(k0 + lk) * SB + lr];
        y0 = Mf<T>::mma(A[sidx(r0, col, pp)], rk, y0);
        y1 = Mf<T>::mma(A[sidx(r1, col, pp)], rk, y1);
      }
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        sb = Mf<T>::mma(R1[(4 * i + lk) * SB + lr], y0[i], sb);
        sb = Mf<T>::mma(R1[(HB + 4 * i + lk) * SB + lr], y1[i], sb);
      }
#pragma unroll
      for (int i = 0; i < 4; ++i) L.S[0][HB * h1 + 4 * i + lk][HB * h2 + lr] = sb[i];
    } else {
      T (&X)[SB][LDS_PAD] = L.S[1];
      T (&RA)[SB][LDS_PAD] = L.R[1];
      T (&RB)[SB][LDS_PAD] = L.R[0];
      // all four blocks of the current matrix and both rotations, loaded at once (thread t
      // owns elements t + 256 q)
      T xr[4][4], ra[4], rb[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int e = t + NTJ * q, i = e / SB, k = e % SB;
        ra[q] = Rc[(long)P[0] * SB * SB + e];
        rb[q] = Rc[(long)P[1] * SB * SB + e];
#pragma unroll
        for (int cmb = 0; cmb < 4; ++cmb) {
          const int h1 = cmb >> 1, h2 = cmb & 1;
          xr[cmb][q] = A[sidx(gidx(i, bi[h1], bj[h1]), gidx(k, bi[h2], bj[h2]), pp)];
        }
      }
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int e = t + NTJ * q, i = e / SB, k = e % SB;
        RA[i][k] = ra[q];  // R_P[0]
        RB[i][k] = rb[q];  // R_P[1]
      }
#pragma unroll
      for (int cmb = 0; cmb < 4; ++cmb) {
        const int h1 = cmb >> 1, h2 = cmb & 1;
        __syncthreads();
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int e = t + NTJ * q;
          X[e / SB][e % SB] = xr[cmb][q];
        }
        __syncthreads();
        // Y = X R_P[h2][:, half H[h2]]  (32 x 16): thread (i = t / 8, columns 2 (t % 8) + {0, 1})
        T (&R2)[SB][LDS_PAD] = h2 == 0 ? RA : RB;
        T (&R1)[SB][LDS_PAD] = h1 == 0 ? RA : RB;
        const int yi = t / 8, yc = 2 * (t % 8);
        T y0 = T(0), y1 = T(0);
        // partial unrolling: fully unrolled, these two loops held their LDS operands in
        // registers and took the round kernel to 124 VGPRs (four waves per SIMD); at 8 it
        // needs under 64, which leaves room for eight binary32 round workgroups per CU
#pragma unroll 8
        for (int k = 0; k < SB; ++k) {
          const T x = X[yi][k];
          y0 += x * R2[k][HB * H[h2] + yc];
          y1 += x * R2[k][HB * H[h2] + yc + 1];
        }
        __syncthreads();
        X[yi][yc] = y0;  // X now holds Y in its first 16 columns
        X[yi][yc + 1] = y1;
        __syncthreads();
        // S block = R_P[h1][:, half H[h1]]^T Y  (16 x 16): thread (i = t / 16, c = t % 16)
        const int si = t / HB, sc = t % HB;
        T sum = T(0);
#pragma unroll 8
        for (int k = 0; k < SB; ++k) sum += R1[k][HB * H[h1] + si] * X[k][sc];
        L.S[0][HB * h1 + si][HB * h2 + sc] = sum;
      }
    }
    __syncthreads();  // RB (in R[0]) no longer read
  }
  for (int e = t; e < SB * SB; e += NTJ) {
    const int i = e / SB, k = e % SB;
    L.R[0][i][k] = (i == k) ? T(1) : T(0);
  }
  __syncthreads();
  subproblem_sweep(L, thr, eps, full);
  T* Ro = Rn + (long)j * SB * SB;
  for (int e = t; e < SB * SB; e += NTJ) Ro[e] = L.R[0][e / SB][e % SB];
  if (t == 0 && L.any) atomicAdd(applied, 1);
}

// First solve of the iteration (subproblems read from A).
template <class T>
__global__ __launch_bounds__(NTJ) void jac_solve0(int pp, int np, const T* __restrict__ A,
                                                  const int* __restrict__ pn, int pseudo,
                                                  const double* __restrict__ thr_dev, double eps,
                                                  T* __restrict__ Rn, int* __restrict__ applied) {
  __shared__ SolveLds<T> L;
  solve_pair<T>(L, pp, np, A, nullptr, nullptr, nullptr, pn, blockIdx.x, pseudo, true,
                (T)*thr_dev, (T)eps, Rn, applied);
}

// One round.  Blocks [0, np): solves of the next round's pairs pn (rotations to Rn; a full
// subproblem sweep when the next round is one of the first two of a sweep, a cross sweep
// otherwise).
// The other blocks are update workers that take items w, w + nw, w + 2 nw, ... of
//   items [0, na), na = np (np + 1) / 2: pair blocks P <= Q, Aout block (pair P rows, pair Q
//                 cols) = R_P^T Ain_PQ R_Q, stored into the upper block triangle,
//   items [na, na + np*nt): V tile (rows 32 t.., cols of pair Q) <- V_tile R_Q (in place),
// loading the operands of their next item into registers while they compute the current one.
// The block products run on the FP64 matrix cores: wave w owns the 16 x 16 tile (w/2, w%2).
struct Item {
  bool isA;
  int P, Q, tile;
};

// A items are the pair blocks with P <= Q in row order (row P starts at P np - P (P - 1) / 2).
__device__ inline int upper_start(int P, int np) { return P * np - P * (P - 1) / 2; }

__device__ inline Item decode_item(int item, int np) {
  Item it;
  const int na = np * (np + 1) / 2;
  it.isA = item < na;
  if (it.isA) {
    const double b = 2.0 * np + 1.0;
    int P = (int)((b - sqrt(b * b - 8.0 * item)) * 0.5);
    P = max(0, min(np - 1, P));
    while (P + 1 < np && upper_start(P + 1, np) <= item) ++P;
    while (P > 0 && upper_start(P, np) > item) --P;
    it.P = P;
    it.Q = P + (item - upper_start(P, np));
    it.tile = 0;
  } else {
    const int b2 = item - na;
    it.Q = b2 % np;
    it.tile = b2 / np;
    it.P = 0;
  }
  return it;
}

// thread t loads elements t + 256 q (q < 4) of the item's three 32 x 32 operands
template <class T>
__device__ inline void load_item(const Item& it, int pp, const int* __restrict__ pc,
                                 const T* __restrict__ Ain, const T* __restrict__ V,
                                 const T* __restrict__ Rc, T (&m)[4], T (&rq)[4], T (&rp)[4]) {
  const int t = threadIdx.x;
  const int qI = pc[2 * it.Q], qJ = pc[2 * it.Q + 1];
  const int pI = pc[2 * it.P], pJ = pc[2 * it.P + 1];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int e = t + NTJ * q, i = e / SB, j = e % SB;
    rq[q] = Rc[(long)it.Q * SB * SB + e];
    if (it.isA) {
      rp[q] = Rc[(long)it.P * SB * SB + e];
      m[q] = Ain[sidx(gidx(i, pI, pJ), gidx(j, qI, qJ), pp)];
    } else {
      m[q] = V[(long)(it.tile * SB + i) * pp + gidx(j, qI, qJ)];
    }
  }
}

template <class T>
__global__ __launch_bounds__(NTJ, sizeof(T) == 8 ? 5 : 1) void jac_round(int pp, int np, const T* __restrict__ Ain,
                                                 T* __restrict__ Aout, T* __restrict__ V,
                                                 const int* __restrict__ pc,
                                                 const int* __restrict__ mc,
                                                 const T* __restrict__ Rc,
                                                 const int* __restrict__ pn, int pseudo, int full,
                                                 T* __restrict__ Rn,
                                                 const double* __restrict__ thr_dev, double eps,
                                                 int* __restrict__ applied) {
  using M4 = Mf<T>;
  __shared__ SolveLds<T> L;
  const int blk = blockIdx.x;
  if (blk < np) {
    solve_pair<T>(L, pp, np, Ain, pc, mc, Rc, pn, blk, pseudo, full != 0, (T)*thr_dev, (T)eps,
                  Rn, applied);
    return;
  }
  const int nw = gridDim.x - np;
  const int nitems = np * (np + 1) / 2 + np * (pp / SB);
  int item = blk - np;
  if (item >= nitems) return;
  T (&M)[SB][LDS_PAD] = L.S[1];
  T (&RQ)[SB][LDS_PAD] = L.S[0];
  T (&RP)[SB][LDS_PAD] = L.R[0];
  T (&T1)[SB][LDS_PAD] = L.S[0];  // the first product's result replaces RQ
  const int t = threadIdx.x;
  const int lane = t & 63, wave = t >> 6;
  const int ti = wave >> 1, tj = wave & 1;
  const int lr = lane & 15, lk = lane >> 4;
  T m[4], rq[4], rp[4];
  Item it = decode_item(item, np);
  load_item<T>(it, pp, pc, Ain, V, Rc, m, rq, rp);
  while (true) {
    __syncthreads();  // the previous item's operands are no longer read
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int e = t + NTJ * q, i = e / SB, j = e % SB;
      M[i][j] = m[q];
      RQ[i][j] = rq[q];
      if (it.isA) RP[i][j] = rp[q];
    }
    __syncthreads();
    const Item cur = it;
    const int next = item + nw;
    if (next < nitems) {
      it = decode_item(next, np);
      load_item<T>(it, pp, pc, Ain, V, Rc, m, rq, rp);
    }
    const int qI = pc[2 * cur.Q], qJ = pc[2 * cur.Q + 1];
    typename M4::V4 acc = {T(0), T(0), T(0), T(0)};
#pragma unroll
    for (int k0 = 0; k0 < SB; k0 += 4)
      acc = M4::mma(M[16 * ti + lr][k0 + lk], RQ[k0 + lk][16 * tj + lr], acc);
    if (!cur.isA) {
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int r = 16 * ti + M4::row(i, lk), c = 16 * tj + lr;
        V[(long)(cur.tile * SB + r) * pp + gidx(c, qI, qJ)] = acc[i];
      }
    } else {
      const int pI = pc[2 * cur.P], pJ = pc[2 * cur.P + 1];
      __syncthreads();  // every wave has read RQ
#pragma unroll
      for (int i = 0; i < 4; ++i) T1[16 * ti + M4::row(i, lk)][16 * tj + lr] = acc[i];
      __syncthreads();
      typename M4::V4 out = {T(0), T(0), T(0), T(0)};
#pragma unroll
      for (int k0 = 0; k0 < SB; k0 += 4)
        out = M4::mma(RP[k0 + lk][16 * ti + lr], T1[k0 + lk][16 * tj + lr], out);
      // staged through M (free since the first product) so that each stored 16 x 16 block
      // is written row by row: block (h1, h2) of the result goes to (x, y) = (its row block,
      // its column block) when x <= y and transposed to (y, x) otherwise; for P == Q the
      // block (1, 0) is the transpose of (0, 1) and is not written
#pragma unroll
      for (int i = 0; i < 4; ++i) M[16 * ti + M4::row(i, lk)][16 * tj + lr] = out[i];
      __syncthreads();
#pragma unroll
      for (int h = 0; h < 4; ++h) {
        const int h1 = h >> 1, h2 = h & 1;
        if (cur.P == cur.Q && h1 == 1 && h2 == 0) continue;
        const int x = h1 ? pJ : pI, y = h2 ? qJ : qI;
        if (x <= y) {
          const int a = t / HB, b = t % HB;
          Aout[(long)(HB * x + a) * pp + HB * y + b] = M[HB * h1 + a][HB * h2 + b];
        } else {
          const int a = t % HB, b = t / HB;
          Aout[(long)(HB * y + b) * pp + HB * x + a] = M[HB * h1 + a][HB * h2 + b];
        }
      }
    }
    item = next;
    if (item >= nitems) break;
  }
}

template <class T>
__global__ void jac_load(int p, int pp, const double* __restrict__ H, long ldh,
                         T* __restrict__ A, T* __restrict__ V) {
  long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (long)pp * pp) return;
  int i = (int)(idx / pp), j = (int)(idx % pp);
  double v = 0.0;
  if (i < p && j < p) v = 0.5 * (H[(long)i * ldh + j] + H[(long)j * ldh + i]);
  A[idx] = (T)v;
  V[idx] = (i == j) ? T(1) : T(0);
}

// partial sums: [0] off-diagonal squares, [1] all squares (rows strided over blocks)
// (entries of the stored upper block triangle; an off-diagonal block counts twice)
template <class T>
__global__ void jac_norms(int pp, const T* __restrict__ A, double* __restrict__ part) {
  __shared__ double r0[256], r1[256];
  double off = 0.0, all = 0.0;
  for (int i = blockIdx.x; i < pp; i += gridDim.x)
    for (int j = threadIdx.x; j < pp; j += 256) {
      if (i / HB > j / HB) continue;
      const double v = (double)A[(long)i * pp + j];
      const double v2 = (i / HB == j / HB) ? v * v : 2.0 * v * v;
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
// rotation since the last call (the counter is reset); *thr_dev = thr_rel ||A||_F.
// One workgroup of 256 threads, fixed summation order.
__global__ void jac_norms_finish(int nparts, const double* __restrict__ part,
                                 double* __restrict__ out, double thr_rel,
                                 double* __restrict__ thr_dev, int* __restrict__ applied) {
  __shared__ double r0[256], r1[256];
  double off = 0.0, all = 0.0;
  for (int i = threadIdx.x; i < nparts; i += 256) {
    off += part[2 * i];
    all += part[2 * i + 1];
  }
  r0[threadIdx.x] = off;
  r1[threadIdx.x] = all;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (threadIdx.x < h) {
      r0[threadIdx.x] += r0[threadIdx.x + h];
      r1[threadIdx.x] += r1[threadIdx.x + h];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out[0] = r0[0];
    out[1] = r1[0];
    out[2] = (double)*applied;
    *applied = 0;
    *thr_dev = thr_rel * sqrt(r1[0]);
  }
}

// Sort the first p diagonal entries by descending |value| (ties by index): the rank of entry i
// is computed by counting; workgroup x ranks entries [256 x, 256 x + 256).
template <class T>
__global__ __launch_bounds__(256) void jac_sort(int p, int pp, const T* __restrict__ A,
                                                int* __restrict__ perm, double* __restrict__ w) {
  __shared__ double dg[4096];
  for (int i = threadIdx.x; i < p; i += 256) dg[i] = (double)A[(long)i * pp + i];
  __syncthreads();
  {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= p) return;
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

template <class T>
__global__ void jac_gather(int p, int pp, const T* __restrict__ Vw, const int* __restrict__ perm,
                           double* __restrict__ V, long ldv) {
  long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (long)p * p) return;
  int i = (int)(idx / p), k = (int)(idx % p);
  V[(long)i * ldv + k] = (double)Vw[(long)i * pp + perm[k]];
}

}  // namespace

// Block pair schedule (modulus ordering): round t rotates the block pairs (i, j), i < j,
// with i + j = t mod nb, listed by i.  Every pair appears once in the nb rounds of a sweep,
// and the sequence of rounds, sweep after sweep, is the row-cyclic sequence of pairs with
// only disjoint (commuting) pairs reordered, so it converges like the row-cyclic ordering.
// Even rounds leave blocks t / 2 and t / 2 + nb / 2 idle: they form the last pair of the
// round with the identity as rotation.  bmap[t][b] = 2 k + h for block b at half h of
// pair k of round t.
int jacobi_schedule(int nb, int* pairs, int* bmap) {
  if (nb < 2 || nb % 2 != 0 || !pairs || !bmap) return LYAP_BADARG;
  const int np = nb / 2;
  for (int r = 0; r < nb; ++r) {
    int* pr = pairs + (size_t)r * np * 2;
    int k = 0;
    for (int i = 0; i < nb; ++i) {
      const int j = (r - i + nb) % nb;
      if (j <= i) continue;
      pr[2 * k] = i;
      pr[2 * k + 1] = j;
      ++k;
    }
    if (r % 2 == 0) {
      pr[2 * k] = r / 2;
      pr[2 * k + 1] = r / 2 + np;
      ++k;
    }
    if (k != np) return LYAP_BADARG;  // not reached: every round holds np pairs
    for (k = 0; k < np; ++k)
      for (int h = 0; h < 2; ++h) bmap[(size_t)r * nb + pr[2 * k + h]] = 2 * k + h;
  }
  return LYAP_OK;
}

size_t syev_workspace_bytes(int p) {
  size_t pp = (size_t)ceil_div(p, SB) * SB;
  size_t nb = pp / HB, np = nb / 2;
  size_t s = 0;
  s += 3 * align_up(pp * pp * 8, 256);
  s += 2 * align_up(np * SB * SB * 8, 256);
  s += align_up(nb * np * 2 * 4 + 8, 256) + align_up(nb * nb * 4 + 8, 256);
  s += align_up(2 * 256 * 8, 256) + align_up(4 * 8, 256) + align_up(pp * 4, 256) + 256;
  return s + 4096;
}

namespace {

template <class T>
int syev_t(hipStream_t s, int p, const double* H, long ldh, double* w, double* V, long ldv,
           Arena& ws, double tol_rel, int* sweeps_out, KernTimer* kt, bool relative) {
  const int pp = ceil_div(p, SB) * SB;
  const int nb = pp / HB, np = nb / 2, rounds = nb;
  T* Aw[2] = {ws.take<T>((size_t)pp * pp), ws.take<T>((size_t)pp * pp)};
  T* Vw = ws.take<T>((size_t)pp * pp);
  T* Rb[2] = {ws.take<T>((size_t)np * SB * SB), ws.take<T>((size_t)np * SB * SB)};
  int* pairs = ws.take<int>((size_t)rounds * np * 2 + 2);
  int* bmap = ws.take<int>((size_t)rounds * nb + 2);
  double* part = ws.take<double>(2 * 256);  // nparts pairs
  double* scal = ws.take<double>(4);
  int* perm = ws.take<int>(pp);
  int* applied = ws.take<int>(1);
  if (!Aw[0] || !Aw[1] || !Vw || !Rb[0] || !Rb[1] || !pairs || !bmap || !part || !scal ||
      !perm || !applied)
    return LYAP_NO_MEMORY;
  if (tol_rel <= 0.0) tol_rel = 1e-15;
  const double eps = relative ? tol_rel : 0.0;
  std::vector<int> sched((size_t)rounds * np * 2), bm((size_t)rounds * nb);
  LYAP_TRY(jacobi_schedule(nb, sched.data(), bm.data()));
  LYAP_HIP(hipMemcpyAsync(pairs, sched.data(), sched.size() * sizeof(int), hipMemcpyHostToDevice,
                          s));
  LYAP_HIP(hipMemcpyAsync(bmap, bm.data(), bm.size() * sizeof(int), hipMemcpyHostToDevice, s));
  hipLaunchKernelGGL((jac_load<T>), dim3((unsigned)ceil_div(pp * pp, 256)), dim3(256), 0, s, p, pp, H,
                     ldh, Aw[0], Vw);
  const int nparts = 256;
  double* thr = scal + 3;
  hipLaunchKernelGGL((jac_norms<T>), dim3(nparts), dim3(256), 0, s, pp, Aw[0], part);
  const double thr_rel = 0.25 * tol_rel / pp;
  hipLaunchKernelGGL(jac_norms_finish, dim3(1), dim3(256), 0, s, nparts, part, scal, thr_rel, thr,
                     applied);
  LYAP_HIP(hipGetLastError());
  double host[3] = {0, 0, 0};
  int sweep = 0;
  const int max_sweeps = 40;
  LYAP_HIP(hipMemcpyAsync(host, scal, 3 * sizeof(double), hipMemcpyDeviceToHost, s));
  LYAP_HIP(hipStreamSynchronize(s));
  const double total = host[1];
  int cur = 0, rc = 0;  // A in Aw[cur], rotations of the next round in Rb[rc]
  bool solved = false;
  // update workers: about as many as fit on the chip next to the solves (6 round workgroups
  // per CU in FP64, bound by LDS; 8 in binary32, bound by registers)
  const int nitems = np * (np + 1) / 2 + np * (pp / SB);
  const int per_cu = sizeof(T) == 4 ? 8 : 6;
  const int nw = std::min(nitems, std::max(256, per_cu * 256 - np));
  while (sweep < max_sweeps && np > 0) {
    if (host[0] <= tol_rel * tol_rel * total) break;
    if (sweep > 0 && host[2] == 0.0) break;
    if (!solved) {
      hipLaunchKernelGGL((jac_solve0<T>), dim3(np), dim3(NTJ), 0, s, pp, np, Aw[cur], pairs,
                         np - 1, thr, eps, Rb[rc], applied);
      solved = true;
    }
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (kt) LYAP_TRY(kt->mark(s, &e0));
    for (int r = 0; r < rounds; ++r) {
      const int* pc = pairs + (size_t)r * np * 2;
      const int rn = (r + 1) % rounds;
      const int* pn = pairs + (size_t)rn * np * 2;
      hipLaunchKernelGGL((jac_round<T>), dim3(np + nw), dim3(NTJ), 0, s, pp, np,
                         Aw[cur], Aw[cur ^ 1], Vw, pc, bmap + (size_t)r * nb, Rb[rc], pn,
                         rn % 2 == 0 ? np - 1 : -1, rn <= 1 ? 1 : 0, Rb[rc ^ 1], thr, eps,
                         applied);
      cur ^= 1;
      rc ^= 1;
    }
    if (kt) {
      // block update traffic per round: the stored pair blocks P <= Q of A read and written,
      // V read and written
      LYAP_TRY(kt->mark(s, &e1));
      const double per_round = ((double)np * (np + 1) * SB * SB + 2.0 * pp * pp) * sizeof(T);
      kt->add(e0, e1, 1, rounds * per_round, rounds);
    }
    hipLaunchKernelGGL((jac_norms<T>), dim3(nparts), dim3(256), 0, s, pp, Aw[cur], part);
    hipLaunchKernelGGL(jac_norms_finish, dim3(1), dim3(256), 0, s, nparts, part, scal, thr_rel, thr,
                       applied);
    LYAP_HIP(hipGetLastError());
    LYAP_HIP(hipMemcpyAsync(host, scal, 3 * sizeof(double), hipMemcpyDeviceToHost, s));
    LYAP_HIP(hipStreamSynchronize(s));
    ++sweep;
  }
  if (sweeps_out) *sweeps_out = sweep;
  hipLaunchKernelGGL((jac_sort<T>), dim3((unsigned)ceil_div(p, 256)), dim3(256), 0, s, p, pp,
                     Aw[cur], perm, w);
  hipLaunchKernelGGL((jac_gather<T>), dim3((unsigned)ceil_div(p * p, 256)), dim3(256), 0, s, p, pp, Vw,
                     perm, V, ldv);
  LYAP_HIP(hipGetLastError());
  return LYAP_OK;
}

}  // namespace

int syev(hipStream_t s, int p, const double* H, long ldh, double* w, double* V, long ldv,
         Arena& ws, double tol_rel, int* sweeps_out, KernTimer* kt, bool relative, bool single) {
  if (p <= 0) return LYAP_OK;
  if (p > 4096) return LYAP_BADARG;
  if (single) return syev_t<float>(s, p, H, ldh, w, V, ldv, ws, tol_rel, sweeps_out, kt, relative);
  return syev_t<double>(s, p, H, ldh, w, V, ldv, ws, tol_rel, sweeps_out, kt, relative);
}

}  // namespace lyap
