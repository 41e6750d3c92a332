// Matrix-core products for gfx950.
//
// Kernel families:
//  * gemm_k4   -- 16x16x4 MFMA with one operand element per lane (FP64: v_mfma_f64_16x16x4f64,
//                 binary32: v_mfma_f32_16x16x4f32).  Block tile 64x64, k-tile 16, 4 waves in
//                 a 2x2 grid, each wave 32x32 (2x2 MFMA tiles).
//  * gemm_big  -- the same MFMA shapes on a 128x128 block tile with eight waves (2x4, each
//                 64x32), a double-buffered 128-byte k-slice in LDS and register prefetch of
//                 the next slice; chosen for products with enough tiles and a long k-loop.
//  * gemm_k32  -- 16x16x32 MFMA with eight operand elements per lane (fp16 / bf16 operands,
//                 binary32 accumulation).  Block tile 64x64, k-tile 32.
//  * gemm_k32s -- split fp16 operands x = hi + 2^-11 lo: three 16x16x32 MFMAs per step
//                 (hi*hi and the two cross terms) in binary32 accumulation.
// Operands are read through generic strides so that transposed views need no copies; the
// loader picks a coalesced thread mapping from whichever stride is unit.  Ragged M, N, K are
// zero-padded in LDS.  Products with few output tiles and a long k-loop (the tall-skinny
// products of the factor iterations and the Gram matrices) split K across blocks when the
// caller gives a workspace: each block writes its scaled partial product in FP64 and a
// deterministic second pass sums them in a fixed order (for reduced-precision operands the
// accumulation is binary32 within a k-chunk and FP64 across chunks).
#include <algorithm>
#include <type_traits>

#include "common.hpp"

namespace lyap {
namespace {

constexpr int BM = 64, BN = 64, NT = 256;

template <class T> __device__ inline double to_d(T x) { return (double)x; }
template <> __device__ inline double to_d<_Float16>(_Float16 x) { return (double)(float)x; }
template <> __device__ inline double to_d<__bf16>(__bf16 x) { return (double)(float)x; }

template <class D> struct Cvt;
template <> struct Cvt<double> {
  template <class S> __device__ static double f(S x) { return to_d(x); }
};
template <> struct Cvt<float> {
  __device__ static float f(double x) { return (float)x; }
  __device__ static float f(float x) { return x; }
  __device__ static float f(_Float16 x) { return (float)x; }
  __device__ static float f(__bf16 x) { return (float)x; }
};
template <> struct Cvt<_Float16> {
  __device__ static _Float16 f(double x) { return rne_from_f64<_Float16>(x); }
  __device__ static _Float16 f(float x) { return (_Float16)x; }
  __device__ static _Float16 f(_Float16 x) { return x; }
  __device__ static _Float16 f(__bf16 x) { return (_Float16)(float)x; }
};
template <> struct Cvt<__bf16> {
  __device__ static __bf16 f(double x) { return rne_from_f64<__bf16>(x); }
  __device__ static __bf16 f(float x) { return (__bf16)x; }
  __device__ static __bf16 f(_Float16 x) { return (__bf16)(float)x; }
  __device__ static __bf16 f(__bf16 x) { return x; }
};

// Operand element rounded to MF after an exact scaling by 2^-e (e = 0: plain rounding).
template <class MF, class S> __device__ inline MF cvt_scaled(S x, int e) {
  if (e == 0) return Cvt<MF>::f(x);
  return Cvt<MF>::f(ldexp(to_d(x), -e));
}

template <class MF> struct Acc;
template <> struct Acc<double> { typedef f64x4 V; typedef double S; };
template <> struct Acc<float> { typedef f32x4 V; typedef float S; };

__device__ inline f64x4 mfma4(double a, double b, f64x4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ inline f32x4 mfma4(float a, float b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

template <class TC, class S> __device__ inline void store_out(TC* p, S v) { *p = (TC)v; }

// ----------------------------------------------------------------------------- k4 kernel
// MF = double (FP64 matrix cores) or float (binary32 matrix cores).
template <class TA, class TB, class MF, class TC, bool AK, bool BN_>
__global__ __launch_bounds__(NT) void gemm_k4(int M, int N, int K, int kchunk, double alpha,
                                              double beta, const TA* __restrict__ A, long sar,
                                              long sac, const TB* __restrict__ B, long sbr,
                                              long sbc, TC* __restrict__ C, long ldc,
                                              TC* __restrict__ part,
                                              const int* __restrict__ aexp,
                                              const int* __restrict__ bexp) {
  constexpr int BK = 16;
  constexpr int PA = (BM * BK) / NT, PB = (BN * BK) / NT;
  typedef typename Acc<MF>::V AV;
  typedef typename Acc<MF>::S AS;
  // double-buffered k-tiles; the next tile is loaded into registers while the current one
  // feeds the matrix cores, so each k-step waits for the global loads at most once
  __shared__ MF As[2][BK][BM + 1];
  __shared__ MF Bs[2][BK][BN + 1];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int m0 = blockIdx.y * BM, n0 = blockIdx.x * BN;
  const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
  const int kbeg = blockIdx.z * kchunk;
  const int kend = min(K, kbeg + kchunk);
  AV acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = AV{0, 0, 0, 0};

  MF ra[PA], rb[PB];
  auto load = [&](int k0) {
#pragma unroll
    for (int r = 0; r < PA; ++r) {
      int e = tid + NT * r;
      int kk, mm;
      if (AK) { kk = e % BK; mm = e / BK; } else { mm = e % BM; kk = e / BM; }
      int gm = m0 + mm, gk = k0 + kk;
      ra[r] = (gm < M && gk < kend) ? Cvt<MF>::f(A[(long)gm * sar + (long)gk * sac]) : (MF)0;
    }
#pragma unroll
    for (int r = 0; r < PB; ++r) {
      int e = tid + NT * r;
      int kk, nn;
      if (BN_) { nn = e % BN; kk = e / BN; } else { kk = e % BK; nn = e / BK; }
      int gn = n0 + nn, gk = k0 + kk;
      rb[r] = (gn < N && gk < kend)
                  ? cvt_scaled<MF>(B[(long)gk * sbr + (long)gn * sbc], bexp ? bexp[gn] : 0)
                  : (MF)0;
    }
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int r = 0; r < PA; ++r) {
      int e = tid + NT * r;
      int kk, mm;
      if (AK) { kk = e % BK; mm = e / BK; } else { mm = e % BM; kk = e / BM; }
      As[buf][kk][mm] = ra[r];
    }
#pragma unroll
    for (int r = 0; r < PB; ++r) {
      int e = tid + NT * r;
      int kk, nn;
      if (BN_) { nn = e % BN; kk = e / BN; } else { kk = e % BK; nn = e / BK; }
      Bs[buf][kk][nn] = rb[r];
    }
  };

  if (kbeg < kend) {
    load(kbeg);
    store(0);
  }
  __syncthreads();
  int buf = 0;
  for (int k0 = kbeg; k0 < kend; k0 += BK) {
    const bool more = k0 + BK < kend;
    if (more) load(k0 + BK);
#pragma unroll
    for (int ks = 0; ks < BK; ks += 4) {
      const int kq = ks + (lane >> 4);
      MF a0 = As[buf][kq][wm + (lane & 15)];
      MF a1 = As[buf][kq][wm + 16 + (lane & 15)];
      MF b0 = Bs[buf][kq][wn + (lane & 15)];
      MF b1 = Bs[buf][kq][wn + 16 + (lane & 15)];
      acc[0][0] = mfma4(a0, b0, acc[0][0]);
      acc[0][1] = mfma4(a0, b1, acc[0][1]);
      acc[1][0] = mfma4(a1, b0, acc[1][0]);
      acc[1][1] = mfma4(a1, b1, acc[1][1]);
    }
    if (more) store(buf ^ 1);
    __syncthreads();
    buf ^= 1;
  }
  // D layout of the 16x16 tile, lane l, register i: column l % 16; row 4*i + l/16 for the
  // FP64 instruction and 4*(l/16) + i for the binary32 one.
  constexpr bool kF64 = sizeof(MF) == 8;
  const int ea = aexp ? *aexp : 0;
#pragma unroll
  for (int ti = 0; ti < 2; ++ti)
#pragma unroll
    for (int tj = 0; tj < 2; ++tj)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        int rr = kF64 ? (4 * i + (lane >> 4)) : (4 * (lane >> 4) + i);
        int gm = m0 + wm + ti * 16 + rr;
        int gn = n0 + wn + tj * 16 + (lane & 15);
        if (gm < M && gn < N) {
          AS v = acc[ti][tj][i];
          const int es = ea + (bexp ? bexp[gn] : 0);
          const double al = es == 0 ? alpha : ldexp(alpha, es);
          if (part) {
            part[((long)blockIdx.z * M + gm) * N + gn] = (TC)((double)v * al);
          } else {
            TC* cp = C + (long)gm * ldc + gn;
            double out = al * (double)v;
            if (beta != 0.0) out += beta * (double)(*cp);
            *cp = (TC)out;
          }
        }
      }
}

// ---------------------------------------------------------------------------- k32 kernel
template <class MF> struct V8;
template <> struct V8<_Float16> { typedef f16x8 T; };
template <> struct V8<__bf16> { typedef bf16x8 T; };

__device__ inline f32x4 mfma32(f16x8 a, f16x8 b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
}
__device__ inline f32x4 mfma32(bf16x8 a, bf16x8 b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

template <class TA, class TB, class MF, class TC, bool AK, bool BN_>
__global__ __launch_bounds__(NT) void gemm_k32(int M, int N, int K, int kchunk, double alpha,
                                               double beta, const TA* __restrict__ A, long sar,
                                               long sac, const TB* __restrict__ B, long sbr,
                                               long sbc, TC* __restrict__ C, long ldc,
                                               TC* __restrict__ part,
                                               const int* __restrict__ aexp,
                                               const int* __restrict__ bexp) {
  constexpr int BK = 32, PK = BK + 8;
  typedef typename V8<MF>::T VT;
  __shared__ __attribute__((aligned(16))) MF As[BM][PK];
  __shared__ __attribute__((aligned(16))) MF Bs[BN][PK];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int m0 = blockIdx.y * BM, n0 = blockIdx.x * BN;
  const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
  const int kbeg = blockIdx.z * kchunk;
  const int kend = min(K, kbeg + kchunk);
  f32x4 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = f32x4{0, 0, 0, 0};

  for (int k0 = kbeg; k0 < kend; k0 += BK) {
#pragma unroll
    for (int r = 0; r < (BM * BK) / NT; ++r) {
      int e = tid + NT * r;
      int kk, mm;
      if (AK) { kk = e % BK; mm = e / BK; } else { mm = e % BM; kk = e / BM; }
      int gm = m0 + mm, gk = k0 + kk;
      MF v = Cvt<MF>::f(0.0f);
      if (gm < M && gk < kend) v = Cvt<MF>::f(A[(long)gm * sar + (long)gk * sac]);
      As[mm][kk] = v;
    }
#pragma unroll
    for (int r = 0; r < (BN * BK) / NT; ++r) {
      int e = tid + NT * r;
      int kk, nn;
      if (BN_) { nn = e % BN; kk = e / BN; } else { kk = e % BK; nn = e / BK; }
      int gn = n0 + nn, gk = k0 + kk;
      MF v = Cvt<MF>::f(0.0f);
      if (gn < N && gk < kend)
        v = cvt_scaled<MF>(B[(long)gk * sbr + (long)gn * sbc], bexp ? bexp[gn] : 0);
      Bs[nn][kk] = v;
    }
    __syncthreads();
    // operand layout: lane l holds row (l % 16), k = 8*(l/16) .. 8*(l/16)+7
    const int kq = 8 * (lane >> 4);
    VT a0 = *reinterpret_cast<const VT*>(&As[wm + (lane & 15)][kq]);
    VT a1 = *reinterpret_cast<const VT*>(&As[wm + 16 + (lane & 15)][kq]);
    VT b0 = *reinterpret_cast<const VT*>(&Bs[wn + (lane & 15)][kq]);
    VT b1 = *reinterpret_cast<const VT*>(&Bs[wn + 16 + (lane & 15)][kq]);
    acc[0][0] = mfma32(a0, b0, acc[0][0]);
    acc[0][1] = mfma32(a0, b1, acc[0][1]);
    acc[1][0] = mfma32(a1, b0, acc[1][0]);
    acc[1][1] = mfma32(a1, b1, acc[1][1]);
    __syncthreads();
  }
  const int ea = aexp ? *aexp : 0;
#pragma unroll
  for (int ti = 0; ti < 2; ++ti)
#pragma unroll
    for (int tj = 0; tj < 2; ++tj)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        int gm = m0 + wm + ti * 16 + 4 * (lane >> 4) + i;
        int gn = n0 + wn + tj * 16 + (lane & 15);
        if (gm < M && gn < N) {
          const int es = ea + (bexp ? bexp[gn] : 0);
          double out = (es == 0 ? alpha : ldexp(alpha, es)) * (double)acc[ti][tj][i];
          if (part) {
            part[((long)blockIdx.z * M + gm) * N + gn] = (TC)out;
          } else {
            TC* cp = C + (long)gm * ldc + gn;
            if (beta != 0.0) out += beta * (double)(*cp);
            *cp = (TC)out;
          }
        }
      }
}

// ------------------------------------------------------------------------- big kernel
// 128 x 128 block tile, eight waves in a 2 x 4 grid, each wave 64 x 32 (4 x 2 MFMA tiles of
// 16 x 16, one operand element per lane: FP64 16x16x4 or binary32 16x16x4); two waves per
// SIMD interleave, so one wave's loads and barriers overlap the other's products.  The k-slice of
// BK elements (BK * sizeof(MF) = 128 bytes) is double-buffered in LDS; the next slice is
// loaded into registers while the current one feeds the matrix cores.  The LDS layout follows
// the operand's layout in memory so that the stores are straight copies: a k-contiguous A is
// kept as As[m][k] (row stride BK + 1, so the 16 lanes reading 16 rows at one k hit distinct
// banks), an m-contiguous A as As[k][m]; B likewise as Bs[k][n] or Bs[n][k].
constexpr int GBM = 128, GBN = 128, GNT = 512;

template <class MF, bool KC, int BK, int BMN>
struct LdsTile {
  // KC: k contiguous -> [BMN][BK + 1]; otherwise [BK][BMN]
  static constexpr int R = KC ? BMN : BK;
  static constexpr int C = KC ? BK + 1 : BMN;
  __device__ static inline int at(int mn, int k) { return KC ? mn * C + k : k * C + mn; }
};

template <class TA, class TB, class MF, class TC, bool AK, bool BN_>
__global__ __launch_bounds__(GNT, 1) void gemm_big(int M, int N, int K, double alpha,
                                                   double beta, const TA* __restrict__ A,
                                                   long sar, long sac, const TB* __restrict__ B,
                                                   long sbr, long sbc, TC* __restrict__ C,
                                                   long ldc, const int* __restrict__ aexp,
                                                   const int* __restrict__ bexp) {
  constexpr int BK = 128 / (int)sizeof(MF);  // 16 (FP64) or 32 (binary32)
  typedef typename Acc<MF>::V AV;
  typedef LdsTile<MF, AK, BK, GBM> LA;
  typedef LdsTile<MF, !BN_, BK, GBN> LB;
  constexpr int AE = LA::R * LA::C, BE = LB::R * LB::C;
  __shared__ MF lds[2 * (AE + BE)];
  // per thread: (GBM * BK) / GNT = 8 (FP64) or 16 (binary32) elements of each operand
  constexpr int PT = GBM * BK / GNT;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int m0 = blockIdx.y * GBM, n0 = blockIdx.x * GBN;
  const int wm = (wave >> 2) * 64, wn = (wave & 3) * 32;

  // global -> register slice loaders: element e of this thread, contiguous runs along the
  // operand's unit-stride dimension
  MF ra[PT], rb[PT];
  auto load_a = [&](int k0) {
#pragma unroll
    for (int e = 0; e < PT; ++e) {
      const int q = tid + GNT * e;
      int mm, kk;
      if (AK) { kk = q % BK; mm = q / BK; } else { mm = q % GBM; kk = q / GBM; }
      const int gm = m0 + mm, gk = k0 + kk;
      ra[e] = (gm < M && gk < K) ? Cvt<MF>::f(A[(long)gm * sar + (long)gk * sac]) : (MF)0;
    }
  };
  auto load_b = [&](int k0) {
#pragma unroll
    for (int e = 0; e < PT; ++e) {
      const int q = tid + GNT * e;
      int nn, kk;
      if (BN_) { nn = q % GBN; kk = q / GBN; } else { kk = q % BK; nn = q / BK; }
      const int gn = n0 + nn, gk = k0 + kk;
      rb[e] = (gn < N && gk < K)
                  ? cvt_scaled<MF>(B[(long)gk * sbr + (long)gn * sbc], bexp ? bexp[gn] : 0)
                  : (MF)0;
    }
  };
  auto store = [&](int buf) {
    MF* As = lds + buf * (AE + BE);
    MF* Bs = As + AE;
#pragma unroll
    for (int e = 0; e < PT; ++e) {
      const int q = tid + GNT * e;
      int mm, kk, nn, kb;
      if (AK) { kk = q % BK; mm = q / BK; } else { mm = q % GBM; kk = q / GBM; }
      if (BN_) { nn = q % GBN; kb = q / GBN; } else { kb = q % BK; nn = q / BK; }
      As[LA::at(mm, kk)] = ra[e];
      Bs[LB::at(nn, kb)] = rb[e];
    }
  };

  AV acc[4][2];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = AV{0, 0, 0, 0};

  const int nk = (K + BK - 1) / BK;
  if (nk > 0) {
    load_a(0);
    load_b(0);
    store(0);
  }
  __syncthreads();
  for (int t = 0; t < nk; ++t) {
    const int buf = t & 1;
    if (t + 1 < nk) {
      load_a((t + 1) * BK);
      load_b((t + 1) * BK);
    }
    const MF* As = lds + buf * (AE + BE);
    const MF* Bs = As + AE;
#pragma unroll
    for (int ks = 0; ks < BK; ks += 4) {
      const int kq = ks + (lane >> 4);
      MF a[4], b[2];
#pragma unroll
      for (int i = 0; i < 4; ++i) a[i] = As[LA::at(wm + 16 * i + (lane & 15), kq)];
#pragma unroll
      for (int j = 0; j < 2; ++j) b[j] = Bs[LB::at(wn + 16 * j + (lane & 15), kq)];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = mfma4(a[i], b[j], acc[i][j]);
    }
    if (t + 1 < nk) store(buf ^ 1);
    __syncthreads();
  }
  // D layout of a 16x16 tile, lane l, register r: column l % 16; row 4 r + l / 16 (FP64
  // instruction) or 4 (l / 16) + r (binary32 instruction).
  constexpr bool kF64 = sizeof(MF) == 8;
  const int ea = aexp ? *aexp : 0;
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int gn = n0 + wn + 16 * j + (lane & 15);
      if (gn >= N) continue;
      const int es = ea + (bexp ? bexp[gn] : 0);
      const double al = es == 0 ? alpha : ldexp(alpha, es);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int rr = kF64 ? (4 * r + (lane >> 4)) : (4 * (lane >> 4) + r);
        const int gm = m0 + wm + 16 * i + rr;
        if (gm < M) {
          TC* cp = C + (long)gm * ldc + gn;
          double out = al * (double)acc[i][j][r];
          if (beta != 0.0) out += beta * (double)(*cp);
          *cp = (TC)out;
        }
      }
    }
}

// ------------------------------------------------------------------- split kernel
// Split-operand binary16 products (the hi/lo operand splitting of Markidis et al. 2018 and
// Ootomo and Yokota 2022): each operand element x is loaded as the pair hi = RNE16(x),
// lo = RNE16(2^11 (x - hi)), so x ~ hi + 2^-11 lo with 22 significand bits, and
// A B ~ Ah Bh + 2^-11 (Ah Bl + Al Bh): three 16x16x32 binary16 MFMAs per tile step, the
// hi*hi and cross sums in separate binary32 accumulators.  Tiles as in gemm_k32.
template <class S> __device__ inline void split16(S x, _Float16& hi, _Float16& lo);
template <> __device__ inline void split16<double>(double x, _Float16& hi, _Float16& lo) {
  hi = rne_from_f64<_Float16>(x);
  lo = rne_from_f64<_Float16>((x - (double)(float)hi) * 2048.0);
}
template <> __device__ inline void split16<float>(float x, _Float16& hi, _Float16& lo) {
  hi = (_Float16)x;
  lo = (_Float16)((x - (float)hi) * 2048.0f);  // x - hi is exact in binary32
}

template <class TA, class TB, class TC, bool AK, bool BN_>
__global__ __launch_bounds__(NT) void gemm_k32s(int M, int N, int K, int kchunk, double alpha,
                                                double beta, const TA* __restrict__ A, long sar,
                                                long sac, const TB* __restrict__ B, long sbr,
                                                long sbc, TC* __restrict__ C, long ldc,
                                                TC* __restrict__ part,
                                                const int* __restrict__ aexp,
                                                const int* __restrict__ bexp) {
  constexpr int BK = 32, PK = BK + 8;
  typedef _Float16 MF;
  typedef f16x8 VT;
  __shared__ __attribute__((aligned(16))) MF AsH[BM][PK];
  __shared__ __attribute__((aligned(16))) MF AsL[BM][PK];
  __shared__ __attribute__((aligned(16))) MF BsH[BN][PK];
  __shared__ __attribute__((aligned(16))) MF BsL[BN][PK];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int m0 = blockIdx.y * BM, n0 = blockIdx.x * BN;
  const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
  f32x4 hh[2][2], xx[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      hh[i][j] = f32x4{0, 0, 0, 0};
      xx[i][j] = f32x4{0, 0, 0, 0};
    }
  const int kbeg = blockIdx.z * kchunk;
  const int kend = min(K, kbeg + kchunk);
  for (int k0 = kbeg; k0 < kend; k0 += BK) {
#pragma unroll
    for (int r = 0; r < (BM * BK) / NT; ++r) {
      int e = tid + NT * r;
      int kk, mm;
      if (AK) { kk = e % BK; mm = e / BK; } else { mm = e % BM; kk = e / BM; }
      int gm = m0 + mm, gk = k0 + kk;
      MF h = (MF)0.0f, l = (MF)0.0f;
      if (gm < M && gk < kend) split16<TA>(A[(long)gm * sar + (long)gk * sac], h, l);
      AsH[mm][kk] = h;
      AsL[mm][kk] = l;
    }
#pragma unroll
    for (int r = 0; r < (BN * BK) / NT; ++r) {
      int e = tid + NT * r;
      int kk, nn;
      if (BN_) { nn = e % BN; kk = e / BN; } else { kk = e % BK; nn = e / BK; }
      int gn = n0 + nn, gk = k0 + kk;
      MF h = (MF)0.0f, l = (MF)0.0f;
      if (gn < N && gk < kend) {
        TB v = B[(long)gk * sbr + (long)gn * sbc];
        if (bexp && bexp[gn] != 0) v = (TB)ldexp((double)v, -bexp[gn]);
        split16<TB>(v, h, l);
      }
      BsH[nn][kk] = h;
      BsL[nn][kk] = l;
    }
    __syncthreads();
    const int kq = 8 * (lane >> 4);
    VT ah[2], al[2], bh[2], bl[2];
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      ah[i] = *reinterpret_cast<const VT*>(&AsH[wm + 16 * i + (lane & 15)][kq]);
      al[i] = *reinterpret_cast<const VT*>(&AsL[wm + 16 * i + (lane & 15)][kq]);
      bh[i] = *reinterpret_cast<const VT*>(&BsH[wn + 16 * i + (lane & 15)][kq]);
      bl[i] = *reinterpret_cast<const VT*>(&BsL[wn + 16 * i + (lane & 15)][kq]);
    }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        hh[i][j] = mfma32(ah[i], bh[j], hh[i][j]);
        xx[i][j] = mfma32(ah[i], bl[j], xx[i][j]);
        xx[i][j] = mfma32(al[i], bh[j], xx[i][j]);
      }
    __syncthreads();
  }
  const int ea = aexp ? *aexp : 0;
#pragma unroll
  for (int ti = 0; ti < 2; ++ti)
#pragma unroll
    for (int tj = 0; tj < 2; ++tj)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        int gm = m0 + wm + ti * 16 + 4 * (lane >> 4) + i;
        int gn = n0 + wn + tj * 16 + (lane & 15);
        if (gm < M && gn < N) {
          const int es = ea + (bexp ? bexp[gn] : 0);
          const double v = (double)hh[ti][tj][i] + (double)xx[ti][tj][i] * (1.0 / 2048.0);
          double out = (es == 0 ? alpha : ldexp(alpha, es)) * v;
          if (part) {
            part[((long)blockIdx.z * M + gm) * N + gn] = (TC)out;
          } else {
            TC* cp = C + (long)gm * ldc + gn;
            if (beta != 0.0) out += beta * (double)(*cp);
            *cp = (TC)out;
          }
        }
      }
}

// Sum split-K partial products in a fixed order: C = sum_z part[z] + beta * C.
__global__ void splitk_reduce(int M, int N, int splits, const double* __restrict__ part,
                              double beta, double* __restrict__ C, long ldc) {
  long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
  long total = (long)M * N;
  if (idx >= total) return;
  int gm = (int)(idx / N), gn = (int)(idx % N);
  double s = 0.0;
  for (int z = 0; z < splits; ++z) s += part[(long)z * total + idx];
  double* cp = C + (long)gm * ldc + gn;
  if (beta != 0.0) s += beta * (*cp);
  *cp = s;
}

// k-chunk of a split product: a multiple of the kernel's k-tile (a chunk past K is empty and
// contributes a zero partial product)
inline int chunk_of(int K, int splits, int bk) {
  return splits > 1 ? ceil_div(ceil_div(K, splits), bk) * bk : K;
}

template <class TA, class TB, class MF, class TC>
int launch_big(hipStream_t s, const GemmDesc& d) {
  dim3 grid(ceil_div(d.N, GBN), ceil_div(d.M, GBM), 1);
  bool ak = (d.sac == 1), bn = (d.sbc == 1);
  auto A = static_cast<const TA*>(d.A);
  auto B = static_cast<const TB*>(d.B);
  auto C = static_cast<TC*>(d.C);
#define KB(a, b)                                                                              \
  hipLaunchKernelGGL((gemm_big<TA, TB, MF, TC, a, b>), grid, dim3(GNT), 0, s, d.M, d.N, d.K,  \
                     d.alpha, d.beta, A, d.sar, d.sac, B, d.sbr, d.sbc, C, d.ldc, d.a_exp,    \
                     d.b_colexp)
  if (ak && bn) KB(true, true);
  else if (ak) KB(true, false);
  else if (bn) KB(false, true);
  else KB(false, false);
#undef KB
  LYAP_HIP(hipGetLastError());
  return LYAP_OK;
}

// The 128 x 128 kernel (one workgroup per CU) pays off once its grid covers every CU and the
// k-loop has a few slices; below that the 64 x 64 kernel's four times as many workgroups keep
// more of the GPU busy (measured on the inversion's updates at n = 4096: a threshold of 256
// tiles instead of 48 made the FP64 butterfly inversion 10.5 -> 9.7 ms).
inline bool use_big(const GemmDesc& d) {
  const long tiles = (long)ceil_div(d.M, GBM) * ceil_div(d.N, GBN);
  return d.M >= 96 && d.N >= 96 && d.K >= 32 && tiles >= 256;
}

template <class TA, class TB, class MF, class TC>
int launch_k4(hipStream_t s, const GemmDesc& d, int splits, TC* part) {
  dim3 grid(ceil_div(d.N, BN), ceil_div(d.M, BM), splits);
  const int kchunk = chunk_of(d.K, splits, 16);
  bool ak = (d.sac == 1), bn = (d.sbc == 1);
  auto A = static_cast<const TA*>(d.A);
  auto B = static_cast<const TB*>(d.B);
  auto C = static_cast<TC*>(d.C);
#define K4(a, b)                                                                              \
  hipLaunchKernelGGL((gemm_k4<TA, TB, MF, TC, a, b>), grid, dim3(NT), 0, s, d.M, d.N, d.K,   \
                     kchunk, d.alpha, d.beta, A, d.sar, d.sac, B, d.sbr, d.sbc, C, d.ldc,  \
                     part, d.a_exp, d.b_colexp)
  if (ak && bn) K4(true, true);
  else if (ak) K4(true, false);
  else if (bn) K4(false, true);
  else K4(false, false);
#undef K4
  LYAP_HIP(hipGetLastError());
  return LYAP_OK;
}

template <class TA, class TB, class MF, class TC>
int launch_k32(hipStream_t s, const GemmDesc& d, int splits, TC* part) {
  dim3 grid(ceil_div(d.N, BN), ceil_div(d.M, BM), splits);
  const int kchunk = chunk_of(d.K, splits, 32);
  bool ak = (d.sac == 1), bn = (d.sbc == 1);
  auto A = static_cast<const TA*>(d.A);
  auto B = static_cast<const TB*>(d.B);
  auto C = static_cast<TC*>(d.C);
#define K32(a, b)                                                                             \
  hipLaunchKernelGGL((gemm_k32<TA, TB, MF, TC, a, b>), grid, dim3(NT), 0, s, d.M, d.N, d.K,  \
                     kchunk, d.alpha, d.beta, A, d.sar, d.sac, B, d.sbr, d.sbc, C, d.ldc,   \
                     part, d.a_exp, d.b_colexp)
  if (ak && bn) K32(true, true);
  else if (ak) K32(true, false);
  else if (bn) K32(false, true);
  else K32(false, false);
#undef K32
  LYAP_HIP(hipGetLastError());
  return LYAP_OK;
}

template <class TA, class TB, class TC>
int launch_k32s(hipStream_t s, const GemmDesc& d, int splits, TC* part) {
  dim3 grid(ceil_div(d.N, BN), ceil_div(d.M, BM), splits);
  const int kchunk = chunk_of(d.K, splits, 32);
  bool ak = (d.sac == 1), bn = (d.sbc == 1);
  auto A = static_cast<const TA*>(d.A);
  auto B = static_cast<const TB*>(d.B);
  auto C = static_cast<TC*>(d.C);
#define KS(a, b)                                                                              \
  hipLaunchKernelGGL((gemm_k32s<TA, TB, TC, a, b>), grid, dim3(NT), 0, s, d.M, d.N, d.K,      \
                     kchunk, d.alpha, d.beta, A, d.sar, d.sac, B, d.sbr, d.sbc, C, d.ldc,    \
                     part, d.a_exp, d.b_colexp)
  if (ak && bn) KS(true, true);
  else if (ak) KS(true, false);
  else if (bn) KS(false, true);
  else KS(false, false);
#undef KS
  LYAP_HIP(hipGetLastError());
  return LYAP_OK;
}

// Split-K for products with fewer output tiles than four workgroups per CU and a long
// k-loop: about 1024 workgroups, at least 256 k per split, at most 64 splits, within the
// workspace (splits x M x N FP64 partial products).  With the 64 x 64 tile at M = n = 4096,
// N <= 320, K = n (the factor products of the solvers) one block per tile left the matrix
// cores idle most of the time: about 500 us per product, regardless of N.
int split_count(const GemmDesc& d, size_t ws_elems) {
  const long tiles = (long)ceil_div(d.M, BM) * ceil_div(d.N, BN);
  if (ws_elems == 0 || tiles >= 256 || d.K < 512) return 1;
  int splits = (int)std::min<long>((1024 + tiles - 1) / tiles, d.K / 256);
  splits = std::min(splits, 64);
  while (splits > 1 && (size_t)splits * d.M * d.N > ws_elems) --splits;
  return std::max(splits, 1);
}

int reduce_splits(hipStream_t s, const GemmDesc& d, int splits, const double* part) {
  const long total = (long)d.M * d.N;
  hipLaunchKernelGGL(splitk_reduce, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, d.M,
                     d.N, splits, part, d.beta, static_cast<double*>(d.C), d.ldc);
  LYAP_HIP(hipGetLastError());
  return LYAP_OK;
}

template <class TA, class TB, class TC>
int dispatch_lp_op(hipStream_t s, Prec op, const GemmDesc& d, int splits, TC* part) {
  switch (op) {
    case Prec::F32:
      if (splits <= 1 && use_big(d)) return launch_big<TA, TB, float, TC>(s, d);
      return launch_k4<TA, TB, float, TC>(s, d, splits, part);
    case Prec::F16: return launch_k32<TA, TB, _Float16, TC>(s, d, splits, part);
    case Prec::BF16: return launch_k32<TA, TB, __bf16, TC>(s, d, splits, part);
    case Prec::F16X2:
      if constexpr ((std::is_same<TA, double>::value || std::is_same<TA, float>::value) &&
                    (std::is_same<TB, double>::value || std::is_same<TB, float>::value))
        return launch_k32s<TA, TB, TC>(s, d, splits, part);
      return LYAP_BADARG;
    default: return LYAP_BADARG;
  }
}

template <class TA, class TB>
int dispatch_lp_c(hipStream_t s, Prec op, Store sc, const GemmDesc& d, double* ws,
                  size_t ws_elems) {
  if (sc == Store::F32) return dispatch_lp_op<TA, TB, float>(s, op, d, 1, nullptr);
  if (sc != Store::F64) return LYAP_BADARG;
  const int splits = split_count(d, ws ? ws_elems : 0);
  LYAP_TRY((dispatch_lp_op<TA, TB, double>(s, op, d, splits, splits > 1 ? ws : nullptr)));
  return splits > 1 ? reduce_splits(s, d, splits, ws) : LYAP_OK;
}

template <class TA>
int dispatch_lp_b(hipStream_t s, Prec op, Store sb, Store sc, const GemmDesc& d, double* ws,
                  size_t ws_elems) {
  switch (sb) {
    case Store::F64: return dispatch_lp_c<TA, double>(s, op, sc, d, ws, ws_elems);
    case Store::F32: return dispatch_lp_c<TA, float>(s, op, sc, d, ws, ws_elems);
    case Store::F16: return dispatch_lp_c<TA, _Float16>(s, op, sc, d, ws, ws_elems);
    case Store::BF16: return dispatch_lp_c<TA, __bf16>(s, op, sc, d, ws, ws_elems);
  }
  return LYAP_BADARG;
}

}  // namespace

int gemm_f64(hipStream_t s, const GemmDesc& d, double* ws, size_t ws_elems) {
  if (d.M <= 0 || d.N <= 0) return LYAP_OK;
  // K == 0 is handled by the kernel itself: the k-loop is empty and C = beta * C.
  const int splits = split_count(d, ws ? ws_elems : 0);
  if (splits <= 1) {
    if (use_big(d)) return launch_big<double, double, double, double>(s, d);
    return launch_k4<double, double, double, double>(s, d, 1, nullptr);
  }
  LYAP_TRY((launch_k4<double, double, double, double>(s, d, splits, ws)));
  return reduce_splits(s, d, splits, ws);
}

int gemm_lp(hipStream_t s, Prec op, Store sa, Store sb, Store sc, const GemmDesc& d, double* ws,
            size_t ws_elems) {
  if (d.M <= 0 || d.N <= 0) return LYAP_OK;
  switch (sa) {
    case Store::F64: return dispatch_lp_b<double>(s, op, sb, sc, d, ws, ws_elems);
    case Store::F32: return dispatch_lp_b<float>(s, op, sb, sc, d, ws, ws_elems);
    case Store::F16: return dispatch_lp_b<_Float16>(s, op, sb, sc, d, ws, ws_elems);
    case Store::BF16: return dispatch_lp_b<__bf16>(s, op, sb, sc, d, ws, ws_elems);
  }
  return LYAP_BADARG;
}

}  // namespace lyap
