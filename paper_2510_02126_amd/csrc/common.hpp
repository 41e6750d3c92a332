// Shared definitions for the gfx950 Lyapunov solver library.
#pragma once

#include <hip/hip_runtime.h>
#include <vector>
#include <hip/hip_fp16.h>
#include <hip/hip_bf16.h>

#include <cstddef>
#include <cstdint>

#include "../../include/lyap.h"

namespace lyap {

typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

// Round-to-nearest-even conversion of a binary64 value to a narrower format, with a single
// rounding.  binary32 is converted directly.  For fp16 and bf16 the value is first rounded to
// binary32 by truncation with the last bit set when inexact ("round to odd"); since binary32
// carries more than p + 1 bits for both targets (p = 11 and 8), the following nearest-even
// rounding then gives the correctly rounded result (Boldo and Melquiond, 2008), where the
// direct route through a nearest-even binary32 value can round twice.
__device__ inline float f32_round_odd(double x) {
  float f = __double2float_rz(x);
  if ((double)f != x) f = __int_as_float(__float_as_int(f) | 1);
  return f;
}
template <class T> __device__ inline T rne_from_f64(double x);
template <> __device__ inline double rne_from_f64<double>(double x) { return x; }
template <> __device__ inline float rne_from_f64<float>(double x) { return (float)x; }
template <> __device__ inline _Float16 rne_from_f64<_Float16>(double x) {
  return (_Float16)f32_round_odd(x);
}
template <> __device__ inline __bf16 rne_from_f64<__bf16>(double x) {
  return (__bf16)f32_round_odd(x);
}

// Operand formats of the matrix-core products.
enum class Prec : int {
  F64 = LYAP_F64, F32 = LYAP_F32, F16 = LYAP_F16, BF16 = LYAP_BF16, F16X2 = LYAP_F16X2
};

inline double unit_roundoff(Prec p) {
  switch (p) {
    case Prec::F64: return 1.1102230246251565e-16;   // 2^-53
    case Prec::F32: return 5.960464477539063e-08;    // 2^-24
    case Prec::F16: return 4.8828125e-04;            // 2^-11
    case Prec::BF16: return 3.90625e-03;             // 2^-8
    case Prec::F16X2: return 2.384185791015625e-07;  // 2^-22: hi + 2^-11 lo, two binary16
  }
  return 0.0;
}

// Status propagated out of the internal routines.
struct Status {
  int code = LYAP_OK;
  bool ok() const { return code == LYAP_OK; }
};

#define LYAP_HIP(expr)                                   \
  do {                                                   \
    hipError_t _e = (expr);                              \
    if (_e != hipSuccess) return LYAP_HIP_ERROR;         \
  } while (0)

#define LYAP_TRY(expr)                                   \
  do {                                                   \
    int _c = (expr);                                     \
    if (_c != LYAP_OK) return _c;                        \
  } while (0)

inline int ceil_div(int a, int b) { return (a + b - 1) / b; }
inline size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// Device workspace owned by a handle: one bump allocator over a growable hipMalloc block.
struct Arena {
  char* base = nullptr;
  size_t cap = 0;
  size_t top = 0;
  int reserve(size_t bytes);          // ensure capacity (frees old block; call when empty)
  void reset() { top = 0; }
  template <class T>
  T* take(size_t count) {
    size_t off = align_up(top, 256);
    size_t need = off + align_up(count * sizeof(T), 256);
    if (need > cap) return nullptr;
    top = need;
    return reinterpret_cast<T*>(base + off);
  }
  void release();
};

// Event timing of kernel families, for the roofline report of a solve: each timed interval
// is a pair of events on the stream, resolved after the solve.  Families: 0 inversions
// (work in flops, 2 n^3 each), 1 Jacobi round kernels (work in bytes, the A and V traffic of
// the block update), 2 thin QR factorisations (work in flops), 3 unused.
struct KernTimer {
  static constexpr int NF = 4;
  double ms[NF] = {0, 0, 0, 0};
  double work[NF] = {0, 0, 0, 0};
  int calls[NF] = {0, 0, 0, 0};
  struct Pending {
    hipEvent_t a, b;
    int fam;
    double work;
    int calls;
  };
  std::vector<Pending> pend;
  std::vector<hipEvent_t> pool;
  // Records an event on s into *e (from the pool).
  int mark(hipStream_t s, hipEvent_t* e);
  void add(hipEvent_t a, hipEvent_t b, int fam, double work, int calls) {
    pend.push_back({a, b, fam, work, calls});
  }
  // Waits for the pending intervals and accumulates them.
  int collect();
  void reset();
  void release();
};

// ------------------------------------------------------------------ launchers
// Generic strided product C = alpha * opA * opB + beta * C, opA(i,k) = A[i*sar + k*sac],
// opB(k,j) = B[k*sbr + j*sbc], C row-major (ldc).  Operand storage types are given by
// the template instantiations in gemm.hip.
struct GemmDesc {
  int M = 0, N = 0, K = 0;
  double alpha = 1.0, beta = 0.0;
  const void* A = nullptr;
  long sar = 0, sac = 0;
  const void* B = nullptr;
  long sbr = 0, sbc = 0;
  void* C = nullptr;
  long ldc = 0;
  // Power-of-two scalings of reduced-precision operands (device ints, may be NULL):
  // op(A) is stored as 2^-a_exp times the matrix it stands for, so the product is multiplied
  // by 2^a_exp; column j of op(B) is multiplied by 2^-b_colexp[j] before it is rounded to the
  // operand format and column j of the product by 2^b_colexp[j] afterwards.  Both are exact.
  const int* a_exp = nullptr;
  const int* b_colexp = nullptr;
};

// Storage type codes for operands/results.
enum class Store : int { F64 = 0, F32 = 1, F16 = 2, BF16 = 3 };

// Product with FP64 matrix cores (all storage F64).  With a workspace (splitk_ws, ws_elems
// doubles) a product with few output tiles and a long k-loop splits K across workgroups.
int gemm_f64(hipStream_t s, const GemmDesc& d, double* splitk_ws = nullptr, size_t ws_elems = 0);
// Product with operands rounded to ``op`` (F32/F16/BF16), binary32 accumulation.  A and B
// stored as ``sa``/``sb``, C stored as ``sc`` (F32 or F64).  For an F64 C a workspace allows
// the same split of K (binary32 accumulation within each k-chunk, FP64 across chunks).
int gemm_lp(hipStream_t s, Prec op, Store sa, Store sb, Store sc, const GemmDesc& d,
            double* splitk_ws = nullptr, size_t ws_elems = 0);

}  // namespace lyap
