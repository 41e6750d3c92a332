// Host driver of the solver: the scaled sign-function Newton A-iteration with its cached
// sequence of inverses (Section 3.4), the factored LDL^T iteration (eq 3.3, Alg 3.2) with
// RankTruncLdlt, and the mixed-precision iterative refinement of Alg 2.2 with the residual
// factorisation (Fragment 2.3) and the projected solution update (Fragment 2.4); the
// Cholesky type (Alg 2.1, Fragments 2.1 / 2.2) shares the same pieces.
//
// Every matrix operation runs in the library's HIP kernels; the host only keeps scalars
// (the scalings mu_k, stopping quantities, the diagonal factors D, kept-index lists) and
// decides ranks and stops from them.  Tall factors are row-major n x cols with a common
// leading dimension ``cap``.  All device memory of a solve is carved from one workspace
// (Layout), so a caller can provide it and the solve allocates nothing.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <vector>

#include "common.hpp"
#include "internal.hpp"
#include "solver.hpp"

namespace lyap {

int DevBuf::ensure(size_t b) {
  if (b <= bytes && p) return LYAP_OK;
  release();
  size_t want = align_up(std::max(b, (size_t)256), (size_t)1 << 16);
  if (hipMalloc(&p, want) != hipSuccess) {
    p = nullptr;
    bytes = 0;
    return LYAP_NO_MEMORY;
  }
  bytes = want;
  return LYAP_OK;
}

void DevBuf::release() {
  if (p) (void)hipFree(p);
  p = nullptr;
  bytes = 0;
}

void Solver::release() {
  key_ = CacheKey();
  kt_.release();
}

namespace {

using clk = std::chrono::steady_clock;

double ms_since(clk::time_point t0) {
  return std::chrono::duration<double, std::milli>(clk::now() - t0).count();
}

// Storage of values held at a precision (the split format keeps binary32 values and splits
// them as they are loaded into a product).
Store store_of(Prec p) {
  switch (p) {
    case Prec::F64: return Store::F64;
    case Prec::F32: return Store::F32;
    case Prec::F16: return Store::F16;
    case Prec::BF16: return Store::BF16;
    case Prec::F16X2: return Store::F32;
  }
  return Store::F64;
}

size_t store_bytes(Store s) {
  return s == Store::F64 ? 8 : (s == Store::F32 ? 4 : 2);
}

// Next precision up for escalation (Table 1.1): bf16 -> fp16 -> fp32 -> fp64 (the split
// format escalates to fp32).
Prec next_up(Prec p) {
  switch (p) {
    case Prec::BF16: return Prec::F16;
    case Prec::F16: return Prec::F32;
    default: return Prec::F64;
  }
}

double round_host(double x, Prec p) {
  if (p == Prec::F32) return (double)(float)x;
  return x;
}

// power-iteration steps of the 2-norm and spectral-radius estimates of the optional scalings
// and of the ADI solver's spectral interval
constexpr int NORM_ITERS = 12;
constexpr int RHO_ITERS = 24;

// ------------------------------------------------- elliptic functions for the ADI shifts
// Arithmetic-geometric mean of x >= y > 0.
double agm(double x, double y) {
  for (int i = 0; i < 64 && x - y > 1e-16 * x; ++i) {
    const double t = 0.5 * (x + y);
    y = std::sqrt(x * y);
    x = t;
  }
  return x;
}

// Complete elliptic integral K of modulus k with complementary modulus kp:
// K = pi / (2 AGM(1, kp)) (Gauss).
double ellip_k(double kp) { return 1.5707963267948966 / agm(1.0, kp); }

// Jacobi dn(u | k) by the descending Landen (AGM) scheme of Abramowitz and Stegun 16.4:
// a_0 = 1, b_0 = kp, c_0 = k; a_{i+1} = (a_i + b_i) / 2, b_{i+1} = sqrt(a_i b_i),
// c_{i+1} = (a_i - b_i) / 2 until c_N is negligible; phi_N = 2^N a_N u,
// phi_{i-1} = (phi_i + asin(c_i sin(phi_i) / a_i)) / 2; dn = cos(phi_0) / cos(phi_1 - phi_0).
double jacobi_dn(double u, double k, double kp) {
  double a[40], c[40];
  a[0] = 1.0;
  c[0] = k;
  double b = kp;
  int N = 0;
  while (N < 38 && std::fabs(c[N]) > 1e-17 * a[N]) {
    a[N + 1] = 0.5 * (a[N] + b);
    c[N + 1] = 0.5 * (a[N] - b);
    b = std::sqrt(a[N] * b);
    ++N;
  }
  if (N == 0) return 1.0;  // k = 0
  double phi = std::ldexp(a[N] * u, N);
  double phi1 = phi;
  for (int i = N; i >= 1; --i) {
    phi1 = phi;
    phi = 0.5 * (phi + std::asin(c[i] * std::sin(phi) / a[i]));
  }
  return std::cos(phi) / std::cos(phi1 - phi);
}

// Wachspress's optimal real ADI shifts for a spectrum of -A inside [a, b]: with kp = a / b,
// k = sqrt(1 - kp^2), K = K(k), the shifts are p_i = -b dn((2i - 1) K / (2J) | k), i <= J.
// J = 0 asks for the count that brings the ADI error function below eps over [a, b]:
// J = ceil(K ln(4 / eps) / (pi K(kp))).
std::vector<double> adi_shifts(double a, double b, int J, double eps) {
  if (!(a < b)) return std::vector<double>(std::max(J, 1), -b);
  const double kp = a / b;
  const double k = std::sqrt((1.0 - kp) * (1.0 + kp));
  const double K = ellip_k(kp), Kp = ellip_k(k);
  if (J <= 0) J = std::max(1, (int)std::ceil(K * std::log(4.0 / eps) / (3.141592653589793 * Kp)));
  std::vector<double> p(J);
  for (int i = 0; i < J; ++i) p[i] = -b * jacobi_dn((2.0 * i + 1.0) * K / (2.0 * J), k, kp);
  return p;
}

}  // namespace

Layout solver_layout(int n, int m, Prec us, const lyap_options& opt) {
  Layout L;
  L.n = n;
  L.m = m;
  L.cap = (opt.form == 1 ? 3 : 2) * n + 2 * m + 64;
  L.slots = std::max(1, std::min(opt.k_max, 64));
  const Prec cache_prec = opt.escalate ? Prec::F64 : us;
  L.slot_bytes = align_up((size_t)n * n * store_bytes(store_of(cache_prec)), 256);
  const size_t nn = (size_t)n * n, ncap = (size_t)n * L.cap, cap = (size_t)L.cap;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t o = off;
    off += align_up(std::max(bytes, (size_t)8), 256);
    return o;
  };
  L.cache = take(L.slot_bytes * L.slots);
  L.cexp = take(64 * sizeof(int));
  L.Ak = take(nn * 8);
  L.An = take(nn * 8);
  L.Ainv = take(nn * 8);
  L.colsum = take((size_t)n * 8);
  L.part = take((2 * 256 + 256 * (size_t)n + 1024) * 8);
  L.scal = take(64 * 8);
  L.flags = take(16 * sizeof(int));
  L.fpr = take(2 * sizeof(unsigned long long));
  L.vecs = take((size_t)(3 + 16) * n * 8);
  L.dvec = take(cap * 8);
  L.dvec2 = take(cap * 8);
  L.idx = take(cap * 4);
  L.colexp = take(cap * 4);
  L.bits = take(cap * 8);
  L.Lq = take((size_t)n * m * 8);
  L.Sm = take((size_t)m * m * 8);
  L.Sv = take((size_t)m * m * 8);
  L.Sw = take((size_t)m * 8);
  L.Zs = take(ncap * 8);
  L.Zc = take(ncap * 8);
  L.Zd = take(ncap * 8);
  L.F = take(ncap * 8);
  L.Uq = take(ncap * 8);
  L.Tq = take(ncap * 8);
  L.TN = take(ncap * 8);
  L.Hm = take(ncap * 8);
  L.Vm = take(ncap * 8);
  L.Gm = take(nn * 8);
  L.wv = take(cap * 8);
  const Prec inv_prec = opt.escalate ? Prec::F64 : us;
  // scratch of one step at a time: a thin QR (qr_lead adds its Gram-Schmidt coefficients and
  // split-K partial products, at most n^2/4 and min(2 n^2, 2^22) doubles, in front of the
  // QR of the rest), a spectral decomposition, or an inversion
  const size_t lead = ((nn / 4) + std::min(2 * nn, (size_t)1 << 22)) * 8 + ((size_t)1 << 16);
  L.arena_bytes = std::max(std::max(qr_workspace_bytes(n, L.cap), syev_workspace_bytes(n)),
                           syev_workspace_bytes(std::max(m, 1))) +
                  std::max(inverse_workspace_bytes(inv_prec, n) + rbt_workspace_bytes(n), lead);
  L.arena = take(L.arena_bytes);
  L.total = off;
  return L;
}

struct Solver::Ctx {
  hipStream_t s;
  char* base;
  Layout lay;
  Arena arena;
  int* flags;
  int n, m;
  const double* A;
  long lda;
  const double* L;
  long ldl;
  Prec us, u, ur, uc;
  Store cstore;
  lyap_options opt;
  bool psd;
  std::vector<double> svec;
  int cap;
  int K = 0;
  int iters = 0;  // steps of the last inner solve (Newton steps or ADI steps)
  std::vector<double> mus;
  double normA = 0.0, normW = 0.0;
  unsigned long long fp = 0;
  unsigned long epoch = 0;
  bool may_reuse = false;
  lyap_info* info;
  double* scal;
  double* part;
  KernTimer* kt = nullptr;
  bool trans = false;  // adjoint equation: products with A^T and with (A_k^{-1})^T
  // Leading columns known to be orthonormal: of Zs during a factor iteration (a truncated
  // factor Q V_kept is), and whether the solution factor in Zc is.  The QRs of the
  // truncation, the residual factorisation and the update then orthogonalise only the rest.
  int orth = 0;
  bool zc_orth = false;
  bool chol = false;  // Cholesky-type IR (Alg 2.1)
  // buffers
  char* cache;
  int* cexp;
  double *Ak, *An, *Ainv, *colsum, *vecs, *dvec, *dvec2;
  int *idx, *colexp;
  unsigned long long *bits, *fpr;
  double *Zs, *Zc, *Zd, *F, *Uq, *Tq, *TN, *Hm, *Vm, *Gm, *wv;
  template <class T> T* at(size_t off) const { return reinterpret_cast<T*>(base + off); }
  void* slot(int k) const { return cache + (size_t)k * lay.slot_bytes; }
};

int Solver::upload_d(Ctx& c, const std::vector<double>& d, double* dst) {
  if (d.empty()) return LYAP_OK;
  LYAP_HIP(hipMemcpyAsync(dst, d.data(), d.size() * sizeof(double), hipMemcpyHostToDevice, c.s));
  return LYAP_OK;
}

// mu_{k-1} of the chosen scaling (Section 3): Frobenius sqrt(||A^-1||_F / ||A||_F),
// determinantal |det A|^(-1/n), 2-norm sqrt(||A^-1||_2 / ||A||_2), spectral
// sqrt(rho(A^-1) / rho(A)); 1 once scaling is switched off.  The 2-norms and spectral radii
// are power-iteration estimates.  Result on the device in mu_dev.
int Solver::scaling_mu(Ctx& c, int mode, const double* Ak, const double* Ainv,
                       const double* a_ss, const double* logdet, bool scaling, double* mu_dev) {
  hipStream_t s = c.s;
  const int n = c.n;
  double* sc = c.scal;
  switch (scaling ? mode : 0) {
    case 1:
      return newton_mu(s, 1, logdet, nullptr, n, scaling ? 1 : 0, mu_dev);
    case 2:
      LYAP_TRY(norm2_est(s, n, Ak, n, NORM_ITERS, sc + 7, c.vecs));
      LYAP_TRY(norm2_est(s, n, Ainv, n, NORM_ITERS, sc + 8, c.vecs));
      return newton_mu(s, 2, sc + 8, sc + 7, n, 1, mu_dev);
    case 3:
      LYAP_TRY(specrad_est(s, n, Ak, n, RHO_ITERS, sc + 7, c.vecs));
      LYAP_TRY(specrad_est(s, n, Ainv, n, RHO_ITERS, sc + 8, c.vecs));
      return newton_mu(s, 2, sc + 8, sc + 7, n, 1, mu_dev);
    default:
      return newton_mu(s, 0, sc + 1, a_ss, n, scaling ? 1 : 0, mu_dev);
  }
}

// ---------------------------------------------------------------------------- A-iteration
// eq (3.1a) with the chosen scaling; stop when ||A_k + I||_1 <= tau_N = 10 sqrt(n u_s), or
// when scaling is already off and delta_k > delta_{k-1}/2; the step that meets the test is
// followed by one further step.  Scaling is switched off for good once delta_k < delta_off.
// Each inverse is cached at u_s as a power of two times a value of the format (per matrix).
int Solver::a_iteration(Ctx& c) {
  const int n = c.n;
  hipStream_t s = c.s;
  double* Ak = c.Ak;
  double* An = c.An;
  double* scal = c.scal;
  c.mus.clear();
  c.K = 0;
  LYAP_TRY(copy_block(s, n, n, c.A, c.lda, Ak, n));
  LYAP_TRY(sumsq(s, n, n, Ak, n, scal + 0, c.part));
  const double tau = 10.0 * std::sqrt(n * unit_roundoff(c.us));
  bool scaling = true;
  int countdown = -1;
  double delta_prev = -1.0;
  double last_onenorm = INFINITY;
  bool stopped = false;
  const double* a_ss = scal + 0;
  const int kmax = std::min(c.opt.k_max, c.lay.slots);
  for (int k = 1; k <= kmax; ++k) {
    double* out = (c.us == Prec::F64) ? static_cast<double*>(c.slot(k - 1)) : c.Ainv;
    // ||A_{k-1} + I||_1 < 1 makes A_{k-1} strictly column diagonally dominant: partial
    // pivoting would pick the diagonal, so the pivot search is skipped (same result).
    // Otherwise, with opt.pivoting = 1, the random butterfly transformation removes the need
    // for pivoting; its residual probe decides whether the step is redone with partial
    // pivoting.
    const bool pivot = !(last_onenorm < 1.0);
    // opt.scaling 4 (combined): determinantal for the first step, Frobenius afterwards
    const int mode = c.opt.scaling == 4 ? (k == 1 ? 1 : 0) : c.opt.scaling;
    const bool want_det = scaling && mode == 1;
    bool rbt = pivot && c.opt.pivoting == 1 && n % 4 == 0;
    double h[6];
    double probe = 0.0;
    int fl[2];
    for (;;) {
      LYAP_TRY(fill_int(s, c.flags, 2, 0));
      c.arena.reset();
      if (rbt) {
        LYAP_TRY(rbt_invert(s, c.us, n, Ak, n, out, n, c.arena, c.flags, c.kt,
                            want_det ? scal + 6 : nullptr, 0x4c59415055ull + (unsigned)k,
                            scal + 13));
      } else {
        LYAP_TRY(invert(s, c.us, n, Ak, n, out, n, c.arena, c.flags, pivot, c.kt,
                        want_det ? scal + 6 : nullptr));
      }
      if (c.us != Prec::F64) {
        // cached copy 2^-e A_k^-1 rounded once to u_s (e from its largest entry)
        LYAP_TRY(absmax_exp(s, n, n, out, n, c.cexp + (k - 1), c.flags + 1, c.part));
        LYAP_TRY(cast_scaled(s, c.cstore, n, n, out, n, c.slot(k - 1), c.cexp + (k - 1)));
      } else {
        LYAP_TRY(fill_int(s, c.cexp + (k - 1), 1, 0));
      }
      LYAP_TRY(sumsq(s, n, n, out, n, scal + 1, c.part));
      LYAP_TRY(scaling_mu(c, mode, Ak, out, a_ss, scal + 6, scaling, scal + 2));
      LYAP_TRY(copy_block(s, 1, 1, a_ss, 1, scal + 14, 1));  // ||A_{k-1}||_F^2, kept
      LYAP_TRY(newton_update(s, n, Ak, n, out, n, scal + 2, An, n, scal + 3, c.colsum, c.part));
      double a2 = 0.0;
      LYAP_HIP(hipMemcpyAsync(h, scal, sizeof(h), hipMemcpyDeviceToHost, s));
      LYAP_HIP(hipMemcpyAsync(&a2, scal + 14, sizeof(double), hipMemcpyDeviceToHost, s));
      LYAP_HIP(hipMemcpyAsync(&probe, scal + 13, sizeof(double), hipMemcpyDeviceToHost, s));
      LYAP_HIP(hipMemcpyAsync(fl, c.flags, sizeof(fl), hipMemcpyDeviceToHost, s));
      LYAP_HIP(hipStreamSynchronize(s));
      c.info->inversions += 1;
      if (!rbt) break;
      // accept when ||A (A^-1 x) - x|| <= 8 sqrt(n) u_s ||A||_F ||A^-1||_F ||x|| (a backward
      // stable inversion's residual is of order u_s kappa); otherwise partial pivoting
      const double bound = 8.0 * std::sqrt((double)n) * unit_roundoff(c.us) *
                           std::sqrt(a2) * std::sqrt(h[1]);
      if (!fl[0] && !fl[1] && std::isfinite(probe) && probe <= bound) {
        c.info->rbt_steps += 1;
        break;
      }
      c.info->rbt_fallbacks += 1;
      rbt = false;
    }
    if (fl[0]) return LYAP_SINGULAR;
    const double mu = h[2], dsq = h[3], anew = h[4], onenorm = h[5];
    if (fl[1] || !std::isfinite(mu) || !(mu > 0.0) || !std::isfinite(anew) ||
        !std::isfinite(onenorm) || !std::isfinite(h[1]))
      return LYAP_NONFINITE;
    const double delta = std::sqrt(dsq / anew);
    c.mus.push_back(mu);
    if (k <= 64) {
      c.info->mus[k - 1] = mu;
      c.info->onenorm[k - 1] = onenorm;
      c.info->n_mu = k;
    }
    std::swap(Ak, An);
    a_ss = scal + 4;
    c.K = k;
    last_onenorm = onenorm;
    if (countdown >= 0) {
      if (--countdown <= 0) {
        stopped = true;
        break;
      }
    } else if (onenorm <= tau || (!scaling && delta_prev >= 0.0 && delta > 0.5 * delta_prev)) {
      countdown = 1;
    }
    if (scaling && delta < c.opt.delta_off) scaling = false;
    delta_prev = delta;
  }
  if (!stopped) return LYAP_NOT_STABLE;
  // sign(A) = -I exactly when A is Hurwitz.  ||A_K + I||_1 < 1 puts every eigenvalue of A_K
  // within distance 1 of -1, so A is Hurwitz; an eigenvalue of A in the right half-plane
  // leaves an eigenvalue of A_K near +1 and ||A_K + I||_1 >= 2 - O(u).  When tau_N >= 1
  // (fp16/bf16 at large n) the loose stop leaves A_K too far from -I to tell, and an
  // unstable A shows up instead as refinement that does not converge.
  if (last_onenorm < 1.0 || tau >= 1.0) return LYAP_OK;
  return LYAP_NOT_STABLE;
}

// ------------------------------------------------------------------- ADI sequence
// Inverse of the n x n FP64 matrix M at ``op`` into ``out`` (n x n): with opt.pivoting = 1
// the butterfly inversion first, checked by its residual probe and redone with partial
// pivoting when the probe fails (as in the A-iteration); otherwise partial pivoting.
int Solver::checked_inverse(Ctx& c, Prec op, const double* M, long ld, double* out,
                            unsigned long long seed) {
  const int n = c.n;
  hipStream_t s = c.s;
  double* scal = c.scal;
  bool rbt = c.opt.pivoting == 1 && n % 4 == 0;
  int fl[2];
  for (;;) {
    LYAP_TRY(fill_int(s, c.flags, 2, 0));
    c.arena.reset();
    if (rbt) {
      LYAP_TRY(rbt_invert(s, op, n, M, ld, out, n, c.arena, c.flags, c.kt, nullptr, seed,
                          scal + 13));
      LYAP_TRY(sumsq(s, n, n, M, ld, scal + 18, c.part));
      LYAP_TRY(sumsq(s, n, n, out, n, scal + 19, c.part));
    } else {
      LYAP_TRY(invert(s, op, n, M, ld, out, n, c.arena, c.flags, true, c.kt, nullptr));
    }
    double h[7];
    LYAP_HIP(hipMemcpyAsync(h, scal + 13, sizeof(h), hipMemcpyDeviceToHost, s));
    LYAP_HIP(hipMemcpyAsync(fl, c.flags, sizeof(fl), hipMemcpyDeviceToHost, s));
    LYAP_HIP(hipStreamSynchronize(s));
    c.info->inversions += 1;
    if (!rbt) break;
    const double bound = 8.0 * std::sqrt((double)n) * unit_roundoff(op) * std::sqrt(h[5]) *
                         std::sqrt(h[6]);
    if (!fl[0] && !fl[1] && std::isfinite(h[0]) && h[0] <= bound) {
      c.info->rbt_steps += 1;
      break;
    }
    c.info->rbt_fallbacks += 1;
    rbt = false;
  }
  if (fl[0]) return LYAP_SINGULAR;
  if (fl[1]) return LYAP_NONFINITE;
  return LYAP_OK;
}

// (A + p I)^{-1} at u_s into slot j (A^T's with the same shifts is its transpose).
int Solver::shifted_inverse(Ctx& c, int j, double p) {
  const int n = c.n;
  hipStream_t s = c.s;
  double* out = (c.us == Prec::F64) ? static_cast<double*>(c.slot(j)) : c.Ainv;
  LYAP_TRY(copy_block(s, n, n, c.A, c.lda, c.Ak, n));
  LYAP_TRY(add_diag(s, n, c.Ak, n, p));
  LYAP_TRY(checked_inverse(c, c.us, c.Ak, n, out, 0x4144495348ull + (unsigned)j));
  if (c.us != Prec::F64) {
    LYAP_TRY(absmax_exp(s, n, n, out, n, c.cexp + j, c.flags + 1, c.part));
    LYAP_TRY(cast_scaled(s, c.cstore, n, n, out, n, c.slot(j), c.cexp + j));
  } else {
    LYAP_TRY(fill_int(s, c.cexp + j, 1, 0));
  }
  return LYAP_OK;
}

// Spectral interval [a, b] of -A by power iteration (b = rho(A), a = 1 / rho(A^{-1}) with
// A^{-1} at u_s, or binary32 for the half-precision solvers; inverted like the shifted
// matrices), the Wachspress shifts for it and the cached shifted inverses.
int Solver::adi_sequence(Ctx& c) {
  const int n = c.n;
  hipStream_t s = c.s;
  double* scal = c.scal;
  c.mus.clear();
  c.K = 0;
  LYAP_TRY(specrad_est(s, n, c.A, c.lda, RHO_ITERS, scal + 15, c.vecs));
  const Prec iop = (c.us == Prec::F64) ? Prec::F64 : Prec::F32;
  LYAP_TRY(checked_inverse(c, iop, c.A, c.lda, c.Ainv, 0x494e54ull));
  LYAP_TRY(specrad_est(s, n, c.Ainv, n, RHO_ITERS, scal + 16, c.vecs));
  double h[2];
  LYAP_HIP(hipMemcpyAsync(h, scal + 15, sizeof(h), hipMemcpyDeviceToHost, s));
  LYAP_HIP(hipStreamSynchronize(s));
  const double b = h[0], a = 1.0 / h[1];
  if (!std::isfinite(a) || !std::isfinite(b) || !(a > 0.0) || !(b > 0.0)) return LYAP_NONFINITE;
  std::vector<double> p = adi_shifts(std::min(a, b), b, c.opt.adi_shifts,
                                     std::sqrt(unit_roundoff(c.us)));
  if ((int)p.size() > c.lay.slots) p = adi_shifts(std::min(a, b), b, c.lay.slots, 0.0);
  for (int j = 0; j < (int)p.size(); ++j) LYAP_TRY(shifted_inverse(c, j, p[j]));
  c.mus = p;
  c.K = (int)p.size();
  c.info->n_mu = std::min(c.K, 64);
  for (int j = 0; j < c.info->n_mu; ++j) {
    c.info->mus[j] = p[j];
    c.info->onenorm[j] = 0.0;
  }
  return LYAP_OK;
}

// The inverse sequence of A at u_s: replayed from the workspace when it holds the sequence of
// this A (content fingerprint, n, u_s, same workspace) and the call allows it, else computed.
int Solver::ensure_sequence(Ctx& c) {
  if (c.K > 0) return LYAP_OK;
  auto t0 = clk::now();
  const bool match = key_.K > 0 && key_.ws == c.base && key_.epoch == c.epoch &&
                     key_.fp == c.fp && key_.n == c.n && key_.us == c.us &&
                     key_.slots == c.lay.slots && key_.solver == c.opt.solver &&
                     key_.adi_shifts == c.opt.adi_shifts;
  if (c.may_reuse && match) {
    c.K = key_.K;
    c.mus = key_.mus;
    c.info->cache_reused = 1;
    c.info->n_mu = std::min(c.K, 64);
    for (int k = 0; k < c.info->n_mu; ++k) {
      c.info->mus[k] = key_.mus[k];
      c.info->onenorm[k] = key_.onenorm[k];
    }
  } else {
    key_ = CacheKey();
    const int code = c.opt.solver == 1 ? adi_sequence(c) : a_iteration(c);
    c.info->phase_ms[0] += ms_since(t0);
    if (code != LYAP_OK) {
      c.K = 0;
      return code;
    }
    key_.ws = c.base;
    key_.epoch = c.epoch;
    key_.fp = c.fp;
    key_.n = c.n;
    key_.us = c.us;
    key_.slots = c.lay.slots;
    key_.solver = c.opt.solver;
    key_.adi_shifts = c.opt.adi_shifts;
    key_.mus = c.mus;
    key_.onenorm.assign(c.info->onenorm, c.info->onenorm + std::min(c.K, 64));
    key_.K = c.K;
    return LYAP_OK;
  }
  c.info->phase_ms[0] += ms_since(t0);
  return LYAP_OK;
}

// -------------------------------------------------------------------- rank truncation
// RankTruncLdlt: Z = Q R, R diag(d) R^T = V Lambda V^T, keep lambda > thr max|lambda|
// (|lambda| for an indefinite problem); Z <- Q V_kept, d <- lambda_kept.
int Solver::rank_trunc(Ctx& c, double* Zb, long ldb, int& cols, std::vector<double>& d,
                       double thr, bool psd) {
  hipStream_t s = c.s;
  const int n = c.n, cap = c.cap;
  if (cols == 0) return LYAP_OK;
  const int k = std::min(n, cols);
  c.arena.reset();
  LYAP_TRY(qr_lead(s, n, cols, std::min(c.orth, cols), Zb, ldb, c.Uq, cap, c.Tq, cap, c.arena,
                   c.kt));
  LYAP_TRY(upload_d(c, d, c.dvec));
  LYAP_TRY(copy_block(s, k, cols, c.Tq, cap, c.TN, cap, c.dvec));
  GemmDesc g;
  g.M = k; g.N = k; g.K = cols;
  g.A = c.TN; g.sar = cap; g.sac = 1;
  g.B = c.Tq; g.sbr = 1; g.sbc = cap;
  g.C = c.Hm; g.ldc = cap;
  LYAP_TRY(gemm_f64(s, g));
  c.arena.reset();
  // Inside the solver only eigenvalues above thr max|lambda| are kept and the solver works
  // at u_s: accuracy relative to ||H|| (absolute rotation threshold) is what it can use;
  // relative accuracy for the discarded small eigenvalues would cost many extra sweeps.  For
  // u_s of FP16 / BF16 the rotations run in FP32 (Alg 3.2 runs at precision u_s; FP32 keeps
  // the threshold far above its own rounding).  For u_s = FP32 they stay FP64: FP32
  // rotations would leave noise eigenvalues at the size of the threshold itself.
  const bool single = c.us == Prec::F16 || c.us == Prec::BF16;
  LYAP_TRY(syev(s, k, c.Hm, cap, c.wv, c.Vm, cap, c.arena, std::max(10.0 * thr, 1e-15), nullptr,
                c.kt, false, single));
  std::vector<double> lam(k);
  LYAP_HIP(hipMemcpyAsync(lam.data(), c.wv, k * sizeof(double), hipMemcpyDeviceToHost, s));
  LYAP_HIP(hipStreamSynchronize(s));
  const double t = thr * std::fabs(lam[0]);
  std::vector<int> keep;
  for (int i = 0; i < k; ++i)
    if (psd ? (lam[i] > t) : (std::fabs(lam[i]) > t)) keep.push_back(i);
  const int r = (int)keep.size();
  d.resize(r);
  for (int i = 0; i < r; ++i) d[i] = lam[keep[i]];
  if (r > 0) {
    LYAP_HIP(hipMemcpyAsync(c.idx, keep.data(), r * sizeof(int), hipMemcpyHostToDevice, s));
    LYAP_TRY(gather_cols(s, k, r, c.Vm, cap, c.idx, c.TN, cap));
    GemmDesc z;
    z.M = n; z.N = r; z.K = k;
    z.A = c.Uq; z.sar = cap; z.sac = 1;
    z.B = c.TN; z.sbr = cap; z.sbc = 1;
    z.C = Zb; z.ldc = ldb;
    LYAP_TRY(gemm_f64(s, z));
  }
  cols = r;
  c.orth = r;  // Q V_kept has orthonormal columns
  return LYAP_OK;
}

// Split-K workspace for a tall-skinny product (n x n times n x c): the arena, which holds
// nothing between the steps that use it (every user resets it first; one stream orders the
// reuse).
static double* splitk_part(Arena& a, size_t& elems) {
  a.reset();
  elems = a.cap > 4096 ? (a.cap - 4096) / sizeof(double) : 0;
  double* p = elems ? a.take<double>(elems) : nullptr;
  if (!p) elems = 0;
  return p;
}

// ------------------------------------------------------------------ factor iteration
// eq (3.3): Z_k = [Z_{k-1}, A_{k-1}^{-1} Z_{k-1}], D_k = (mu D, D / mu) / 2, truncating
// whenever the column count exceeds floor(rho n) (threshold max(u_s, trunc_thr) relative);
// finally D <- D / 2.  The products use the
// cached inverses with operands at the solver precision: the cache holds 2^-e_k A_k^-1 and each
// column j of Z enters as 2^-f_j Z_:j rounded once to u_s, both scales undone exactly in the
// product.  Result in Zs (n x cols); the first ``orth0`` columns of L0 are orthonormal, and
// c.orth tells the same of the result.
int Solver::factor_iteration(Ctx& c, const double* L0, long ld0, int m0, int orth0,
                             const std::vector<double>& d0, bool psd, int& cols,
                             std::vector<double>& d, double trunc_thr) {
  hipStream_t s = c.s;
  const int n = c.n, cap = c.cap;
  double* Zs = c.Zs;
  LYAP_TRY(copy_block(s, n, m0, L0, ld0, Zs, cap));
  cols = m0;
  c.orth = std::min(orth0, m0);
  d = d0;
  const int trunc_at = (int)std::floor(c.opt.rho * n);
  for (int k = 0; k < c.K; ++k) {
    if (2 * cols > cap) return LYAP_CAPACITY;
    if (cols > 0) {
      GemmDesc g;
      g.M = n; g.N = cols; g.K = n;
      g.A = c.slot(k);
      if (c.trans) { g.sar = 1; g.sac = n; }  // (A_k^{-1})^T = (A_k^T)^{-1}
      else { g.sar = n; g.sac = 1; }
      g.B = Zs; g.sbr = cap; g.sbc = 1;
      g.C = Zs + cols; g.ldc = cap;
      size_t pe = 0;
      double* part = splitk_part(c.arena, pe);
      if (c.us == Prec::F64) {
        LYAP_TRY(gemm_f64(s, g, part, pe));
      } else {
        LYAP_TRY(col_exponents(s, n, cols, Zs, cap, c.colexp, c.flags + 1, c.bits));
        g.a_exp = c.cexp + k;
        g.b_colexp = c.colexp;
        LYAP_TRY(gemm_lp(s, c.us, c.cstore, Store::F64, Store::F64, g, part, pe));
      }
    }
    const double mu = c.mus[k];
    const int c0 = cols;
    d.resize(2 * c0);
    for (int i = 0; i < c0; ++i) {
      d[c0 + i] = 0.5 / mu * d[i];
      d[i] = 0.5 * mu * d[i];
    }
    cols = 2 * c0;
    if (cols > trunc_at)
      LYAP_TRY(rank_trunc(c, Zs, cap, cols, d, std::max(unit_roundoff(c.us), trunc_thr), psd));
  }
  for (double& x : d) x *= 0.5;
  return LYAP_OK;
}

// ------------------------------------------------------------------ ADI iteration
// Low-rank ADI in LDL^T form with real shifts on the cached (A + p_j I)^{-1}: W_0 = L0,
// V = (A + p I)^{-1} W (operands at u_s, as in the Newton products), W <- W - 2 p V,
// Z <- [Z, V], d <- [d, -2 p d0], until ||W diag(d0) W^T||_F <= tol ||L0 diag(d0) L0^T||_F
// with tol = max(10 u_s, trunc_thr), or opt.adi_max steps.  W is kept in FP64 in Gm
// (n x m0, leading dimension m0); its Gram matrix W^T W (in Hm) gives the residual norm.
// Result in Zs (n x cols); c.iters receives the step count.
int Solver::adi_iteration(Ctx& c, const double* L0, long ld0, int m0,
                          const std::vector<double>& d0, bool psd, int& cols,
                          std::vector<double>& d, double trunc_thr) {
  hipStream_t s = c.s;
  const int n = c.n, cap = c.cap;
  double* Zs = c.Zs;
  double* W = c.Gm;
  cols = 0;
  d.clear();
  c.orth = 0;
  c.iters = 0;
  if (m0 == 0) return LYAP_OK;
  if (m0 > n) return LYAP_CAPACITY;
  LYAP_TRY(copy_block(s, n, m0, L0, ld0, W, m0));
  LYAP_TRY(upload_d(c, d0, c.dvec2));
  auto wnorm = [&](double& out) -> int {
    GemmDesc g;
    g.M = m0; g.N = m0; g.K = n;
    g.A = W; g.sar = 1; g.sac = m0;
    g.B = W; g.sbr = m0; g.sbc = 1;
    g.C = c.Hm; g.ldc = m0;
    c.arena.reset();
    size_t welems = std::min((size_t)64 * m0 * m0, (c.arena.cap - 4096) / sizeof(double));
    double* part = c.arena.take<double>(welems);
    LYAP_TRY(gemm_f64(s, g, part, part ? welems : 0));
    LYAP_TRY(wsumsq(s, m0, c.Hm, m0, c.dvec2, c.scal + 17, c.part));
    double v[2];
    int fl = 0;
    LYAP_HIP(hipMemcpyAsync(v, c.scal + 17, sizeof(double), hipMemcpyDeviceToHost, s));
    LYAP_HIP(hipMemcpyAsync(&fl, c.flags + 1, sizeof(int), hipMemcpyDeviceToHost, s));
    LYAP_HIP(hipStreamSynchronize(s));
    if (fl) return LYAP_NONFINITE;
    out = std::sqrt(std::max(v[0], 0.0));
    return LYAP_OK;
  };
  LYAP_TRY(fill_int(s, c.flags + 1, 1, 0));
  double nrm0 = 0.0;
  LYAP_TRY(wnorm(nrm0));
  if (!std::isfinite(nrm0)) return LYAP_NONFINITE;
  if (nrm0 == 0.0) return LYAP_OK;
  const double tol = std::max(10.0 * unit_roundoff(c.us), trunc_thr);
  const double thr = std::max(unit_roundoff(c.us), trunc_thr);
  const int trunc_at = (int)std::floor(c.opt.rho * n);
  const int J = c.K;
  for (int t = 0; t < c.opt.adi_max; ++t) {
    const int j = t % J;
    const double p = c.mus[j];
    if (cols + m0 > cap) {
      LYAP_TRY(rank_trunc(c, Zs, cap, cols, d, thr, psd));
      if (cols + m0 > cap) return LYAP_CAPACITY;
    }
    GemmDesc g;
    g.M = n; g.N = m0; g.K = n;
    g.A = c.slot(j);
    if (c.trans) { g.sar = 1; g.sac = n; }  // (A + p I)^{-T} = (A^T + p I)^{-1}
    else { g.sar = n; g.sac = 1; }
    g.B = W; g.sbr = m0; g.sbc = 1;
    g.C = Zs + cols; g.ldc = cap;
    size_t pe = 0;
    double* part = splitk_part(c.arena, pe);
    if (c.us == Prec::F64) {
      LYAP_TRY(gemm_f64(s, g, part, pe));
    } else {
      LYAP_TRY(col_exponents(s, n, m0, W, m0, c.colexp, c.flags + 1, c.bits));
      g.a_exp = c.cexp + j;
      g.b_colexp = c.colexp;
      LYAP_TRY(gemm_lp(s, c.us, c.cstore, Store::F64, Store::F64, g, part, pe));
    }
    LYAP_TRY(add_block(s, n, m0, -2.0 * p, Zs + cols, cap, W, m0));
    for (int k = 0; k < m0; ++k) d.push_back(-2.0 * p * d0[k]);
    cols += m0;
    if (cols > trunc_at) LYAP_TRY(rank_trunc(c, Zs, cap, cols, d, thr, psd));
    c.iters = t + 1;
    double nrm = 0.0;
    LYAP_TRY(wnorm(nrm));
    if (!std::isfinite(nrm)) return LYAP_NONFINITE;
    if (nrm <= tol * nrm0) break;
  }
  return LYAP_OK;
}

int Solver::inner_solve(Ctx& c, const double* L0, long ld0, int m0, int orth0,
                        const std::vector<double>& d0, bool psd, int& cols,
                        std::vector<double>& d, double trunc_thr) {
  if (c.opt.solver == 1) return adi_iteration(c, L0, ld0, m0, d0, psd, cols, d, trunc_thr);
  c.iters = c.K;
  return factor_iteration(c, L0, ld0, m0, orth0, d0, psd, cols, d, trunc_thr);
}

// ||Z diag(d) Z^T||_F = sqrt(sum_ij d_i d_j (Z^T Z)_ij^2)
int Solver::xnorm(Ctx& c, const double* Zb, long ldb, int cols, const std::vector<double>& d,
                  double& out) {
  hipStream_t s = c.s;
  if (cols == 0) {
    out = 0.0;
    return LYAP_OK;
  }
  GemmDesc g;
  g.M = cols; g.N = cols; g.K = c.n;
  g.A = Zb; g.sar = 1; g.sac = ldb;
  g.B = Zb; g.sbr = ldb; g.sbc = 1;
  g.C = c.Gm; g.ldc = cols;
  c.arena.reset();
  size_t welems = std::min((size_t)64 * cols * cols, (c.arena.cap - 4096) / sizeof(double));
  double* part = c.arena.take<double>(welems);
  LYAP_TRY(gemm_f64(s, g, part, part ? welems : 0));
  LYAP_TRY(upload_d(c, d, c.dvec));
  LYAP_TRY(wsumsq(s, cols, c.Gm, cols, c.dvec, c.scal + 9, c.part));
  double v = 0.0;
  LYAP_HIP(hipMemcpyAsync(&v, c.scal + 9, sizeof(double), hipMemcpyDeviceToHost, s));
  LYAP_HIP(hipStreamSynchronize(s));
  out = std::sqrt(std::max(v, 0.0));
  return LYAP_OK;
}

// ------------------------------------------------------------ residual factorisation
// Fragment 2.3: F = [Z, AZ, L] = U T, H = T N T^T with N = [[0, D, 0], [D, 0, 0], [0, 0, S]],
// ||R||_F = ||H||_F; with want_factor, H = Q Lambda Q^T and the residual factor
// L^D = U Q_t (into Zd), S^D = Lambda_t for |lambda| >= eta_r max|lambda|.  At u_r = FP32 the
// product AZ runs on the binary32 matrix cores and U, T, H are rounded to binary32.
int Solver::res_fac(Ctx& c, const double* Zb, long ldb, int cols, const std::vector<double>& d,
                    bool want_factor, double& normR, int& rd, std::vector<double>& sd) {
  hipStream_t s = c.s;
  const int n = c.n, m = c.m, cap = c.cap;
  const int p = 2 * cols + m;
  if (p > cap) return LYAP_CAPACITY;
  const int k = std::min(n, p);
  const Store rs = store_of(c.ur);
  LYAP_TRY(copy_block(s, n, cols, Zb, ldb, c.F, cap));
  if (cols > 0) {
    GemmDesc g;
    g.M = n; g.N = cols; g.K = n;
    g.A = c.A;
    if (c.trans) { g.sar = 1; g.sac = c.lda; }
    else { g.sar = c.lda; g.sac = 1; }
    g.B = Zb; g.sbr = ldb; g.sbc = 1;
    g.C = c.F + cols; g.ldc = cap;
    size_t pe = 0;
    double* part = splitk_part(c.arena, pe);
    if (c.ur == Prec::F64) LYAP_TRY(gemm_f64(s, g, part, pe));
    else LYAP_TRY(gemm_lp(s, c.ur, Store::F64, Store::F64, Store::F64, g, part, pe));
  }
  LYAP_TRY(copy_block(s, n, m, c.L, c.ldl, c.F + 2 * cols, cap));
  c.arena.reset();
  // the plain QR when p > n: the completed basis (T = U^T F by one long product) gave a
  // residual a few units of u less accurate, which the residual factorisation cannot afford
  LYAP_TRY(qr_lead(s, n, p, c.zc_orth ? cols : 0, c.F, cap, c.Uq, cap, c.Tq, cap, c.arena, c.kt,
                   false));
  LYAP_TRY(round_block(s, rs, n, k, c.Uq, cap));
  LYAP_TRY(round_block(s, rs, k, p, c.Tq, cap));
  // TN = T N = [T2 D, T1 D, T3 S]
  LYAP_TRY(upload_d(c, d, c.dvec));
  LYAP_TRY(upload_d(c, c.svec, c.dvec2));
  if (cols > 0) {
    LYAP_TRY(copy_block(s, k, cols, c.Tq + cols, cap, c.TN, cap, c.dvec));
    LYAP_TRY(copy_block(s, k, cols, c.Tq, cap, c.TN + cols, cap, c.dvec));
  }
  LYAP_TRY(copy_block(s, k, m, c.Tq + 2 * cols, cap, c.TN + 2 * cols, cap, c.dvec2));
  GemmDesc h;
  h.M = k; h.N = k; h.K = p;
  h.A = c.TN; h.sar = cap; h.sac = 1;
  h.B = c.Tq; h.sbr = 1; h.sbc = cap;
  h.C = c.Hm; h.ldc = cap;
  LYAP_TRY(gemm_f64(s, h));
  LYAP_TRY(round_block(s, rs, k, k, c.Hm, cap));
  LYAP_TRY(sumsq(s, k, k, c.Hm, cap, c.scal + 10, c.part));
  double ss = 0.0;
  LYAP_HIP(hipMemcpyAsync(&ss, c.scal + 10, sizeof(double), hipMemcpyDeviceToHost, s));
  LYAP_HIP(hipStreamSynchronize(s));
  normR = std::sqrt(std::max(ss, 0.0));
  rd = 0;
  sd.clear();
  last_k_ = k;
  if (!want_factor) return LYAP_OK;
  return res_factor(c, rd, sd);
}

// Second half of Fragment 2.3 on the H and U left by res_fac: H = Q Lambda Q^T, keep
// |lambda| >= eta_r max|lambda| (a prefix, eigenvalues being sorted by magnitude),
// L^D = U Q_t into Zd, S^D = Lambda_t.
int Solver::res_factor(Ctx& c, int& rd, std::vector<double>& sd) {
  hipStream_t s = c.s;
  const int n = c.n, cap = c.cap, k = last_k_;
  rd = 0;
  sd.clear();
  if (k == 0) return LYAP_OK;
  c.arena.reset();
  const bool single = c.ur != Prec::F64;
  LYAP_TRY(syev(s, k, c.Hm, cap, c.wv, c.Vm, cap, c.arena, single ? 1e-6 : 1e-10, nullptr, c.kt,
                true, single));
  std::vector<double> lam(k);
  LYAP_HIP(hipMemcpyAsync(lam.data(), c.wv, k * sizeof(double), hipMemcpyDeviceToHost, s));
  LYAP_HIP(hipStreamSynchronize(s));
  const double t = c.opt.eta_r * std::fabs(lam[0]);
  while (rd < k && std::fabs(lam[rd]) >= t && lam[rd] != 0.0) ++rd;
  sd.assign(lam.begin(), lam.begin() + rd);
  for (double& x : sd) x = round_host(x, c.ur);
  if (rd > 0) {
    GemmDesc z;
    z.M = n; z.N = rd; z.K = k;
    z.A = c.Uq; z.sar = cap; z.sac = 1;
    z.B = c.Vm; z.sbr = cap; z.sbc = 1;
    z.C = c.Zd; z.ldc = cap;
    LYAP_TRY(gemm_f64(s, z));
    LYAP_TRY(round_block(s, store_of(c.ur), n, rd, c.Zd, cap));
  }
  return LYAP_OK;
}

// ------------------------------------------------------------------ solution update
// Fragment 2.4: G = [Z, Z^D] = V Gamma, K = Gamma blkdiag(D, D^D) Gamma^T = Theta Sigma Theta^T,
// keep sigma >= eta_s max|sigma| (|sigma| when the PSD projection is off);
// Z <- V Theta_t (into Zc), D <- Sigma_t.  The correction Z^D (cd columns) is read from Zcor.
// Fragment 2.2 (Cholesky type) is the same with Z^D = [Z+, Z-], D^D = (D+, -D-) and the PSD
// projection: G = [Z, Z+, Z-] scaled by the square roots of the weights gives its K.  At
// u_c = FP32 the rotations run in binary32 and V, Gamma, K are rounded to binary32; the new
// factor is stored at the working precision u.
int Solver::sol_upt(Ctx& c, int& cols, std::vector<double>& d, const double* Zcor, int cd,
                    const std::vector<double>& dd, double eta_s, bool psd) {
  hipStream_t s = c.s;
  const int n = c.n, cap = c.cap;
  const int q = cols + cd;
  if (q > cap) return LYAP_CAPACITY;
  if (q == 0) return LYAP_OK;
  const int k = std::min(n, q);
  const Store cs = store_of(c.uc);
  LYAP_TRY(copy_block(s, n, cols, c.Zc, cap, c.F, cap));
  LYAP_TRY(copy_block(s, n, cd, Zcor, cap, c.F + cols, cap));
  c.arena.reset();
  LYAP_TRY(qr_lead(s, n, q, c.zc_orth ? cols : 0, c.F, cap, c.Uq, cap, c.Tq, cap, c.arena, c.kt));
  LYAP_TRY(round_block(s, cs, n, k, c.Uq, cap));
  LYAP_TRY(round_block(s, cs, k, q, c.Tq, cap));
  std::vector<double> ups(d);
  ups.insert(ups.end(), dd.begin(), dd.end());
  LYAP_TRY(upload_d(c, ups, c.dvec));
  LYAP_TRY(copy_block(s, k, q, c.Tq, cap, c.TN, cap, c.dvec));
  GemmDesc g;
  g.M = k; g.N = k; g.K = q;
  g.A = c.TN; g.sar = cap; g.sac = 1;
  g.B = c.Tq; g.sbr = 1; g.sbc = cap;
  g.C = c.Hm; g.ldc = cap;
  LYAP_TRY(gemm_f64(s, g));
  LYAP_TRY(round_block(s, cs, k, k, c.Hm, cap));
  c.arena.reset();
  const bool single = c.uc != Prec::F64;
  LYAP_TRY(syev(s, k, c.Hm, cap, c.wv, c.Vm, cap, c.arena, single ? 1e-6 : 0.0, nullptr, c.kt,
                true, single));
  std::vector<double> sig(k);
  LYAP_HIP(hipMemcpyAsync(sig.data(), c.wv, k * sizeof(double), hipMemcpyDeviceToHost, s));
  LYAP_HIP(hipStreamSynchronize(s));
  const double t = eta_s * std::fabs(sig[0]);
  std::vector<int> keep;
  for (int i = 0; i < k; ++i)
    if (psd ? (sig[i] >= t && sig[i] > 0.0) : (std::fabs(sig[i]) >= t && sig[i] != 0.0))
      keep.push_back(i);
  const int r = (int)keep.size();
  d.resize(r);
  for (int i = 0; i < r; ++i) d[i] = round_host(sig[keep[i]], c.u);
  if (r > 0) {
    LYAP_HIP(hipMemcpyAsync(c.idx, keep.data(), r * sizeof(int), hipMemcpyHostToDevice, s));
    LYAP_TRY(gather_cols(s, k, r, c.Vm, cap, c.idx, c.TN, cap));
    GemmDesc z;
    z.M = n; z.N = r; z.K = k;
    z.A = c.Uq; z.sar = cap; z.sac = 1;
    z.B = c.TN; z.sbr = cap; z.sbc = 1;
    z.C = c.Zc; z.ldc = cap;
    LYAP_TRY(gemm_f64(s, z));
    LYAP_TRY(round_block(s, store_of(c.u), n, r, c.Zc, cap));
  }
  cols = r;
  c.zc_orth = c.u == Prec::F64;  // U Theta_t (orthonormal to working precision)
  return LYAP_OK;
}

// ------------------------------------------------------------------ refinement loop
// Alg 2.1 / 2.2 from the current iterate (Zc, d): residual test (eq 4.1) against tau_I, the
// early stop of eq (4.2), then the correction solve(s) reusing the cached inverses and the
// projected update.  ``status`` receives OK / NOT_CONVERGED / STAGNATED / NONFINITE; the
// return value is a hard error code (or LYAP_OK).
int Solver::refine_loop(Ctx& c, int& cols, std::vector<double>& d, int steps, int& status) {
  hipStream_t s = c.s;
  const int n = c.n, cap = c.cap;
  lyap_info* info = c.info;
  const double eta_s = c.opt.eta_s > 0.0 ? c.opt.eta_s : 10.0 * unit_roundoff(c.u);
  std::vector<double> hist;  // residuals of this stage (the eq (4.2) test looks at these)
  bool inexact = c.opt.adaptive != 0;
  status = LYAP_NOT_CONVERGED;
  for (int i = 1; i <= steps; ++i) {
    auto t0 = clk::now();
    double normR = 0.0, nx = 0.0;
    int rd = 0;
    std::vector<double> sd;
    LYAP_TRY(res_fac(c, c.Zc, cap, cols, d, false, normR, rd, sd));
    LYAP_TRY(xnorm(c, c.Zc, cap, cols, d, nx));
    // eq (4.1); W = 0 with X = 0 is the exact solution (R = 0): res 0, not 0 / 0
    const double den = c.normW + 2.0 * nx * c.normA;
    const double res = den > 0.0 ? normR / den : (normR == 0.0 ? 0.0 : INFINITY);
    if (info->n_res < 64) info->res_hist[info->n_res++] = res;
    info->res = res;
    hist.push_back(res);
    // the inexact thresholds only drop what the next correction fixes: a step that contracts
    // the residual by less than half switches them off for the rest of the refinement
    if (inexact && hist.size() >= 2 && res > 0.5 * hist[hist.size() - 2]) inexact = false;
    info->phase_ms[4] += ms_since(t0);
    if (!std::isfinite(res)) {
      status = LYAP_NONFINITE;
      return LYAP_OK;
    }
    if (res <= c.opt.tol) {
      status = LYAP_OK;
      return LYAP_OK;
    }
    if (!c.opt.refine) return LYAP_OK;
    const int nh = (int)hist.size();
    if (nh >= 3 && hist[nh - 1] > c.opt.theta * hist[nh - 2] &&
        hist[nh - 2] > c.opt.theta * hist[nh - 3]) {
      status = LYAP_STAGNATED;
      return LYAP_OK;
    }
    if (i == steps) return LYAP_OK;
    // the inverse sequence (computed on demand when the refinement started from a given X_0)
    {
      const int code = ensure_sequence(c);
      if (code != LYAP_OK) {
        status = code;
        return LYAP_OK;
      }
    }
    // residual factor (Fragment 2.3, truncated at eta_r), from the H and U just formed
    t0 = clk::now();
    LYAP_TRY(res_factor(c, rd, sd));
    info->phase_ms[4] += ms_since(t0);
    // correction equation(s) at the solver precision, reusing the cached inverses; with
    // adaptive tolerances the correction is truncated at eta_r / 10 (its right-hand side is
    // itself truncated at eta_r) and the update at omega res_i
    const double inner_thr = inexact ? c.opt.eta_r / 10.0 : 0.0;
    const double eta_i = inexact ? std::max(eta_s, c.opt.omega * res) : eta_s;
    t0 = clk::now();
    int cd = 0;
    std::vector<double> dd;
    const double* Zcor = c.Zs;
    if (!c.chol) {
      // the correction is solved for 2^-e W^D (largest |S^D| in [1/2, 1)) and scaled back
      int e = 0;
      if (rd > 0) std::frexp(std::fabs(sd[0]), &e);
      std::vector<double> sds(sd);
      for (double& x : sds) x = std::ldexp(x, -e);
      LYAP_TRY(inner_solve(c, c.Zd, cap, rd, rd, sds, false, cd, dd, inner_thr));  // U Q_t
      for (double& x : dd) x = std::ldexp(x, e);
    } else {
      // Fragment 2.1: R = L+ L+^T - L- L-^T with L+- = U Q_+- |Lambda_+-|^(1/2), here as
      // (U Q_+-, |lambda|); the two correction equations (Alg 2.1) share the inverse sequence
      // and are truncated independently.  U Q_t is gathered into F (positive part first),
      // and the corrections Z+ and Z- are collected in Zd.
      std::vector<int> order;
      std::vector<double> dp, dm;
      for (int j = 0; j < rd; ++j)
        if (sd[j] > 0.0) { order.push_back(j); dp.push_back(sd[j]); }
      const int rp = (int)order.size();
      for (int j = 0; j < rd; ++j)
        if (sd[j] < 0.0) { order.push_back(j); dm.push_back(-sd[j]); }
      const int rm = (int)order.size() - rp;
      double* Fb = c.F;
      double* Zpm = c.Zd;
      if (!order.empty()) {
        LYAP_HIP(hipMemcpyAsync(c.idx, order.data(), order.size() * sizeof(int),
                                hipMemcpyHostToDevice, s));
        LYAP_TRY(gather_cols(s, n, (int)order.size(), c.Zd, cap, c.idx, Fb, cap));
      }
      int cp = 0, cm = 0;
      std::vector<double> ddp, ddm;
      LYAP_TRY(inner_solve(c, Fb, cap, rp, rp, dp, true, cp, ddp, inner_thr));
      const int iters_p = c.iters;
      LYAP_TRY(copy_block(s, n, cp, c.Zs, cap, Zpm, cap));
      LYAP_TRY(inner_solve(c, Fb + rp, cap, rm, rm, dm, true, cm, ddm, inner_thr));
      c.iters = std::max(c.iters, iters_p);
      if (cp + cm > cap) return LYAP_CAPACITY;
      LYAP_TRY(copy_block(s, n, cm, c.Zs, cap, Zpm + cp, cap));
      cd = cp + cm;
      dd = ddp;
      for (double x : ddm) dd.push_back(-x);
      Zcor = Zpm;
    }
    // the correction is stored at the working precision
    LYAP_TRY(round_block(s, store_of(c.u), n, cd, const_cast<double*>(Zcor), cap));
    for (double& x : dd) x = round_host(x, c.u);
    LYAP_HIP(hipStreamSynchronize(s));
    info->phase_ms[2] += ms_since(t0);
    info->newton_total += c.iters;
    info->newton_max = std::max(info->newton_max, c.iters);
    info->refinements += 1;
    // projected solution update (Fragment 2.4; Fragment 2.2 for the Cholesky type)
    t0 = clk::now();
    LYAP_TRY(sol_upt(c, cols, d, Zcor, cd, dd, eta_i, c.psd));
    info->phase_ms[5] += ms_since(t0);
  }
  return LYAP_OK;
}

// ------------------------------------------------------------------------ driver
int Solver::solve(hipStream_t s, char* ws, size_t ws_bytes, unsigned long ws_epoch, int n, int m,
                  const double* A, int lda, const double* L, int ldl, const double* S, int lds,
                  const lyap_precisions& prec, const lyap_options& opt, const double* Z0,
                  int ldz0, const double* D0, int r0, double* Z, int ldz, int z_cap, double* D,
                  int* rank, lyap_info* info, bool adjoint, bool timing) {
  const auto t_start = clk::now();
  Ctx c;
  c.s = s;
  c.base = ws;
  c.epoch = ws_epoch;
  c.us = (Prec)prec.u_s;
  c.u = (Prec)prec.u;
  c.ur = (Prec)prec.u_r;
  c.uc = (Prec)prec.u_c;
  c.lay = solver_layout(n, m, c.us, opt);
  if (!ws || ws_bytes < c.lay.total || ((uintptr_t)ws & 255) != 0) return LYAP_WORKSPACE;
  const Layout& ly = c.lay;
  c.arena.base = ws + ly.arena;
  c.arena.cap = ly.arena_bytes;
  c.arena.top = 0;
  c.cache = ws + ly.cache;
  c.cexp = c.at<int>(ly.cexp);
  c.Ak = c.at<double>(ly.Ak);
  c.An = c.at<double>(ly.An);
  c.Ainv = c.at<double>(ly.Ainv);
  c.colsum = c.at<double>(ly.colsum);
  c.part = c.at<double>(ly.part);
  c.scal = c.at<double>(ly.scal);
  c.flags = c.at<int>(ly.flags);
  c.fpr = c.at<unsigned long long>(ly.fpr);
  c.vecs = c.at<double>(ly.vecs);
  c.dvec = c.at<double>(ly.dvec);
  c.dvec2 = c.at<double>(ly.dvec2);
  c.idx = c.at<int>(ly.idx);
  c.colexp = c.at<int>(ly.colexp);
  c.bits = c.at<unsigned long long>(ly.bits);
  c.Zs = c.at<double>(ly.Zs);
  c.Zc = c.at<double>(ly.Zc);
  c.Zd = c.at<double>(ly.Zd);
  c.F = c.at<double>(ly.F);
  c.Uq = c.at<double>(ly.Uq);
  c.Tq = c.at<double>(ly.Tq);
  c.TN = c.at<double>(ly.TN);
  c.Hm = c.at<double>(ly.Hm);
  c.Vm = c.at<double>(ly.Vm);
  c.Gm = c.at<double>(ly.Gm);
  c.wv = c.at<double>(ly.wv);
  c.n = n;
  c.m = m;
  c.A = A;
  c.lda = lda;
  c.L = L;
  c.ldl = ldl;
  c.cstore = store_of(c.us);
  c.opt = opt;
  c.info = info;
  c.trans = adjoint;
  c.cap = ly.cap;
  kt_.reset();
  c.kt = timing ? &kt_ : nullptr;
  const int cap = c.cap;

  // A0: S.  A diagonal S is taken as given; a full symmetric S = Q_s diag(s) Q_s^T is
  // diagonalised on the device once and L replaced by L Q_s (an exact orthogonal change:
  // L S L^T = (L Q_s) diag(s) (L Q_s)^T).
  c.svec.assign(m, 1.0);
  if (S && lds == 0) {
    LYAP_HIP(hipMemcpyAsync(c.svec.data(), S, m * sizeof(double), hipMemcpyDeviceToHost, s));
    LYAP_HIP(hipStreamSynchronize(s));
  } else if (S) {
    double* Sm = c.at<double>(ly.Sm);
    double* Sv = c.at<double>(ly.Sv);
    double* Sw = c.at<double>(ly.Sw);
    double* Lq = c.at<double>(ly.Lq);
    LYAP_TRY(copy_block(s, m, m, S, lds, Sm, m));
    c.arena.reset();
    LYAP_TRY(syev(s, m, Sm, m, Sw, Sv, m, c.arena, 0.0, nullptr, nullptr, true, false));
    GemmDesc g;
    g.M = n; g.N = m; g.K = m;
    g.A = L; g.sar = ldl; g.sac = 1;
    g.B = Sv; g.sbr = m; g.sbc = 1;
    g.C = Lq; g.ldc = m;
    LYAP_TRY(gemm_f64(s, g));
    LYAP_HIP(hipMemcpyAsync(c.svec.data(), Sw, m * sizeof(double), hipMemcpyDeviceToHost, s));
    LYAP_HIP(hipStreamSynchronize(s));
    c.L = Lq;
    c.ldl = m;
  }
  for (double v : c.svec)
    if (!std::isfinite(v)) return LYAP_BADARG;
  bool all_nonneg = true;
  for (double v : c.svec) all_nonneg = all_nonneg && v >= 0.0;
  c.chol = opt.form == 1;
  c.psd = c.chol || (opt.psd < 0 ? all_nonneg : (opt.psd != 0));

  // ||A||_F, ||W||_F = sqrt(tr((L^T L S)^2)) and the content fingerprint of A
  LYAP_TRY(sumsq(s, n, n, A, lda, c.scal + 11, c.part));
  {
    GemmDesc g;
    g.M = m; g.N = m; g.K = n;
    g.A = c.L; g.sar = 1; g.sac = c.ldl;
    g.B = c.L; g.sbr = c.ldl; g.sbc = 1;
    g.C = c.Gm; g.ldc = m;
    LYAP_TRY(gemm_f64(s, g));
    LYAP_TRY(upload_d(c, c.svec, c.dvec2));
    LYAP_TRY(wsumsq(s, m, c.Gm, m, c.dvec2, c.scal + 12, c.part));
    LYAP_TRY(fingerprint(s, n, n, A, lda, c.fpr));
    double h2[2];
    LYAP_HIP(hipMemcpyAsync(h2, c.scal + 11, sizeof(h2), hipMemcpyDeviceToHost, s));
    LYAP_HIP(hipMemcpyAsync(&c.fp, c.fpr, sizeof(c.fp), hipMemcpyDeviceToHost, s));
    LYAP_HIP(hipStreamSynchronize(s));
    c.normA = std::sqrt(h2[0]);
    c.normW = std::sqrt(std::max(h2[1], 0.0));
    if (!std::isfinite(c.normA) || !std::isfinite(c.normW)) return LYAP_BADARG;
  }
  const bool warm = r0 >= 0;
  c.may_reuse = opt.reuse > 0 || (opt.reuse < 0 && (adjoint || warm));
  info->u_s_final = (int)c.us;

  int cols = 0;
  std::vector<double> d;
  int status = LYAP_OK;
  int refinements_left = opt.refine ? std::max(opt.i_max, 1) : 1;
  bool fresh = !warm;
  if (warm) {
    // X_0 = Z0 diag(D0) Z0^T, stored at the working precision
    if (r0 > cap) return LYAP_CAPACITY;
    d.assign(r0, 0.0);
    if (r0 > 0) {
      LYAP_TRY(copy_block(s, n, r0, Z0, ldz0, c.Zc, cap));
      LYAP_TRY(round_block(s, store_of(c.u), n, r0, c.Zc, cap));
      LYAP_HIP(hipMemcpyAsync(d.data(), D0, r0 * sizeof(double), hipMemcpyDeviceToHost, s));
      LYAP_HIP(hipStreamSynchronize(s));
      for (double& x : d) {
        if (!std::isfinite(x)) return LYAP_BADARG;
        x = round_host(x, c.u);
      }
    }
    cols = r0;
    c.zc_orth = false;
  }
  for (;;) {
    int code = LYAP_OK;
    if (fresh) {
      // first solve (Alg 2.2, line 1)
      code = ensure_sequence(c);
      if (code == LYAP_OK) {
        auto t0 = clk::now();
        LYAP_TRY(inner_solve(c, c.L, c.ldl, m, 0, c.svec, c.psd, cols, d));
        // the factor counts as orthonormal for the FP64 steps only when the truncation that
        // made it rotated in FP64: binary32 rotations (fp16 / bf16 solvers) leave it
        // orthonormal to about 1e-6, and the residual factorisation's QR would then assume
        // an orthonormal leading block that is not one
        const bool f64_rotations = !(c.us == Prec::F16 || c.us == Prec::BF16);
        c.zc_orth = cols > 0 && c.orth >= cols && c.u == Prec::F64 && f64_rotations;
        LYAP_TRY(copy_block(s, n, cols, c.Zs, cap, c.Zc, cap));
        LYAP_TRY(round_block(s, store_of(c.u), n, cols, c.Zc, cap));
        for (double& x : d) x = round_host(x, c.u);
        LYAP_HIP(hipStreamSynchronize(s));
        info->phase_ms[2] += ms_since(t0);
        info->newton_total += c.iters;
        info->newton_max = std::max(info->newton_max, c.iters);
      }
    }
    if (code == LYAP_OK) {
      const int before = info->refinements;
      LYAP_TRY(refine_loop(c, cols, d, refinements_left, code));
      refinements_left = std::max(1, refinements_left - (info->refinements - before));
    }
    // precision escalation: a stage that stagnated, overflowed, hit an exact zero pivot or
    // ran out of steps at a reduced solver precision is continued one precision up
    const bool escalatable = code == LYAP_STAGNATED || code == LYAP_NOT_CONVERGED ||
                             code == LYAP_NONFINITE || code == LYAP_SINGULAR;
    if (!(opt.escalate && opt.refine && escalatable &&
          unit_roundoff(c.us) > unit_roundoff(c.u))) {
      status = code;
      break;
    }
    const bool have_iterate = code == LYAP_STAGNATED || code == LYAP_NOT_CONVERGED;
    c.us = next_up(c.us);
    c.cstore = store_of(c.us);
    c.K = 0;
    c.mus.clear();
    info->escalations += 1;
    info->u_s_final = (int)c.us;
    fresh = !(have_iterate && cols > 0);
    if (fresh) {
      cols = 0;
      d.clear();
    }
  }
  info->rank = cols;
  *rank = cols;
  if (status != LYAP_OK && status != LYAP_NOT_CONVERGED && status != LYAP_STAGNATED)
    return status;
  if (cols > z_cap) return LYAP_CAPACITY;
  if (!c.chol) {
    LYAP_TRY(copy_block(s, n, cols, c.Zc, cap, Z, ldz));
    if (cols > 0)
      LYAP_HIP(hipMemcpyAsync(D, d.data(), cols * sizeof(double), hipMemcpyHostToDevice, s));
  } else if (cols > 0) {
    // Cholesky-type factor Z diag(d)^(1/2) (d >= 0 after the PSD projection), D = 1
    std::vector<double> sq(cols), ones(cols, 1.0);
    for (int i = 0; i < cols; ++i) sq[i] = std::sqrt(std::max(d[i], 0.0));
    LYAP_TRY(upload_d(c, sq, c.dvec));
    LYAP_TRY(copy_block(s, n, cols, c.Zc, cap, Z, ldz, c.dvec));
    LYAP_HIP(hipMemcpyAsync(D, ones.data(), cols * sizeof(double), hipMemcpyHostToDevice, s));
  }
  LYAP_HIP(hipStreamSynchronize(s));
  if (kt_.collect() == LYAP_OK) {
    for (int f = 0; f < KernTimer::NF; ++f) {
      info->kern_ms[f] = kt_.ms[f];
      info->kern_work[f] = kt_.work[f];
      info->kern_calls[f] = kt_.calls[f];
    }
  }
  info->phase_ms[7] = ms_since(t_start);
  return status;
}

}  // namespace lyap
