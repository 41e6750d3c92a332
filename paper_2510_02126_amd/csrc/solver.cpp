// Host driver of the solver: the scaled sign-function Newton A-iteration with its cached
// sequence of inverses (Section 3.4), the factored LDL^T iteration (eq 3.3, Alg 3.2) with
// RankTruncLdlt, and the mixed-precision iterative refinement of Alg 2.2 with the residual
// factorisation (Fragment 2.3) and the projected solution update (Fragment 2.4).
//
// Every matrix operation runs in the library's HIP kernels; the host only keeps scalars
// (the scalings mu_k, stopping quantities, the diagonal factors D, kept-index lists) and
// decides ranks and stops from them.  Tall factors are row-major n x cols with a common
// leading dimension ``cap``.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
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
  DevBuf* all[] = {&Ak_, &An_, &Ainv_, &colsum_, &part_, &scal_, &dvec_, &dvec2_, &idx_, &Zs_,
                   &Zc_, &Zd_, &F_, &Uq_, &Tq_, &TN_, &Hm_, &Vm_, &wv_, &Gm_};
  for (DevBuf* b : all) b->release();
  for (auto& b : cache_) b.release();
  cache_.clear();
  kt_.release();
}

namespace {

using clk = std::chrono::steady_clock;

double ms_since(clk::time_point t0) {
  return std::chrono::duration<double, std::milli>(clk::now() - t0).count();
}

Store store_of(Prec p) {
  switch (p) {
    case Prec::F64: return Store::F64;
    case Prec::F32: return Store::F32;
    case Prec::F16: return Store::F16;
    case Prec::BF16: return Store::BF16;
  }
  return Store::F64;
}

size_t store_bytes(Store s) {
  return s == Store::F64 ? 8 : (s == Store::F32 ? 4 : 2);
}

}  // namespace

struct Solver::Ctx {
  hipStream_t s;
  Arena* ws;
  int* flags;
  int n, m;
  const double* A;
  long lda;
  const double* L;
  long ldl;
  Prec us;
  Store cstore;
  lyap_options opt;
  bool psd;
  std::vector<double> svec;
  int cap;
  int K = 0;
  std::vector<double> mus;
  double normA = 0.0, normW = 0.0;
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
};

int Solver::upload_d(Ctx& c, const std::vector<double>& d, double* dst) {
  if (d.empty()) return LYAP_OK;
  LYAP_HIP(hipMemcpyAsync(dst, d.data(), d.size() * sizeof(double), hipMemcpyHostToDevice, c.s));
  return LYAP_OK;
}

// ---------------------------------------------------------------------------- A-iteration
// eq (3.1a) with Frobenius scaling; stop when ||A_k + I||_1 <= tau_N = 10 sqrt(n u_s), or
// when scaling is already off and delta_k > delta_{k-1}/2; the step that meets the test is
// followed by one further step.  Scaling is switched off for good once delta_k < delta_off.
int Solver::a_iteration(Ctx& c) {
  const int n = c.n;
  hipStream_t s = c.s;
  double* Ak = Ak_.as<double>();
  double* An = An_.as<double>();
  double* scal = c.scal;
  LYAP_TRY(copy_block(s, n, n, c.A, c.lda, Ak, n));
  LYAP_TRY(sumsq(s, n, n, Ak, n, scal + 0, c.part));
  const double tau = 10.0 * std::sqrt(n * unit_roundoff(c.us));
  bool scaling = true;
  int countdown = -1;
  double delta_prev = -1.0;
  double last_onenorm = INFINITY;
  bool stopped = false;
  const double* a_ss = scal + 0;
  for (int k = 1; k <= c.opt.k_max; ++k) {
    if ((int)cache_.size() < k) cache_.emplace_back();
    size_t eb = store_bytes(c.cstore);
    LYAP_TRY(cache_[k - 1].ensure((size_t)n * n * eb));
    double* out = (c.us == Prec::F64) ? cache_[k - 1].as<double>() : Ainv_.as<double>();
    LYAP_TRY(fill_int(s, c.flags, 2, 0));
    c.ws->reset();
    // ||A_{k-1} + I||_1 < 1 makes A_{k-1} strictly column diagonally dominant: partial
    // pivoting would pick the diagonal, so the pivot search is skipped (same result)
    const bool pivot = !(last_onenorm < 1.0);
    LYAP_TRY(invert(s, c.us, n, Ak, n, out, n, *c.ws, c.flags, pivot, c.kt));
    if (c.us != Prec::F64) LYAP_TRY(cast_store(s, c.cstore, n, n, out, n, cache_[k - 1].p));
    LYAP_TRY(sumsq(s, n, n, out, n, scal + 1, c.part));
    LYAP_TRY(newton_mu(s, scal + 1, a_ss, scaling ? 1 : 0, scal + 2));
    LYAP_TRY(newton_update(s, n, Ak, n, out, n, scal + 2, An, n, scal + 3,
                           colsum_.as<double>(), c.part));
    double h[6];
    int fl[2];
    LYAP_HIP(hipMemcpyAsync(h, scal, sizeof(h), hipMemcpyDeviceToHost, s));
    LYAP_HIP(hipMemcpyAsync(fl, c.flags, sizeof(fl), hipMemcpyDeviceToHost, s));
    LYAP_HIP(hipStreamSynchronize(s));
    if (fl[0]) return LYAP_SINGULAR;
    const double mu = h[2], dsq = h[3], anew = h[4], onenorm = h[5];
    if (fl[1] || !std::isfinite(mu) || !std::isfinite(anew) || !std::isfinite(onenorm))
      return LYAP_NONFINITE;
    const double delta = std::sqrt(dsq / anew);
    c.mus.push_back(mu);
    if (k <= 64) {
      c.info->mus[k - 1] = mu;
      c.info->onenorm[k - 1] = onenorm;
      c.info->n_mu = k;
    }
    std::swap(Ak, An);
    std::swap(Ak_, An_);
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

// -------------------------------------------------------------------- rank truncation
// RankTruncLdlt: Z = Q R, R diag(d) R^T = V Lambda V^T, keep lambda > thr max|lambda|
// (|lambda| for an indefinite problem); Z <- Q V_kept, d <- lambda_kept.
int Solver::rank_trunc(Ctx& c, double* Zb, long ldb, int& cols, std::vector<double>& d,
                       double thr, bool psd) {
  hipStream_t s = c.s;
  const int n = c.n, cap = c.cap;
  if (cols == 0) return LYAP_OK;
  const int k = std::min(n, cols);
  double* Uq = Uq_.as<double>();
  double* Tq = Tq_.as<double>();
  double* TN = TN_.as<double>();
  double* Hm = Hm_.as<double>();
  double* Vm = Vm_.as<double>();
  double* wv = wv_.as<double>();
  c.ws->reset();
  LYAP_TRY(qr_lead(s, n, cols, std::min(c.orth, cols), Zb, ldb, Uq, cap, Tq, cap, *c.ws, c.kt));
  LYAP_TRY(upload_d(c, d, dvec_.as<double>()));
  LYAP_TRY(copy_block(s, k, cols, Tq, cap, TN, cap, dvec_.as<double>()));
  GemmDesc g;
  g.M = k; g.N = k; g.K = cols;
  g.A = TN; g.sar = cap; g.sac = 1;
  g.B = Tq; g.sbr = 1; g.sbc = cap;
  g.C = Hm; g.ldc = cap;
  LYAP_TRY(gemm_f64(s, g));
  c.ws->reset();
  // Inside the solver only eigenvalues above thr max|lambda| are kept and the solver works
  // at u_s: accuracy relative to ||H|| (absolute rotation threshold) is what it can use;
  // relative accuracy for the discarded small eigenvalues would cost many extra sweeps.  For
  // u_s of FP16 / BF16 the rotations run in FP32 (Alg 3.2 runs at precision u_s; FP32 keeps
  // the threshold far above its own rounding).  For u_s = FP32 they stay FP64: FP32
  // rotations would leave noise eigenvalues at the size of the threshold itself.
  const bool single = c.us == Prec::F16 || c.us == Prec::BF16;
  LYAP_TRY(syev(s, k, Hm, cap, wv, Vm, cap, *c.ws, std::max(10.0 * thr, 1e-15), nullptr, c.kt,
                false, single));
  std::vector<double> lam(k);
  LYAP_HIP(hipMemcpyAsync(lam.data(), wv, k * sizeof(double), hipMemcpyDeviceToHost, s));
  LYAP_HIP(hipStreamSynchronize(s));
  const double t = thr * std::fabs(lam[0]);
  std::vector<int> keep;
  for (int i = 0; i < k; ++i)
    if (psd ? (lam[i] > t) : (std::fabs(lam[i]) > t)) keep.push_back(i);
  const int r = (int)keep.size();
  d.resize(r);
  for (int i = 0; i < r; ++i) d[i] = lam[keep[i]];
  if (r > 0) {
    LYAP_HIP(hipMemcpyAsync(idx_.p, keep.data(), r * sizeof(int), hipMemcpyHostToDevice, s));
    LYAP_TRY(gather_cols(s, k, r, Vm, cap, idx_.as<int>(), TN, cap));
    GemmDesc z;
    z.M = n; z.N = r; z.K = k;
    z.A = Uq; z.sar = cap; z.sac = 1;
    z.B = TN; z.sbr = cap; z.sbc = 1;
    z.C = Zb; z.ldc = ldb;
    LYAP_TRY(gemm_f64(s, z));
  }
  cols = r;
  c.orth = r;  // Q V_kept has orthonormal columns
  return LYAP_OK;
}

// ------------------------------------------------------------------ factor iteration
// eq (3.3): Z_k = [Z_{k-1}, A_{k-1}^{-1} Z_{k-1}], D_k = (mu D, D / mu) / 2, truncating
// whenever the column count exceeds floor(rho n); finally D <- D / 2.  The products use the
// cached inverses with operands at the solver precision.  Result in Zs (n x cols); the first
// ``orth0`` columns of L0 are orthonormal, and c.orth tells the same of the result.
int Solver::factor_iteration(Ctx& c, const double* L0, long ld0, int m0, int orth0,
                             const std::vector<double>& d0, bool psd, int& cols,
                             std::vector<double>& d) {
  hipStream_t s = c.s;
  const int n = c.n, cap = c.cap;
  double* Zs = Zs_.as<double>();
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
      g.A = cache_[k].p;
      if (c.trans) { g.sar = 1; g.sac = n; }  // (A_k^{-1})^T = (A_k^T)^{-1}
      else { g.sar = n; g.sac = 1; }
      g.B = Zs; g.sbr = cap; g.sbc = 1;
      g.C = Zs + cols; g.ldc = cap;
      if (c.us == Prec::F64) LYAP_TRY(gemm_f64(s, g));
      else LYAP_TRY(gemm_lp(s, c.us, c.cstore, Store::F64, Store::F64, g));
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
      LYAP_TRY(rank_trunc(c, Zs, cap, cols, d, unit_roundoff(c.us), psd));
  }
  for (double& x : d) x *= 0.5;
  return LYAP_OK;
}

// ||Z diag(d) Z^T||_F = sqrt(sum_ij d_i d_j (Z^T Z)_ij^2)
int Solver::xnorm(Ctx& c, const double* Zb, long ldb, int cols, const std::vector<double>& d,
                  double& out) {
  hipStream_t s = c.s;
  if (cols == 0) {
    out = 0.0;
    return LYAP_OK;
  }
  double* Gm = Gm_.as<double>();
  GemmDesc g;
  g.M = cols; g.N = cols; g.K = c.n;
  g.A = Zb; g.sar = 1; g.sac = ldb;
  g.B = Zb; g.sbr = ldb; g.sbc = 1;
  g.C = Gm; g.ldc = cols;
  c.ws->reset();
  size_t welems = std::min((size_t)64 * cols * cols, (c.ws->cap - 4096) / sizeof(double));
  double* part = c.ws->take<double>(welems);
  LYAP_TRY(gemm_f64(s, g, part, part ? welems : 0));
  LYAP_TRY(upload_d(c, d, dvec_.as<double>()));
  LYAP_TRY(wsumsq(s, cols, Gm, cols, dvec_.as<double>(), c.scal + 9, c.part));
  double v = 0.0;
  LYAP_HIP(hipMemcpyAsync(&v, c.scal + 9, sizeof(double), hipMemcpyDeviceToHost, s));
  LYAP_HIP(hipStreamSynchronize(s));
  out = std::sqrt(std::max(v, 0.0));
  return LYAP_OK;
}

// ------------------------------------------------------------ residual factorisation
// Fragment 2.3: F = [Z, AZ, L] = U T, H = T N T^T with N = [[0, D, 0], [D, 0, 0], [0, 0, S]],
// ||R||_F = ||H||_F; with want_factor, H = Q Lambda Q^T and the residual factor
// L^D = U Q_t (into Zd), S^D = Lambda_t for |lambda| >= eta_r max|lambda|.
int Solver::res_fac(Ctx& c, const double* Zb, long ldb, int cols, const std::vector<double>& d,
                    bool want_factor, double& normR, int& rd, std::vector<double>& sd) {
  hipStream_t s = c.s;
  const int n = c.n, m = c.m, cap = c.cap;
  const int p = 2 * cols + m;
  if (p > cap) return LYAP_CAPACITY;
  const int k = std::min(n, p);
  double* F = F_.as<double>();
  double* Uq = Uq_.as<double>();
  double* Tq = Tq_.as<double>();
  double* TN = TN_.as<double>();
  double* Hm = Hm_.as<double>();
  LYAP_TRY(copy_block(s, n, cols, Zb, ldb, F, cap));
  if (cols > 0) {
    GemmDesc g;
    g.M = n; g.N = cols; g.K = n;
    g.A = c.A;
    if (c.trans) { g.sar = 1; g.sac = c.lda; }
    else { g.sar = c.lda; g.sac = 1; }
    g.B = Zb; g.sbr = ldb; g.sbc = 1;
    g.C = F + cols; g.ldc = cap;
    LYAP_TRY(gemm_f64(s, g));
  }
  LYAP_TRY(copy_block(s, n, m, c.L, c.ldl, F + 2 * cols, cap));
  c.ws->reset();
  LYAP_TRY(qr_lead(s, n, p, c.zc_orth ? cols : 0, F, cap, Uq, cap, Tq, cap, *c.ws, c.kt));
  // TN = T N = [T2 D, T1 D, T3 S]
  LYAP_TRY(upload_d(c, d, dvec_.as<double>()));
  LYAP_TRY(upload_d(c, c.svec, dvec2_.as<double>()));
  if (cols > 0) {
    LYAP_TRY(copy_block(s, k, cols, Tq + cols, cap, TN, cap, dvec_.as<double>()));
    LYAP_TRY(copy_block(s, k, cols, Tq, cap, TN + cols, cap, dvec_.as<double>()));
  }
  LYAP_TRY(copy_block(s, k, m, Tq + 2 * cols, cap, TN + 2 * cols, cap, dvec2_.as<double>()));
  GemmDesc h;
  h.M = k; h.N = k; h.K = p;
  h.A = TN; h.sar = cap; h.sac = 1;
  h.B = Tq; h.sbr = 1; h.sbc = cap;
  h.C = Hm; h.ldc = cap;
  LYAP_TRY(gemm_f64(s, h));
  LYAP_TRY(sumsq(s, k, k, Hm, cap, c.scal + 10, c.part));
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
  double* Uq = Uq_.as<double>();
  double* Hm = Hm_.as<double>();
  double* Vm = Vm_.as<double>();
  double* wv = wv_.as<double>();
  rd = 0;
  sd.clear();
  if (k == 0) return LYAP_OK;
  c.ws->reset();
  LYAP_TRY(syev(s, k, Hm, cap, wv, Vm, cap, *c.ws, 1e-10, nullptr, c.kt));
  std::vector<double> lam(k);
  LYAP_HIP(hipMemcpyAsync(lam.data(), wv, k * sizeof(double), hipMemcpyDeviceToHost, s));
  LYAP_HIP(hipStreamSynchronize(s));
  const double t = c.opt.eta_r * std::fabs(lam[0]);
  while (rd < k && std::fabs(lam[rd]) >= t && lam[rd] != 0.0) ++rd;
  sd.assign(lam.begin(), lam.begin() + rd);
  if (rd > 0) {
    GemmDesc z;
    z.M = n; z.N = rd; z.K = k;
    z.A = Uq; z.sar = cap; z.sac = 1;
    z.B = Vm; z.sbr = cap; z.sbc = 1;
    z.C = Zd_.as<double>(); z.ldc = cap;
    LYAP_TRY(gemm_f64(s, z));
  }
  return LYAP_OK;
}

// ------------------------------------------------------------------ solution update
// Fragment 2.4: G = [Z, Z^D] = V Gamma, K = Gamma blkdiag(D, D^D) Gamma^T = Theta Sigma Theta^T,
// keep sigma >= eta_s max|sigma| (|sigma| when the PSD projection is off);
// Z <- V Theta_t (into Zc), D <- Sigma_t.  The correction Z^D (cd columns) is read from Zcor.
// Fragment 2.2 (Cholesky type) is the same with Z^D = [Z+, Z-], D^D = (D+, -D-) and the PSD
// projection: G = [Z, Z+, Z-] scaled by the square roots of the weights gives its K.
int Solver::sol_upt(Ctx& c, int& cols, std::vector<double>& d, const double* Zcor, int cd,
                    const std::vector<double>& dd, double eta_s, bool psd) {
  hipStream_t s = c.s;
  const int n = c.n, cap = c.cap;
  const int q = cols + cd;
  if (q > cap) return LYAP_CAPACITY;
  if (q == 0) return LYAP_OK;
  const int k = std::min(n, q);
  double* F = F_.as<double>();
  double* Zc = Zc_.as<double>();
  double* Uq = Uq_.as<double>();
  double* Tq = Tq_.as<double>();
  double* TN = TN_.as<double>();
  double* Hm = Hm_.as<double>();
  double* Vm = Vm_.as<double>();
  double* wv = wv_.as<double>();
  LYAP_TRY(copy_block(s, n, cols, Zc, cap, F, cap));
  LYAP_TRY(copy_block(s, n, cd, Zcor, cap, F + cols, cap));
  c.ws->reset();
  LYAP_TRY(qr_lead(s, n, q, c.zc_orth ? cols : 0, F, cap, Uq, cap, Tq, cap, *c.ws, c.kt));
  std::vector<double> ups(d);
  ups.insert(ups.end(), dd.begin(), dd.end());
  LYAP_TRY(upload_d(c, ups, dvec_.as<double>()));
  LYAP_TRY(copy_block(s, k, q, Tq, cap, TN, cap, dvec_.as<double>()));
  GemmDesc g;
  g.M = k; g.N = k; g.K = q;
  g.A = TN; g.sar = cap; g.sac = 1;
  g.B = Tq; g.sbr = 1; g.sbc = cap;
  g.C = Hm; g.ldc = cap;
  LYAP_TRY(gemm_f64(s, g));
  c.ws->reset();
  LYAP_TRY(syev(s, k, Hm, cap, wv, Vm, cap, *c.ws, 0.0, nullptr, c.kt));
  std::vector<double> sig(k);
  LYAP_HIP(hipMemcpyAsync(sig.data(), wv, k * sizeof(double), hipMemcpyDeviceToHost, s));
  LYAP_HIP(hipStreamSynchronize(s));
  const double t = eta_s * std::fabs(sig[0]);
  std::vector<int> keep;
  for (int i = 0; i < k; ++i)
    if (psd ? (sig[i] >= t && sig[i] > 0.0) : (std::fabs(sig[i]) >= t && sig[i] != 0.0))
      keep.push_back(i);
  const int r = (int)keep.size();
  d.resize(r);
  for (int i = 0; i < r; ++i) d[i] = sig[keep[i]];
  if (r > 0) {
    LYAP_HIP(hipMemcpyAsync(idx_.p, keep.data(), r * sizeof(int), hipMemcpyHostToDevice, s));
    LYAP_TRY(gather_cols(s, k, r, Vm, cap, idx_.as<int>(), TN, cap));
    GemmDesc z;
    z.M = n; z.N = r; z.K = k;
    z.A = Uq; z.sar = cap; z.sac = 1;
    z.B = TN; z.sbr = cap; z.sbc = 1;
    z.C = Zc; z.ldc = cap;
    LYAP_TRY(gemm_f64(s, z));
  }
  cols = r;
  c.zc_orth = true;  // U Theta_t
  return LYAP_OK;
}

// ------------------------------------------------------------------------ IR driver
int Solver::solve(hipStream_t s, Arena& ws, int* flags, int n, int m, const double* A, int lda,
                  const double* L, int ldl, const double* S, Prec us, const lyap_options& opt,
                  double* Z, int ldz, int z_cap, double* D, int* rank, lyap_info* info,
                  bool adjoint) {
  const auto t_start = clk::now();
  Ctx c;
  c.s = s;
  c.ws = &ws;
  c.flags = flags;
  c.n = n;
  c.m = m;
  c.A = A;
  c.lda = lda;
  c.L = L;
  c.ldl = ldl;
  c.us = us;
  c.cstore = store_of(us);
  c.opt = opt;
  c.info = info;
  c.trans = adjoint;
  kt_.reset();
  c.kt = &kt_;
  c.svec.assign(m, 1.0);
  if (S) {
    LYAP_HIP(hipMemcpyAsync(c.svec.data(), S, m * sizeof(double), hipMemcpyDeviceToHost, s));
    LYAP_HIP(hipStreamSynchronize(s));
    for (double v : c.svec)
      if (!std::isfinite(v)) return LYAP_BADARG;
  }
  bool all_nonneg = true;
  for (double v : c.svec) all_nonneg = all_nonneg && v >= 0.0;
  c.chol = opt.form == 1;
  c.psd = c.chol || (opt.psd < 0 ? all_nonneg : (opt.psd != 0));
  // column capacity of the tall buffers: [Z, AZ, L] and [Z, Z^D]; the Cholesky type keeps two
  // corrections, [Z, Z+, Z-]
  c.cap = (c.chol ? 3 : 2) * n + 2 * m + 64;
  const int cap = c.cap;
  const size_t nn = (size_t)n * n, ncap = (size_t)n * cap;
  const size_t RP = 256;
  LYAP_TRY(Ak_.ensure(nn * 8));
  LYAP_TRY(An_.ensure(nn * 8));
  if (us != Prec::F64) LYAP_TRY(Ainv_.ensure(nn * 8));
  LYAP_TRY(colsum_.ensure((size_t)n * 8));
  LYAP_TRY(part_.ensure((2 * RP + RP * (size_t)n) * 8));
  LYAP_TRY(scal_.ensure(64 * 8));
  LYAP_TRY(dvec_.ensure((size_t)cap * 8));
  LYAP_TRY(dvec2_.ensure((size_t)cap * 8));
  LYAP_TRY(idx_.ensure((size_t)cap * 4));
  DevBuf* tall[] = {&Zs_, &Zc_, &Zd_, &F_, &Uq_, &Tq_, &TN_};
  for (DevBuf* b : tall) LYAP_TRY(b->ensure(ncap * 8));
  LYAP_TRY(Hm_.ensure(ncap * 8));
  LYAP_TRY(Vm_.ensure(ncap * 8));
  LYAP_TRY(Gm_.ensure((size_t)cap * cap * 8));
  LYAP_TRY(wv_.ensure((size_t)cap * 8));
  LYAP_TRY(ws.reserve(std::max(qr_workspace_bytes(n, cap), syev_workspace_bytes(n)) +
                      std::max(inverse_workspace_bytes(us, n), (size_t)64 << 20)));
  c.scal = scal_.as<double>();
  c.part = part_.as<double>();

  // ||A||_F and ||W||_F = sqrt(tr((L^T L S)^2))
  LYAP_TRY(sumsq(s, n, n, A, lda, c.scal + 11, c.part));
  {
    GemmDesc g;
    g.M = m; g.N = m; g.K = n;
    g.A = L; g.sar = 1; g.sac = ldl;
    g.B = L; g.sbr = ldl; g.sbc = 1;
    g.C = Gm_.as<double>(); g.ldc = m;
    LYAP_TRY(gemm_f64(s, g));
    LYAP_TRY(upload_d(c, c.svec, dvec2_.as<double>()));
    LYAP_TRY(wsumsq(s, m, Gm_.as<double>(), m, dvec2_.as<double>(), c.scal + 12, c.part));
    double h2[2];
    LYAP_HIP(hipMemcpyAsync(h2, c.scal + 11, sizeof(h2), hipMemcpyDeviceToHost, s));
    LYAP_HIP(hipStreamSynchronize(s));
    c.normA = std::sqrt(h2[0]);
    c.normW = std::sqrt(std::max(h2[1], 0.0));
    if (!std::isfinite(c.normA) || !std::isfinite(c.normW)) return LYAP_BADARG;
  }

  // The sign iteration of A^T is the transpose of that of A (same mu_k: transposition keeps
  // Frobenius norms), so the adjoint equation runs on A's inverse sequence with transposed
  // products.  It replays the sequence of the previous forward solve when that was computed
  // for the same A and solver precision (its stop is then the forward's, on ||A_k + I||_1).
  auto t0 = clk::now();
  const bool reuse = adjoint && key_.K > 0 && key_.A == A && key_.n == n && key_.lda == lda &&
                     key_.us == us && key_.normA == c.normA && (int)cache_.size() >= key_.K;
  if (reuse) {
    c.K = key_.K;
    c.mus = key_.mus;
    info->inversions = 0;
    info->n_mu = std::min(c.K, 64);
    for (int k = 0; k < info->n_mu; ++k) {
      info->mus[k] = key_.mus[k];
      info->onenorm[k] = key_.onenorm[k];
    }
  } else {
    key_ = CacheKey();
    LYAP_TRY(a_iteration(c));
    info->inversions = c.K;
    key_.A = A;
    key_.n = n;
    key_.lda = lda;
    key_.us = us;
    key_.normA = c.normA;
    key_.mus = c.mus;
    key_.onenorm.assign(info->onenorm, info->onenorm + std::min(c.K, 64));
    key_.K = c.K;
  }
  info->phase_ms[0] += ms_since(t0);

  // first solve (Alg 2.2, line 1)
  t0 = clk::now();
  int cols = 0;
  std::vector<double> d;
  LYAP_TRY(factor_iteration(c, L, ldl, m, 0, c.svec, c.psd, cols, d));
  c.zc_orth = cols > 0 && c.orth >= cols;
  LYAP_TRY(copy_block(s, n, cols, Zs_.as<double>(), cap, Zc_.as<double>(), cap));
  LYAP_HIP(hipStreamSynchronize(s));
  info->phase_ms[2] += ms_since(t0);
  info->newton_total = info->newton_max = c.K;

  const double eta_s = opt.eta_s > 0.0 ? opt.eta_s : 10.0 * unit_roundoff(Prec::F64);
  int status = LYAP_NOT_CONVERGED;
  const int steps = opt.refine ? std::max(opt.i_max, 1) : 1;
  for (int i = 1; i <= steps; ++i) {
    t0 = clk::now();
    double normR = 0.0, nx = 0.0;
    int rd = 0;
    std::vector<double> sd;
    LYAP_TRY(res_fac(c, Zc_.as<double>(), cap, cols, d, false, normR, rd, sd));
    LYAP_TRY(xnorm(c, Zc_.as<double>(), cap, cols, d, nx));
    const double res = normR / (c.normW + 2.0 * nx * c.normA);
    if (info->n_res < 64) info->res_hist[info->n_res++] = res;
    info->res = res;
    info->phase_ms[4] += ms_since(t0);
    if (!std::isfinite(res)) {
      status = LYAP_NONFINITE;
      break;
    }
    if (res <= opt.tol) {
      status = LYAP_OK;
      break;
    }
    if (!opt.refine) break;
    const int nh = info->n_res;
    if (nh >= 3 && info->res_hist[nh - 1] > opt.theta * info->res_hist[nh - 2] &&
        info->res_hist[nh - 2] > opt.theta * info->res_hist[nh - 3]) {
      status = LYAP_STAGNATED;
      break;
    }
    if (i == steps) break;
    // residual factor (Fragment 2.3, truncated at eta_r), from the H and U just formed
    t0 = clk::now();
    LYAP_TRY(res_factor(c, rd, sd));
    info->phase_ms[4] += ms_since(t0);
    // correction equation(s) at the solver precision, reusing the cached inverses
    t0 = clk::now();
    int cd = 0;
    std::vector<double> dd;
    const double* Zcor = Zs_.as<double>();
    if (!c.chol) {
      LYAP_TRY(factor_iteration(c, Zd_.as<double>(), cap, rd, rd, sd, false, cd, dd));  // U Q_t
    } else {
      // Fragment 2.1: R = L+ L+^T - L- L-^T with L+- = U Q_+- |Lambda_+-|^(1/2), here as
      // (U Q_+-, |lambda|); the two correction equations (Alg 2.1) share the inverse sequence
      // and are truncated independently.  U Q_t is gathered into F (positive part first),
      // and the corrections Z+ and Z- are collected in Zd.
      std::vector<int> order;
      std::vector<double> dp, dm;
      for (int i = 0; i < rd; ++i)
        if (sd[i] > 0.0) { order.push_back(i); dp.push_back(sd[i]); }
      const int rp = (int)order.size();
      for (int i = 0; i < rd; ++i)
        if (sd[i] < 0.0) { order.push_back(i); dm.push_back(-sd[i]); }
      const int rm = (int)order.size() - rp;
      double* Fb = F_.as<double>();
      double* Zpm = Zd_.as<double>();
      if (!order.empty()) {
        LYAP_HIP(hipMemcpyAsync(idx_.p, order.data(), order.size() * sizeof(int),
                                hipMemcpyHostToDevice, s));
        LYAP_TRY(gather_cols(s, n, (int)order.size(), Zd_.as<double>(), cap, idx_.as<int>(), Fb,
                             cap));
      }
      int cp = 0, cm = 0;
      std::vector<double> ddp, ddm;
      LYAP_TRY(factor_iteration(c, Fb, cap, rp, rp, dp, true, cp, ddp));
      LYAP_TRY(copy_block(s, n, cp, Zs_.as<double>(), cap, Zpm, cap));
      LYAP_TRY(factor_iteration(c, Fb + rp, cap, rm, rm, dm, true, cm, ddm));
      if (cp + cm > cap) return LYAP_CAPACITY;
      LYAP_TRY(copy_block(s, n, cm, Zs_.as<double>(), cap, Zpm + cp, cap));
      cd = cp + cm;
      dd = ddp;
      for (double x : ddm) dd.push_back(-x);
      Zcor = Zpm;
    }
    LYAP_HIP(hipStreamSynchronize(s));
    info->phase_ms[2] += ms_since(t0);
    info->newton_total += c.K;
    info->refinements += 1;
    // projected solution update (Fragment 2.4; Fragment 2.2 for the Cholesky type)
    t0 = clk::now();
    LYAP_TRY(sol_upt(c, cols, d, Zcor, cd, dd, eta_s, c.psd));
    info->phase_ms[5] += ms_since(t0);
  }
  info->rank = cols;
  *rank = cols;
  if (cols > z_cap) return LYAP_CAPACITY;
  if (!c.chol) {
    LYAP_TRY(copy_block(s, n, cols, Zc_.as<double>(), cap, Z, ldz));
    if (cols > 0)
      LYAP_HIP(hipMemcpyAsync(D, d.data(), cols * sizeof(double), hipMemcpyHostToDevice, s));
  } else if (cols > 0) {
    // Cholesky-type factor Z diag(d)^(1/2) (d >= 0 after the PSD projection), D = 1
    std::vector<double> sq(cols), ones(cols, 1.0);
    for (int i = 0; i < cols; ++i) sq[i] = std::sqrt(std::max(d[i], 0.0));
    LYAP_TRY(upload_d(c, sq, dvec_.as<double>()));
    LYAP_TRY(copy_block(s, n, cols, Zc_.as<double>(), cap, Z, ldz, dvec_.as<double>()));
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
