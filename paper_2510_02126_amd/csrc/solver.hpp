// Host driver of the factored sign-function Newton solver (Alg 3.2) and of the LDL^T-type
// mixed-precision iterative refinement (Alg 2.2 with Fragments 2.3 and 2.4).
#pragma once

#include <vector>

#include "common.hpp"

namespace lyap {

// A device allocation that grows on demand (used for a handle's own workspace).
struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  int ensure(size_t b);
  void release();
  template <class T> T* as() const { return static_cast<T*>(p); }
};

// Byte offsets of every buffer of one solve inside a workspace.  The cached inverse sequence
// comes first, so its place depends only on n, the cache format and the slot count: a later
// call on the same workspace (adjoint solve, warm-started refinement) finds it there.
struct Layout {
  int n = 0, m = 0, cap = 0, slots = 0;
  size_t slot_bytes = 0;
  size_t cache = 0, cexp = 0;
  size_t Ak = 0, An = 0, Ainv = 0, colsum = 0, part = 0, scal = 0, flags = 0, fpr = 0, vecs = 0;
  size_t dvec = 0, dvec2 = 0, idx = 0, colexp = 0, bits = 0, Lq = 0, Sm = 0, Sv = 0, Sw = 0;
  size_t Zs = 0, Zc = 0, Zd = 0, F = 0, Uq = 0, Tq = 0, TN = 0, Hm = 0, Vm = 0, Gm = 0, wv = 0;
  size_t arena = 0, arena_bytes = 0;
  size_t total = 0;
};
// Workspace of a solve of order n with m right-hand-side columns; ``us`` the solver precision
// (the cache is sized for FP64 when opt.escalate is set, since escalation can end there).
Layout solver_layout(int n, int m, Prec us, const lyap_options& opt);

class Solver {
 public:
  void release();
  // Solve A X + X A^T + L S L^T = 0 (adjoint = false) or A^T Y + Y A + L S L^T = 0
  // (adjoint = true) in the workspace ws (at least solver_layout(...).total bytes, 256-byte
  // aligned).  S: NULL (S = I), the m diagonal entries (lds == 0) or an m x m symmetric
  // matrix (lds >= m).  With r0 >= 0 the refinement starts from X_0 = Z0 diag(D0) Z0^T
  // (r0 columns) instead of a first solve.  The inverse sequence left in ws by an earlier call
  // is replayed when the option allows it and the content fingerprint of A, n, the solver
  // precision and the workspace match.
  int solve(hipStream_t s, char* ws, size_t ws_bytes, unsigned long ws_epoch, int n, int m,
            const double* A, int lda, const double* L, int ldl, const double* S, int lds,
            const lyap_precisions& prec, const lyap_options& opt, const double* Z0, int ldz0,
            const double* D0, int r0, double* Z, int ldz, int z_cap, double* D, int* rank,
            lyap_info* info, bool adjoint, bool timing = true);

 private:
  struct Ctx;
  int a_iteration(Ctx& c);
  int adi_sequence(Ctx& c);
  int shifted_inverse(Ctx& c, int j, double p);
  int checked_inverse(Ctx& c, Prec op, const double* M, long ld, double* out,
                      unsigned long long seed);
  int ensure_sequence(Ctx& c);
  int refine_loop(Ctx& c, int& cols, std::vector<double>& d, int steps, int& status);
  int factor_iteration(Ctx& c, const double* L0, long ld0, int m0, int orth0,
                       const std::vector<double>& d0, bool psd, int& cols,
                       std::vector<double>& d, double trunc_thr = 0.0);
  int adi_iteration(Ctx& c, const double* L0, long ld0, int m0, const std::vector<double>& d0,
                    bool psd, int& cols, std::vector<double>& d, double trunc_thr);
  // the chosen inner solver on the cached sequence; c.iters receives its step count
  int inner_solve(Ctx& c, const double* L0, long ld0, int m0, int orth0,
                  const std::vector<double>& d0, bool psd, int& cols, std::vector<double>& d,
                  double trunc_thr = 0.0);
  int rank_trunc(Ctx& c, double* Zb, long ldb, int& cols, std::vector<double>& d, double thr,
                 bool psd);
  int xnorm(Ctx& c, const double* Zb, long ldb, int cols, const std::vector<double>& d,
            double& out);
  int res_fac(Ctx& c, const double* Zb, long ldb, int cols, const std::vector<double>& d,
              bool want_factor, double& normR, int& rd, std::vector<double>& sd);
  int res_factor(Ctx& c, int& rd, std::vector<double>& sd);
  int sol_upt(Ctx& c, int& cols, std::vector<double>& d, const double* Zcor, int cd,
              const std::vector<double>& dd, double eta_s, bool psd);
  int upload_d(Ctx& c, const std::vector<double>& d, double* dst);
  int scaling_mu(Ctx& c, int mode, const double* Ak, const double* Ainv, const double* a_ss,
                 const double* logdet, bool scaling, double* mu_dev);

  int last_k_ = 0;
  KernTimer kt_;
  // the matrix whose inverse sequence the workspace holds
  struct CacheKey {
    const char* ws = nullptr;
    unsigned long epoch = 0;
    unsigned long long fp = 0;
    int n = 0, slots = 0, solver = 0, adi_shifts = 0;
    Prec us = Prec::F64;
    std::vector<double> mus, onenorm;
    int K = 0;
  } key_;
};

}  // namespace lyap
