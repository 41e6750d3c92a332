// Host driver of the factored sign-function Newton solver (Alg 3.2) and of the LDL^T-type
// mixed-precision iterative refinement (Alg 2.2 with Fragments 2.3 and 2.4).
#pragma once

#include <vector>

#include "common.hpp"

namespace lyap {

// A device allocation that grows on demand.
struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  int ensure(size_t b);
  void release();
  template <class T> T* as() const { return static_cast<T*>(p); }
};

class Solver {
 public:
  void release();
  // adjoint = false: A X + X A^T + L S L^T = 0.  adjoint = true: A^T Y + Y A + L S L^T = 0,
  // replaying the inverse sequence of the previous forward solve when it was computed for
  // the same A (pointer, n, lda, ||A||_F) and solver precision.
  int solve(hipStream_t s, Arena& ws, int* flags, int n, int m, const double* A, int lda,
            const double* L, int ldl, const double* S, Prec us, const lyap_options& opt,
            double* Z, int ldz, int z_cap, double* D, int* rank, lyap_info* info,
            bool adjoint = false);

 private:
  struct Ctx;
  int a_iteration(Ctx& c);
  int factor_iteration(Ctx& c, const double* L0, long ld0, int m0, int orth0,
                       const std::vector<double>& d0, bool psd, int& cols,
                       std::vector<double>& d);
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

  // persistent buffers (grown to the largest problem seen)
  DevBuf Ak_, An_, Ainv_, colsum_, part_, scal_, dvec_, dvec2_, idx_;
  DevBuf Zs_, Zc_, Zd_, F_, Uq_, Tq_, TN_, Hm_, Vm_, wv_, Gm_;
  std::vector<DevBuf> cache_;
  int last_k_ = 0;
  KernTimer kt_;
  // the matrix the cached inverse sequence belongs to
  struct CacheKey {
    const double* A = nullptr;
    int n = 0, lda = 0;
    Prec us = Prec::F64;
    double normA = -1.0;
    std::vector<double> mus, onenorm;
    int K = 0;
  } key_;
};

}  // namespace lyap
