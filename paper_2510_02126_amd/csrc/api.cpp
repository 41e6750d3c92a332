// C ABI of the solver library (declared in include/lyap.h).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cstring>
#include <memory>
#include <mutex>
#include <new>
#include <numeric>
#include <thread>
#include <vector>

#include "common.hpp"
#include "internal.hpp"
#include "solver.hpp"

using namespace lyap;

namespace lyap {

int Arena::reserve(size_t bytes) {
  if (bytes <= cap) return LYAP_OK;
  release();
  size_t want = align_up(bytes, (size_t)1 << 20);
  if (hipMalloc(&base, want) != hipSuccess) {
    base = nullptr;
    return LYAP_NO_MEMORY;
  }
  cap = want;
  top = 0;
  return LYAP_OK;
}

void Arena::release() {
  if (base) (void)hipFree(base);
  base = nullptr;
  cap = 0;
  top = 0;
}

int KernTimer::mark(hipStream_t s, hipEvent_t* e) {
  if (pool.empty()) {
    hipEvent_t x;
    LYAP_HIP(hipEventCreate(&x));
    pool.push_back(x);
  }
  *e = pool.back();
  pool.pop_back();
  LYAP_HIP(hipEventRecord(*e, s));
  return LYAP_OK;
}

int KernTimer::collect() {
  int code = LYAP_OK;
  for (const Pending& q : pend) {
    float t = 0.0f;
    if (code == LYAP_OK && hipEventSynchronize(q.b) == hipSuccess &&
        hipEventElapsedTime(&t, q.a, q.b) == hipSuccess) {
      ms[q.fam] += t;
      work[q.fam] += q.work;
      calls[q.fam] += q.calls;
    } else {
      code = LYAP_HIP_ERROR;
    }
    pool.push_back(q.a);
    pool.push_back(q.b);
  }
  pend.clear();
  return code;
}

void KernTimer::reset() {
  for (int f = 0; f < NF; ++f) {
    ms[f] = 0.0;
    work[f] = 0.0;
    calls[f] = 0;
  }
  for (const Pending& q : pend) {
    pool.push_back(q.a);
    pool.push_back(q.b);
  }
  pend.clear();
}

void KernTimer::release() {
  reset();
  for (hipEvent_t e : pool) (void)hipEventDestroy(e);
  pool.clear();
}

}  // namespace lyap

// Solver state of one batched-solve worker: its own stream, workspace and solver.
struct BatchWorker {
  hipStream_t stream = nullptr;
  DevBuf own;              // used when the caller gives no workspace
  unsigned long epoch = 0;
  Solver solver;
  ~BatchWorker() {
    solver.release();
    own.release();
    if (stream) (void)hipStreamDestroy(stream);
  }
};

struct lyap_handle_s {
  int device = 0;
  Arena ws;              // scratch of the component entry points
  DevBuf own;            // the handle's own solve workspace (ws == NULL)
  unsigned long epoch = 0;  // bumped whenever ``own`` is reallocated
  Solver solver;         // host state, including which workspace holds which inverse sequence
  int* flags = nullptr;  // device status flags of the component entry points
  std::vector<std::unique_ptr<BatchWorker>> workers;  // batched solves
};

static bool valid_dtype(int d) { return d >= LYAP_F64 && d <= LYAP_F16X2; }

static double uroff(int d) { return unit_roundoff((Prec)d); }

// u_s >= u >= u_r, u_c in unit roundoff, with u in {F64, F32}; u_s = F64 only with u = F64.
static bool valid_precisions(const lyap_precisions& p) {
  if (!valid_dtype(p.u_s) || !valid_dtype(p.u) || !valid_dtype(p.u_r) || !valid_dtype(p.u_c))
    return false;
  if (p.u != LYAP_F64 && p.u != LYAP_F32) return false;
  if (p.u_r != LYAP_F64 && p.u_r != LYAP_F32) return false;
  if (p.u_c != LYAP_F64 && p.u_c != LYAP_F32) return false;
  return uroff(p.u_s) >= uroff(p.u) && uroff(p.u) >= uroff(p.u_r) &&
         uroff(p.u) >= uroff(p.u_c);
}

static bool valid_options(const lyap_options& o, const double* S, int lds) {
  return o.tol >= 0 && o.i_max >= 0 && o.i_max <= 63 && o.k_max >= 1 && o.k_max <= 64 &&
         o.rho > 0 && o.eta_r >= 0 && o.theta > 0 && (o.form == 0 || o.form == 1) &&
         !(o.form == 1 && S != nullptr) && o.scaling >= 0 && o.scaling <= 4 &&
         (o.escalate == 0 || o.escalate == 1) && o.reuse >= -1 && o.reuse <= 1 &&
         o.delta_off >= 0 && lds >= 0 && (o.adaptive == 0 || o.adaptive == 1) &&
         o.omega >= 0 && (o.pivoting == 0 || o.pivoting == 1) && (o.solver == 0 || o.solver == 1) &&
         o.adi_shifts >= 0 && o.adi_shifts <= 64 && o.adi_max >= 1;
}

// ws == NULL: the solve runs in ``own`` (grown on demand, ``epoch`` bumped on every
// reallocation).  Otherwise in ws, whose contents are identified by ws_epoch.  With
// ``static_max`` > 0 the workspace is the fixed scratch of lyap_solve_static: problems whose
// workspace exceeds it are rejected, and no kernel timing events are recorded.
static int solve_on(Solver& solver, DevBuf& own, unsigned long& epoch, hipStream_t stream,
                    int n, int m, const double* A, int lda, const double* L, int ldl,
                    const double* S, int lds, lyap_precisions prec, const lyap_options* opt,
                    const double* Z0, int ldz0, const double* D0, int r0, double* Z, int ldz,
                    int z_cap, double* D, int* rank, void* ws, size_t ws_bytes, lyap_info* info,
                    bool adjoint, unsigned long ws_epoch = 0, size_t static_max = 0) {
  if (n <= 0 || m <= 0 || m > n || !A || !L || !Z || !D || !rank || lda < n || ldl < m ||
      z_cap < 1 || ldz < z_cap || (S && lds != 0 && lds < m))
    return LYAP_BADARG;
  if (r0 >= 0 && (r0 > n || (r0 > 0 && (!Z0 || !D0 || ldz0 < r0)))) return LYAP_BADARG;
  if (!valid_precisions(prec)) return LYAP_BADARG;
  if (n > 4096) return LYAP_BADARG;
  lyap_options o;
  if (opt) o = *opt;
  else lyap_default_options(&o);
  if (!valid_options(o, S, lds)) return LYAP_BADARG;
  lyap_info local;
  lyap_info* inf = info ? info : &local;
  std::memset(inf, 0, sizeof(*inf));
  const Layout lay = solver_layout(n, m, (Prec)prec.u_s, o);
  if (static_max > 0 && lay.total > static_max) return inf->status = LYAP_TOO_LARGE;
  char* base = static_cast<char*>(ws);
  unsigned long ep = ws_epoch;
  if (!ws) {
    if (own.bytes < lay.total) {
      ++epoch;
      if (own.ensure(lay.total) != LYAP_OK) return inf->status = LYAP_NO_MEMORY;
    }
    base = own.as<char>();
    ws_bytes = own.bytes;
    ep = epoch;
  }
  int code = solver.solve(stream, base, ws_bytes, ep, n, m, A, lda, L, ldl, S, lds, prec, o, Z0,
                          ldz0, D0, r0, Z, ldz, z_cap, D, rank, inf, adjoint, static_max == 0);
  inf->status = code;
  return code;
}

static int solve_impl(bool adjoint, lyap_handle h, void* stream, int n, int m, const double* A,
                      int lda, const double* L, int ldl, const double* S, int lds,
                      lyap_precisions prec, const lyap_options* opt, const double* Z0, int ldz0,
                      const double* D0, int r0, double* Z, int ldz, int z_cap, double* D,
                      int* rank, void* ws, size_t ws_bytes, lyap_info* info) {
  if (!h) return LYAP_BADARG;
  return solve_on(h->solver, h->own, h->epoch, (hipStream_t)stream, n, m, A, lda, L, ldl, S, lds,
                  prec, opt, Z0, ldz0, D0, r0, Z, ldz, z_cap, D, rank, ws, ws_bytes, info,
                  adjoint);
}

// ---------------------------------------------------------------- allocation-free solve
// The workspace of lyap_solve_static: a fixed device array, one copy per GPU, held for the
// life of the process.  Host code uses only the per-device address returned by
// hipGetSymbolAddress (taken once per device in lyap_create, with that device current); the
// array's name itself is a host-side stand-in, not a device address.
static constexpr size_t kStaticScratchBytes = (size_t)64 << 20;
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};
// Every static call gets a fresh epoch, so no call replays an inverse sequence another call
// left in the shared array (the high bit keeps these apart from handle workspace epochs).
std::atomic<unsigned long> g_scratch_epoch[kMaxDevices];
}  // namespace

static int static_scratch_init(int device) {
  if (device < 0 || device >= kMaxDevices) return LYAP_BADARG;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_ptr[device]) return LYAP_OK;
  void* ptr = nullptr;
  if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr)
    return LYAP_HIP_ERROR;
  g_scratch_ptr[device] = ptr;
  return LYAP_OK;
}

extern "C" {

const char* lyap_strerror(int code) {
  switch (code) {
    case LYAP_OK: return "ok";
    case LYAP_NOT_CONVERGED: return "refinement did not reach the tolerance within i_max steps";
    case LYAP_STAGNATED: return "refinement stagnated (residual ratio above theta twice)";
    case LYAP_NONFINITE: return "non-finite value at the solver precision";
    case LYAP_SINGULAR: return "exact zero pivot in an inversion";
    case LYAP_NOT_STABLE: return "Newton iteration did not converge to -I (A not Hurwitz?)";
    case LYAP_CAPACITY: return "factor needs more columns than z_cap";
    case LYAP_BADARG: return "invalid argument";
    case LYAP_HIP_ERROR: return "HIP runtime error";
    case LYAP_NO_MEMORY: return "device memory allocation failed";
    case LYAP_WORKSPACE: return "workspace smaller than lyap_workspace_size() or misaligned";
    case LYAP_TOO_LARGE:
      return "problem needs more workspace than lyap_solve_static's 64 MiB device scratch";
    default: return "unknown status";
  }
}

const char* lyap_version(void) { return "lyap-mi355x 0.1 (gfx950)"; }

void lyap_default_options(lyap_options* o) {
  if (!o) return;
  o->tol = 1e-13;
  o->i_max = 50;
  o->k_max = 50;
  o->rho = 0.1;
  o->eta_r = 1e-4;
  o->eta_s = 0.0;
  o->delta_off = 1e-2;
  o->theta = 0.9;
  o->refine = 1;
  o->psd = -1;
  o->form = 0;
  o->scaling = 0;
  o->escalate = 0;
  o->reuse = -1;
  o->adaptive = 0;
  o->pivoting = 0;
  o->omega = 0.1;
  o->solver = 0;
  o->adi_shifts = 0;
  o->adi_max = 100;
}

int lyap_workspace_size(int n, int m, int u_s, const lyap_options* opt, size_t* bytes) {
  if (!bytes || n <= 0 || m <= 0 || m > n || n > 4096 || !valid_dtype(u_s)) return LYAP_BADARG;
  lyap_options o;
  if (opt) o = *opt;
  else lyap_default_options(&o);
  if (o.k_max < 1 || o.k_max > 64 || (o.form != 0 && o.form != 1)) return LYAP_BADARG;
  *bytes = solver_layout(n, m, (Prec)u_s, o).total;
  return LYAP_OK;
}

static int batch_workers(int count, int workers) {
  return std::max(1, std::min(workers > 0 ? workers : 8, std::min(count, 32)));
}

// One worker slice: large enough for the largest instance (every layout buffer grows with
// n and m, so the maximum over the instances is taken per dimension).
static size_t batch_slice(int count, const int* n, const int* m, int u_s, const lyap_options& o) {
  int nmax = 1, mmax = 1;
  for (int i = 0; i < count; ++i) {
    nmax = std::max(nmax, n[i]);
    mmax = std::max(mmax, m[i]);
  }
  return align_up(solver_layout(nmax, std::min(mmax, nmax), (Prec)u_s, o).total, 256);
}

int lyap_workspace_size_batched(int count, const int* n, const int* m, int u_s,
                                const lyap_options* opt, int workers, size_t* bytes) {
  if (!bytes || count < 0 || (count > 0 && (!n || !m)) || !valid_dtype(u_s)) return LYAP_BADARG;
  *bytes = 0;
  if (count == 0) return LYAP_OK;
  for (int i = 0; i < count; ++i)
    if (n[i] <= 0 || m[i] <= 0 || m[i] > n[i] || n[i] > 4096) return LYAP_BADARG;
  lyap_options o;
  if (opt) o = *opt;
  else lyap_default_options(&o);
  if (o.k_max < 1 || o.k_max > 64 || (o.form != 0 && o.form != 1)) return LYAP_BADARG;
  *bytes = batch_slice(count, n, m, u_s, o) * (size_t)batch_workers(count, workers);
  return LYAP_OK;
}

int lyap_create(lyap_handle* h, int device) {
  if (!h) return LYAP_BADARG;
  *h = nullptr;
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count)
    return LYAP_HIP_ERROR;
  if (hipSetDevice(device) != hipSuccess) return LYAP_HIP_ERROR;
  lyap_handle_s* p = new (std::nothrow) lyap_handle_s();
  if (!p) return LYAP_NO_MEMORY;
  p->device = device;
  if (hipMalloc(&p->flags, 16 * sizeof(int)) != hipSuccess) {
    delete p;
    return LYAP_NO_MEMORY;
  }
  const int sc = static_scratch_init(device);
  if (sc != LYAP_OK) {
    (void)hipFree(p->flags);
    delete p;
    return sc;
  }
  *h = p;
  return LYAP_OK;
}

int lyap_destroy(lyap_handle h) {
  if (!h) return LYAP_OK;
  (void)hipDeviceSynchronize();
  h->workers.clear();
  h->solver.release();
  h->own.release();
  h->ws.release();
  if (h->flags) (void)hipFree(h->flags);
  delete h;
  return LYAP_OK;
}

int lyap_inverse(lyap_handle h, void* stream, int dtype, int pivot, int n, const double* A,
                 int lda, double* Ainv, int ldi) {
  if (!h || !valid_dtype(dtype) || n < 0 || (n > 0 && (!A || !Ainv || lda < n || ldi < n)))
    return LYAP_BADARG;
  if (n == 0) return LYAP_OK;
  if (n > 4096) return LYAP_BADARG;
  hipStream_t s = (hipStream_t)stream;
  if (pivot == 2 && n % 4 != 0) return LYAP_BADARG;
  LYAP_TRY(h->ws.reserve(inverse_workspace_bytes((Prec)dtype, n) + rbt_workspace_bytes(n) +
                         (1 << 20)));
  h->ws.reset();
  LYAP_TRY(fill_int(s, h->flags, 2, 0));
  if (pivot == 2)
    LYAP_TRY(rbt_invert(s, (Prec)dtype, n, A, lda, Ainv, ldi, h->ws, h->flags, nullptr, nullptr,
                        0x4c59415055ull, nullptr));
  else
    LYAP_TRY(invert(s, (Prec)dtype, n, A, lda, Ainv, ldi, h->ws, h->flags, pivot != 0));
  int f[2] = {0, 0};
  LYAP_HIP(hipMemcpyAsync(f, h->flags, sizeof(f), hipMemcpyDeviceToHost, s));
  LYAP_HIP(hipStreamSynchronize(s));
  if (f[0]) return LYAP_SINGULAR;
  if (f[1]) return LYAP_NONFINITE;
  return LYAP_OK;
}

int lyap_gemm(lyap_handle h, void* stream, int dtype, int transa, int transb, int M, int N, int K,
              double alpha, const double* A, int lda, const double* B, int ldb, double beta,
              double* C, int ldc) {
  if (!h || !valid_dtype(dtype) || M < 0 || N < 0 || K < 0) return LYAP_BADARG;
  if (M == 0 || N == 0) return LYAP_OK;
  if (!C || ldc < N || (K > 0 && (!A || !B))) return LYAP_BADARG;
  if (K > 0) {
    if (lda < (transa ? M : K) || ldb < (transb ? K : N)) return LYAP_BADARG;
  }
  hipStream_t s = (hipStream_t)stream;
  GemmDesc g;
  g.M = M; g.N = N; g.K = K;
  g.alpha = alpha; g.beta = beta;
  g.A = A;
  if (!transa) { g.sar = lda; g.sac = 1; } else { g.sar = 1; g.sac = lda; }
  g.B = B;
  if (!transb) { g.sbr = ldb; g.sbc = 1; } else { g.sbr = 1; g.sbc = ldb; }
  g.C = C; g.ldc = ldc;
  // split-K partial products (used for products with few output tiles and a long k-loop)
  size_t ws_elems = (size_t)64 * M * N;
  ws_elems = std::min(ws_elems, (size_t)1 << 26);
  LYAP_TRY(h->ws.reserve(ws_elems * sizeof(double) + (1 << 20)));
  h->ws.reset();
  double* part = h->ws.take<double>(ws_elems);
  if (dtype == LYAP_F64) LYAP_TRY(gemm_f64(s, g, part, ws_elems));
  else LYAP_TRY(gemm_lp(s, (Prec)dtype, Store::F64, Store::F64, Store::F64, g, part, ws_elems));
  LYAP_HIP(hipStreamSynchronize(s));
  return LYAP_OK;
}

int lyap_qr(lyap_handle h, void* stream, int n, int p, const double* F, int ldf, double* U,
            int ldu, double* T, int ldt) {
  const int k = n < p ? n : p;
  if (!h || n < 0 || p < 0 || n > 4096 ||
      (p > 0 && (!F || !U || !T || ldf < p || ldu < k || ldt < p)))
    return LYAP_BADARG;
  if (p == 0) return LYAP_OK;
  hipStream_t s = (hipStream_t)stream;
  LYAP_TRY(h->ws.reserve(qr_workspace_bytes(n, p) + (1 << 20)));
  h->ws.reset();
  LYAP_TRY(qr(s, n, p, F, ldf, U, ldu, T, ldt, h->ws));
  LYAP_HIP(hipStreamSynchronize(s));
  return LYAP_OK;
}

int lyap_qr_lead(lyap_handle h, void* stream, int n, int p, int c, const double* F, int ldf,
                 double* U, int ldu, double* T, int ldt) {
  const int k = std::min(n, p);
  if (!h || n < 0 || p < 0 || n > 4096 || c < 0 || c > p || c > n ||
      (p > 0 && (!F || !U || !T || ldf < p || ldu < k || ldt < p)))
    return LYAP_BADARG;
  if (p == 0) return LYAP_OK;
  hipStream_t s = (hipStream_t)stream;
  const size_t q = (size_t)(p - c);
  LYAP_TRY(h->ws.reserve(qr_workspace_bytes(n, p) + (size_t)n * p * 8 + (size_t)c * q * 8 +
                         (size_t)2 * n * n * 8 + ((size_t)4 << 23) + (2 << 20)));
  h->ws.reset();
  double* W = h->ws.take<double>((size_t)n * p);
  if (!W) return LYAP_NO_MEMORY;
  LYAP_TRY(copy_block(s, n, p, F, ldf, W, p));
  LYAP_TRY(qr_lead(s, n, p, c, W, p, U, ldu, T, ldt, h->ws));
  LYAP_HIP(hipStreamSynchronize(s));
  return LYAP_OK;
}

int lyap_jacobi_schedule(int nb, int* pairs, int* bmap) {
  if (nb < 2 || nb > 256 || nb % 2 != 0 || !pairs || !bmap) return LYAP_BADARG;
  return jacobi_schedule(nb, pairs, bmap);
}

int lyap_syev(lyap_handle h, void* stream, int p, const double* H, int ldh, double* w, double* V,
              int ldv) {
  if (!h || p < 0 || (p > 0 && (!H || !w || !V || ldh < p || ldv < p))) return LYAP_BADARG;
  if (p == 0) return LYAP_OK;
  hipStream_t s = (hipStream_t)stream;
  LYAP_TRY(h->ws.reserve(syev_workspace_bytes(p) + (1 << 20)));
  h->ws.reset();
  LYAP_TRY(syev(s, p, H, ldh, w, V, ldv, h->ws, 0.0, nullptr));
  LYAP_HIP(hipStreamSynchronize(s));
  return LYAP_OK;
}

int lyap_trace_loss(lyap_handle h, void* stream, int n, int k, const double* C, int ldc, int r,
                    const double* Z, int ldz, const double* D, double* loss) {
  if (!h || n <= 0 || k <= 0 || r < 0 || !loss || (r > 0 && (!C || !Z || !D)) || ldc < n ||
      (r > 0 && ldz < r))
    return LYAP_BADARG;
  *loss = 0.0;
  if (r == 0) return LYAP_OK;
  hipStream_t s = (hipStream_t)stream;
  LYAP_TRY(h->ws.reserve(((size_t)k * r + 64) * sizeof(double) + (1 << 20)));
  h->ws.reset();
  double* CZ = h->ws.take<double>((size_t)k * r);
  double* out = h->ws.take<double>(1);
  if (!CZ || !out) return LYAP_NO_MEMORY;
  GemmDesc g;
  g.M = k; g.N = r; g.K = n;
  g.A = C; g.sar = ldc; g.sac = 1;
  g.B = Z; g.sbr = ldz; g.sbc = 1;
  g.C = CZ; g.ldc = r;
  LYAP_TRY(gemm_f64(s, g));
  LYAP_TRY(colw_sumsq(s, k, r, CZ, r, D, out));
  LYAP_HIP(hipMemcpyAsync(loss, out, sizeof(double), hipMemcpyDeviceToHost, s));
  LYAP_HIP(hipStreamSynchronize(s));
  return LYAP_OK;
}

int lyap_trace_loss_grad(lyap_handle h, void* stream, int n, int m, int k, const double* L,
                         int ldl, const double* S, const double* C, int ldc, int r,
                         const double* Z, int ldz, const double* D, int ry, const double* ZY,
                         int ldzy, const double* DY, double scale, double* dA, int ldda,
                         double* dL, int lddl, double* dS, double* dC, int lddc) {
  if (!h || n <= 0 || m <= 0 || k <= 0 || r < 0 || ry < 0 || !L || !C || ldl < m || ldc < n ||
      (r > 0 && (!Z || !D || ldz < r)) || (ry > 0 && (!ZY || !DY || ldzy < ry)) ||
      (dA && ldda < n) || (dL && lddl < m) || (dC && lddc < n))
    return LYAP_BADARG;
  hipStream_t s = (hipStream_t)stream;
  const size_t need = (size_t)n * ry + (size_t)n * r + (size_t)ry * r + (size_t)n * r +
                      2 * (size_t)ry * m + (size_t)k * r + (size_t)m + 64;
  LYAP_TRY(h->ws.reserve(need * sizeof(double) + (16 << 20)));
  h->ws.reset();
  double* ZYD = h->ws.take<double>((size_t)n * std::max(ry, 1));   // ZY diag(DY)
  double* ZD = h->ws.take<double>((size_t)n * std::max(r, 1));     // Z diag(D)
  double* M = h->ws.take<double>((size_t)std::max(ry, 1) * std::max(r, 1));
  double* P = h->ws.take<double>((size_t)n * std::max(r, 1));
  double* N = h->ws.take<double>((size_t)std::max(ry, 1) * m);
  double* NS = h->ws.take<double>((size_t)std::max(ry, 1) * m);
  double* CZD = h->ws.take<double>((size_t)k * std::max(r, 1));
  double* ones = h->ws.take<double>((size_t)m);
  if (!ZYD || !ZD || !M || !P || !N || !NS || !CZD || !ones) return LYAP_NO_MEMORY;
  if (r > 0) LYAP_TRY(copy_block(s, n, r, Z, ldz, ZD, r, D));
  if (ry > 0) LYAP_TRY(copy_block(s, n, ry, ZY, ldzy, ZYD, ry, DY));
  GemmDesc g;
  if (dA) {
    // dA = 2 Y X = 2 (ZY diag(DY)) (ZY^T (Z diag(D))) Z^T
    if (r == 0 || ry == 0) {
      LYAP_TRY(fill_f64(s, dA, (long)(n - 1) * ldda + n, 0.0));
    } else {
      g = GemmDesc();
      g.M = ry; g.N = r; g.K = n;
      g.A = ZY; g.sar = 1; g.sac = ldzy;
      g.B = ZD; g.sbr = r; g.sbc = 1;
      g.C = M; g.ldc = r;
      LYAP_TRY(gemm_f64(s, g));
      g = GemmDesc();
      g.M = n; g.N = r; g.K = ry;
      g.A = ZYD; g.sar = ry; g.sac = 1;
      g.B = M; g.sbr = r; g.sbc = 1;
      g.C = P; g.ldc = r;
      LYAP_TRY(gemm_f64(s, g));
      g = GemmDesc();
      g.M = n; g.N = n; g.K = r;
      g.alpha = 2.0 * scale;
      g.A = P; g.sar = r; g.sac = 1;
      g.B = Z; g.sbr = 1; g.sbc = ldz;
      g.C = dA; g.ldc = ldda;
      LYAP_TRY(gemm_f64(s, g));
    }
  }
  if (dL || dS) {
    // N = ZY^T L; dL = 2 ZY diag(DY) N diag(S); dS = diag(L^T Y L) = sum_j DY_j N_j.^2
    if (ry > 0) {
      g = GemmDesc();
      g.M = ry; g.N = m; g.K = n;
      g.A = ZY; g.sar = 1; g.sac = ldzy;
      g.B = L; g.sbr = ldl; g.sbc = 1;
      g.C = N; g.ldc = m;
      LYAP_TRY(gemm_f64(s, g));
    }
    if (dL) {
      if (ry == 0) {
        LYAP_TRY(fill_f64(s, dL, (long)(n - 1) * lddl + m, 0.0));
      } else {
        if (!S) LYAP_TRY(fill_f64(s, ones, m, 1.0));
        LYAP_TRY(copy_block(s, ry, m, N, m, NS, m, S ? S : ones));
        g = GemmDesc();
        g.M = n; g.N = m; g.K = ry;
        g.alpha = 2.0 * scale;
        g.A = ZYD; g.sar = ry; g.sac = 1;
        g.B = NS; g.sbr = m; g.sbc = 1;
        g.C = dL; g.ldc = lddl;
        LYAP_TRY(gemm_f64(s, g));
      }
    }
    if (dS) {
      if (ry == 0) LYAP_TRY(fill_f64(s, dS, m, 0.0));
      else LYAP_TRY(roww_colsumsq(s, ry, m, N, m, DY, dS));
      if (scale != 1.0 && ry > 0) LYAP_TRY(copy_block(s, 1, m, dS, m, dS, m, nullptr, scale));
    }
  }
  if (dC) {
    // dC = 2 C X = 2 (C Z diag(D)) Z^T
    if (r == 0) {
      LYAP_TRY(fill_f64(s, dC, (long)(k - 1) * lddc + n, 0.0));
    } else {
      g = GemmDesc();
      g.M = k; g.N = r; g.K = n;
      g.A = C; g.sar = ldc; g.sac = 1;
      g.B = ZD; g.sbr = r; g.sbc = 1;
      g.C = CZD; g.ldc = r;
      LYAP_TRY(gemm_f64(s, g));
      g = GemmDesc();
      g.M = k; g.N = n; g.K = r;
      g.alpha = 2.0 * scale;
      g.A = CZD; g.sar = r; g.sac = 1;
      g.B = Z; g.sbr = 1; g.sbc = ldz;
      g.C = dC; g.ldc = lddc;
      LYAP_TRY(gemm_f64(s, g));
    }
  }
  LYAP_HIP(hipStreamSynchronize(s));
  return LYAP_OK;
}

int lyap_solve_batched(lyap_handle h, void* stream, int count, const int* n, const int* m,
                       const double* const* A, const int* lda, const double* const* L,
                       const int* ldl, const double* const* S, lyap_precisions prec,
                       const lyap_options* opt, double* const* Z, const int* ldz,
                       const int* z_cap, double* const* D, int* rank, lyap_info* infos,
                       int* codes, int workers, void* ws, size_t ws_bytes) {
  if (!h || count < 0 || (count > 0 && (!n || !m || !A || !lda || !L || !ldl || !Z || !ldz ||
                                        !z_cap || !D || !rank || !codes)))
    return LYAP_BADARG;
  if (count == 0) return LYAP_OK;
  for (int i = 0; i < count; ++i)
    if (n[i] <= 0 || m[i] <= 0 || m[i] > n[i] || n[i] > 4096 || !A[i] || !L[i] || !Z[i] ||
        !D[i] || lda[i] < n[i] || ldl[i] < m[i] || z_cap[i] < 1 || ldz[i] < z_cap[i])
      return LYAP_BADARG;
  lyap_options o;
  if (opt) o = *opt;
  else lyap_default_options(&o);
  const int W = batch_workers(count, workers);
  size_t slice = 0;
  if (ws) {
    slice = batch_slice(count, n, m, prec.u_s, o);
    if (ws_bytes < slice * W || ((uintptr_t)ws & 255) != 0) return LYAP_WORKSPACE;
  }
  // inputs are ready once the caller's stream has drained; outputs are complete on return
  LYAP_HIP(hipStreamSynchronize((hipStream_t)stream));
  while ((int)h->workers.size() < W) {
    std::unique_ptr<BatchWorker> w(new (std::nothrow) BatchWorker());
    if (!w) return LYAP_NO_MEMORY;
    LYAP_HIP(hipStreamCreateWithFlags(&w->stream, hipStreamNonBlocking));
    h->workers.push_back(std::move(w));
  }
  // longest-processing-time first: instances by decreasing n^3
  std::vector<int> order(count);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return n[a] > n[b]; });
  std::atomic<int> next(0);
  auto run = [&](int wi) {
    BatchWorker& w = *h->workers[wi];
    if (hipSetDevice(h->device) != hipSuccess) return;
    char* mine = ws ? static_cast<char*>(ws) + slice * wi : nullptr;
    for (int q = next.fetch_add(1); q < count; q = next.fetch_add(1)) {
      const int i = order[q];
      lyap_info local;
      lyap_info* inf = infos ? &infos[i] : &local;
      codes[i] = solve_on(w.solver, w.own, w.epoch, w.stream, n[i], m[i], A[i], lda[i], L[i],
                          ldl[i], S ? S[i] : nullptr, 0, prec, opt, nullptr, 0, nullptr, -1, Z[i],
                          ldz[i], z_cap[i], D[i], &rank[i], mine, slice, inf, false);
    }
  };
  std::vector<std::thread> pool;
  for (int wi = 1; wi < W; ++wi) pool.emplace_back(run, wi);
  run(0);
  for (auto& t : pool) t.join();
  for (int i = 0; i < count; ++i)
    if (codes[i] != LYAP_OK) return codes[i];
  return LYAP_OK;
}

int lyap_solve(lyap_handle h, void* stream, int n, int m, const double* A, int lda,
               const double* L, int ldl, const double* S, int lds, lyap_precisions prec,
               const lyap_options* opt, double* Z, int ldz, int z_cap, double* D, int* rank,
               void* ws, size_t ws_bytes, lyap_info* info) {
  return solve_impl(false, h, stream, n, m, A, lda, L, ldl, S, lds, prec, opt, nullptr, 0,
                    nullptr, -1, Z, ldz, z_cap, D, rank, ws, ws_bytes, info);
}

int lyap_solve_static(lyap_handle h, void* stream, int n, int m, const double* A, int lda,
                      const double* L, int ldl, const double* S, int lds, lyap_precisions prec,
                      const lyap_options* opt, double* Z, int ldz, int z_cap, double* D,
                      int* rank, lyap_info* info) {
  if (!h || h->device < 0 || h->device >= kMaxDevices) return LYAP_BADARG;
  void* ptr = g_scratch_ptr[h->device];
  if (!ptr) return LYAP_HIP_ERROR;
  const unsigned long ep = (1ul << 63) | (g_scratch_epoch[h->device].fetch_add(1) + 1);
  return solve_on(h->solver, h->own, h->epoch, (hipStream_t)stream, n, m, A, lda, L, ldl, S, lds,
                  prec, opt, nullptr, 0, nullptr, -1, Z, ldz, z_cap, D, rank, ptr,
                  kStaticScratchBytes, info, false, ep, kStaticScratchBytes);
}

int lyap_refine(lyap_handle h, void* stream, int n, int m, const double* A, int lda,
                const double* L, int ldl, const double* S, int lds, lyap_precisions prec,
                const lyap_options* opt, const double* Z0, int ldz0, const double* D0, int r0,
                double* Z, int ldz, int z_cap, double* D, int* rank, void* ws,
                size_t ws_bytes, lyap_info* info) {
  if (r0 < 0) return LYAP_BADARG;
  return solve_impl(false, h, stream, n, m, A, lda, L, ldl, S, lds, prec, opt, Z0, ldz0, D0, r0,
                    Z, ldz, z_cap, D, rank, ws, ws_bytes, info);
}

int lyap_solve_adjoint(lyap_handle h, void* stream, int n, int m, const double* A, int lda,
                       const double* L, int ldl, const double* S, int lds, lyap_precisions prec,
                       const lyap_options* opt, double* Z, int ldz, int z_cap, double* D,
                       int* rank, void* ws, size_t ws_bytes, lyap_info* info) {
  return solve_impl(true, h, stream, n, m, A, lda, L, ldl, S, lds, prec, opt, nullptr, 0,
                    nullptr, -1, Z, ldz, z_cap, D, rank, ws, ws_bytes, info);
}

}  // extern "C"
