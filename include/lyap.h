/*
 * lyap.h -- C ABI of the MI355X (gfx950) low-rank Lyapunov solver.
 *
 * Solves A X + X A^T + W = 0 with A Hurwitz and W = L L^T or W = L S L^T (S symmetric,
 * possibly indefinite) by the factored, scaled sign-function Newton iteration
 * (Section 3, eq (3.2)/(3.3), Alg 3.1/3.2) wrapped in mixed-precision iterative
 * refinement (Section 2, Alg 2.1/2.2, Fragments 2.1-2.4), returning X ~ Z diag(D) Z^T.
 *
 * Conventions shared by every entry point
 *  - Matrices are row-major (C order): element (i, j) of a matrix with leading dimension
 *    ld lives at ptr[i * ld + j].
 *  - Every matrix/vector pointer is a DEVICE pointer (hipMalloc'd or a torch CUDA tensor)
 *    unless stated otherwise; info structs are HOST pointers.
 *  - ``stream`` is a hipStream_t passed as void* (NULL = the default stream).  Every call
 *    is stream-ordered and returns after its results are valid (host-synchronous), since
 *    ranks and stopping decisions are taken on the host from a few device scalars.
 *  - Ownership: the caller owns all input and output buffers; the library never frees or
 *    keeps caller memory.  Every solve works in a device workspace of
 *    lyap_workspace_size() bytes: either the caller's (``ws``, ``ws_bytes``; the call then
 *    allocates no device memory) or, with ws == NULL, one the handle allocates with hipMalloc
 *    on first use, grows when a larger problem needs it and frees in lyap_destroy.  The
 *    workspace also keeps the cached sequence of inverses of the last solve made in it, which
 *    adjoint solves and warm-started refinement replay (see lyap_options.reuse).
 *  - Errors: every entry point returns an int status (LYAP_OK = 0 or one of the codes
 *    below); nothing throws across the ABI.  On error the outputs are unspecified unless
 *    the code's description says otherwise.
 *  - Thread safety: a handle must not be used by two host threads at once.
 */
#ifndef LYAP_H
#define LYAP_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Status codes. */
enum {
  LYAP_OK = 0,
  LYAP_NOT_CONVERGED = 1, /* i_max refinements done; outputs hold the last iterate       */
  LYAP_STAGNATED = 2,     /* res_i/res_{i-1} > theta twice in a row (eq 4.2); outputs valid */
  LYAP_NONFINITE = 3,     /* an inverse or iterate overflowed at the solver precision       */
  LYAP_SINGULAR = 4,      /* an exact zero pivot in an inversion                            */
  LYAP_NOT_STABLE = 5,    /* A-iteration did not converge to -I (A not Hurwitz) in k_max    */
  LYAP_CAPACITY = 6,      /* the factor needs more than z_cap columns; *rank = needed       */
  LYAP_BADARG = 7,        /* invalid size, pointer, precision order or option               */
  LYAP_HIP_ERROR = 8,     /* a HIP runtime call failed                                      */
  LYAP_NO_MEMORY = 9,     /* the handle could not allocate its workspace                    */
  LYAP_WORKSPACE = 10,    /* the caller's workspace is smaller than lyap_workspace_size()
                             or not 256-byte aligned                                        */
  LYAP_TOO_LARGE = 11     /* lyap_solve_static: the problem's workspace exceeds its fixed
                             64 MiB device scratch                                          */
};

/* Arithmetic formats of Table 1.1, and the split-operand binary16 format F16X2 (not in the
 * paper: x ~ hi + 2^-11 lo with hi, lo binary16, products hi*hi + 2^-11 (hi*lo + lo*hi) on
 * the binary16 matrix cores with binary32 sums; 22 significand bits, unit roundoff 2^-22;
 * the operand splitting of Markidis et al. 2018 and Ootomo and Yokota 2022), usable as a
 * solver precision u_s.  Order of "precision" (larger unit roundoff first):
 * BF16 > F16 > F16X2 > F32 > F64. */
typedef enum {
  LYAP_F64 = 0, LYAP_F32 = 1, LYAP_F16 = 2, LYAP_BF16 = 3, LYAP_F16X2 = 4
} lyap_dtype;

/* Precisions of Alg 2.1/2.2: solver u_s, working u, residual factorisation u_r and solution
 * update u_c, with u_s >= u >= u_r, u_c in unit roundoff (Table 1.1).  Supported: u = F64
 * with u_r = u_c = F64 and any u_s (u_s = F64 gives the plain FP64 sign-function Newton
 * solve), and u = F32 with u_r, u_c in {F32, F64} and u_s in {F32, F16, BF16} (Table 3.1's
 * rows with u = fp32; the attainable residual is then at the binary32 level, about 1e-8).
 * At u = F32 the factor Z and D are stored rounded to binary32; at u_r = F32 the product AZ
 * of the residual factorisation runs on the binary32 matrix cores and the spectral
 * decompositions of the residual (u_r = F32) and of the update (u_c = F32) use binary32
 * rotations, their results rounded to binary32. */
typedef struct {
  int u_s, u, u_r, u_c; /* lyap_dtype values */
} lyap_precisions;

/* Options; lyap_default_options fills in the paper's Section 4.1 values. */
typedef struct {
  double tol;        /* tau_I on the relative residual of eq (4.1); default 1e-13        */
  int i_max;         /* refinement steps; default 50                                      */
  int k_max;         /* Newton steps per solver call; default 50                          */
  double rho;        /* in-solver truncation when columns exceed floor(rho n); 0.1        */
  double eta_r;      /* residual truncation, relative to max|lambda|; 1e-4               */
  double eta_s;      /* solution truncation, relative to max|sigma|; <= 0 means 10 u     */
  double delta_off;  /* Frobenius scaling switched off once delta_k < delta_off; 1e-2     */
  double theta;      /* stagnation ratio of eq (4.2); 0.9                                 */
  int refine;        /* 1: iterative refinement (Alg 2.2); 0: one solve + residual check  */
  int psd;           /* -1 auto (S == NULL or S >= 0), 0 off, 1 on: PSD projection        */
  int form;          /* 0: LDL^T type (Alg 2.2, default).  1: Cholesky type (Alg 2.1,
                        Fragments 2.1 / 2.2), only for W = L L^T (S must be NULL): the
                        residual is split into R = L+ L+^T - L- L-^T, the two correction
                        equations are solved separately (sharing the inverse sequence) and
                        the update keeps [Z, Z+, Z-] with signature (+, +, -) projected onto
                        the PSD cone; Z is returned as the Cholesky-type factor
                        (X ~ Z Z^T) and D is filled with ones.  The in-solver
                        truncation keeps singular values above sqrt(u_s) sigma_1 of the
                        factor (SVD reading of RankTruncChol).                              */
  int scaling;       /* Newton scaling mu_k (Section 3): 0 Frobenius-norm (default, the one
                        Section 4 uses), 1 determinantal |det A_k|^(-1/n) (log|det| from the
                        pivots of the inversion), 2 2-norm sqrt(||A_k^-1||_2 / ||A_k||_2) and
                        3 spectral sqrt(rho(A_k^-1) / rho(A_k)), the last two from power-
                        iteration estimates (12 steps on A^T A; 24 steps on A), and 4 the
                        combined Frobenius + determinantal scaling Section 4 mentions:
                        determinantal for the first step, Frobenius afterwards.  Scaling is
                        switched off once delta_k < delta_off in every case.               */
  int escalate;      /* 1: when a refinement at reduced u_s stagnates (eq 4.2), runs out of
                        steps, overflows or meets an exact zero pivot, continue it at the next
                        solver precision (bf16 -> fp16 -> fp32 -> fp64, Table 1.1), from the
                        current iterate when it is valid; 0 (default): stop there.  Table
                        3.1 ties each u_s to the conditioning it can handle, so escalation
                        picks the cheapest precision that converges.  The workspace is then
                        sized for the FP64 inverse sequence.                                */
  int reuse;         /* inverse-sequence replay: -1 (default) for lyap_solve_adjoint and
                        lyap_refine when the workspace holds the sequence of the same A
                        (64-bit content fingerprint of A, n, u_s and k_max), never for
                        lyap_solve; 1 also for lyap_solve; 0 never.                          */
  int adaptive;      /* 1: inexact inner solves with tolerances tied to the refinement (the
                        adaptivity the Conclusions point to): each correction solve's in-solver
                        truncation keeps |lambda| > max(u_s, eta_r / 10) max|lambda| (the
                        residual factor is itself truncated at eta_r), and the update after a
                        step with residual res_i keeps |sigma| >= max(eta_s, omega res_i)
                        max|sigma|; a step that contracts the residual by less than half
                        (res_i > res_{i-1} / 2) switches both back to the fixed thresholds
                        for the rest of the refinement.  0 (default): the fixed thresholds
                        of Alg 3.2 and Fragment 2.4.                                        */
  int pivoting;      /* inversions of A_k while ||A_{k-1} + I||_1 >= 1 (afterwards A_k is
                        strictly column diagonally dominant and no pivoting is needed):
                        0 (default) Gauss-Jordan with partial pivoting; 1 random butterfly
                        transformation (Parker's RBT, depth 2, seeded) and Gauss-Jordan
                        without pivoting on U^T A_k V, checked by a residual probe
                        ||A_k (A_k^-1 x) - x|| <= 8 sqrt(n) u_s ||A_k||_F ||A_k^-1||_F ||x||
                        and redone with partial pivoting when the probe fails (needs
                        n % 4 == 0, otherwise partial pivoting).  The ADI solver's shifted
                        inverses and its spectral-interval inverse are treated alike.      */
  double omega;      /* the factor omega of the adaptive update threshold; default 0.1:
                        directions that small are the ones the next correction fixes
                        anyway (measured at n = 4096: fp16 inner, omega 1e-3 / 0.1 / 0.3:
                        rank 3796 / 1071 / 289 with the same six or five refinements)   */
  int solver;        /* inner solver of the first solve and of every correction: 0 (default)
                        the sign-function Newton iteration (Alg 3.2 / 3.1); 1 the low-rank
                        ADI method in LDL^T form, the other solver Section 3 says the
                        refinement's precision settings carry over to.  Residual-factor
                        recurrence with real shifts p_j < 0: V_j = (A + p_j I)^{-1} W_{j-1},
                        W_j = W_{j-1} - 2 p_j V_j, Z_j = [Z_{j-1}, V_j], D_j = blkdiag(D_{j-1},
                        -2 p_j S); the residual of Z_j D_j Z_j^T is W_j S W_j^T.  Shifts:
                        Wachspress's optimal real shifts for [a, b], b = rho(A) and
                        a = 1 / rho(A^{-1}) estimated by 24 power-iteration steps (A^{-1} at
                        u_s, binary32 for fp16 / bf16 / split fp16), J of them for a
                        reduction of sqrt(u_s) per cycle.  The J shifted inverses are formed
                        at u_s once (J + 1 inversions with the interval's) and cached like
                        the Newton sequence; the shifts are used cyclically until
                        ||W_j S W_j^T||_F <= max(10 u_s, inner) ||W_0 S W_0^T||_F (inner =
                        eta_r / 10 with ``adaptive``, else 0) or adi_max steps.  Z is
                        truncated by RankTruncLdlt past rho n columns as in the Newton
                        solver.  With solver = 1, info.mus holds the shifts and
                        newton_total / newton_max count ADI steps.                          */
  int adi_shifts;    /* number J of ADI shifts; 0 (default): from the bound above; at most
                        min(k_max, 64)                                                      */
  int adi_max;       /* ADI steps per solve; default 100                                    */
} lyap_options;

/* Per-solve diagnostics (Table 4.1 columns plus timings). */
typedef struct {
  int status;             /* same as the return code                                     */
  double res;             /* relative residual (eq 4.1) of the returned factors          */
  int n_res;              /* entries used in res_hist                                    */
  double res_hist[64];    /* res_i per refinement step                                   */
  int newton_total;       /* varsigma: Newton steps over all solver calls                */
  int newton_max;         /* alpha: largest number of Newton steps in one call           */
  int inversions;         /* inverses actually computed (the cached sequence length K)   */
  int refinements;        /* correction solves performed                                 */
  int rank;               /* columns of the returned Z                                   */
  int n_mu;               /* entries used in mus                                         */
  double mus[64];         /* scalings mu_0 .. mu_{K-1} (ADI solver: the shifts p_1 .. p_J) */
  double onenorm[64];     /* ||A_k + I||_1 after each Newton step                        */
  double phase_ms[8];     /* 0 inversions, 1 Newton update+norms, 2 factor products,
                             3 in-solver truncation, 4 residual factorisation,
                             5 solution update, 6 other, 7 total                          */
  /* Kernel families timed with HIP events on the solve's stream (for roofline reports):
     0 inversions (work = 2 n^3 flops each), 1 Jacobi round kernels of the spectral
     decompositions (work = bytes of A and V read and written by the block updates),
     2 thin QR factorisations including the formation of U (work = Householder flops),
     3 unused.  kern_ms is the summed event time, kern_calls the number of kernel
     launches (family 1) or calls (families 0 and 2).                                    */
  double kern_ms[4];
  double kern_work[4];
  int kern_calls[4];
  int u_s_final;          /* solver precision (lyap_dtype) of the last stage (escalate)   */
  int escalations;        /* precision escalations performed                             */
  int cache_reused;       /* 1 when the inverse sequence was replayed from the workspace  */
  int rbt_steps;          /* inversions done through the random butterfly transformation  */
  int rbt_fallbacks;      /* butterfly inversions whose probe failed, redone with pivoting */
} lyap_info;

typedef struct lyap_handle_s* lyap_handle;

/* Create a handle bound to HIP device ``device`` (the device must be current in the
 * calling thread for every later call).  *h receives the handle. */
int lyap_create(lyap_handle* h, int device);
/* Destroy a handle and free its workspace.  NULL is accepted. */
int lyap_destroy(lyap_handle h);
/* Section 4.1 defaults: tol 1e-13, i_max 50, k_max 50, rho 0.1, eta_r 1e-4, eta_s 10u,
 * delta_off 1e-2, theta 0.9, refine 1, psd -1, form 0, scaling 0 (Frobenius), escalate 0,
 * reuse -1, adaptive 0, pivoting 0, omega 0.1, solver 0 (Newton), adi_shifts 0 (automatic),
 * adi_max 100. */
void lyap_default_options(lyap_options* opt);
/* Human-readable text of a status code (static string). */
const char* lyap_strerror(int code);
/* Library version string and the GPU architecture it was built for. */
const char* lyap_version(void);

/*
 * lyap_workspace_size -- bytes of device workspace (256-byte aligned) that lyap_solve,
 * lyap_refine and lyap_solve_adjoint need for order n, m right-hand-side columns, solver
 * precision u_s (a lyap_dtype) and the options ``opt`` (NULL: defaults; k_max fixes the
 * number of cached inverses, form and escalate the buffer shapes).  About
 * k_max n^2 b_s + (9 (2n + 2m + 64) n + 5 n^2) 8 bytes, b_s the bytes of a u_s value (8 with
 * escalate): 6.5 GB at n = 4096, u_s = fp32 and the default k_max.  Returns LYAP_BADARG for
 * sizes outside 1 <= m <= n <= 4096.
 */
int lyap_workspace_size(int n, int m, int u_s, const lyap_options* opt, size_t* bytes);

/*
 * lyap_solve -- Alg 2.2 (LDL^T-type mixed-precision IR) with Alg 3.2 as the solver, or with
 * opt->form == 1 Alg 2.1 (Cholesky type, W = L L^T only).
 *
 *  n, m      order of A (n <= 4096) and number of columns of L (1 <= m <= n).
 *  A         n x n FP64, row-major, leading dimension lda >= n; A must be Hurwitz.
 *  L         n x m FP64, row-major, ldl >= m.
 *  S, lds    NULL for W = L L^T; with lds == 0, the m diagonal entries of S
 *            (W = L diag(S) L^T); with lds >= m, an m x m symmetric S (row-major, only its
 *            symmetric part is used), diagonalised once on the device as S = Q_s diag(s) Q_s^T
 *            with L replaced by L Q_s (the change of basis the paper's LDL^T form allows).
 *  prec      precisions {u_s, u, u_r, u_c} (see lyap_precisions).
 *  opt       options or NULL for the defaults.
 *  Z         n x z_cap FP64 output, row-major, ldz >= z_cap; columns 0..rank-1 receive
 *            orthonormal factor columns (form 0) or the Cholesky-type factor (form 1).
 *  D         z_cap FP64 output: the diagonal of D (X ~ Z diag(D) Z^T).  For W = L L^T
 *            (S == NULL) D > 0 and Z diag(sqrt D) is a Cholesky-type factor; with form 1,
 *            D = 1.
 *  rank      host int: the number of columns written.
 *  ws        device workspace of ws_bytes >= lyap_workspace_size(n, m, prec.u_s, opt) bytes,
 *            256-byte aligned, or NULL for the handle's own.  The solve allocates no device
 *            memory when ws is given.  Two calls that overlap in time must not share ws.
 *  info      host lyap_info or NULL.
 * Returns LYAP_OK when res <= tol.  LYAP_NOT_CONVERGED / LYAP_STAGNATED still write the
 * last iterate.  With opt->refine == 0 the call runs the plain sign-function Newton solve
 * at u_s and one residual evaluation (the FP64 baseline when u_s = LYAP_F64).  Non-finite
 * values in A, L or S give LYAP_BADARG; overflow inside the iteration LYAP_NONFINITE.
 */
int lyap_solve(lyap_handle h, void* stream, int n, int m, const double* A, int lda,
               const double* L, int ldl, const double* S, int lds, lyap_precisions prec,
               const lyap_options* opt, double* Z, int ldz, int z_cap, double* D, int* rank,
               void* ws, size_t ws_bytes, lyap_info* info);

/*
 * lyap_solve_static -- lyap_solve for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc): the solve runs in
 * a fixed 64 MiB device scratch array compiled into the library, one per GPU, held until the
 * process ends; the call makes no hipMalloc / hipFree and creates no events (info->kern_*
 * stay zero).  Arguments, outputs and status codes as for lyap_solve; a problem whose
 * lyap_workspace_size() exceeds 64 MiB (for example n > 256 at the default k_max with m = 8
 * and u_s = fp64; the limit grows when k_max is lowered) is rejected with LYAP_TOO_LARGE
 * before any device work.  Every call on a GPU shares that GPU's scratch, which keeps the
 * last call's contents: calls that overlap in time on one GPU (two streams, two threads,
 * two handles) race and must be serialised by the caller.  No call replays an inverse
 * sequence left in the scratch by an earlier call.
 */
int lyap_solve_static(lyap_handle h, void* stream, int n, int m, const double* A, int lda,
                      const double* L, int ldl, const double* S, int lds, lyap_precisions prec,
                      const lyap_options* opt, double* Z, int ldz, int z_cap, double* D,
                      int* rank, lyap_info* info);

/*
 * lyap_refine -- Alg 2.1 / 2.2 started from a given approximation X_0 = Z0 diag(D0) Z0^T
 * (r0 >= 0 columns, Z0 n x r0 row-major with ldz0 >= r0, D0 r0 values, device pointers) in
 * place of the first solve (the first line of either algorithm accepts any starting factor):
 * the residual of X_0 is tested, and while it exceeds tol the corrections are solved and
 * the update applied exactly as in lyap_solve.  The inverse sequence is computed only if a
 * correction is needed, and is replayed (no inversion) when the workspace holds the sequence
 * of the same A and u_s, e.g. from a lyap_solve just made in it.  Z0/D0 may be the same
 * buffers as Z/D.  Other arguments and return codes as for lyap_solve.
 */
int lyap_refine(lyap_handle h, void* stream, int n, int m, const double* A, int lda,
                const double* L, int ldl, const double* S, int lds, lyap_precisions prec,
                const lyap_options* opt, const double* Z0, int ldz0, const double* D0, int r0,
                double* Z, int ldz, int z_cap, double* D, int* rank, void* ws,
                size_t ws_bytes, lyap_info* info);

/*
 * lyap_solve_batched -- ``count`` independent equations A_i X_i + X_i A_i^T + L_i S_i L_i^T = 0
 * of uneven n_i (<= 4096) and m_i, each solved exactly as lyap_solve would on its own.  The
 * instances are taken longest first (by n_i) by ``workers`` host threads (0: 8; at most
 * 32), each driving its own HIP stream and its own slice of the workspace, so the
 * latency-bound steps of different instances overlap on the GPU.  Per-instance arrays of
 * device pointers and leading dimensions (host arrays of length count); S may be NULL (all
 * instances W = L L^T) or hold NULL entries; a non-NULL S_i is the diagonal of S (m_i
 * values).  ws: NULL (the handle's workers allocate their own) or a device workspace of
 * ws_bytes >= lyap_workspace_size_batched(...) bytes split between the workers.  rank, infos
 * (may be NULL) and codes are host arrays of length count receiving each instance's rank,
 * info and return code.  The call waits for ``stream`` before starting and returns when every
 * instance is complete; it returns the first nonzero per-instance code in instance order, or
 * LYAP_OK.
 */
int lyap_solve_batched(lyap_handle h, void* stream, int count, const int* n, const int* m,
                       const double* const* A, const int* lda, const double* const* L,
                       const int* ldl, const double* const* S, lyap_precisions prec,
                       const lyap_options* opt, double* const* Z, const int* ldz,
                       const int* z_cap, double* const* D, int* rank, lyap_info* infos,
                       int* codes, int workers, void* ws, size_t ws_bytes);
/* Workspace bytes of lyap_solve_batched for these instances and worker count (``workers``
 * as in lyap_solve_batched, 0 meaning 8): one slice per worker, each large enough for the
 * largest instance. */
int lyap_workspace_size_batched(int count, const int* n, const int* m, int u_s,
                                const lyap_options* opt, int workers, size_t* bytes);

/*
 * lyap_trace_loss -- loss = tr(C X C^T) for X = Z diag(D) Z^T: sum_j D_j ||C z_j||^2.
 *  C  k x n FP64 row-major (ldc >= n); Z n x r (ldz >= r); D r values; loss: host double.
 */
int lyap_trace_loss(lyap_handle h, void* stream, int n, int k, const double* C, int ldc, int r,
                    const double* Z, int ldz, const double* D, double* loss);

/*
 * lyap_trace_loss_grad -- gradients of scale * tr(C X C^T), X solving
 * A X + X A^T + L diag(S) L^T = 0, from the factors X = Z diag(D) Z^T (r columns) and
 * Y = ZY diag(DY) ZY^T (ry columns) of the adjoint solution A^T Y + Y A + C^T C = 0
 * (lyap_solve_adjoint with L = C^T):
 *   dA = 2 scale Y X (n x n, ldda), dL = 2 scale Y L diag(S) (n x m, lddl),
 *   dS = scale diag(L^T Y L) (m), dC = 2 scale C X (k x n, lddc).
 * S NULL means S = I.  Any of dA, dL, dS, dC may be NULL (not computed).  All products run
 * on the FP64 matrix cores; only dA is dense n x n.  Device pointers, row-major; the call
 * returns after the results are written.
 */
int lyap_trace_loss_grad(lyap_handle h, void* stream, int n, int m, int k, const double* L,
                         int ldl, const double* S, const double* C, int ldc, int r,
                         const double* Z, int ldz, const double* D, int ry, const double* ZY,
                         int ldzy, const double* DY, double scale, double* dA, int ldda,
                         double* dL, int lddl, double* dS, double* dC, int lddc);

/*
 * lyap_solve_adjoint -- the adjoint equation A^T Y + Y A + L S L^T = 0 of the same A, by the
 * same method (Alg 2.2 with Alg 3.2 as the solver), for gradients of losses of X: with
 * G = dloss/dX symmetric and Y solving A^T Y + Y A + G = 0, dloss/dA = 2 Y X and
 * dloss/dL = 2 Y L S.  Arguments, outputs and return codes as for lyap_solve
 * (Y ~ Z diag(D) Z^T).  The sign iteration of A^T is the transpose of that of A, so when the
 * workspace holds the inverse sequence of this A at this u_s (the 64-bit content fingerprint
 * of A, n and k_max are compared, not the pointer: an A edited in place is recognised as a
 * different matrix), it is replayed with transposed products and no inversion is computed
 * (info->inversions = 0, info->cache_reused = 1).  Otherwise the sequence is computed.
 */
int lyap_solve_adjoint(lyap_handle h, void* stream, int n, int m, const double* A, int lda,
                       const double* L, int ldl, const double* S, int lds, lyap_precisions prec,
                       const lyap_options* opt, double* Z, int ldz, int z_cap, double* D,
                       int* rank, void* ws, size_t ws_bytes, lyap_info* info);

/* ---------------------------------------------------------------------------------
 * Component entry points.  Each runs one hot-path kernel family on the handle's stream
 * ordering; they exist so that each step of the path can be checked on its own.
 * ------------------------------------------------------------------------------ */

/*
 * lyap_inverse -- inverse of the n x n FP64 matrix A (row-major, lda) at solver precision
 * ``dtype`` (the inversion of Alg 3.1/3.2, first line of the loop): Gauss-Jordan
 * elimination.  pivot == 1: partial pivoting (ties to the lowest row index).  pivot == 2:
 * random butterfly transformation and no pivoting (lyap_options.pivoting = 1; n % 4 == 0,
 * else LYAP_BADARG; no probe, no fallback).  pivot == 0:
 * no row interchanges, which is the same elimination whenever A is strictly column
 * diagonally dominant (partial pivoting then never interchanges rows); for other A the
 * unpivoted elimination may be unstable.  For F32/F16/BF16 the matrix is held in binary32,
 * scaled by a power of two, and every block-update product takes its operands rounded to
 * ``dtype`` with binary32 accumulation.  The result is written in FP64 to Ainv (row-major,
 * ldi).  Returns LYAP_SINGULAR on an exact zero pivot, LYAP_NONFINITE on a NaN/Inf input or
 * result, LYAP_BADARG for n > 4096.
 */
int lyap_inverse(lyap_handle h, void* stream, int dtype, int pivot, int n, const double* A,
                 int lda, double* Ainv, int ldi);

/*
 * lyap_gemm -- C = alpha * op(A) * op(B) + beta * C in FP64 on the FP64 matrix cores, or
 * with operands rounded to ``dtype`` (F32/F16/BF16) and binary32 accumulation.  op(X) is
 * X or X^T (transa/transb = 0/1).  All matrices FP64 row-major.  op(A) is M x K, op(B) is
 * K x N, C is M x N.  A product with few 64 x 64 output tiles (fewer than 256) and K >= 512
 * splits K over several workgroups (as the solver's tall-skinny products do): the partial
 * products are summed in FP64 in a fixed order, so for reduced-precision operands the
 * accumulation is binary32 within each k-chunk (at least 256 long) and FP64 across chunks.
 * The handle keeps a workspace for the partial products.
 */
int lyap_gemm(lyap_handle h, void* stream, int dtype, int transa, int transb, int M, int N,
              int K, double alpha, const double* A, int lda, const double* B, int ldb,
              double beta, double* C, int ldc);

/*
 * lyap_qr_lead -- the same thin QR F = U T when the first c columns Z of F are orthonormal
 * to working precision, as the truncated and updated factors of the solver are
 * (RankTruncLdlt in Alg 3.2, Fragments 2.3 / 2.4).  For p <= n: C = Z^T Y and Y <- Y - Z C
 * twice (block Gram-Schmidt with reorthogonalisation), then the Householder QR of lyap_qr of
 * the projected Y = Q2 R2, so U = [Z, Q2] and T = [[I, C], [0, R2]].  For p > n the columns
 * span the whole space: U = [Z, Q2] (n x n) with Q2 an orthonormal completion of Z (from a
 * seeded random block projected off range(Z) and factored twice) and T = U^T F (n x p,
 * [[I, Z^T Y], [0, Q2^T Y]], not triangular).  Same layouts and errors as lyap_qr (U is
 * n x min(n, p), ldu >= min(n, p)); 0 <= c <= min(n, p) (c < 32 gives lyap_qr's
 * factorisation).  F is not modified.  If Z is not orthonormal the result is not a
 * factorisation of F.
 */
int lyap_qr_lead(lyap_handle h, void* stream, int n, int p, int c, const double* F, int ldf,
                 double* U, int ldu, double* T, int ldt);
/*
 * lyap_qr -- thin QR F = U T of the n x p FP64 matrix F, as used by the residual
 * factorisation and solution update (Fragments 2.1-2.4) and RankTruncLdlt (Alg 3.2):
 * right-looking blocked Householder QR whose panels are factored by a two-level
 * tall-skinny (TSQR) reduction; stable for rank-deficient F.  With k = min(n, p), U is
 * n x k with orthonormal columns (row-major, ldu >= k) and T is k x p upper trapezoidal
 * (row-major, ldt >= p).  F is not modified.
 */
int lyap_qr(lyap_handle h, void* stream, int n, int p, const double* F, int ldf, double* U,
            int ldu, double* T, int ldt);

/*
 * lyap_syev -- spectral decomposition H = V diag(w) V^T of the symmetric p x p FP64 matrix
 * H (row-major, ldh; only its symmetric part is used), as needed by Fragments 2.1-2.4 and
 * the in-solver truncation: cyclic block Jacobi.  w (p) receives the eigenvalues in
 * descending order of magnitude; V (p x p, row-major, ldv) the orthonormal eigenvectors as
 * columns.  H is not modified.
 */
int lyap_syev(lyap_handle h, void* stream, int p, const double* H, int ldh, double* w,
              double* V, int ldv);

/*
 * lyap_jacobi_schedule -- the block-pair schedule lyap_syev sweeps with (host only, no GPU
 * call, no handle): the spectral decompositions of Fragments 2.1-2.4 and Alg 3.2 are
 * computed by cyclic Jacobi, whose pair ordering this fixes.  The matrix is cut into nb
 * blocks (nb even, 2 <= nb <= 256); a sweep is nb rounds of nb/2 disjoint pairs, round t
 * holding the pairs (i, j), i < j, with i + j = t mod nb in increasing i, and in even rounds
 * last the pseudo-pair (t/2, t/2 + nb/2) of the two blocks the round leaves idle (rotated by
 * the identity).  pairs (caller-owned, nb * nb ints): pairs[(t * nb/2 + k) * 2 + h] is block
 * h of pair k of round t.  bmap (caller-owned, nb * nb ints): bmap[t * nb + b] = 2 k + h for
 * block b at half h of pair k of round t.  Returns LYAP_BADARG for an odd or out-of-range nb
 * or a NULL pointer.
 */
int lyap_jacobi_schedule(int nb, int* pairs, int* bmap);

#ifdef __cplusplus
}
#endif
#endif /* LYAP_H */
