// Internal entry points shared between the kernel files and the host driver.
#pragma once

#include "common.hpp"

namespace lyap {

// ---- inverse.hip
size_t inverse_workspace_bytes(Prec op, int n);
// A^{-1} at solver precision ``op`` into ``out`` (FP64).  flags_dev[0] <- 1 on an exact zero
// pivot, flags_dev[1] <- 1 on a non-finite input or result (device ints zeroed by caller).
// pivot = false skips the pivot search (pivot row = diagonal row); valid when A is strictly
// column diagonally dominant, where partial pivoting makes no interchanges.
// With logdet_dev, log|det A| (from the pivots) is written to logdet_dev[0].
int invert(hipStream_t s, Prec op, int n, const double* A, long lda, double* out, long ldo,
           Arena& ws, int* flags_dev, bool pivot = true, KernTimer* kt = nullptr,
           double* logdet_dev = nullptr);

// ---- rbt.hip
size_t rbt_workspace_bytes(int n);
// A^{-1} = V (U^T A V)^{-1} U^T with random depth-2 butterflies U, V (seeded) and Gauss-Jordan
// without pivoting on the transformed matrix; n must be a multiple of 4.  With probe, the
// residual ||A (A^{-1} x) - x||_2 / ||x||_2 for a seeded random x is written to probe[0]; with
// logdet, log|det A|.  Timed as one inversion (family 0) when kt is given.
int rbt_invert(hipStream_t s, Prec op, int n, const double* A, long lda, double* out, long ldo,
               Arena& ws, int* flags_dev, KernTimer* kt, double* logdet,
               unsigned long long seed, double* probe);
// The same residual probe for any computed inverse.
int probe_inverse(hipStream_t s, int n, const double* A, long lda, const double* Ainv, long ldi,
                  Arena& ws, unsigned long long seed, double* probe);

// ---- elem.hip
int fill_int(hipStream_t s, int* p, int count, int value);
int fill_f64(hipStream_t s, double* p, long count, double value);
// Copy a rows x cols block (row-major, lds / ldd) with optional per-column scale (may be NULL)
// and global scale.
int copy_block(hipStream_t s, int rows, int cols, const double* src, long lds, double* dst,
               long ldd, const double* colscale = nullptr, double scale = 1.0);
// dst += alpha src over a rows x cols block.
int add_block(hipStream_t s, int rows, int cols, double alpha, const double* src, long lds,
              double* dst, long ldd);
// M_ii += p for i < n.
int add_diag(hipStream_t s, int n, double* M, long ld, double p);
// Round an FP64 rows x cols block to storage ``st`` (F64/F32/F16/BF16) into dst (ld = cols).
int cast_store(hipStream_t s, Store st, int rows, int cols, const double* src, long lds,
               void* dst);
// e_dev[0] <- e with 2^(e-1) <= max|A_ij| < 2^e (0 for a zero block); bad_dev[0] <- 1 for a
// NaN or infinite entry (bad_dev may be NULL).  partial >= 1024 doubles.
int absmax_exp(hipStream_t s, int rows, int cols, const double* A, long lda, int* e_dev,
               int* bad_dev, double* partial);
// dst = RNE(2^-e src) at storage ``st`` (row-major, ld = cols), e = e_dev[0] (NULL: 0); one
// rounding from FP64 for every format.
int cast_scaled(hipStream_t s, Store st, int rows, int cols, const double* src, long lds,
                void* dst, const int* e_dev);
// X <- RNE(X) at storage ``st`` in place (the values stay in FP64 storage).
int round_block(hipStream_t s, Store st, int rows, int cols, double* X, long ldx);
// e_dev[j] <- e_j with 2^(e_j-1) <= max_i |X_ij| < 2^e_j (0 for a zero column); bad_dev[0] <- 1
// for a non-finite entry.  bits: cols scratch words.
int col_exponents(hipStream_t s, int rows, int cols, const double* X, long ldx, int* e_dev,
                  int* bad_dev, unsigned long long* bits);
// 64-bit content fingerprint of a rows x cols FP64 block (order-independent integer sum).
int fingerprint(hipStream_t s, int rows, int cols, const double* A, long lda,
                unsigned long long* out);
// sum of squares of a rows x cols FP64 block into out[0] (deterministic two-stage).
int sumsq(hipStream_t s, int rows, int cols, const double* A, long lda, double* out,
          double* partial /* >= 256 doubles, >= 1024 when rows >= 1024 */);
// Newton update: Anew = 0.5 (mu A + Ainv / mu), mu = mu_dev[0]; accumulates into out4:
// out4[0] = ||Anew - A||_F^2, out4[1] = ||Anew||_F^2, out4[2] = ||Anew + I||_1.
// colsum must hold n doubles, partial >= 3*256 doubles.
int newton_update(hipStream_t s, int n, const double* A, long lda, const double* Ainv, long ldi,
                  const double* mu_dev, double* Anew, long ldn, double* out4, double* colsum,
                  double* partial);
// Scaling parameter (device scalars, 1 when scaling == 0): mode 0 Frobenius
// sqrt(sqrt(x) / sqrt(y)) from x = ||A^-1||_F^2, y = ||A||_F^2; mode 1 determinantal
// exp(-x / n) from x = log|det A|; mode 2 sqrt(x / y) from estimates x of A^-1 and y of A.
int newton_mu(hipStream_t s, int mode, const double* x, const double* y, int n, int scaling,
              double* mu_dev);
// Power-iteration estimate of ||M||_2 (iters steps on M^T M from the normalised ones vector)
// into out[0]; work: 19 n doubles.
int norm2_est(hipStream_t s, int n, const double* M, long ld, int iters, double* out,
              double* work);
// Estimate of the spectral radius rho(M): the geometric mean of ||M x_k|| over the last half
// of ``iters`` normalised power steps, into out[0]; work: 19 n doubles.
int specrad_est(hipStream_t s, int n, const double* M, long ld, int iters, double* out,
                double* work);

// sum_ij d_i d_j G_ij^2 for a symmetric c x c G into out[0]; partial >= 256 doubles.
int wsumsq(hipStream_t s, int c, const double* G, long ldg, const double* d, double* out,
           double* partial);
// dst[:, k] = src[:, idx[k]] (idx on the device), rows x count.
int gather_cols(hipStream_t s, int rows, int count, const double* src, long lds, const int* idx,
                double* dst, long ldd);
// out[0] = sum_ij w[j] X_ij^2 (rows x cols, one block).
int colw_sumsq(hipStream_t s, int rows, int cols, const double* X, long ldx, const double* w,
               double* out);
// out[c] = sum_i w[i] X_ic^2.
int roww_colsumsq(hipStream_t s, int rows, int cols, const double* X, long ldx, const double* w,
                  double* out);
// out[0] = trace(A) (n x n).
int trace(hipStream_t s, int n, const double* A, long lda, double* out);

// ---- qr.hip
size_t qr_workspace_bytes(int n, int p);
// Thin QR F = U T (U n x min(n,p) explicit, T min(n,p) x p upper trapezoidal); F is copied
// first.
int qr(hipStream_t s, int n, int p, const double* F, long ldf, double* U, long ldu, double* T,
       long ldt, Arena& ws, KernTimer* kt = nullptr);
// The same factorisation when the first c columns of F are orthonormal (block Gram-Schmidt
// against them, Householder QR of the rest); overwrites columns c.. of F.  With p > n and
// ``complete`` (32 <= c <= n, scratch permitting) U = [Z, Q2] is an orthonormal completion of
// Z and T = U^T F (n x p, not triangular).  Falls back to ``qr`` otherwise when c < 32,
// c >= p or p > n.
int qr_lead(hipStream_t s, int n, int p, int c, double* F, long ldf, double* U, long ldu,
            double* T, long ldt, Arena& ws, KernTimer* kt = nullptr, bool complete = true);

// ---- eig.hip
size_t syev_workspace_bytes(int p);
// The block-pair schedule of the Jacobi sweeps for nb (even) blocks: pairs[(t np + k) 2 + h]
// is block h of pair k of round t (np = nb / 2 pairs, nb rounds), bmap[t nb + b] = 2 k + h.
// Host only.
int jacobi_schedule(int nb, int* pairs, int* bmap);
// H = V diag(w) V^T, w sorted by descending |w|.  ``sweeps_out`` (host, optional).
// Rotations are skipped below tol ||H||_F / (4 p) and, with ``relative``, also below
// tol sqrt(|h_pp h_qq|) (eigenvalues accurate relative to their own size rather than to
// ||H||).  With ``single`` the rotations run in FP32 (tol must then be >= 1e-6); H, w and V
// stay FP64.
int syev(hipStream_t s, int p, const double* H, long ldh, double* w, double* V, long ldv,
         Arena& ws, double tol_rel, int* sweeps_out, KernTimer* kt = nullptr,
         bool relative = true, bool single = false);

}  // namespace lyap
