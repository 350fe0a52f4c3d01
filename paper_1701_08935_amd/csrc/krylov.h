// Block Arnoldi / shifted least-squares / Rayleigh-Ritz helper kernels.
#pragma once

#include "dev_common.h"

namespace zolo {

// out(i,j) (ld_out) = [out +] sum_s partial[s](i,j)  (each partial M x N col-major, ld M)
void reduce_partials(double* out, int64_t ld_out, const double* partial, int S, int M, int N, bool add,
                     hipStream_t s);

// Cholesky of a p x p symmetric positive matrix G (col-major): G + shift*I = R^T R,
// R upper; writes R and R^{-1} (col-major p x p).  flag[0] = 1 on a nonpositive pivot.
void chol_upper_inv(const double* G, int p, double rel_shift, double* R, double* Rinv, int* flag, hipStream_t s);
// C = A * B for upper-triangular p x p matrices (col-major)
void upper_mul(const double* A, const double* B, double* C, int p, hipStream_t s);
// copy a p x p block into H at (row0, col0), ld
void put_block(double* H, int64_t ldh, int64_t row0, int64_t col0, const double* X, int p, hipStream_t s);

// ---- shifted block Hessenberg least squares (one problem per shift) ----
struct HlsState {
  zd* R;        // per shift: ldr x (mmax p), col-major
  zd* refl;     // per shift: mmax * p reflectors of length p+1
  double* tau;  // per shift: mmax * p
  zd* g;        // per shift: ldr x p, col-major (transformed E1 R0)
  int64_t ldr;  // (mmax + 1) p
  int mmax, p, nshift;
  const double* shift_im;  // device: imaginary parts (shifts are i * shift_im[s])
};
// initialise g = E1 R0 for every shift
void hls_init(const HlsState& st, const double* R0, hipStream_t s);
// bring block column k of H (ldh) into every shift's R, apply the earlier
// reflectors, factor the new panel and update g; res[s*p + c] = LS residual
// norm of column c for shift s.
void hls_step(const HlsState& st, const double* H, int64_t ldh, int k, double* res, hipStream_t s);
// Y_s = R_s^{-1} g_s (first mp rows), Y: per shift (m p) x p col-major ld m p
void hls_backsolve(const HlsState& st, int m, zd* Y, hipStream_t s);
// C(i,c) = coef * sum_s a[s] * Re(Y_s(i,c))  (real pencils), C: (m p) x p col-major
void hls_combine_real(const zd* Y, int m, int p, int nshift, const double* coef, double* C, hipStream_t s);

// ---- Rayleigh-Ritz reduction on the device (single workgroup) ----
// Inputs At, Bt (n x n, col-major, symmetric).  Outputs theta[k] (ascending),
// Cmat (n x k col-major, ld n) with X = Y Cmat B-orthonormal, *k_out.
// work: 6 n^2 + 8 n doubles.
void rr_reduce(const double* At, const double* Bt, int n, double tau_rank, double* theta, double* Cmat, int* k_out,
               double* work, hipStream_t s);

// per column c < k: out[3c..3c+2] partial sums of |AX - theta BX|^2, |X|^2, |BX|^2
void resid_norms(const double* AX, const double* BX, const double* X, const double* theta, int64_t n, int k,
                 double* partial, double* out, hipStream_t s);

}  // namespace zolo
