// Block Arnoldi / shifted least-squares / Rayleigh-Ritz helper kernels.
#pragma once

#include "dev_common.h"

namespace zolo {

// Functions templated on the block scalar T: double (real pencils) or zd
// (complex Hermitian pencils); "^T" below reads "^H" for complex T.

// out(i,j) (ld_out) = [out +] sum_s partial[s](i,j)  (each partial M x N col-major, ld M),
// summed in a fixed order (groups of kReduceGroup consecutive partials, then
// the groups); with S > kReduceGroup the partials are overwritten.
constexpr int kReduceGroup = 32;
template <typename T>
void reduce_partials(T* out, int64_t ld_out, T* partial, int S, int M, int N, bool add, hipStream_t s);

// Cholesky of a p x p Hermitian positive matrix G (col-major): G + shift*I = R^H R,
// R upper; writes R and R^{-1} (col-major p x p).  flag[0] = 1 on a nonpositive pivot.
template <typename T>
void chol_upper_inv(const T* G, int p, double rel_shift, T* R, T* Rinv, int* flag, hipStream_t s);
// C = A * B for upper-triangular p x p matrices (col-major)
template <typename T>
void upper_mul(const T* A, const T* B, T* C, int p, hipStream_t s);
// copy a p x p block into H at (row0, col0), ld
template <typename T>
void put_block(T* H, int64_t ldh, int64_t row0, int64_t col0, const T* X, int p, hipStream_t s);

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
template <typename T>
void hls_init(const HlsState& st, const T* R0, hipStream_t s);
// bring block column k of H (ldh) into every shift's R, apply the earlier
// reflectors, factor the new panel and update g; res[s*p + c] = LS residual
// norm of column c for shift s.
template <typename T>
void hls_step(const HlsState& st, const T* H, int64_t ldh, int k, double* res, hipStream_t s);
// Y_s = R_s^{-1} g_s (first mp rows), Y: per shift (m p) x p col-major ld m p
void hls_backsolve(const HlsState& st, int m, zd* Y, hipStream_t s);
// Restarted multi-shift block GMRES with collinear residuals:
// g_s = G0_s (p x p col-major at G0 + s p p) in the first p rows, zero below
void hls_init_multi(const HlsState& st, const zd* G0, hipStream_t s);
// columns of Z (ld ldz, rows [0, (m+1)p)) times Q_s (adjoint: Q_s^H), Q_s the
// product of shift s's reflectors of blocks 0..m-1; shift < 0: every shift, its
// columns at Z + s zstride
void hls_apply_q(const HlsState& st, int shift, int m, zd* Z, int64_t ldz, int64_t zstride, int ncols, bool adjoint,
                 hipStream_t s);
// g_s(0:mp, :) -= T_s(0:mp, :) W_s for every shift s != skip (T_s: (m+1)p x p
// col-major at T + s tstride, W_s: p x p col-major at W + s p p)
void hls_collinear_rhs(const HlsState& st, int m, const zd* T, int64_t tstride, const zd* W, int skip, hipStream_t s);
// Er (rows x 2p col-major doubles): columns 2c, 2c + 1 = Re, Im of column c of Z (ld ldz)
void cols_re_im(const zd* Z, int64_t ldz, int64_t rows, int p, double* Er, hipStream_t s);
// C(i,c) = sum_s coef[s] * Y_s(i,c): real part for real pencils (double C),
// complex for complex pencils (zd C).  C: (m p) x p col-major
void hls_combine(const zd* Y, int m, int p, int nshift, const double* coef, double* C, hipStream_t s);
void hls_combine(const zd* Y, int m, int p, int nshift, const double* coef, zd* C, hipStream_t s);

// ---- Rayleigh-Ritz reduction on the device (single workgroup) ----
// Inputs At, Bt (n x n, col-major, Hermitian).  Outputs theta[k] (ascending),
// Cmat (n x k col-major, ld n) with X = Y Cmat B-orthonormal, *k_out (-1 when
// one of the two Hermitian eigensolves did not converge).
// work: 6 n^2 T values + 2 n doubles + 2 n ints.
template <typename T>
void rr_reduce(const T* At, const T* Bt, int n, double tau_rank, double* theta, T* Cmat, int* k_out, T* work,
               hipStream_t s);

// per column c < k: out[3c..3c+2] partial sums of |AX - theta BX|^2, |X|^2, |BX|^2
template <typename T>
void resid_norms(const T* AX, const T* BX, const T* X, const double* theta, int64_t n, int k, double* partial,
                 double* out, hipStream_t s);

}  // namespace zolo
