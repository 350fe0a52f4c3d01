// CSR products and elementwise kernels on N x p row-major blocks.
#pragma once

#include "dev_common.h"

namespace zolo {

// Ya = A X, and Yb = B X when Yb != null (A, B share the CSR pattern).
void spmm_real(int64_t n, const int64_t* rowptr, const int32_t* colind, const double* a, const double* b,
               const double* X, int64_t ldx, int p, double* Ya, int64_t ldya, double* Yb, int64_t ldyb,
               hipStream_t s);
// complex Hermitian pencils: the same with complex values and blocks
void spmm_cplx(int64_t n, const int64_t* rowptr, const int32_t* colind, const zd* a, const zd* b, const zd* X,
               int64_t ldx, int p, zd* Ya, int64_t ldya, zd* Yb, int64_t ldyb, hipStream_t s);
// R = T - (A - sigma B) X  with X complex, T real (refinement residual, FP64).
void spmm_shift_resid(int64_t n, const int64_t* rowptr, const int32_t* colind, const double* a, const double* b,
                      double sr, double si, const zd* X, const double* T, int64_t ldt, int p, zd* R, hipStream_t s);
// complex Hermitian pencils: the same with complex values and a complex T
void spmm_shift_resid(int64_t n, const int64_t* rowptr, const int32_t* colind, const zd* a, const zd* b, double sr,
                      double si, const zd* X, const zd* T, int64_t ldt, int p, zd* R, hipStream_t s);
// row permutations of N x p blocks: gather dst[i] = src[idx[i]], scatter dst[idx[i]] = src[i]
template <typename T>
void rows_gather(T* dst, int64_t ldd, const T* src, int64_t lds, const int32_t* idx, int64_t n, int p, hipStream_t s);
template <typename T>
void rows_scatter(T* dst, int64_t ldd, const T* src, int64_t lds, const int32_t* idx, int64_t n, int p,
                  hipStream_t s);
// W = alpha V (real)
void scale_copy(double* W, int64_t ldw, const double* V, int64_t ldv, double alpha, int64_t n, int p, hipStream_t s);
void scale_copy(zd* W, int64_t ldw, const zd* V, int64_t ldv, double alpha, int64_t n, int p, hipStream_t s);
// W += w X + conj(w) Xc  (complex pencils: a pole and its conjugate, X and Xc contiguous N x p)
void axpy_pair(zd* W, int64_t ldw, const zd* X, const zd* Xc, double wr, double wi, int64_t n, int p, hipStream_t s);
// W += 2 * Re(w * X)  (X complex, contiguous N x p)
void axpy_re(double* W, int64_t ldw, const zd* X, double wr, double wi, int64_t n, int p, hipStream_t s);
// W = alpha V + sum_{j < r} 2 Re(w_j X_j), X_j complex N x p (ld p) at X + j * xstride; r <= 16.
// One pass, the terms added in the order scale_copy then axpy_re for j = 0, 1, ... would add them.
struct GCombineCoef {
  double wr[16], wi[16];
};
void g_combine_real(double* W, int64_t ldw, const double* V, int64_t ldv, double alpha, const zd* X, int64_t xstride,
                    const GCombineCoef& w, int r, int64_t n, int p, hipStream_t s);
// dst = conj(src)
template <typename T>
void conj_copy(T* dst, const T* src, int64_t n, hipStream_t s);
// X = cvt(D); X += cvt(D)
void set_lowp(zd* X, const zf* D, int64_t n, hipStream_t s);
void add_lowp(zd* X, const zf* D, int64_t n, hipStream_t s);
void add_same(zd* X, const zd* D, int64_t n, hipStream_t s);
// column sums of |x|^2 (N x p row-major, real or complex) into out[p] (device)
void colnorm2_real(const double* X, int64_t ldx, int64_t n, int p, double* partial, double* out, hipStream_t s);
void colnorm2_cplx(const zd* X, int64_t n, int p, double* partial, double* out, hipStream_t s);
int colnorm_partials(int64_t n);
// Residual norms of approximate eigenpairs of (A, B) (rows in the pencil's ordering, X
// in the caller's: X row perm[i] belongs to pencil row i):
//   out[c] = ||A x_c - lam_c B x_c||_2 / ((normA + |lam_c| normB) ||x_c||_2),  c < p <= kResidMaxCols.
// partial: kResidGroups * 2 * p doubles of device scratch (fully overwritten); lam, out: device.
constexpr int kResidGroups = 512;
constexpr int kResidMaxCols = 512;
template <typename T>
void eig_resid_norms(int64_t n, const int64_t* rowptr, const int32_t* colind, const T* a, const T* b,
                     const int32_t* perm, const T* X, int64_t ldx, int p, const double* lam, double normA,
                     double normB, double* partial, double* out, hipStream_t s);
// Y = s1 Y + s0 V (N x p row-major blocks)
template <typename T>
void axpby_rows(T* Y, int64_t ldy, const T* V, int64_t ldv, double s0, double s1, int64_t n, int p, hipStream_t s);
// out[0 .. n) = i.i.d. N(0, 1) draws of the seeded generator (the start block
// zolo_solve and the serving loop draw when the caller passes none)
void gaussian_fill(uint64_t seed, int64_t n, double* out, hipStream_t s);
// asynchronous clear of device memory
void fill_zero_bytes(void* p, size_t bytes, hipStream_t s);

}  // namespace zolo
