// CSR sparse products (S3: B V, A Y, B Y; S4': refinement residuals) and
// elementwise kernels (S5: the G combine of eq. solve).  Blocks are N x p
// row-major, so the p columns of one row are contiguous and every nonzero
// reads one contiguous row of X.
#include "sparse.h"

namespace zolo {
namespace {

__global__ void spmm_real_kernel(int64_t n, const int64_t* __restrict__ rp, const int32_t* __restrict__ ci,
                                 const double* __restrict__ a, const double* __restrict__ b,
                                 const double* __restrict__ X, int64_t ldx, int p, double* __restrict__ Ya,
                                 int64_t ldya, double* __restrict__ Yb, int64_t ldyb) {
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n * p) return;
  int64_t i = e / p;
  int c = (int)(e % p);
  double sa = 0.0, sb = 0.0;
  const int64_t e0 = rp[i], e1 = rp[i + 1];
  if (Yb) {
    for (int64_t q = e0; q < e1; ++q) {
      double x = X[(int64_t)ci[q] * ldx + c];
      sa = fma(a[q], x, sa);
      sb = fma(b[q], x, sb);
    }
    Yb[i * ldyb + c] = sb;
  } else {
    for (int64_t q = e0; q < e1; ++q) sa = fma(a[q], X[(int64_t)ci[q] * ldx + c], sa);
  }
  Ya[i * ldya + c] = sa;
}

// complex Hermitian pencils: complex values, complex blocks
__global__ void spmm_cplx_kernel(int64_t n, const int64_t* __restrict__ rp, const int32_t* __restrict__ ci,
                                 const zd* __restrict__ a, const zd* __restrict__ b, const zd* __restrict__ X,
                                 int64_t ldx, int p, zd* __restrict__ Ya, int64_t ldya, zd* __restrict__ Yb,
                                 int64_t ldyb) {
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n * p) return;
  int64_t i = e / p;
  int c = (int)(e % p);
  zd sa{0.0, 0.0}, sb{0.0, 0.0};
  const int64_t e0 = rp[i], e1 = rp[i + 1];
  for (int64_t q = e0; q < e1; ++q) {
    const zd x = X[(int64_t)ci[q] * ldx + c];
    sa = fma_(sa, a[q], x);
    if (Yb) sb = fma_(sb, b[q], x);
  }
  Ya[i * ldya + c] = sa;
  if (Yb) Yb[i * ldyb + c] = sb;
}

__global__ void spmm_shift_resid_kernel(int64_t n, const int64_t* __restrict__ rp, const int32_t* __restrict__ ci,
                                        const double* __restrict__ a, const double* __restrict__ b, double sr,
                                        double si, const zd* __restrict__ X, const double* __restrict__ T,
                                        int64_t ldt, int p, zd* __restrict__ R) {
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n * p) return;
  int64_t i = e / p;
  int c = (int)(e % p);
  double re = 0.0, im = 0.0;
  for (int64_t q = rp[i]; q < rp[i + 1]; ++q) {
    zd x = X[(int64_t)ci[q] * p + c];
    double kr = a[q] - sr * b[q], ki = -si * b[q];  // (A - sigma B)_iq
    re = fma(kr, x.re, fma(-ki, x.im, re));
    im = fma(kr, x.im, fma(ki, x.re, im));
  }
  R[i * p + c] = zd{T[i * ldt + c] - re, -im};
}

template <typename T>
__global__ void rows_gather_kernel(T* __restrict__ dst, int64_t ldd, const T* __restrict__ src, int64_t lds,
                                   const int32_t* __restrict__ idx, int64_t n, int p) {
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n * p) return;
  int64_t i = e / p;
  int c = (int)(e % p);
  dst[i * ldd + c] = src[(int64_t)idx[i] * lds + c];
}

template <typename T>
__global__ void rows_scatter_kernel(T* __restrict__ dst, int64_t ldd, const T* __restrict__ src, int64_t lds,
                                    const int32_t* __restrict__ idx, int64_t n, int p) {
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n * p) return;
  int64_t i = e / p;
  int c = (int)(e % p);
  dst[(int64_t)idx[i] * ldd + c] = src[i * lds + c];
}

__global__ void scale_copy_kernel(double* __restrict__ W, int64_t ldw, const double* __restrict__ V, int64_t ldv,
                                  double alpha, int64_t n, int p) {
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n * p) return;
  int64_t i = e / p;
  int c = (int)(e % p);
  W[i * ldw + c] = alpha * V[i * ldv + c];
}

__global__ void scale_copy_cplx_kernel(zd* __restrict__ W, int64_t ldw, const zd* __restrict__ V, int64_t ldv,
                                       double alpha, int64_t n, int p) {
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n * p) return;
  int64_t i = e / p;
  int c = (int)(e % p);
  W[i * ldw + c] = scl(V[i * ldv + c], alpha);
}

// W += w X + conj(w) Xc  (the pole and its conjugate, complex pencils)
__global__ void axpy_pair_kernel(zd* __restrict__ W, int64_t ldw, const zd* __restrict__ X, const zd* __restrict__ Xc,
                                 double wr, double wi, int64_t n, int p) {
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n * p) return;
  int64_t i = e / p;
  int c = (int)(e % p);
  const zd x = X[e], y = Xc[e];
  zd& o = W[i * ldw + c];
  o.re += wr * x.re - wi * x.im + wr * y.re + wi * y.im;
  o.im += wr * x.im + wi * x.re + wr * y.im - wi * y.re;
}

template <typename T>
__global__ void conj_copy_kernel(T* __restrict__ dst, const T* __restrict__ src, int64_t n) {
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < n) dst[e] = conj_(src[e]);
}

__global__ void axpy_re_kernel(double* __restrict__ W, int64_t ldw, const zd* __restrict__ X, double wr, double wi,
                               int64_t n, int p) {
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n * p) return;
  int64_t i = e / p;
  int c = (int)(e % p);
  zd x = X[e];
  W[i * ldw + c] += 2.0 * (wr * x.re - wi * x.im);
}

__global__ void add_lowp_kernel(zd* __restrict__ X, const zf* __restrict__ D, int64_t n) {
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  zf d = D[e];
  X[e].re += (double)d.re;
  X[e].im += (double)d.im;
}

__global__ void add_same_kernel(zd* __restrict__ X, const zd* __restrict__ D, int64_t n) {
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  X[e].re += D[e].re;
  X[e].im += D[e].im;
}

constexpr int CN_ROWS = 1024;  // rows per partial sum

// partial[b][c] = sum over rows of chunk b of |x_ic|^2
template <bool CPLX>
__global__ void colnorm_partial_kernel(const double* __restrict__ X, int64_t ldx, int64_t n, int p,
                                       double* __restrict__ partial) {
  const int64_t r0 = (int64_t)blockIdx.x * CN_ROWS;
  const int64_t r1 = (r0 + CN_ROWS < n) ? r0 + CN_ROWS : n;
  for (int c = threadIdx.x; c < p; c += blockDim.x) {
    double s = 0.0;
    for (int64_t i = r0; i < r1; ++i) {
      if (CPLX) {
        double re = X[2 * (i * ldx + c)], im = X[2 * (i * ldx + c) + 1];
        s = fma(re, re, fma(im, im, s));
      } else {
        double v = X[i * ldx + c];
        s = fma(v, v, s);
      }
    }
    partial[(int64_t)blockIdx.x * p + c] = s;
  }
}

__global__ void colnorm_final_kernel(const double* __restrict__ partial, int nb, int p, double* __restrict__ out) {
  int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= p) return;
  double s = 0.0;
  for (int b = 0; b < nb; ++b) s += partial[(int64_t)b * p + c];
  out[c] = s;
}

inline unsigned nblk(int64_t tot) { return (unsigned)((tot + 255) / 256); }

}  // namespace

template <typename T>
void conj_copy(T* dst, const T* src, int64_t n, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(conj_copy_kernel<T>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, dst, src, n);
}
template void conj_copy<zd>(zd*, const zd*, int64_t, hipStream_t);
template void conj_copy<zf>(zf*, const zf*, int64_t, hipStream_t);

void spmm_cplx(int64_t n, const int64_t* rowptr, const int32_t* colind, const zd* a, const zd* b, const zd* X,
               int64_t ldx, int p, zd* Ya, int64_t ldya, zd* Yb, int64_t ldyb, hipStream_t s) {
  int64_t tot = n * p;
  if (tot == 0) return;
  hipLaunchKernelGGL(spmm_cplx_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, n, rowptr, colind, a, b,
                     X, ldx, p, Ya, ldya, Yb, ldyb);
}

void scale_copy(zd* W, int64_t ldw, const zd* V, int64_t ldv, double alpha, int64_t n, int p, hipStream_t s) {
  int64_t tot = n * p;
  if (tot == 0) return;
  hipLaunchKernelGGL(scale_copy_cplx_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, W, ldw, V, ldv,
                     alpha, n, p);
}

void axpy_pair(zd* W, int64_t ldw, const zd* X, const zd* Xc, double wr, double wi, int64_t n, int p, hipStream_t s) {
  int64_t tot = n * p;
  if (tot == 0) return;
  hipLaunchKernelGGL(axpy_pair_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, W, ldw, X, Xc, wr, wi, n,
                     p);
}

void spmm_real(int64_t n, const int64_t* rp, const int32_t* ci, const double* a, const double* b, const double* X,
               int64_t ldx, int p, double* Ya, int64_t ldya, double* Yb, int64_t ldyb, hipStream_t s) {
  if (n * p == 0) return;
  hipLaunchKernelGGL(spmm_real_kernel, dim3(nblk(n * p)), dim3(256), 0, s, n, rp, ci, a, b, X, ldx, p, Ya, ldya, Yb,
                     ldyb);
}

void spmm_shift_resid(int64_t n, const int64_t* rp, const int32_t* ci, const double* a, const double* b, double sr,
                      double si, const zd* X, const double* T, int64_t ldt, int p, zd* R, hipStream_t s) {
  if (n * p == 0) return;
  hipLaunchKernelGGL(spmm_shift_resid_kernel, dim3(nblk(n * p)), dim3(256), 0, s, n, rp, ci, a, b, sr, si, X, T, ldt,
                     p, R);
}

template <typename T>
void rows_gather(T* dst, int64_t ldd, const T* src, int64_t lds, const int32_t* idx, int64_t n, int p,
                 hipStream_t s) {
  if (n * p == 0) return;
  hipLaunchKernelGGL(rows_gather_kernel<T>, dim3(nblk(n * p)), dim3(256), 0, s, dst, ldd, src, lds, idx, n, p);
}
template <typename T>
void rows_scatter(T* dst, int64_t ldd, const T* src, int64_t lds, const int32_t* idx, int64_t n, int p,
                  hipStream_t s) {
  if (n * p == 0) return;
  hipLaunchKernelGGL(rows_scatter_kernel<T>, dim3(nblk(n * p)), dim3(256), 0, s, dst, ldd, src, lds, idx, n, p);
}
template void rows_gather<double>(double*, int64_t, const double*, int64_t, const int32_t*, int64_t, int, hipStream_t);
template void rows_scatter<double>(double*, int64_t, const double*, int64_t, const int32_t*, int64_t, int,
                                   hipStream_t);
template void rows_gather<zd>(zd*, int64_t, const zd*, int64_t, const int32_t*, int64_t, int, hipStream_t);
template void rows_scatter<zd>(zd*, int64_t, const zd*, int64_t, const int32_t*, int64_t, int, hipStream_t);

void scale_copy(double* W, int64_t ldw, const double* V, int64_t ldv, double alpha, int64_t n, int p, hipStream_t s) {
  if (n * p == 0) return;
  hipLaunchKernelGGL(scale_copy_kernel, dim3(nblk(n * p)), dim3(256), 0, s, W, ldw, V, ldv, alpha, n, p);
}
void axpy_re(double* W, int64_t ldw, const zd* X, double wr, double wi, int64_t n, int p, hipStream_t s) {
  if (n * p == 0) return;
  hipLaunchKernelGGL(axpy_re_kernel, dim3(nblk(n * p)), dim3(256), 0, s, W, ldw, X, wr, wi, n, p);
}
void add_lowp(zd* X, const zf* D, int64_t n, hipStream_t s) {
  if (n == 0) return;
  hipLaunchKernelGGL(add_lowp_kernel, dim3(nblk(n)), dim3(256), 0, s, X, D, n);
}
void add_same(zd* X, const zd* D, int64_t n, hipStream_t s) {
  if (n == 0) return;
  hipLaunchKernelGGL(add_same_kernel, dim3(nblk(n)), dim3(256), 0, s, X, D, n);
}

int colnorm_partials(int64_t n) { return (int)((n + CN_ROWS - 1) / CN_ROWS); }

void colnorm2_real(const double* X, int64_t ldx, int64_t n, int p, double* partial, double* out, hipStream_t s) {
  int nb = colnorm_partials(n);
  if (nb == 0) return;
  hipLaunchKernelGGL(colnorm_partial_kernel<false>, dim3(nb), dim3(128), 0, s, X, ldx, n, p, partial);
  hipLaunchKernelGGL(colnorm_final_kernel, dim3((p + 127) / 128), dim3(128), 0, s, partial, nb, p, out);
}
void colnorm2_cplx(const zd* X, int64_t n, int p, double* partial, double* out, hipStream_t s) {
  int nb = colnorm_partials(n);
  if (nb == 0) return;
  hipLaunchKernelGGL(colnorm_partial_kernel<true>, dim3(nb), dim3(128), 0, s, (const double*)X, (int64_t)p, n, p,
                     partial);
  hipLaunchKernelGGL(colnorm_final_kernel, dim3((p + 127) / 128), dim3(128), 0, s, partial, nb, p, out);
}

void fill_zero_bytes(void* p, size_t bytes, hipStream_t s) {
  if (bytes) (void)hipMemsetAsync(p, 0, bytes, s);
}

}  // namespace zolo
