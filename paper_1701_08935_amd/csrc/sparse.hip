// CSR sparse products (S3: B V, A Y, B Y; S4': refinement residuals) and
// elementwise kernels (S5: the G combine of eq. solve).  Blocks are N x p
// row-major, so the p columns of one row are contiguous and every nonzero
// reads one contiguous row of X.
#include "sparse.h"

namespace zolo {
namespace {

// The SpMMs below give one wave to one matrix row: lanes cover the p columns
// (two per lane per pass of 128), so every X row a nonzero selects is read as
// whole 512-byte segments, and the row's column indices and values are
// wave-uniform (scalar loads).  The hardware hands workgroups to the 8 XCDs
// round-robin and each XCD has its own L2; the logical row block is remapped
// so that every XCD takes one contiguous range of rows, and the X rows that
// neighbouring matrix rows share are fetched into one L2, not several.
constexpr int kSpmmRows = 4;  // rows (waves) per 256-thread workgroup

// streaming (non-temporal) stores of a 16-byte pair
__device__ inline void store_stream(double* p, double2 v) {
  __builtin_nontemporal_store(v.x, p);
  __builtin_nontemporal_store(v.y, p + 1);
}

// logical workgroup of physical workgroup blk in a grid of nb8 (a multiple of 8)
__device__ inline int64_t xcd_block(int64_t blk, int64_t nb8) { return (blk & 7) * (nb8 >> 3) + (blk >> 3); }
inline unsigned xcd_grid(int64_t rows) { return (unsigned)((((rows + kSpmmRows - 1) / kSpmmRows) + 7) & ~int64_t(7)); }

__device__ inline int64_t spmm_row() {
  const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  return xcd_block(blockIdx.x, gridDim.x) * kSpmmRows + w;
}

template <bool HB>
__global__ __launch_bounds__(256) void spmm_real_kernel(int64_t n, const int64_t* __restrict__ rp,
                                                        const int32_t* __restrict__ ci, const double* __restrict__ a,
                                                        const double* __restrict__ b, const double* __restrict__ X,
                                                        int64_t ldx, int p, double* __restrict__ Ya, int64_t ldya,
                                                        double* __restrict__ Yb, int64_t ldyb) {
  const int64_t i = spmm_row();
  if (i >= n) return;
  const int lane = threadIdx.x & 63;
  const int64_t e0 = rp[i], e1 = rp[i + 1];
  for (int c0 = 0; c0 < p; c0 += 128) {
    const int c1 = c0 + lane, c2 = c1 + 64;
    const bool v1 = c1 < p, v2 = c2 < p;
    const int l1 = v1 ? c1 : p - 1, l2 = v2 ? c2 : p - 1;  // loads stay in the row; unused lanes are not stored
    double sa1 = 0.0, sa2 = 0.0, sb1 = 0.0, sb2 = 0.0;
#pragma unroll 4
    for (int64_t q = e0; q < e1; ++q) {
      const double* xr = X + (int64_t)ci[q] * ldx;
      const double x1 = xr[l1], x2 = xr[l2];
      const double av = a[q];
      sa1 = fma(av, x1, sa1);
      sa2 = fma(av, x2, sa2);
      if constexpr (HB) {
        const double bv = b[q];
        sb1 = fma(bv, x1, sb1);
        sb2 = fma(bv, x2, sb2);
      }
    }
    if (v1) {
      Ya[i * ldya + c1] = sa1;
      if constexpr (HB) Yb[i * ldyb + c1] = sb1;
    }
    if (v2) {
      Ya[i * ldya + c2] = sa2;
      if constexpr (HB) Yb[i * ldyb + c2] = sb2;
    }
  }
}

// Eight lanes per matrix row and eight rows per wave (32 per workgroup): a
// lane holds columns 2 (l + 8 u), u < 6, of each 96-column pass as 16-byte
// pairs, so every lane is busy at 96 columns, a wave keeps eight rows' index
// and value loads and their X rows in flight at once (one wave per row left
// the dependent loads of a row exposed), and the products are written with
// streaming stores, which leave the L2 to the X rows that neighbouring rows
// share.  Each entry sums the row's nonzeros in order, as spmm_real_kernel does.  On
// the 64^3 7-point stencil in the dissection order, a contiguous 96-column
// block: B X 158 -> 86 us, A X and B X 241 -> 138 us (a 96-column slice of a
// wider basis gains less: 161 -> 133 us).  Needs p and the leading dimensions
// even and the blocks 16-byte aligned.
constexpr int kR8Lanes = 8, kR8Rows = 256 / kR8Lanes, kR8Pairs = 6;
inline unsigned r8_grid(int64_t rows) { return (unsigned)((((rows + kR8Rows - 1) / kR8Rows) + 7) & ~int64_t(7)); }

template <bool HB>
__global__ __launch_bounds__(256) void spmm_real_r8_kernel(int64_t n, const int64_t* __restrict__ rp,
                                                           const int32_t* __restrict__ ci, const double* __restrict__ a,
                                                           const double* __restrict__ b, const double* __restrict__ X,
                                                           int64_t ldx, int p, double* __restrict__ Ya, int64_t ldya,
                                                           double* __restrict__ Yb, int64_t ldyb) {
  const int64_t i = xcd_block(blockIdx.x, gridDim.x) * kR8Rows + (threadIdx.x / kR8Lanes);
  if (i >= n) return;
  const int l = threadIdx.x % kR8Lanes;
  const int64_t e0 = rp[i], e1 = rp[i + 1];
  for (int c0 = 0; c0 < p; c0 += 2 * kR8Lanes * kR8Pairs) {
    double2 sa[kR8Pairs], sb[kR8Pairs];
    int cc[kR8Pairs];
#pragma unroll
    for (int u = 0; u < kR8Pairs; ++u) {
      const int c = c0 + 2 * (l + kR8Lanes * u);
      cc[u] = c < p ? c : p - 2;  // loads stay in the row; columns past p are not stored
      sa[u] = double2{0.0, 0.0};
      sb[u] = double2{0.0, 0.0};
    }
    for (int64_t q = e0; q < e1; ++q) {
      const double* xr = X + (int64_t)ci[q] * ldx;
      const double av = a[q];
      const double bv = HB ? b[q] : 0.0;
#pragma unroll
      for (int u = 0; u < kR8Pairs; ++u) {
        const double2 x = *reinterpret_cast<const double2*>(xr + cc[u]);
        sa[u].x = fma(av, x.x, sa[u].x);
        sa[u].y = fma(av, x.y, sa[u].y);
        if constexpr (HB) {
          sb[u].x = fma(bv, x.x, sb[u].x);
          sb[u].y = fma(bv, x.y, sb[u].y);
        }
      }
    }
#pragma unroll
    for (int u = 0; u < kR8Pairs; ++u) {
      const int c = c0 + 2 * (l + kR8Lanes * u);
      if (c < p) {
        store_stream(Ya + i * ldya + c, sa[u]);
        if constexpr (HB) store_stream(Yb + i * ldyb + c, sb[u]);
      }
    }
  }
}

// complex Hermitian pencils: complex values, complex blocks
template <bool HB>
__global__ __launch_bounds__(256) void spmm_cplx_kernel(int64_t n, const int64_t* __restrict__ rp,
                                                        const int32_t* __restrict__ ci, const zd* __restrict__ a,
                                                        const zd* __restrict__ b, const zd* __restrict__ X, int64_t ldx,
                                                        int p, zd* __restrict__ Ya, int64_t ldya, zd* __restrict__ Yb,
                                                        int64_t ldyb) {
  const int64_t i = spmm_row();
  if (i >= n) return;
  const int lane = threadIdx.x & 63;
  const int64_t e0 = rp[i], e1 = rp[i + 1];
  const zd z0{0.0, 0.0};
  for (int c0 = 0; c0 < p; c0 += 128) {
    const int c1 = c0 + lane, c2 = c1 + 64;
    const bool v1 = c1 < p, v2 = c2 < p;
    const int l1 = v1 ? c1 : p - 1, l2 = v2 ? c2 : p - 1;  // loads stay in the row; unused lanes are not stored
    zd sa1 = z0, sa2 = z0, sb1 = z0, sb2 = z0;
#pragma unroll 4
    for (int64_t q = e0; q < e1; ++q) {
      const zd* xr = X + (int64_t)ci[q] * ldx;
      const zd x1 = xr[l1], x2 = xr[l2];
      const zd av = a[q];
      sa1 = fma_(sa1, av, x1);
      sa2 = fma_(sa2, av, x2);
      if constexpr (HB) {
        const zd bv = b[q];
        sb1 = fma_(sb1, bv, x1);
        sb2 = fma_(sb2, bv, x2);
      }
    }
    if (v1) {
      Ya[i * ldya + c1] = sa1;
      if constexpr (HB) Yb[i * ldyb + c1] = sb1;
    }
    if (v2) {
      Ya[i * ldya + c2] = sa2;
      if constexpr (HB) Yb[i * ldyb + c2] = sb2;
    }
  }
}

// Residual norms of approximate eigenpairs, ||A x_c - lam_c B x_c||^2 and ||x_c||^2,
// fused into one pass over the CSR rows: the rows are in the pencil's ordering,
// the block X in the caller's (X row of pencil row i is perm[i]), so every row of
// the residual is formed from gathered X rows and squared at once; nothing N x p
// is written.  A fixed grid of kResidGroups workgroups: each wave sums a
// contiguous range of rows (ranges of one XCD are contiguous), the four waves of
// a workgroup are added through LDS and the workgroup writes 2 p partial sums.
template <typename T>
__global__ __launch_bounds__(256) void eig_resid_partial_kernel(int64_t n, const int64_t* __restrict__ rp,
                                                                const int32_t* __restrict__ ci,
                                                                const T* __restrict__ a, const T* __restrict__ b,
                                                                const int32_t* __restrict__ perm,
                                                                const T* __restrict__ X, int64_t ldx, int p,
                                                                const double* __restrict__ lam,
                                                                double* __restrict__ partial) {
  __shared__ double red[2][4][kResidMaxCols];
  const int lane = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const int64_t nw = (int64_t)gridDim.x * 4;
  const int64_t w = xcd_block(blockIdx.x, gridDim.x) * 4 + wv;
  const int64_t per = (n + nw - 1) / nw;
  const int64_t i0 = w * per < n ? w * per : n;
  const int64_t i1 = i0 + per < n ? i0 + per : n;
  const int nch = (p + 63) >> 6;
  double rr[kResidMaxCols / 64], xx[kResidMaxCols / 64], lm[kResidMaxCols / 64];
#pragma unroll
  for (int h = 0; h < kResidMaxCols / 64; ++h) {
    rr[h] = 0.0;
    xx[h] = 0.0;
    const int c = h * 64 + lane;
    lm[h] = c < p ? lam[c] : 0.0;
  }
  for (int64_t i = i0; i < i1; ++i) {
    const int64_t e0 = rp[i], e1 = rp[i + 1];
    const T* xo = X + (int64_t)perm[i] * ldx;
#pragma unroll
    for (int h = 0; h < kResidMaxCols / 64; ++h) {
      if (h >= nch) break;
      const int c = h * 64 + lane;
      const int lc = c < p ? c : p - 1;  // loads stay in the row; the sums of unused lanes are never read
      T sa = ST<T>::zero(), sb = ST<T>::zero();
      for (int64_t q = e0; q < e1; ++q) {
        const T xv = X[(int64_t)perm[ci[q]] * ldx + lc];
        sa = fma_(sa, a[q], xv);
        sb = fma_(sb, b[q], xv);
      }
      rr[h] += abs2(sub(sa, scl(sb, lm[h])));
      xx[h] += abs2(xo[lc]);
    }
  }
#pragma unroll
  for (int h = 0; h < kResidMaxCols / 64; ++h) {
    if (h >= nch) break;
    red[0][wv][h * 64 + lane] = rr[h];
    red[1][wv][h * 64 + lane] = xx[h];
  }
  __syncthreads();
  for (int c = threadIdx.x; c < p; c += blockDim.x) {
    double* o = partial + (int64_t)blockIdx.x * 2 * p;
    o[c] = ((red[0][0][c] + red[0][1][c]) + red[0][2][c]) + red[0][3][c];
    o[p + c] = ((red[1][0][c] + red[1][1][c]) + red[1][2][c]) + red[1][3][c];
  }
}

// out[c] = sqrt(sum |r|^2) / ((normA + |lam_c| normB) sqrt(sum |x|^2)), partial
// sums added in workgroup order (the result does not depend on timing)
__global__ void eig_resid_final_kernel(const double* __restrict__ partial, int groups, int p,
                                       const double* __restrict__ lam, double normA, double normB,
                                       double* __restrict__ out) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= p) return;
  double sr = 0.0, sx = 0.0;
  for (int g = 0; g < groups; ++g) {
    sr += partial[(int64_t)g * 2 * p + c];
    sx += partial[(int64_t)g * 2 * p + p + c];
  }
  const double den = (normA + fabs(lam[c]) * normB) * sqrt(sx);
  out[c] = den > 0.0 ? sqrt(sr) / den : (sr == 0.0 ? 0.0 : INFINITY);
}

// R = T - (A - sigma B) X  (X complex, ld p; T real, ld ldt; R complex, ld p)
__global__ __launch_bounds__(256) void spmm_shift_resid_kernel(int64_t n, const int64_t* __restrict__ rp,
                                                               const int32_t* __restrict__ ci,
                                                               const double* __restrict__ a,
                                                               const double* __restrict__ b, double sr, double si,
                                                               const zd* __restrict__ X, const double* __restrict__ T,
                                                               int64_t ldt, int p, zd* __restrict__ R) {
  const int64_t i = spmm_row();
  if (i >= n) return;
  const int lane = threadIdx.x & 63;
  const int64_t e0 = rp[i], e1 = rp[i + 1];
  for (int c0 = 0; c0 < p; c0 += 128) {
    const int c1 = c0 + lane, c2 = c1 + 64;
    const bool v1 = c1 < p, v2 = c2 < p;
    const int l1 = v1 ? c1 : p - 1, l2 = v2 ? c2 : p - 1;  // loads stay in the row; unused lanes are not stored
    double r1 = 0.0, i1 = 0.0, r2 = 0.0, i2 = 0.0;
#pragma unroll 4
    for (int64_t q = e0; q < e1; ++q) {
      const zd* xr = X + (int64_t)ci[q] * p;
      const zd x1 = xr[l1], x2 = xr[l2];
      const double kr = a[q] - sr * b[q], ki = -si * b[q];  // (A - sigma B)_iq
      r1 = fma(kr, x1.re, fma(-ki, x1.im, r1));
      i1 = fma(kr, x1.im, fma(ki, x1.re, i1));
      r2 = fma(kr, x2.re, fma(-ki, x2.im, r2));
      i2 = fma(kr, x2.im, fma(ki, x2.re, i2));
    }
    if (v1) R[i * p + c1] = zd{T[i * ldt + c1] - r1, -i1};
    if (v2) R[i * p + c2] = zd{T[i * ldt + c2] - r2, -i2};
  }
}

// complex Hermitian pencils: R = T - (A - sigma B) X  (X, T, R complex; A, B complex values)
__global__ __launch_bounds__(256) void spmm_shift_resid_cplx_kernel(int64_t n, const int64_t* __restrict__ rp,
                                                                    const int32_t* __restrict__ ci,
                                                                    const zd* __restrict__ a,
                                                                    const zd* __restrict__ b, double sr, double si,
                                                                    const zd* __restrict__ X, const zd* __restrict__ T,
                                                                    int64_t ldt, int p, zd* __restrict__ R) {
  const int64_t i = spmm_row();
  if (i >= n) return;
  const int lane = threadIdx.x & 63;
  const int64_t e0 = rp[i], e1 = rp[i + 1];
  for (int c0 = 0; c0 < p; c0 += 128) {
    const int c1 = c0 + lane, c2 = c1 + 64;
    const bool v1 = c1 < p, v2 = c2 < p;
    const int l1 = v1 ? c1 : p - 1, l2 = v2 ? c2 : p - 1;  // loads stay in the row; unused lanes are not stored
    zd s1{0.0, 0.0}, s2{0.0, 0.0};
#pragma unroll 4
    for (int64_t q = e0; q < e1; ++q) {
      const zd* xr = X + (int64_t)ci[q] * p;
      const zd x1 = xr[l1], x2 = xr[l2];
      const zd av = a[q], bv = b[q];
      const zd kv{av.re - (sr * bv.re - si * bv.im), av.im - (sr * bv.im + si * bv.re)};  // (A - sigma B)_iq
      s1 = fma_(s1, kv, x1);
      s2 = fma_(s2, kv, x2);
    }
    if (v1) R[i * p + c1] = sub(T[i * ldt + c1], s1);
    if (v2) R[i * p + c2] = sub(T[i * ldt + c2], s2);
  }
}

// Y = s1 Y + s0 V (N x p blocks, real or complex, real scalars)
template <typename T>
__global__ void axpby_rows_kernel(T* __restrict__ Y, int64_t ldy, const T* __restrict__ V, int64_t ldv, double s0,
                                  double s1, int64_t n, int p) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n * p) return;
  const int64_t i = e / p;
  const int c = (int)(e % p);
  Y[i * ldy + c] = add(scl(Y[i * ldy + c], s1), scl(V[i * ldv + c], s0));
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

__global__ void g_combine_real_kernel(double* __restrict__ W, int64_t ldw, const double* __restrict__ V, int64_t ldv,
                                      double alpha, const zd* __restrict__ X, int64_t xstride, GCombineCoef w, int r,
                                      int64_t n, int p) {
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n * p) return;
  int64_t i = e / p;
  int c = (int)(e % p);
  double acc = alpha * V[i * ldv + c];
  for (int j = 0; j < r; ++j) {
    const zd x = X[(int64_t)j * xstride + e];
    acc += 2.0 * (w.wr[j] * x.re - w.wi[j] * x.im);
  }
  W[i * ldw + c] = acc;
}

__global__ void set_lowp_kernel(zd* __restrict__ X, const zf* __restrict__ D, int64_t n) {
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  const zf d = D[e];
  X[e] = zd{(double)d.re, (double)d.im};
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

constexpr int CN_ROWS = 256;  // rows per partial sum (one workgroup)

template <bool CPLX>
__device__ __forceinline__ double cn_sq(const double* __restrict__ X, int64_t row, int64_t ldx, int c) {
  if (CPLX) {
    const double re = X[2 * (row * ldx + c)], im = X[2 * (row * ldx + c) + 1];
    return fma(re, re, im * im);
  }
  const double v = X[row * ldx + c];
  return v * v;
}

// partial[b][c] = sum over the rows of chunk b of |x_ic|^2.  The four waves of
// the workgroup take every fourth row of the chunk; lane l holds columns
// c0 + l and c0 + 64 + l (so each row is read as one contiguous run across the
// wave), with eight rows in flight per column; the waves' sums meet in LDS.
template <bool CPLX>
__global__ __launch_bounds__(256) void colnorm_partial_kernel(const double* __restrict__ X, int64_t ldx, int64_t n,
                                                              int p, double* __restrict__ partial) {
  __shared__ double red[4][128];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int64_t r0 = (int64_t)blockIdx.x * CN_ROWS;
  const int64_t r1 = (r0 + CN_ROWS < n) ? r0 + CN_ROWS : n;
  for (int c0 = 0; c0 < p; c0 += 128) {
    const int ca = c0 + lane, cb = c0 + 64 + lane;
    const bool va = ca < p, vb = cb < p;
    double sa[8] = {}, sb[8] = {};
    int64_t i = r0 + w;
    for (; i + 28 < r1; i += 32) {
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        if (va) sa[u] += cn_sq<CPLX>(X, i + 4 * u, ldx, ca);
        if (vb) sb[u] += cn_sq<CPLX>(X, i + 4 * u, ldx, cb);
      }
    }
    for (; i < r1; i += 4) {
      if (va) sa[0] += cn_sq<CPLX>(X, i, ldx, ca);
      if (vb) sb[0] += cn_sq<CPLX>(X, i, ldx, cb);
    }
    red[w][lane] = ((sa[0] + sa[1]) + (sa[2] + sa[3])) + ((sa[4] + sa[5]) + (sa[6] + sa[7]));
    red[w][64 + lane] = ((sb[0] + sb[1]) + (sb[2] + sb[3])) + ((sb[4] + sb[5]) + (sb[6] + sb[7]));
    __syncthreads();
    if (tid < 128 && c0 + tid < p)
      partial[(int64_t)blockIdx.x * p + c0 + tid] = (red[0][tid] + red[1][tid]) + (red[2][tid] + red[3][tid]);
    __syncthreads();
  }
}

// out[c] = sum over b of partial[b][c]: one workgroup per column, a fixed
// summation order (strided partial sums, then a tree in LDS)
__global__ __launch_bounds__(256) void colnorm_final_kernel(const double* __restrict__ partial, int nb, int p,
                                                            double* __restrict__ out) {
  __shared__ double red[256];
  const int c = blockIdx.x, tid = threadIdx.x;
  double s = 0.0;
  for (int b = tid; b < nb; b += 256) s += partial[(int64_t)b * p + c];
  red[tid] = s;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (tid < h) red[tid] += red[tid + h];
    __syncthreads();
  }
  if (tid == 0) out[c] = red[0];
}

inline unsigned nblk(int64_t tot) { return (unsigned)((tot + 255) / 256); }

// Seeded Gaussian block: splitmix64 (a Weyl sequence x0 + k gamma through the
// splitmix finalizer, so draw k is a function of k alone) and the Box-Muller
// transform, one thread per pair of values (draws 2j+1 and 2j+2 of the
// sequence give out[2j] = r cos(2 pi u2), out[2j+1] = r sin(2 pi u2)).
__device__ inline uint64_t splitmix(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}
__global__ void gaussian_fill_kernel(uint64_t x0, int64_t n, double* __restrict__ out) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (2 * j >= n) return;
  constexpr uint64_t kGamma = 0x9E3779B97F4A7C15ULL;
  const double u1 = ((splitmix(x0 + (uint64_t)(2 * j + 1) * kGamma) >> 11) + 0.5) * (1.0 / 9007199254740992.0);
  const double u2 = ((splitmix(x0 + (uint64_t)(2 * j + 2) * kGamma) >> 11) + 0.5) * (1.0 / 9007199254740992.0);
  const double r = sqrt(-2.0 * log(u1));
  const double t = 6.283185307179586 * u2;
  out[2 * j] = r * cos(t);
  if (2 * j + 1 < n) out[2 * j + 1] = r * sin(t);
}

}  // namespace

template <typename T>
void conj_copy(T* dst, const T* src, int64_t n, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(conj_copy_kernel<T>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, dst, src, n);
}
template void conj_copy<zd>(zd*, const zd*, int64_t, hipStream_t);
template void conj_copy<zf>(zf*, const zf*, int64_t, hipStream_t);
template void conj_copy<double>(double*, const double*, int64_t, hipStream_t);

void spmm_cplx(int64_t n, const int64_t* rowptr, const int32_t* colind, const zd* a, const zd* b, const zd* X,
               int64_t ldx, int p, zd* Ya, int64_t ldya, zd* Yb, int64_t ldyb, hipStream_t s) {
  if (n * p == 0) return;
  if (Yb)
    hipLaunchKernelGGL(spmm_cplx_kernel<true>, dim3(xcd_grid(n)), dim3(256), 0, s, n, rowptr, colind, a, b, X, ldx, p,
                       Ya, ldya, Yb, ldyb);
  else
    hipLaunchKernelGGL(spmm_cplx_kernel<false>, dim3(xcd_grid(n)), dim3(256), 0, s, n, rowptr, colind, a, b, X, ldx,
                       p, Ya, ldya, Yb, ldyb);
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
  auto al16 = [](const void* q) { return ((uintptr_t)q & 15) == 0; };
  if (p % 2 == 0 && ldx % 2 == 0 && ldya % 2 == 0 && al16(X) && al16(Ya) && (!Yb || (ldyb % 2 == 0 && al16(Yb)))) {
    if (Yb)
      hipLaunchKernelGGL(spmm_real_r8_kernel<true>, dim3(r8_grid(n)), dim3(256), 0, s, n, rp, ci, a, b, X, ldx, p, Ya,
                         ldya, Yb, ldyb);
    else
      hipLaunchKernelGGL(spmm_real_r8_kernel<false>, dim3(r8_grid(n)), dim3(256), 0, s, n, rp, ci, a, b, X, ldx, p, Ya,
                         ldya, Yb, ldyb);
    return;
  }
  if (Yb)
    hipLaunchKernelGGL(spmm_real_kernel<true>, dim3(xcd_grid(n)), dim3(256), 0, s, n, rp, ci, a, b, X, ldx, p, Ya,
                       ldya, Yb, ldyb);
  else
    hipLaunchKernelGGL(spmm_real_kernel<false>, dim3(xcd_grid(n)), dim3(256), 0, s, n, rp, ci, a, b, X, ldx, p, Ya,
                       ldya, Yb, ldyb);
}

void spmm_shift_resid(int64_t n, const int64_t* rp, const int32_t* ci, const double* a, const double* b, double sr,
                      double si, const zd* X, const double* T, int64_t ldt, int p, zd* R, hipStream_t s) {
  if (n * p == 0) return;
  hipLaunchKernelGGL(spmm_shift_resid_kernel, dim3(xcd_grid(n)), dim3(256), 0, s, n, rp, ci, a, b, sr, si, X, T, ldt, p,
                     R);
}

void spmm_shift_resid(int64_t n, const int64_t* rp, const int32_t* ci, const zd* a, const zd* b, double sr,
                      double si, const zd* X, const zd* T, int64_t ldt, int p, zd* R, hipStream_t s) {
  if (n * p == 0) return;
  hipLaunchKernelGGL(spmm_shift_resid_cplx_kernel, dim3(xcd_grid(n)), dim3(256), 0, s, n, rp, ci, a, b, sr, si, X, T,
                     ldt, p, R);
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
void g_combine_real(double* W, int64_t ldw, const double* V, int64_t ldv, double alpha, const zd* X, int64_t xstride,
                    const GCombineCoef& w, int r, int64_t n, int p, hipStream_t s) {
  if (n * p == 0) return;
  hipLaunchKernelGGL(g_combine_real_kernel, dim3(nblk(n * p)), dim3(256), 0, s, W, ldw, V, ldv, alpha, X, xstride, w,
                     r, n, p);
}
void set_lowp(zd* X, const zf* D, int64_t n, hipStream_t s) {
  if (n == 0) return;
  hipLaunchKernelGGL(set_lowp_kernel, dim3(nblk(n)), dim3(256), 0, s, X, D, n);
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
  if (nb == 0 || p <= 0) return;
  hipLaunchKernelGGL(colnorm_partial_kernel<false>, dim3(nb), dim3(256), 0, s, X, ldx, n, p, partial);
  hipLaunchKernelGGL(colnorm_final_kernel, dim3(p), dim3(256), 0, s, partial, nb, p, out);
}
void colnorm2_cplx(const zd* X, int64_t n, int p, double* partial, double* out, hipStream_t s) {
  int nb = colnorm_partials(n);
  if (nb == 0 || p <= 0) return;
  hipLaunchKernelGGL(colnorm_partial_kernel<true>, dim3(nb), dim3(256), 0, s, (const double*)X, (int64_t)p, n, p,
                     partial);
  hipLaunchKernelGGL(colnorm_final_kernel, dim3(p), dim3(256), 0, s, partial, nb, p, out);
}

template <typename T>
void eig_resid_norms(int64_t n, const int64_t* rp, const int32_t* ci, const T* a, const T* b, const int32_t* perm,
                     const T* X, int64_t ldx, int p, const double* lam, double normA, double normB, double* partial,
                     double* out, hipStream_t s) {
  if (p <= 0) return;
  hipLaunchKernelGGL(eig_resid_partial_kernel<T>, dim3(kResidGroups), dim3(256), 0, s, n, rp, ci, a, b, perm, X, ldx, p,
                     lam, partial);
  hipLaunchKernelGGL(eig_resid_final_kernel, dim3((p + 127) / 128), dim3(128), 0, s, partial, kResidGroups, p, lam,
                     normA, normB, out);
}
template void eig_resid_norms<double>(int64_t, const int64_t*, const int32_t*, const double*, const double*,
                                      const int32_t*, const double*, int64_t, int, const double*, double, double,
                                      double*, double*, hipStream_t);
template void eig_resid_norms<zd>(int64_t, const int64_t*, const int32_t*, const zd*, const zd*, const int32_t*,
                                  const zd*, int64_t, int, const double*, double, double, double*, double*,
                                  hipStream_t);

void gaussian_fill(uint64_t seed, int64_t n, double* out, hipStream_t s) {
  if (n <= 0) return;
  const uint64_t x0 = seed * 0x9E3779B97F4A7C15ULL + 0x1234567ULL;
  hipLaunchKernelGGL(gaussian_fill_kernel, dim3(nblk((n + 1) / 2)), dim3(256), 0, s, x0, n, out);
}

template <typename T>
void axpby_rows(T* Y, int64_t ldy, const T* V, int64_t ldv, double s0, double s1, int64_t n, int p, hipStream_t s) {
  if (n * p == 0) return;
  hipLaunchKernelGGL(axpby_rows_kernel<T>, dim3(nblk(n * p)), dim3(256), 0, s, Y, ldy, V, ldv, s0, s1, n, p);
}
template void axpby_rows<double>(double*, int64_t, const double*, int64_t, double, double, int64_t, int, hipStream_t);
template void axpby_rows<zd>(zd*, int64_t, const zd*, int64_t, double, double, int64_t, int, hipStream_t);

void fill_zero_bytes(void* p, size_t bytes, hipStream_t s) {
  if (bytes) (void)hipMemsetAsync(p, 0, bytes, s);
}

}  // namespace zolo
