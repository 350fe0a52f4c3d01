// Multifrontal LDL^T kernels (numeric factorization and solve helpers) for
// the r1 shifted matrices K_j = A - sigma_hat_j B of Algorithm 2, lines 5-6.
// Real pencils give complex-symmetric K_j, factored without pivoting in the
// nested-dissection order (A - sigma B with Im sigma != 0 has a definite
// skew-Hermitian part, so every leading principal block is nonsingular).
#include "front.h"

namespace zolo {
namespace {

template <typename T>
__global__ void assemble_kernel(T* __restrict__ panel, const int64_t* __restrict__ dst, const int64_t* __restrict__ src,
                                int64_t n, const double* __restrict__ a, const double* __restrict__ b, double sr,
                                double si) {
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  int64_t s = src[e];
  double av = a[s], bv = b[s];
  zd v{av - sr * bv, -si * bv};
  panel[dst[e]] = cvt<T, zd>(v);
}

// complex Hermitian pencils: a, b interleaved complex values
template <typename T>
__global__ void assemble_cplx_kernel(T* __restrict__ panel, const int64_t* __restrict__ dst,
                                     const int64_t* __restrict__ src, int64_t n, const zd* __restrict__ a,
                                     const zd* __restrict__ b, double sr, double si) {
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  int64_t s = src[e];
  zd av = a[s], bv = b[s];
  zd v{av.re - (sr * bv.re - si * bv.im), av.im - (sr * bv.im + si * bv.re)};
  panel[dst[e]] = cvt<T, zd>(v);
}

// LU fronts: the child's update block is full; entry (i, j) goes to the
// parent's L panel (lower part of the front, diagonal included), its U panel
// (upper part, stored transposed so that it is laid out like L), or its
// update block.
template <typename T>
__global__ void extend_add_lu_kernel(T* __restrict__ panel, T* __restrict__ upanel, T* __restrict__ upd,
                                     const int32_t* __restrict__ pmap, const ExtDesc* __restrict__ descs) {
  const ExtDesc d = descs[blockIdx.y];
  const int64_t nb = d.nb_c;
  const int64_t j = blockIdx.x;
  if (j >= nb) return;
  const int32_t* pm = pmap + d.pmap;
  const T* cu = upd + d.child_upd;
  const int pj = pm[j];
  const int64_t nbp = (int64_t)d.k_p - d.ns_p;
  for (int64_t i = threadIdx.x; i < nb; i += blockDim.x) {
    T v = cu[i + j * nb];
    const int pi = pm[i];
    T* dst;
    if (pj < d.ns_p && pi >= pj)
      dst = panel + d.par_panel + pi + (int64_t)pj * d.k_p;
    else if (pi < d.ns_p)
      dst = upanel + d.par_panel + pj + (int64_t)pi * d.k_p;
    else
      dst = upd + d.par_upd + (pi - d.ns_p) + (int64_t)(pj - d.ns_p) * nbp;
    *dst = add(*dst, v);
  }
}

template <typename T>
__global__ void extend_add_kernel(T* __restrict__ panel, T* __restrict__ upd, const int32_t* __restrict__ pmap,
                                  const ExtDesc* __restrict__ descs) {
  const ExtDesc d = descs[blockIdx.y];
  const int64_t nb = d.nb_c;
  // column j of the child block handled by blockIdx.x, rows by threads
  const int64_t j = blockIdx.x;
  if (j >= nb) return;
  const int32_t* pm = pmap + d.pmap;
  const T* cu = upd + d.child_upd;
  const int pj = pm[j];
  for (int64_t i = j + threadIdx.x; i < nb; i += blockDim.x) {
    T v = cu[i + j * nb];
    int pi = pm[i];
    if (pj < d.ns_p) {
      T* dst = panel + d.par_panel + pi + (int64_t)pj * d.k_p;
      *dst = add(*dst, v);
    } else {
      int64_t nbp = (int64_t)d.k_p - d.ns_p;
      T* dst = upd + d.par_upd + (pi - d.ns_p) + (int64_t)(pj - d.ns_p) * nbp;
      *dst = add(*dst, v);
    }
  }
}

// One workgroup per front: LDL^T of the jb x jb diagonal block in LDS, then the
// inverse of its unit lower factor.
// Inverse of the unit lower triangle stored in Ab (jb x jb) into Xb, by
// 16 x 16 sub-blocks:
//  (1) X_II = L_II^-1 for every diagonal sub-block (in parallel);
//  (2) for block rows I = 1, 2, ...: X_IJ = -X_II sum_{J <= K < I} L_IK X_KJ.
template <typename T>
__device__ void unit_lower_inverse(T (*Ab)[FB + 1], T (*Xb)[FB + 1], T (*Tm)[FB], int jb) {
  const int tid = threadIdx.x;
  constexpr int SB = 16;
  const int nsb = (jb + SB - 1) / SB;
  for (int e = tid; e < jb * jb; e += blockDim.x) {
    int r = e % jb, c = e / jb;
    Xb[r][c] = (r == c) ? ST<T>::one() : ST<T>::zero();
  }
  __syncthreads();
  if (tid < nsb * SB) {
    const int b = tid / SB, c = b * SB + tid % SB;
    const int rend = min(jb, (b + 1) * SB);
    if (c < jb)
      for (int r = c + 1; r < rend; ++r) {
        T s = ST<T>::zero();
        for (int t = c; t < r; ++t) s = fma_(s, Ab[r][t], Xb[t][c]);
        Xb[r][c] = neg(s);
      }
  }
  __syncthreads();
  for (int I = 1; I < nsb; ++I) {
    const int r0 = I * SB, rn = min(SB, jb - r0), cols = r0;
    for (int e = tid; e < rn * cols; e += blockDim.x) {
      int r = e % rn, c = e / rn;
      T s = ST<T>::zero();
      for (int t = (c / SB) * SB; t < r0; ++t) s = fma_(s, Ab[r0 + r][t], Xb[t][c]);
      Tm[r][c] = s;
    }
    __syncthreads();
    for (int e = tid; e < rn * cols; e += blockDim.x) {
      int r = e % rn, c = e / rn;
      T s = ST<T>::zero();
      for (int t = 0; t <= r; ++t) s = fma_(s, Xb[r0 + r][r0 + t], Tm[t][c]);
      Xb[r0 + r][c] = neg(s);
    }
    __syncthreads();
  }
}

// LU of the jb x jb diagonal block of a front without pivoting (complex
// Hermitian pencils): L (unit lower) into the L panel, U^T (unit lower) into
// the U panel, D into dvec, and the inverses of both unit lower blocks.
template <typename T>
__global__ __launch_bounds__(256) void diag_block_lu_kernel(T* __restrict__ panel, T* __restrict__ upanel,
                                                            T* __restrict__ inv, T* __restrict__ uinv,
                                                            T* __restrict__ dvec, const DiagDesc* __restrict__ descs,
                                                            int J, int* breakdown) {
  const DiagDesc d = descs[blockIdx.x];
  if (J >= d.ns) return;
  const int jb = (d.ns - J) < FB ? (d.ns - J) : FB;
  __shared__ T Ab[FB][FB + 1];
  __shared__ T Xb[FB][FB + 1];
  __shared__ T Tm[16][FB];
  const int tid = threadIdx.x;
  T* P = panel + d.panel;
  T* U = upanel + d.panel;
  const int64_t k = d.k, ns = d.ns;
  for (int e = tid; e < jb * jb; e += blockDim.x) {
    int r = e % jb, c = e / jb;
    Ab[r][c] = (r >= c) ? P[(J + r) + (int64_t)(J + c) * k] : U[(J + c) + (int64_t)(J + r) * k];
  }
  __syncthreads();
  for (int c = 0; c < jb; ++c) {
    T dc = Ab[c][c];
    if (abs2(dc) == 0.0) {
      if (tid == 0) atomicExch(breakdown, 1);
      dc = ST<T>::one();
    }
    const T dinv = inv_(dc);
    __syncthreads();
    for (int r = c + 1 + tid; r < jb; r += blockDim.x) {
      Ab[r][c] = mul(Ab[r][c], dinv);  // L(r, c)
      Ab[c][r] = mul(Ab[c][r], dinv);  // U(c, r)
    }
    __syncthreads();
    // trailing update: A(r, q) -= L(r, c) d U(c, q) for r, q in (c, jb)
    const int m = jb - c - 1;
    for (int e = tid; e < m * m; e += blockDim.x) {
      int r = c + 1 + e % m, q = c + 1 + e / m;
      Ab[r][q] = sub(Ab[r][q], mul(mul(Ab[r][c], dc), Ab[c][q]));
    }
    __syncthreads();
  }
  for (int e = tid; e < jb * jb; e += blockDim.x) {
    int r = e % jb, c = e / jb;
    if (r >= c) {
      P[(J + r) + (int64_t)(J + c) * k] = Ab[r][c];
      U[(J + r) + (int64_t)(J + c) * k] = (r == c) ? Ab[r][c] : Ab[c][r];
    }
  }
  for (int c = tid; c < jb; c += blockDim.x) dvec[d.first + J + c] = Ab[c][c];
  __syncthreads();
  unit_lower_inverse<T>(Ab, Xb, Tm, jb);
  T* X = inv + d.inv;
  for (int e = tid; e < jb * jb; e += blockDim.x) {
    int r = e % jb, c = e / jb;
    X[(J + r) + (int64_t)(J + c) * ns] = (r >= c) ? Xb[r][c] : ST<T>::zero();
  }
  __syncthreads();
  // the same for U^T: move its strict lower part into Ab's lower triangle
  for (int e = tid; e < jb * jb; e += blockDim.x) {
    int r = e % jb, c = e / jb;
    if (r > c) Xb[r][c] = Ab[c][r];
  }
  __syncthreads();
  for (int e = tid; e < jb * jb; e += blockDim.x) {
    int r = e % jb, c = e / jb;
    if (r > c) Ab[r][c] = Xb[r][c];
  }
  __syncthreads();
  unit_lower_inverse<T>(Ab, Xb, Tm, jb);
  T* XU = uinv + d.inv;
  for (int e = tid; e < jb * jb; e += blockDim.x) {
    int r = e % jb, c = e / jb;
    XU[(J + r) + (int64_t)(J + c) * ns] = (r >= c) ? Xb[r][c] : ST<T>::zero();
  }
}

template <typename T>
__global__ __launch_bounds__(256) void diag_block_kernel(T* __restrict__ panel, T* __restrict__ inv,
                                                         T* __restrict__ dvec, const DiagDesc* __restrict__ descs,
                                                         int J, int* breakdown) {
  const DiagDesc d = descs[blockIdx.x];
  if (J >= d.ns) return;
  const int jb = (d.ns - J) < FB ? (d.ns - J) : FB;
  __shared__ T Ab[FB][FB + 1];  // Ab[r][c]
  __shared__ T Xb[FB][FB + 1];
  __shared__ T Tm[16][FB];
  const int tid = threadIdx.x;
  T* P = panel + d.panel;
  const int64_t k = d.k;
  for (int e = tid; e < jb * jb; e += blockDim.x) {
    int r = e % jb, c = e / jb;
    Ab[r][c] = (r >= c) ? P[(J + r) + (int64_t)(J + c) * k] : ST<T>::zero();
  }
  __syncthreads();
  // right-looking unblocked LDL^T
  for (int c = 0; c < jb; ++c) {
    T dc = Ab[c][c];
    if (abs2(dc) == 0.0) {
      if (tid == 0) atomicExch(breakdown, 1);
      dc = ST<T>::one();
    }
    T dinv = inv_(dc);
    __syncthreads();
    for (int r = c + 1 + tid; r < jb; r += blockDim.x) Ab[r][c] = mul(Ab[r][c], dinv);
    __syncthreads();
    // trailing lower update: A(r, q) -= L(r,c) d L(q,c), q in (c, jb), r >= q
    const int m = jb - c - 1;
    for (int e = tid; e < m * m; e += blockDim.x) {
      int r = c + 1 + e % m, q = c + 1 + e / m;
      if (r >= q) Ab[r][q] = sub(Ab[r][q], mul(mul(Ab[r][c], dc), Ab[q][c]));
    }
    __syncthreads();
  }
  // write back L (strict lower) and D
  for (int e = tid; e < jb * jb; e += blockDim.x) {
    int r = e % jb, c = e / jb;
    if (r >= c) P[(J + r) + (int64_t)(J + c) * k] = Ab[r][c];
  }
  for (int c = tid; c < jb; c += blockDim.x) dvec[d.first + J + c] = Ab[c][c];
  // inverse of the unit lower block, by 16 x 16 sub-blocks:
  //  (1) X_II = L_II^-1 for every diagonal sub-block (in parallel);
  //  (2) for block rows I = 1, 2, ...: X_IJ = -X_II sum_{J <= K < I} L_IK X_KJ.
  constexpr int SB = 16;
  const int nsb = (jb + SB - 1) / SB;
  for (int e = tid; e < jb * jb; e += blockDim.x) {
    int r = e % jb, c = e / jb;
    Xb[r][c] = (r == c) ? ST<T>::one() : ST<T>::zero();
  }
  __syncthreads();
  if (tid < nsb * SB) {
    const int b = tid / SB, c = b * SB + tid % SB;
    const int rend = min(jb, (b + 1) * SB);
    if (c < jb)
      for (int r = c + 1; r < rend; ++r) {
        T s = ST<T>::zero();
        for (int t = c; t < r; ++t) s = fma_(s, Ab[r][t], Xb[t][c]);
        Xb[r][c] = neg(s);
      }
  }
  __syncthreads();
  for (int I = 1; I < nsb; ++I) {
    const int r0 = I * SB, rn = min(SB, jb - r0), cols = r0;
    // Tm(r, c) = sum_{t in [c's block start, r0)} L(r0 + r, t) X(t, c)
    for (int e = tid; e < rn * cols; e += blockDim.x) {
      int r = e % rn, c = e / rn;
      T s = ST<T>::zero();
      for (int t = (c / SB) * SB; t < r0; ++t) s = fma_(s, Ab[r0 + r][t], Xb[t][c]);
      Tm[r][c] = s;
    }
    __syncthreads();
    for (int e = tid; e < rn * cols; e += blockDim.x) {
      int r = e % rn, c = e / rn;
      T s = ST<T>::zero();
      for (int t = 0; t <= r; ++t) s = fma_(s, Xb[r0 + r][r0 + t], Tm[t][c]);
      Xb[r0 + r][c] = neg(s);
    }
    __syncthreads();
  }
  T* X = inv + d.inv;
  const int64_t ns = d.ns;
  for (int e = tid; e < jb * jb; e += blockDim.x) {
    int r = e % jb, c = e / jb;
    X[(J + r) + (int64_t)(J + c) * ns] = (r >= c) ? Xb[r][c] : ST<T>::zero();
  }
}

template <typename Ts, typename T>
__global__ void gather_own_kernel(T* __restrict__ W, const Ts* __restrict__ src, int64_t ldsrc,
                                  const SolveDesc* __restrict__ descs, int p) {
  const SolveDesc d = descs[blockIdx.y];
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t tot = (int64_t)d.k * p;
  if (e >= tot) return;
  int64_t r = e / p, c = e % p;
  T v = ST<T>::zero();
  if (r < d.ns) v = cvt<T, Ts>(src[d.so + (d.first + r) * ldsrc + c]);
  W[d.w + e] = v;
}

template <typename T>
__global__ void solve_ext_kernel(T* __restrict__ W, const T* __restrict__ U, const int32_t* __restrict__ pmap,
                                 const SolveExt* __restrict__ descs, int p) {
  const SolveExt d = descs[blockIdx.y];
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t tot = (int64_t)d.nb_c * p;
  if (e >= tot) return;
  int64_t i = e / p, c = e % p;
  int64_t pr = pmap[d.pmap + i];
  T* dst = W + d.par_w + pr * p + c;
  *dst = add(*dst, U[d.child_u + e]);
}

template <typename T>
__global__ void gather_back_kernel(T* __restrict__ W, const T* __restrict__ Y, const T* __restrict__ X,
                                   const int32_t* __restrict__ srows, const SolveDesc* __restrict__ descs, int p) {
  const SolveDesc d = descs[blockIdx.y];
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t tot = (int64_t)d.k * p;
  if (e >= tot) return;
  int64_t r = e / p, c = e % p;
  T v;
  if (r < d.ns) {
    const T* dv = (const T*)d.dv;
    v = mul(Y[d.xo + (d.first + r) * p + c], inv_(dv[d.first + r]));
  } else {
    v = X[d.xo + (int64_t)srows[d.srow + r - d.ns] * p + c];
  }
  W[d.w + e] = v;
}

template <typename T>
__global__ void stack_kernel(const StackDesc<T>* __restrict__ descs) {
  const StackDesc<T> d = descs[blockIdx.y];
  const int64_t k = (int64_t)d.ns + d.nb;
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= k * d.ns) return;
  const int64_t c = e / k, r = e % k;
  d.dst[e] = r < d.ns ? d.top[r + c * d.ns] : d.bot[(r - d.ns) + c * d.nb];
}

}  // namespace

template <typename T>
void front_assemble(T* panel, const int64_t* dst, const int64_t* src, int64_t n, const double* a, const double* b,
                    double sr, double si, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(assemble_kernel<T>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, panel, dst, src, n, a, b,
                     sr, si);
}

template <typename T>
void front_assemble_cplx(T* panel, const int64_t* dst, const int64_t* src, int64_t n, const zd* a, const zd* b,
                         double sr, double si, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(assemble_cplx_kernel<T>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, panel, dst, src, n,
                     a, b, sr, si);
}

template <typename T>
void front_extend_add_lu(T* panel, T* upanel, T* upd, const int32_t* pmap, const ExtDesc* d, int nd, int max_nb,
                         hipStream_t s) {
  if (nd <= 0 || max_nb <= 0) return;
  hipLaunchKernelGGL(extend_add_lu_kernel<T>, dim3(max_nb, nd), dim3(256), 0, s, panel, upanel, upd, pmap, d);
}

template <typename T>
void front_diag_block_lu(T* panel, T* upanel, T* inv, T* uinv, T* dvec, const DiagDesc* d, int nd, int J,
                         int* breakdown, hipStream_t s) {
  if (nd <= 0) return;
  hipLaunchKernelGGL(diag_block_lu_kernel<T>, dim3(nd), dim3(256), 0, s, panel, upanel, inv, uinv, dvec, d, J,
                     breakdown);
}

template <typename T>
void front_extend_add(T* panel, T* upd, const int32_t* pmap, const ExtDesc* d, int nd, int max_nb, hipStream_t s) {
  if (nd <= 0 || max_nb <= 0) return;
  hipLaunchKernelGGL(extend_add_kernel<T>, dim3(max_nb, nd), dim3(256), 0, s, panel, upd, pmap, d);
}

template <typename T>
void front_diag_block(T* panel, T* inv, T* dvec, const DiagDesc* d, int nd, int J, int* breakdown, hipStream_t s) {
  if (nd <= 0) return;
  hipLaunchKernelGGL(diag_block_kernel<T>, dim3(nd), dim3(256), 0, s, panel, inv, dvec, d, J, breakdown);
}

template <typename Ts, typename T>
void solve_gather_own(T* W, const Ts* src, int64_t ldsrc, const SolveDesc* d, int nd, int p, int max_k,
                      hipStream_t s) {
  if (nd <= 0) return;
  int64_t tot = (int64_t)max_k * p;
  hipLaunchKernelGGL((gather_own_kernel<Ts, T>), dim3((unsigned)((tot + 255) / 256), nd), dim3(256), 0, s, W, src,
                     ldsrc, d, p);
}

template <typename T>
void solve_extend_add(T* W, const T* U, const int32_t* pmap, const SolveExt* d, int nd, int p, int max_nb,
                      hipStream_t s) {
  if (nd <= 0 || max_nb <= 0) return;
  int64_t tot = (int64_t)max_nb * p;
  hipLaunchKernelGGL(solve_ext_kernel<T>, dim3((unsigned)((tot + 255) / 256), nd), dim3(256), 0, s, W, U, pmap, d, p);
}

template <typename T>
void solve_gather_back(T* W, const T* Y, const T* X, const int32_t* srows, const SolveDesc* d, int nd, int p,
                       int max_k, hipStream_t s) {
  if (nd <= 0 || max_k <= 0) return;
  int64_t tot = (int64_t)max_k * p;
  hipLaunchKernelGGL(gather_back_kernel<T>, dim3((unsigned)((tot + 255) / 256), nd), dim3(256), 0, s, W, Y, X, srows,
                     d, p);
}

template <typename T>
void front_stack(const StackDesc<T>* d, int nd, int64_t max_elems, hipStream_t s) {
  if (nd <= 0 || max_elems <= 0) return;
  hipLaunchKernelGGL(stack_kernel<T>, dim3((unsigned)((max_elems + 255) / 256), nd), dim3(256), 0, s, d);
}

#define INST(T)                                                                                                      \
  template void front_assemble<T>(T*, const int64_t*, const int64_t*, int64_t, const double*, const double*, double, \
                                  double, hipStream_t);                                                              \
  template void front_extend_add<T>(T*, T*, const int32_t*, const ExtDesc*, int, int, hipStream_t);                  \
  template void front_assemble_cplx<T>(T*, const int64_t*, const int64_t*, int64_t, const zd*, const zd*, double,    \
                                       double, hipStream_t);                                                         \
  template void front_extend_add_lu<T>(T*, T*, T*, const int32_t*, const ExtDesc*, int, int, hipStream_t);           \
  template void front_diag_block_lu<T>(T*, T*, T*, T*, T*, const DiagDesc*, int, int, int*, hipStream_t);            \
  template void front_diag_block<T>(T*, T*, T*, const DiagDesc*, int, int, int*, hipStream_t);                       \
  template void solve_extend_add<T>(T*, const T*, const int32_t*, const SolveExt*, int, int, int, hipStream_t);      \
  template void solve_gather_back<T>(T*, const T*, const T*, const int32_t*, const SolveDesc*, int, int, int,        \
                                     hipStream_t);                                                                   \
  template void front_stack<T>(const StackDesc<T>*, int, int64_t, hipStream_t);
INST(zd)
INST(zf)
#undef INST
template void solve_gather_own<double, zd>(zd*, const double*, int64_t, const SolveDesc*, int, int, int, hipStream_t);
template void solve_gather_own<zd, zd>(zd*, const zd*, int64_t, const SolveDesc*, int, int, int, hipStream_t);
template void solve_gather_own<double, zf>(zf*, const double*, int64_t, const SolveDesc*, int, int, int, hipStream_t);
template void solve_gather_own<zd, zf>(zf*, const zd*, int64_t, const SolveDesc*, int, int, int, hipStream_t);

}  // namespace zolo
