// Kernels of the multi-shift block GMRES (Algorithm 2, line 8; eq. solve2)
// and of the Rayleigh-Ritz step (Algorithm 1, lines 4-6).
//
// Shifted least squares.  Block Arnoldi gives G V_m = V_{m+1} Hbar_m with a
// real block upper Hessenberg Hbar; by shift invariance
// (G + s I) V_m = V_{m+1} (Hbar_m + s Ibar), so each outer shift s = i sqrt(c_j)
// needs min || E1 R0 - (Hbar + s Ibar) Y ||.  Every shift keeps its own
// incremental QR: each new block column receives the earlier Householder
// reflectors, its 2p x p panel (upper-triangular subdiagonal block) is reduced
// by p new reflectors of length p + 1, and the transformed right-hand side
// gives the residual norm of every column.  Reductions are wave-level
// (64-lane shuffles); one wave owns the rows r with r % 64 == lane, so no
// barrier is needed between reflectors applied to one column.
#include "krylov.h"

namespace zolo {
namespace {

__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// partial q sits at partial + q * step * M N; summed in q order
template <typename T>
__global__ void reduce_partials_kernel(T* __restrict__ out, int64_t ld_out, const T* __restrict__ partial, int S,
                                       int step, int M, int N, int addto) {
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t MN = (int64_t)M * N;
  if (e >= MN) return;
  T s = ST<T>::zero();
  for (int q = 0; q < S; ++q) s = add(s, partial[(int64_t)q * step * MN + e]);
  int64_t i = e % M, j = e / M;
  T* o = out + i + j * ld_out;
  *o = addto ? add(*o, s) : s;
}

// First level of a long reduction: group g of gs consecutive partials is
// summed, in order, into its first partial (grid.y = number of groups).
template <typename T>
__global__ void reduce_groups_kernel(T* __restrict__ partial, int S, int gs, int64_t MN) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= MN) return;
  const int q0 = (int)blockIdx.y * gs, q1 = q0 + gs < S ? q0 + gs : S;
  T s = partial[(int64_t)q0 * MN + e];
  for (int q = q0 + 1; q < q1; ++q) s = add(s, partial[(int64_t)q * MN + e]);
  partial[(int64_t)q0 * MN + e] = s;
}

// single workgroup; G is read, R/Rinv written (all col-major p x p).  With
// USE_LDS the factorization runs in LDS (p <= 128) and only R, R^-1 are
// written to global memory.  Hermitian G = R^H R for complex T.
template <typename T, bool USE_LDS>
__global__ __launch_bounds__(1024) void chol_upper_inv_kernel(const T* __restrict__ G, int p, double rel_shift,
                                                              T* __restrict__ Rg, T* __restrict__ Rinv, int* flag) {
  extern __shared__ __align__(16) char lds_raw[];
  T* lds_R = (T*)lds_raw;
  T* R = USE_LDS ? lds_R : Rg;
  // the inverse also lives in LDS when both fit
  const bool inv_lds = USE_LDS && (int64_t)2 * p * p * sizeof(T) <= 160 * 1024 - 4096;
  T* Ri = inv_lds ? lds_R + p * p : Rinv;
  const int tid = threadIdx.x, nt = blockDim.x;
  __shared__ double trace_s;
  __shared__ int bad_s;
  if (tid == 0) {
    double tr = 0.0;
    for (int i = 0; i < p; ++i) tr += re_(G[i + (int64_t)i * p]);
    trace_s = tr;
    bad_s = 0;
  }
  __syncthreads();
  const double shift = rel_shift * trace_s / (p > 0 ? p : 1);
  for (int e = tid; e < p * p; e += nt) {
    int i = e % p, j = e / p;
    T v = (i <= j) ? G[e] : ST<T>::zero();
    if (i == j) v = cvt<T, double>(re_(v) + shift);
    R[e] = v;
  }
  __syncthreads();
  for (int k = 0; k < p; ++k) {
    double dkk = re_(R[k + (int64_t)k * p]);
    if (!(dkk > 1e-300)) {
      if (tid == 0) bad_s = 1;
      dkk = 1.0;
    }
    double rk = sqrt(dkk);
    __syncthreads();
    for (int j = k + tid; j < p; j += nt) {
      if (j == k)
        R[k + (int64_t)k * p] = cvt<T, double>(rk);
      else
        R[k + (int64_t)j * p] = scl(R[k + (int64_t)j * p], 1.0 / rk);
    }
    __threadfence_block();
    __syncthreads();
    int m = p - k - 1;
    for (int e = tid; e < m * m; e += nt) {
      int i = k + 1 + e % m, j = k + 1 + e / m;
      if (i <= j) R[i + (int64_t)j * p] = sub(R[i + (int64_t)j * p], mul(conj_(R[k + (int64_t)i * p]), R[k + (int64_t)j * p]));
    }
    __threadfence_block();
    __syncthreads();
  }
  if (tid == 0 && bad_s) *flag = 1;
  // R^-1: column j by back substitution, x_i = -(sum_{t=i+1..j} R(i,t) x_t) / R(i,i)
  for (int j = tid; j < p; j += nt) {
    for (int i = j + 1; i < p; ++i) Ri[i + (int64_t)j * p] = ST<T>::zero();
    Ri[j + (int64_t)j * p] = inv_(R[j + (int64_t)j * p]);
    for (int i = j - 1; i >= 0; --i) {
      T acc = ST<T>::zero();
      for (int t = i + 1; t <= j; ++t) acc = fma_(acc, R[i + (int64_t)t * p], Ri[t + (int64_t)j * p]);
      Ri[i + (int64_t)j * p] = neg(mul(acc, inv_(R[i + (int64_t)i * p])));
    }
  }
  if (USE_LDS) {
    __syncthreads();
    for (int e = tid; e < p * p; e += nt) {
      int i = e % p, j = e / p;
      Rg[e] = (i <= j) ? R[e] : ST<T>::zero();
      if (Ri != Rinv) Rinv[e] = Ri[e];
    }
  }
}

// Cholesky G + shift I = R^H R together with R^-1, for p small enough that both
// live in LDS: one workgroup, one barrier per elimination step.  Step k reads the
// (not yet scaled) row k of A and of Z and updates the rows below it:
//   A(i, j) -= conj(A(k, i)) A(k, j) / d_k         (k < i <= j, the trailing upper part)
//   Z(i, c) -= conj(A(k, i)) Z(k, c) / d_k         (i > k, c <= k)
// where Z starts as I and ends, row by row, as R(k, k) Y with Y = R^-H (forward
// substitution on R^H run right-looking); row k of both is scaled by 1 / sqrt(d_k)
// at the next step, when nothing reads it.  R^-1 = Y^H.
template <typename T>
__global__ __launch_bounds__(1024) void chol_inv_lds_kernel(const T* __restrict__ G, int p, double rel_shift,
                                                            T* __restrict__ Rg, T* __restrict__ Rinv, int* flag) {
  extern __shared__ __align__(16) char lds_raw[];
  // LDS leading dimension p + 1: the row of A read across lanes at every step
  // would otherwise sit in one bank (column stride a multiple of the 64 banks)
  const int ld = p + 1;
  T* A = (T*)lds_raw;
  T* Z = A + (int64_t)p * ld;
  const int tid = threadIdx.x, nt = blockDim.x, tx = tid & 31, ty = tid >> 5;
  __shared__ double trace_s;
  __shared__ int bad_s;
  if (tid == 0) {
    double tr = 0.0;
    for (int i = 0; i < p; ++i) tr += re_(G[i + (int64_t)i * p]);
    trace_s = tr;
    bad_s = 0;
  }
  __syncthreads();
  const double shift = rel_shift * trace_s / (p > 0 ? p : 1);
  for (int e = tid; e < p * p; e += nt) {
    const int i = e % p, j = e / p;
    T v = (i <= j) ? G[e] : ST<T>::zero();
    if (i == j) v = cvt<T, double>(re_(v) + shift);
    A[i + (int64_t)j * ld] = v;
    Z[i + (int64_t)j * ld] = i == j ? ST<T>::one() : ST<T>::zero();
  }
  __syncthreads();
  double irk_prev = 1.0;
  for (int k = 0; k <= p; ++k) {
    // scale row k - 1 (final values of R and of Y)
    if (k > 0) {
      const int r = k - 1;
      for (int j = r + tid; j < p; j += nt) A[r + (int64_t)j * ld] = scl(A[r + (int64_t)j * ld], irk_prev);
      for (int c = tid; c <= r; c += nt) Z[r + (int64_t)c * ld] = scl(Z[r + (int64_t)c * ld], irk_prev);
    }
    if (k == p) break;
    double dkk = re_(A[k + (int64_t)k * ld]);
    if (!(dkk > 1e-300)) {
      if (tid == 0) bad_s = 1;
      dkk = 1.0;
    }
    const double idk = 1.0 / dkk;
    irk_prev = 1.0 / sqrt(dkk);
    for (int j = k + 1 + ty; j < p; j += 32) {
      const T akj = scl(A[k + (int64_t)j * ld], idk);
      for (int i = k + 1 + tx; i <= j; i += 32)
        A[i + (int64_t)j * ld] = sub(A[i + (int64_t)j * ld], mul(conj_(A[k + (int64_t)i * ld]), akj));
    }
    for (int c = ty; c <= k; c += 32) {
      const T zkc = scl(Z[k + (int64_t)c * ld], idk);
      for (int i = k + 1 + tx; i < p; i += 32)
        Z[i + (int64_t)c * ld] = sub(Z[i + (int64_t)c * ld], mul(conj_(A[k + (int64_t)i * ld]), zkc));
    }
    __syncthreads();
  }
  __syncthreads();
  if (tid == 0 && bad_s) *flag = 1;
  for (int e = tid; e < p * p; e += nt) {
    const int i = e % p, j = e / p;
    Rg[e] = i <= j ? A[i + (int64_t)j * ld] : ST<T>::zero();
    Rinv[e] = i <= j ? conj_(Z[j + (int64_t)i * ld]) : ST<T>::zero();
  }
}

template <typename T>
__global__ void upper_mul_kernel(const T* __restrict__ A, const T* __restrict__ B, T* __restrict__ C, int p) {
  int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= p * p) return;
  int i = e % p, j = e / p;
  T s = ST<T>::zero();
  for (int t = i; t <= j; ++t) s = fma_(s, A[i + t * p], B[t + j * p]);
  C[e] = (i <= j) ? s : ST<T>::zero();
}

template <typename T>
__global__ void put_block_kernel(T* __restrict__ H, int64_t ldh, int64_t r0, int64_t c0, const T* __restrict__ X,
                                 int p) {
  int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= p * p) return;
  int i = e % p, j = e / p;
  H[(r0 + i) + (c0 + j) * ldh] = X[e];
}

// ---------------- shifted least squares ----------------
template <typename T>
__global__ void hls_init_kernel(HlsState st, const T* __restrict__ R0) {
  const int s = blockIdx.y;
  const int64_t tot = st.ldr * st.p;
  zd* g = st.g + (int64_t)s * tot;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < tot; e += (int64_t)gridDim.x * blockDim.x) {
    int64_t i = e % st.ldr, c = e / st.ldr;
    g[e] = (i < st.p) ? cvt<zd, T>(R0[i + c * st.p]) : zd{0.0, 0.0};
  }
}

// one wave per (column c, shift s): load block column k, apply reflectors of blocks < k
template <typename HT>
__global__ __launch_bounds__(64) void hls_apply_prev_kernel(HlsState st, const HT* __restrict__ H, int64_t ldh, int k) {
  const int c = blockIdx.x, s = blockIdx.y, lane = threadIdx.x;
  const int p = st.p;
  const int64_t ldr = st.ldr;
  zd* Rs = st.R + (int64_t)s * ldr * st.mmax * p;
  zd* col = Rs + ((int64_t)k * p + c) * ldr;
  const int64_t rows = (int64_t)(k + 2) * p;
  const HT* hc = H + ((int64_t)k * p + c) * ldh;
  const double sh = st.shift_im[s];
  for (int64_t i = lane; i < ldr; i += 64) {
    zd v = i < rows ? cvt<zd, HT>(hc[i]) : zd{0.0, 0.0};
    if (i == (int64_t)k * p + c) v.im += sh;
    col[i] = v;
  }
  const zd* refl = st.refl + (int64_t)s * st.mmax * p * (p + 1);
  const double* tau = st.tau + (int64_t)s * st.mmax * p;
  for (int j = 0; j < k; ++j) {
    for (int q = 0; q < p; ++q) {
      const zd* v = refl + ((int64_t)j * p + q) * (p + 1);
      const double t = tau[(int64_t)j * p + q];
      const int64_t base = (int64_t)j * p + q;
      // lane owns rows r with r % 64 == lane: i = r - base
      int i0 = (int)((lane - base % 64 + 64) % 64);
      double dr = 0.0, di = 0.0;
      for (int i = i0; i <= p; i += 64) {
        zd vv = v[i], x = col[base + i];
        dr += vv.re * x.re + vv.im * x.im;  // conj(v) x
        di += vv.re * x.im - vv.im * x.re;
      }
      dr = wave_sum(dr);
      di = wave_sum(di);
      const double fr = t * dr, fi = t * di;
      for (int i = i0; i <= p; i += 64) {
        zd vv = v[i];
        zd x = col[base + i];
        x.re -= fr * vv.re - fi * vv.im;
        x.im -= fr * vv.im + fi * vv.re;
        col[base + i] = x;
      }
    }
  }
}

// one workgroup (4 waves) per shift: reduce the new panel, update g, residuals
__global__ __launch_bounds__(256) void hls_factor_kernel(HlsState st, int k, double* __restrict__ res) {
  const int s = blockIdx.x;
  const int p = st.p;
  const int64_t ldr = st.ldr;
  const int tid = threadIdx.x, lane = tid % 64, wave = tid / 64;
  zd* Rs = st.R + (int64_t)s * ldr * st.mmax * p;
  zd* g = st.g + (int64_t)s * ldr * p;
  zd* refl = st.refl + (int64_t)s * st.mmax * p * (p + 1);
  double* tau = st.tau + (int64_t)s * st.mmax * p;
  __shared__ double tau_s;
  for (int q = 0; q < p; ++q) {
    const int64_t base = (int64_t)k * p + q;
    zd* colq = Rs + base * ldr;  // column k p + q
    zd* v = refl + ((int64_t)k * p + q) * (p + 1);
    if (wave == 0) {
      int i0 = (int)((lane - base % 64 + 64) % 64);
      double nrm = 0.0;
      for (int i = i0; i <= p; i += 64) {
        zd x = colq[base + i];
        nrm += x.re * x.re + x.im * x.im;
      }
      nrm = sqrt(wave_sum(nrm));
      zd x0 = colq[base];
      double ax0 = sqrt(x0.re * x0.re + x0.im * x0.im);
      double phr = ax0 > 0.0 ? x0.re / ax0 : 1.0, phi = ax0 > 0.0 ? x0.im / ax0 : 0.0;
      // v = x + phase(x0) ||x|| e1 ; P = I - tau v v^H ; P x = -phase ||x|| e1
      double vn2 = 0.0;
      for (int i = i0; i <= p; i += 64) {
        zd x = colq[base + i];
        if (i == 0) {
          x.re += phr * nrm;
          x.im += phi * nrm;
        }
        v[i] = x;
        vn2 += x.re * x.re + x.im * x.im;
      }
      vn2 = wave_sum(vn2);
      double t = vn2 > 0.0 ? 2.0 / vn2 : 0.0;
      for (int i = i0; i <= p; i += 64) colq[base + i] = (i == 0) ? zd{-phr * nrm, -phi * nrm} : zd{0.0, 0.0};
      if (lane == 0) {
        tau[(int64_t)k * p + q] = t;
        tau_s = t;
      }
    }
    __threadfence_block();
    __syncthreads();
    const double t = tau_s;
    // apply to panel columns q+1..p-1 and to the p columns of g (fixed wave per column)
    const int ncols = (p - q - 1) + p;
    for (int cc = wave; cc < ncols; cc += 4) {
      zd* y = (cc < p - q - 1) ? Rs + ((int64_t)k * p + q + 1 + cc) * ldr : g + (int64_t)(cc - (p - q - 1)) * ldr;
      int i0 = (int)((lane - base % 64 + 64) % 64);
      double dr = 0.0, di = 0.0;
      for (int i = i0; i <= p; i += 64) {
        zd vv = v[i], x = y[base + i];
        dr += vv.re * x.re + vv.im * x.im;
        di += vv.re * x.im - vv.im * x.re;
      }
      dr = wave_sum(dr);
      di = wave_sum(di);
      const double fr = t * dr, fi = t * di;
      for (int i = i0; i <= p; i += 64) {
        zd vv = v[i], x = y[base + i];
        x.re -= fr * vv.re - fi * vv.im;
        x.im -= fr * vv.im + fi * vv.re;
        y[base + i] = x;
      }
    }
    __threadfence_block();
    __syncthreads();
  }
  // residual norms: rows (k+1)p .. (k+2)p of g
  for (int c = wave; c < p; c += 4) {
    const zd* y = g + (int64_t)c * ldr;
    double n2 = 0.0;
    for (int i = lane; i < p; i += 64) {
      zd x = y[(int64_t)(k + 1) * p + i];
      n2 += x.re * x.re + x.im * x.im;
    }
    n2 = wave_sum(n2);
    if (lane == 0) res[(int64_t)s * p + c] = sqrt(n2);
  }
}

// ---- faster variants for p <= 128 ----------------------------------------
// Active-window formulation: reflectors of block j touch rows [jp, (j+2)p).
// Each wave owns one column and keeps that window in LDS as a circular buffer
// of W = roundup(2p, 64) slots; lane l only ever touches rows r = l (mod 64),
// which always map to its own slots, so a wave needs no barrier.
__device__ inline int win_slots(int p) { return ((2 * p + 63) / 64) * 64; }

template <typename HT>
__global__ __launch_bounds__(256) void hls_apply_prev_lds_kernel(HlsState st, const HT* __restrict__ H, int64_t ldh,
                                                                 int k) {
  extern __shared__ zd win_all[];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int c = blockIdx.x * 4 + wave, s = blockIdx.y;
  const int p = st.p;
  if (c >= p) return;
  const int W = win_slots(p);
  zd* win = win_all + wave * W;
  const int64_t ldr = st.ldr;
  zd* col = st.R + (int64_t)s * ldr * st.mmax * p + ((int64_t)k * p + c) * ldr;
  const HT* hc = H + ((int64_t)k * p + c) * ldh;
  const double sh = st.shift_im[s];
  const int64_t diag = (int64_t)k * p + c;
  auto load_rows = [&](int64_t r0, int64_t r1) {  // rows [r0, r1) from H into the window
    for (int64_t r = r0 + ((lane - r0 % 64) + 64) % 64; r < r1; r += 64) {
      zd v = cvt<zd, HT>(hc[r]);
      if (r == diag) v.im += sh;
      win[r % W] = v;
    }
  };
  load_rows(0, 2 * (int64_t)p);
  const zd* refl = st.refl + (int64_t)s * st.mmax * p * (p + 1);
  const double* tau = st.tau + (int64_t)s * st.mmax * p;
  for (int j = 0; j < k; ++j) {
    for (int q = 0; q < p; ++q) {
      const zd* v = refl + ((int64_t)j * p + q) * (p + 1);
      const double t = tau[(int64_t)j * p + q];
      const int64_t base = (int64_t)j * p + q;
      const int i0 = (int)(((lane - base % 64) + 64) % 64);
      double dr = 0.0, di = 0.0;
      for (int i = i0; i <= p; i += 64) {
        zd vv = v[i], x = win[(base + i) % W];
        dr += vv.re * x.re + vv.im * x.im;
        di += vv.re * x.im - vv.im * x.re;
      }
      dr = wave_sum(dr);
      di = wave_sum(di);
      const double fr = t * dr, fi = t * di;
      for (int i = i0; i <= p; i += 64) {
        zd vv = v[i];
        zd& x = win[(base + i) % W];
        x.re -= fr * vv.re - fi * vv.im;
        x.im -= fr * vv.im + fi * vv.re;
      }
    }
    // rows [jp, (j+1)p) are final; rows [(j+2)p, (j+3)p) enter the window
    const int64_t r0 = (int64_t)j * p, r1 = r0 + p;
    for (int64_t r = r0 + ((lane - r0 % 64) + 64) % 64; r < r1; r += 64) col[r] = win[r % W];
    load_rows((int64_t)(j + 2) * p, (int64_t)(j + 3) * p);
  }
  const int64_t r0 = (int64_t)k * p, r1 = r0 + 2 * (int64_t)p;
  for (int64_t r = r0 + ((lane - r0 % 64) + 64) % 64; r < r1; r += 64) col[r] = win[r % W];
  // rows below the window are zero
  for (int64_t r = r1 + ((lane - r1 % 64) + 64) % 64; r < ldr; r += 64) col[r] = zd{0.0, 0.0};
}

// Panel reduction with the 2p x p panel in registers: 8 lanes per column,
// lane `sub` owns window rows w = sub + 8 t.
template <int PB>
__global__ __launch_bounds__(8 * PB) void hls_factor_reg_kernel(HlsState st, int k) {
  constexpr int NT = PB / 4;  // 2 PB rows / 8 lanes
  const int s = blockIdx.x;
  const int p = st.p;
  const int tid = threadIdx.x, c = tid >> 3, sub = tid & 7;
  const int64_t ldr = st.ldr;
  const bool active = c < p;
  zd* Rs = st.R + (int64_t)s * ldr * st.mmax * p;
  zd* colp = Rs + ((int64_t)k * p + (active ? c : 0)) * ldr + (int64_t)k * p;
  zd* refl = st.refl + (int64_t)s * st.mmax * p * (p + 1);
  double* tau = st.tau + (int64_t)s * st.mmax * p;
  double xr[NT], xi[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    int w = sub + 8 * t;
    zd v = (active && w < 2 * p) ? colp[w] : zd{0.0, 0.0};
    xr[t] = v.re;
    xi[t] = v.im;
  }
  __shared__ double vre[2][PB + 1], vim[2][PB + 1], tau_s[2];
  const int gbase = (tid & 63) & ~7;
  for (int q = 0; q < p; ++q) {
    const int b = q & 1;
    if (c == q) {
      double n2 = 0.0, x0r = 0.0, x0i = 0.0;
#pragma unroll
      for (int t = 0; t < NT; ++t) {
        int w = sub + 8 * t;
        if (w >= q && w <= q + p) n2 += xr[t] * xr[t] + xi[t] * xi[t];
        if (w == q) {
          x0r = xr[t];
          x0i = xi[t];
        }
      }
      n2 += __shfl_xor(n2, 1, 64);
      n2 += __shfl_xor(n2, 2, 64);
      n2 += __shfl_xor(n2, 4, 64);
      x0r = __shfl(x0r, gbase + (q & 7), 64);
      x0i = __shfl(x0i, gbase + (q & 7), 64);
      const double nrm = sqrt(n2), ax0 = sqrt(x0r * x0r + x0i * x0i);
      const double phr = ax0 > 0.0 ? x0r / ax0 : 1.0, phi = ax0 > 0.0 ? x0i / ax0 : 0.0;
      const double tq = nrm > 0.0 ? 1.0 / (n2 + ax0 * nrm) : 0.0;  // 2 / ||v||^2
      zd* vg = refl + ((int64_t)k * p + q) * (p + 1);
#pragma unroll
      for (int t = 0; t < NT; ++t) {
        int w = sub + 8 * t;
        if (w >= q && w <= q + p) {
          double a = xr[t], bb = xi[t];
          if (w == q) {
            a += phr * nrm;
            bb += phi * nrm;
          }
          vre[b][w - q] = a;
          vim[b][w - q] = bb;
          vg[w - q] = zd{a, bb};
          xr[t] = (w == q) ? -phr * nrm : 0.0;
          xi[t] = (w == q) ? -phi * nrm : 0.0;
        }
      }
      if (sub == 0) {
        tau_s[b] = tq;
        tau[(int64_t)k * p + q] = tq;
      }
    }
    __syncthreads();
    if (active && c > q) {
      double dr = 0.0, di = 0.0;
#pragma unroll
      for (int t = 0; t < NT; ++t) {
        int w = sub + 8 * t;
        if (w >= q && w <= q + p) {
          double a = vre[b][w - q], bb = vim[b][w - q];
          dr += a * xr[t] + bb * xi[t];
          di += a * xi[t] - bb * xr[t];
        }
      }
      dr += __shfl_xor(dr, 1, 64);
      dr += __shfl_xor(dr, 2, 64);
      dr += __shfl_xor(dr, 4, 64);
      di += __shfl_xor(di, 1, 64);
      di += __shfl_xor(di, 2, 64);
      di += __shfl_xor(di, 4, 64);
      const double fr = tau_s[b] * dr, fi = tau_s[b] * di;
#pragma unroll
      for (int t = 0; t < NT; ++t) {
        int w = sub + 8 * t;
        if (w >= q && w <= q + p) {
          double a = vre[b][w - q], bb = vim[b][w - q];
          xr[t] -= fr * a - fi * bb;
          xi[t] -= fr * bb + fi * a;
        }
      }
    }
  }
  if (active) {
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      int w = sub + 8 * t;
      if (w < 2 * p) colp[w] = zd{xr[t], xi[t]};
    }
  }
}

// apply the p reflectors of block k to the right-hand side g, then the
// residual norms of rows [(k+1)p, (k+2)p): one wave per (column, shift)
__global__ __launch_bounds__(256) void hls_apply_g_kernel(HlsState st, int k, double* __restrict__ res) {
  extern __shared__ zd gwin_all[];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int c = blockIdx.x * 4 + wave, s = blockIdx.y;
  const int p = st.p;
  if (c >= p) return;
  const int W = win_slots(p);
  zd* win = gwin_all + wave * W;
  const int64_t ldr = st.ldr;
  zd* gc = st.g + (int64_t)s * ldr * p + (int64_t)c * ldr + (int64_t)k * p;  // window row 0
  for (int w = lane; w < 2 * p; w += 64) win[w] = gc[w];
  const zd* refl = st.refl + (int64_t)s * st.mmax * p * (p + 1);
  const double* tau = st.tau + (int64_t)s * st.mmax * p;
  for (int q = 0; q < p; ++q) {
    const zd* v = refl + ((int64_t)k * p + q) * (p + 1);
    const double t = tau[(int64_t)k * p + q];
    const int i0 = ((lane - q % 64) + 64) % 64;
    double dr = 0.0, di = 0.0;
    for (int i = i0; i <= p; i += 64) {
      zd vv = v[i], x = win[q + i];
      dr += vv.re * x.re + vv.im * x.im;
      di += vv.re * x.im - vv.im * x.re;
    }
    dr = wave_sum(dr);
    di = wave_sum(di);
    const double fr = t * dr, fi = t * di;
    for (int i = i0; i <= p; i += 64) {
      zd vv = v[i];
      zd& x = win[q + i];
      x.re -= fr * vv.re - fi * vv.im;
      x.im -= fr * vv.im + fi * vv.re;
    }
  }
  double n2 = 0.0;
  for (int w = lane; w < 2 * p; w += 64) {
    gc[w] = win[w];
    if (w >= p) n2 += win[w].re * win[w].re + win[w].im * win[w].im;
  }
  n2 = wave_sum(n2);
  if (lane == 0) res[(int64_t)s * p + c] = sqrt(n2);
}

// one wave per (column c, shift s): Y = R^{-1} g over the first m p rows
__global__ __launch_bounds__(64) void hls_backsolve_kernel(HlsState st, int m, zd* __restrict__ Y) {
  const int c = blockIdx.x, s = blockIdx.y, lane = threadIdx.x;
  const int p = st.p;
  const int64_t ldr = st.ldr, mp = (int64_t)m * p;
  const zd* Rs = st.R + (int64_t)s * ldr * st.mmax * p;
  const zd* gs = st.g + (int64_t)s * ldr * p + (int64_t)c * ldr;
  zd* y = Y + (int64_t)s * mp * p + (int64_t)c * mp;
  for (int64_t i = lane; i < mp; i += 64) y[i] = gs[i];
  for (int64_t t = mp - 1; t >= 0; --t) {
    // owner lane of row t computes y_t and broadcasts it
    zd yt{0.0, 0.0};
    if (lane == (int)(t % 64)) {
      zd r = Rs[t + t * ldr], v = y[t];
      double den = r.re * r.re + r.im * r.im;
      yt = zd{(v.re * r.re + v.im * r.im) / den, (v.im * r.re - v.re * r.im) / den};
      y[t] = yt;
    }
    yt.re = __shfl(yt.re, (int)(t % 64), 64);
    yt.im = __shfl(yt.im, (int)(t % 64), 64);
    const zd* rc = Rs + t * ldr;
    for (int64_t i = lane; i < t; i += 64) {
      zd r = rc[i], v = y[i];
      v.re -= r.re * yt.re - r.im * yt.im;
      v.im -= r.re * yt.im + r.im * yt.re;
      y[i] = v;
    }
  }
}

// ---- restarts (collinear residuals) ----
// g_s = per-shift right-hand side G0_s (p x p col-major at G0 + s p p) in the
// first p rows, zero below
__global__ void hls_init_multi_kernel(HlsState st, const zd* __restrict__ G0) {
  const int s = blockIdx.y;
  const int64_t tot = st.ldr * st.p;
  zd* g = st.g + (int64_t)s * tot;
  const zd* g0 = G0 + (int64_t)s * st.p * st.p;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < tot; e += (int64_t)gridDim.x * blockDim.x) {
    int64_t i = e % st.ldr, c = e / st.ldr;
    g[e] = (i < st.p) ? g0[i + c * st.p] : zd{0.0, 0.0};
  }
}

// one wave per (column c, shift): Z_c <- Q_s Z_c (adjoint = 0: reflectors of the
// first m blocks in reverse order) or Q_s^H Z_c (adjoint = 1: forward order);
// rows [0, (m+1) p) of each column.  shift < 0: blockIdx.y is the shift and its
// columns start at Z + y zstride; otherwise every column uses that one shift.
__global__ __launch_bounds__(64) void hls_apply_q_kernel(HlsState st, int shift, int m, zd* __restrict__ Z,
                                                          int64_t ldz, int64_t zstride, int adjoint) {
  const int c = blockIdx.x, lane = threadIdx.x;
  const int s = shift < 0 ? (int)blockIdx.y : shift;
  const int p = st.p;
  zd* col = Z + (shift < 0 ? (int64_t)blockIdx.y * zstride : 0) + (int64_t)c * ldz;
  const zd* refl = st.refl + (int64_t)s * st.mmax * p * (p + 1);
  const double* tau = st.tau + (int64_t)s * st.mmax * p;
  const int nref = m * p;
  for (int r = 0; r < nref; ++r) {
    const int idx = adjoint ? r : nref - 1 - r;  // reflector j p + q acts on rows [idx, idx + p]
    const zd* v = refl + (int64_t)idx * (p + 1);
    const double t = tau[idx];
    const int i0 = (int)((lane - idx % 64 + 64) % 64);
    double dr = 0.0, di = 0.0;
    for (int i = i0; i <= p; i += 64) {
      zd vv = v[i], x = col[idx + i];
      dr += vv.re * x.re + vv.im * x.im;
      di += vv.re * x.im - vv.im * x.re;
    }
    dr = wave_sum(dr);
    di = wave_sum(di);
    const double fr = t * dr, fi = t * di;
    for (int i = i0; i <= p; i += 64) {
      zd vv = v[i], x = col[idx + i];
      x.re -= fr * vv.re - fi * vv.im;
      x.im -= fr * vv.im + fi * vv.re;
      col[idx + i] = x;
    }
  }
}

// g_s(i, c) -= sum_t T_s(i, t) W_s(t, c) for i < m p, every shift but `skip`
// (T_s: (m+1) p x p col-major at T + s tstride; W_s: p x p col-major)
__global__ void hls_collinear_rhs_kernel(HlsState st, int m, const zd* __restrict__ T, int64_t tstride,
                                         const zd* __restrict__ Wc, int skip) {
  const int s = blockIdx.y;
  if (s == skip) return;
  const int p = st.p;
  const int64_t mp = (int64_t)m * p, ldt = (int64_t)(m + 1) * p;
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= mp * p) return;
  const int64_t i = e % mp;
  const int c = (int)(e / mp);
  const zd* Ts = T + (int64_t)s * tstride;
  const zd* Ws = Wc + (int64_t)s * p * p;
  zd acc{0.0, 0.0};
  for (int t = 0; t < p; ++t) acc = fma_(acc, Ts[i + t * ldt], Ws[t + (int64_t)c * p]);
  zd* g = st.g + (int64_t)s * st.ldr * p + (int64_t)c * st.ldr + i;
  *g = sub(*g, acc);
}

// Er (rows x 2p col-major doubles): column 2c = Re Z(:, c), 2c + 1 = Im Z(:, c)
__global__ void cols_re_im_kernel(const zd* __restrict__ Z, int64_t ldz, int64_t rows, int p, double* __restrict__ Er) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= rows * p) return;
  const int64_t i = e % rows;
  const int c = (int)(e / rows);
  const zd z = Z[i + (int64_t)c * ldz];
  Er[i + (int64_t)(2 * c) * rows] = z.re;
  Er[i + (int64_t)(2 * c + 1) * rows] = z.im;
}

__global__ void hls_combine_real_kernel(const zd* __restrict__ Y, int64_t mp, int p, int nshift,
                                        const double* __restrict__ coef, double* __restrict__ C) {
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= mp * p) return;
  double s = 0.0;
  for (int q = 0; q < nshift; ++q) s += coef[q] * Y[(int64_t)q * mp * p + e].re;
  C[e] = s;
}

__global__ void hls_combine_cplx_kernel(const zd* __restrict__ Y, int64_t mp, int p, int nshift,
                                        const double* __restrict__ coef, zd* __restrict__ C) {
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= mp * p) return;
  zd s{0.0, 0.0};
  for (int q = 0; q < nshift; ++q) s = add(s, scl(Y[(int64_t)q * mp * p + e], coef[q]));
  C[e] = s;
}

// ---------------- Rayleigh-Ritz (single workgroup) ----------------
// Hermitian eigensolver of one workgroup (1024 threads) for the Rayleigh-Ritz
// reductions: Householder reduction to tridiagonal form, symmetric QR steps with
// Wilkinson shifts on the real tridiagonal, and the accumulated transformations
// (Golub & Van Loan, Matrix Computations, sections 8.3.1-8.3.3).
//   1. For k = 0 .. m-3: H_k = I - tau v v^H maps A(k+1:, k) to alpha_k e_1, and
//      A22 <- H_k A22 H_k by p = tau A22 v, w = p - (tau/2)(v^H p) v,
//      A22 -= v w^H + w v^H.  v overwrites A(k+1:, k).
//   2. Unit phases delta (delta_0 = 1, delta_{k+1} = delta_k alpha_k / |alpha_k|)
//      give T = D T_r D^H with T_r real, subdiagonal |alpha_k|.
//   3. Thread 0 runs the implicit QR steps on T_r; each step is a chain of plane
//      rotations on neighbouring columns (k, k+1), which the other 15 waves apply
//      to the rows of V = D (one row per thread) one step behind the producer.
//   4. V <- H_0 H_1 ... H_{m-3} V, so that A = V diag(d) V^H.
// In: M (m x m, col-major, global), Hermitian.  Out: the eigenvalues on M's
// diagonal (unsorted), V (m x m, global) the eigenvectors as columns; M's strict
// lower part holds the reflectors.  The matrix stage runs in LDS when m^2 values
// fit beside the vectors, else in global memory.
constexpr double kHeevEps = 1.1102230246251565e-16;  // 2^-53

// plane rotation (c, s) with c x - s z = r, s x + c z = 0: 1/r from the hardware
// reciprocal square root and two Newton steps (no divide on the serial chain)
__device__ inline void heev_givens(double x, double z, double& c, double& s, double& r) {
  const double r2 = fma(x, x, z * z);
  if (r2 > 0.0) {
    double y = __builtin_amdgcn_rsq(r2);
    const double hh = 0.5 * r2;
    y = y * fma(-hh * y, y, 1.5);
    y = y * fma(-hh * y, y, 1.5);
    c = x * y;
    s = -z * y;
    r = r2 * y;
  } else {
    c = 1.0;
    s = 0.0;
    r = 0.0;
  }
}

// LDS layout: dd, ee, tau, rc[2m], rs[2m] (double), ph, pv, vs (T), then the matrix
template <typename T>
__device__ inline size_t heev_mat_off(int m) {
  return ((size_t)m * (7 * sizeof(double) + 3 * sizeof(T)) + 255) & ~(size_t)255;
}

__device__ inline bool heev_negligible(double e, double d0, double d1) {
  return fabs(e) <= kHeevEps * (fabs(d0) + fabs(d1));
}

// L: the matrix stage (A, then V) is in LDS.  A compile-time choice, so that every
// matrix access has a fixed address space (LDS or global), never a flat one.
template <typename T, bool L>
__device__ __attribute__((always_inline)) bool heev_run(T* __restrict__ Mg, T* __restrict__ Vg, int m, char* lds) {
  const int tid = threadIdx.x, nt = blockDim.x;
  const int wv = tid >> 6, ln = tid & 63, nw = nt >> 6;
  __shared__ int sw_l[2], sw_h[2], ql_done[2], q_capped;
  // vectors first, the matrix after them
  double* dd = (double*)lds;  // diagonal of T_r
  double* ee = dd + m;        // ee[k] couples k and k+1
  double* tau = ee + m;
  double* rc = tau + m;       // rotation buffers [2][m] cosines, [2][m] sines
  double* rs = rc + 2 * m;
  T* ph = (T*)(rs + 2 * m);   // alpha_k / |alpha_k|
  T* pv = ph + m;             // p, then the phases delta, then v^H V
  T* vs = pv + m;             // staged reflector
  constexpr bool in_lds = L;
  T* A = L ? (T*)(lds + heev_mat_off<T>(m)) : Mg;
  if (in_lds) {
    for (int j = wv; j < m; j += nw)
      for (int i = ln; i < m; i += 64) A[i + (int64_t)j * m] = Mg[i + (int64_t)j * m];
    __syncthreads();
  }
  // 1. Householder tridiagonalization
  for (int k = 0; k + 2 < m; ++k) {
    const int r0 = k + 1, len = m - r0;
    T* x = A + r0 + (int64_t)k * m;
    if (tid < 64) {
      double rest = 0.0;
      for (int i = 1 + tid; i < len; i += 64) rest += abs2(x[i]);
      rest = wave_sum(rest);
      if (tid == 0) {
        const T x0 = x[0];
        const double ax0 = sqrt(abs2(x0));
        const T phase = ax0 > 0.0 ? scl(x0, 1.0 / ax0) : ST<T>::one();
        dd[k] = re_(A[k + (int64_t)k * m]);
        if (rest == 0.0) {  // column already reduced
          tau[k] = 0.0;
          ee[k] = ax0;
          ph[k] = phase;
        } else {
          const double nrm = sqrt(rest + ax0 * ax0);
          const T v0 = add(x0, scl(phase, nrm));  // v = x - alpha e_1, alpha = -phase |x|
          tau[k] = 2.0 / (rest + abs2(v0));
          ee[k] = nrm;
          ph[k] = neg(phase);
          x[0] = v0;
        }
      }
    }
    __threadfence_block();
    __syncthreads();
    const double tk = tau[k];
    if (tk == 0.0) continue;
    {  // p = tau A22 v, 8 lanes per row
      const int row = tid >> 3, l8 = tid & 7;
      for (int i = row; i < len; i += nt >> 3) {
        const T* arow = A + (r0 + i) + (int64_t)r0 * m;
        T acc = ST<T>::zero();
        for (int j = l8; j < len; j += 8) acc = fma_(acc, arow[(int64_t)j * m], x[j]);
        double ar = re_(acc), ai = 0.0;
        if constexpr (ST<T>::cplx) ai = acc.im;
#pragma unroll
        for (int o = 4; o > 0; o >>= 1) {
          ar += __shfl_xor(ar, o, 8);
          if constexpr (ST<T>::cplx) ai += __shfl_xor(ai, o, 8);
        }
        if (l8 == 0) {
          if constexpr (ST<T>::cplx)
            pv[i] = T{ar * tk, ai * tk};
          else
            pv[i] = ar * tk;
        }
      }
    }
    __threadfence_block();
    __syncthreads();
    // K = (tau / 2) v^H p is real: one reduction per wave
    double kk = 0.0;
    for (int j = ln; j < len; j += 64) kk += re_(mul(conj_(x[j]), pv[j]));
    kk = 0.5 * tk * wave_sum(kk);
    for (int j = wv; j < len; j += nw) {
      const T xj = x[j];
      const T wjc = conj_(sub(pv[j], scl(xj, kk))), xjc = conj_(xj);
      T* acol = A + r0 + (int64_t)(r0 + j) * m;
      for (int i = ln; i < len; i += 64) {
        const T xi = x[i];
        const T wi = sub(pv[i], scl(xi, kk));
        acol[i] = sub(acol[i], add(mul(xi, wjc), mul(wi, xjc)));
      }
    }
    __threadfence_block();
    __syncthreads();
  }
  if (tid == 0) {
    const int k = m - 2;
    dd[k] = re_(A[k + (int64_t)k * m]);
    dd[k + 1] = re_(A[(k + 1) + (int64_t)(k + 1) * m]);
    const T x0 = A[(k + 1) + (int64_t)k * m];
    const double ax0 = sqrt(abs2(x0));
    ee[k] = ax0;
    ph[k] = ax0 > 0.0 ? scl(x0, 1.0 / ax0) : ST<T>::one();
    tau[k] = 0.0;
    ee[m - 1] = 0.0;
    T dl = ST<T>::one();
    pv[0] = dl;
    for (int i = 0; i + 1 < m; ++i) {
      dl = mul(dl, ph[i]);
      pv[i + 1] = dl;
    }
  }
  __threadfence_block();
  __syncthreads();
  // the reflectors go back to M; V = D takes the matrix space
  T* V = in_lds ? A : Vg;
  if (in_lds) {
    for (int j = wv; j + 2 < m; j += nw)
      for (int i = j + 1 + ln; i < m; i += 64) Mg[i + (int64_t)j * m] = A[i + (int64_t)j * m];
    __syncthreads();
  }
  for (int j = wv; j < m; j += nw)
    for (int i = ln; i < m; i += 64) V[i + (int64_t)j * m] = i == j ? pv[i] : ST<T>::zero();
  __threadfence_block();
  __syncthreads();
  // 3. implicit QR steps: thread 0 produces the rotations of step r into buffer r & 1
  //    while the other waves apply step r - 1 to their rows of V.  The active block
  //    is [q_l, q_h]: everything below q_h has converged, ee[q_l - 1] is zero.
  int q_iter = 0, q_h = m - 1, q_l = 0;
  bool q_done = false;
  if (tid == 0) q_capped = 0;  // read after the rounds, which end with a barrier
  for (int round = 0;; ++round) {
    const int b = round & 1;
    if (tid == 0) {
      int l = 0, h = -1;
      while (!q_done) {
        while (q_h > q_l && heev_negligible(ee[q_h - 1], dd[q_h - 1], dd[q_h])) {
          ee[q_h - 1] = 0.0;
          --q_h;
        }
        if (q_h > q_l) break;
        if (q_l == 0) {
          q_done = true;
          break;
        }
        // the block above
        q_h = q_l - 1;
        int nl = q_h;
        while (nl > 0 && !heev_negligible(ee[nl - 1], dd[nl - 1], dd[nl])) --nl;
        if (nl > 0) ee[nl - 1] = 0.0;
        q_l = nl;
      }
      if (!q_done && q_iter >= 30 * m) {  // not converged: reported to the caller
        q_done = true;
        q_capped = 1;
      }
      if (!q_done) {
        l = q_l;
        h = q_h;
        ++q_iter;
        // Wilkinson shift from the trailing 2 x 2 block
        const double da = dd[h - 1], dc = dd[h], eb = ee[h - 1];
        const double dl2 = 0.5 * (da - dc);
        const double den = dl2 + (dl2 >= 0.0 ? 1.0 : -1.0) * sqrt(fma(dl2, dl2, eb * eb));
        const double mu = dc - eb * eb / den;
        // bulge chase, the state of the moving 2 x 2 window in registers
        double a0 = dd[l], b0 = ee[l], d0 = dd[l + 1];
        double e1 = l + 1 < h ? ee[l + 1] : 0.0;
        double xv = a0 - mu, zv = b0, dprev = 0.0, en = 0.0;
        double* rcb = rc + b * m;
        double* rsb = rs + b * m;
        int split = -1;
        for (int k = l; k < h; ++k) {
          const double d_nx = k + 2 <= h ? dd[k + 2] : 0.0;
          const double e_nx = k + 2 < h ? ee[k + 2] : 0.0;
          double c, sn, r;
          heev_givens(xv, zv, c, sn, r);
          const double cc = c * c, ss = sn * sn, cs = c * sn;
          const double an = fma(a0, cc, fma(-2.0 * b0, cs, d0 * ss));
          const double dn = fma(a0, ss, fma(2.0 * b0, cs, d0 * cc));
          en = fma(a0 - d0, cs, b0 * (cc - ss));
          dd[k] = an;
          if (k > l) {
            ee[k - 1] = r;
            if (heev_negligible(r, dprev, an)) split = k - 1;
          }
          rcb[k - l] = c;
          rsb[k - l] = sn;
          dprev = an;
          xv = en;
          zv = -sn * e1;
          b0 = c * e1;
          a0 = dn;
          d0 = d_nx;
          e1 = e_nx;
        }
        dd[h] = a0;
        ee[h - 1] = en;
        if (split >= 0) {
          ee[split] = 0.0;
          q_l = split + 1;
        }
      }
      sw_l[b] = l;
      sw_h[b] = h;
      ql_done[b] = q_done ? 1 : 0;
    } else if (tid >= 64 && round > 0) {
      const int pb = b ^ 1;
      const int l = sw_l[pb], h = sw_h[pb];
      if (h > l) {
        const double* cb = rc + pb * m;
        const double* sb = rs + pb * m;
        for (int r = tid - 64; r < m; r += nt - 64) {
          T* vr = V + r;
          T carry = vr[(int64_t)l * m];
          T zn = vr[(int64_t)(l + 1) * m];
          for (int k = l; k < h; ++k) {
            const T znext = k + 2 <= h ? vr[(int64_t)(k + 2) * m] : ST<T>::zero();
            const double c = cb[k - l], sn = sb[k - l];
            // columns (k, k+1) <- (c z_k - s z_{k+1}, s z_k + c z_{k+1})
            vr[(int64_t)k * m] = sub(scl(carry, c), scl(zn, sn));
            carry = add(scl(carry, sn), scl(zn, c));
            zn = znext;
          }
          vr[(int64_t)h * m] = carry;
        }
      }
    }
    __threadfence_block();
    __syncthreads();
    if (ql_done[b]) break;
  }
  // 4. back-transformation V <- H_k V, k = m-3 .. 0 (reflectors from M)
  for (int k = m - 3; k >= 0; --k) {
    const double tk = tau[k];
    if (tk == 0.0) continue;
    const int r0 = k + 1, len = m - r0;
    for (int i = tid; i < len; i += nt) vs[i] = Mg[(r0 + i) + (int64_t)k * m];
    __threadfence_block();
    __syncthreads();
    {  // pv[c] = tau v^H V(r0:, c), 8 lanes per column
      const int col = tid >> 3, l8 = tid & 7;
      for (int c = col; c < m; c += nt >> 3) {
        const T* vc = V + r0 + (int64_t)c * m;
        T acc = ST<T>::zero();
        for (int i = l8; i < len; i += 8) acc = fma_(acc, conj_(vs[i]), vc[i]);
        double ar = re_(acc), ai = 0.0;
        if constexpr (ST<T>::cplx) ai = acc.im;
#pragma unroll
        for (int o = 4; o > 0; o >>= 1) {
          ar += __shfl_xor(ar, o, 8);
          if constexpr (ST<T>::cplx) ai += __shfl_xor(ai, o, 8);
        }
        if (l8 == 0) {
          if constexpr (ST<T>::cplx)
            pv[c] = T{ar * tk, ai * tk};
          else
            pv[c] = ar * tk;
        }
      }
    }
    __threadfence_block();
    __syncthreads();
    for (int c = wv; c < m; c += nw) {
      const T sc = pv[c];
      T* vcol = V + r0 + (int64_t)c * m;
      for (int i = ln; i < len; i += 64) vcol[i] = sub(vcol[i], mul(vs[i], sc));
    }
    __threadfence_block();
    __syncthreads();
  }
  if (in_lds)
    for (int j = wv; j < m; j += nw)
      for (int i = ln; i < m; i += 64) Vg[i + (int64_t)j * m] = V[i + (int64_t)j * m];
  for (int i = tid; i < m; i += nt) Mg[i + (int64_t)i * m] = cvt<T, double>(dd[i]);
  __threadfence_block();
  __syncthreads();
  return q_capped == 0;
}

// returns false when the QR steps did not converge (iteration cap reached)
template <typename T>
__device__ __attribute__((always_inline)) bool heev_tridiag(T* __restrict__ Mg, T* __restrict__ Vg, int m, char* lds,
                                                            size_t lds_bytes) {
  if (m <= 0) return true;
  if (m == 1) {
    if (threadIdx.x == 0) {
      Vg[0] = ST<T>::one();
      Mg[0] = cvt<T, double>(re_(Mg[0]));
    }
    __threadfence_block();
    __syncthreads();
    return true;
  }
  if (heev_mat_off<T>(m) + (size_t)m * m * sizeof(T) <= lds_bytes) return heev_run<T, true>(Mg, Vg, m, lds);
  return heev_run<T, false>(Mg, Vg, m, lds);
}

// dynamic LDS of the Rayleigh-Ritz kernel: the 160 KB of a CU less its few static words
constexpr size_t kRrLdsBytes = 160 * 1024 - 256;

// Rank-revealing Rayleigh-Ritz: scale to unit diagonal of Bt, eigendecompose
// Bt, keep directions with eigenvalue > tau_rank * max, reduce At on them and
// eigendecompose the reduced Hermitian matrix.
template <typename T>
__global__ __launch_bounds__(1024) void rr_reduce_kernel(const T* __restrict__ At, const T* __restrict__ Bt, int n,
                                                         double tau_rank, double* __restrict__ theta,
                                                         T* __restrict__ Cmat, int* k_out, T* work) {
  extern __shared__ __align__(16) char rr_raw[];
  const int tid = threadIdx.x, nt = blockDim.x;
  const int64_t nn = (int64_t)n * n;
  T* As = work;
  T* Bs = work + nn;
  T* U = work + 2 * nn;
  T* Tm = work + 3 * nn;
  T* M1 = work + 4 * nn;
  T* W = work + 5 * nn;
  double* d = (double*)(work + 6 * nn);
  double* sv = d + n;
  int* idx = (int*)(sv + n);
  int* rank = idx + n;
  __shared__ int k_s;
  for (int i = tid; i < n; i += nt) {
    double b = re_(Bt[i + (int64_t)i * n]);
    d[i] = b > 0.0 ? sqrt(b) : 1.0;
  }
  __threadfence_block();
  __syncthreads();
  for (int64_t e = tid; e < nn; e += nt) {
    int i = (int)(e % n), j = (int)(e / n);
    double sc = 0.5 / (d[i] * d[j]);
    // Hermitian part
    As[e] = scl(add(At[e], conj_(At[j + (int64_t)i * n])), sc);
    Bs[e] = scl(add(Bt[e], conj_(Bt[j + (int64_t)i * n])), sc);
  }
  __threadfence_block();
  __syncthreads();
  const bool ok_b = heev_tridiag<T>(Bs, U, n, rr_raw, kRrLdsBytes);
  __syncthreads();
  for (int i = tid; i < n; i += nt) sv[i] = re_(Bs[i + (int64_t)i * n]);
  __threadfence_block();
  __syncthreads();
  if (tid == 0) {
    double mx = 0.0;
    for (int i = 0; i < n; ++i) mx = sv[i] > mx ? sv[i] : mx;
    int k = 0;
    for (int i = 0; i < n; ++i)
      if (sv[i] > tau_rank * mx) idx[k++] = i;
    k_s = k;
  }
  __threadfence_block();
  __syncthreads();
  const int k = k_s;
  // Tm(:, j) = U(:, idx_j) / sqrt(s_idx_j)   (n x k, ld n)
  for (int64_t e = tid; e < (int64_t)n * k; e += nt) {
    int i = (int)(e % n), j = (int)(e / n);
    int c = idx[j];
    Tm[e] = scl(U[i + (int64_t)c * n], 1.0 / sqrt(sv[c]));
  }
  __threadfence_block();
  __syncthreads();
  // M1 = As Tm (n x k); Ar = Tm^H M1 (k x k, ld k) into As
  for (int64_t e = tid; e < (int64_t)n * k; e += nt) {
    int i = (int)(e % n), j = (int)(e / n);
    T sacc = ST<T>::zero();
    for (int t = 0; t < n; ++t) sacc = fma_(sacc, As[i + (int64_t)t * n], Tm[t + (int64_t)j * n]);
    M1[e] = sacc;
  }
  __threadfence_block();
  __syncthreads();
  for (int64_t e = tid; e < (int64_t)k * k; e += nt) {
    int i = (int)(e % k), j = (int)(e / k);
    T sacc = ST<T>::zero();
    for (int t = 0; t < n; ++t) sacc = fma_(sacc, conj_(Tm[t + (int64_t)i * n]), M1[t + (int64_t)j * n]);
    As[i + (int64_t)j * k] = sacc;
  }
  __threadfence_block();
  __syncthreads();
  for (int64_t e = tid; e < (int64_t)k * k; e += nt) {
    int i = (int)(e % k), j = (int)(e / k);
    Bs[e] = scl(add(As[i + (int64_t)j * k], conj_(As[j + (int64_t)i * k])), 0.5);
  }
  __threadfence_block();
  __syncthreads();
  const bool ok_a = heev_tridiag<T>(Bs, W, k, rr_raw, kRrLdsBytes);
  __syncthreads();
  // ascending order of the Ritz values
  for (int i = tid; i < k; i += nt) {
    double ti = re_(Bs[i + (int64_t)i * k]);
    int r = 0;
    for (int j = 0; j < k; ++j) {
      double tj = re_(Bs[j + (int64_t)j * k]);
      if (tj < ti || (tj == ti && j < i)) ++r;
    }
    rank[i] = r;
    theta[r] = ti;
  }
  __threadfence_block();
  __syncthreads();
  // Cmat(:, rank_j) = D^-1 Tm W(:, j)
  for (int64_t e = tid; e < (int64_t)n * k; e += nt) {
    int i = (int)(e % n), j = (int)(e / n);
    T sacc = ST<T>::zero();
    for (int t = 0; t < k; ++t) sacc = fma_(sacc, Tm[i + (int64_t)t * n], W[t + (int64_t)j * k]);
    Cmat[i + (int64_t)rank[j] * n] = scl(sacc, 1.0 / d[i]);
  }
  if (tid == 0) *k_out = ok_b && ok_a ? k : -1;
}

constexpr int RN_ROWS = 512;

template <typename T>
__global__ void resid_partial_kernel(const T* __restrict__ AX, const T* __restrict__ BX, const T* __restrict__ X,
                                     const double* __restrict__ theta, int64_t n, int k, double* __restrict__ partial) {
  const int64_t r0 = (int64_t)blockIdx.x * RN_ROWS;
  const int64_t r1 = r0 + RN_ROWS < n ? r0 + RN_ROWS : n;
  for (int c = threadIdx.x; c < k; c += blockDim.x) {
    double th = theta[c], s1 = 0.0, s2 = 0.0, s3 = 0.0;
    for (int64_t i = r0; i < r1; ++i) {
      T bx = BX[i * k + c], ax = AX[i * k + c], x = X[i * k + c];
      T r = sub(ax, scl(bx, th));
      s1 += abs2(r);
      s2 += abs2(x);
      s3 += abs2(bx);
    }
    double* o = partial + (int64_t)blockIdx.x * 3 * k;
    o[3 * c] = s1;
    o[3 * c + 1] = s2;
    o[3 * c + 2] = s3;
  }
}

__global__ void resid_final_kernel(const double* __restrict__ partial, int nb, int k3, double* __restrict__ out) {
  int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= k3) return;
  double s = 0.0;
  for (int b = 0; b < nb; ++b) s += partial[(int64_t)b * k3 + c];
  out[c] = s;
}

}  // namespace

template <typename T>
void reduce_partials(T* out, int64_t ld_out, T* partial, int S, int M, int N, bool add, hipStream_t s) {
  int64_t MN = (int64_t)M * N;
  if (MN == 0) return;
  const unsigned nb = (unsigned)((MN + 255) / 256);
  int step = 1;
  if (S > kReduceGroup) {  // groups of kReduceGroup in parallel, then the group sums
    const int groups = (S + kReduceGroup - 1) / kReduceGroup;
    hipLaunchKernelGGL(reduce_groups_kernel<T>, dim3(nb, groups), dim3(256), 0, s, partial, S, kReduceGroup, MN);
    S = groups;
    step = kReduceGroup;
  }
  hipLaunchKernelGGL(reduce_partials_kernel<T>, dim3(nb), dim3(256), 0, s, out, ld_out, (const T*)partial, S, step, M,
                     N, add ? 1 : 0);
}

template <typename T>
void chol_upper_inv(const T* G, int p, double rel_shift, T* R, T* Rinv, int* flag, hipStream_t s) {
  const size_t one = sizeof(T) * (size_t)p * p;
  const size_t one_pad = sizeof(T) * (size_t)p * (p + 1);  // chol_inv_lds_kernel: leading dimension p + 1
  const bool use_lds = one <= 160 * 1024 - 4096;
  if (2 * one_pad <= 160 * 1024 - 4096) {
    (void)hipFuncSetAttribute((const void*)chol_inv_lds_kernel<T>, hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)(2 * one_pad));
    hipLaunchKernelGGL(chol_inv_lds_kernel<T>, dim3(1), dim3(1024), 2 * one_pad, s, G, p, rel_shift, R, Rinv, flag);
  } else if (use_lds) {
    const size_t lds = 2 * one <= 160 * 1024 - 4096 ? 2 * one : one;
    (void)hipFuncSetAttribute((const void*)chol_upper_inv_kernel<T, true>, hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)lds);
    hipLaunchKernelGGL((chol_upper_inv_kernel<T, true>), dim3(1), dim3(1024), lds, s, G, p, rel_shift, R, Rinv, flag);
  } else {
    hipLaunchKernelGGL((chol_upper_inv_kernel<T, false>), dim3(1), dim3(1024), 0, s, G, p, rel_shift, R, Rinv, flag);
  }
}

template <typename T>
void upper_mul(const T* A, const T* B, T* C, int p, hipStream_t s) {
  hipLaunchKernelGGL(upper_mul_kernel<T>, dim3((p * p + 255) / 256), dim3(256), 0, s, A, B, C, p);
}

template <typename T>
void put_block(T* H, int64_t ldh, int64_t r0, int64_t c0, const T* X, int p, hipStream_t s) {
  hipLaunchKernelGGL(put_block_kernel<T>, dim3((p * p + 255) / 256), dim3(256), 0, s, H, ldh, r0, c0, X, p);
}

template <typename T>
void hls_init(const HlsState& st, const T* R0, hipStream_t s) {
  hipLaunchKernelGGL(hls_init_kernel<T>, dim3(64, st.nshift), dim3(256), 0, s, st, R0);
}

template <typename T>
void hls_step(const HlsState& st, const T* H, int64_t ldh, int k, double* res, hipStream_t s) {
  if (st.p > 128) {
    hipLaunchKernelGGL(hls_apply_prev_kernel<T>, dim3(st.p, st.nshift), dim3(64), 0, s, st, H, ldh, k);
    hipLaunchKernelGGL(hls_factor_kernel, dim3(st.nshift), dim3(256), 0, s, st, k, res);
    return;
  }
  const size_t lds = sizeof(zd) * 4 * (size_t)(((2 * st.p + 63) / 64) * 64);
  const dim3 g4((st.p + 3) / 4, st.nshift);
  hipLaunchKernelGGL(hls_apply_prev_lds_kernel<T>, g4, dim3(256), lds, s, st, H, ldh, k);
  if (st.p <= 32)
    hipLaunchKernelGGL(hls_factor_reg_kernel<32>, dim3(st.nshift), dim3(256), 0, s, st, k);
  else if (st.p <= 64)
    hipLaunchKernelGGL(hls_factor_reg_kernel<64>, dim3(st.nshift), dim3(512), 0, s, st, k);
  else if (st.p <= 96)
    hipLaunchKernelGGL(hls_factor_reg_kernel<96>, dim3(st.nshift), dim3(768), 0, s, st, k);
  else
    hipLaunchKernelGGL(hls_factor_reg_kernel<128>, dim3(st.nshift), dim3(1024), 0, s, st, k);
  hipLaunchKernelGGL(hls_apply_g_kernel, g4, dim3(256), lds, s, st, k, res);
}

void hls_backsolve(const HlsState& st, int m, zd* Y, hipStream_t s) {
  hipLaunchKernelGGL(hls_backsolve_kernel, dim3(st.p, st.nshift), dim3(64), 0, s, st, m, Y);
}

void hls_init_multi(const HlsState& st, const zd* G0, hipStream_t s) {
  hipLaunchKernelGGL(hls_init_multi_kernel, dim3(64, st.nshift), dim3(256), 0, s, st, G0);
}

void hls_apply_q(const HlsState& st, int shift, int m, zd* Z, int64_t ldz, int64_t zstride, int ncols, bool adjoint,
                 hipStream_t s) {
  if (ncols <= 0 || m <= 0) return;
  hipLaunchKernelGGL(hls_apply_q_kernel, dim3(ncols, shift < 0 ? st.nshift : 1), dim3(64), 0, s, st, shift, m, Z, ldz,
                     zstride, adjoint ? 1 : 0);
}

void hls_collinear_rhs(const HlsState& st, int m, const zd* T, int64_t tstride, const zd* W, int skip,
                       hipStream_t s) {
  const int64_t tot = (int64_t)m * st.p * st.p;
  if (tot == 0) return;
  hipLaunchKernelGGL(hls_collinear_rhs_kernel, dim3((unsigned)((tot + 255) / 256), st.nshift), dim3(256), 0, s, st, m,
                     T, tstride, W, skip);
}

void cols_re_im(const zd* Z, int64_t ldz, int64_t rows, int p, double* Er, hipStream_t s) {
  const int64_t tot = rows * p;
  if (tot == 0) return;
  hipLaunchKernelGGL(cols_re_im_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, Z, ldz, rows, p, Er);
}

void hls_combine(const zd* Y, int m, int p, int nshift, const double* coef, double* C, hipStream_t s) {
  int64_t mp = (int64_t)m * p;
  hipLaunchKernelGGL(hls_combine_real_kernel, dim3((unsigned)((mp * p + 255) / 256)), dim3(256), 0, s, Y, mp, p,
                     nshift, coef, C);
}
void hls_combine(const zd* Y, int m, int p, int nshift, const double* coef, zd* C, hipStream_t s) {
  int64_t mp = (int64_t)m * p;
  hipLaunchKernelGGL(hls_combine_cplx_kernel, dim3((unsigned)((mp * p + 255) / 256)), dim3(256), 0, s, Y, mp, p,
                     nshift, coef, C);
}

template <typename T>
void rr_reduce(const T* At, const T* Bt, int n, double tau_rank, double* theta, T* Cmat, int* k_out, T* work,
               hipStream_t s) {
  const size_t lds = kRrLdsBytes;
  (void)hipFuncSetAttribute((const void*)rr_reduce_kernel<T>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  hipLaunchKernelGGL(rr_reduce_kernel<T>, dim3(1), dim3(1024), lds, s, At, Bt, n, tau_rank, theta, Cmat, k_out, work);
}

template <typename T>
void resid_norms(const T* AX, const T* BX, const T* X, const double* theta, int64_t n, int k, double* partial,
                 double* out, hipStream_t s) {
  int nb = (int)((n + RN_ROWS - 1) / RN_ROWS);
  if (nb == 0 || k == 0) return;
  hipLaunchKernelGGL(resid_partial_kernel<T>, dim3(nb), dim3(128), 0, s, AX, BX, X, theta, n, k, partial);
  hipLaunchKernelGGL(resid_final_kernel, dim3((3 * k + 127) / 128), dim3(128), 0, s, partial, nb, 3 * k, out);
}

#define KRYLOV_INST(T)                                                                                        \
  template void reduce_partials<T>(T*, int64_t, T*, int, int, int, bool, hipStream_t);                        \
  template void chol_upper_inv<T>(const T*, int, double, T*, T*, int*, hipStream_t);                         \
  template void upper_mul<T>(const T*, const T*, T*, int, hipStream_t);                                      \
  template void put_block<T>(T*, int64_t, int64_t, int64_t, const T*, int, hipStream_t);                     \
  template void hls_init<T>(const HlsState&, const T*, hipStream_t);                                         \
  template void hls_step<T>(const HlsState&, const T*, int64_t, int, double*, hipStream_t);                   \
  template void rr_reduce<T>(const T*, const T*, int, double, double*, T*, int*, T*, hipStream_t);            \
  template void resid_norms<T>(const T*, const T*, const T*, const double*, int64_t, int, double*, double*, \
                               hipStream_t);
KRYLOV_INST(double)
KRYLOV_INST(zd)
#undef KRYLOV_INST

}  // namespace zolo
