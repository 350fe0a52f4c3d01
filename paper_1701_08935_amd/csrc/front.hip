// Multifrontal LDL^T kernels (numeric factorization and solve helpers) for
// the r1 shifted matrices K_j = A - sigma_hat_j B of Algorithm 2, lines 5-6.
// Real pencils give complex-symmetric K_j, factored without pivoting in the
// nested-dissection order (A - sigma B with Im sigma != 0 has a definite
// skew-Hermitian part, so every leading principal block is nonsingular).
#include "front.h"

namespace zolo {
namespace {

// Every kernel of the factorization runs the same step for a batch of poles
// at once: the pole is the last grid dimension and pb[pole] its arrays.
template <typename T>
__global__ void assemble_kernel(const PoleBase<T>* __restrict__ pb, const int64_t* __restrict__ dst,
                                const int64_t* __restrict__ src, int64_t n, const double* __restrict__ a,
                                const double* __restrict__ b) {
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  const PoleBase<T>& q = pb[blockIdx.y];
  T* panel = q.panel;
  const double sr = q.sr, si = q.si;
  int64_t s = src[e];
  double av = a[s], bv = b[s];
  zd v{av - sr * bv, -si * bv};
  panel[dst[e]] = cvt<T, zd>(v);
}

// complex Hermitian pencils: a, b interleaved complex values
template <typename T>
__global__ void assemble_cplx_kernel(const PoleBase<T>* __restrict__ pb, bool upper, const int64_t* __restrict__ dst,
                                     const int64_t* __restrict__ src, int64_t n, const zd* __restrict__ a,
                                     const zd* __restrict__ b) {
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  const PoleBase<T>& q = pb[blockIdx.y];
  T* panel = upper ? q.upanel : q.panel;
  const double sr = q.sr, si = q.si;
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
__global__ void extend_add_lu_kernel(const PoleBase<T>* __restrict__ pb, const int32_t* __restrict__ pmap,
                                     const ExtDesc* __restrict__ descs) {
  const ExtDesc d = descs[blockIdx.y];
  const PoleBase<T>& q = pb[blockIdx.z];
  T* panel = q.panel;
  T* upanel = q.upanel;
  T* upd = q.upd;
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
__global__ void extend_add_kernel(const PoleBase<T>* __restrict__ pb, const int32_t* __restrict__ pmap,
                                  const ExtDesc* __restrict__ descs) {
  const ExtDesc d = descs[blockIdx.y];
  const PoleBase<T>& q = pb[blockIdx.z];
  T* panel = q.panel;
  T* upd = q.upd;
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

// Blocked factorization of the jb x jb diagonal block of step J (jb <= FB =
// 64), one workgroup (4 waves) per front, in 16-column panels so that only
// the 16 x 16 diagonal sub-blocks are eliminated column by column (by one
// wave, exchanging through LDS without workgroup barriers); everything else is
// small dense products over all threads.  For panel p (columns c0 = 16p ..):
//  A. wave 0: LDL^T (LU: L D U) of the 16 x 16 sub-block A_pp, and the
//     inverse X_pp of its unit lower factor (LU: also Y_pp = (U_pp^T)^-1);
//  B. rows below: L_ip = A_ip X_pp^T D_p^-1 (LU: A_ip U_pp^-1 D_p^-1 with
//     U_pp^-1 = Y_pp^T, and the row panel U_pi = D_p^-1 X_pp A_pi);
//  C. trailing block: A_ij -= L_ip D_p L_jp^T (LU: L_ip D_p U_pj).
// Then the off-diagonal blocks of X = L^-1 by block rows,
// X_IJ = -X_II sum_{J <= K < I} L_IK X_KJ (LU: Y from U^T likewise).
// LDS: A holds the block, then L (strict lower), D (diagonal) and, for LU,
// U (strict upper).  LU: X holds L^-1 in its lower triangle and (U^T)^-1
// transposed in its upper triangle (both unit diagonal).  LDL^T: the strict
// lower triangle of L^-1 is kept transposed in A's (otherwise unused) strict
// upper triangle, so the kernel needs about half the LDS (two workgroups, or
// one beside a GEMM workgroup, fit on a CU).
constexpr int SBK = 16;  // sub-block (panel) width

// 1 / d for a pivot: conj(d) / |d|^2 with one real division (the pivots here
// are far from the range where |d|^2 under- or overflows).
__device__ inline zd recip(zd a) {
  const double s = 1.0 / (a.re * a.re + a.im * a.im);
  return zd{a.re * s, -a.im * s};
}
__device__ inline zf recip(zf a) {
  const float s = 1.0f / (a.re * a.re + a.im * a.im);
  return zf{a.re * s, -a.im * s};
}
__device__ inline double recip(double a) { return 1.0 / a; }

// Component-wise select.  Writing c ? a : b on the complex structs makes the
// compiler select between their addresses, which keeps register arrays of
// them in scratch memory.
__device__ inline zd sel(bool c, zd a, zd b) { return zd{c ? a.re : b.re, c ? a.im : b.im}; }
__device__ inline zf sel(bool c, zf a, zf b) { return zf{c ? a.re : b.re, c ? a.im : b.im}; }
__device__ inline double sel(bool c, double a, double b) { return c ? a : b; }

template <typename T, bool LU>
__global__ __launch_bounds__(256) void diag_blocked_kernel(const PoleBase<T>* __restrict__ pb,
                                                           const DiagDesc* __restrict__ descs, int J) {
  const DiagDesc d = descs[blockIdx.x];
  const PoleBase<T>& q = pb[blockIdx.y];
  T* panel = q.panel;
  T* upanel = q.upanel;
  T* inv = q.inv;
  T* uinv = q.uinv;
  T* dvec = q.dvec;
  int* breakdown = q.flag;
  if (J >= d.ns) return;
  const int jb = (d.ns - J) < FB ? (d.ns - J) : FB;
  __shared__ T A[FB][FB + 1];
  __shared__ T X[LU ? FB : 1][LU ? FB + 1 : 1];
  __shared__ T Tm[SBK][FB - SBK + 1];            // block-row products of the inverse
  __shared__ T Dv[FB], Di[FB];                    // pivots and their inverses
  __shared__ T cb[2][SBK], rb[2][LU ? SBK : 1];  // column / row exchange inside a sub-block
  // entry (r, c), r > c, of the lower inverse L^-1
  auto XL = [&](int r, int c) -> T& {
    if constexpr (LU)
      return X[r][c];
    else
      return A[c][r];
  };
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const T one = ST<T>::one(), zero = ST<T>::zero();
  T* P = panel + d.panel;
  T* U = LU ? upanel + d.panel : nullptr;
  const int64_t k = d.k, ns = d.ns;

  for (int e = tid; e < FB * FB; e += blockDim.x) {
    const int r = e & (FB - 1), c = e >> 6;
    T v = zero;
    if (r < jb && c < jb) {
      if (r >= c)
        v = P[(J + r) + (int64_t)(J + c) * k];
      else if (LU)
        v = U[(J + c) + (int64_t)(J + r) * k];
    }
    A[r][c] = v;
    if constexpr (LU) X[r][c] = zero;
  }
  __syncthreads();

  const int np = (jb + SBK - 1) / SBK;
  for (int p = 0; p < np; ++p) {
    const int c0 = p * SBK, pb = min(SBK, jb - c0);
    // ---- A: the diagonal sub-block, by wave 0 ----
    if (wave == 0) {
      const int l = lane & (SBK - 1);
      T a[SBK];
#pragma unroll
      for (int t = 0; t < SBK; ++t) a[t] = A[c0 + l][c0 + t];
#pragma unroll
      for (int j = 0; j < SBK; ++j) {
        if (j >= pb) continue;  // partial last panel (uniform)
        const int b = j & 1;
        if (lane < SBK) {
          cb[b][lane] = a[j];  // column j
          if constexpr (LU) {
            if (lane == j) {
#pragma unroll
              for (int t = j + 1; t < SBK; ++t) rb[b][t] = a[t];  // row j
            }
          }
        }
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "workgroup");
        T dj = cb[b][j];
        if (abs2(dj) == 0.0) {
          if (lane == 0) atomicExch(breakdown, 1);
          dj = one;
        }
        const T dinv = recip(dj);
        const bool below = l > j;
        const T g = mul(a[j], dinv);  // L(l, j) for l > j
#pragma unroll
        for (int t = j + 1; t < SBK; ++t) {
          T w;  // A(j, t) (= A(t, j) for LDL^T)
          if constexpr (LU)
            w = rb[b][t];
          else
            w = cb[b][t];
          const T nv = sub(a[t], mul(g, w));
          a[t] = sel(below, nv, a[t]);
        }
        a[j] = sel(below, g, a[j]);
        if (LU && l == j) {
#pragma unroll
          for (int t = j + 1; t < SBK; ++t) a[t] = mul(a[t], dinv);  // U(j, t)
        }
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_sched_barrier(0);
      }
      if (lane < pb) {
#pragma unroll
        for (int t = 0; t < SBK; ++t)
          if (t < pb && (LU || t <= l)) A[c0 + l][c0 + t] = a[t];
        T dl = zero;  // the diagonal entry, selected with static register indices
#pragma unroll
        for (int t = 0; t < SBK; ++t) dl = sel(t == l, a[t], dl);
        Dv[c0 + l] = dl;
      }
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "workgroup");
      // inverses of the unit triangles: lanes 0..15 column l of X_pp (from L),
      // lanes 16..31 column l of Y_pp (from U^T, i.e. U read transposed)
      if (lane < (LU ? 2 * SBK : SBK)) {
        const bool upper = lane >= SBK;
        T x[SBK];
#pragma unroll
        for (int r = 0; r < SBK; ++r) {
          T s = zero;
#pragma unroll
          for (int t = 0; t < r; ++t) s = fma_(s, upper ? A[c0 + t][c0 + r] : A[c0 + r][c0 + t], x[t]);
          x[r] = sel(r < l, zero, sel(r == l, one, neg(s)));
          __builtin_amdgcn_sched_barrier(0);  // keep each row's loads with it (register pressure)
        }
        if (l < pb) {
#pragma unroll
          for (int r = 0; r < SBK; ++r) {
            if (r < pb && r > l) {  // the unit diagonal is implicit
              if constexpr (LU) {
                if (upper)
                  X[c0 + l][c0 + r] = x[r];  // Y(r, l), stored transposed
                else
                  X[c0 + r][c0 + l] = x[r];
              } else {
                XL(c0 + r, c0 + l) = x[r];
              }
            }
          }
          if (!upper) Di[c0 + l] = recip(Dv[c0 + l]);
        }
      }
    }
    __syncthreads();
    // ---- B: the panel below (and, for LU, the row panel to the right) ----
    const int r1 = c0 + SBK, nr = jb - r1;
    if (nr > 0) {
      const int items = nr * SBK * (LU ? 2 : 1);
      constexpr int NIT = (FB - SBK) * SBK * (LU ? 2 : 1) / 256;  // items per thread at most
      T res[NIT];
#pragma unroll
      for (int it = 0; it < NIT; ++it) {
        const int e = tid + 256 * it;
        res[it] = zero;
        if (e >= items) continue;
        const int side = e / (nr * SBK), f = e % (nr * SBK);
        const int i = r1 + f / SBK, t = f % SBK;
        T s = zero;
        // (unrolled over the 16 terms; the zero triangle of Z contributes 0)
        if (side == 0) {
          // L(i, c0+t) = sum_q A(i, c0+q) Z(t, q) / D_t, Z = X_pp (LDL^T) or Y_pp (LU)
#pragma unroll
          for (int q = 0; q < SBK; ++q) {
            T zq;
            if constexpr (LU)
              zq = X[c0 + q][c0 + t];
            else
              zq = XL(c0 + t, c0 + q);
            const T z = sel(q == t, one, sel(q < t, zq, zero));
            s = fma_(s, A[i][c0 + q], z);
          }
        } else {
          // U(c0+t, i) = D_t^-1 sum_q X_pp(t, q) A(c0+q, i)
          if constexpr (LU) {
#pragma unroll
            for (int q = 0; q < SBK; ++q)
              s = fma_(s, sel(q == t, one, sel(q < t, X[c0 + t][c0 + q], zero)), A[c0 + q][i]);
          }
        }
        res[it] = mul(s, Di[c0 + t]);
      }
      __syncthreads();
#pragma unroll
      for (int it = 0; it < NIT; ++it) {
        const int e = tid + 256 * it;
        if (e >= items) continue;
        const int side = e / (nr * SBK), f = e % (nr * SBK);
        const int i = r1 + f / SBK, t = f % SBK;
        if (side == 0)
          A[i][c0 + t] = res[it];
        else
          A[c0 + t][i] = res[it];
      }
      __syncthreads();
      // ---- C: trailing update, 3 x 3 tiles per thread ----
      const int nt = (nr + 2) / 3;
      for (int e = tid; e < nt * nt; e += blockDim.x) {
        const int ti = e % nt, tj = e / nt;
        const int i0 = r1 + 3 * ti, j0 = r1 + 3 * tj;
        if (!LU && i0 + 2 < j0) continue;  // strictly above the diagonal
        T acc[3][3];
#pragma unroll
        for (int u = 0; u < 3; ++u)
#pragma unroll
          for (int v = 0; v < 3; ++v) acc[u][v] = zero;
#pragma unroll 4
        for (int q = 0; q < SBK; ++q) {
          T li[3], rj[3];
#pragma unroll
          for (int u = 0; u < 3; ++u) {
            const int i = min(i0 + u, FB - 1), j = min(j0 + u, FB - 1);
            li[u] = A[i][c0 + q];
            rj[u] = LU ? A[c0 + q][j] : mul(Dv[c0 + q], A[j][c0 + q]);
          }
          if (LU) {
#pragma unroll
            for (int u = 0; u < 3; ++u) li[u] = mul(li[u], Dv[c0 + q]);
          }
#pragma unroll
          for (int u = 0; u < 3; ++u)
#pragma unroll
            for (int v = 0; v < 3; ++v) acc[u][v] = fma_(acc[u][v], li[u], rj[v]);
        }
#pragma unroll
        for (int u = 0; u < 3; ++u)
#pragma unroll
          for (int v = 0; v < 3; ++v) {
            const int i = i0 + u, j = j0 + v;
            if (i < jb && j < jb && (LU || i >= j)) A[i][j] = sub(A[i][j], acc[u][v]);
          }
      }
      __syncthreads();
    }
  }

  // ---- off-diagonal blocks of the inverse(s), by block rows ----
  for (int I = 1; I < np; ++I) {
    const int ri = I * SBK, nri = min(SBK, jb - ri), ncol = ri;  // block row I, columns [0, ri)
    for (int side = 0; side < (LU ? 2 : 1); ++side) {
      // Tm(r, c) = sum_{t in [c's block start, ri)} Lt(ri + r, t) Z(t, c), with Lt = L (side 0)
      // or U^T (side 1) and Z = X or Y
      for (int e = tid; e < SBK * ncol; e += blockDim.x) {
        const int r = e % SBK, c = e / SBK;
        T s = zero;
        if (r < nri) {
          for (int t0 = (c / SBK) * SBK; t0 < ri; t0 += SBK) {
#pragma unroll
            for (int u = 0; u < SBK; ++u) {
              const int t = t0 + u;
              const T lt = side ? A[t][ri + r] : A[ri + r][t];
              T zt;
              if constexpr (LU)
                zt = side ? X[c][t] : X[t][c];
              else
                zt = XL(t, c);
              const T z = sel(t == c, one, sel(t > c, zt, zero));
              s = fma_(s, lt, z);
            }
          }
        }
        Tm[r][c] = s;
      }
      __syncthreads();
      // Z(ri + r, c) = -sum_{t <= r} Z_II(r, t) Tm(t, c)
      for (int e = tid; e < SBK * ncol; e += blockDim.x) {
        const int r = e % SBK, c = e / SBK;
        if (r >= nri) continue;
        T s = zero;
#pragma unroll
        for (int t = 0; t < SBK; ++t) {
          T zt;
          if constexpr (LU)
            zt = side ? X[ri + t][ri + r] : X[ri + r][ri + t];
          else
            zt = XL(ri + r, ri + t);
          const T z = sel(t == r, one, sel(t < r, zt, zero));
          s = fma_(s, z, Tm[t][c]);
        }
        if constexpr (LU) {
          if (side)
            X[c][ri + r] = neg(s);
          else
            X[ri + r][c] = neg(s);
        } else {
          XL(ri + r, c) = neg(s);
        }
      }
      __syncthreads();
    }
  }

  for (int c = tid; c < jb; c += blockDim.x) dvec[d.first + J + c] = Dv[c];
  T* Xo = inv + d.inv;
  T* Yo = LU ? uinv + d.inv : nullptr;
  for (int e = tid; e < FB * FB; e += blockDim.x) {
    const int r = e & (FB - 1), c = e >> 6;
    if (r >= jb || c >= jb) continue;
    if (r >= c) {
      P[(J + r) + (int64_t)(J + c) * k] = sel(r == c, Dv[c], A[r][c]);
      if (LU) U[(J + r) + (int64_t)(J + c) * k] = sel(r == c, Dv[c], A[c][r]);
    }
    Xo[(J + r) + (int64_t)(J + c) * ns] = sel(r > c, XL(r, c), sel(r == c, one, zero));
    if constexpr (LU) Yo[(J + r) + (int64_t)(J + c) * ns] = sel(r > c, X[c][r], sel(r == c, one, zero));
  }
}

// Half a wave (32 lanes) per W row, eight rows per workgroup: a lane takes
// columns c, c + 32 and c + 64 of each 96-column pass, so a 96-column block
// keeps every lane busy (one wave per row left a third of the lanes idle in
// the second pass) and each contribution row is read with three independent
// loads per lane.
constexpr int kRowLanes = 32, kRowsPerGroup = 256 / kRowLanes, kColsPerLane = 3;

template <typename Ts, typename T>
__global__ __launch_bounds__(256) void solve_fill_kernel(T* __restrict__ W, int64_t wstride, const Ts* __restrict__ src,
                                                         int64_t ldsrc, int64_t sstride, const T* __restrict__ U,
                                                         int64_t ustride, const int32_t* __restrict__ own,
                                                         const int32_t* __restrict__ cbeg,
                                                         const int32_t* __restrict__ cidx, int64_t rows, int p) {
  const int64_t r = (int64_t)blockIdx.x * kRowsPerGroup + (threadIdx.x / kRowLanes);
  if (r >= rows) return;
  const int j = blockIdx.y, lane = threadIdx.x % kRowLanes;
  const int o = own[r], q0 = cbeg[r], q1 = cbeg[r + 1];
  T* wr = W + (int64_t)j * wstride + r * p;
  const Ts* sr = src + (int64_t)j * sstride + (int64_t)(o < 0 ? 0 : o) * ldsrc;
  const T* ub = U + (int64_t)j * ustride;
  for (int c0 = 0; c0 < p; c0 += kRowLanes * kColsPerLane) {
    T acc[kColsPerLane];
    int cc[kColsPerLane];
#pragma unroll
    for (int u = 0; u < kColsPerLane; ++u) {
      const int c = c0 + lane + kRowLanes * u;
      cc[u] = c < p ? c : p - 1;  // loads stay in the row; columns past p are not stored
      acc[u] = o >= 0 ? cvt<T, Ts>(sr[cc[u]]) : ST<T>::zero();
    }
    for (int q = q0; q < q1; ++q) {
      const T* ur = ub + (int64_t)cidx[q] * p;
#pragma unroll
      for (int u = 0; u < kColsPerLane; ++u) acc[u] = add(acc[u], ur[cc[u]]);
    }
#pragma unroll
    for (int u = 0; u < kColsPerLane; ++u)
      if (c0 + lane + kRowLanes * u < p) wr[c0 + lane + kRowLanes * u] = acc[u];
  }
}

// the same layout: half a wave per row of a front's W
template <typename T>
__global__ __launch_bounds__(256) void gather_back_kernel(T* __restrict__ W, const T* __restrict__ Y,
                                                          const T* __restrict__ X, const int32_t* __restrict__ srows,
                                                          const SolveDesc* __restrict__ descs, int p) {
  const SolveDesc d = descs[blockIdx.y];
  const int64_t r = (int64_t)blockIdx.x * kRowsPerGroup + (threadIdx.x / kRowLanes);
  if (r >= d.k) return;
  const int lane = threadIdx.x % kRowLanes;
  T* wr = W + d.w + r * p;
  const bool top = r < d.ns;
  const T dinv = top ? inv_(((const T*)d.dv)[d.first + r]) : ST<T>::one();
  const T* xr = top ? Y + d.xo + (d.first + r) * p : X + d.xo + (int64_t)srows[d.srow + r - d.ns] * p;
  for (int c0 = 0; c0 < p; c0 += kRowLanes * kColsPerLane) {
    T v[kColsPerLane];
#pragma unroll
    for (int u = 0; u < kColsPerLane; ++u) {
      const int c = c0 + lane + kRowLanes * u;
      v[u] = xr[c < p ? c : p - 1];  // loads stay in the row; columns past p are not stored
    }
#pragma unroll
    for (int u = 0; u < kColsPerLane; ++u) {
      const int c = c0 + lane + kRowLanes * u;
      if (c < p) wr[c] = top ? mul(v[u], dinv) : v[u];
    }
  }
}

// one workgroup per column of a front's panel, threads over its k rows
template <typename T>
__global__ __launch_bounds__(256) void stack_kernel(const StackDesc<T>* __restrict__ descs) {
  const StackDesc<T> d = descs[blockIdx.y];
  const int64_t c = blockIdx.x;
  if (c >= d.ns) return;
  const int64_t k = (int64_t)d.ns + d.nb;
  T* dst = d.dst + c * k;
  const T* top = d.top + c * d.ns;
  const T* bot = d.bot + c * d.nb;
  for (int64_t r = threadIdx.x; r < k; r += blockDim.x) dst[r] = r < d.ns ? top[r] : bot[r - d.ns];
}

}  // namespace

template <typename T>
void front_assemble(const PoleBase<T>* pb, int np, const int64_t* dst, const int64_t* src, int64_t n, const double* a,
                    const double* b, hipStream_t s) {
  if (n <= 0 || np <= 0) return;
  hipLaunchKernelGGL(assemble_kernel<T>, dim3((unsigned)((n + 255) / 256), np), dim3(256), 0, s, pb, dst, src, n, a,
                     b);
}

template <typename T>
void front_assemble_cplx(const PoleBase<T>* pb, int np, bool upper, const int64_t* dst, const int64_t* src, int64_t n,
                         const zd* a, const zd* b, hipStream_t s) {
  if (n <= 0 || np <= 0) return;
  hipLaunchKernelGGL(assemble_cplx_kernel<T>, dim3((unsigned)((n + 255) / 256), np), dim3(256), 0, s, pb, upper, dst,
                     src, n, a, b);
}

template <typename T>
void front_extend_add_lu(const PoleBase<T>* pb, int np, const int32_t* pmap, const ExtDesc* d, int nd, int max_nb,
                         hipStream_t s) {
  if (nd <= 0 || max_nb <= 0 || np <= 0) return;
  hipLaunchKernelGGL(extend_add_lu_kernel<T>, dim3(max_nb, nd, np), dim3(256), 0, s, pb, pmap, d);
}

template <typename T>
void front_diag_block_lu(const PoleBase<T>* pb, int np, const DiagDesc* d, int nd, int J, hipStream_t s) {
  if (nd <= 0 || np <= 0) return;
  hipLaunchKernelGGL((diag_blocked_kernel<T, true>), dim3(nd, np), dim3(256), 0, s, pb, d, J);
}

template <typename T>
void front_extend_add(const PoleBase<T>* pb, int np, const int32_t* pmap, const ExtDesc* d, int nd, int max_nb,
                      hipStream_t s) {
  if (nd <= 0 || max_nb <= 0 || np <= 0) return;
  hipLaunchKernelGGL(extend_add_kernel<T>, dim3(max_nb, nd, np), dim3(256), 0, s, pb, pmap, d);
}

template <typename T>
void front_diag_block(const PoleBase<T>* pb, int np, const DiagDesc* d, int nd, int J, hipStream_t s) {
  if (nd <= 0 || np <= 0) return;
  hipLaunchKernelGGL((diag_blocked_kernel<T, false>), dim3(nd, np), dim3(256), 0, s, pb, d, J);
}

template <typename Ts, typename T>
void solve_fill(T* W, int64_t wstride, const Ts* src, int64_t ldsrc, int64_t sstride, const T* U, int64_t ustride,
                const int32_t* own, const int32_t* cbeg, const int32_t* cidx, int64_t rows, int p, int np,
                hipStream_t s) {
  if (rows <= 0 || p <= 0 || np <= 0) return;
  hipLaunchKernelGGL((solve_fill_kernel<Ts, T>), dim3((unsigned)((rows + kRowsPerGroup - 1) / kRowsPerGroup), np),
                     dim3(256), 0, s, W, wstride,
                     src, ldsrc, sstride, U, ustride, own, cbeg, cidx, rows, p);
}

template <typename T>
void solve_gather_back(T* W, const T* Y, const T* X, const int32_t* srows, const SolveDesc* d, int nd, int p,
                       int max_k, hipStream_t s) {
  if (nd <= 0 || max_k <= 0) return;
  hipLaunchKernelGGL(gather_back_kernel<T>, dim3((unsigned)((max_k + kRowsPerGroup - 1) / kRowsPerGroup), nd), dim3(256),
                     0, s, W, Y, X, srows, d, p);
}

template <typename T>
void front_stack(const StackDesc<T>* d, int nd, int64_t max_cols, hipStream_t s) {
  if (nd <= 0 || max_cols <= 0) return;
  hipLaunchKernelGGL(stack_kernel<T>, dim3((unsigned)max_cols, nd), dim3(256), 0, s, d);
}

#define INST(T)                                                                                                      \
  template void front_assemble<T>(const PoleBase<T>*, int, const int64_t*, const int64_t*, int64_t, const double*,   \
                                  const double*, hipStream_t);                                                        \
  template void front_extend_add<T>(const PoleBase<T>*, int, const int32_t*, const ExtDesc*, int, int, hipStream_t);  \
  template void front_assemble_cplx<T>(const PoleBase<T>*, int, bool, const int64_t*, const int64_t*, int64_t,        \
                                       const zd*, const zd*, hipStream_t);                                            \
  template void front_extend_add_lu<T>(const PoleBase<T>*, int, const int32_t*, const ExtDesc*, int, int,             \
                                       hipStream_t);                                                                  \
  template void front_diag_block_lu<T>(const PoleBase<T>*, int, const DiagDesc*, int, int, hipStream_t);             \
  template void front_diag_block<T>(const PoleBase<T>*, int, const DiagDesc*, int, int, hipStream_t);                \
  template void solve_gather_back<T>(T*, const T*, const T*, const int32_t*, const SolveDesc*, int, int, int,        \
                                     hipStream_t);                                                                   \
  template void front_stack<T>(const StackDesc<T>*, int, int64_t, hipStream_t);
INST(zd)
INST(zf)
INST(double)
#undef INST
#define INST_FILL(Ts, T)                                                                                    \
  template void solve_fill<Ts, T>(T*, int64_t, const Ts*, int64_t, int64_t, const T*, int64_t, const int32_t*, \
                                  const int32_t*, const int32_t*, int64_t, int, int, hipStream_t);
INST_FILL(double, zd)
INST_FILL(zd, zd)
INST_FILL(double, zf)
INST_FILL(zd, zf)
#undef INST_FILL

}  // namespace zolo
