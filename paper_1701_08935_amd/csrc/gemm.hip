// Batched tiled matrix product (LDS tiles of 64 x 16, 4 x 4 outputs per
// thread).  See gemm.h for the operation.
#include "gemm.h"

namespace zolo {

namespace {

constexpr int TK = 16;

template <typename T, bool CONJ>
__device__ inline T maybe_conj(T x) {
  if constexpr (CONJ) return conj_(x);
  return x;
}

template <typename T>
__global__ __launch_bounds__(256) void gemm_batched_kernel(const GemmDesc<T>* __restrict__ descs) {
  const GemmDesc<T> d = descs[blockIdx.y];
  const int tilesM = (d.M + GEMM_TILE - 1) / GEMM_TILE;
  const int tilesN = (d.N + GEMM_TILE - 1) / GEMM_TILE;
  const int tile = blockIdx.x;
  if (tile >= tilesM * tilesN) return;
  const int m0 = (tile % tilesM) * GEMM_TILE;
  const int n0 = (tile / tilesM) * GEMM_TILE;
  const bool tri = (d.flags & GF_TRI) != 0;
  if (tri && (m0 + GEMM_TILE - 1) - n0 < d.tri_off) return;

  __shared__ T As[TK][GEMM_TILE + 1];
  __shared__ T Bs[TK][GEMM_TILE + 1];

  const int tid = threadIdx.x;
  const int tx = tid % 16, ty = tid / 16;
  T acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = ST<T>::zero();

  const bool ta = (d.flags & GF_TRANSA) != 0, tb = (d.flags & GF_TRANSB) != 0;
  const bool ca = (d.flags & GF_CONJA) != 0, cb = (d.flags & GF_CONJB) != 0;

  for (int k0 = 0; k0 < d.K; k0 += TK) {
    // A tile: 64 rows x 16 inner
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      int e = tid + 256 * q;
      int i, t;
      if (!ta) {
        i = e % GEMM_TILE;
        t = e / GEMM_TILE;
      } else {
        i = e / TK;
        t = e % TK;
      }
      int gi = m0 + i, gt = k0 + t;
      T v = ST<T>::zero();
      if (gi < d.M && gt < d.K) {
        v = ta ? d.A[gt + (int64_t)gi * d.lda] : d.A[gi + (int64_t)gt * d.lda];
        if (ca) v = conj_(v);
        if (d.dk) v = mul(v, d.dk[gt]);
      }
      As[t][i] = v;
    }
    // B tile: 16 inner x 64 cols
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      int e = tid + 256 * q;
      int t, j;
      if (!tb) {
        t = e % TK;
        j = e / TK;
      } else {
        j = e % GEMM_TILE;
        t = e / GEMM_TILE;
      }
      int gj = n0 + j, gt = k0 + t;
      T v = ST<T>::zero();
      if (gj < d.N && gt < d.K) {
        v = tb ? d.B[gj + (int64_t)gt * d.ldb] : d.B[gt + (int64_t)gj * d.ldb];
        if (cb) v = conj_(v);
      }
      Bs[t][j] = v;
    }
    __syncthreads();
#pragma unroll
    for (int t = 0; t < TK; ++t) {
      T ar[4], br[4];
#pragma unroll
      for (int a = 0; a < 4; ++a) ar[a] = As[t][tx + 16 * a];
#pragma unroll
      for (int b = 0; b < 4; ++b) br[b] = Bs[t][ty + 16 * b];
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = fma_(acc[a][b], ar[a], br[b]);
    }
    __syncthreads();
  }

  const bool tc = (d.flags & GF_TRANSC) != 0;
  const bool use_crs = (d.flags & (GF_CRS | GF_CRS_INV)) != 0;
  const bool crs_inv = (d.flags & GF_CRS_INV) != 0;
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    int i = m0 + tx + 16 * a;
    if (i >= d.M) continue;
    T s = d.beta;
    if (use_crs) s = crs_inv ? inv_(d.crs[i]) : d.crs[i];
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      int j = n0 + ty + 16 * b;
      if (j >= d.N) continue;
      if (tri && i - j < d.tri_off) continue;
      T out = mul(d.alpha, acc[a][b]);
      if (d.Cin) {
        T cin = tc ? d.Cin[(int64_t)i * d.ldcin + j] : d.Cin[i + (int64_t)j * d.ldcin];
        out = fma_(out, s, cin);
      }
      if (tc)
        d.C[(int64_t)i * d.ldc + j] = out;
      else
        d.C[i + (int64_t)j * d.ldc] = out;
    }
  }
}

}  // namespace

template <typename T>
void gemm_batched(const GemmDesc<T>* d_desc, int n, int max_tiles, hipStream_t s) {
  if (n <= 0 || max_tiles <= 0) return;
  for (int b0 = 0; b0 < n; b0 += 65535) {
    int nb = n - b0 < 65535 ? n - b0 : 65535;
    hipLaunchKernelGGL(gemm_batched_kernel<T>, dim3(max_tiles, nb), dim3(256), 0, s, d_desc + b0);
  }
}

template void gemm_batched<double>(const GemmDesc<double>*, int, int, hipStream_t);
template void gemm_batched<zd>(const GemmDesc<zd>*, int, int, hipStream_t);
template void gemm_batched<zf>(const GemmDesc<zf>*, int, int, hipStream_t);

}  // namespace zolo
