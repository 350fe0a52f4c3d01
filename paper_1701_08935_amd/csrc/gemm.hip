// Batched matrix product on the CDNA4 matrix cores (see gemm.h for the
// operation).
//
// Tiling: a workgroup computes a TM x TN tile of C (shapes below, chosen per
// launch from the largest M and N of its products); each wave owns a 32-row
// strip of half the tile's columns as 16 x 16 blocks.  The inner dimension
// advances in chunks staged through LDS (real and imaginary parts in separate
// arrays), double-buffered: the global loads of chunk c+1 are issued into
// registers before the MFMAs of chunk c and written to the other LDS buffer
// after them, with one barrier per chunk.  Each 16 x 16 x 4 step uses
// v_mfma_f64_16x16x4_f64 (double, complex double) or v_mfma_f32_16x16x4_f32
// (complex float); a complex product is four real ones:
//   Cre += Are Bre - Aim Bim,  Cim += Are Bim + Aim Bre.
// Fragment layout of the 16x16x4 instructions (lane l of 64, checked on the
// device):
//   A(i, k): i = l % 16, k = l / 16;  B(k, j): j = l % 16, k = l / 16;
//   D(i, j): j = l % 16 and, for accumulator value v = 0..3,
//            i = l / 16 + 4 v      (f64 instruction)
//            i = 4 (l / 16) + v    (f32 instruction).
#include "gemm.h"

namespace zolo {

namespace {

template <typename T>
struct MfmaTraits;
template <>
struct MfmaTraits<double> {
  typedef double R;
  typedef double __attribute__((ext_vector_type(4))) V4;
  static constexpr bool cplx = false;
  __device__ static inline int row(int lk, int v) { return lk + 4 * v; }
};
template <>
struct MfmaTraits<zd> {
  typedef double R;
  typedef double __attribute__((ext_vector_type(4))) V4;
  static constexpr bool cplx = true;
  __device__ static inline int row(int lk, int v) { return lk + 4 * v; }
};
template <>
struct MfmaTraits<zf> {
  typedef float R;
  typedef float __attribute__((ext_vector_type(4))) V4;
  static constexpr bool cplx = true;
  __device__ static inline int row(int lk, int v) { return 4 * lk + v; }
};

__device__ inline MfmaTraits<double>::V4 mfma(double a, double b, MfmaTraits<double>::V4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ inline MfmaTraits<zf>::V4 mfma(float a, float b, MfmaTraits<zf>::V4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

template <typename T>
__device__ inline void split(const T& v, typename MfmaTraits<T>::R* re, typename MfmaTraits<T>::R* im);
template <>
__device__ inline void split<double>(const double& v, double* re, double* im) {
  *re = v;
  (void)im;
}
template <>
__device__ inline void split<zd>(const zd& v, double* re, double* im) {
  *re = v.re;
  *im = v.im;
}
template <>
__device__ inline void split<zf>(const zf& v, float* re, float* im) {
  *re = v.re;
  *im = v.im;
}

// Tile shapes (TM x TN per workgroup, TM/32 x 2 waves, each wave 32 x TN/2 as
// 2 x TN/32 blocks of 16 x 16):
//   64 x 64  : 256 threads, TK 16
//   64 x 96  : 256 threads, TK 8  (N in (64, 96], e.g. a 96-column block)
// Both fit two or more workgroups per CU, so one workgroup's barrier and LDS
// writes overlap the other's MFMAs.  LDS rows are padded to an odd number of elements so that both the row-wise
// fragment reads and the column-wise stores of transposed operands spread over
// all banks.
template <int TM, int TN>
struct TileCfg {
  static constexpr int NT = TM * 4;                          // threads
  static constexpr int TK = (TM == 64 && TN == 96) ? 8 : 16;  // inner chunk
  static constexpr int LDA = TM + 1, LDB = TN + 1;
  static constexpr int NLA = TM * TK / NT, NLB = TN * TK / NT;
  static constexpr int NB = TN / 32;  // 16-column blocks per wave
};

// TAG only separates the uses in profiles: 0 front updates, 1 supernodal
// solves, 2 Krylov / Rayleigh-Ritz products.
template <typename T, int TAG, int TM, int TN>
__global__ __launch_bounds__((TM * 4), 2) void gemm_batched_kernel(
    const GemmDesc<T>* __restrict__ descs) {
  typedef typename MfmaTraits<T>::R R;
  typedef typename MfmaTraits<T>::V4 V4;
  typedef TileCfg<TM, TN> C;
  constexpr bool CPLX = MfmaTraits<T>::cplx;
  constexpr int NP = CPLX ? 2 : 1;  // real planes
  constexpr int TK = C::TK, NT = C::NT, NLA = C::NLA, NLB = C::NLB, NB = C::NB;
  static_assert(NLA * NT == TM * TK && NLB * NT == TN * TK, "staging must cover the chunk");

  const GemmDesc<T> d = descs[blockIdx.y];
  const int tilesM = (d.M + TM - 1) / TM;
  const int tilesN = (d.N + TN - 1) / TN;
  const int ntiles = tilesM * tilesN;
  const int S = d.splitk > 1 ? d.splitk : 1;
  if ((int)blockIdx.x >= ntiles * S) return;
  const int tile = blockIdx.x % ntiles, ks = blockIdx.x / ntiles;  // tile, K split
  const int m0 = (tile % tilesM) * TM;
  const int n0 = (tile / tilesM) * TN;
  const bool tri = (d.flags & GF_TRI) != 0;
  if (tri && (m0 + TM - 1) - n0 < d.tri_off) return;

  // [buffer][plane][k][row]: double-buffered chunks
  __shared__ R As[2][NP][TK][C::LDA];
  __shared__ R Bs[2][NP][TK][C::LDB];

  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int wm = (wave % (TM / 32)) * 32, wn = (wave / (TM / 32)) * (TN / 2);
  const int li = lane & 15, lk = lane >> 4;

  const bool ta = (d.flags & GF_TRANSA) != 0, tb = (d.flags & GF_TRANSB) != 0;
  const bool ca = (d.flags & GF_CONJA) != 0, cb = (d.flags & GF_CONJB) != 0;

  V4 acc[NP][2][NB];
#pragma unroll
  for (int q = 0; q < NP; ++q)
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < NB; ++b) acc[q][a][b] = V4{0, 0, 0, 0};

  // element e of a TM x TK (A) or TK x TN (B) chunk, laid out so that
  // consecutive threads read consecutive addresses
  auto a_idx = [&](int e, int* i, int* t) {
    if (!ta) {
      *i = e % TM;
      *t = e / TM;
    } else {
      *i = e / TK;
      *t = e % TK;
    }
  };
  auto b_idx = [&](int e, int* t, int* j) {
    if (!tb) {
      *t = e % TK;
      *j = e / TK;
    } else {
      *j = e % TN;
      *t = e / TN;
    }
  };

  // inner range: all of K, or the nonzero part of a triangular opA
  int kbeg = 0, kend = d.K;
  if (d.flags & GF_ALOW) kend = min(d.K, m0 + TM);
  if (d.flags & GF_AUP) kbeg = m0;
  const bool has_dk = d.dk != nullptr;

  // Global loads of a chunk go straight into registers: out-of-range elements
  // read the (valid) first element instead and are zeroed when the chunk is
  // written to LDS, so no load waits on a branch and all of them are in
  // flight together while the MFMAs of the previous chunk run.
  T ra[NLA], rb[NLB], rd[NLA];
  auto gload = [&](int k0) {
#pragma unroll
    for (int q = 0; q < NLA; ++q) {
      int i, t;
      a_idx(tid + NT * q, &i, &t);
      const int gi = m0 + i, gt = k0 + t;
      const bool ok = gi < d.M && gt < kend;
      ra[q] = gld(ok ? (ta ? d.A + gt + (int64_t)gi * d.lda : d.A + gi + (int64_t)gt * d.lda) : d.A);
      if (has_dk) rd[q] = gld(d.dk + (ok ? gt : 0));
    }
#pragma unroll
    for (int q = 0; q < NLB; ++q) {
      int t, j;
      b_idx(tid + NT * q, &t, &j);
      const int gj = n0 + j, gt = k0 + t;
      const bool ok = gj < d.N && gt < kend;
      rb[q] = gld(ok ? (tb ? d.B + gj + (int64_t)gt * d.ldb : d.B + gt + (int64_t)gj * d.ldb) : d.B);
    }
  };
  auto sstore = [&](int buf, int k0) {
#pragma unroll
    for (int q = 0; q < NLA; ++q) {
      int i, t;
      a_idx(tid + NT * q, &i, &t);
      const bool ok = m0 + i < d.M && k0 + t < kend;
      T v = ok ? ra[q] : ST<T>::zero();
      if (ca) v = conj_(v);
      if (has_dk) v = mul(v, rd[q]);
      R re, im = 0;
      split<T>(v, &re, &im);
      As[buf][0][t][i] = re;
      if constexpr (CPLX) As[buf][NP - 1][t][i] = im;
    }
#pragma unroll
    for (int q = 0; q < NLB; ++q) {
      int t, j;
      b_idx(tid + NT * q, &t, &j);
      const bool ok = n0 + j < d.N && k0 + t < kend;
      T v = ok ? rb[q] : ST<T>::zero();
      if (cb) v = conj_(v);
      R re, im = 0;
      split<T>(v, &re, &im);
      Bs[buf][0][t][j] = re;
      if constexpr (CPLX) Bs[buf][NP - 1][t][j] = im;
    }
  };

  if (S > 1) {  // this split's share of the chunks
    const int ctot = kend > kbeg ? (kend - kbeg + TK - 1) / TK : 0;
    const int c0 = (int)((int64_t)ks * ctot / S), c1 = (int)((int64_t)(ks + 1) * ctot / S);
    const int kb = kbeg + c0 * TK;
    kend = min(kend, kbeg + c1 * TK);
    kbeg = kb;
  }
  const int nchunk = kend > kbeg ? (kend - kbeg + TK - 1) / TK : 0;
  if (nchunk > 0) {
    gload(kbeg);
    sstore(0, kbeg);
  }
  __syncthreads();
  for (int c = 0; c < nchunk; ++c) {
    const int k0 = kbeg + c * TK;
    const int buf = c & 1;
    if (c + 1 < nchunk) gload(k0 + TK);  // in flight during this chunk's MFMAs
    const int ksteps = min(TK, kend - k0);  // a short last chunk skips its empty steps
#pragma unroll
    for (int kk = 0; kk < TK / 4; ++kk) {
      if (4 * kk >= ksteps) break;
      const int k = 4 * kk + lk;
      R are[2], aim[2], bre[NB], bim[NB];
#pragma unroll
      for (int a = 0; a < 2; ++a) {
        are[a] = As[buf][0][k][wm + 16 * a + li];
        if constexpr (CPLX) aim[a] = As[buf][NP - 1][k][wm + 16 * a + li];
      }
#pragma unroll
      for (int b = 0; b < NB; ++b) {
        bre[b] = Bs[buf][0][k][wn + 16 * b + li];
        if constexpr (CPLX) bim[b] = Bs[buf][NP - 1][k][wn + 16 * b + li];
      }
      // independent accumulators within each group, so dependent MFMAs are spaced
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < NB; ++b) acc[0][a][b] = mfma(are[a], bre[b], acc[0][a][b]);
      if constexpr (CPLX) {
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
          for (int b = 0; b < NB; ++b) acc[1][a][b] = mfma(are[a], bim[b], acc[1][a][b]);
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
          for (int b = 0; b < NB; ++b) acc[0][a][b] = mfma(-aim[a], bim[b], acc[0][a][b]);
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
          for (int b = 0; b < NB; ++b) acc[1][a][b] = mfma(aim[a], bre[b], acc[1][a][b]);
      }
    }
    if (c + 1 < nchunk) sstore(buf ^ 1, k0 + TK);
    __syncthreads();  // buf^1 is written; every wave is done reading buf
  }

  if (S > 1) {
    // Partial sums in fragment order: value q of thread tid at q * NT + tid.
    constexpr int NV = NP * 2 * NB * 4;
    R* P = (R*)d.part;
    const int64_t tstride = (int64_t)NV * NT;
    R* mine = P + ((int64_t)tile * S + ks) * tstride;
#pragma unroll
    for (int q = 0; q < NP; ++q)
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < NB; ++b)
#pragma unroll
          for (int v = 0; v < 4; ++v) gst(mine + (int64_t)(((q * 2 + a) * NB + b) * 4 + v) * NT + tid, acc[q][a][b][v]);
    __threadfence();  // partials visible device-wide before the arrival count
    __syncthreads();
    __shared__ int last_s;
    if (tid == 0) last_s = atomicAdd(d.cnt + tile, 1) == S - 1;
    __syncthreads();
    if (!last_s) return;
    __threadfence();  // see every split's partials
#pragma unroll
    for (int q = 0; q < NP; ++q)
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < NB; ++b) acc[q][a][b] = V4{0, 0, 0, 0};
    for (int sp = 0; sp < S; ++sp) {  // fixed order: independent of which split came last
      const R* src = P + ((int64_t)tile * S + sp) * tstride;
#pragma unroll
      for (int q = 0; q < NP; ++q)
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
          for (int b = 0; b < NB; ++b)
#pragma unroll
            for (int v = 0; v < 4; ++v) acc[q][a][b][v] += gld(src + (int64_t)(((q * 2 + a) * NB + b) * 4 + v) * NT + tid);
    }
    if (tid == 0) d.cnt[tile] = 0;  // ready for the next launch
  }

  // Epilogue.  All loads (row scales, Cin) are issued before any of them is
  // used, so their latency is paid once per tile.
  const bool tc = (d.flags & GF_TRANSC) != 0;
  const bool use_crs = (d.flags & (GF_CRS | GF_CRS_INV)) != 0;
  const bool crs_inv = (d.flags & GF_CRS_INV) != 0;
  const bool crs_acc = (d.flags & GF_CRS_ACC) != 0;
  const bool has_cin = d.Cin != nullptr;
  T rs[2][4], cv[2][4][NB];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int i = m0 + wm + 16 * a + MfmaTraits<T>::row(lk, v);
      const bool iok = i < d.M;
      if (use_crs) rs[a][v] = gld(d.crs + (iok ? i : 0));
      if (has_cin) {
#pragma unroll
        for (int b = 0; b < NB; ++b) {
          const int j = n0 + wn + 16 * b + li;
          const bool ok = iok && j < d.N;
          cv[a][v][b] = gld(ok ? (tc ? d.Cin + (int64_t)i * d.ldcin + j : d.Cin + i + (int64_t)j * d.ldcin) : d.Cin);
        }
      }
    }
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int i = m0 + wm + 16 * a + MfmaTraits<T>::row(lk, v);
      if (i >= d.M) continue;
      T s = d.beta, ra = d.alpha;
      if (use_crs) {
        const T r = crs_inv ? inv_(rs[a][v]) : rs[a][v];
        if (crs_acc)
          ra = mul(ra, r);
        else
          s = r;
      }
#pragma unroll
      for (int b = 0; b < NB; ++b) {
        const int j = n0 + wn + 16 * b + li;
        if (j >= d.N) continue;
        if (tri && i - j < d.tri_off) continue;
        T accv;
        if constexpr (CPLX)
          accv = T{acc[0][a][b][v], acc[1][a][b][v]};
        else
          accv = acc[0][a][b][v];
        T out = mul(ra, accv);
        if (has_cin) out = fma_(out, s, cv[a][v][b]);
        gst(tc ? d.C + (int64_t)i * d.ldc + j : d.C + i + (int64_t)j * d.ldc, out);
      }
    }
}

template <typename T, int TM, int TN>
void launch_cfg(const GemmDesc<T>* d_desc, int n, int maxM, int maxN, hipStream_t s, int tag, int max_split) {
  const int tiles = ((maxM + TM - 1) / TM) * ((maxN + TN - 1) / TN) * (max_split > 1 ? max_split : 1);
  const dim3 blk(TileCfg<TM, TN>::NT);
  for (int b0 = 0; b0 < n; b0 += 65535) {
    const int nb = n - b0 < 65535 ? n - b0 : 65535;
    if (tag == 0)
      hipLaunchKernelGGL((gemm_batched_kernel<T, 0, TM, TN>), dim3(tiles, nb), blk, 0, s, d_desc + b0);
    else if (tag == 1)
      hipLaunchKernelGGL((gemm_batched_kernel<T, 1, TM, TN>), dim3(tiles, nb), blk, 0, s, d_desc + b0);
    else
      hipLaunchKernelGGL((gemm_batched_kernel<T, 2, TM, TN>), dim3(tiles, nb), blk, 0, s, d_desc + b0);
  }
}

}  // namespace

int gemm_tile_m(int) { return 64; }
int gemm_tile_n(int maxN) { return (maxN > 64 && maxN <= 96) ? 96 : 64; }
int gemm_tiles(int maxM, int maxN) {
  const int tm = gemm_tile_m(maxM), tn = gemm_tile_n(maxN);
  return ((maxM + tm - 1) / tm) * ((maxN + tn - 1) / tn);
}
int64_t gemm_part_elems(int maxN, bool cplx) { return (int64_t)64 * gemm_tile_n(maxN) * (cplx ? 2 : 1); }

template <typename T>
void gemm_batched(const GemmDesc<T>* d_desc, int n, int maxM, int maxN, hipStream_t s, int tag, int max_split) {
  if (n <= 0 || maxM <= 0 || maxN <= 0) return;
  if (gemm_tile_n(maxN) == 64)
    launch_cfg<T, 64, 64>(d_desc, n, maxM, maxN, s, tag, max_split);
  else
    launch_cfg<T, 64, 96>(d_desc, n, maxM, maxN, s, tag, max_split);
}

template void gemm_batched<double>(const GemmDesc<double>*, int, int, int, hipStream_t, int, int);
template void gemm_batched<zd>(const GemmDesc<zd>*, int, int, int, hipStream_t, int, int);
template void gemm_batched<zf>(const GemmDesc<zf>*, int, int, int, hipStream_t, int, int);

}  // namespace zolo
