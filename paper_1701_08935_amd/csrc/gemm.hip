// Batched matrix product on the CDNA4 matrix cores (see gemm.h for the
// operation).
//
// Tiling: a workgroup computes a TM x TN tile of C (shapes below, chosen per
// launch from the largest M and N of its products); each wave owns a 32-row
// strip of half the tile's columns as 16 x 16 blocks.  The inner dimension
// advances in chunks staged through LDS (real and imaginary parts in separate
// arrays) in two buffers with one barrier per chunk.  Two schedules:
//  * two chunks deep (every tile but the 64 x 96 complex-double one): while
//    chunk c is multiplied out of one buffer, chunk c+1, already in registers,
//    is written to the other and the global loads of chunk c+2 are issued; the
//    staging addresses are computed once per tile;
//  * one chunk deep (64 x 96 complex double, which would spill otherwise): the
//    loads of chunk c+1 are issued before the MFMAs of chunk c and written to
//    the other buffer after them.
// The loop bodies have no branches: out-of-range elements (and chunks past the
// end) read a valid address and are zeroed on their way to LDS, and a short
// last chunk is zero-padded.  Each 16 x 16 x 4 step uses
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
// Both fit two workgroups per CU, so one workgroup's barrier and LDS writes
// overlap the other's MFMAs.  LDS rows are padded to an odd number of elements
// so that both the row-wise fragment reads and the column-wise stores of
// transposed operands spread over all banks.
template <int TM, int TN>
struct TileCfg {
  static constexpr int NT = TM * 4;                          // threads
  static constexpr int TK = (TM == 64 && TN == 96) ? 8 : 16;  // inner chunk
  static constexpr int LDA = TM + 1, LDB = TN + 1;
  static constexpr int NLA = TM * TK / NT, NLB = TN * TK / NT;
  static constexpr int NB = TN / 32;  // 16-column blocks per wave
};

// Main-loop schedule per tile type: the two-deep pipeline keeps a second
// chunk's staging registers live across the MFMAs, which the 64 x 96
// complex-double tile cannot afford without spilling.
template <typename T, int TN>
struct PipelinedLoop {
  static constexpr bool value = !(MfmaTraits<T>::cplx && sizeof(typename MfmaTraits<T>::R) == 8 && TN == 96);
};

// First tile row of tile column j holding an entry i - j >= tri_off (rows i of
// tile row t span [t TM, t TM + TM)): the smallest t with t TM + TM - 1 >= j TN + tri_off.
template <int TM, int TN>
__host__ __device__ inline int tri_first_row(int j, int tri_off, int tilesM) {
  const int need = j * TN + tri_off - (TM - 1);  // t * TM >= need
  const int t = need <= 0 ? 0 : (need + TM - 1) / TM;
  return t < tilesM ? t : tilesM;
}

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
  const int S = d.splitk > 1 ? d.splitk : 1;
  const bool tri = (d.flags & GF_TRI) != 0;
  // Tiles are numbered column by column; a lower-triangular product numbers
  // only the tiles that hold kept entries (rows i with i - j >= tri_off), so
  // no workgroup of the grid is spent on the empty upper part.
  int ntiles = tilesM * tilesN;
  if (tri) {
    ntiles = 0;
    for (int j = 0; j < tilesN; ++j) ntiles += tilesM - tri_first_row<TM, TN>(j, d.tri_off, tilesM);
  }
  if ((int)blockIdx.x >= ntiles * S) return;
  const int tile = blockIdx.x % ntiles, ks = blockIdx.x / ntiles;  // tile, K split
  int m0, n0;
  if (tri) {
    int a = tile, j = 0;
    for (;; ++j) {
      const int i0 = tri_first_row<TM, TN>(j, d.tri_off, tilesM), cnt = tilesM - i0;
      if (a < cnt) {
        m0 = (i0 + a) * TM;
        break;
      }
      a -= cnt;
    }
    n0 = j * TN;
  } else {
    m0 = (tile % tilesM) * TM;
    n0 = (tile / tilesM) * TN;
  }

  // two LDS buffers as separate arrays, so the compiler can tell the chunk
  // being read from the one being written: [plane][k][row]
  __shared__ R As0[NP][TK][C::LDA], As1[NP][TK][C::LDA];
  __shared__ R Bs0[NP][TK][C::LDB], Bs1[NP][TK][C::LDB];

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

  // inner range: all of K, or the nonzero part of a triangular opA; a split
  // takes its share of the chunks
  int kbeg = 0, kend = d.K;
  if (d.flags & GF_ALOW) kend = min(d.K, m0 + TM);
  if (d.flags & GF_AUP) kbeg = m0;
  if (d.flags & GF_BLOW) kbeg = max(kbeg, n0);
  if (S > 1) {
    const int ctot = kend > kbeg ? (kend - kbeg + TK - 1) / TK : 0;
    const int c0 = (int)((int64_t)ks * ctot / S), c1 = (int)((int64_t)(ks + 1) * ctot / S);
    const int kb = kbeg + c0 * TK;
    kend = min(kend, kbeg + c1 * TK);
    kbeg = kb;
  }
  const int nchunk = kend > kbeg ? (kend - kbeg + TK - 1) / TK : 0;
  const bool has_dk = d.dk != nullptr;

  // MFMAs of one chunk held in (As, Bs); a short last chunk is zero-padded
  auto compute = [&](const R* As, const R* Bs) {
#pragma unroll
    for (int kk = 0; kk < TK / 4; ++kk) {
      const int k = 4 * kk + lk;
      R are[2], aim[2], bre[NB], bim[NB];
#pragma unroll
      for (int a = 0; a < 2; ++a) {
        are[a] = As[k * C::LDA + wm + 16 * a + li];
        if constexpr (CPLX) aim[a] = As[TK * C::LDA + k * C::LDA + wm + 16 * a + li];
      }
#pragma unroll
      for (int b = 0; b < NB; ++b) {
        bre[b] = Bs[k * C::LDB + wn + 16 * b + li];
        if constexpr (CPLX) bim[b] = Bs[TK * C::LDB + k * C::LDB + wn + 16 * b + li];
      }
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
  };

  if constexpr (PipelinedLoop<T, TN>::value) {
    // Staging geometry, fixed for the whole loop: element q of this thread is
    // (row or column, k offset) of every chunk; consecutive threads read
    // consecutive addresses.  The global address of a chunk at k0 is the
    // thread's base plus k0 times a uniform step.
    const T* pa[NLA];
    int at[NLA], la[NLA];
    bool arow[NLA];
#pragma unroll
    for (int q = 0; q < NLA; ++q) {
      const int e = tid + NT * q;
      const int i = ta ? e / TK : e % TM, t = ta ? e % TK : e / TM;
      arow[q] = m0 + i < d.M;
      at[q] = t;
      la[q] = t * C::LDA + i;
      pa[q] = ta ? d.A + t + (int64_t)(m0 + i) * d.lda : d.A + (m0 + i) + (int64_t)t * d.lda;
    }
    const T* pb[NLB];
    int bt[NLB], lb[NLB];
    bool bcol[NLB];
#pragma unroll
    for (int q = 0; q < NLB; ++q) {
      const int e = tid + NT * q;
      const int j = tb ? e % TN : e / TK, t = tb ? e / TN : e % TK;
      bcol[q] = n0 + j < d.N;
      bt[q] = t;
      lb[q] = t * C::LDB + j;
      pb[q] = tb ? d.B + (n0 + j) + (int64_t)t * d.ldb : d.B + t + (int64_t)(n0 + j) * d.ldb;
    }
    const int64_t sa = ta ? 1 : d.lda, sb = tb ? d.ldb : 1;

    // Global loads of a chunk go straight into registers; out-of-range elements
    // (and chunks past the end) read the first element instead and are zeroed
    // when written to LDS, so the loop body has no branches.
    T ra[NLA], rb[NLB], rd[NLA];
    auto gload = [&](int k0) {
      const int64_t oa = (int64_t)k0 * sa, ob = (int64_t)k0 * sb;
#pragma unroll
      for (int q = 0; q < NLA; ++q) {
        const bool ok = arow[q] && at[q] + k0 < kend;
        ra[q] = gld(ok ? pa[q] + oa : d.A);
        if (has_dk) rd[q] = gld(d.dk + (ok ? k0 + at[q] : 0));
      }
#pragma unroll
      for (int q = 0; q < NLB; ++q) {
        const bool ok = bcol[q] && bt[q] + k0 < kend;
        rb[q] = gld(ok ? pb[q] + ob : d.B);
      }
    };
    auto sstore = [&](R* As, R* Bs, int k0) {
#pragma unroll
      for (int q = 0; q < NLA; ++q) {
        const bool ok = arow[q] && at[q] + k0 < kend;
        T v = ok ? ra[q] : ST<T>::zero();
        if (ca) v = conj_(v);
        if (has_dk) v = mul(v, rd[q]);
        R re, im = 0;
        split<T>(v, &re, &im);
        As[la[q]] = re;
        if constexpr (CPLX) As[TK * C::LDA + la[q]] = im;
      }
#pragma unroll
      for (int q = 0; q < NLB; ++q) {
        const bool ok = bcol[q] && bt[q] + k0 < kend;
        T v = ok ? rb[q] : ST<T>::zero();
        if (cb) v = conj_(v);
        R re, im = 0;
        split<T>(v, &re, &im);
        Bs[lb[q]] = re;
        if constexpr (CPLX) Bs[TK * C::LDB + lb[q]] = im;
      }
    };
    // Software pipeline, two chunks deep: while chunk c is multiplied out of
    // one buffer, chunk c+1 (already in registers) is written to the other
    // and the loads of chunk c+2 are issued.  One barrier per chunk.
    if (nchunk > 0) {
      gload(kbeg);
      sstore(&As0[0][0][0], &Bs0[0][0][0], kbeg);
      gload(kbeg + TK);
    }
    __syncthreads();
    for (int c = 0; c < nchunk; c += 2) {
      const int k0 = kbeg + c * TK;
      sstore(&As1[0][0][0], &Bs1[0][0][0], k0 + TK);
      gload(k0 + 2 * TK);
      compute(&As0[0][0][0], &Bs0[0][0][0]);
      __syncthreads();
      if (c + 1 >= nchunk) break;
      sstore(&As0[0][0][0], &Bs0[0][0][0], k0 + 2 * TK);
      gload(k0 + 3 * TK);
      compute(&As1[0][0][0], &Bs1[0][0][0]);
      __syncthreads();
    }
  } else {
    // Staging geometry: element q of this thread is (row or column, k offset)
    // within every chunk, consecutive threads reading consecutive addresses;
    // recomputed per chunk (a few integer ops) rather than kept in registers.
    auto ageo = [&](int q, int* i, int* t) {
      const int e = tid + NT * q;
      *i = ta ? e / TK : e % TM;
      *t = ta ? e % TK : e / TM;
    };
    auto bgeo = [&](int q, int* t, int* j) {
      const int e = tid + NT * q;
      *j = tb ? e % TN : e / TK;
      *t = tb ? e / TN : e % TK;
    };

    T ra[NLA], rb[NLB], rd[NLA];
    auto gload = [&](int k0) {
#pragma unroll
      for (int q = 0; q < NLA; ++q) {
        int i, t;
        ageo(q, &i, &t);
        const int gi = m0 + i, gt = k0 + t;
        const bool ok = gi < d.M && gt < kend;
        const int64_t off = ta ? gt + (int64_t)gi * d.lda : gi + (int64_t)gt * d.lda;
        ra[q] = gld(d.A + (ok ? off : 0));
        if (has_dk) rd[q] = gld(d.dk + (ok ? gt : 0));
      }
#pragma unroll
      for (int q = 0; q < NLB; ++q) {
        int t, j;
        bgeo(q, &t, &j);
        const int gj = n0 + j, gt = k0 + t;
        const bool ok = gj < d.N && gt < kend;
        const int64_t off = tb ? gj + (int64_t)gt * d.ldb : gt + (int64_t)gj * d.ldb;
        rb[q] = gld(d.B + (ok ? off : 0));
      }
    };
    auto sstore = [&](R* As, R* Bs, int k0) {
#pragma unroll
      for (int q = 0; q < NLA; ++q) {
        int i, t;
        ageo(q, &i, &t);
        const bool ok = m0 + i < d.M && k0 + t < kend;
        T v = ok ? ra[q] : ST<T>::zero();
        if (ca) v = conj_(v);
        if (has_dk) v = mul(v, rd[q]);
        R re, im = 0;
        split<T>(v, &re, &im);
        As[t * C::LDA + i] = re;
        if constexpr (CPLX) As[TK * C::LDA + t * C::LDA + i] = im;
      }
#pragma unroll
      for (int q = 0; q < NLB; ++q) {
        int t, j;
        bgeo(q, &t, &j);
        const bool ok = n0 + j < d.N && k0 + t < kend;
        T v = ok ? rb[q] : ST<T>::zero();
        if (cb) v = conj_(v);
        R re, im = 0;
        split<T>(v, &re, &im);
        Bs[t * C::LDB + j] = re;
        if constexpr (CPLX) Bs[TK * C::LDB + t * C::LDB + j] = im;
      }
    };
    // One chunk ahead: the loads of chunk c+1 are issued before the MFMAs of
    // chunk c and written to the other buffer after them (fewer registers
    // live across the MFMAs, for the widest complex tile).
    if (nchunk > 0) {
      gload(kbeg);
      sstore(&As0[0][0][0], &Bs0[0][0][0], kbeg);
    }
    __syncthreads();
    for (int c = 0; c < nchunk; ++c) {
      const int k0 = kbeg + c * TK;
      R* curA = (c & 1) ? &As1[0][0][0] : &As0[0][0][0];
      R* curB = (c & 1) ? &Bs1[0][0][0] : &Bs0[0][0][0];
      R* nxtA = (c & 1) ? &As0[0][0][0] : &As1[0][0][0];
      R* nxtB = (c & 1) ? &Bs0[0][0][0] : &Bs1[0][0][0];
      if (c + 1 < nchunk) gload(k0 + TK);
      compute(curA, curB);
      if (c + 1 < nchunk) sstore(nxtA, nxtB, k0 + TK);
      __syncthreads();
    }
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
void launch_cfg(const GemmDesc<T>* d_desc, int n, int maxM, int maxN, hipStream_t s, int tag, int max_split,
                int grid_tiles) {
  const int per = grid_tiles > 0 ? grid_tiles : ((maxM + TM - 1) / TM) * ((maxN + TN - 1) / TN);
  const int tiles = per * (max_split > 1 ? max_split : 1);
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

// The tag is part of the interface so that a use class can get shapes of its
// own; every class shares these today.
int gemm_tile_m(int, int, int) { return 64; }
int gemm_tile_n(int, int maxN, int) { return (maxN > 64 && maxN <= 96) ? 96 : 64; }
int gemm_tile_k(int maxM, int maxN, int tag) { return gemm_tile_n(maxM, maxN, tag) == 96 ? 8 : 16; }
int gemm_tiles(int maxM, int maxN, int tag) {
  const int tm = gemm_tile_m(maxM, maxN, tag), tn = gemm_tile_n(maxM, maxN, tag);
  return ((maxM + tm - 1) / tm) * ((maxN + tn - 1) / tn);
}
int64_t gemm_part_elems(int maxM, int maxN, int tag, bool cplx) {
  return (int64_t)gemm_tile_m(maxM, maxN, tag) * gemm_tile_n(maxM, maxN, tag) * (cplx ? 2 : 1);
}
int gemm_desc_tiles(int M, int N, int flags, int tri_off, int maxM, int maxN, int tag) {
  const int tn = gemm_tile_n(maxM, maxN, tag);
  const int tilesM = (M + 63) / 64, tilesN = (N + tn - 1) / tn;
  if (!(flags & GF_TRI)) return tilesM * tilesN;
  int n = 0;
  for (int j = 0; j < tilesN; ++j)
    n += tilesM - (tn == 64 ? tri_first_row<64, 64>(j, tri_off, tilesM) : tri_first_row<64, 96>(j, tri_off, tilesM));
  return n;
}

template <typename T>
void gemm_batched(const GemmDesc<T>* d_desc, int n, int maxM, int maxN, hipStream_t s, int tag, int max_split,
                  int grid_tiles) {
  if (n <= 0 || maxM <= 0 || maxN <= 0) return;
  if (gemm_tile_n(maxM, maxN, tag) == 64)
    launch_cfg<T, 64, 64>(d_desc, n, maxM, maxN, s, tag, max_split, grid_tiles);
  else
    launch_cfg<T, 64, 96>(d_desc, n, maxM, maxN, s, tag, max_split, grid_tiles);
}

template <typename T>
__global__ void gemm_desc_series_kernel(GemmDesc<T> base, int count, int64_t a_step, int64_t b_step, int64_t c_step,
                                        int64_t kchunk, int64_t ktotal, GemmDesc<T>* out) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= count) return;
  GemmDesc<T> d = base;
  d.A += q * a_step;
  d.B += q * b_step;
  d.C += q * c_step;
  const int64_t k0 = q * kchunk;
  d.K = (int)(ktotal - k0 < kchunk ? ktotal - k0 : kchunk);
  out[q] = d;
}

template <typename T>
void gemm_desc_series(const GemmDesc<T>& base, int count, int64_t a_step, int64_t b_step, int64_t c_step,
                      int64_t kchunk, int64_t ktotal, GemmDesc<T>* out, hipStream_t s) {
  if (count <= 0) return;
  hipLaunchKernelGGL(gemm_desc_series_kernel<T>, dim3((count + 63) / 64), dim3(64), 0, s, base, count, a_step, b_step,
                     c_step, kchunk, ktotal, out);
}

template void gemm_batched<double>(const GemmDesc<double>*, int, int, int, hipStream_t, int, int, int);
template void gemm_batched<zd>(const GemmDesc<zd>*, int, int, int, hipStream_t, int, int, int);
template void gemm_batched<zf>(const GemmDesc<zf>*, int, int, int, hipStream_t, int, int, int);
#define ZOLO_SERIES(T)                                                                                         \
  template void gemm_desc_series<T>(const GemmDesc<T>&, int, int64_t, int64_t, int64_t, int64_t, int64_t, GemmDesc<T>*, \
                                    hipStream_t);
ZOLO_SERIES(double)
ZOLO_SERIES(zd)
ZOLO_SERIES(zf)
#undef ZOLO_SERIES

}  // namespace zolo
