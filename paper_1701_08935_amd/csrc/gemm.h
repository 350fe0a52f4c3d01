// Batched dense matrix product used by the factorization, the solves, the
// block Arnoldi process and Rayleigh-Ritz.
//
//   C(i,j) = s(i) Cin(i,j) + alpha * sum_t opA(i,t) * dk(t) * opB(t,j)
//
// with s(i) = beta, or crs(i) (row scale), or 1/crs(i) (flag GF_CRS_INV);
// with GF_CRS_ACC the row scale multiplies the product instead:
//   C(i,j) = beta Cin(i,j) + r(i) alpha sum_t ...;
// opA/opB optionally transposed / conjugated; C and Cin column-major with
// leading dimensions ldc/ldcin, or row-major with GF_TRANSC.  GF_TRI keeps
// only entries with i - j >= tri_off (lower-triangular updates of symmetric
// fronts).  GF_ALOW / GF_AUP declare opA lower / upper trapezoidal
// (opA(i,t) = 0 for t > i, resp. t < i; those entries are stored as zeros):
// each row tile then runs its inner loop only over the nonzero part, which
// halves the work of products with an explicit triangular inverse, square or
// stacked on a dense panel; GF_BLOW does the same for a lower trapezoidal opB
// (opB(t,j) = 0 for t < j; each column tile starts its inner loop at its
// first column).  One descriptor per independent product; a launch covers a
// list.
#pragma once

#include "dev_common.h"

namespace zolo {

enum GemmFlags {
  GF_TRANSA = 1,
  GF_TRANSB = 2,
  GF_TRANSC = 4,
  GF_CONJA = 8,
  GF_CONJB = 16,
  GF_TRI = 32,
  GF_CRS_INV = 64,
  GF_CRS = 128,
  GF_ALOW = 256,
  GF_AUP = 512,
  GF_CRS_ACC = 1024,  // the row scale (crs or 1/crs) multiplies the product instead of Cin
  GF_BLOW = 2048,     // opB lower trapezoidal: column j sums over t >= j only
};

template <typename T>
struct GemmDesc {
  const T* A;
  const T* B;
  T* C;
  const T* Cin;  // may equal C; null when beta == 0 and no row scale
  const T* dk;   // inner-dimension scale (length K), may be null
  const T* crs;  // row scale of Cin (GF_CRS / GF_CRS_INV), may be null
  // Split of the inner dimension (splitk > 1): the product is computed by
  // splitk workgroups per tile over consecutive K ranges; each writes its
  // partial sums to part (splitk * tiles * gemm_part_elems(maxM, maxN) real
  // scalars) and bumps cnt[tile] (zero before the launch, reset to zero by
  // the workgroup that arrives last); that one adds the partials in split
  // order, so the result does not depend on arrival order, and applies the
  // epilogue.
  void* part;
  int* cnt;
  int splitk;
  int64_t lda, ldb, ldc, ldcin;
  int M, N, K;
  int tri_off;
  int flags;
  T alpha, beta;
};

// Tile shape the launcher picks for a launch of tag `tag` whose products are
// at most maxM x maxN: 64 rows; 96 columns when maxN is in (64, 96], else 64.
int gemm_tile_m(int maxM, int maxN, int tag);
int gemm_tile_n(int maxM, int maxN, int tag);
int gemm_tile_k(int maxM, int maxN, int tag);  // inner chunk of that shape
// workgroups of one maxM x maxN product (per split) in such a launch
int gemm_tiles(int maxM, int maxN, int tag);
// real scalars of partial sums one split of one tile writes
int64_t gemm_part_elems(int maxM, int maxN, int tag, bool cplx);
// workgroups (per split) one M x N descriptor needs in a launch with bounds
// maxM x maxN: its tiles, or only those holding kept entries for GF_TRI
int gemm_desc_tiles(int M, int N, int flags, int tri_off, int maxM, int maxN, int tag);

// d_desc: device array of n descriptors; maxM / maxN: upper bounds of every
// descriptor's M and N (they size the grid and select the tile shape);
// max_split: largest splitk of the descriptors; grid_tiles: the largest
// gemm_desc_tiles of the descriptors (0: the tiles of maxM x maxN).
// tag: 0 front updates, 1 supernodal solves, 2 Krylov / Rayleigh-Ritz (profile names only).
template <typename T>
void gemm_batched(const GemmDesc<T>* d_desc, int n, int maxM, int maxN, hipStream_t s, int tag, int max_split = 1,
                  int grid_tiles = 0);

// Writes count descriptors to the device array out, in stream order on s:
// descriptor q is base with A, B and C advanced by q * a_step, q * b_step and
// q * c_step elements and K = min(kchunk, ktotal - q * kchunk).  base travels
// as a kernel argument, so nothing on the host has to outlive the call and the
// caller need not wait for the copy.  count <= 1024.
template <typename T>
void gemm_desc_series(const GemmDesc<T>& base, int count, int64_t a_step, int64_t b_step, int64_t c_step,
                      int64_t kchunk, int64_t ktotal, GemmDesc<T>* out, hipStream_t s);

// Algorithmic work of one descriptor: entries of C computed and flops
// (8 per complex multiply-add, 2 per real one), and the bytes a product
// must move at least once: A, B, C written, Cin read.
template <typename T>
inline void gemm_work(const GemmDesc<T>& d, double* flops, double* bytes) {
  double M = d.M, N = d.N, K = d.K;
  double ent = M * N;
  if (d.flags & GF_TRI) {
    ent = 0.0;
    for (int j = 0; j < d.N; ++j) {
      int i0 = j + d.tri_off;
      if (i0 < 0) i0 = 0;
      if (i0 < d.M) ent += (double)(d.M - i0);
    }
  }
  const double fm = ST<T>::cplx ? 8.0 : 2.0;
  // nonzeros of an R x K operand whose row r holds min(r + 1, K) entries (lower)
  // or max(K - r, 0) entries (upper)
  auto nz_lower = [](double R, double KK) { return R <= KK ? R * (R + 1.0) / 2.0 : KK * (KK + 1.0) / 2.0 + (R - KK) * KK; };
  auto nz_upper = [](double R, double KK) {
    const double r = R < KK ? R : KK;
    return r * KK - r * (r - 1.0) / 2.0;
  };
  if (d.flags & GF_BLOW) {
    const double nzb = nz_upper(N, K);  // column j of opB sums over t >= j
    *flops += fm * M * nzb;
    *bytes += (double)sizeof(T) * (M * K + nzb + ent * (d.Cin ? 2.0 : 1.0));
    return;
  }
  if (d.flags & (GF_ALOW | GF_AUP)) {
    const double nza = (d.flags & GF_ALOW) ? nz_lower(M, K) : nz_upper(M, K);
    *flops += fm * N * nza;
    *bytes += (double)sizeof(T) * (nza + K * N + ent * (d.Cin ? 2.0 : 1.0));
    return;
  }
  *flops += fm * ent * K;
  *bytes += (double)sizeof(T) * (M * K + K * N + ent * (d.Cin ? 2.0 : 1.0));
}

}  // namespace zolo
