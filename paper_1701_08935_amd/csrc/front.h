// Multifrontal kernels: front assembly, extend-add, diagonal-block
// factorization and inversion, the stacking of each front's solve panel, and
// the row gathers / extend-adds of the supernodal triangular solves.
#pragma once

#include "dev_common.h"

namespace zolo {

constexpr int FB = 64;  // block size of the blocked partial factorization
constexpr int FOB = 256;  // outer block of the trailing updates (a multiple of FB)

// One extend-add: child contribution block (nb_c x nb_c, column-major, lower
// triangle) into the parent front (panel k_p x ns_p col-major + update block
// nb_p x nb_p col-major), rows mapped by pmap.
struct ExtDesc {
  int64_t child_upd;  // element offset of the child's update block
  int64_t pmap;       // offset into the parent-map array (nb_c entries)
  int64_t par_panel;  // element offset of the parent panel
  int64_t par_upd;    // element offset of the parent update block
  int32_t nb_c, k_p, ns_p, pad;
};

struct DiagDesc {
  int64_t panel;  // element offset of the panel (k x ns, col-major, ld k)
  int64_t inv;    // element offset of the ns x ns inverse block (ld ns)
  int32_t k, ns, first, pad;
};

// Solve: per front RHS block W (k x p row-major), contributions U (nb x p).
struct SolveDesc {
  const void* dv;  // pivots D of this solve's factor (the backward gather scales by D^-1)
  int64_t w;       // element offset of W in the level's W buffer
  int64_t u;       // element offset of U in the U buffer (global over fronts)
  int64_t srow;    // offset into struct_rows
  int64_t xo;      // element offset of this solve's blocks in X and Y
  int32_t first, ns, nb, k;
};

// A pole's arrays for the factorization kernels, which run one step for a
// batch of poles at once (the pole is the last grid dimension; pb is a device
// array of np entries): its panels, diagonal-block inverses, pivots, update
// blocks, breakdown flag and shift sigma = sr + i si.
template <typename T>
struct PoleBase {
  T* panel;
  T* upanel;  // LU only
  T* inv;
  T* uinv;    // LU only
  T* dvec;
  T* upd;
  int* flag;
  double sr, si;
};

// assembly: panel[dst[e]] = a[src[e]] - sigma * b[src[e]]  (real pencil values)
template <typename T>
void front_assemble(const PoleBase<T>* pb, int np, const int64_t* dst, const int64_t* src, int64_t n, const double* a,
                    const double* b, hipStream_t s);

template <typename T>
void front_extend_add(const PoleBase<T>* pb, int np, const int32_t* pmap, const ExtDesc* d, int nd, int max_nb,
                      hipStream_t s);

// Factor the FB x FB (or smaller) diagonal block at step J of each listed front,
// write L (unit lower, strictly lower part), D (into dvec at first + J + c and the
// panel diagonal) and the inverse of the unit lower block into the inverse array;
// a zero pivot sets the pole's flag.
template <typename T>
void front_diag_block(const PoleBase<T>* pb, int np, const DiagDesc* d, int nd, int J, hipStream_t s);

// LU fronts of complex Hermitian pencils (no pivoting).  Each front keeps an
// L panel (k x ns: the front's lower part) and a U panel of the same layout
// holding the transpose of its upper part, so L, U^T, their diagonal-block
// inverses and D are laid out as in the LDL^T case.  upper: assemble into the
// U panels.
template <typename T>
void front_assemble_cplx(const PoleBase<T>* pb, int np, bool upper, const int64_t* dst, const int64_t* src, int64_t n,
                         const zd* a, const zd* b, hipStream_t s);
template <typename T>
void front_extend_add_lu(const PoleBase<T>* pb, int np, const int32_t* pmap, const ExtDesc* d, int nd, int max_nb,
                         hipStream_t s);
template <typename T>
void front_diag_block_lu(const PoleBase<T>* pb, int np, const DiagDesc* d, int nd, int J, hipStream_t s);

// Forward right-hand sides of one level for np solves at once.  Row r of the
// level's W (its fronts' k x p blocks one after the other, row-major; solve j
// at j * wstride) = right-hand-side row own[r] (converted to T; zero where
// own[r] < 0, the border rows) plus the children's update rows
// cidx[cbeg[r]] .. cidx[cbeg[r+1] - 1] of U (solve j at j * ustride), added in
// that order.  src: solve j at j * sstride (0: one right-hand side for all).
template <typename Ts, typename T>
void solve_fill(T* W, int64_t wstride, const Ts* src, int64_t ldsrc, int64_t sstride, const T* U, int64_t ustride,
                const int32_t* own, const int32_t* cbeg, const int32_t* cidx, int64_t rows, int p, int np,
                hipStream_t s);
// Backward right-hand side of each front, into W (k x p, row-major):
// rows [0, ns): D^-1 Y[first + r]; rows [ns, k): X[struct_rows[srow + r - ns]].
template <typename T>
void solve_gather_back(T* W, const T* Y, const T* X, const int32_t* struct_rows, const SolveDesc* d, int nd, int p,
                       int max_k, hipStream_t s);

// Solve panel of a front, stacked in place of its factor panel (k x ns,
// col-major, ld k): rows [0, ns) <- top (ns x ns, ld ns), rows [ns, k) <- bot
// (nb x ns, ld nb).
template <typename T>
struct StackDesc {
  T* dst;
  const T* top;
  const T* bot;
  int32_t ns, nb;
};
template <typename T>
void front_stack(const StackDesc<T>* d, int nd, int64_t max_cols, hipStream_t s);  // max_cols: largest ns

}  // namespace zolo
