// Internal declarations shared by the host code of the library.
#pragma once

#include <cstddef>
#include <cstdint>
#include <cstdio>
#include <string>
#include <vector>

#include "../../include/zolo.h"

namespace zolo {

void set_error(const char* fmt, ...);

int plan_filter(double am, double ap, double bm, double bp, int r1, int r2, double eps, zolo_filter_coeffs* out,
                char* err, size_t errlen);

// ---------------------------------------------------------------------------
// Symbolic analysis (multifrontal method, Sec. 2.3 pre-factorization phase).
// Vertices are renumbered by nested dissection in post-order, so the
// vertices of a front are a contiguous range [first, first + ns) and all its
// off-diagonal rows ("struct") belong to ancestors (indices >= first + ns).
// ---------------------------------------------------------------------------
struct Front {
  int32_t first = 0;
  int32_t ns = 0;          // fully summed (eliminated) variables
  int32_t nb = 0;          // rows of the update (contribution) block
  int32_t parent = -1;
  int32_t level = 0;       // height: leaves 0
  int64_t struct_off = 0;  // into Symbolic::struct_rows, nb entries
  int32_t child_begin = 0; // into Symbolic::children
  int32_t child_count = 0;
  int64_t asm_begin = 0, asm_end = 0;  // into asm_entry / asm_pos
};

struct Symbolic {
  int64_t n = 0;
  std::vector<int32_t> perm;   // perm[new] = old
  std::vector<int32_t> iperm;  // iperm[old] = new
  std::vector<Front> fronts;   // post-order
  std::vector<int32_t> struct_rows;  // concatenated struct lists (new indices, ascending)
  std::vector<int32_t> parent_map;   // per struct entry: local row in the parent front
  std::vector<int32_t> children;
  std::vector<std::vector<int32_t>> levels;  // front ids by height
  // permuted CSR (new ordering); psrc[e_new] = e_old
  std::vector<int64_t> prow;
  std::vector<int32_t> pcol;
  std::vector<int64_t> psrc;
  // assembly of original entries: lower-triangle entries of each front's columns
  std::vector<int64_t> asm_entry;  // entry index in the permuted CSR
  std::vector<int64_t> asm_pos;    // row_local + col_local * k in the front panel
  // figures
  int64_t panel_entries = 0;   // sum k * ns
  int64_t inv_entries = 0;     // sum ns * ns
  int64_t update_entries = 0;  // sum nb * nb
  int64_t struct_total = 0;    // sum nb
  int64_t max_front = 0;
  int max_children = 0;
  double flops = 0.0;          // real flops of one complex factorization (with the L11^-1 blocks)
  double elim_flops = 0.0;     // the elimination alone (complex LDL^T: sum over fronts of 8 (k^3 - nb^3) / 6)
};

// Build the symbolic structure.  grid may be null.  Returns ZOLO_OK or an error code.
int symbolic_analyze(int64_t n, const int64_t* rowptr, const int32_t* colind, const int32_t* grid, int leaf_size,
                     Symbolic* S);

// For the serving loop: device bytes one query needs at most (factors of r1
// poles, solve program, Krylov basis of maxit block steps, subspace blocks);
// a deep copy of a result.
// zolo_solve with resident factors of the same filter (F_in, used and kept by
// the caller) or, with F_in null and F_keep non-null, handing the new
// factorization to the caller instead of freeing it (serving loop)
zolo_status solve_resident(zolo_ctx* ctx, zolo_pencil* P, double a, double b, int n_lambda_est,
                           const zolo_opts* opts, const double* d_Q0, void* stream, zolo_factors* F_in,
                           zolo_factors** F_keep, zolo_result** out);
int64_t factors_bytes(const zolo_factors* F);
// drops the solve programs and the Krylov workspace, keeping the factors (a
// resident factorization holds only what its bytes count)
void factors_keep_only(zolo_factors* F);
// the calling thread's cap on the shifts zolo_inertia factors together (0 = none)
void set_inertia_cap(int shifts);
// device bytes of one real-shift factorization of the inertia count
int64_t inertia_shift_bytes(const zolo_pencil* P);
int plan_contour(int kind, double a, double b, int npole, zolo_filter_coeffs* out, char* err, size_t errlen);
int64_t query_bytes_estimate(const zolo_pencil* P, int r1, int nss, int maxit, int restart, int precision,
                             int block_cols);
int64_t pencil_n(const zolo_pencil* P);
bool pencil_cplx(const zolo_pencil* P);
zolo_result* result_clone(const zolo_result* r);
// device bytes of a result's vectors
int64_t result_bytes(const zolo_result* r);
// max over the result's pairs of the residual norm of zolo_residuals, on stream s
zolo_status result_verify(zolo_pencil* P, const zolo_result* r, void* s, double* worst);
// marks a copy handed out from a resident subspace: its max_resid recomputed
// now, t_total the time of that check
void result_mark_reused(zolo_result* r, double max_resid, double t_check);
// a stream the library created: its release events may be queried until
// retire_stream (which synchronizes it) is called before it is destroyed
void register_stream(void* s);
void retire_stream(void* s);
// the seeded Gaussian start block zolo_solve draws, written on the device (n doubles)
void gaussian_device(uint64_t seed, int64_t n, double* d_out, void* stream);

}  // namespace zolo
