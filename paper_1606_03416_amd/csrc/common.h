// Internal declarations shared by the library's translation units (gfx950).
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_bf16.h>

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/chefsi.h"

namespace chefsi {

// ---------------------------------------------------------------- errors
void set_error(const std::string& msg);
int fail(int code, const std::string& msg);

#define CHEFSI_HIP(call)                                                              \
  do {                                                                                \
    hipError_t e_ = (call);                                                           \
    if (e_ != hipSuccess)                                                             \
      return ::chefsi::fail(CHEFSI_ERR_HIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

#define CHEFSI_LAUNCHED(what)                                                         \
  do {                                                                                \
    hipError_t e_ = hipGetLastError();                                                \
    if (e_ != hipSuccess)                                                             \
      return ::chefsi::fail(CHEFSI_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e_)); \
  } while (0)

#define CHEFSI_TRY(expr)               \
  do {                                 \
    int r_ = (expr);                   \
    if (r_ != CHEFSI_OK) return r_;    \
  } while (0)

// ---------------------------------------------------------------- sizes
constexpr int kMaxJ = 256;          // largest ALB count per element supported
constexpr int kMaxLanczos = 64;     // largest Lanczos step count
#ifndef CHEFSI_STEP_KC
#define CHEFSI_STEP_KC 16
#endif
constexpr int kStepKC = CHEFSI_STEP_KC;  // reduction rows of an element padded to this (FP64/FP32 chunks)
constexpr int kPadK = 32;           // reduction rows of an element padded to this (BF16 chunk)

__host__ __device__ inline int64_t round_up(int64_t v, int64_t m) { return (v + m - 1) / m * m; }
__host__ __device__ inline int64_t ceil_div(int64_t v, int64_t m) { return (v + m - 1) / m; }

// ---------------------------------------------------------------- plan
struct Plan {
  int nx = 0, ny = 0, nz = 0, stencil = 0, M = 0;
  int64_t N = 0;
  int64_t h_elems = 0;      // block-list layout size
  int64_t panel_elems = 0;  // internal packed panel size (elements)
  int64_t kmap_len = 0;
  int maxJ = 0, maxRB = 0;
  bool uniform = true;
  int device = 0;
  std::vector<int32_t> J, nbr, ktot, kpad, rb;
  std::vector<int64_t> rowoff, hoff, poff, koff;
  // device tables
  int32_t* d_J = nullptr;       // [M]
  int32_t* d_nbr = nullptr;     // [M*S]
  int32_t* d_rb = nullptr;      // [M] row blocks (ceil(J/16))
  int32_t* d_kpad = nullptr;    // [M] reduction rows padded to kPadK
  int32_t* d_order = nullptr;   // [M] element processing order, grouped by row-block count
  // launch groups of the step kernels: elements order[start .. start+count)
  // all have rb row blocks (one group for uniform plans)
  std::vector<int> grp_rb, grp_start, grp_count;
  int64_t* d_rowoff = nullptr;  // [M+1]
  int64_t* d_hoff = nullptr;    // [M*S] block offsets in block-list layout
  int64_t* d_poff = nullptr;    // [M] panel offsets (elements)
  int64_t* d_koff = nullptr;    // [M] kmap offsets
  int32_t* d_kmap = nullptr;    // [sum kpad] global row of each reduction row (-1 pad)
  int32_t* d_kslot = nullptr;   // [sum kpad] (slot << 8 | row-in-slot) of each reduction row
  // BF16 filter: multivectors in 8-row tiles whose element row ranges are
  // padded to multiples of 8 (zero rows), so every 8 consecutive reduction
  // rows of a neighbour segment are one tile, contiguous per state.
  int64_t N8 = 0;               // padded row count (state stride)
  int64_t panel8_elems = 0;     // BF16 panel size (elements)
  std::vector<int64_t> rowoff8, poff8, kgoff;
  std::vector<int32_t> kpad8;
  int64_t* d_rowoff8 = nullptr; // [M+1] padded row offsets
  int64_t* d_poff8 = nullptr;   // [M] BF16 panel offsets
  int32_t* d_kpad8 = nullptr;   // [M] padded reduction rows, multiple of kPadK
  int64_t* d_kgoff = nullptr;   // [M] offsets into d_kg8
  int32_t* d_kg8 = nullptr;     // [sum kpad8/8] 8-row tile of each reduction-row group (-1 pad)
  int32_t* d_rowsrc8 = nullptr; // [N8] source row of each padded row (-1 padding)
  // element blocks J_K x J_K (density-matrix blocks, basis overlaps), row-major,
  // back to back: element K's block starts at sqoff[K]; sqtot = sum_K J_K^2
  std::vector<int64_t> sqoff;
  int64_t sqtot = 0;
  int64_t* d_sqoff = nullptr;   // [M+1]
  void* rocblas = nullptr;      // rocblas_handle for the dense eigensolver
  void* scratch = nullptr;      // this device's address of the library's static scratch array (or null)
  size_t eig_ws_cache_n = 0, eig_ws_cache_bytes = 0, eig_ws_cache_roc = 0;
};

inline Plan* P(chefsi_plan p) { return reinterpret_cast<Plan*>(p); }

// ---------------------------------------------------------------- workspace carving
struct Carver {
  char* base;
  size_t cap, used = 0;
  bool dry;
  Carver(void* b, size_t c) : base(static_cast<char*>(b)), cap(c), dry(b == nullptr) {}
  template <typename T>
  T* take(int64_t count) {
    size_t bytes = static_cast<size_t>(round_up(static_cast<int64_t>(count * sizeof(T)), 256));
    size_t off = used;
    used += bytes;
    if (dry) return nullptr;
    return reinterpret_cast<T*>(base + off);
  }
  bool ok() const { return dry || used <= cap; }
};

// ---------------------------------------------------------------- kernels (launchers)
// All launchers enqueue on `st` and return a chefsi_status.
int launch_set_bounds(double a, double b, double a0, double* d_bounds, hipStream_t st);
int launch_cheb_coef(const double* d_bounds, int m, double* d_coef, hipStream_t st);
int launch_const_coef(double alpha, double c, double* d_coef, hipStream_t st);
int launch_const_coef3(double alpha, double beta, double c, double* d_coef, hipStream_t st);

// Repack H (block-list, fp64) into per-element transposed panels of type dtype.
// transpose_h = true packs H^T (uses the opposite slot of each neighbour).
// BF16 panels use the 8-padded reduction rows and 32-row chunks (panel8_elems).
// d_shift (device, may be null) is subtracted from the diagonal of the self
// block; used for BF16 panels, which carry H - cI.
int launch_repack(const Plan& p, const double* d_H, int dtype, bool transpose_h, void* d_panel,
                  hipStream_t st, const double* d_shift = nullptr);

// One Chebyshev step / SpMM: out = alpha_k (H*in - c*in) - beta_k*prev on all
// element rows, columns [0, ns). coef points at (alpha, beta, c) of this step.
// in/prev/out element types follow dtype (F64: double; F32: float; BF16: bf16),
// except out_f64 forces a float64 output and in_f64/prev_f64 a float64 input.
struct StepIO {
  const void* in; int64_t ldi; bool in_f64;
  const void* prev; int64_t ldp; bool prev_f64;   // prev may be null
  void* out; int64_t ldo; bool out_f64;
  bool shifted = false;   // no c*in term: out = alpha*(panel*in) - beta*prev (the panel carries H - cI, or c = 0)
};
int launch_step(const Plan& p, const void* d_panel, int dtype, const double* d_coef,
                const StepIO& io, int ns, hipStream_t st);
// BF16 step on 8-row-tiled buffers (rows padded per element to multiples of
// 8; element (row, state j) at ((row/8)*ns + j)*8 + row%8), with a panel that
// carries H - cI: out = alpha*(panel*in) - beta*prev.  in/prev bf16; out bf16
// tiled, or float64 row-major (ldo) when out_f64.  split: every buffer holds
// hi and lo halves (lo at N8*ns elements on, the lo panel at panel8_elems on)
// and each product takes three BF16 MFMAs.
int launch_step_b16(const Plan& p, const void* d_panel8, const double* d_coef, const void* in, const void* prev,
                    void* out, bool out_f64, int64_t ldo, int ns, hipStream_t st, bool split = false);
// float64 row-major X (ldx) -> bf16 8-row tiles with zero padding rows (split:
// also the lo halves, N8*ns elements after the hi ones).
int launch_to_tiles_b16(const Plan& p, const double* X, int64_t ldx, void* out, int ns, hipStream_t st,
                        bool split = false);
// Residual partials: part[K*ns + j] = sum_{i in K} (H x_j - theta_j x_j)_i^2 (fp64).
int launch_resid_partial(const Plan& p, const void* d_panel, const double* d_X, int64_t ldx,
                         const double* d_theta, int ns, double* d_part, hipStream_t st);
int launch_colsum_sqrt(const double* d_part, int rows, int ns, double* d_out, hipStream_t st);

// Conversions / copies of N x ns multivectors.
int launch_convert(const double* src, int64_t lds, void* dst, int dst_dtype, int64_t ldd,
                   int64_t n, int ns, hipStream_t st);
int launch_copy_f64(const double* src, int64_t lds, double* dst, int64_t ldd, int64_t n, int ns,
                    hipStream_t st);

// Dense FP64 kernels (dense.hip).
// C(m x n) = alpha * A^T B + beta * C, A (k x m, lda), B (k x n, ldb), row-major.
// upper_only: compute only tiles on/above the diagonal (symmetric results).
// kmin: fewest reduction rows per split-K part (splits fill the chip when the
// result has few tiles; the partial sums need d_split_ws).
int gemm_tn(int64_t m, int64_t n, int64_t k, double alpha, const double* A, int64_t lda,
            const double* B, int64_t ldb, double beta, double* C, int64_t ldc, bool upper_only,
            double* d_split_ws, size_t split_ws_elems, hipStream_t st, int64_t kmin = 1024);
// C(m x n) = alpha * A B + beta * C, A (m x k, lda), B (k x n, ldb), row-major.
// b_upper: B is upper triangular (its zero part is skipped).  skip_if
// (device, 3 ints, may be null): if any is nonzero when the kernel runs, C is
// left untouched (status words of earlier steps of the same stream).
int gemm_nn(int64_t m, int64_t n, int64_t k, double alpha, const double* A, int64_t lda,
            const double* B, int64_t ldb, double beta, double* C, int64_t ldc, hipStream_t st,
            bool b_upper = false, const int* skip_if = nullptr);
// Upper triangle (j >= i) of a row-major n x n C += alpha (A1 B1^T + A2 B2^T),
// the four operands n x k row-major with stride ld; entries below the
// diagonal are not touched.
int syr2k_upper(int64_t n, int64_t k, double alpha, const double* A1, const double* B1, const double* A2,
                const double* B2, int64_t ld, double* C, int64_t ldc, hipStream_t st);
// T = U^{-1} for an upper triangular n x n U (T upper triangular); W is
// scratch of (n/2 + 64)^2 doubles.
int upper_inverse(const double* U, int n, double* T, double* W, hipStream_t st);
size_t gemm_tn_split_ws_elems(int64_t m, int64_t n, int64_t k, int64_t kmin = 1024);
// mode 0: (A + A^T)/2; 1: upper -> lower; 2: lower -> upper.
int launch_symmetrize(double* A, int64_t lda, int n, int mode, hipStream_t st);
// d_scr: device scratch of at least min(n, 64)^2 doubles.
int cholesky_upper(double* S, int64_t lds, int n, int* d_status, double* d_scr, hipStream_t st);
// Upper bound on the 2-norm condition number of the column-equilibrated block
// from its Cholesky factor U and T = U^{-1} (n x n, row-major, upper parts
// used); d_scr holds cholqr_cond_scratch_elems(n) doubles; d_out 1 double.
size_t cholqr_cond_scratch_elems(int n);
int cholqr_cond_bound(const double* U, const double* T, int n, double* d_scr, double* d_out, hipStream_t st);
int trsm_right_upper(double* Y, int64_t ldy, int64_t nrows, const double* U, int64_t ldu, int n,
                     hipStream_t st);
// Solve X L = Y in place (L lower triangular, n x n row-major).
int trsm_right_lower(double* Y, int64_t ldy, int64_t nrows, const double* L, int64_t ldl, int n,
                     hipStream_t st);
// Hbar_{K;s} += alpha * (*d_alpha if non-null) * A[K rows] B[K'_s rows]^T for every stored block.
int sddmm_accumulate(const Plan& p, const double* A, int64_t lda, const double* B, int64_t ldb, int ns,
                     double alpha, const double* d_alpha, double* d_Hbar, hipStream_t st);
// rcoef[3j..] = (alpha_j, beta_{j+1} (0 for j = m-1), c): coefficients of the reverse sweep.
int launch_rev_coef(const double* d_coef, int m, double* d_rcoef, hipStream_t st);
// out[0] = sum_{i<k} v[i]
int launch_sum_first(const double* d_v, int k, double* d_out, hipStream_t st);
int launch_fill(double* d, int64_t count, double v, hipStream_t st);
int launch_fill_int(int* d, int64_t count, int v, hipStream_t st);
int trmm_upper_upper(const double* A, const double* B, double* C, int n, hipStream_t st);
int launch_eigvec_fix(const double* Vcm, int64_t ldv, int n, double* Q, int64_t ldq,
                      hipStream_t st);
// B[c][r] = A[r][c] * (row_scale ? row_scale[r] : 1)
int launch_transpose(const double* A, int64_t lda, double* B, int64_t ldb, int rows, int cols,
                     hipStream_t st, const double* row_scale = nullptr);

// Eigensolver (eig.hip)
int eig_workspace_bytes(Plan& p, int n, size_t* bytes);
// *d_info: 0 ok, > 0 the tridiagonal solver failed, -1 A was not finite.
// skip (device, 3 ints, may be null): if any is set, the identity is solved
// instead of A (a failed earlier step; the caller reports it).
int eig_sym(Plan& p, double* A, int64_t lda, int n, double* d_w, double* d_E, int* d_info, double* Z,
            void* d_ws, size_t ws_bytes, hipStream_t st, const int* skip = nullptr);
// Householder tridiagonalisation (tridiag.hip), LAPACK lower format
size_t tridiag_scratch_bytes(int n);
int tridiag_lower(double* A, int64_t lda, int n, double* D, double* E, double* tau, void* scratch,
                  hipStream_t st);
// Back-transformation (backtr.hip): out = Q C for the reflectors of
// tridiag_lower in A and tau; C (n x n column-major, leading dimension n, the
// eigenvectors of T) is overwritten; out is column-major with leading
// dimension ldo and may be A itself.
size_t backtr_scratch_bytes(int n);
int backtr_lower(const double* A, int64_t lda, int n, const double* tau, double* C, double* out, int64_t ldo,
                 void* scratch, size_t scratch_bytes, hipStream_t st);

// Lanczos (lanczos.hip)
size_t lanczos_ws_bytes(const Plan& p, int k);
int lanczos_bounds(const Plan& p, const void* d_panel64, const double* d_v0, int k,
                   const double* d_ritz_prev, int ns, double* d_bounds, void* ws, size_t ws_bytes,
                   hipStream_t st);
// d_bounds = (a, b, a0) with b = d_bounds_src[1] and a, a0 from the ascending
// Ritz values (largest, smallest; a0 separated from a as in chefsi_bounds).
int launch_warm_bounds(const double* d_ritz, int ns, const double* d_bounds_src, double* d_bounds,
                       hipStream_t st);
// *d_status = 1 if the bounds (a, b, a0) are not finite, 2 if a0 < a < b fails.
int launch_check_bounds(const double* d_bounds, int* d_status, hipStream_t st);

// Steps around the cycle (post.hip).
// Fermi level mu (sum_i f_i = n_occ) by bisection and occupations f (device).
int launch_fermi(const double* d_theta, int ns, double n_occ, double kT, double* d_f, double* d_mu,
                 hipStream_t st);
// Slices the element products split a reduction of length L into; the
// partial buffer of elem_nt holds elem_nt_slices(p, L) * p.sqtot doubles.
int elem_nt_slices(const Plan& p, int64_t L);
// C_K = A_K diag(w) B_K^T for every element (J_K x J_K, reduction over L
// columns; A_K = rows rowoff[K].. of A with row stride lda; w may be null);
// sym: B = A and C symmetric (only the upper part computed, then mirrored).
// Result in d_out at sqoff[K]; d_part is the slice scratch.
int elem_nt(const Plan& p, const double* A, int64_t lda, const double* B, int64_t ldb, const double* w,
            int64_t L, bool sym, double* d_part, double* d_out, hipStream_t st);
// X_K <- R_K X_K in place for every element (R_K at d_R + sqoff[K]).
int elem_apply(const Plan& p, const double* d_R, double* X, int64_t ldx, int ns, hipStream_t st);

}  // namespace chefsi
