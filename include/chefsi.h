/*
 * chefsi.h -- C ABI of the MI355X (gfx950) DG-CheFSI hot-path library.
 *
 * The library runs one cycle of Chebyshev-filtered subspace iteration
 * (Algorithm 1 of Banerjee, Lin, Hu, Yang, Pask, "Chebyshev polynomial
 * filtered subspace iteration in the Discontinuous Galerkin method for
 * large-scale electronic structure calculations", arXiv:1606.03416) on a
 * block-sparse DG Hamiltonian held in GPU memory.
 *
 * Problem data (Sec. II A and Sec. II B 1 of the paper):
 *   - a periodic nx x ny x nz grid of M = nx*ny*nz elements, element id
 *     K = ix + nx*(iy + ny*iz);
 *   - J_K adaptive local basis functions in element K (alb_counts[K]);
 *     N = sum_K J_K is the matrix order;
 *   - H^DG is symmetric and block-sparse: H_{K;K'} (J_K x J_K') is nonzero only
 *     for face neighbours (block-partition equation of H^DG and eqs.
 *     matvec_1..3).  Each element stores one block per stencil slot, in the
 *     order self, -x, +x, -y, +y, -z, +z (stencil 7) or self, -x, +x, -y, +y
 *     (stencil 5).  A periodic dimension of length 2 reaches one neighbour
 *     through two slots, length 1 reaches the element itself; such blocks add.
 *   - "block-list" layout of H (float64, device): for K = 0..M-1, for each slot
 *     s, the J_K x J_{K'_s} block row-major, back to back.  Its element count
 *     is chefsi_plan_h_elems().
 *   - multivectors (X, Y, ...) are N x ns float64, row-major, element-major rows
 *     (element K owns rows rowoff[K] .. rowoff[K]+J_K-1), row stride ld >= ns.
 *
 * Conventions:
 *   - Pointers named d_* are device memory owned by the caller; the library
 *     never frees or keeps them beyond the call.  Host pointers are marked.
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).  All
 *     kernels of a call are enqueued on it; calls that return host values or a
 *     status that is only known on the device synchronise that stream.
 *   - `ws` is caller-provided device workspace of at least the size returned by
 *     chefsi_workspace_bytes() for the same operation and sizes (256-byte
 *     aligned).  The library allocates device memory only in
 *     chefsi_plan_create (index tables) and, once per plan, when the first
 *     workspace query or call that needs the dense eigensolver creates the
 *     plan's rocBLAS handle.
 *   - Every entry point returns a chefsi_status; argument checks happen on the
 *     host before any HIP call.  chefsi_last_error() gives a message for the
 *     calling thread's most recent failure.  No C++ exception crosses the ABI.
 *   - A plan may be used from one host thread at a time.
 */
#ifndef CHEFSI_H
#define CHEFSI_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  CHEFSI_OK = 0,
  CHEFSI_ERR_ARG = 1,         /* invalid argument (checked on the host)          */
  CHEFSI_ERR_HIP = 2,         /* a HIP runtime / launch error                     */
  CHEFSI_ERR_WORKSPACE = 3,   /* ws is NULL, too small or misaligned              */
  CHEFSI_ERR_NOT_PD = 4,      /* Cholesky met a pivot <= 0                        */
  CHEFSI_ERR_EIG = 5,         /* the dense eigensolver did not converge           */
  CHEFSI_ERR_NONFINITE = 6,   /* a non-finite value where a finite one is needed  */
  CHEFSI_ERR_UNSUPPORTED = 7  /* valid request the library does not implement     */
} chefsi_status;

/* Arithmetic of the filter's recurrence.  CHEFSI_BF16X3 (split BF16) stores
 * every value v as hi + lo with hi = bf16(v), lo = bf16(v - hi) (about 16
 * significant bits) and forms each product from three BF16 MFMAs,
 * A_hi B_hi + A_hi B_lo + A_lo B_hi, accumulated in FP32. */
typedef enum { CHEFSI_F64 = 0, CHEFSI_F32 = 1, CHEFSI_BF16 = 2, CHEFSI_BF16X3 = 3 } chefsi_dtype;

typedef enum {
  CHEFSI_OP_BOUNDS = 0,
  CHEFSI_OP_FILTER = 1,
  CHEFSI_OP_ORTHONORMALIZE = 2,
  CHEFSI_OP_RAYLEIGH_RITZ = 3,
  CHEFSI_OP_SWEEP = 4,
  CHEFSI_OP_FILTER_BACKWARD = 5,
  CHEFSI_OP_LOSS_BACKWARD = 6,
  CHEFSI_OP_DENSITY = 7,
  CHEFSI_OP_LOSS = 8,
  CHEFSI_OP_RAYLEIGH_RITZ_BACKWARD = 9
} chefsi_op;

typedef struct chefsi_plan_s* chefsi_plan;

/* Per-stage device times of one chefsi_sweep call, in milliseconds, measured
 * with HIP events on the call's stream.  filter_steps_ms covers only the m
 * Chebyshev step launches (the dominant kernel).  cholqr_passes is the number
 * of Cholesky-QR passes the call took (1 or 2) and cholqr_cond_bound the
 * condition bound of its first factor (see chefsi_sweep). */
typedef struct {
  double bounds_ms;
  double filter_ms;
  double filter_steps_ms;
  double orthonormalize_ms;
  double rayleigh_ritz_ms;
  double total_ms;
  double cholqr_passes;
  double cholqr_cond_bound;
} chefsi_stats;

/* Library version string and the last error message of this thread. */
const char* chefsi_version(void);
const char* chefsi_last_error(void);

/* ---------------------------------------------------------------- plan ----
 * Element grid, stencil and ALB counts (Sec. II A; Sec. II B 1, the element-
 * wise storage of H^DG).  alb_counts: host array of M int32, each in [1, 256]
 * (the paper's bulk system uses 200 ALBs per element).
 * stencil: 7 (self + 6 faces) or 5 (self + 4 in-plane faces).
 * Builds the neighbour, row-offset and block-offset tables, uploads them to
 * the current HIP device, and keeps no copy of H's values.
 * Errors: CHEFSI_ERR_ARG for bad sizes/stencil/counts, CHEFSI_ERR_HIP. */
int chefsi_plan_create(chefsi_plan* out, int nx, int ny, int nz, int stencil,
                       const int32_t* alb_counts);
void chefsi_plan_destroy(chefsi_plan plan);
/* N = sum_K J_K, and the element count of H in block-list layout. */
int64_t chefsi_plan_n(chefsi_plan plan);
int64_t chefsi_plan_h_elems(chefsi_plan plan);
/* sum_K J_K^2: the element count of a set of element blocks (density-matrix
 * blocks, basis overlaps), stored row-major and back to back in element order. */
int64_t chefsi_plan_block_elems(chefsi_plan plan);
/* Element reached from K through slot s (the plan's table), or -1 on bad args. */
int chefsi_plan_neighbour(chefsi_plan plan, int K, int s);

/* Workspace size in bytes for `op` with ns columns, filter dtype `dtype`,
 * Cholesky-QR passes `passes` and Lanczos steps `lanczos_steps` (ops that do
 * not use an argument ignore it). */
int chefsi_workspace_bytes(chefsi_plan plan, int op, int ns, int dtype, int passes,
                           int lanczos_steps, size_t* bytes);

/* ---------------------------------------------------------------- bounds --
 * Algorithm 1 step 1.  b = b_up from `lanczos_steps` (1..64) steps of Lanczos
 * with full reorthogonalisation started from d_v0 (N float64, need not be
 * normalised): b = largest Ritz value of T_k + beta_k.
 * If d_ritz_prev is non-NULL (ns Ritz values of the previous cycle, ascending)
 *   a = b_low = d_ritz_prev[ns-1], a0 = d_ritz_prev[0];
 * else (first cycle from a random block, no Ritz values yet)
 *   a0 = smallest Ritz value of T_k and a = the smallest Ritz value of T_k
 *   whose cumulative weight sum_{i<=j} tau_i^2 (tau = first components of T_k's
 *   eigenvectors) reaches ns/N.
 * If a0 >= a - 1e-12|b| then a0 = a - 1e-3 (b - a).
 * Writes (a, b, a0) to d_bounds (device, 3 doubles, may be NULL) and to
 * h_bounds (host, 3 doubles, may be NULL).  Synchronises the stream.
 * Returns CHEFSI_ERR_NONFINITE if a bound is not finite and CHEFSI_ERR_ARG if
 * a0 < a < b fails (previous Ritz values at or above the Lanczos bound: they
 * belong to another H); the bounds are written in either case. */
int chefsi_bounds(chefsi_plan plan, const double* d_H, const double* d_v0, int lanczos_steps,
                  const double* d_ritz_prev, int ns, double* d_bounds, double* h_bounds,
                  void* ws, size_t ws_bytes, void* stream);

/* ---------------------------------------------------------------- filter --
 * Algorithm 1 step 2: d_Y = p_m(H) d_X with the three-term recurrence
 *   Y_0 = X, Y_1 = (s_1/e)(H - cI)Y_0,
 *   Y_{k+1} = (2 s_{k+1}/e)(H - cI)Y_k - s_k s_{k+1} Y_{k-1},
 * c = (a+b)/2, e = (b-a)/2, s_1 = e/(a0-c), s_{k+1} = 1/(2/s_1 - s_k), i.e.
 * p_m(t) = T_m((t-c)/e) / T_m((a0-c)/e): [a, b] is mapped to [-1, 1] and the
 * filter is 1 at a0.  Requires a0 < a < b (finite) and m >= 0.
 * dtype selects the arithmetic of the recurrence: CHEFSI_F64 (MFMA FP64),
 * CHEFSI_F32 (FP32 storage and MFMA, FP32 accumulation), CHEFSI_BF16 (bf16
 * storage and MFMA operands, FP32 accumulation and epilogue) or CHEFSI_BF16X3
 * (split bf16 pairs, three BF16 MFMAs per product, FP32 accumulation); H is
 * rounded to that type once per call, X is read in FP64 and Y is written in
 * FP64.
 * d_X and d_Y must not overlap.  Asynchronous. */
int chefsi_filter(chefsi_plan plan, const double* d_H, int m, double a, double b, double a0,
                  int dtype, const double* d_X, int64_t ldx, double* d_Y, int64_t ldy, int ns,
                  void* ws, size_t ws_bytes, void* stream);

/* Allocation-free variant of chefsi_filter, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc).  Same arguments and result as chefsi_filter without
 * the workspace: the filter's scratch is a static device array of the library,
 * CHEFSI_NOALLOC_SCRATCH_BYTES per GPU, held until the process ends (its
 * per-device address is looked up by chefsi_plan_create).  The call allocates
 * nothing.  Returns CHEFSI_ERR_WORKSPACE when the filter's workspace
 * (chefsi_workspace_bytes with CHEFSI_OP_FILTER) exceeds the array: e.g.
 * N * ns * 8 bytes for FP64 plus the packed H and 2.4 MB of coefficients.
 * Every call on a GPU uses that GPU's one array, which keeps the last call's
 * contents: calls that overlap in time on one GPU (several streams or host
 * threads) race and give wrong results.  Asynchronous. */
#define CHEFSI_NOALLOC_SCRATCH_BYTES (256u * 1024u * 1024u)
int chefsi_filter_noalloc(chefsi_plan plan, const double* d_H, int m, double a, double b, double a0,
                          int dtype, const double* d_X, int64_t ldx, double* d_Y, int64_t ldy, int ns,
                          void* stream);

/* ------------------------------------------------------- orthonormalize ---
 * Algorithm 1 step 3 (Cholesky-QR): S = Y^T Y, U^T U = S, solve Yhat U = Y,
 * in place on d_Y (n x ns, float64).  passes = 2 repeats it once on Yhat
 * (CholeskyQR2); passes = 0 repeats it only when the first factor's condition
 * bound asks for it (the rule of chefsi_sweep; one extra synchronisation).
 * d_U (ns x ns row-major, may be NULL) receives U_2 U_1 (or U_1).
 * Returns CHEFSI_ERR_NOT_PD if the first failing pivot was <= 0 and
 * CHEFSI_ERR_NONFINITE if it was not finite (Y held NaN or Inf, or the
 * factorisation overflowed).  Synchronises
 * the stream to read the pivot status. */
int chefsi_orthonormalize(int64_t n, int ns, double* d_Y, int64_t ldy, int passes,
                          double* d_U, void* ws, size_t ws_bytes, void* stream);
/* Workspace bytes of chefsi_orthonormalize for an n x ns block (no plan needed). */
int chefsi_orthonormalize_workspace_bytes(int64_t n, int ns, int passes, size_t* bytes);

/* -------------------------------------------------------- rayleigh_ritz ---
 * Algorithm 1 steps 4-5: W = H Yhat, Hhat = (Yhat^T W + W^T Yhat)/2,
 * Hhat Q = Q D (D ascending; each column of Q has its largest-magnitude entry
 * positive, lowest index on ties), X_new = Yhat Q, and residual norms
 * r_i = ||H x_i - theta_i x_i||_2.  d_ritz (ns), d_resid (ns, may be NULL),
 * d_Q (ns x ns row-major, may be NULL) are device outputs.  d_Xnew must not
 * overlap d_Yhat.  Returns CHEFSI_ERR_EIG if the eigensolver fails.
 * Synchronises the stream to read the eigensolver status. */
int chefsi_rayleigh_ritz(chefsi_plan plan, const double* d_H, const double* d_Yhat, int64_t ldy,
                         int ns, double* d_Xnew, int64_t ldx, double* d_ritz, double* d_resid,
                         double* d_Q, void* ws, size_t ws_bytes, void* stream);

/* ----------------------------------------------------------------- sweep --
 * One CheFSI cycle (Algorithm 1, steps 1-5), X updated in place.
 * Bounds: if d_bounds_in (device, a, b, a0) is non-NULL and warm == 0 they are
 * used as given; if d_bounds_in is non-NULL and warm != 0, b is taken from
 * d_bounds_in[1] (the Lanczos upper bound depends only on H, so a later cycle
 * may reuse it) and a, a0 come from d_ritz on entry by the rule of
 * chefsi_bounds; otherwise step 1 runs as in chefsi_bounds with d_v0 and
 * lanczos_steps, warm (a, a0 from d_ritz on entry) if `warm` != 0, cold
 * otherwise.  filter_dtype as in chefsi_filter.
 * passes: 1 = one Cholesky-QR pass (as in the paper), 2 = CholeskyQR2,
 * 0 = automatic: one pass when the first factor U_1 shows it is enough, i.e.
 * 10 eps B^2 <= 1e-12 for B = sqrt(k_1 k_inf), k_1 and k_inf the 1- and
 * inf-norm condition numbers of U_1 D^{-1} (D = column norms of the filtered
 * block Y), an upper bound on the 2-norm condition number of the
 * column-equilibrated Y (one pass loses orthogonality like eps kappa^2);
 * otherwise two.  The last factor is folded into Rayleigh-Ritz: with B the
 * block before that factor (Y after one pass, Yhat_1 = Y U_1^{-1} after two)
 * and T = U_last^{-1}, Hhat = T^T (B^T H B) T and X = B (T Q), equal to
 * Rayleigh-Ritz on the orthonormalised block in exact arithmetic.
 * Outputs: d_X (new Ritz vectors), d_ritz (ns), d_resid (ns, may be NULL),
 * d_bounds_out (3, may be NULL: the bounds used), stats (host, may be NULL:
 * per-stage event times, passes taken, condition bound).  Synchronises the
 * stream once at the end to read status words, and with passes = 0 also once
 * after the first factor to read its condition bound (a failed first factor
 * then returns at once).
 * Errors found on the device: CHEFSI_ERR_NONFINITE (bounds not finite),
 * CHEFSI_ERR_ARG (bounds with a0 < a < b violated, e.g. warm Ritz values at or
 * above a reused upper bound), CHEFSI_ERR_NOT_PD (the first failing Cholesky pivot
 * <= 0) or CHEFSI_ERR_NONFINITE (it was not finite: X or H held NaN or Inf),
 * CHEFSI_ERR_EIG, reported in that order of precedence.  On every error return d_X is unchanged (the final
 * rotation checks the status words on the device before writing); d_ritz,
 * d_resid and d_bounds_out are then undefined. */
int chefsi_sweep(chefsi_plan plan, const double* d_H, int m, int filter_dtype, int passes,
                 int lanczos_steps, const double* d_v0, const double* d_bounds_in, int warm,
                 double* d_X, int64_t ldx, int ns, double* d_ritz, double* d_resid,
                 double* d_bounds_out, chefsi_stats* stats, void* ws, size_t ws_bytes,
                 void* stream);

/* ------------------------------------------------------------- adjoint ----
 * Reverse-mode gradient of L = sum_{i<k} theta_i, the k lowest Ritz values of
 * one filter (FP64, bounds held constant) + Cholesky-QR (`passes`) +
 * Rayleigh-Ritz pass from X.  Not part of the paper; it differentiates the
 * steps of Algorithm 1 (2-4) by the textbook reverse-mode rules: eigenvalue
 * derivative, projection, thin-QR backward with R_bar = 0, and the reverse
 * three-term sweep Lambda_j = alpha_j (H^T - cI) Lambda_{j+1} - beta_{j+1}
 * Lambda_{j+2}.  The recurrence is recomputed from checkpoints every
 * `ckpt_stride` steps.  Outputs: d_Hbar (block-list layout, overwritten: the
 * gradient w.r.t. every stored block, not symmetrised), d_Xbar (N x ns,
 * ld = ldxb), *h_loss (host, may be NULL).  Synchronises the stream. */
int chefsi_loss_backward(chefsi_plan plan, const double* d_H, int m, double a, double b,
                         double a0, int passes, int k, int ckpt_stride, const double* d_X,
                         int64_t ldx, int ns, double* d_Hbar, double* d_Xbar, int64_t ldxb,
                         double* h_loss, void* ws, size_t ws_bytes, void* stream);

/* The loss alone, L = sum_{i<k} theta_i of the same pass, with exactly the
 * arithmetic of chefsi_loss_backward's forward part (so both report the same
 * value) and no checkpoints, adjoint or rotation: what a forward evaluation
 * without gradients costs.  *h_loss (host).  Synchronises the stream.
 * Workspace: chefsi_backward_workspace_bytes(op = CHEFSI_OP_LOSS). */
int chefsi_loss(chefsi_plan plan, const double* d_H, int m, double a, double b, double a0, int passes,
                int k, const double* d_X, int64_t ldx, int ns, double* h_loss, void* ws,
                size_t ws_bytes, void* stream);

/* Workspace bytes of chefsi_loss_backward (op = CHEFSI_OP_LOSS_BACKWARD),
 * chefsi_loss (op = CHEFSI_OP_LOSS) or chefsi_filter_backward
 * (op = CHEFSI_OP_FILTER_BACKWARD) for degree m, ns columns, `passes`
 * Cholesky-QR passes and checkpoint stride ckpt_stride. */
int chefsi_backward_workspace_bytes(chefsi_plan plan, int op, int m, int ns, int passes,
                                    int ckpt_stride, size_t* bytes);

/* Adjoint of chefsi_orthonormalize (Algorithm 1 step 3): Yhat = Y U^{-1} is
 * the thin QR factorisation of Y (U upper triangular with positive diagonal,
 * d_U as chefsi_orthonormalize returns it: U_2 U_1 after two passes, which is
 * the same factorisation).  Given Yhat_bar = dL/dYhat and no dependence of L
 * on U, writes dL/dY by the textbook QR backward rule
 *   M = -Yhat_bar^T Yhat,  Y_bar = (Yhat_bar + Yhat copyltu(M)) U^{-T},
 * copyltu(M) = tril(M) + tril(M, -1)^T (the last product by triangular
 * substitution).  d_Yhat, d_Yhat_bar, d_Y_bar: n x ns float64 row-major
 * (device); d_U: ns x ns row-major (device).  d_Y_bar may be d_Yhat_bar itself
 * (in place, same leading dimension) but must not otherwise overlap an
 * input.  Workspace: chefsi_orthonormalize_backward_workspace_bytes.
 * Asynchronous. */
int chefsi_orthonormalize_backward(int64_t n, int ns, const double* d_Yhat, int64_t ldy,
                                   const double* d_U, const double* d_Yhat_bar, int64_t ldyb,
                                   double* d_Y_bar, int64_t ldb, void* ws, size_t ws_bytes,
                                   void* stream);
int chefsi_orthonormalize_backward_workspace_bytes(int64_t n, int ns, size_t* bytes);

/* Adjoint of chefsi_rayleigh_ritz's Ritz values (Algorithm 1 step 4): for
 * Hhat = sym(Yhat^T H Yhat) = Q diag(theta) Q^T and a cotangent theta_bar of
 * the Ritz values, Hhat_bar = Q diag(theta_bar) Q^T and
 *   Yhat_bar = H Yhat Hhat_bar + H^T Yhat Hhat_bar   (d_Yhat_bar, written),
 *   H_bar    = Yhat Hhat_bar Yhat^T on the stored blocks (d_Hbar, block-list
 *              layout; overwritten, or added to when accumulate != 0).
 * d_Q: the ns x ns eigenvector matrix chefsi_rayleigh_ritz returns (row-major,
 * column j = eigenvector j); d_ritz_bar: ns float64 (device).  The gradient of
 * the rotated vectors (X_new = Yhat Q) is not part of this rule.
 * d_Yhat_bar and d_Hbar must not overlap any input.  Workspace:
 * chefsi_workspace_bytes(op = CHEFSI_OP_RAYLEIGH_RITZ_BACKWARD, ns).
 * Asynchronous. */
int chefsi_rayleigh_ritz_backward(chefsi_plan plan, const double* d_H, const double* d_Yhat,
                                  int64_t ldy, int ns, const double* d_Q, const double* d_ritz_bar,
                                  double* d_Yhat_bar, int64_t ldyb, double* d_Hbar, int accumulate,
                                  void* ws, size_t ws_bytes, void* stream);

/* Adjoint of chefsi_filter alone (FP64): given Ybar = dL/dY for Y = p_m(H)X,
 * accumulates dL/dH onto d_Hbar (block-list layout, added to) and writes
 * d_Xbar = dL/dX.  Checkpoints every ckpt_stride steps (1..m). Asynchronous. */
int chefsi_filter_backward(chefsi_plan plan, const double* d_H, int m, double a, double b,
                           double a0, int ckpt_stride, const double* d_X, int64_t ldx,
                           const double* d_Ybar, int64_t ldyb, int ns, double* d_Hbar,
                           double* d_Xbar, int64_t ldxb, void* ws, size_t ws_bytes,
                           void* stream);

/* ------------------------------------------------------- occupations ----
 * Fermi-Dirac occupations of the Ritz values (Sec. II A: occupations by
 * Fermi-Dirac smearing; Sec. II B 2: the Ritz values give the Fermi energy and
 * the occupation numbers).  f_i = 1/(1 + exp((theta_i - mu)/kT)) per spatial
 * orbital (the spin factor 2 is left to the density), and the Fermi level mu
 * satisfies sum_i f_i = n_occ (= N_e/2).  mu is found by bisection on
 * [min theta - 50 kT, max theta + 50 kT], halving until the midpoint is no
 * longer strictly inside the bracket (or 200 halvings), mu = the final
 * midpoint.  d_ritz: ns float64 (device, any order); d_f: ns float64 (device,
 * may equal d_ritz for an in-place update); d_mu: 1 float64 (device).
 * Requires 0 < n_occ < ns and kT > 0 (finite).  A non-finite Ritz value gives
 * NaN in d_f and d_mu.  Asynchronous; no workspace. */
int chefsi_occupations(int ns, const double* d_ritz, double n_occ, double kT, double* d_f,
                       double* d_mu, void* stream);

/* ------------------------------------------------ density-matrix blocks ---
 * Diagonal blocks of the density matrix (eq. densitymatrix with K = K'):
 *   P_KK[j][j'] = sum_i f_i X[rowoff[K]+j][i] X[rowoff[K]+j'][i],
 * one J_K x J_K block per element, which is all the electron density needs
 * and is local to each element.  d_X: N x ns Ritz vectors (row stride ldx);
 * d_f: ns weights (device; the occupations); d_P: chefsi_plan_block_elems()
 * float64 (device), element K's block row-major at sum_{K'<K} J_K'^2, exactly
 * symmetric.  d_P must not overlap d_X or d_f.  Workspace:
 * chefsi_workspace_bytes(op = CHEFSI_OP_DENSITY, ns).  Asynchronous.
 * Plans with an ALB count above 128 return CHEFSI_ERR_UNSUPPORTED. */
int chefsi_density_blocks(chefsi_plan plan, const double* d_X, int64_t ldx, int ns, const double* d_f,
                          double* d_P, void* ws, size_t ws_bytes, void* stream);

/* ------------------------------------------------------------ realign -----
 * Re-alignment of the coefficients to a changed ALB basis (Sec. II B 3,
 * eqs. basis_rotation_1-3): X_K <- (V_new,K)^T V_old,K X_K for every element,
 * in place on d_X (N x ns, row stride ldx).  V_K (nr x J_K) samples element
 * K's J_K ALBs on its nr grid points; d_Vnew and d_Vold (device, N*nr float64
 * each) hold, element after element, V_K^T row-major (row j = ALB j's nr
 * samples), element K starting at nr * rowoff[K].  The ALB counts are the
 * plan's for both bases.  d_X must not overlap d_Vnew or d_Vold (d_Vnew may
 * equal d_Vold).  Workspace: chefsi_realign_workspace_bytes.  Asynchronous.
 * Plans with an ALB count above 128 return CHEFSI_ERR_UNSUPPORTED. */
int chefsi_realign(chefsi_plan plan, int nr, const double* d_Vnew, const double* d_Vold, double* d_X,
                   int64_t ldx, int ns, void* ws, size_t ws_bytes, void* stream);
int chefsi_realign_workspace_bytes(chefsi_plan plan, int nr, size_t* bytes);

#ifdef __cplusplus
}
#endif

#endif /* CHEFSI_H */
