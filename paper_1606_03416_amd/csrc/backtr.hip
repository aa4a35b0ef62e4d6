// Back-transformation of the tridiagonal eigenvectors by the reflectors of the
// Householder reduction (the last stage of the dense eigensolve of Algorithm 1
// step 4): C <- Q C with Q = H(0) H(1) ... H(n-2), the reflectors in LAPACK's
// lower format (tridiag.hip), FP64.
//
// The reflectors are taken kBB at a time and aggregated into one block
// reflector H(p0) ... H(p0+nb-1) = I - V T V^T (V unit lower trapezoidal, T
// upper triangular).  T comes from the identity T^{-1} = striu(V^T V) +
// diag(1/tau) (Joffrain, Low, Quintana-Orti, van de Geijn, "Accumulating
// Householder transformations, revisited", ACM TOMS 2006), inverted with the
// library's blocked triangular inverse; it equals LAPACK's forward recurrence
// T(0:k, k) = -tau_k T(0:k, 0:k) V(:, 0:k)^T v_k, T(k, k) = tau_k, without its
// column-by-column dependency.  A reflector with tau = 0 (the identity) enters
// as v = 0 with tau = 1.  Each block is applied to the trailing rows of C with
// three of the library's MFMA GEMMs,
//   W = V^T C,  W = T W,  C -= V W,
// last block first.  C is worked on row-major with rows = the reduction's
// coordinate (one in-place transpose of the column-major eigenvectors of T at
// the start), so that every product is a plain row-major GEMM.
#include "common.h"

namespace chefsi {
namespace {

#ifndef CHEFSI_BACKTR_BB
#define CHEFSI_BACKTR_BB 512
#endif
constexpr int kBB = CHEFSI_BACKTR_BB;   // reflectors per block reflector (a multiple of 64)
static_assert(kBB % 64 == 0, "whole transpose tiles per block");
constexpr int kXT = 64;    // transpose tile edge
constexpr int kSplitK = 256;   // fewest rows per split-K part of V^T C (its result has few tiles)

__device__ __forceinline__ int tri_row(int64_t p) {
  // largest R with R (R + 1) / 2 <= p
  int R = static_cast<int>((sqrt(8.0 * static_cast<double>(p) + 1.0) - 1.0) * 0.5);
  while (static_cast<int64_t>(R) * (R + 1) / 2 > p) --R;
  while (static_cast<int64_t>(R + 1) * (R + 2) / 2 <= p) ++R;
  return R;
}

// In-place transpose of an n x n matrix (leading dimension ld): one
// work-group per tile pair (I, J), I <= J, swaps the two tiles through LDS.
__global__ __launch_bounds__(256) void transpose_sq_kernel(double* A, int64_t ld, int n) {
  __shared__ double s0[kXT][kXT + 1], s1[kXT][kXT + 1];
  const int64_t p = blockIdx.x;
  const int J = tri_row(p);
  const int I = static_cast<int>(p - static_cast<int64_t>(J) * (J + 1) / 2);
  const int x = threadIdx.x & 63, y0 = threadIdx.x >> 6;
  for (int y = y0; y < kXT; y += 4) {
    const int r = I * kXT + y, c = J * kXT + x;
    s0[y][x] = (r < n && c < n) ? A[r * ld + c] : 0.0;
    const int r2 = J * kXT + y, c2 = I * kXT + x;
    s1[y][x] = (I != J && r2 < n && c2 < n) ? A[r2 * ld + c2] : 0.0;
  }
  __syncthreads();
  for (int y = y0; y < kXT; y += 4) {
    const int r = I * kXT + y, c = J * kXT + x;
    if (r < n && c < n) A[r * ld + c] = (I == J) ? s0[x][y] : s1[x][y];
    const int r2 = J * kXT + y, c2 = I * kXT + x;
    if (I != J && r2 < n && c2 < n) A[r2 * ld + c2] = s0[x][y];
  }
}

// V of the block of reflectors p0 .. p0+nb-1 as an m x kBB row-major array
// (m = n - p0 - 1 rows, row rr = coordinate p0 + 1 + rr): v_c(rr) = 0 above
// rr = c, 1 at rr = c, A(p0 + 1 + rr, p0 + c) below; columns nb .. kBB-1 and
// columns of identity reflectors (tau = 0) zero.
// One work-group per 64 x 64 tile (rows of V x columns of V), through LDS.
__global__ __launch_bounds__(256) void build_v_kernel(const double* A, int64_t lda, int n, int p0, int nb,
                                                      const double* tau, double* V) {
  __shared__ double s[kXT][kXT + 1];
  const int m = n - p0 - 1;
  const int rb = blockIdx.x, cb = blockIdx.y;
  const int x = threadIdx.x & 63, y0 = threadIdx.x >> 6;
  // load: column c = cb*64 + y of V, rows rr = rb*64 + x (contiguous in A)
  for (int y = y0; y < kXT; y += 4) {
    const int c = cb * kXT + y, rr = rb * kXT + x;
    double v = 0.0;
    if (c < nb && rr < m && tau[p0 + c] != 0.0) {
      if (rr == c) v = 1.0;
      else if (rr > c) v = A[(p0 + 1 + rr) + static_cast<int64_t>(p0 + c) * lda];
    }
    s[y][x] = v;
  }
  __syncthreads();
  for (int y = y0; y < kXT; y += 4) {
    const int rr = rb * kXT + y, c = cb * kXT + x;
    if (rr < m) V[static_cast<int64_t>(rr) * kBB + c] = s[x][y];
  }
}

// T^{-1} of one block (kBB x kBB row-major, upper triangular): G = V^T V above
// the diagonal, 1/tau on it (1 for identity reflectors and padding columns).
__global__ __launch_bounds__(256) void ut_kernel(const double* G, const double* tau, int nb, double* M) {
  for (int e = threadIdx.x + blockIdx.x * 256; e < kBB * kBB; e += 256 * gridDim.x) {
    const int i = e / kBB, k = e - i * kBB;
    double v = 0.0;
    if (i < k) {
      v = G[e];
    } else if (i == k) {
      const double t = (k < nb) ? tau[k] : 0.0;
      v = (t != 0.0) ? 1.0 / t : 1.0;
    }
    M[e] = v;
  }
}

}  // namespace

size_t backtr_scratch_bytes(int n) {
  if (n <= 1) return 0;
  const int64_t nn = n;
  const size_t split = gemm_tn_split_ws_elems(kBB, nn, nn, kSplitK);
  const size_t splitg = gemm_tn_split_ws_elems(kBB, kBB, nn, kSplitK);
  const int64_t inv = (kBB / 2 + 64) * (kBB / 2 + 64);   // blocked triangular inverse
  const int64_t elems = nn * kBB + 3 * static_cast<int64_t>(kBB) * kBB + inv + 2 * static_cast<int64_t>(kBB) * nn +
                        static_cast<int64_t>(split > splitg ? split : splitg) + 64;
  return static_cast<size_t>(elems) * sizeof(double);
}

int backtr_lower(const double* A, int64_t lda, int n, const double* tau, double* C, double* out, int64_t ldo,
                 void* scratch, size_t scratch_bytes, hipStream_t st) {
  if (n <= 0) return CHEFSI_OK;
  if (n == 1) return launch_copy_f64(C, 1, out, ldo, 1, 1, st);
  if (scratch_bytes < backtr_scratch_bytes(n)) return fail(CHEFSI_ERR_WORKSPACE, "back-transformation scratch too small");
  const int64_t nn = n;
  const int nt = static_cast<int>(ceil_div(n, kXT));
  // C (column-major eigenvectors of T, leading dimension n) -> row-major by coordinate
  transpose_sq_kernel<<<static_cast<unsigned>(static_cast<int64_t>(nt) * (nt + 1) / 2), 256, 0, st>>>(C, nn, n);
  CHEFSI_LAUNCHED("transpose_sq");
  double* s = static_cast<double*>(scratch);
  double* V = s;
  s += nn * kBB;
  double* G = s;
  s += kBB * kBB;
  double* T = s;
  s += kBB * kBB;
  double* M = s;
  s += kBB * kBB;
  double* Wi = s;
  s += (kBB / 2 + 64) * (kBB / 2 + 64);
  double* W = s;
  s += kBB * nn;
  double* W2 = s;
  s += kBB * nn;
  double* split = s;
  const size_t split_elems = backtr_scratch_bytes(n) / sizeof(double) - static_cast<size_t>(s - static_cast<double*>(scratch));
  const int nref = n - 1;   // reflectors 0 .. n-2
  for (int p0 = nref > 0 ? ((nref - 1) / kBB) * kBB : -1; p0 >= 0; p0 -= kBB) {
    const int nb = (nref - p0 < kBB) ? nref - p0 : kBB;
    const int m = n - p0 - 1;
    dim3 gv(static_cast<unsigned>(ceil_div(m, kXT)), static_cast<unsigned>(kBB / kXT));
    build_v_kernel<<<gv, 256, 0, st>>>(A, lda, n, p0, nb, tau, V);
    CHEFSI_LAUNCHED("build_v");
    CHEFSI_TRY(gemm_tn(kBB, kBB, m, 1.0, V, kBB, V, kBB, 0.0, G, kBB, false, split, split_elems, st, kSplitK));
    ut_kernel<<<8, 256, 0, st>>>(G, tau + p0, nb, M);
    CHEFSI_LAUNCHED("ut");
    CHEFSI_TRY(upper_inverse(M, kBB, T, Wi, st));
    double* Cs = C + static_cast<int64_t>(p0 + 1) * nn;
    CHEFSI_TRY(gemm_tn(nb, nn, m, 1.0, V, kBB, Cs, nn, 0.0, W, nn, false, split, split_elems, st, kSplitK));
    CHEFSI_TRY(gemm_nn(nb, nn, nb, 1.0, T, kBB, W, nn, 0.0, W2, nn, st));
    CHEFSI_TRY(gemm_nn(m, nn, nb, -1.0, V, kBB, W2, nn, 1.0, Cs, nn, st));
  }
  // back to column-major eigenvectors in out
  return launch_transpose(C, nn, out, ldo, n, n, st);
}
}  // namespace chefsi
