// Dense symmetric eigensolve of the projected matrix Hhat (Algorithm 1 step 4)
// on the GPU, in FP64: Householder reduction to tridiagonal form by the
// library's own kernels (tridiag.hip), rocSOLVER's tridiagonal
// divide-and-conquer (dstedc, eigenvectors of T), and the back-transformation
// by the reflectors as block reflectors on the library's GEMMs (backtr.hip).
// rocSOLVER's device scratch and the library's scratch come from the caller's
// workspace (rocblas_set_workspace), so the call allocates nothing itself.
#include <rocblas/rocblas.h>
#include <rocsolver/rocsolver.h>

#include "common.h"

namespace chefsi {

namespace {

// *flag |= 1 if any entry of the n x n matrix is not finite.
__global__ __launch_bounds__(256) void nonfinite_scan_kernel(const double* A, int64_t lda, int n, int* flag) {
  const int64_t total = static_cast<int64_t>(n) * n;
  bool bad = false;
  for (int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; t < total;
       t += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const int64_t i = t / n, j = t - i * n;
    bad |= !isfinite(A[i * lda + j]);
  }
  if (bad) atomicOr(flag, 1);
}

// If the matrix is not finite (*flag) or an earlier step of the caller failed
// (skip[0..2], may be null), replace it by the identity so that the
// tridiagonal solver only ever sees finite input; the caller reports the error.
__global__ __launch_bounds__(256) void identity_if_kernel(double* A, int64_t lda, int n, const int* flag,
                                                          const int* skip) {
  const bool bad = (*flag != 0) || (skip != nullptr && (skip[0] | skip[1] | skip[2]) != 0);
  if (!bad) return;
  const int64_t total = static_cast<int64_t>(n) * n;
  for (int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; t < total;
       t += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const int64_t i = t / n, j = t - i * n;
    A[i * lda + j] = (i == j) ? 1.0 : 0.0;
  }
}

// info = -1 when the input was not finite (the solver's own info otherwise).
__global__ void merge_flag_kernel(int* info, const int* flag) {
  if (threadIdx.x == 0 && *flag != 0) *info = -1;
}

unsigned grid_for(int64_t total) {
  int64_t g = (total + 255) / 256;
  if (g < 1) g = 1;
  if (g > 2048) g = 2048;
  return static_cast<unsigned>(g);
}

}  // namespace

static int ensure_handle(Plan& p) {
  if (p.rocblas) return CHEFSI_OK;
  rocblas_handle h = nullptr;
  if (rocblas_create_handle(&h) != rocblas_status_success)
    return fail(CHEFSI_ERR_HIP, "rocblas_create_handle failed");
  p.rocblas = h;
  return CHEFSI_OK;
}

int eig_workspace_bytes(Plan& p, int n, size_t* bytes) {
  if (n <= 0) {
    *bytes = 0;
    return CHEFSI_OK;
  }
  if (p.eig_ws_cache_n == static_cast<size_t>(n)) {
    *bytes = p.eig_ws_cache_bytes;
    return CHEFSI_OK;
  }
  CHEFSI_TRY(ensure_handle(p));
  rocblas_handle h = static_cast<rocblas_handle>(p.rocblas);
  if (rocblas_start_device_memory_size_query(h) != rocblas_status_success)
    return fail(CHEFSI_ERR_HIP, "rocblas size query start failed");
  rocsolver_dstedc(h, rocblas_evect_tridiagonal, n, nullptr, nullptr, nullptr, n, nullptr);
  size_t sz = 0;
  if (rocblas_stop_device_memory_size_query(h, &sz) != rocblas_status_success)
    return fail(CHEFSI_ERR_HIP, "rocblas size query stop failed");
  const size_t roc = static_cast<size_t>(round_up(static_cast<int64_t>(sz), 256));
  const size_t tau = static_cast<size_t>(round_up(static_cast<int64_t>(n) * 8, 256));
  p.eig_ws_cache_n = static_cast<size_t>(n);
  p.eig_ws_cache_roc = roc;
  const size_t td = tridiag_scratch_bytes(n), bt = backtr_scratch_bytes(n);
  p.eig_ws_cache_bytes = roc + tau + 256 + (td > bt ? td : bt);
  *bytes = p.eig_ws_cache_bytes;
  return CHEFSI_OK;
}

// A (n x n, symmetric, lower triangle read) is overwritten by eigenvectors in
// column-major order; d_w gets the eigenvalues ascending; d_E (n) and Z (n x n,
// leading dimension n) are scratch.  *d_info: 0 on success, > 0 if the
// tridiagonal solver failed, -1 if A was not finite.  skip (device, 3 ints, may
// be null): if any is set the solve runs on the identity instead of A.
int eig_sym(Plan& p, double* A, int64_t lda, int n, double* d_w, double* d_E, int* d_info, double* Z,
            void* d_ws, size_t ws_bytes, hipStream_t st, const int* skip) {
  if (n <= 0) return CHEFSI_OK;
  CHEFSI_TRY(ensure_handle(p));
  size_t need = 0;
  CHEFSI_TRY(eig_workspace_bytes(p, n, &need));
  if (ws_bytes < need) return fail(CHEFSI_ERR_WORKSPACE, "eigensolver workspace too small");
  rocblas_handle h = static_cast<rocblas_handle>(p.rocblas);
  if (rocblas_set_stream(h, st) != rocblas_status_success)
    return fail(CHEFSI_ERR_HIP, "rocblas_set_stream failed");
  const size_t roc = p.eig_ws_cache_roc;
  if (rocblas_set_workspace(h, roc ? d_ws : nullptr, roc) != rocblas_status_success)
    return fail(CHEFSI_ERR_HIP, "rocblas_set_workspace failed");
  const size_t taub = static_cast<size_t>(round_up(static_cast<int64_t>(n) * 8, 256));
  double* tau = reinterpret_cast<double*>(static_cast<char*>(d_ws) + roc);
  int* flag = reinterpret_cast<int*>(static_cast<char*>(d_ws) + roc + taub);
  void* scratch = static_cast<char*>(d_ws) + roc + taub + 256;
  const int64_t nn = static_cast<int64_t>(n) * n;
  CHEFSI_TRY(launch_fill_int(flag, 1, 0, st));
  nonfinite_scan_kernel<<<grid_for(nn), 256, 0, st>>>(A, lda, n, flag);
  identity_if_kernel<<<grid_for(nn), 256, 0, st>>>(A, lda, n, flag, skip);
  CHEFSI_LAUNCHED("eig input guard");
  CHEFSI_TRY(tridiag_lower(A, lda, n, d_w, d_E, tau, scratch, st));
  rocblas_status s = rocsolver_dstedc(h, rocblas_evect_tridiagonal, n, d_w, d_E, Z, n, d_info);
  if (s != rocblas_status_success)
    return fail(CHEFSI_ERR_EIG, std::string("rocsolver_dstedc: ") + rocblas_status_to_string(s));
  merge_flag_kernel<<<1, 64, 0, st>>>(d_info, flag);
  CHEFSI_LAUNCHED("eig info");
  const size_t scratch_bytes = need - roc - taub - 256;
  return backtr_lower(A, lda, n, tau, Z, A, lda, scratch, scratch_bytes, st);
}

void destroy_eig_handle(Plan& p) {
  if (p.rocblas) {
    rocblas_destroy_handle(static_cast<rocblas_handle>(p.rocblas));
    p.rocblas = nullptr;
  }
}

}  // namespace chefsi
