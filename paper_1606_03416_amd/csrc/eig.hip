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
  p.eig_ws_cache_bytes = roc + tau + (td > bt ? td : bt);
  *bytes = p.eig_ws_cache_bytes;
  return CHEFSI_OK;
}

// A (n x n, symmetric, lower triangle read) is overwritten by eigenvectors in
// column-major order; d_w gets the eigenvalues ascending; d_E (n) and Z (n x n,
// leading dimension n) are scratch.
int eig_sym(Plan& p, double* A, int64_t lda, int n, double* d_w, double* d_E, int* d_info, double* Z,
            void* d_ws, size_t ws_bytes, hipStream_t st) {
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
  double* tau = reinterpret_cast<double*>(static_cast<char*>(d_ws) + roc);
  void* scratch = static_cast<char*>(d_ws) + roc + round_up(static_cast<int64_t>(n) * 8, 256);
  CHEFSI_TRY(tridiag_lower(h, A, lda, n, d_w, d_E, tau, scratch, st));
  rocblas_status s = rocsolver_dstedc(h, rocblas_evect_tridiagonal, n, d_w, d_E, Z, n, d_info);
  if (s != rocblas_status_success)
    return fail(CHEFSI_ERR_EIG, std::string("rocsolver_dstedc: ") + rocblas_status_to_string(s));
  const size_t scratch_bytes = need - roc - static_cast<size_t>(round_up(static_cast<int64_t>(n) * 8, 256));
  return backtr_lower(A, lda, n, tau, Z, A, lda, scratch, scratch_bytes, st);
}

void destroy_eig_handle(Plan& p) {
  if (p.rocblas) {
    rocblas_destroy_handle(static_cast<rocblas_handle>(p.rocblas));
    p.rocblas = nullptr;
  }
}

}  // namespace chefsi
