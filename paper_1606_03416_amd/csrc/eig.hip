// Dense symmetric eigensolve of the projected matrix Hhat (Algorithm 1 step 4)
// on the GPU through rocSOLVER's divide-and-conquer driver (dsyevd), in FP64.
// rocSOLVER's device scratch comes from the caller's workspace
// (rocblas_set_workspace), so the call allocates nothing itself.
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
  rocsolver_dsyevd(h, rocblas_evect_original, rocblas_fill_upper, n, nullptr, n, nullptr, nullptr,
                   nullptr);
  size_t sz = 0;
  if (rocblas_stop_device_memory_size_query(h, &sz) != rocblas_status_success)
    return fail(CHEFSI_ERR_HIP, "rocblas size query stop failed");
  p.eig_ws_cache_n = static_cast<size_t>(n);
  p.eig_ws_cache_bytes = sz;
  *bytes = sz;
  return CHEFSI_OK;
}

// A (n x n, symmetric, upper triangle read) is overwritten by eigenvectors in
// column-major order; d_w gets the eigenvalues ascending; d_E (n) is scratch.
int eig_sym(Plan& p, double* A, int64_t lda, int n, double* d_w, double* d_E, int* d_info,
            void* d_ws, size_t ws_bytes, hipStream_t st) {
  CHEFSI_TRY(ensure_handle(p));
  size_t need = 0;
  CHEFSI_TRY(eig_workspace_bytes(p, n, &need));
  if (ws_bytes < need) return fail(CHEFSI_ERR_WORKSPACE, "eigensolver workspace too small");
  rocblas_handle h = static_cast<rocblas_handle>(p.rocblas);
  if (rocblas_set_stream(h, st) != rocblas_status_success)
    return fail(CHEFSI_ERR_HIP, "rocblas_set_stream failed");
  if (rocblas_set_workspace(h, need ? d_ws : nullptr, need) != rocblas_status_success)
    return fail(CHEFSI_ERR_HIP, "rocblas_set_workspace failed");
  rocblas_status s = rocsolver_dsyevd(h, rocblas_evect_original, rocblas_fill_upper, n, A,
                                      static_cast<rocblas_int>(lda), d_w, d_E, d_info);
  if (s != rocblas_status_success)
    return fail(CHEFSI_ERR_EIG, std::string("rocsolver_dsyevd: ") + rocblas_status_to_string(s));
  return CHEFSI_OK;
}

void destroy_eig_handle(Plan& p) {
  if (p.rocblas) {
    rocblas_destroy_handle(static_cast<rocblas_handle>(p.rocblas));
    p.rocblas = nullptr;
  }
}

}  // namespace chefsi
