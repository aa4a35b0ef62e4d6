// C ABI of the DG-CheFSI library: plan, argument checks, workspace carving,
// and the orchestration of Algorithm 1 (bounds, filter, Cholesky-QR,
// Rayleigh-Ritz, rotation) over the kernels in filter.hip, dense.hip,
// lanczos.hip and eig.hip.  Every argument check runs on the host before the
// first HIP call of an entry point.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <exception>
#include <mutex>
#include <numeric>

#include "common.h"

// Device scratch of chefsi_filter_noalloc: one copy per GPU, held until the
// process ends.  Host code never uses this name as an address; it uses the
// per-device pointer that scratch_address() obtains once per device.
constexpr size_t kNoallocScratchBytes = size_t(256) << 20;
static __device__ __attribute__((aligned(256))) unsigned char scratch[kNoallocScratchBytes];
static_assert(kNoallocScratchBytes == CHEFSI_NOALLOC_SCRATCH_BYTES, "header and library agree on the size");

namespace chefsi {

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// This device's address of `scratch` (looked up once per device, with that
// device current), or null if the lookup failed.
void* scratch_address(int dev) {
  if (dev < 0 || dev >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_ptr[dev] == nullptr) {
    void* ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess) {
      (void)hipGetLastError();
      return nullptr;
    }
    g_scratch_ptr[dev] = ptr;
  }
  return g_scratch_ptr[dev];
}

}  // namespace

void destroy_eig_handle(Plan& p);

static thread_local std::string g_err;

void set_error(const std::string& msg) { g_err = msg; }

int fail(int code, const std::string& msg) {
  g_err = msg;
  return code;
}

namespace {

constexpr int kMaxDegree = 100000;

bool aligned256(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 255u) == 0; }

int check_device(const Plan& p) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return fail(CHEFSI_ERR_HIP, "hipGetDevice failed");
  if (dev != p.device) return fail(CHEFSI_ERR_ARG, "current HIP device differs from the plan's device");
  return CHEFSI_OK;
}

int check_ws(void* ws, size_t ws_bytes, size_t need) {
  if (need == 0) return CHEFSI_OK;
  if (ws == nullptr) return fail(CHEFSI_ERR_WORKSPACE, "workspace pointer is NULL");
  if (!aligned256(ws)) return fail(CHEFSI_ERR_WORKSPACE, "workspace must be 256-byte aligned");
  if (ws_bytes < need)
    return fail(CHEFSI_ERR_WORKSPACE, "workspace too small: need " + std::to_string(need) +
                                          " bytes, got " + std::to_string(ws_bytes));
  return CHEFSI_OK;
}

bool overlaps(const void* a, size_t an, const void* b, size_t bn) {
  const char* pa = static_cast<const char*>(a);
  const char* pb = static_cast<const char*>(b);
  return pa < pb + bn && pb < pa + an;
}

size_t mv_bytes(int64_t n, int64_t ld, int ns, size_t elt) {
  if (n <= 0 || ns <= 0) return 0;
  return static_cast<size_t>((n - 1) * ld + ns) * elt;
}

int elt_size(int dtype) { return dtype == CHEFSI_F64 ? 8 : (dtype == CHEFSI_F32 ? 4 : 2); }

bool is_b16(int dtype) { return dtype == CHEFSI_BF16 || dtype == CHEFSI_BF16X3; }

bool valid_dtype(int dtype) {
  return dtype == CHEFSI_F64 || dtype == CHEFSI_F32 || dtype == CHEFSI_BF16 || dtype == CHEFSI_BF16X3;
}

// ------------------------------------------------------------ workspace layouts
struct FilterWs {
  double* coef;
  double* bounds;
  void* panel;
  void* buf0;   // F64: recurrence buffer; low precision: converted X
  void* buf1;   // low precision recurrence buffers
  void* buf2;
};

void carve_filter(Carver& c, const Plan& p, int ns, int dtype, bool need_panel, FilterWs& f) {
  const int e = elt_size(dtype);
  f.coef = c.take<double>(3 * static_cast<int64_t>(kMaxDegree));
  f.bounds = c.take<double>(4);
  // split BF16 holds hi and lo halves of every buffer
  const int parts = (dtype == CHEFSI_BF16X3) ? 2 : 1;
  const int64_t pe = is_b16(dtype) ? parts * p.panel8_elems : p.panel_elems;
  f.panel = need_panel ? c.take<char>(pe * e) : nullptr;
  const int64_t mv = p.N * static_cast<int64_t>(ns);
  if (dtype == CHEFSI_F64) {
    f.buf0 = c.take<double>(mv);
    f.buf1 = f.buf2 = nullptr;
  } else if (is_b16(dtype)) {
    const int64_t mvp = parts * p.N8 * static_cast<int64_t>(ns);
    f.buf0 = c.take<char>(mvp * e);
    f.buf1 = c.take<char>(mvp * e);
    f.buf2 = c.take<char>(mvp * e);
  } else {
    f.buf0 = c.take<char>(mv * e);
    f.buf1 = c.take<char>(mv * e);
    f.buf2 = c.take<char>(mv * e);
  }
}

struct OrthWs {
  double* S;
  double* U1;
  double* U2;
  double* T;      // U^{-1}
  double* Wt;     // scratch of the triangular inverse
  double* B;      // n x ns block the passes alternate with
  double* split;
  size_t split_elems;
  int* status;
  double* cond;   // condition bound of the first factor (1 double)
  double* cscr;   // its scratch
};

void carve_orth(Carver& c, int64_t n, int ns, OrthWs& o) {
  const int64_t nn = static_cast<int64_t>(ns) * ns;
  o.S = c.take<double>(nn);
  o.U1 = c.take<double>(nn);
  o.U2 = c.take<double>(nn);
  o.T = c.take<double>(nn);
  o.Wt = c.take<double>((static_cast<int64_t>(ns) / 2 + 64) * (static_cast<int64_t>(ns) / 2 + 64));
  o.B = c.take<double>(n * static_cast<int64_t>(ns));
  o.split_elems = gemm_tn_split_ws_elems(ns, ns, n);
  o.split = o.split_elems ? c.take<double>(static_cast<int64_t>(o.split_elems)) : nullptr;
  o.status = c.take<int>(4);
  o.cond = c.take<double>(8);
  o.cscr = c.take<double>(static_cast<int64_t>(cholqr_cond_scratch_elems(ns)));
}

struct RrWs {
  void* panel;     // FP64 panel (may be shared)
  double* W;
  double* Hh;
  double* Q;       // ns*ns + ns (signs)
  double* E;
  double* w;
  double* part;
  double* coef;
  double* split;
  size_t split_elems;
  int* info;
  void* eig;
  size_t eig_bytes;
};

int carve_rr(Carver& c, Plan& p, int ns, bool need_panel, RrWs& r) {
  const int64_t nn = static_cast<int64_t>(ns) * ns;
  r.panel = need_panel ? c.take<double>(p.panel_elems) : nullptr;
  r.W = c.take<double>(p.N * static_cast<int64_t>(ns));
  r.Hh = c.take<double>(nn);
  r.Q = c.take<double>(nn + ns);
  r.E = c.take<double>(ns);
  r.w = c.take<double>(ns);
  r.part = c.take<double>(static_cast<int64_t>(p.M) * ns);
  r.coef = c.take<double>(4);
  r.split_elems = gemm_tn_split_ws_elems(ns, ns, p.N);
  r.split = r.split_elems ? c.take<double>(static_cast<int64_t>(r.split_elems)) : nullptr;
  r.info = c.take<int>(4);
  size_t eb = 0;
  int rc = eig_workspace_bytes(p, ns, &eb);
  r.eig_bytes = eb;
  r.eig = eb ? c.take<char>(static_cast<int64_t>(eb)) : nullptr;
  return rc;
}

// ------------------------------------------------------------ building blocks
int run_filter(const Plan& p, const void* panel, int dtype, const double* coef, int m,
               const double* X, int64_t ldx, double* Y, int64_t ldy, int ns, const FilterWs& f,
               hipStream_t st) {
  if (m == 0) return launch_copy_f64(X, ldx, Y, ldy, p.N, ns, st);
  if (dtype == CHEFSI_F64) {
    double* B[2] = {Y, static_cast<double*>(f.buf0)};
    const int64_t LD[2] = {ldy, ns};
    for (int k = 0; k < m; ++k) {
      const int bi = (m - k) % 2, bp = (m - k + 1) % 2, bo = (m - k - 1) % 2;
      StepIO io{};
      io.in = (k == 0) ? static_cast<const void*>(X) : B[bi];
      io.ldi = (k == 0) ? ldx : LD[bi];
      io.in_f64 = true;
      io.prev = (k == 0) ? nullptr : (k == 1 ? static_cast<const void*>(X) : B[bp]);
      io.ldp = (k == 1) ? ldx : LD[bp];
      io.prev_f64 = true;
      io.out = B[bo];
      io.ldo = LD[bo];
      io.out_f64 = true;
      io.shifted = true;
      CHEFSI_TRY(launch_step(p, panel, dtype, coef + 3 * k, io, ns, st));
    }
    return CHEFSI_OK;
  }
  // low precision: X converted once, Y_1..Y_{m-1} in two rotating buffers,
  // Y_m written in FP64.
  void* L[2] = {f.buf1, f.buf2};
  if (is_b16(dtype)) {
    const bool split = (dtype == CHEFSI_BF16X3);
    CHEFSI_TRY(launch_to_tiles_b16(p, X, ldx, f.buf0, ns, st, split));
    for (int k = 0; k < m; ++k) {
      const bool last = (k == m - 1);
      const void* in = (k == 0) ? f.buf0 : L[k % 2];
      const void* prev = (k == 0) ? nullptr : (k == 1 ? f.buf0 : L[(k - 1) % 2]);
      void* out = last ? static_cast<void*>(Y) : L[(k + 1) % 2];
      CHEFSI_TRY(launch_step_b16(p, panel, coef + 3 * k, in, prev, out, last, ldy, ns, st, split));
    }
    return CHEFSI_OK;
  }
  CHEFSI_TRY(launch_convert(X, ldx, f.buf0, dtype, ns, p.N, ns, st));
  for (int k = 0; k < m; ++k) {
    StepIO io{};
    io.in = (k == 0) ? f.buf0 : L[k % 2];
    io.ldi = ns;
    io.in_f64 = false;
    io.prev = (k == 0) ? nullptr : (k == 1 ? f.buf0 : L[(k - 1) % 2]);
    io.ldp = ns;
    io.prev_f64 = false;
    const bool last = (k == m - 1);
    io.out = last ? static_cast<void*>(Y) : L[(k + 1) % 2];
    io.ldo = last ? ldy : ns;
    io.out_f64 = last;
    io.shifted = true;
    CHEFSI_TRY(launch_step(p, panel, dtype, coef + 3 * k, io, ns, st));
  }
  return CHEFSI_OK;
}

// passes = 0 (auto): one pass is kept when 10 eps B^2 <= 1e-12 for the
// condition bound B of the first factor (B >= kappa_2 of the
// column-equilibrated block; one pass loses orthogonality like eps kappa^2).
constexpr double kAutoLossLimit = 1e-12;
constexpr double kAutoLossFactor = 10.0;

int auto_passes_from_bound(double B) {
  const double eps = 2.220446049250313e-16;
  return (kAutoLossFactor * eps * B * B <= kAutoLossLimit) ? 1 : 2;
}

// Error of a Cholesky status word: 1 = a pivot not above zero (the block is
// rank deficient), 2 = a pivot that is not finite (the block holds NaN or Inf).
int chol_fail(int h) {
  if (h == 2) return fail(CHEFSI_ERR_NONFINITE, "Cholesky factorisation met a non-finite pivot (input not finite)");
  return fail(CHEFSI_ERR_NOT_PD, "Cholesky factorisation met a non-positive pivot");
}

// Cholesky-QR, `passes` times: S = Y^T Y (upper triangle, mirrored),
// U^T U = S, and Yhat = Y U^{-1} as one GEMM with the triangular inverse
// (its zero part skipped).  The passes alternate between Y and o.B so that
// the result ends in Y.  passes = 0: the second pass runs only if the first
// factor's condition bound asks for it (auto_passes_from_bound), which reads
// the bound on the host (one stream synchronisation).
int run_orth(int64_t n, int ns, double* Y, int64_t ldy, int passes, double* Uout, const OrthWs& o,
             hipStream_t st) {
  CHEFSI_TRY(launch_fill_int(o.status, 1, 0, st));
  double* Us[2] = {o.U1, o.U2};
  double* src = Y;
  int64_t lds = ldy;
  int used = passes ? passes : 2;
  for (int pass = 0; pass < used; ++pass) {
    const bool last = (pass == used - 1);
    double* dst = (used == 2 && last) ? Y : o.B;
    const int64_t ldd = (dst == Y) ? ldy : ns;
    CHEFSI_TRY(gemm_tn(ns, ns, n, 1.0, src, lds, src, lds, 0.0, o.S, ns, true, o.split, o.split_elems, st));
    CHEFSI_TRY(launch_symmetrize(o.S, ns, ns, 1, st));
    CHEFSI_TRY(cholesky_upper(o.S, ns, ns, o.status, o.Wt, st));
    CHEFSI_TRY(launch_copy_f64(o.S, ns, Us[pass], ns, ns, ns, st));
    CHEFSI_TRY(upper_inverse(o.S, ns, o.T, o.Wt, st));
    CHEFSI_TRY(gemm_nn(n, ns, ns, 1.0, src, lds, o.T, ns, 0.0, dst, ldd, st, true));
    src = dst;
    lds = ldd;
    if (passes == 0 && pass == 0) {
      CHEFSI_TRY(cholqr_cond_bound(o.S, o.T, ns, o.cscr, o.cond, st));
      double h = 0.0;
      int hs0 = 0;
      CHEFSI_HIP(hipMemcpyAsync(&h, o.cond, sizeof(double), hipMemcpyDeviceToHost, st));
      CHEFSI_HIP(hipMemcpyAsync(&hs0, o.status, sizeof(int), hipMemcpyDeviceToHost, st));
      CHEFSI_HIP(hipStreamSynchronize(st));
      if (hs0 != 0) return chol_fail(hs0);
      used = auto_passes_from_bound(h);
    }
  }
  if (src != Y) CHEFSI_TRY(launch_copy_f64(src, lds, Y, ldy, n, ns, st));
  if (Uout != nullptr) {
    if (used == 1) {
      CHEFSI_TRY(launch_copy_f64(o.U1, ns, Uout, ns, ns, ns, st));
    } else {
      CHEFSI_TRY(trmm_upper_upper(o.U2, o.U1, Uout, ns, st));
    }
  }
  return CHEFSI_OK;
}

// Cholesky-QR inside a sweep.  The first factor: S = Y^T Y (upper triangle,
// mirrored), U1^T U1 = S (U1 left in o.S), T = U1^{-1}.
int run_orth_factor1(int64_t n, int ns, const double* Y, int64_t ldy, double* T, const OrthWs& o,
                     hipStream_t st) {
  CHEFSI_TRY(launch_fill_int(o.status, 1, 0, st));
  CHEFSI_TRY(gemm_tn(ns, ns, n, 1.0, Y, ldy, Y, ldy, 0.0, o.S, ns, true, o.split, o.split_elems, st));
  CHEFSI_TRY(launch_symmetrize(o.S, ns, ns, 1, st));
  CHEFSI_TRY(cholesky_upper(o.S, ns, ns, o.status, o.Wt, st));
  return upper_inverse(o.S, ns, T, o.Wt, st);
}

// The second pass of CholeskyQR2, factor only: Yhat1 = Y T1 (into Y1out),
// U2 from Yhat1^T Yhat1, and T <- U2^{-1}.
int run_orth_pass2(int64_t n, int ns, const double* Y, int64_t ldy, double* T, double* Y1out, int64_t ld1,
                   const OrthWs& o, hipStream_t st) {
  CHEFSI_TRY(gemm_nn(n, ns, ns, 1.0, Y, ldy, T, ns, 0.0, Y1out, ld1, st, true));
  CHEFSI_TRY(gemm_tn(ns, ns, n, 1.0, Y1out, ld1, Y1out, ld1, 0.0, o.S, ns, true, o.split, o.split_elems, st));
  CHEFSI_TRY(launch_symmetrize(o.S, ns, ns, 1, st));
  CHEFSI_TRY(cholesky_upper(o.S, ns, ns, o.status, o.Wt, st));
  return upper_inverse(o.S, ns, T, o.Wt, st);
}

// Rayleigh-Ritz with the last Cholesky factor folded in.  B is the block whose
// orthonormalisation is B T (T = U^{-1} of B's last factor): the filtered
// block itself after one pass, Yhat1 after two.  Then
//   Hhat = T^T (B^T H B) T,   X = B (T Q),
// which equals Rayleigh-Ritz on B T in exact arithmetic and never forms B T.
// X must not alias B.  The rotation into X is skipped on the device when any of
// status[0..2] is set, so that a failed cycle leaves X as it was.
int run_rr_fold(Plan& p, const void* panel64, const double* B, int64_t ldb, int ns, const double* T, double* X,
                int64_t ldx, const int* status, double* ritz, double* resid, const RrWs& r, hipStream_t st) {
  CHEFSI_TRY(launch_const_coef(1.0, 0.0, r.coef, st));
  StepIO io{B, ldb, true, nullptr, 0, true, r.W, ns, true, true};   // W = H B (no c term)
  CHEFSI_TRY(launch_step(p, panel64, CHEFSI_F64, r.coef, io, ns, st));
  CHEFSI_TRY(gemm_tn(ns, ns, p.N, 1.0, B, ldb, r.W, ns, 0.0, r.Hh, ns, true, r.split, r.split_elems, st));
  CHEFSI_TRY(launch_symmetrize(r.Hh, ns, ns, 1, st));
  // Hhat = T^T (B^T W) T (upper triangle, mirrored)
  CHEFSI_TRY(gemm_nn(ns, ns, ns, 1.0, r.Hh, ns, T, ns, 0.0, r.Q, ns, st, true));
  CHEFSI_TRY(gemm_tn(ns, ns, ns, 1.0, T, ns, r.Q, ns, 0.0, r.Hh, ns, true, r.split, r.split_elems, st));
  CHEFSI_TRY(launch_symmetrize(r.Hh, ns, ns, 1, st));
  CHEFSI_TRY(launch_fill_int(r.info, 1, 0, st));
  CHEFSI_TRY(eig_sym(p, r.Hh, ns, ns, ritz, r.E, r.info, r.Q, r.eig, r.eig_bytes, st, status));
  CHEFSI_TRY(launch_eigvec_fix(r.Hh, ns, ns, r.Q, ns, st));
  // X = B (T Q)
  CHEFSI_TRY(gemm_nn(ns, ns, ns, 1.0, T, ns, r.Q, ns, 0.0, r.Hh, ns, st));
  CHEFSI_TRY(gemm_nn(p.N, ns, ns, 1.0, B, ldb, r.Hh, ns, 0.0, X, ldx, st, false, status));
  if (resid != nullptr) {
    CHEFSI_TRY(launch_resid_partial(p, panel64, X, ldx, ritz, ns, r.part, st));
    CHEFSI_TRY(launch_colsum_sqrt(r.part, p.M, ns, resid, st));
  }
  return CHEFSI_OK;
}

int run_rr(Plan& p, const void* panel64, const double* Yh, int64_t ldy, int ns, double* Xn,
           int64_t ldx, double* ritz, double* resid, double* Qout, const RrWs& r, hipStream_t st) {
  CHEFSI_TRY(launch_const_coef(1.0, 0.0, r.coef, st));
  StepIO io{Yh, ldy, true, nullptr, 0, true, r.W, ns, true, true};   // W = H Yhat (no c term)
  CHEFSI_TRY(launch_step(p, panel64, CHEFSI_F64, r.coef, io, ns, st));
  // Hhat = Yhat^T (H Yhat) is symmetric: form its upper triangle and mirror it
  CHEFSI_TRY(gemm_tn(ns, ns, p.N, 1.0, Yh, ldy, r.W, ns, 0.0, r.Hh, ns, true, r.split, r.split_elems, st));
  CHEFSI_TRY(launch_symmetrize(r.Hh, ns, ns, 1, st));
  CHEFSI_TRY(launch_fill_int(r.info, 1, 0, st));
  CHEFSI_TRY(eig_sym(p, r.Hh, ns, ns, ritz, r.E, r.info, r.Q, r.eig, r.eig_bytes, st));
  CHEFSI_TRY(launch_eigvec_fix(r.Hh, ns, ns, r.Q, ns, st));
  CHEFSI_TRY(gemm_nn(p.N, ns, ns, 1.0, Yh, ldy, r.Q, ns, 0.0, Xn, ldx, st));
  if (resid != nullptr) {
    CHEFSI_TRY(launch_resid_partial(p, panel64, Xn, ldx, ritz, ns, r.part, st));
    CHEFSI_TRY(launch_colsum_sqrt(r.part, p.M, ns, resid, st));
  }
  if (Qout != nullptr) CHEFSI_TRY(launch_copy_f64(r.Q, ns, Qout, ns, ns, ns, st));
  return CHEFSI_OK;
}

int read_status(const int* d_status, int code_if_set, const char* what, hipStream_t st) {
  int h = 0;
  CHEFSI_HIP(hipMemcpyAsync(&h, d_status, sizeof(int), hipMemcpyDeviceToHost, st));
  CHEFSI_HIP(hipStreamSynchronize(st));
  if (h < 0) return fail(CHEFSI_ERR_NONFINITE, "the projected matrix is not finite");
  if (h != 0) return fail(code_if_set, std::string(what) + " (device status " + std::to_string(h) + ")");
  return CHEFSI_OK;
}

#ifdef CHEFSI_DEBUG
// Debug builds: every index a kernel takes from the plan's tables stays inside
// the buffer it indexes (checked on the host before the upload).  A failure is
// a bug of the library, reported as CHEFSI_ERR_ARG with "table check" in the
// message.
int verify_plan_tables(const Plan& p, const std::vector<int32_t>& kmap, const std::vector<int32_t>& kg8,
                       const std::vector<int32_t>& rowsrc8, const std::vector<int32_t>& order) {
  auto bad = [](const std::string& what) { return fail(CHEFSI_ERR_ARG, "plan table check: " + what); };
  const int M = p.M, S = p.stencil;
  if (p.rowoff.size() != static_cast<size_t>(M) + 1 || p.rowoff[0] != 0 || p.rowoff[M] != p.N) return bad("rowoff");
  for (int K = 0; K < M; ++K) {
    if (p.J[K] < 1 || p.J[K] > kMaxJ || p.rowoff[K + 1] - p.rowoff[K] != p.J[K]) return bad("J / rowoff");
    if (p.rb[K] * 16 < p.J[K] || p.rb[K] > p.maxRB) return bad("rb");
    int kt = 0;
    int64_t h = p.hoff[static_cast<size_t>(K) * S];
    for (int s = 0; s < S; ++s) {
      const int Kp = p.nbr[static_cast<size_t>(K) * S + s];
      if (Kp < 0 || Kp >= M) return bad("nbr");
      if (p.hoff[static_cast<size_t>(K) * S + s] != h) return bad("hoff contiguity");
      h += static_cast<int64_t>(p.J[K]) * p.J[Kp];
      kt += p.J[Kp];
    }
    if (h > p.h_elems) return bad("hoff range");
    if (kt != p.ktot[K] || p.kpad[K] < kt || p.kpad[K] % kStepKC != 0 || p.kpad[K] > 7 * kMaxJ) return bad("kpad");
    if (p.koff[K] + p.kpad[K] > p.kmap_len) return bad("koff");
    for (int k = 0; k < p.kpad[K]; ++k) {
      const int32_t g = kmap[p.koff[K] + k];
      if (k < kt ? (g < 0 || g >= p.N) : (g != -1)) return bad("kmap entry");
    }
    if (p.poff[K] + static_cast<int64_t>(p.kpad[K]) * p.rb[K] * 16 > p.panel_elems) return bad("poff");
    if (p.kpad8[K] % kPadK != 0 || p.kpad8[K] > 7 * kMaxJ) return bad("kpad8");
    if (p.kgoff[K] + p.kpad8[K] / 8 > static_cast<int64_t>(kg8.size())) return bad("kgoff");
    for (int t = 0; t < p.kpad8[K] / 8; ++t) {
      const int32_t G = kg8[p.kgoff[K] + t];
      if (G < -1 || static_cast<int64_t>(G) * 8 >= p.N8) return bad("kg8 entry");
    }
    if (p.poff8[K] + static_cast<int64_t>(p.kpad8[K]) * p.rb[K] * 16 > p.panel8_elems) return bad("poff8");
    if (p.rowoff8[K + 1] - p.rowoff8[K] != round_up(p.J[K], 8)) return bad("rowoff8");
    if (p.sqoff[K + 1] - p.sqoff[K] != static_cast<int64_t>(p.J[K]) * p.J[K]) return bad("sqoff");
  }
  if (p.rowoff8[M] != p.N8 || static_cast<int64_t>(rowsrc8.size()) != p.N8) return bad("N8");
  for (int32_t r : rowsrc8)
    if (r < -1 || r >= p.N) return bad("rowsrc8 entry");
  std::vector<char> seen(M, 0);
  for (int32_t K : order) {
    if (K < 0 || K >= M || seen[K]) return bad("order is not a permutation");
    seen[K] = 1;
  }
  int covered = 0;
  for (size_t g = 0; g < p.grp_rb.size(); ++g) {
    if (p.grp_start[g] != covered) return bad("launch groups");
    for (int e = p.grp_start[g]; e < p.grp_start[g] + p.grp_count[g]; ++e)
      if (p.rb[order[e]] != p.grp_rb[g]) return bad("group row-block count");
    covered += p.grp_count[g];
  }
  if (covered != M) return bad("launch groups cover");
  return CHEFSI_OK;
}
#endif

int validate_mv(const char* name, const void* d, int64_t ld, int ns) {
  if (ns > 0 && d == nullptr) return fail(CHEFSI_ERR_ARG, std::string(name) + " is NULL");
  if (ld < ns || ld < 1) return fail(CHEFSI_ERR_ARG, std::string(name) + ": leading dimension < ns");
  return CHEFSI_OK;
}

int validate_bounds(double a, double b, double a0) {
  if (!std::isfinite(a) || !std::isfinite(b) || !std::isfinite(a0))
    return fail(CHEFSI_ERR_ARG, "filter bounds must be finite");
  if (!(a0 < a && a < b)) return fail(CHEFSI_ERR_ARG, "filter bounds must satisfy a0 < a < b");
  return CHEFSI_OK;
}

template <typename F>
int guarded(F&& f) {
  try {
    return f();
  } catch (const std::exception& e) {
    return fail(CHEFSI_ERR_HIP, std::string("internal error: ") + e.what());
  } catch (...) {
    return fail(CHEFSI_ERR_HIP, "internal error");
  }
}

// Workspace of a sweep: a common part, then the filter, Cholesky-QR and
// Rayleigh-Ritz carvings one after the other in the same region, except that
// with a second pass (passes != 1) the Rayleigh-Ritz carving follows the
// Cholesky-QR one, whose block B then holds Yhat1 = Y U1^{-1} (so d_X is
// written only by the final rotation).
size_t sweep_bytes(Plan& p, int ns, int dtype, int k, int passes) {
  Carver c(nullptr, 0);
  c.take<double>(p.panel_elems);                        // FP64 panel
  c.take<double>(p.N * static_cast<int64_t>(ns));       // filtered block
  c.take<double>(8);                                    // bounds
  c.take<int>(8);                                       // status words
  c.take<double>(static_cast<int64_t>(ns) * ns);        // inverse of the last Cholesky factor
  c.take<double>(8);                                    // condition bound
  c.take<double>(static_cast<int64_t>(cholqr_cond_scratch_elems(ns)));
  const size_t base = c.used;
  Carver cf(nullptr, 0);
  FilterWs f;
  carve_filter(cf, p, ns, dtype, true, f);
  Carver co(nullptr, 0);
  OrthWs o;
  carve_orth(co, p.N, ns, o);
  Carver cr(nullptr, 0);
  RrWs r;
  carve_rr(cr, p, ns, false, r);
  size_t lz = lanczos_ws_bytes(p, k);
  const size_t subspace = (passes == 1) ? std::max(co.used, cr.used) : co.used + cr.used;
  return base + std::max(std::max(cf.used, subspace), lz);
}


// ------------------------------------------------------------ adjoint
struct BwdWs {
  double* panel = nullptr;
  double* panelT = nullptr;
  double* coef = nullptr;
  double* rcoef = nullptr;
  double* bounds = nullptr;
  double* cconst = nullptr;
  double* F[2] = {nullptr, nullptr};
  std::vector<double*> ckY, ckP, seg;
  double* LA = nullptr;
  double* LB = nullptr;
  // loss path
  double *P1 = nullptr, *P2 = nullptr, *W = nullptr, *YH = nullptr, *G = nullptr;
  double *S = nullptr, *U0 = nullptr, *U1 = nullptr, *Mb = nullptr, *Lt = nullptr, *Hh = nullptr;
  double *Q = nullptr, *QT = nullptr, *Hhb = nullptr, *split = nullptr;
  size_t split_elems = 0;
  double *theta = nullptr, *E = nullptr, *loss = nullptr;
  int* status = nullptr;
  void* eig = nullptr;
  size_t eig_bytes = 0;
};

// reverse = false: the forward of the loss only (no checkpoints, no H^T
// panel, no reverse-sweep buffers).
int carve_bwd(Carver& c, Plan& p, int m, int ns, int passes, int stride, bool loss_path, BwdWs& b,
              bool reverse = true) {
  const int64_t mv = p.N * static_cast<int64_t>(ns);
  const int64_t nn = static_cast<int64_t>(ns) * ns;
  const int nseg = (m > 0 && reverse) ? static_cast<int>(ceil_div(m, stride)) : 0;
  b.panel = c.take<double>(p.panel_elems);
  b.panelT = reverse ? c.take<double>(p.panel_elems) : nullptr;
  b.coef = c.take<double>(3 * static_cast<int64_t>(std::max(m, 1)));
  b.rcoef = reverse ? c.take<double>(3 * static_cast<int64_t>(std::max(m, 1))) : nullptr;
  b.bounds = c.take<double>(4);
  b.cconst = c.take<double>(8);
  b.F[0] = c.take<double>(mv);
  b.F[1] = c.take<double>(mv);
  b.ckY.assign(nseg, nullptr);
  b.ckP.assign(nseg, nullptr);
  for (int i = 1; i < nseg; ++i) {
    b.ckY[i] = c.take<double>(mv);
    b.ckP[i] = c.take<double>(mv);
  }
  b.seg.assign(std::max(stride, 1), nullptr);
  if (reverse)
    for (int t = 1; t < stride && t < m; ++t) b.seg[t] = c.take<double>(mv);
  b.LA = reverse ? c.take<double>(mv) : nullptr;
  b.LB = reverse ? c.take<double>(mv) : nullptr;
  b.status = c.take<int>(8);
  if (!loss_path) return CHEFSI_OK;
  b.P1 = c.take<double>(mv);
  b.P2 = passes == 2 ? c.take<double>(mv) : nullptr;
  b.W = c.take<double>(mv);
  b.YH = reverse ? c.take<double>(mv) : nullptr;
  b.G = reverse ? c.take<double>(mv) : nullptr;
  b.S = c.take<double>(nn);
  b.U0 = c.take<double>(nn);
  b.U1 = c.take<double>(nn);
  b.Mb = c.take<double>(nn);
  b.Lt = c.take<double>(nn);
  b.Hh = c.take<double>(nn);
  b.Q = c.take<double>(nn + ns);
  b.QT = c.take<double>(nn);
  b.Hhb = c.take<double>(nn);
  b.split_elems = gemm_tn_split_ws_elems(ns, ns, p.N);
  b.split = b.split_elems ? c.take<double>(static_cast<int64_t>(b.split_elems)) : nullptr;
  b.theta = c.take<double>(ns);
  b.E = c.take<double>(ns);
  b.loss = c.take<double>(4);
  int rc = eig_workspace_bytes(p, ns, &b.eig_bytes);
  b.eig = b.eig_bytes ? c.take<char>(static_cast<int64_t>(b.eig_bytes)) : nullptr;
  return rc;
}

// Forward recurrence from X, keeping (Y_{i*stride - 1}, Y_{i*stride}) for each
// segment start i >= 1.  Runs `steps` steps; *Ylast / *ldlast get Y_steps.
int forward_checkpointed(const Plan& p, const double* panel, const double* coef, int steps, int stride,
                         const double* X, int64_t ldx, int ns, BwdWs& b, const double** Ylast,
                         int64_t* ldlast, hipStream_t st) {
  const double* Yk = X;
  int64_t ldk = ldx;
  const double* Ykm1 = nullptr;
  int64_t ldkm1 = 0;
  for (int k = 0; k < steps; ++k) {
    double* out = b.F[(k + 1) % 2];
    StepIO io{Yk, ldk, true, Ykm1, ldkm1, true, out, ns, true};
    CHEFSI_TRY(launch_step(p, panel, CHEFSI_F64, coef + 3 * k, io, ns, st));
    Ykm1 = Yk;
    ldkm1 = ldk;
    Yk = out;
    ldk = ns;
    if ((k + 1) % stride == 0) {
      const int i = (k + 1) / stride;
      if (i < static_cast<int>(b.ckY.size())) {
        CHEFSI_TRY(launch_copy_f64(Yk, ldk, b.ckY[i], ns, p.N, ns, st));
        CHEFSI_TRY(launch_copy_f64(Ykm1, ldkm1, b.ckP[i], ns, p.N, ns, st));
      }
    }
  }
  *Ylast = Yk;
  *ldlast = ldk;
  return CHEFSI_OK;
}

// Reverse three-term sweep from Lambda_m (already in b.LA):
//   Hbar += sum_j alpha_j Lambda_{j+1} Y_j^T (stored blocks),
//   Lambda_j = alpha_j (H^T - cI) Lambda_{j+1} - beta_{j+1} Lambda_{j+2},
// recomputing Y_j segment by segment from the checkpoints; Xbar = Lambda_0.
int reverse_sweep(const Plan& p, int m, int stride, const double* X, int64_t ldx, int ns, BwdWs& b,
                  double* Hbar, double* Xbar, int64_t ldxb, hipStream_t st) {
  const int nseg = static_cast<int>(ceil_div(m, stride));
  double* lam1 = b.LA;       // Lambda_{j+1}
  double* lam2 = nullptr;    // Lambda_{j+2}
  std::vector<const double*> Yseg(std::max(stride, 1));
  std::vector<int64_t> ldseg(std::max(stride, 1));
  for (int sg = nseg - 1; sg >= 0; --sg) {
    const int j0 = sg * stride;
    const int j1 = std::min(j0 + stride, m);
    Yseg[0] = (sg == 0) ? X : b.ckY[sg];
    ldseg[0] = (sg == 0) ? ldx : ns;
    const double* Yprev0 = (sg == 0) ? nullptr : b.ckP[sg];
    for (int t = 1; t < j1 - j0; ++t) {
      const int k = j0 + t - 1;
      const double* prev = (t == 1) ? Yprev0 : Yseg[t - 2];
      const int64_t ldp = (t == 1) ? ns : ldseg[t - 2];
      StepIO io{Yseg[t - 1], ldseg[t - 1], true, prev, ldp, true, b.seg[t], ns, true};
      CHEFSI_TRY(launch_step(p, b.panel, CHEFSI_F64, b.coef + 3 * k, io, ns, st));
      Yseg[t] = b.seg[t];
      ldseg[t] = ns;
    }
    for (int j = j1 - 1; j >= j0; --j) {
      CHEFSI_TRY(sddmm_accumulate(p, lam1, ns, Yseg[j - j0], ldseg[j - j0], ns, 1.0, b.coef + 3 * j, Hbar, st));
      double* out = lam2 ? lam2 : (lam1 == b.LA ? b.LB : b.LA);
      StepIO io{lam1, ns, true, lam2, ns, true, out, ns, true};
      CHEFSI_TRY(launch_step(p, b.panelT, CHEFSI_F64, b.rcoef + 3 * j, io, ns, st));
      lam2 = lam1;
      lam1 = out;
    }
  }
  return launch_copy_f64(lam1, ns, Xbar, ldxb, p.N, ns, st);
}

int validate_bwd_common(Plan& p, int m, double a, double bb, double a0, int ns, int ckpt_stride) {
  if (m < 0 || m > kMaxDegree) return fail(CHEFSI_ERR_ARG, "filter degree must be in [0, 100000]");
  if (ns < 1 || ns > p.N) return fail(CHEFSI_ERR_ARG, "ns must be in [1, N]");
  if (m > 0 && (ckpt_stride < 1 || ckpt_stride > m)) return fail(CHEFSI_ERR_ARG, "ckpt_stride must be in [1, m]");
  return validate_bounds(a, bb, a0);
}

// Adjoint of the thin QR Y = Yhat U (U upper with positive diagonal) with
// R_bar = 0, in place on G (Yhat_bar on entry, Y_bar on exit):
//   M = -G^T Yhat,  G <- (G + Yhat copyltu(M)) U^{-T},
// copyltu(M) = tril(M) + tril(M, -1)^T.  M, Lt: ns x ns scratch.
int run_qr_backward(int64_t n, int ns, const double* Yh, int64_t ldy, const double* U, double* G, int64_t ldg,
                    double* M, double* Lt, double* split, size_t split_elems, hipStream_t st) {
  CHEFSI_TRY(gemm_tn(ns, ns, n, -1.0, G, ldg, Yh, ldy, 0.0, M, ns, false, split, split_elems, st));
  CHEFSI_TRY(launch_symmetrize(M, ns, ns, 2, st));
  CHEFSI_TRY(gemm_nn(n, ns, ns, 1.0, Yh, ldy, M, ns, 1.0, G, ldg, st));
  CHEFSI_TRY(launch_transpose(U, ns, Lt, ns, ns, ns, st));
  return trsm_right_lower(G, ldg, n, Lt, ns, ns, st);
}

// Adjoint of Hhat = sym(Yhat^T H Yhat) and Hhat Q = Q diag(theta) for the
// Ritz-value cotangent theta_bar: Hhat_bar = Q diag(theta_bar) Q^T,
// YH = Yhat Hhat_bar, G = H YH + H^T YH (into G, ld ldg) and
// Hbar += YH Yhat^T on the stored blocks.  Q: ns x ns row-major (column j =
// eigenvector j); QT, QD, Hhb: ns x ns scratch; YH: N x ns scratch;
// cconst: the constant coefficients (1, 0, 0) and, 4 doubles on, (1, -1, 0).
int run_rr_backward(const Plan& p, const double* panel, const double* panelT, const double* cconst,
                    const double* Yh, int64_t ldy, int ns, const double* Q, const double* theta_bar,
                    double* QT, double* QD, double* Hhb, double* YH, double* G, int64_t ldg, double* Hbar,
                    hipStream_t st) {
  CHEFSI_TRY(launch_transpose(Q, ns, QT, ns, ns, ns, st));
  CHEFSI_TRY(launch_transpose(QT, ns, QD, ns, ns, ns, st, theta_bar));   // Q diag(theta_bar)
  CHEFSI_TRY(gemm_nn(ns, ns, ns, 1.0, QD, ns, QT, ns, 0.0, Hhb, ns, st));
  CHEFSI_TRY(gemm_nn(p.N, ns, ns, 1.0, Yh, ldy, Hhb, ns, 0.0, YH, ns, st));
  StepIO io{YH, ns, true, nullptr, 0, true, G, ldg, true};
  CHEFSI_TRY(launch_step(p, panel, CHEFSI_F64, cconst, io, ns, st));
  StepIO io2{YH, ns, true, G, ldg, true, G, ldg, true};
  CHEFSI_TRY(launch_step(p, panelT, CHEFSI_F64, cconst + 4, io2, ns, st));
  return sddmm_accumulate(p, YH, ns, Yh, ldy, ns, 1.0, nullptr, Hbar, st);
}

// Forward of the differentiated pass, as the adjoint sees it: the filter with
// checkpoints every `stride` steps (none when b.ckY is empty), `passes`
// Cholesky-QR passes with their factors kept (Qp[pass] = output of the pass,
// Up[pass] = its factor), Hhat = sym(Yhat^T H Yhat), its eigenpairs
// (b.theta, b.Q) and the loss sum_{i<k} theta_i (b.loss).  Status words:
// b.status[0] Cholesky, b.status[1] eigensolver.
int loss_forward_dev(Plan& p, const double* d_H, int m, double a, double bb, double a0, int passes, int k,
                     int stride, const double* d_X, int64_t ldx, int ns, BwdWs& w, hipStream_t st) {
  const int64_t N = p.N;
  CHEFSI_TRY(launch_repack(p, d_H, CHEFSI_F64, false, w.panel, st));
  if (w.panelT) CHEFSI_TRY(launch_repack(p, d_H, CHEFSI_F64, true, w.panelT, st));
  CHEFSI_TRY(launch_set_bounds(a, bb, a0, w.bounds, st));
  CHEFSI_TRY(launch_cheb_coef(w.bounds, m, w.coef, st));
  if (m > 0 && w.rcoef) CHEFSI_TRY(launch_rev_coef(w.coef, m, w.rcoef, st));
  CHEFSI_TRY(launch_fill_int(w.status, 2, 0, st));
  const double* Ym = nullptr;
  int64_t ldm = 0;
  CHEFSI_TRY(forward_checkpointed(p, w.panel, w.coef, m, stride, d_X, ldx, ns, w, &Ym, &ldm, st));
  double* Qp[2] = {w.P1, w.P2};
  double* Up[2] = {w.U0, w.U1};
  CHEFSI_TRY(launch_copy_f64(Ym, ldm, w.P1, ns, N, ns, st));
  for (int pass = 0; pass < passes; ++pass) {
    if (pass == 1) CHEFSI_TRY(launch_copy_f64(w.P1, ns, w.P2, ns, N, ns, st));
    double* Y = Qp[pass];
    CHEFSI_TRY(gemm_tn(ns, ns, N, 1.0, Y, ns, Y, ns, 0.0, w.S, ns, true, w.split, w.split_elems, st));
    CHEFSI_TRY(launch_symmetrize(w.S, ns, ns, 1, st));
    CHEFSI_TRY(cholesky_upper(w.S, ns, ns, w.status, w.Mb, st));
    CHEFSI_TRY(trsm_right_upper(Y, ns, N, w.S, ns, ns, st));
    CHEFSI_TRY(launch_copy_f64(w.S, ns, Up[pass], ns, ns, ns, st));
  }
  double* Yh = Qp[passes - 1];
  CHEFSI_TRY(launch_const_coef3(1.0, 0.0, 0.0, w.cconst, st));        // plain H x
  CHEFSI_TRY(launch_const_coef3(1.0, -1.0, 0.0, w.cconst + 4, st));   // H x + prev
  {
    StepIO io{Yh, ns, true, nullptr, 0, true, w.W, ns, true};
    CHEFSI_TRY(launch_step(p, w.panel, CHEFSI_F64, w.cconst, io, ns, st));
  }
  CHEFSI_TRY(gemm_tn(ns, ns, N, 1.0, Yh, ns, w.W, ns, 0.0, w.Hh, ns, false, w.split, w.split_elems, st));
  CHEFSI_TRY(launch_symmetrize(w.Hh, ns, ns, 0, st));
  CHEFSI_TRY(eig_sym(p, w.Hh, ns, ns, w.theta, w.E, w.status + 1, w.Q, w.eig, w.eig_bytes, st));
  CHEFSI_TRY(launch_eigvec_fix(w.Hh, ns, ns, w.Q, ns, st));
  return launch_sum_first(w.theta, k, w.loss, st);
}

int read_loss_status(const BwdWs& w, double* h_loss, hipStream_t st) {
  double hl = 0.0;
  int hs[2] = {0, 0};
  CHEFSI_HIP(hipMemcpyAsync(&hl, w.loss, sizeof(double), hipMemcpyDeviceToHost, st));
  CHEFSI_HIP(hipMemcpyAsync(hs, w.status, 2 * sizeof(int), hipMemcpyDeviceToHost, st));
  CHEFSI_HIP(hipStreamSynchronize(st));
  if (h_loss) *h_loss = hl;
  if (hs[0] != 0) return chol_fail(hs[0]);
  if (hs[1] < 0) return fail(CHEFSI_ERR_NONFINITE, "the projected matrix is not finite");
  if (hs[1] != 0) return fail(CHEFSI_ERR_EIG, "dense eigensolver did not converge");
  return CHEFSI_OK;
}

struct QrBwdWs {
  double* M;
  double* Lt;
  double* split;
  size_t split_elems;
};

void carve_qr_bwd(Carver& c, int64_t n, int ns, QrBwdWs& q) {
  const int64_t nn = static_cast<int64_t>(ns) * ns;
  q.M = c.take<double>(nn);
  q.Lt = c.take<double>(nn);
  q.split_elems = gemm_tn_split_ws_elems(ns, ns, n);
  q.split = q.split_elems ? c.take<double>(static_cast<int64_t>(q.split_elems)) : nullptr;
}

struct RrBwdWs {
  double* panel;
  double* panelT;
  double* cconst;
  double* QT;
  double* QD;
  double* Hhb;
  double* YH;
};

void carve_rr_bwd(Carver& c, const Plan& p, int ns, RrBwdWs& r) {
  const int64_t nn = static_cast<int64_t>(ns) * ns;
  r.panel = c.take<double>(p.panel_elems);
  r.panelT = c.take<double>(p.panel_elems);
  r.cconst = c.take<double>(8);
  r.QT = c.take<double>(nn);
  r.QD = c.take<double>(nn);
  r.Hhb = c.take<double>(nn);
  r.YH = c.take<double>(p.N * static_cast<int64_t>(ns));
}

}  // namespace
}  // namespace chefsi

using namespace chefsi;

// ====================================================================== ABI
extern "C" {

const char* chefsi_version(void) { return "chefsi-gfx950 1.0"; }

const char* chefsi_last_error(void) { return g_err.c_str(); }

int chefsi_plan_create(chefsi_plan* out, int nx, int ny, int nz, int stencil, const int32_t* alb_counts) {
  return guarded([&]() -> int {
    if (out == nullptr) return fail(CHEFSI_ERR_ARG, "out is NULL");
    *out = nullptr;
    if (nx < 1 || ny < 1 || nz < 1) return fail(CHEFSI_ERR_ARG, "grid dimensions must be >= 1");
    const int64_t M64 = static_cast<int64_t>(nx) * ny * nz;
    if (M64 > (1 << 22)) return fail(CHEFSI_ERR_ARG, "too many elements");
    if (stencil != 5 && stencil != 7) return fail(CHEFSI_ERR_ARG, "stencil must be 5 or 7");
    if (alb_counts == nullptr) return fail(CHEFSI_ERR_ARG, "alb_counts is NULL");
    const int M = static_cast<int>(M64);
    for (int K = 0; K < M; ++K)
      if (alb_counts[K] < 1 || alb_counts[K] > kMaxJ)
        return fail(CHEFSI_ERR_ARG, "alb_counts[" + std::to_string(K) + "] must be in [1, 256]");

    Plan* p = new Plan();
    p->nx = nx;
    p->ny = ny;
    p->nz = nz;
    p->stencil = stencil;
    p->M = M;
    const int S = stencil;
    p->J.assign(alb_counts, alb_counts + M);
    p->rowoff.assign(M + 1, 0);
    for (int K = 0; K < M; ++K) p->rowoff[K + 1] = p->rowoff[K] + p->J[K];
    p->N = p->rowoff[M];
    if (p->N >= (int64_t(1) << 31)) {
      delete p;
      return fail(CHEFSI_ERR_ARG, "N must be < 2^31");
    }
    static const int dirs[7][3] = {{0, 0, 0}, {-1, 0, 0}, {1, 0, 0}, {0, -1, 0}, {0, 1, 0}, {0, 0, -1}, {0, 0, 1}};
    p->nbr.resize(static_cast<size_t>(M) * S);
    for (int K = 0; K < M; ++K) {
      const int ix = K % nx, iy = (K / nx) % ny, iz = K / (nx * ny);
      for (int s = 0; s < S; ++s) {
        const int jx = ((ix + dirs[s][0]) % nx + nx) % nx;
        const int jy = ((iy + dirs[s][1]) % ny + ny) % ny;
        const int jz = ((iz + dirs[s][2]) % nz + nz) % nz;
        p->nbr[static_cast<size_t>(K) * S + s] = jx + nx * (jy + ny * jz);
      }
    }
    p->hoff.resize(static_cast<size_t>(M) * S);
    p->ktot.resize(M);
    p->kpad.resize(M);
    p->rb.resize(M);
    p->poff.resize(M);
    p->koff.resize(M);
    int64_t h = 0, po = 0, ko = 0;
    p->maxJ = 0;
    p->maxRB = 0;
    p->uniform = true;
    for (int K = 0; K < M; ++K) {
      int kt = 0;
      for (int s = 0; s < S; ++s) {
        const int Kp = p->nbr[static_cast<size_t>(K) * S + s];
        p->hoff[static_cast<size_t>(K) * S + s] = h;
        h += static_cast<int64_t>(p->J[K]) * p->J[Kp];
        kt += p->J[Kp];
      }
      p->ktot[K] = kt;
      p->kpad[K] = static_cast<int32_t>(round_up(kt, kStepKC));
      p->rb[K] = static_cast<int32_t>(ceil_div(p->J[K], 16));
      p->poff[K] = po;
      po += static_cast<int64_t>(p->kpad[K]) * p->rb[K] * 16;
      p->koff[K] = ko;
      ko += p->kpad[K];
      p->maxJ = std::max(p->maxJ, p->J[K]);
      p->maxRB = std::max(p->maxRB, static_cast<int>(p->rb[K]));
      if (p->rb[K] != p->rb[0]) p->uniform = false;
    }
    p->h_elems = h;
    p->panel_elems = po;
    p->kmap_len = ko;
    std::vector<int32_t> kmap(static_cast<size_t>(ko), -1);
    for (int K = 0; K < M; ++K) {
      int k = 0;
      for (int s = 0; s < S; ++s) {
        const int Kp = p->nbr[static_cast<size_t>(K) * S + s];
        for (int r = 0; r < p->J[Kp]; ++r) kmap[p->koff[K] + k++] = static_cast<int32_t>(p->rowoff[Kp] + r);
      }
    }
    // BF16 layout: element rows padded to multiples of 8
    p->rowoff8.assign(M + 1, 0);
    for (int K = 0; K < M; ++K) p->rowoff8[K + 1] = p->rowoff8[K] + round_up(p->J[K], 8);
    p->N8 = p->rowoff8[M];
    p->kpad8.assign(M, 0);
    p->poff8.assign(M, 0);
    p->kgoff.assign(M, 0);
    int64_t po8 = 0, kg = 0;
    for (int K = 0; K < M; ++K) {
      int kt8 = 0;
      for (int s = 0; s < S; ++s) kt8 += static_cast<int>(round_up(p->J[p->nbr[static_cast<size_t>(K) * S + s]], 8));
      p->kpad8[K] = static_cast<int32_t>(round_up(kt8, kPadK));
      p->poff8[K] = po8;
      po8 += static_cast<int64_t>(p->kpad8[K]) * p->rb[K] * 16;
      p->kgoff[K] = kg;
      kg += p->kpad8[K] / 8;
    }
    p->panel8_elems = po8;
    std::vector<int32_t> kg8(static_cast<size_t>(kg), -1);
    for (int K = 0; K < M; ++K) {
      int64_t g = p->kgoff[K];
      for (int s = 0; s < S; ++s) {
        const int Kp = p->nbr[static_cast<size_t>(K) * S + s];
        const int J8 = static_cast<int>(round_up(p->J[Kp], 8));
        for (int r = 0; r < J8; r += 8) kg8[g++] = static_cast<int32_t>((p->rowoff8[Kp] + r) / 8);
      }
    }
    std::vector<int32_t> rowsrc8(static_cast<size_t>(p->N8), -1);
    for (int K = 0; K < M; ++K)
      for (int i = 0; i < p->J[K]; ++i) rowsrc8[p->rowoff8[K] + i] = static_cast<int32_t>(p->rowoff[K] + i);
    if (p->N8 > 0x7fffffff) {
      delete p;
      return fail(CHEFSI_ERR_ARG, "plan_create: too many rows");
    }
    // Element processing order of the step kernels.  Consecutive work-groups
    // of one XCD take consecutive entries, so a compact traversal keeps the
    // neighbour rows they gather in that XCD's L2: columns of BX x BY
    // elements, walked z-slab by z-slab.
#ifndef CHEFSI_ELEM_ORDER
#define CHEFSI_ELEM_ORDER 1
#endif
    std::vector<int32_t> order;
    order.reserve(M);
    if (CHEFSI_ELEM_ORDER >= 1) {
#ifndef CHEFSI_ORDER_BX
#define CHEFSI_ORDER_BX 4
#endif
#ifndef CHEFSI_ORDER_BY
#define CHEFSI_ORDER_BY 4
#endif
      const int BX = std::min(nx, CHEFSI_ORDER_BX), BY = std::min(ny, CHEFSI_ORDER_BY);
      for (int by = 0; by < ny; by += BY)
        for (int bx = 0; bx < nx; bx += BX)
          for (int z = 0; z < nz; ++z)
            for (int y = by; y < std::min(ny, by + BY); ++y)
              for (int x = bx; x < std::min(nx, bx + BX); ++x) order.push_back(x + nx * (y + ny * z));
    } else {
      order.resize(M);
      std::iota(order.begin(), order.end(), 0);
    }
    // mixed block sizes: grouped by row-block count (one launch per group),
    // the walk order kept within a group
    if (!p->uniform)
      std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return p->rb[x] > p->rb[y]; });
    for (int e = 0; e < M; ++e) {
      const int rb = p->rb[order[e]];
      if (p->grp_rb.empty() || p->grp_rb.back() != rb) {
        p->grp_rb.push_back(rb);
        p->grp_start.push_back(e);
        p->grp_count.push_back(0);
      }
      ++p->grp_count.back();
    }
    p->sqoff.assign(M + 1, 0);
    for (int K = 0; K < M; ++K) p->sqoff[K + 1] = p->sqoff[K] + static_cast<int64_t>(p->J[K]) * p->J[K];
    p->sqtot = p->sqoff[M];
#ifdef CHEFSI_DEBUG
    {
      const int rc = verify_plan_tables(*p, kmap, kg8, rowsrc8, order);
      if (rc != CHEFSI_OK) {
        delete p;
        return rc;
      }
    }
#endif
    if (hipGetDevice(&p->device) != hipSuccess) {
      delete p;
      return fail(CHEFSI_ERR_HIP, "hipGetDevice failed (no GPU?)");
    }
    // set-up of the allocation-free filter: this device's scratch address
    p->scratch = scratch_address(p->device);
    auto up = [&](auto** dst, const auto& vec) -> int {
      using T = typename std::remove_reference<decltype(vec)>::type::value_type;
      const size_t bytes = std::max<size_t>(vec.size(), 1) * sizeof(T);
      if (hipMalloc(reinterpret_cast<void**>(dst), bytes) != hipSuccess) return CHEFSI_ERR_HIP;
      if (!vec.empty() && hipMemcpy(*dst, vec.data(), vec.size() * sizeof(T), hipMemcpyHostToDevice) != hipSuccess)
        return CHEFSI_ERR_HIP;
      return CHEFSI_OK;
    };
    int rc = CHEFSI_OK;
    rc |= up(&p->d_J, p->J);
    rc |= up(&p->d_nbr, p->nbr);
    rc |= up(&p->d_rb, p->rb);
    rc |= up(&p->d_kpad, p->kpad);
    rc |= up(&p->d_order, order);
    rc |= up(&p->d_rowoff, p->rowoff);
    rc |= up(&p->d_hoff, p->hoff);
    rc |= up(&p->d_poff, p->poff);
    rc |= up(&p->d_koff, p->koff);
    rc |= up(&p->d_kmap, kmap);
    rc |= up(&p->d_rowoff8, p->rowoff8);
    rc |= up(&p->d_poff8, p->poff8);
    rc |= up(&p->d_kpad8, p->kpad8);
    rc |= up(&p->d_kgoff, p->kgoff);
    rc |= up(&p->d_kg8, kg8);
    rc |= up(&p->d_rowsrc8, rowsrc8);
    rc |= up(&p->d_sqoff, p->sqoff);
    if (rc != CHEFSI_OK) {
      chefsi_plan_destroy(reinterpret_cast<chefsi_plan>(p));
      return fail(CHEFSI_ERR_HIP, "plan_create: device table upload failed");
    }
    *out = reinterpret_cast<chefsi_plan>(p);
    return CHEFSI_OK;
  });
}

void chefsi_plan_destroy(chefsi_plan plan) {
  if (plan == nullptr) return;
  Plan* p = P(plan);
  void* ptrs[] = {p->d_J, p->d_nbr, p->d_rb, p->d_kpad, p->d_order, p->d_rowoff,
                  p->d_hoff, p->d_poff, p->d_koff, p->d_kmap, p->d_kslot, p->d_rowoff8,
                  p->d_poff8, p->d_kpad8, p->d_kgoff, p->d_kg8, p->d_rowsrc8, p->d_sqoff};
  for (void* q : ptrs)
    if (q) (void)hipFree(q);
  destroy_eig_handle(*p);
  delete p;
}

int64_t chefsi_plan_n(chefsi_plan plan) { return plan ? P(plan)->N : -1; }

int64_t chefsi_plan_h_elems(chefsi_plan plan) { return plan ? P(plan)->h_elems : -1; }

int64_t chefsi_plan_block_elems(chefsi_plan plan) { return plan ? P(plan)->sqtot : -1; }

int chefsi_plan_neighbour(chefsi_plan plan, int K, int s) {
  if (!plan) return -1;
  const Plan* p = P(plan);
  if (K < 0 || K >= p->M || s < 0 || s >= p->stencil) return -1;
  return p->nbr[static_cast<size_t>(K) * p->stencil + s];
}

int chefsi_workspace_bytes(chefsi_plan plan, int op, int ns, int dtype, int passes, int lanczos_steps,
                           size_t* bytes) {
  return guarded([&]() -> int {
    if (plan == nullptr || bytes == nullptr) return fail(CHEFSI_ERR_ARG, "plan/bytes is NULL");
    if (ns < 0) return fail(CHEFSI_ERR_ARG, "ns must be >= 0");
    Plan& p = *P(plan);
    *bytes = 0;
    switch (op) {
      case CHEFSI_OP_BOUNDS: {
        if (lanczos_steps < 1 || lanczos_steps > kMaxLanczos)
          return fail(CHEFSI_ERR_ARG, "lanczos_steps must be in [1, 64]");
        Carver c(nullptr, 0);
        c.take<double>(p.panel_elems);
        c.take<double>(8);
        *bytes = c.used + lanczos_ws_bytes(p, lanczos_steps);
        return CHEFSI_OK;
      }
      case CHEFSI_OP_FILTER: {
        if (!valid_dtype(dtype)) return fail(CHEFSI_ERR_ARG, "bad dtype");
        Carver c(nullptr, 0);
        FilterWs f;
        carve_filter(c, p, ns, dtype, true, f);
        *bytes = c.used;
        return CHEFSI_OK;
      }
      case CHEFSI_OP_ORTHONORMALIZE: {
        Carver c(nullptr, 0);
        OrthWs o;
        carve_orth(c, p.N, ns, o);
        *bytes = c.used;
        return CHEFSI_OK;
      }
      case CHEFSI_OP_RAYLEIGH_RITZ: {
        Carver c(nullptr, 0);
        RrWs r;
        CHEFSI_TRY(carve_rr(c, p, ns, true, r));
        *bytes = c.used;
        return CHEFSI_OK;
      }
      case CHEFSI_OP_DENSITY: {
        Carver c(nullptr, 0);
        c.take<double>(static_cast<int64_t>(elem_nt_slices(p, ns)) * p.sqtot);
        *bytes = c.used;
        return CHEFSI_OK;
      }
      case CHEFSI_OP_RAYLEIGH_RITZ_BACKWARD: {
        Carver c(nullptr, 0);
        RrBwdWs r;
        carve_rr_bwd(c, p, ns, r);
        *bytes = c.used;
        return CHEFSI_OK;
      }
      case CHEFSI_OP_SWEEP: {
        if (!valid_dtype(dtype)) return fail(CHEFSI_ERR_ARG, "bad dtype");
        if (lanczos_steps < 1 || lanczos_steps > kMaxLanczos)
          return fail(CHEFSI_ERR_ARG, "lanczos_steps must be in [1, 64]");
        if (passes < 0 || passes > 2) return fail(CHEFSI_ERR_ARG, "passes must be 0 (auto), 1 or 2");
        *bytes = sweep_bytes(p, ns, dtype, lanczos_steps, passes);
        return CHEFSI_OK;
      }
      default:
        return fail(CHEFSI_ERR_UNSUPPORTED, "unknown op");
    }
  });
}

int chefsi_bounds(chefsi_plan plan, const double* d_H, const double* d_v0, int lanczos_steps,
                  const double* d_ritz_prev, int ns, double* d_bounds, double* h_bounds, void* ws,
                  size_t ws_bytes, void* stream) {
  return guarded([&]() -> int {
    if (plan == nullptr) return fail(CHEFSI_ERR_ARG, "plan is NULL");
    Plan& p = *P(plan);
    if (d_H == nullptr || d_v0 == nullptr) return fail(CHEFSI_ERR_ARG, "H or v0 is NULL");
    if (lanczos_steps < 1 || lanczos_steps > kMaxLanczos)
      return fail(CHEFSI_ERR_ARG, "lanczos_steps must be in [1, 64]");
    if (ns < 1 || ns > p.N) return fail(CHEFSI_ERR_ARG, "ns must be in [1, N]");
    size_t need = 0;
    CHEFSI_TRY(chefsi_workspace_bytes(plan, CHEFSI_OP_BOUNDS, ns, 0, 1, lanczos_steps, &need));
    CHEFSI_TRY(check_ws(ws, ws_bytes, need));
    CHEFSI_TRY(check_device(p));
    hipStream_t st = static_cast<hipStream_t>(stream);
    Carver c(ws, ws_bytes);
    double* panel = c.take<double>(p.panel_elems);
    double* bnd = c.take<double>(8);
    CHEFSI_TRY(launch_repack(p, d_H, CHEFSI_F64, false, panel, st));
    CHEFSI_TRY(lanczos_bounds(p, panel, d_v0, lanczos_steps, d_ritz_prev, ns, bnd,
                              static_cast<char*>(ws) + c.used, ws_bytes - c.used, st));
    if (d_bounds) CHEFSI_HIP(hipMemcpyAsync(d_bounds, bnd, 3 * sizeof(double), hipMemcpyDeviceToDevice, st));
    double hb[3];
    CHEFSI_HIP(hipMemcpyAsync(hb, bnd, 3 * sizeof(double), hipMemcpyDeviceToHost, st));
    CHEFSI_HIP(hipStreamSynchronize(st));
    if (h_bounds) std::memcpy(h_bounds, hb, sizeof(hb));
    if (!std::isfinite(hb[0]) || !std::isfinite(hb[1]) || !std::isfinite(hb[2]))
      return fail(CHEFSI_ERR_NONFINITE, "bounds are not finite");
    if (!(hb[2] < hb[0] && hb[0] < hb[1]))
      return fail(CHEFSI_ERR_ARG, "bounds violate a0 < a < b (previous Ritz values above the upper bound?)");
    return CHEFSI_OK;
  });
}

int chefsi_filter(chefsi_plan plan, const double* d_H, int m, double a, double b, double a0, int dtype,
                  const double* d_X, int64_t ldx, double* d_Y, int64_t ldy, int ns, void* ws,
                  size_t ws_bytes, void* stream) {
  return guarded([&]() -> int {
    if (plan == nullptr) return fail(CHEFSI_ERR_ARG, "plan is NULL");
    Plan& p = *P(plan);
    if (d_H == nullptr) return fail(CHEFSI_ERR_ARG, "H is NULL");
    if (m < 0 || m > kMaxDegree) return fail(CHEFSI_ERR_ARG, "filter degree must be in [0, 100000]");
    if (!valid_dtype(dtype)) return fail(CHEFSI_ERR_ARG, "bad dtype");
    if (ns < 0) return fail(CHEFSI_ERR_ARG, "ns must be >= 0");
    CHEFSI_TRY(validate_bounds(a, b, a0));
    CHEFSI_TRY(validate_mv("X", d_X, ldx, ns));
    CHEFSI_TRY(validate_mv("Y", d_Y, ldy, ns));
    if (ns > 0 && overlaps(d_X, mv_bytes(p.N, ldx, ns, 8), d_Y, mv_bytes(p.N, ldy, ns, 8)))
      return fail(CHEFSI_ERR_ARG, "X and Y overlap");
    size_t need = 0;
    CHEFSI_TRY(chefsi_workspace_bytes(plan, CHEFSI_OP_FILTER, ns, dtype, 1, 1, &need));
    CHEFSI_TRY(check_ws(ws, ws_bytes, need));
    if (ns == 0) return CHEFSI_OK;
    CHEFSI_TRY(check_device(p));
    hipStream_t st = static_cast<hipStream_t>(stream);
    Carver c(ws, ws_bytes);
    FilterWs f;
    carve_filter(c, p, ns, dtype, true, f);
    CHEFSI_TRY(launch_set_bounds(a, b, a0, f.bounds, st));
    CHEFSI_TRY(launch_cheb_coef(f.bounds, m, f.coef, st));
    if (m > 0) CHEFSI_TRY(launch_repack(p, d_H, dtype, false, f.panel, st, f.coef + 2));
    return run_filter(p, f.panel, dtype, f.coef, m, d_X, ldx, d_Y, ldy, ns, f, st);
  });
}

int chefsi_filter_noalloc(chefsi_plan plan, const double* d_H, int m, double a, double b, double a0, int dtype,
                          const double* d_X, int64_t ldx, double* d_Y, int64_t ldy, int ns, void* stream) {
  return guarded([&]() -> int {
    if (plan == nullptr) return fail(CHEFSI_ERR_ARG, "plan is NULL");
    Plan& p = *P(plan);
    if (!valid_dtype(dtype)) return fail(CHEFSI_ERR_ARG, "bad dtype");
    if (ns < 0) return fail(CHEFSI_ERR_ARG, "ns must be >= 0");
    size_t need = 0;
    CHEFSI_TRY(chefsi_workspace_bytes(plan, CHEFSI_OP_FILTER, ns, dtype, 1, 1, &need));
    if (need > kNoallocScratchBytes)
      return fail(CHEFSI_ERR_WORKSPACE, "filter_noalloc: the filter needs " + std::to_string(need) +
                                            " bytes of scratch, more than the library's " +
                                            std::to_string(kNoallocScratchBytes) + " (use chefsi_filter)");
    if (p.scratch == nullptr) return fail(CHEFSI_ERR_HIP, "filter_noalloc: the device scratch is unavailable");
    // every other check, and the filter itself, as chefsi_filter
    return chefsi_filter(plan, d_H, m, a, b, a0, dtype, d_X, ldx, d_Y, ldy, ns, p.scratch, kNoallocScratchBytes,
                         stream);
  });
}

int chefsi_orthonormalize(int64_t n, int ns, double* d_Y, int64_t ldy, int passes, double* d_U, void* ws,
                          size_t ws_bytes, void* stream) {
  return guarded([&]() -> int {
    if (n < 1 || ns < 1) return fail(CHEFSI_ERR_ARG, "n and ns must be >= 1");
    if (ns > n) return fail(CHEFSI_ERR_ARG, "ns must be <= n");
    if (passes < 0 || passes > 2) return fail(CHEFSI_ERR_ARG, "passes must be 0 (auto), 1 or 2");
    CHEFSI_TRY(validate_mv("Y", d_Y, ldy, ns));
    if (d_U && overlaps(d_U, static_cast<size_t>(ns) * ns * 8, d_Y, mv_bytes(n, ldy, ns, 8)))
      return fail(CHEFSI_ERR_ARG, "U and Y overlap");
    Carver dry(nullptr, 0);
    OrthWs o;
    carve_orth(dry, n, ns, o);
    CHEFSI_TRY(check_ws(ws, ws_bytes, dry.used));
    hipStream_t st = static_cast<hipStream_t>(stream);
    Carver c(ws, ws_bytes);
    carve_orth(c, n, ns, o);
    CHEFSI_TRY(run_orth(n, ns, d_Y, ldy, passes, d_U, o, st));
    int h = 0;
    CHEFSI_HIP(hipMemcpyAsync(&h, o.status, sizeof(int), hipMemcpyDeviceToHost, st));
    CHEFSI_HIP(hipStreamSynchronize(st));
    return h != 0 ? chol_fail(h) : CHEFSI_OK;
  });
}

int chefsi_orthonormalize_workspace_bytes(int64_t n, int ns, int passes, size_t* bytes) {
  return guarded([&]() -> int {
    if (bytes == nullptr) return fail(CHEFSI_ERR_ARG, "bytes is NULL");
    if (n < 1 || ns < 1 || ns > n) return fail(CHEFSI_ERR_ARG, "need 1 <= ns <= n");
    if (passes < 0 || passes > 2) return fail(CHEFSI_ERR_ARG, "passes must be 0 (auto), 1 or 2");
    Carver c(nullptr, 0);
    OrthWs o;
    carve_orth(c, n, ns, o);
    *bytes = c.used;
    return CHEFSI_OK;
  });
}

int chefsi_rayleigh_ritz(chefsi_plan plan, const double* d_H, const double* d_Yhat, int64_t ldy, int ns,
                         double* d_Xnew, int64_t ldx, double* d_ritz, double* d_resid, double* d_Q, void* ws,
                         size_t ws_bytes, void* stream) {
  return guarded([&]() -> int {
    if (plan == nullptr) return fail(CHEFSI_ERR_ARG, "plan is NULL");
    Plan& p = *P(plan);
    if (d_H == nullptr || d_ritz == nullptr) return fail(CHEFSI_ERR_ARG, "H or ritz is NULL");
    if (ns < 1 || ns > p.N) return fail(CHEFSI_ERR_ARG, "ns must be in [1, N]");
    CHEFSI_TRY(validate_mv("Yhat", d_Yhat, ldy, ns));
    CHEFSI_TRY(validate_mv("Xnew", d_Xnew, ldx, ns));
    if (overlaps(d_Yhat, mv_bytes(p.N, ldy, ns, 8), d_Xnew, mv_bytes(p.N, ldx, ns, 8)))
      return fail(CHEFSI_ERR_ARG, "Yhat and Xnew overlap");
    size_t need = 0;
    CHEFSI_TRY(chefsi_workspace_bytes(plan, CHEFSI_OP_RAYLEIGH_RITZ, ns, 0, 1, 1, &need));
    CHEFSI_TRY(check_ws(ws, ws_bytes, need));
    CHEFSI_TRY(check_device(p));
    hipStream_t st = static_cast<hipStream_t>(stream);
    Carver c(ws, ws_bytes);
    RrWs r;
    CHEFSI_TRY(carve_rr(c, p, ns, true, r));
    CHEFSI_TRY(launch_repack(p, d_H, CHEFSI_F64, false, r.panel, st));
    CHEFSI_TRY(run_rr(p, r.panel, d_Yhat, ldy, ns, d_Xnew, ldx, d_ritz, d_resid, d_Q, r, st));
    return read_status(r.info, CHEFSI_ERR_EIG, "dense eigensolver did not converge", st);
  });
}

int chefsi_sweep(chefsi_plan plan, const double* d_H, int m, int filter_dtype, int passes, int lanczos_steps,
                 const double* d_v0, const double* d_bounds_in, int warm, double* d_X, int64_t ldx, int ns,
                 double* d_ritz, double* d_resid, double* d_bounds_out, chefsi_stats* stats, void* ws,
                 size_t ws_bytes, void* stream) {
  return guarded([&]() -> int {
    if (plan == nullptr) return fail(CHEFSI_ERR_ARG, "plan is NULL");
    Plan& p = *P(plan);
    if (d_H == nullptr || d_ritz == nullptr) return fail(CHEFSI_ERR_ARG, "H or ritz is NULL");
    if (m < 0 || m > kMaxDegree) return fail(CHEFSI_ERR_ARG, "filter degree must be in [0, 100000]");
    if (!valid_dtype(filter_dtype)) return fail(CHEFSI_ERR_ARG, "bad dtype");
    if (passes < 0 || passes > 2) return fail(CHEFSI_ERR_ARG, "passes must be 0 (auto), 1 or 2");
    if (ns < 1 || ns > p.N) return fail(CHEFSI_ERR_ARG, "ns must be in [1, N]");
    if (d_bounds_in == nullptr) {
      if (d_v0 == nullptr) return fail(CHEFSI_ERR_ARG, "v0 is NULL and no bounds were given");
      if (lanczos_steps < 1 || lanczos_steps > kMaxLanczos)
        return fail(CHEFSI_ERR_ARG, "lanczos_steps must be in [1, 64]");
    }
    CHEFSI_TRY(validate_mv("X", d_X, ldx, ns));
    const int lk = (lanczos_steps >= 1 && lanczos_steps <= kMaxLanczos) ? lanczos_steps : 1;
    const size_t need = sweep_bytes(p, ns, filter_dtype, lk, passes);
    CHEFSI_TRY(check_ws(ws, ws_bytes, need));
    CHEFSI_TRY(check_device(p));
    hipStream_t st = static_cast<hipStream_t>(stream);

    hipEvent_t ev[6] = {};
    if (stats) {
      for (auto& e : ev) CHEFSI_HIP(hipEventCreate(&e));
    }
    auto mark = [&](int i) -> int {
      if (stats) CHEFSI_HIP(hipEventRecord(ev[i], st));
      return CHEFSI_OK;
    };
    auto run = [&]() -> int {
      Carver c(ws, ws_bytes);
      double* panel64 = c.take<double>(p.panel_elems);
      double* Y = c.take<double>(p.N * static_cast<int64_t>(ns));
      double* bnd = c.take<double>(8);
      int* status = c.take<int>(8);
      double* Tk = c.take<double>(static_cast<int64_t>(ns) * ns);
      double* cond = c.take<double>(8);
      double* cscr = c.take<double>(static_cast<int64_t>(cholqr_cond_scratch_elems(ns)));
      char* rest = static_cast<char*>(ws) + c.used;
      const size_t rest_bytes = ws_bytes - c.used;
      CHEFSI_TRY(mark(0));
      // status words: [0] Cholesky pivot, [1] eigensolver, [2] bounds
      CHEFSI_TRY(launch_fill_int(status, 3, 0, st));
      CHEFSI_TRY(launch_repack(p, d_H, CHEFSI_F64, false, panel64, st));
      // step 1: bounds
      if (d_bounds_in && warm) {
        // the upper bound b is fixed per H: taken from the given bounds, with
        // a and a0 from the previous Ritz values
        CHEFSI_TRY(launch_warm_bounds(d_ritz, ns, d_bounds_in, bnd, st));
      } else if (d_bounds_in) {
        CHEFSI_HIP(hipMemcpyAsync(bnd, d_bounds_in, 3 * sizeof(double), hipMemcpyDeviceToDevice, st));
      } else {
        CHEFSI_TRY(lanczos_bounds(p, panel64, d_v0, lanczos_steps, warm ? d_ritz : nullptr, ns, bnd, rest,
                                  rest_bytes, st));
      }
      CHEFSI_TRY(launch_check_bounds(bnd, status + 2, st));
      CHEFSI_TRY(mark(1));
      // step 2: filter
      {
        Carver cf(rest, rest_bytes);
        FilterWs f;
        carve_filter(cf, p, ns, filter_dtype, true, f);
        CHEFSI_TRY(launch_cheb_coef(bnd, m, f.coef, st));
        // the filter's own panel carries H - cI (c of this call's bounds)
        if (m > 0) CHEFSI_TRY(launch_repack(p, d_H, filter_dtype, false, f.panel, st, f.coef + 2));
        const void* fpanel = f.panel;
        CHEFSI_TRY(mark(2));
        CHEFSI_TRY(run_filter(p, fpanel, filter_dtype, f.coef, m, d_X, ldx, Y, ns, ns, f, st));
      }
      CHEFSI_TRY(mark(3));
      // step 3: Cholesky-QR.  The first factor's condition bound decides the
      // pass count when passes = 0; the last factor's inverse stays in Tk and
      // is folded into Rayleigh-Ritz.
      int used = passes;
      double hcond = 0.0;
      size_t orth_used = 0;
      double* Y1 = nullptr;   // Yhat1 = Y U1^{-1} when a second pass runs
      {
        Carver co(rest, rest_bytes);
        OrthWs o;
        carve_orth(co, p.N, ns, o);
        orth_used = co.used;
        o.status = status;
        CHEFSI_TRY(run_orth_factor1(p.N, ns, Y, ns, Tk, o, st));
        CHEFSI_TRY(cholqr_cond_bound(o.S, Tk, ns, cscr, cond, st));
        if (passes == 0) {
          int hs0[3] = {0, 0, 0};
          CHEFSI_HIP(hipMemcpyAsync(&hcond, cond, sizeof(double), hipMemcpyDeviceToHost, st));
          CHEFSI_HIP(hipMemcpyAsync(hs0, status, 3 * sizeof(int), hipMemcpyDeviceToHost, st));
          CHEFSI_HIP(hipStreamSynchronize(st));
          // the host has synchronised anyway: stop here if the bounds or the
          // factor failed (d_X is untouched so far)
          if (hs0[2] == 1) return fail(CHEFSI_ERR_NONFINITE, "filter bounds are not finite");
          if (hs0[2] != 0)
            return fail(CHEFSI_ERR_ARG, "filter bounds violate a0 < a < b (previous Ritz values above the upper bound?)");
          if (hs0[0] != 0) return chol_fail(hs0[0]);
          used = auto_passes_from_bound(hcond);
        }
        if (used == 2) {
          Y1 = o.B;
          CHEFSI_TRY(run_orth_pass2(p.N, ns, Y, ns, Tk, Y1, ns, o, st));
        }
      }
      CHEFSI_TRY(mark(4));
      // steps 4-5: Rayleigh-Ritz and rotation
      {
        // after a second pass the carving starts behind Cholesky-QR's, which
        // holds Yhat1
        const size_t off = (used == 2) ? orth_used : 0;
        Carver cr(rest + off, rest_bytes - off);
        RrWs r;
        CHEFSI_TRY(carve_rr(cr, p, ns, false, r));
        if (!cr.ok()) return fail(CHEFSI_ERR_WORKSPACE, "sweep: workspace too small for two passes");
        r.info = status + 1;
        if (used == 2)
          CHEFSI_TRY(run_rr_fold(p, panel64, Y1, ns, ns, Tk, d_X, ldx, status, d_ritz, d_resid, r, st));
        else
          CHEFSI_TRY(run_rr_fold(p, panel64, Y, ns, ns, Tk, d_X, ldx, status, d_ritz, d_resid, r, st));
      }
      CHEFSI_TRY(mark(5));
      if (d_bounds_out)
        CHEFSI_HIP(hipMemcpyAsync(d_bounds_out, bnd, 3 * sizeof(double), hipMemcpyDeviceToDevice, st));
      int hs[3] = {0, 0, 0};
      CHEFSI_HIP(hipMemcpyAsync(hs, status, 3 * sizeof(int), hipMemcpyDeviceToHost, st));
      if (passes != 0) CHEFSI_HIP(hipMemcpyAsync(&hcond, cond, sizeof(double), hipMemcpyDeviceToHost, st));
      CHEFSI_HIP(hipStreamSynchronize(st));
      if (stats) {
        float t[5];
        for (int i = 0; i < 5; ++i) CHEFSI_HIP(hipEventElapsedTime(&t[i], ev[i], ev[i + 1]));
        float tf = 0.f, tot = 0.f;
        CHEFSI_HIP(hipEventElapsedTime(&tf, ev[1], ev[3]));
        CHEFSI_HIP(hipEventElapsedTime(&tot, ev[0], ev[5]));
        stats->bounds_ms = t[0];
        stats->filter_ms = tf;
        stats->filter_steps_ms = t[2];
        stats->orthonormalize_ms = t[3];
        stats->rayleigh_ritz_ms = t[4];
        stats->total_ms = tot;
        stats->cholqr_passes = used;
        stats->cholqr_cond_bound = hcond;
      }
      if (hs[2] == 1) return fail(CHEFSI_ERR_NONFINITE, "filter bounds are not finite");
      if (hs[2] != 0)
        return fail(CHEFSI_ERR_ARG, "filter bounds violate a0 < a < b (previous Ritz values above the upper bound?)");
      if (hs[0] != 0) return chol_fail(hs[0]);
      if (hs[1] < 0) return fail(CHEFSI_ERR_NONFINITE, "the projected matrix is not finite");
      if (hs[1] != 0) return fail(CHEFSI_ERR_EIG, "dense eigensolver did not converge");
      return CHEFSI_OK;
    };
    int rc = run();
    if (stats)
      for (auto& e : ev)
        if (e) (void)hipEventDestroy(e);
    return rc;
  });
}

int chefsi_backward_workspace_bytes(chefsi_plan plan, int op, int m, int ns, int passes, int ckpt_stride,
                                    size_t* bytes) {
  return guarded([&]() -> int {
    if (plan == nullptr || bytes == nullptr) return fail(CHEFSI_ERR_ARG, "plan/bytes is NULL");
    if (op != CHEFSI_OP_LOSS_BACKWARD && op != CHEFSI_OP_FILTER_BACKWARD && op != CHEFSI_OP_LOSS)
      return fail(CHEFSI_ERR_ARG, "bad op");
    if (passes != 1 && passes != 2) return fail(CHEFSI_ERR_ARG, "passes must be 1 or 2");
    Plan& p = *P(plan);
    if (m < 0 || ns < 1) return fail(CHEFSI_ERR_ARG, "need m >= 0 and ns >= 1");
    const bool loss_only = (op == CHEFSI_OP_LOSS);
    const int stride = loss_only ? std::max(m, 1) : (m > 0 ? std::max(1, std::min(ckpt_stride, m)) : 1);
    Carver c(nullptr, 0);
    BwdWs b;
    CHEFSI_TRY(carve_bwd(c, p, m, ns, passes, stride, op != CHEFSI_OP_FILTER_BACKWARD, b, !loss_only));
    *bytes = c.used;
    return CHEFSI_OK;
  });
}

int chefsi_loss_backward(chefsi_plan plan, const double* d_H, int m, double a, double b, double a0, int passes,
                         int k, int ckpt_stride, const double* d_X, int64_t ldx, int ns, double* d_Hbar,
                         double* d_Xbar, int64_t ldxb, double* h_loss, void* ws, size_t ws_bytes, void* stream) {
  return guarded([&]() -> int {
    if (plan == nullptr) return fail(CHEFSI_ERR_ARG, "plan is NULL");
    Plan& p = *P(plan);
    if (d_H == nullptr || d_Hbar == nullptr) return fail(CHEFSI_ERR_ARG, "H or Hbar is NULL");
    CHEFSI_TRY(validate_bwd_common(p, m, a, b, a0, ns, ckpt_stride));
    if (passes != 1 && passes != 2) return fail(CHEFSI_ERR_ARG, "passes must be 1 or 2");
    if (k < 1 || k > ns) return fail(CHEFSI_ERR_ARG, "k must be in [1, ns]");
    CHEFSI_TRY(validate_mv("X", d_X, ldx, ns));
    CHEFSI_TRY(validate_mv("Xbar", d_Xbar, ldxb, ns));
    if (overlaps(d_X, mv_bytes(p.N, ldx, ns, 8), d_Xbar, mv_bytes(p.N, ldxb, ns, 8)))
      return fail(CHEFSI_ERR_ARG, "X and Xbar overlap");
    const int stride = m > 0 ? ckpt_stride : 1;
    size_t need = 0;
    CHEFSI_TRY(chefsi_backward_workspace_bytes(plan, CHEFSI_OP_LOSS_BACKWARD, m, ns, passes, stride, &need));
    CHEFSI_TRY(check_ws(ws, ws_bytes, need));
    CHEFSI_TRY(check_device(p));
    hipStream_t st = static_cast<hipStream_t>(stream);
    Carver c(ws, ws_bytes);
    BwdWs w;
    CHEFSI_TRY(carve_bwd(c, p, m, ns, passes, stride, true, w));
    const int64_t N = p.N;
    // ---- forward: filter (checkpointed), Cholesky-QR (per-pass factors kept), Rayleigh-Ritz
    CHEFSI_TRY(loss_forward_dev(p, d_H, m, a, b, a0, passes, k, stride, d_X, ldx, ns, w, st));
    double* Qp[2] = {w.P1, w.P2};
    double* Up[2] = {w.U0, w.U1};
    double* Yh = Qp[passes - 1];
    // ---- backward: Rayleigh-Ritz (theta_bar = 1 on the k lowest, 0 above)
    CHEFSI_TRY(launch_fill(w.E, ns, 0.0, st));
    CHEFSI_TRY(launch_fill(w.E, k, 1.0, st));
    CHEFSI_TRY(launch_fill(d_Hbar, p.h_elems, 0.0, st));
    CHEFSI_TRY(run_rr_backward(p, w.panel, w.panelT, w.cconst, Yh, ns, ns, w.Q, w.E, w.QT, w.Lt, w.Hhb, w.YH, w.G,
                               ns, d_Hbar, st));
    // ---- backward: Cholesky-QR passes in reverse
    for (int pass = passes - 1; pass >= 0; --pass)
      CHEFSI_TRY(run_qr_backward(N, ns, Qp[pass], ns, Up[pass], w.G, ns, w.Mb, w.Lt, w.split, w.split_elems, st));
    // ---- backward: filter
    if (m == 0) {
      CHEFSI_TRY(launch_copy_f64(w.G, ns, d_Xbar, ldxb, N, ns, st));
    } else {
      CHEFSI_TRY(launch_copy_f64(w.G, ns, w.LA, ns, N, ns, st));
      CHEFSI_TRY(reverse_sweep(p, m, stride, d_X, ldx, ns, w, d_Hbar, d_Xbar, ldxb, st));
    }
    return read_loss_status(w, h_loss, st);
  });
}

int chefsi_loss(chefsi_plan plan, const double* d_H, int m, double a, double b, double a0, int passes, int k,
                const double* d_X, int64_t ldx, int ns, double* h_loss, void* ws, size_t ws_bytes, void* stream) {
  return guarded([&]() -> int {
    if (plan == nullptr) return fail(CHEFSI_ERR_ARG, "plan is NULL");
    Plan& p = *P(plan);
    if (d_H == nullptr || h_loss == nullptr) return fail(CHEFSI_ERR_ARG, "H or loss is NULL");
    CHEFSI_TRY(validate_bwd_common(p, m, a, b, a0, ns, m > 0 ? m : 1));
    if (passes != 1 && passes != 2) return fail(CHEFSI_ERR_ARG, "passes must be 1 or 2");
    if (k < 1 || k > ns) return fail(CHEFSI_ERR_ARG, "k must be in [1, ns]");
    CHEFSI_TRY(validate_mv("X", d_X, ldx, ns));
    size_t need = 0;
    CHEFSI_TRY(chefsi_backward_workspace_bytes(plan, CHEFSI_OP_LOSS, m, ns, passes, 1, &need));
    CHEFSI_TRY(check_ws(ws, ws_bytes, need));
    CHEFSI_TRY(check_device(p));
    hipStream_t st = static_cast<hipStream_t>(stream);
    Carver c(ws, ws_bytes);
    BwdWs w;
    const int stride = std::max(m, 1);
    CHEFSI_TRY(carve_bwd(c, p, m, ns, passes, stride, true, w, false));
    CHEFSI_TRY(loss_forward_dev(p, d_H, m, a, b, a0, passes, k, stride, d_X, ldx, ns, w, st));
    return read_loss_status(w, h_loss, st);
  });
}

int chefsi_orthonormalize_backward_workspace_bytes(int64_t n, int ns, size_t* bytes) {
  return guarded([&]() -> int {
    if (bytes == nullptr) return fail(CHEFSI_ERR_ARG, "bytes is NULL");
    if (n < 1 || ns < 1 || ns > n) return fail(CHEFSI_ERR_ARG, "need 1 <= ns <= n");
    Carver c(nullptr, 0);
    QrBwdWs q;
    carve_qr_bwd(c, n, ns, q);
    *bytes = c.used;
    return CHEFSI_OK;
  });
}

int chefsi_orthonormalize_backward(int64_t n, int ns, const double* d_Yhat, int64_t ldy, const double* d_U,
                                   const double* d_Yhat_bar, int64_t ldyb, double* d_Y_bar, int64_t ldb, void* ws,
                                   size_t ws_bytes, void* stream) {
  return guarded([&]() -> int {
    if (n < 1 || ns < 1 || ns > n) return fail(CHEFSI_ERR_ARG, "need 1 <= ns <= n");
    if (d_U == nullptr) return fail(CHEFSI_ERR_ARG, "U is NULL");
    CHEFSI_TRY(validate_mv("Yhat", d_Yhat, ldy, ns));
    CHEFSI_TRY(validate_mv("Yhat_bar", d_Yhat_bar, ldyb, ns));
    CHEFSI_TRY(validate_mv("Y_bar", d_Y_bar, ldb, ns));
    const size_t yb = mv_bytes(n, ldy, ns, 8), gb = mv_bytes(n, ldyb, ns, 8), ob = mv_bytes(n, ldb, ns, 8);
    const size_t ub = static_cast<size_t>(ns) * ns * 8;
    if (overlaps(d_Y_bar, ob, d_Yhat, yb) || overlaps(d_Y_bar, ob, d_U, ub))
      return fail(CHEFSI_ERR_ARG, "Y_bar overlaps Yhat or U");
    const bool in_place = (d_Y_bar == d_Yhat_bar);
    if (in_place && ldb != ldyb) return fail(CHEFSI_ERR_ARG, "in place needs ld(Y_bar) == ld(Yhat_bar)");
    if (!in_place && overlaps(d_Y_bar, ob, d_Yhat_bar, gb)) return fail(CHEFSI_ERR_ARG, "Y_bar partially overlaps Yhat_bar");
    size_t need = 0;
    CHEFSI_TRY(chefsi_orthonormalize_backward_workspace_bytes(n, ns, &need));
    CHEFSI_TRY(check_ws(ws, ws_bytes, need));
    hipStream_t st = static_cast<hipStream_t>(stream);
    Carver c(ws, ws_bytes);
    QrBwdWs q;
    carve_qr_bwd(c, n, ns, q);
    if (!in_place) CHEFSI_TRY(launch_copy_f64(d_Yhat_bar, ldyb, d_Y_bar, ldb, n, ns, st));
    return run_qr_backward(n, ns, d_Yhat, ldy, d_U, d_Y_bar, ldb, q.M, q.Lt, q.split, q.split_elems, st);
  });
}

int chefsi_rayleigh_ritz_backward(chefsi_plan plan, const double* d_H, const double* d_Yhat, int64_t ldy, int ns,
                                  const double* d_Q, const double* d_ritz_bar, double* d_Yhat_bar, int64_t ldyb,
                                  double* d_Hbar, int accumulate, void* ws, size_t ws_bytes, void* stream) {
  return guarded([&]() -> int {
    if (plan == nullptr) return fail(CHEFSI_ERR_ARG, "plan is NULL");
    Plan& p = *P(plan);
    if (d_H == nullptr || d_Q == nullptr || d_ritz_bar == nullptr || d_Hbar == nullptr)
      return fail(CHEFSI_ERR_ARG, "H, Q, ritz_bar or Hbar is NULL");
    if (ns < 1 || ns > p.N) return fail(CHEFSI_ERR_ARG, "ns must be in [1, N]");
    CHEFSI_TRY(validate_mv("Yhat", d_Yhat, ldy, ns));
    CHEFSI_TRY(validate_mv("Yhat_bar", d_Yhat_bar, ldyb, ns));
    const size_t ob = mv_bytes(p.N, ldyb, ns, 8), hb = static_cast<size_t>(p.h_elems) * 8;
    const size_t nn8 = static_cast<size_t>(ns) * ns * 8;
    if (overlaps(d_Yhat_bar, ob, d_Yhat, mv_bytes(p.N, ldy, ns, 8)) || overlaps(d_Yhat_bar, ob, d_H, hb) ||
        overlaps(d_Yhat_bar, ob, d_Q, nn8) || overlaps(d_Yhat_bar, ob, d_Hbar, hb) ||
        overlaps(d_Yhat_bar, ob, d_ritz_bar, static_cast<size_t>(ns) * 8))
      return fail(CHEFSI_ERR_ARG, "Yhat_bar overlaps another argument");
    if (overlaps(d_Hbar, hb, d_H, hb) || overlaps(d_Hbar, hb, d_Yhat, mv_bytes(p.N, ldy, ns, 8)) ||
        overlaps(d_Hbar, hb, d_Q, nn8))
      return fail(CHEFSI_ERR_ARG, "Hbar overlaps another argument");
    size_t need = 0;
    CHEFSI_TRY(chefsi_workspace_bytes(plan, CHEFSI_OP_RAYLEIGH_RITZ_BACKWARD, ns, 0, 1, 1, &need));
    CHEFSI_TRY(check_ws(ws, ws_bytes, need));
    CHEFSI_TRY(check_device(p));
    hipStream_t st = static_cast<hipStream_t>(stream);
    Carver c(ws, ws_bytes);
    RrBwdWs r;
    carve_rr_bwd(c, p, ns, r);
    CHEFSI_TRY(launch_repack(p, d_H, CHEFSI_F64, false, r.panel, st));
    CHEFSI_TRY(launch_repack(p, d_H, CHEFSI_F64, true, r.panelT, st));
    CHEFSI_TRY(launch_const_coef3(1.0, 0.0, 0.0, r.cconst, st));
    CHEFSI_TRY(launch_const_coef3(1.0, -1.0, 0.0, r.cconst + 4, st));
    if (!accumulate) CHEFSI_TRY(launch_fill(d_Hbar, p.h_elems, 0.0, st));
    return run_rr_backward(p, r.panel, r.panelT, r.cconst, d_Yhat, ldy, ns, d_Q, d_ritz_bar, r.QT, r.QD, r.Hhb,
                           r.YH, d_Yhat_bar, ldyb, d_Hbar, st);
  });
}

int chefsi_filter_backward(chefsi_plan plan, const double* d_H, int m, double a, double b, double a0,
                           int ckpt_stride, const double* d_X, int64_t ldx, const double* d_Ybar, int64_t ldyb,
                           int ns, double* d_Hbar, double* d_Xbar, int64_t ldxb, void* ws, size_t ws_bytes,
                           void* stream) {
  return guarded([&]() -> int {
    if (plan == nullptr) return fail(CHEFSI_ERR_ARG, "plan is NULL");
    Plan& p = *P(plan);
    if (d_H == nullptr || d_Hbar == nullptr) return fail(CHEFSI_ERR_ARG, "H or Hbar is NULL");
    CHEFSI_TRY(validate_bwd_common(p, m, a, b, a0, ns, ckpt_stride));
    CHEFSI_TRY(validate_mv("X", d_X, ldx, ns));
    CHEFSI_TRY(validate_mv("Ybar", d_Ybar, ldyb, ns));
    CHEFSI_TRY(validate_mv("Xbar", d_Xbar, ldxb, ns));
    if (overlaps(d_Ybar, mv_bytes(p.N, ldyb, ns, 8), d_Xbar, mv_bytes(p.N, ldxb, ns, 8)) ||
        overlaps(d_X, mv_bytes(p.N, ldx, ns, 8), d_Xbar, mv_bytes(p.N, ldxb, ns, 8)))
      return fail(CHEFSI_ERR_ARG, "Xbar overlaps X or Ybar");
    const int stride = m > 0 ? ckpt_stride : 1;
    size_t need = 0;
    CHEFSI_TRY(chefsi_backward_workspace_bytes(plan, CHEFSI_OP_FILTER_BACKWARD, m, ns, 2, stride, &need));
    CHEFSI_TRY(check_ws(ws, ws_bytes, need));
    CHEFSI_TRY(check_device(p));
    hipStream_t st = static_cast<hipStream_t>(stream);
    Carver c(ws, ws_bytes);
    BwdWs w;
    CHEFSI_TRY(carve_bwd(c, p, m, ns, 2, stride, false, w));
    if (m == 0) return launch_copy_f64(d_Ybar, ldyb, d_Xbar, ldxb, p.N, ns, st);
    CHEFSI_TRY(launch_repack(p, d_H, CHEFSI_F64, false, w.panel, st));
    CHEFSI_TRY(launch_repack(p, d_H, CHEFSI_F64, true, w.panelT, st));
    CHEFSI_TRY(launch_set_bounds(a, b, a0, w.bounds, st));
    CHEFSI_TRY(launch_cheb_coef(w.bounds, m, w.coef, st));
    CHEFSI_TRY(launch_rev_coef(w.coef, m, w.rcoef, st));
    const int nseg = static_cast<int>(ceil_div(m, stride));
    const double* Ylast = nullptr;
    int64_t ldl = 0;
    CHEFSI_TRY(forward_checkpointed(p, w.panel, w.coef, (nseg - 1) * stride, stride, d_X, ldx, ns, w, &Ylast,
                                    &ldl, st));
    CHEFSI_TRY(launch_copy_f64(d_Ybar, ldyb, w.LA, ns, p.N, ns, st));
    return reverse_sweep(p, m, stride, d_X, ldx, ns, w, d_Hbar, d_Xbar, ldxb, st);
  });
}

// ------------------------------------------------- steps around the cycle

int chefsi_occupations(int ns, const double* d_ritz, double n_occ, double kT, double* d_f, double* d_mu,
                       void* stream) {
  return guarded([&]() -> int {
    if (ns < 1) return fail(CHEFSI_ERR_ARG, "ns must be >= 1");
    if (d_ritz == nullptr || d_f == nullptr || d_mu == nullptr)
      return fail(CHEFSI_ERR_ARG, "ritz, f or mu is NULL");
    if (!(kT > 0.0) || !std::isfinite(kT)) return fail(CHEFSI_ERR_ARG, "kT must be positive and finite");
    if (!(n_occ > 0.0 && n_occ < static_cast<double>(ns)))
      return fail(CHEFSI_ERR_ARG, "n_occ must lie strictly between 0 and ns");
    const size_t vb = static_cast<size_t>(ns) * sizeof(double);
    if (overlaps(d_mu, sizeof(double), d_ritz, vb) || overlaps(d_mu, sizeof(double), d_f, vb))
      return fail(CHEFSI_ERR_ARG, "mu overlaps ritz or f");
    if (d_f != d_ritz && overlaps(d_f, vb, d_ritz, vb))
      return fail(CHEFSI_ERR_ARG, "f partially overlaps ritz");
    return launch_fermi(d_ritz, ns, n_occ, kT, d_f, d_mu, static_cast<hipStream_t>(stream));
  });
}

int chefsi_density_blocks(chefsi_plan plan, const double* d_X, int64_t ldx, int ns, const double* d_f,
                          double* d_P, void* ws, size_t ws_bytes, void* stream) {
  return guarded([&]() -> int {
    if (plan == nullptr) return fail(CHEFSI_ERR_ARG, "plan is NULL");
    Plan& p = *P(plan);
    if (ns < 0) return fail(CHEFSI_ERR_ARG, "ns must be >= 0");
    if (d_P == nullptr) return fail(CHEFSI_ERR_ARG, "P is NULL");
    if (p.maxJ > 128) return fail(CHEFSI_ERR_UNSUPPORTED, "density blocks: ALB counts above 128 are not implemented");
    if (ns > 0 && d_f == nullptr) return fail(CHEFSI_ERR_ARG, "f is NULL");
    CHEFSI_TRY(validate_mv("X", d_X, ldx, ns));
    const size_t pb = static_cast<size_t>(p.sqtot) * sizeof(double);
    if (ns > 0 && (overlaps(d_P, pb, d_X, mv_bytes(p.N, ldx, ns, 8)) ||
                   overlaps(d_P, pb, d_f, static_cast<size_t>(ns) * sizeof(double))))
      return fail(CHEFSI_ERR_ARG, "P overlaps X or f");
    size_t need = 0;
    CHEFSI_TRY(chefsi_workspace_bytes(plan, CHEFSI_OP_DENSITY, ns, 0, 1, 1, &need));
    CHEFSI_TRY(check_ws(ws, ws_bytes, need));
    CHEFSI_TRY(check_device(p));
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (ns == 0) return launch_fill(d_P, p.sqtot, 0.0, st);
    Carver c(ws, ws_bytes);
    double* part = c.take<double>(static_cast<int64_t>(elem_nt_slices(p, ns)) * p.sqtot);
    return elem_nt(p, d_X, ldx, d_X, ldx, d_f, ns, true, part, d_P, st);
  });
}

int chefsi_realign_workspace_bytes(chefsi_plan plan, int nr, size_t* bytes) {
  return guarded([&]() -> int {
    if (plan == nullptr || bytes == nullptr) return fail(CHEFSI_ERR_ARG, "plan/bytes is NULL");
    if (nr < 1) return fail(CHEFSI_ERR_ARG, "nr must be >= 1");
    Plan& p = *P(plan);
    Carver c(nullptr, 0);
    c.take<double>(p.sqtot);
    c.take<double>(static_cast<int64_t>(elem_nt_slices(p, nr)) * p.sqtot);
    *bytes = c.used;
    return CHEFSI_OK;
  });
}

int chefsi_realign(chefsi_plan plan, int nr, const double* d_Vnew, const double* d_Vold, double* d_X,
                   int64_t ldx, int ns, void* ws, size_t ws_bytes, void* stream) {
  return guarded([&]() -> int {
    if (plan == nullptr) return fail(CHEFSI_ERR_ARG, "plan is NULL");
    Plan& p = *P(plan);
    if (nr < 1) return fail(CHEFSI_ERR_ARG, "nr must be >= 1");
    if (ns < 0) return fail(CHEFSI_ERR_ARG, "ns must be >= 0");
    if (d_Vnew == nullptr || d_Vold == nullptr) return fail(CHEFSI_ERR_ARG, "Vnew or Vold is NULL");
    if (p.maxJ > 128) return fail(CHEFSI_ERR_UNSUPPORTED, "re-alignment: ALB counts above 128 are not implemented");
    CHEFSI_TRY(validate_mv("X", d_X, ldx, ns));
    const size_t vb = static_cast<size_t>(p.N) * nr * sizeof(double);
    const size_t xb = mv_bytes(p.N, ldx, ns, 8);
    if (ns > 0 && (overlaps(d_X, xb, d_Vnew, vb) || overlaps(d_X, xb, d_Vold, vb)))
      return fail(CHEFSI_ERR_ARG, "X overlaps the ALB samples");
    size_t need = 0;
    CHEFSI_TRY(chefsi_realign_workspace_bytes(plan, nr, &need));
    CHEFSI_TRY(check_ws(ws, ws_bytes, need));
    if (ns == 0) return CHEFSI_OK;
    CHEFSI_TRY(check_device(p));
    hipStream_t st = static_cast<hipStream_t>(stream);
    Carver c(ws, ws_bytes);
    double* R = c.take<double>(p.sqtot);
    double* part = c.take<double>(static_cast<int64_t>(elem_nt_slices(p, nr)) * p.sqtot);
    CHEFSI_TRY(elem_nt(p, d_Vnew, nr, d_Vold, nr, nullptr, nr, false, part, R, st));
    return elem_apply(p, R, d_X, ldx, ns, st);
  });
}

}  // extern "C"
