// Filter bounds (Algorithm 1 step 1) on the GPU: k steps of Lanczos with full
// reorthogonalisation give b_up = theta_max(T_k) + beta_k; the lower bound and
// the scaling point come from Ritz values (previous cycle) or, on a first cycle
// from a random block, from the Lanczos quadrature weights.  Everything stays
// on the device; the host only reads the three bounds at the end.
#include "common.h"

namespace chefsi {

namespace {

constexpr int LT = 1024;  // threads of the single-work-group kernels

struct LanczosState {
  double alpha[kMaxLanczos];
  double beta[kMaxLanczos];
  int steps;    // number of alpha values produced
  int stopped;  // invariant subspace found
};

__device__ double block_sum(double v, double* red) {
  const int tid = threadIdx.x;
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  __syncthreads();
  if ((tid & 63) == 0) red[tid >> 6] = v;
  __syncthreads();
  double s = 0.0;
  if (tid < 64) {
    s = (tid < static_cast<int>(blockDim.x >> 6)) ? red[tid] : 0.0;
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
    if (tid == 0) red[32] = s;
  }
  __syncthreads();
  s = red[32];
  __syncthreads();
  return s;
}

__global__ __launch_bounds__(LT) void lanczos_init_kernel(const double* v0, int64_t N, double* V,
                                                          LanczosState* stt) {
  __shared__ double red[64];
  double s = 0.0;
  for (int64_t i = threadIdx.x; i < N; i += LT) s += v0[i] * v0[i];
  s = block_sum(s, red);
  const double inv = 1.0 / sqrt(s);
  for (int64_t i = threadIdx.x; i < N; i += LT) V[i] = v0[i] * inv;
  if (threadIdx.x == 0) {
    stt->steps = 0;
    stt->stopped = 0;
  }
}

// Given w = H v_j: alpha_j = v_j^T w, w -= alpha_j v_j + beta_{j-1} v_{j-1},
// two classical Gram-Schmidt passes against v_0..v_j, beta_j = ||w||,
// v_{j+1} = w / beta_j (unless beta_j <= 1e-14 |alpha_0|).
__global__ __launch_bounds__(LT) void lanczos_orth_kernel(double* V, double* w, int64_t N, int j,
                                                          LanczosState* stt) {
  __shared__ double red[64];
  if (stt->stopped) return;
  const int tid = threadIdx.x;
  const double* vj = V + static_cast<int64_t>(j) * N;
  double s = 0.0;
  for (int64_t i = tid; i < N; i += LT) s += vj[i] * w[i];
  const double alpha = block_sum(s, red);
  const double bprev = (j > 0) ? stt->beta[j - 1] : 0.0;
  const double* vp = (j > 0) ? V + static_cast<int64_t>(j - 1) * N : nullptr;
  for (int64_t i = tid; i < N; i += LT) w[i] -= alpha * vj[i] + (vp ? bprev * vp[i] : 0.0);
  __syncthreads();
  __shared__ double h[kMaxLanczos + 1];
  for (int pass = 0; pass < 2; ++pass) {
    for (int t = 0; t <= j; ++t) {
      const double* vt = V + static_cast<int64_t>(t) * N;
      double d = 0.0;
      for (int64_t i = tid; i < N; i += LT) d += vt[i] * w[i];
      d = block_sum(d, red);
      if (tid == 0) h[t] = d;
    }
    __syncthreads();
    for (int64_t i = tid; i < N; i += LT) {
      double acc = w[i];
      for (int t = 0; t <= j; ++t) acc -= h[t] * V[static_cast<int64_t>(t) * N + i];
      w[i] = acc;
    }
    __syncthreads();
  }
  s = 0.0;
  for (int64_t i = tid; i < N; i += LT) s += w[i] * w[i];
  const double beta = sqrt(block_sum(s, red));
  if (tid == 0) {
    stt->alpha[j] = alpha;
    stt->beta[j] = beta;
    stt->steps = j + 1;
  }
  const double a0 = (j == 0) ? alpha : stt->alpha[0];
  if (beta <= 1e-14 * fabs(a0)) {
    if (tid == 0) stt->stopped = 1;
    return;
  }
  double* vn = V + static_cast<int64_t>(j + 1) * N;
  const double inv = 1.0 / beta;
  for (int64_t i = tid; i < N; i += LT) vn[i] = w[i] * inv;
}

// Eigenpairs of the tridiagonal T (order n <= 64) by cyclic Jacobi on one
// thread, then the bounds policy.  ritz == nullptr selects the first-cycle rule.
__global__ void lanczos_bounds_kernel(const LanczosState* stt, const double* ritz, int ns,
                                      double frac, double* bounds) {
  __shared__ double T[kMaxLanczos][kMaxLanczos];
  __shared__ double V[kMaxLanczos][kMaxLanczos];
  if (threadIdx.x != 0) return;
  const int n = stt->steps;
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) {
      T[i][j] = 0.0;
      V[i][j] = (i == j) ? 1.0 : 0.0;
    }
  for (int i = 0; i < n; ++i) T[i][i] = stt->alpha[i];
  for (int i = 0; i + 1 < n; ++i) {
    T[i][i + 1] = stt->beta[i];
    T[i + 1][i] = stt->beta[i];
  }
  double fro = 0.0;
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) fro += T[i][j] * T[i][j];
  fro = sqrt(fro);
  for (int sweep = 0; sweep < 60 && n > 1; ++sweep) {
    double off = 0.0;
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j)
        if (i != j) off += T[i][j] * T[i][j];
    if (sqrt(off) <= 1e-15 * fro) break;
    for (int p = 0; p < n - 1; ++p)
      for (int q = p + 1; q < n; ++q) {
        const double apq = T[p][q];
        if (fabs(apq) <= 1e-300) continue;
        const double tau = (T[q][q] - T[p][p]) / (2.0 * apq);
        const double t = (tau >= 0.0) ? 1.0 / (tau + sqrt(1.0 + tau * tau))
                                      : -1.0 / (-tau + sqrt(1.0 + tau * tau));
        const double c = 1.0 / sqrt(1.0 + t * t), s = t * c;
        for (int r = 0; r < n; ++r) {
          const double xp = T[r][p], xq = T[r][q];
          T[r][p] = c * xp - s * xq;
          T[r][q] = s * xp + c * xq;
        }
        for (int r = 0; r < n; ++r) {
          const double xp = T[p][r], xq = T[q][r];
          T[p][r] = c * xp - s * xq;
          T[q][r] = s * xp + c * xq;
        }
        T[p][q] = 0.0;
        T[q][p] = 0.0;
        for (int r = 0; r < n; ++r) {
          const double xp = V[r][p], xq = V[r][q];
          V[r][p] = c * xp - s * xq;
          V[r][q] = s * xp + c * xq;
        }
      }
  }
  // ascending order of the diagonal (stable selection)
  int idx[kMaxLanczos];
  for (int i = 0; i < n; ++i) idx[i] = i;
  for (int i = 1; i < n; ++i) {
    const int v = idx[i];
    int j = i - 1;
    while (j >= 0 && T[idx[j]][idx[j]] > T[v][v]) {
      idx[j + 1] = idx[j];
      --j;
    }
    idx[j + 1] = v;
  }
  const double theta_min = T[idx[0]][idx[0]];
  const double theta_max = T[idx[n - 1]][idx[n - 1]];
  const double b = theta_max + stt->beta[n - 1];
  double a, a0;
  if (ritz != nullptr) {
    a = ritz[ns - 1];
    a0 = ritz[0];
  } else {
    double cum = 0.0;
    int js = n - 1;
    for (int i = 0; i < n; ++i) {
      const double tau = V[0][idx[i]];
      cum += tau * tau;
      if (cum >= frac) {
        js = i;
        break;
      }
    }
    a = T[idx[js]][idx[js]];
    a0 = theta_min;
  }
  if (a0 >= a - 1e-12 * fabs(b)) a0 = a - 1e-3 * (b - a);
  bounds[0] = a;
  bounds[1] = b;
  bounds[2] = a0;
}

__global__ void warm_bounds_kernel(const double* ritz, int ns, const double* bsrc, double* bounds) {
  if (threadIdx.x != 0) return;
  const double b = bsrc[1];
  const double a = ritz[ns - 1];
  double a0 = ritz[0];
  if (a0 >= a - 1e-12 * fabs(b)) a0 = a - 1e-3 * (b - a);
  bounds[0] = a;
  bounds[1] = b;
  bounds[2] = a0;
}

}  // namespace

size_t lanczos_ws_bytes(const Plan& p, int k) {
  Carver c(nullptr, 0);
  c.take<double>(static_cast<int64_t>(k + 1) * p.N);
  c.take<double>(p.N);
  c.take<LanczosState>(1);
  c.take<double>(4);
  return c.used;
}

int lanczos_bounds(const Plan& p, const void* d_panel64, const double* d_v0, int k,
                   const double* d_ritz_prev, int ns, double* d_bounds, void* ws, size_t ws_bytes,
                   hipStream_t st) {
  Carver c(ws, ws_bytes);
  double* V = c.take<double>(static_cast<int64_t>(k + 1) * p.N);
  double* w = c.take<double>(p.N);
  LanczosState* stt = c.take<LanczosState>(1);
  double* coef = c.take<double>(4);
  if (!c.ok()) return fail(CHEFSI_ERR_WORKSPACE, "bounds: workspace too small");
  lanczos_init_kernel<<<1, LT, 0, st>>>(d_v0, p.N, V, stt);
  CHEFSI_LAUNCHED("lanczos_init");
  CHEFSI_TRY(launch_const_coef(1.0, 0.0, coef, st));
  for (int j = 0; j < k; ++j) {
    StepIO io{V + static_cast<int64_t>(j) * p.N, 1, true, nullptr, 0, true, w, 1, true};
    CHEFSI_TRY(launch_step(p, d_panel64, CHEFSI_F64, coef, io, 1, st));
    lanczos_orth_kernel<<<1, LT, 0, st>>>(V, w, p.N, j, stt);
    CHEFSI_LAUNCHED("lanczos_orth");
  }
  const double frac = static_cast<double>(ns) / static_cast<double>(p.N);
  lanczos_bounds_kernel<<<1, 64, 0, st>>>(stt, d_ritz_prev, ns, frac, d_bounds);
  CHEFSI_LAUNCHED("lanczos_bounds");
  return CHEFSI_OK;
}

int launch_warm_bounds(const double* d_ritz, int ns, const double* d_b_src, double* d_bounds,
                       hipStream_t st) {
  warm_bounds_kernel<<<1, 64, 0, st>>>(d_ritz, ns, d_b_src, d_bounds);
  CHEFSI_LAUNCHED("warm_bounds");
  return CHEFSI_OK;
}

}  // namespace chefsi
