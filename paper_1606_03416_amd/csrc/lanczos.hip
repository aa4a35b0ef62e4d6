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

// y = H x for one vector, straight from the FP64 panel: one work-group of
// kSpmvThreads per element.  Rows of up to 64 ALBs take 4 waves, rows of up
// to 128 take 2 and rows of up to 256 one (lane group = row), each wave a
// quarter, a half or all of the concatenated neighbour rows (pairs k, k+1
// interleaved), and the parts are added in a fixed order (HBM-bound; the
// panel is read once).
constexpr int kSpmvThreads = 256;
// reduction rows of one element: at most 7 neighbours of up to kMaxJ ALBs
// each, padded to the step kernels' chunk of 16
constexpr int kMaxSpmvK = ((7 * kMaxJ + 15) / 16) * 16;

__global__ __launch_bounds__(kSpmvThreads) void spmv_kernel(const double* panel, const int64_t* poff,
                                                            const int32_t* kpad, const int64_t* koff,
                                                            const int32_t* kmap, const int32_t* J,
                                                            const int32_t* rb, const int64_t* rowoff,
                                                            const double* x, double* y) {
  __shared__ double red[kSpmvThreads];
  const int K = blockIdx.x;
  const int JK = J[K];
  const int splits = (JK <= 64) ? 4 : (JK <= 128 ? 2 : 1);
  const int rows = kSpmvThreads / splits;
  const int i = threadIdx.x % rows, sp = threadIdx.x / rows;
  const int kp = kpad[K];
  const int32_t* km = kmap + koff[K];
  // the element's gathered x entries first (one pass over its reduction
  // rows), so that the product loop reads only the panel from memory
  __shared__ double xs[kMaxSpmvK];
  for (int k = threadIdx.x; k < kp; k += kSpmvThreads) {
    const int g = km[k];
    xs[k] = g >= 0 ? x[g] : 0.0;
  }
  __syncthreads();
  double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
  if (i < JK) {
    const int JP = rb[K] * 16;
    const double* pk = panel + poff[K] + i;
#pragma unroll 2
    for (int k = 4 * sp; k < kp; k += 4 * splits) {
      a0 += pk[static_cast<int64_t>(k) * JP] * xs[k];
      a1 += pk[static_cast<int64_t>(k + 1) * JP] * xs[k + 1];
      a2 += pk[static_cast<int64_t>(k + 2) * JP] * xs[k + 2];
      a3 += pk[static_cast<int64_t>(k + 3) * JP] * xs[k + 3];
    }
  }
  red[threadIdx.x] = (a0 + a1) + (a2 + a3);
  __syncthreads();
  if (sp == 0 && i < JK) {
    double s = 0.0;
    for (int q = 0; q < splits; ++q) s += red[q * rows + i];
    y[rowoff[K] + i] = s;
  }
}

constexpr int RG = 256;   // work-groups of the reduction kernels
constexpr int RT = 256;   // threads per work-group

// Work-group sum of one value per thread (result valid in all threads).
__device__ double wg_sum(double v, double* red) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  const int tid = threadIdx.x;
  __syncthreads();
  if ((tid & 63) == 0) red[tid >> 6] = v;
  __syncthreads();
  double s = 0.0;
  for (int w = 0; w < RT / 64; ++w) s += red[w];
  return s;
}

// Sum of partials[g * stride + t] over g, in a fixed order.
__device__ __forceinline__ double sum_partials(const double* part, int stride, int t) {
  double s = 0.0;
  for (int g = 0; g < RG; ++g) s += part[g * stride + t];
  return s;
}

// Partial dots of w with the vectors V[0..nv-1] over this work-group's rows.
__device__ void partial_dots(const double* V, const double* w, int64_t N, int nv, double* part,
                             double* red) {
  const int64_t r0 = static_cast<int64_t>(blockIdx.x) * RT + threadIdx.x;
  const int64_t stride = static_cast<int64_t>(RG) * RT;
  for (int t = 0; t < nv; ++t) {
    const double* vt = V + static_cast<int64_t>(t) * N;
    double d = 0.0;
    for (int64_t i = r0; i < N; i += stride) d += vt[i] * w[i];
    d = wg_sum(d, red);
    if (threadIdx.x == 0) part[blockIdx.x * (kMaxLanczos + 1) + t] = d;
  }
}

// phase 0: partial v_j^T w
__global__ __launch_bounds__(RT) void lz_alpha_partial(const double* V, const double* w, int64_t N, int j,
                                                       double* part, const LanczosState* stt) {
  __shared__ double red[RT / 64];
  if (stt->stopped) return;
  partial_dots(V + static_cast<int64_t>(j) * N, w, N, 1, part, red);
}

// phase 1: alpha_j = sum; w -= alpha_j v_j + beta_{j-1} v_{j-1}; partial V^T w
__global__ __launch_bounds__(RT) void lz_three_term(double* V, double* w, int64_t N, int j, const double* part_in,
                                                    double* part_out, LanczosState* stt) {
  __shared__ double red[RT / 64];
  if (stt->stopped) return;
  const double alpha = sum_partials(part_in, kMaxLanczos + 1, 0);
  const double bprev = (j > 0) ? stt->beta[j - 1] : 0.0;
  const double* vj = V + static_cast<int64_t>(j) * N;
  const double* vp = (j > 0) ? V + static_cast<int64_t>(j - 1) * N : nullptr;
  const int64_t r0 = static_cast<int64_t>(blockIdx.x) * RT + threadIdx.x;
  const int64_t stride = static_cast<int64_t>(RG) * RT;
  for (int64_t i = r0; i < N; i += stride) w[i] -= alpha * vj[i] + (vp ? bprev * vp[i] : 0.0);
  if (blockIdx.x == 0 && threadIdx.x == 0) stt->alpha[j] = alpha;
  partial_dots(V, w, N, j + 1, part_out, red);
}

// phase 2: h = V^T w (summed partials); w -= V h; then partial V^T w again
// (second Gram-Schmidt pass) or, on the last pass, partial ||w||^2.
__global__ __launch_bounds__(RT) void lz_cgs(const double* V, double* w, int64_t N, int j, const double* part_in,
                                             double* part_out, int last, const LanczosState* stt) {
  __shared__ double red[RT / 64];
  __shared__ double h[kMaxLanczos + 1];
  if (stt->stopped) return;
  if (threadIdx.x <= j) h[threadIdx.x] = sum_partials(part_in, kMaxLanczos + 1, threadIdx.x);
  __syncthreads();
  const int64_t r0 = static_cast<int64_t>(blockIdx.x) * RT + threadIdx.x;
  const int64_t stride = static_cast<int64_t>(RG) * RT;
  for (int64_t i = r0; i < N; i += stride) {
    double acc = w[i];
    for (int t = 0; t <= j; ++t) acc -= h[t] * V[static_cast<int64_t>(t) * N + i];
    w[i] = acc;
  }
  if (!last) {
    partial_dots(V, w, N, j + 1, part_out, red);
  } else {
    double d = 0.0;
    for (int64_t i = r0; i < N; i += stride) d += w[i] * w[i];
    d = wg_sum(d, red);
    if (threadIdx.x == 0) part_out[blockIdx.x * (kMaxLanczos + 1)] = d;
  }
}

// phase 3: beta_j = ||w||; v_{j+1} = w / beta_j unless beta_j <= 1e-14 |alpha_0|.
__global__ __launch_bounds__(RT) void lz_normalize(double* V, const double* w, int64_t N, int j,
                                                   const double* part_in, LanczosState* stt) {
  if (stt->stopped) return;
  const double beta = sqrt(sum_partials(part_in, kMaxLanczos + 1, 0));
  const double a0 = stt->alpha[0];
  const bool stop = beta <= 1e-14 * fabs(a0);
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    stt->beta[j] = beta;
    stt->steps = j + 1;
  }
  if (stop) return;
  double* vn = V + static_cast<int64_t>(j + 1) * N;
  const double inv = 1.0 / beta;
  const int64_t r0 = static_cast<int64_t>(blockIdx.x) * RT + threadIdx.x;
  const int64_t stride = static_cast<int64_t>(RG) * RT;
  for (int64_t i = r0; i < N; i += stride) vn[i] = w[i] * inv;
}

__global__ void lz_check_stop(LanczosState* stt, int j) {
  if (threadIdx.x == 0 && !stt->stopped && stt->steps == j + 1) {
    if (stt->beta[j] <= 1e-14 * fabs(stt->alpha[0])) stt->stopped = 1;
  }
}

// Largest eigenvalue of the symmetric tridiagonal T_k (diagonal al[0..n-1],
// off-diagonal be[0..n-2]) by bisection on Sturm counts: count(x) = number of
// eigenvalues below x = number of negative pivots of the LDL^T factorisation
// of T_k - xI.  The bracket starts from the Gershgorin interval and halves
// until it cannot shrink; the upper end is returned (at most one unit in the
// last place above the eigenvalue).
__device__ double tridiag_max_eig(const double* al, const double* be, int n) {
  if (n == 1) return al[0];
  double gl = al[0], gu = al[0], b2 = 0.0;
  for (int i = 0; i < n; ++i) {
    const double r = (i > 0 ? fabs(be[i - 1]) : 0.0) + (i + 1 < n ? fabs(be[i]) : 0.0);
    gl = fmin(gl, al[i] - r);
    gu = fmax(gu, al[i] + r);
    if (i + 1 < n) b2 = fmax(b2, be[i] * be[i]);
  }
  const double pivmin = 2.2250738585072014e-308 * fmax(1.0, b2);
  double lo = gl, hi = gu + fmax(1e-3 * (gu - gl), 1e-12 * fmax(fabs(gu), 1.0));
  for (int it = 0; it < 2200; ++it) {
    const double mid = 0.5 * (lo + hi);
    if (!(mid > lo && mid < hi)) break;
    int c = 0;
    double q = al[0] - mid;
    if (fabs(q) < pivmin) q = -pivmin;
    c += q < 0.0;
    for (int i = 1; i < n; ++i) {
      q = al[i] - mid - be[i - 1] * be[i - 1] / q;
      if (fabs(q) < pivmin) q = -pivmin;
      c += q < 0.0;
    }
    if (c == n) hi = mid;
    else lo = mid;
  }
  return hi;
}

// Bounds from the Lanczos tridiagonal T: b = (largest eigenvalue of T, by
// bisection) + the last beta in every cycle.  The first-cycle rule (ritz ==
// nullptr) also needs every eigenvalue and the first component of every
// eigenvector: eigenpairs of T (order n <= 64) by parallel Jacobi, each round
// rotating n/2 disjoint (p, q) pairs of a round-robin tournament (a sweep of
// n-1 rounds meets every pair once), thread t applying the rotations to
// row / column t.  Warm cycles take a and a0 from the previous Ritz values
// and skip the Jacobi sweeps.
__global__ __launch_bounds__(64) void lanczos_bounds_kernel(const LanczosState* stt, const double* ritz, int ns,
                                                            double frac, double* bounds) {
  __shared__ double T[kMaxLanczos][kMaxLanczos + 1];
  __shared__ double V[kMaxLanczos][kMaxLanczos + 1];
  __shared__ double cs[kMaxLanczos / 2][2];
  __shared__ int pq[kMaxLanczos / 2][2];
  __shared__ int done;
  __shared__ double sal[kMaxLanczos], sbe[kMaxLanczos];   // alpha, beta of T
  const int t = threadIdx.x;
  const int n = stt->steps;
  const int m = (n + 1) & ~1;   // players incl. an idle one when n is odd
  for (int j = 0; j < kMaxLanczos; ++j) {
    T[t][j] = 0.0;
    V[t][j] = (t == j) ? 1.0 : 0.0;
  }
  __syncthreads();
  if (t < n) {
    sal[t] = stt->alpha[t];
    sbe[t] = stt->beta[t];
    T[t][t] = stt->alpha[t];
    if (t + 1 < n) {
      T[t][t + 1] = stt->beta[t];
      T[t + 1][t] = stt->beta[t];
    }
  }
  __syncthreads();
  double fro = 0.0;
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) fro += T[i][j] * T[i][j];
  fro = sqrt(fro);
  const bool cold = (ritz == nullptr);
  for (int sweep = 0; sweep < 60 && n > 1 && cold; ++sweep) {
    if (t == 0) {
      double off = 0.0;
      for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j)
          if (i != j) off += T[i][j] * T[i][j];
      done = sqrt(off) <= 1e-15 * fro;
    }
    __syncthreads();
    if (done) break;
    for (int r = 0; r < m - 1; ++r) {
      if (t < m / 2) {
        // position i of the circle holds player ((i + r) % (m - 1)) + 1; player 0 is fixed
        int p, q;
        if (t == 0) {
          p = 0;
          q = (r % (m - 1)) + 1;
        } else {
          p = ((t + r) % (m - 1)) + 1;
          q = ((m - 1 - t + r) % (m - 1)) + 1;
        }
        if (p > q) {
          const int x = p;
          p = q;
          q = x;
        }
        double c = 1.0, sn = 0.0;
        if (q < n) {
          const double apq = T[p][q];
          if (fabs(apq) > 1e-300) {
            const double tau = (T[q][q] - T[p][p]) / (2.0 * apq);
            const double tt = (tau >= 0.0) ? 1.0 / (tau + sqrt(1.0 + tau * tau))
                                           : -1.0 / (-tau + sqrt(1.0 + tau * tau));
            c = 1.0 / sqrt(1.0 + tt * tt);
            sn = tt * c;
          }
        }
        cs[t][0] = c;
        cs[t][1] = sn;
        pq[t][0] = p;
        pq[t][1] = q < n ? q : p;   // idle pair: identity on p
      }
      __syncthreads();
      // T <- T J and V <- V J on row t
      if (t < n) {
        for (int k = 0; k < m / 2; ++k) {
          const int p = pq[k][0], q = pq[k][1];
          if (p == q) continue;
          const double c = cs[k][0], sn = cs[k][1];
          const double xp = T[t][p], xq = T[t][q];
          T[t][p] = c * xp - sn * xq;
          T[t][q] = sn * xp + c * xq;
          const double vp = V[t][p], vq = V[t][q];
          V[t][p] = c * vp - sn * vq;
          V[t][q] = sn * vp + c * vq;
        }
      }
      __syncthreads();
      // T <- J^T T on column t
      if (t < n) {
        for (int k = 0; k < m / 2; ++k) {
          const int p = pq[k][0], q = pq[k][1];
          if (p == q) continue;
          const double c = cs[k][0], sn = cs[k][1];
          const double xp = T[p][t], xq = T[q][t];
          T[p][t] = c * xp - sn * xq;
          T[q][t] = sn * xp + c * xq;
        }
      }
      __syncthreads();
      if (t < m / 2 && pq[t][0] != pq[t][1]) {
        T[pq[t][0]][pq[t][1]] = 0.0;
        T[pq[t][1]][pq[t][0]] = 0.0;
      }
      __syncthreads();
    }
  }
  if (t != 0) return;
  const double b = tridiag_max_eig(sal, sbe, n) + sbe[n - 1];
  double a, a0;
  if (!cold) {
    a = ritz[ns - 1];
    a0 = ritz[0];
  } else {
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
    a0 = T[idx[0]][idx[0]];
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

// The filter needs finite bounds with a0 < a < b: previous Ritz values above
// a reused upper bound (H changed since) or a failed Lanczos run break that.
// *status = 1 (bounds not finite) or 2 (not ordered); untouched otherwise.
__global__ void check_bounds_kernel(const double* bounds, int* status) {
  if (threadIdx.x != 0) return;
  const double a = bounds[0], b = bounds[1], a0 = bounds[2];
  if (!isfinite(a) || !isfinite(b) || !isfinite(a0)) {
    *status = 1;
  } else if (!(a0 < a && a < b)) {
    *status = 2;
  }
}

}  // namespace

size_t lanczos_ws_bytes(const Plan& p, int k) {
  Carver c(nullptr, 0);
  c.take<double>(static_cast<int64_t>(k + 1) * p.N);
  c.take<double>(p.N);
  c.take<LanczosState>(1);
  c.take<double>(2 * static_cast<int64_t>(RG) * (kMaxLanczos + 1));
  return c.used;
}

int lanczos_bounds(const Plan& p, const void* d_panel64, const double* d_v0, int k,
                   const double* d_ritz_prev, int ns, double* d_bounds, void* ws, size_t ws_bytes,
                   hipStream_t st) {
  Carver c(ws, ws_bytes);
  double* V = c.take<double>(static_cast<int64_t>(k + 1) * p.N);
  double* w = c.take<double>(p.N);
  LanczosState* stt = c.take<LanczosState>(1);
  double* partA = c.take<double>(2 * static_cast<int64_t>(RG) * (kMaxLanczos + 1));
  double* partB = partA + static_cast<int64_t>(RG) * (kMaxLanczos + 1);
  if (!c.ok()) return fail(CHEFSI_ERR_WORKSPACE, "bounds: workspace too small");
  lanczos_init_kernel<<<1, LT, 0, st>>>(d_v0, p.N, V, stt);
  CHEFSI_LAUNCHED("lanczos_init");
  const double* panel = static_cast<const double*>(d_panel64);
  for (int j = 0; j < k; ++j) {
    spmv_kernel<<<p.M, kSpmvThreads, 0, st>>>(panel, p.d_poff, p.d_kpad, p.d_koff, p.d_kmap, p.d_J, p.d_rb, p.d_rowoff,
                                     V + static_cast<int64_t>(j) * p.N, w);
    lz_alpha_partial<<<RG, RT, 0, st>>>(V, w, p.N, j, partA, stt);
    lz_three_term<<<RG, RT, 0, st>>>(V, w, p.N, j, partA, partB, stt);
    lz_cgs<<<RG, RT, 0, st>>>(V, w, p.N, j, partB, partA, 0, stt);
    lz_cgs<<<RG, RT, 0, st>>>(V, w, p.N, j, partA, partB, 1, stt);
    lz_normalize<<<RG, RT, 0, st>>>(V, w, p.N, j, partB, stt);
    lz_check_stop<<<1, 64, 0, st>>>(stt, j);
    CHEFSI_LAUNCHED("lanczos step");
  }
  const double frac = static_cast<double>(ns) / static_cast<double>(p.N);
  lanczos_bounds_kernel<<<1, 64, 0, st>>>(stt, d_ritz_prev, ns, frac, d_bounds);
  CHEFSI_LAUNCHED("lanczos_bounds");
  return CHEFSI_OK;
}

int launch_warm_bounds(const double* d_ritz, int ns, const double* d_bounds_src, double* d_bounds,
                       hipStream_t st) {
  warm_bounds_kernel<<<1, 64, 0, st>>>(d_ritz, ns, d_bounds_src, d_bounds);
  CHEFSI_LAUNCHED("warm_bounds");
  return CHEFSI_OK;
}

int launch_check_bounds(const double* d_bounds, int* d_status, hipStream_t st) {
  check_bounds_kernel<<<1, 64, 0, st>>>(d_bounds, d_status);
  CHEFSI_LAUNCHED("check_bounds");
  return CHEFSI_OK;
}

}  // namespace chefsi
