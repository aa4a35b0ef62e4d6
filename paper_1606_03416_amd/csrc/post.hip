// Steps around the CheFSI cycle (gfx950):
//  * the Fermi level by bisection and the Fermi-Dirac occupations of the Ritz
//    values (Sec. II A, Fermi-Dirac smearing of the occupations; Sec. II B 2,
//    the Ritz values give the Fermi energy and the occupation numbers);
//  * element-local products C_K = A_K diag(w) B_K^T, which give the diagonal
//    density-matrix blocks P_KK = X_K diag(f) X_K^T (eq. densitymatrix with
//    K = K') and the basis overlaps R_K = V_new,K^T V_old,K (eq.
//    basis_rotation_3);
//  * the element-local rotation X_K <- R_K X_K (eq. basis_rotation_3).
//
// The element products stream X (or the ALB samples) once from HBM: a
// work-group owns one element and one slice of the reduction columns, stages
// 32-column chunks of the element's rows in LDS (the next chunk is loaded into
// registers while the current one is multiplied) and accumulates 16x16 tiles
// with v_mfma_f64_16x16x4f64.  Symmetric products compute only the tiles on
// and above the diagonal.  Slices are summed, in a fixed order, by a second
// small kernel that also mirrors the symmetric result.
//
// MFMA operand layout (v_mfma_f64_16x16x4f64): lane l supplies A[l%16][k] and
// B[k][l%16] for one k of four, and receives D[4v + l/16][l%16], v = 0..3.  Two
// consecutive MFMAs take the k pairs (8g + 2(l/16), 8g + 2(l/16) + 1): any
// assignment of the reduction index to (lane group, MFMA) is valid as long as
// A and B use the same one, and this one lets each lane read its two k values
// of a row with one 16-byte LDS load.
#include <cmath>

#include "common.h"

namespace chefsi {
namespace {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef double d2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ d4 mfma64(double a, double b, d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// Work-group id -> linear work index such that the work-groups one XCD runs
// (hardware id b goes to XCD b % 8) are consecutive work items.
__device__ __forceinline__ int xcd_linear(int b, int nwg) {
  const int q = nwg >> 3, r = nwg & 7;
  const int x = b & 7, i = b >> 3;
  return x * q + (x < r ? x : r) + i;
}

// ----------------------------------------------------------- Fermi level
constexpr int kFermiThreads = 1024;
constexpr int kBisectMax = 200;
constexpr double kBracketKT = 50.0;

// Deterministic block reductions: a fixed xor butterfly in each wave, then
// the wave results in wave order.
__device__ double block_sum(double v, double* red) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  const int w = threadIdx.x >> 6, nw = blockDim.x >> 6;
  if ((threadIdx.x & 63) == 0) red[w] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int i = 0; i < nw; ++i) s += red[i];
    red[32] = s;
  }
  __syncthreads();
  const double r = red[32];
  __syncthreads();
  return r;
}

__device__ double block_minmax(double v, double* red, bool is_max) {
  for (int o = 32; o > 0; o >>= 1) {
    const double u = __shfl_xor(v, o);
    v = is_max ? fmax(v, u) : fmin(v, u);
  }
  const int w = threadIdx.x >> 6, nw = blockDim.x >> 6;
  if ((threadIdx.x & 63) == 0) red[w] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = red[0];
    for (int i = 1; i < nw; ++i) s = is_max ? fmax(s, red[i]) : fmin(s, red[i]);
    red[32] = s;
  }
  __syncthreads();
  const double r = red[32];
  __syncthreads();
  return r;
}

__device__ __forceinline__ double fermi_dirac(double theta, double mu, double kT) {
  return 1.0 / (1.0 + exp((theta - mu) / kT));
}

// One work-group: mu with sum_i f_i(mu) = n_occ by bisection on
// [min theta - 50 kT, max theta + 50 kT], halving until the midpoint is no
// longer strictly inside the bracket or 200 halvings; mu = the final
// midpoint; then f_i = f(theta_i; mu).  Every thread takes the same branch
// (the block sum is broadcast).  A non-finite Ritz value gives NaN outputs.
__global__ __launch_bounds__(kFermiThreads) void fermi_kernel(const double* __restrict__ theta, int ns,
                                                             double n_occ, double kT, double* __restrict__ f,
                                                             double* __restrict__ mu_out) {
  __shared__ double red[33];
  double tmin = INFINITY, tmax = -INFINITY, bad = 0.0;
  for (int i = threadIdx.x; i < ns; i += blockDim.x) {
    const double t = theta[i];
    if (!isfinite(t)) bad = 1.0;
    tmin = fmin(tmin, t);
    tmax = fmax(tmax, t);
  }
  bad = block_sum(bad, red);
  tmin = block_minmax(tmin, red, false);
  tmax = block_minmax(tmax, red, true);
  if (bad > 0.0) {
    for (int i = threadIdx.x; i < ns; i += blockDim.x) f[i] = NAN;
    if (threadIdx.x == 0) mu_out[0] = NAN;
    return;
  }
  double lo = tmin - kBracketKT * kT, hi = tmax + kBracketKT * kT;
  for (int it = 0; it < kBisectMax; ++it) {
    const double mid = 0.5 * (lo + hi);
    if (!(lo < mid && mid < hi)) break;
    double s = 0.0;
    for (int i = threadIdx.x; i < ns; i += blockDim.x) s += fermi_dirac(theta[i], mid, kT);
    s = block_sum(s, red);
    if (s < n_occ)
      lo = mid;
    else
      hi = mid;
  }
  const double mu = 0.5 * (lo + hi);
  for (int i = threadIdx.x; i < ns; i += blockDim.x) f[i] = fermi_dirac(theta[i], mu, kT);
  if (threadIdx.x == 0) mu_out[0] = mu;
}

// ------------------------------------------------------- element products
constexpr int kNtThreads = 256;
#ifndef CHEFSI_NT_KC
#define CHEFSI_NT_KC 32
#endif
#ifndef CHEFSI_NT_TARGET
#define CHEFSI_NT_TARGET 4096
#endif
#ifndef CHEFSI_AP_TARGET
#define CHEFSI_AP_TARGET 8192
#endif
constexpr int kNtKC = CHEFSI_NT_KC;          // reduction columns per chunk
constexpr int kNtLD = kNtKC + 2;             // LDS row stride in doubles (rows 4 banks apart)
constexpr int kNtTargetWG = CHEFSI_NT_TARGET;  // work-groups a launch aims at (element x slice)

struct NtArgs {
  const double* A; int64_t lda;      // rows rowoff[K] .. rowoff[K]+J_K-1, row stride lda
  const double* B; int64_t ldb;      // same rows of B (B = A for symmetric products)
  const double* w;                   // column weights (L) or null (all 1)
  const int64_t* rowoff; const int32_t* J; const int64_t* sqoff; const int32_t* order;
  int start, count;                  // elements order[start .. start+count)
  int64_t L;                         // reduction length
  int S; int64_t SL;                 // slices and slice length (multiple of kNtKC)
  double* part; int64_t pstride;     // slice s of element K at part + s*pstride + sqoff[K]
  bool vec;                          // 16-byte global loads allowed
};

// Tiles of an RB x RB tile grid handled by one product: all of them, or the
// ones on and above the diagonal (symmetric products).  Up to 16 tiles, the
// work-group has the fewest waves, from 4 to 8, that gives the fewest tiles per
// wave, so the waves carry equal MFMA work (10 upper tiles of a 64-row element:
// 5 waves of 2); larger grids keep 4 waves.  The first kNtThreads threads stage
// the operands.
template <int RB, bool SYM>
struct NtTiles {
  static constexpr int T = SYM ? RB * (RB + 1) / 2 : RB * RB;
  static constexpr int waves() {
    int best = 4;
    if (T > 16) return best;
    for (int w = 5; w <= 8; ++w)
      if ((T + w - 1) / w < (T + best - 1) / best) best = w;
    return best;
  }
  static constexpr int NW = waves();
  static constexpr int PER_WAVE = (T + NW - 1) / NW;
};

template <int RB, bool SYM>
__global__ __launch_bounds__((NtTiles<RB, SYM>::NW * 64)) void elem_nt_kernel(NtArgs a) {
  constexpr int ROWS = RB * 16;
  constexpr int PW = NtTiles<RB, SYM>::PER_WAVE;
  constexpr int T = NtTiles<RB, SYM>::T;
  constexpr int NW = NtTiles<RB, SYM>::NW;
  __shared__ __attribute__((aligned(16))) double xs[ROWS * kNtLD];
  __shared__ __attribute__((aligned(16))) double ys[ROWS * kNtLD];

  const int id = xcd_linear(blockIdx.x, gridDim.x);
  const int e = id / a.S, s = id - e * a.S;
  const int K = a.order[a.start + e];
  const int JK = a.J[K];
  const int64_t r0 = a.rowoff[K];
  const int64_t cbeg = s * a.SL;
  const int64_t cend = (cbeg + a.SL < a.L) ? cbeg + a.SL : a.L;
  const int nchunk = static_cast<int>((cend - cbeg + kNtKC - 1) / kNtKC);

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int li = lane & 15, lq = lane >> 4;

  // this wave's tiles (row tile, column tile), -1 past the end
  int ti[PW], tj[PW];
#pragma unroll
  for (int u = 0; u < PW; ++u) {
    const int t = wave + NW * u;
    ti[u] = -1;
    tj[u] = -1;
    if (t < T) {
      if (SYM) {
        int r = 0, rem = t;
        while (rem >= RB - r) { rem -= RB - r; ++r; }
        ti[u] = r;
        tj[u] = r + rem;
      } else {
        ti[u] = t / RB;
        tj[u] = t % RB;
      }
    }
  }
  d4 acc[PW];
#pragma unroll
  for (int u = 0; u < PW; ++u) acc[u] = d4{0.0, 0.0, 0.0, 0.0};

  // staging: thread -> (row tid/TPR + RPP*p, column pair 2(tid%TPR)), TPR
  // threads per chunk row, RPP rows per pass, NP passes
  constexpr int TPR = kNtKC / 2, RPP = kNtThreads / TPR, NP = ROWS / RPP;
  static_assert(ROWS % RPP == 0, "chunk rows split evenly over the passes");
  const int srow = tid / TPR, scol = (tid % TPR) * 2;
  d2 ra[NP], rb[NP], rw;
  auto load = [&](int chunk) {
    const int64_t col = cbeg + static_cast<int64_t>(chunk) * kNtKC + scol;
    const bool c0 = col < cend, c1 = col + 1 < cend;
    if (a.w) {
      rw.x = c0 ? a.w[col] : 0.0;
      rw.y = c1 ? a.w[col + 1] : 0.0;
    } else {
      rw = d2{1.0, 1.0};
    }
#pragma unroll
    for (int p = 0; p < NP; ++p) {
      const int row = srow + RPP * p;
      d2 va = d2{0.0, 0.0}, vb = d2{0.0, 0.0};
      if (row < JK && c0) {
        const double* pa = a.A + (r0 + row) * a.lda + col;
        const double* pb = a.B + (r0 + row) * a.ldb + col;
        if (a.vec && c1) {
          va = *reinterpret_cast<const d2*>(pa);
          if (!SYM) vb = *reinterpret_cast<const d2*>(pb);
        } else {
          va.x = pa[0];
          if (c1) va.y = pa[1];
          if (!SYM) {
            vb.x = pb[0];
            if (c1) vb.y = pb[1];
          }
        }
      }
      ra[p] = va;
      rb[p] = SYM ? va : vb;
    }
  };

  const bool stager = tid < kNtThreads;
  if (stager && nchunk > 0) load(0);
  for (int c = 0; c < nchunk; ++c) {
    __syncthreads();  // the previous chunk's tiles are no longer read
    if (stager) {
#pragma unroll
      for (int p = 0; p < NP; ++p) {
        const int row = srow + RPP * p;
        *reinterpret_cast<d2*>(&xs[row * kNtLD + scol]) = ra[p];
        *reinterpret_cast<d2*>(&ys[row * kNtLD + scol]) = rb[p] * rw;
      }
    }
    __syncthreads();
    if (stager && c + 1 < nchunk) load(c + 1);
#pragma unroll
    for (int g = 0; g < kNtKC / 8; ++g) {
      const int k = 8 * g + 2 * lq;
#pragma unroll
      for (int u = 0; u < PW; ++u) {
        if (ti[u] >= 0) {
          const d2 av = *reinterpret_cast<const d2*>(&xs[(ti[u] * 16 + li) * kNtLD + k]);
          const d2 bv = *reinterpret_cast<const d2*>(&ys[(tj[u] * 16 + li) * kNtLD + k]);
          acc[u] = mfma64(av.x, bv.x, acc[u]);
          acc[u] = mfma64(av.y, bv.y, acc[u]);
        }
      }
    }
  }

  double* out = a.part + s * a.pstride + a.sqoff[K];
#pragma unroll
  for (int u = 0; u < PW; ++u) {
    if (ti[u] < 0) continue;
    const int col = tj[u] * 16 + li;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int row = ti[u] * 16 + 4 * v + lq;
      if (row < JK && col < JK) out[static_cast<int64_t>(row) * JK + col] = acc[u][v];
    }
  }
}

// out_K[i][j] = sum_s part_s,K[i][j] (s in order); symmetric products read the
// entry on or above the diagonal for both (i, j) and (j, i).
// One-dimensional grid: nb work-groups of 256 entries per element.
__global__ __launch_bounds__(256) void nt_reduce_kernel(const double* __restrict__ part, int64_t pstride, int S,
                                                        int nb, const int32_t* __restrict__ J,
                                                        const int64_t* __restrict__ sqoff, bool sym,
                                                        double* __restrict__ out) {
  const int K = blockIdx.x / nb;
  const int JK = J[K];
  const int e = (blockIdx.x - K * nb) * blockDim.x + threadIdx.x;
  if (e >= JK * JK) return;
  const int i = e / JK, j = e - i * JK;
  const int src = (sym && i > j) ? j * JK + i : e;
  const double* p = part + sqoff[K] + src;
  double acc = 0.0;
  for (int t = 0; t < S; ++t) acc += p[t * pstride];
  out[sqoff[K] + e] = acc;
}

// --------------------------------------------------- element rotation
constexpr int kApThreads = 256;
constexpr int kApCW = 64;              // columns per chunk (16 per wave)
constexpr int kApTargetWG = CHEFSI_AP_TARGET;

struct ApplyArgs {
  const double* R;                     // R_K (J_K x J_K row-major) at R + sqoff[K]
  double* X; int64_t ldx; int ns;
  const int64_t* rowoff; const int32_t* J; const int64_t* sqoff; const int32_t* order;
  int start, count, G;                 // elements order[start .. start+count), G column groups each
};

// X_K[:, cols] <- R_K X_K[:, cols] in place.  A work-group owns element K and
// a range of 64-column chunks; R_K sits in LDS (zero padded to RB*16 square);
// wave w owns columns 16w .. 16w+15 of each chunk and holds all rows of them in
// registers before it writes any (the chunk's columns belong to this wave
// only), loading the next chunk while it multiplies the current one.
template <int RB>
__global__ __launch_bounds__(kApThreads) void elem_apply_kernel(ApplyArgs a) {
  constexpr int ROWS = RB * 16;
  constexpr int LDR = ROWS + 2;
  constexpr int NG = ROWS / 8;         // 8-row groups of the reduction
  extern __shared__ __attribute__((aligned(16))) double rs[];

  const int id = xcd_linear(blockIdx.x, gridDim.x);
  const int e = id / a.G, g = id - e * a.G;
  const int K = a.order[a.start + e];
  const int JK = a.J[K];
  const int64_t r0 = a.rowoff[K];
  const double* RK = a.R + a.sqoff[K];
  for (int idx = threadIdx.x; idx < ROWS * ROWS; idx += blockDim.x) {
    const int i = idx / ROWS, k = idx - i * ROWS;
    rs[i * LDR + k] = (i < JK && k < JK) ? RK[i * JK + k] : 0.0;
  }
  __syncthreads();

  const int nchunk = (a.ns + kApCW - 1) / kApCW;
  const int cb = static_cast<int>((static_cast<int64_t>(nchunk) * g) / a.G);
  const int ce = static_cast<int>((static_cast<int64_t>(nchunk) * (g + 1)) / a.G);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int li = lane & 15, lq = lane >> 4;

  // RB > 4: no prefetch (the next chunk's rows would not fit in registers)
  constexpr bool PREFETCH = RB <= 4;
  double xr[NG][2];
  auto load = [&](int chunk) {
    const int col = chunk * kApCW + 16 * wave + li;
#pragma unroll
    for (int q = 0; q < NG; ++q) {
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int row = 8 * q + 2 * lq + h;
        xr[q][h] = (row < JK && col < a.ns) ? a.X[(r0 + row) * a.ldx + col] : 0.0;
      }
    }
  };
  if (PREFETCH && cb < ce) load(cb);
  for (int c = cb; c < ce; ++c) {
    // keep R's fragments in LDS: read them inside the loop, not hoisted into
    // registers for all chunks
    asm volatile("" ::: "memory");
    double cur[NG][2];
    if (!PREFETCH) load(c);
#pragma unroll
    for (int q = 0; q < NG; ++q) {
      cur[q][0] = xr[q][0];
      cur[q][1] = xr[q][1];
    }
    if (PREFETCH && c + 1 < ce) load(c + 1);
    d4 acc[RB];
#pragma unroll
    for (int t = 0; t < RB; ++t) acc[t] = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int q = 0; q < NG; ++q) {
      const int k = 8 * q + 2 * lq;
#pragma unroll
      for (int t = 0; t < RB; ++t) {
        const d2 rv = *reinterpret_cast<const d2*>(&rs[(t * 16 + li) * LDR + k]);
        acc[t] = mfma64(rv.x, cur[q][0], acc[t]);
        acc[t] = mfma64(rv.y, cur[q][1], acc[t]);
      }
    }
    const int col = c * kApCW + 16 * wave + li;
    if (col < a.ns) {
#pragma unroll
      for (int t = 0; t < RB; ++t) {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int row = t * 16 + 4 * v + lq;
          if (row < JK) a.X[(r0 + row) * a.ldx + col] = acc[t][v];
        }
      }
    }
  }
}

template <int RB>
size_t apply_lds_bytes() {
  return static_cast<size_t>(RB * 16) * (RB * 16 + 2) * sizeof(double);
}

template <int RB, bool SYM>
int launch_nt_group(const NtArgs& a, int nwg, hipStream_t st) {
  hipLaunchKernelGGL((elem_nt_kernel<RB, SYM>), dim3(nwg), dim3(NtTiles<RB, SYM>::NW * 64), 0, st, a);
  CHEFSI_LAUNCHED("elem_nt_kernel");
  return CHEFSI_OK;
}

template <bool SYM>
int dispatch_nt(int rb, const NtArgs& a, int nwg, hipStream_t st) {
  switch (rb) {
    case 1: return launch_nt_group<1, SYM>(a, nwg, st);
    case 2: return launch_nt_group<2, SYM>(a, nwg, st);
    case 3: return launch_nt_group<3, SYM>(a, nwg, st);
    case 4: return launch_nt_group<4, SYM>(a, nwg, st);
    case 5: return launch_nt_group<5, SYM>(a, nwg, st);
    case 6: return launch_nt_group<6, SYM>(a, nwg, st);
    case 7: return launch_nt_group<7, SYM>(a, nwg, st);
    case 8: return launch_nt_group<8, SYM>(a, nwg, st);
    default: return fail(CHEFSI_ERR_ARG, "element products: ALB count above 128");
  }
}

template <int RB>
int launch_apply_group(const ApplyArgs& a, int nwg, hipStream_t st) {
  const size_t lds = apply_lds_bytes<RB>();
  if (lds > 65536) {
    // R_K of 96..128-row elements needs more than 64 KB of LDS (gfx950 has 160 KB)
    static bool raised = false;
    if (!raised) {
      CHEFSI_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(&elem_apply_kernel<RB>),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds)));
      raised = true;
    }
  }
  hipLaunchKernelGGL((elem_apply_kernel<RB>), dim3(nwg), dim3(kApThreads), lds, st, a);
  CHEFSI_LAUNCHED("elem_apply_kernel");
  return CHEFSI_OK;
}

int dispatch_apply(int rb, const ApplyArgs& a, int nwg, hipStream_t st) {
  switch (rb) {
    case 1: return launch_apply_group<1>(a, nwg, st);
    case 2: return launch_apply_group<2>(a, nwg, st);
    case 3: return launch_apply_group<3>(a, nwg, st);
    case 4: return launch_apply_group<4>(a, nwg, st);
    case 5: return launch_apply_group<5>(a, nwg, st);
    case 6: return launch_apply_group<6>(a, nwg, st);
    case 7: return launch_apply_group<7>(a, nwg, st);
    case 8: return launch_apply_group<8>(a, nwg, st);
    default: return fail(CHEFSI_ERR_ARG, "element rotation: ALB count above 128");
  }
}

bool aligned16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }

}  // namespace

int launch_fermi(const double* d_theta, int ns, double n_occ, double kT, double* d_f, double* d_mu,
                 hipStream_t st) {
  hipLaunchKernelGGL(fermi_kernel, dim3(1), dim3(kFermiThreads), 0, st, d_theta, ns, n_occ, kT, d_f, d_mu);
  CHEFSI_LAUNCHED("fermi_kernel");
  return CHEFSI_OK;
}

int elem_nt_slices(const Plan& p, int64_t L) {
  if (L <= 0) return 1;
  const int64_t by_wg = ceil_div(kNtTargetWG, std::max(p.M, 1));
  const int64_t by_len = std::max<int64_t>(1, L / (4 * kNtKC));
  const int64_t S = std::max<int64_t>(1, std::min(by_wg, by_len));
  // slice length rounded to whole chunks; recount the slices it implies
  const int64_t SL = round_up(ceil_div(L, S), kNtKC);
  return static_cast<int>(ceil_div(L, SL));
}

int elem_nt(const Plan& p, const double* A, int64_t lda, const double* B, int64_t ldb, const double* w,
            int64_t L, bool sym, double* d_part, double* d_out, hipStream_t st) {
  const int S = elem_nt_slices(p, L);
  const int64_t SL = L > 0 ? round_up(ceil_div(L, S), kNtKC) : kNtKC;
  NtArgs a;
  a.A = A;
  a.lda = lda;
  a.B = sym ? A : B;
  a.ldb = sym ? lda : ldb;
  a.w = w;
  a.rowoff = p.d_rowoff;
  a.J = p.d_J;
  a.sqoff = p.d_sqoff;
  a.order = p.d_order;
  a.L = L;
  a.S = S;
  a.SL = SL;
  a.part = d_part;
  a.pstride = p.sqtot;
  a.vec = (lda % 2 == 0) && aligned16(A) && (sym || ((ldb % 2 == 0) && aligned16(B)));
  for (size_t gi = 0; gi < p.grp_rb.size(); ++gi) {
    a.start = p.grp_start[gi];
    a.count = p.grp_count[gi];
    const int nwg = a.count * S;
    CHEFSI_TRY(sym ? dispatch_nt<true>(p.grp_rb[gi], a, nwg, st) : dispatch_nt<false>(p.grp_rb[gi], a, nwg, st));
  }
  const int nb = static_cast<int>(ceil_div(static_cast<int64_t>(p.maxJ) * p.maxJ, 256));
  hipLaunchKernelGGL(nt_reduce_kernel, dim3(static_cast<unsigned>(static_cast<int64_t>(nb) * p.M)), dim3(256), 0, st,
                     d_part, p.sqtot, S, nb, p.d_J, p.d_sqoff, sym, d_out);
  CHEFSI_LAUNCHED("nt_reduce_kernel");
  return CHEFSI_OK;
}

int elem_apply(const Plan& p, const double* d_R, double* X, int64_t ldx, int ns, hipStream_t st) {
  if (ns <= 0) return CHEFSI_OK;
  const int nchunk = static_cast<int>(ceil_div(ns, kApCW));
  ApplyArgs a;
  a.R = d_R;
  a.X = X;
  a.ldx = ldx;
  a.ns = ns;
  a.rowoff = p.d_rowoff;
  a.J = p.d_J;
  a.sqoff = p.d_sqoff;
  a.order = p.d_order;
  for (size_t gi = 0; gi < p.grp_rb.size(); ++gi) {
    a.start = p.grp_start[gi];
    a.count = p.grp_count[gi];
    a.G = static_cast<int>(std::max<int64_t>(1, std::min<int64_t>(nchunk, ceil_div(kApTargetWG, a.count))));
    CHEFSI_TRY(dispatch_apply(p.grp_rb[gi], a, a.count * a.G, st));
  }
  return CHEFSI_OK;
}

}  // namespace chefsi
