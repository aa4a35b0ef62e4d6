// Dense FP64 kernels of the subspace problem (Algorithm 1 steps 3-5) for
// gfx950: tall-skinny GEMMs on FP64 MFMA (Gram matrix Y^T Y, projection
// Yhat^T (H Yhat), rotation Yhat Q, blocked triangular-solve updates),
// blocked Cholesky, row-wise triangular substitution, and small helpers.
#include "common.h"

namespace chefsi {

namespace {

typedef double d4 __attribute__((ext_vector_type(4)));

constexpr int GT = 128;   // output tile (rows and columns)
constexpr int GK = 16;    // reduction rows per LDS chunk
constexpr int GNT = 256;  // threads: 2 x 2 waves of 64 x 64 outputs
// LDS operand chunk, two layouts of 2304 doubles each:
//   k-major  [GK][LDK]: rows 144 doubles apart, so the two k rows a half-wave
//            reads fall on disjoint halves of the 64 banks;
//   idx-major [GT][LDI]: rows 17 doubles apart (an odd stride), so the 16
//            rows a quarter-wave reads fall on distinct bank pairs.
constexpr int LDK = 144;
constexpr int LDI = 17;
constexpr int GBUF = GK * LDK;
static_assert(GT * LDI <= GBUF, "both operand layouts fit one buffer");

typedef double d4 __attribute__((ext_vector_type(4)));

// FP64 MFMA 16x16x4: lane l supplies A[l%16][l/16] and B[l/16][l%16]; output
// element v of lane l is D[4v + l/16][l%16].
__device__ __forceinline__ d4 mma64(double a, double b, d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

struct GemmArgs {
  const double* A;
  int64_t lda;
  const double* B;
  int64_t ldb;
  double* C;
  int64_t ldc;
  int64_t m, n, k;
  double alpha, beta;
  int64_t kper;     // reduction rows per split (multiple of GK)
  double* part;     // split partials [split][m][n] or null (direct epilogue)
  bool upper_only;
  bool b_upper;     // B is upper triangular: column tile tj needs k < (tj+1)*GT only
  int tri_tiles;    // upper_only: number of upper-triangle tiles (1-D grid)
  int tn_tiles;     // upper_only: tiles per row of the square tile grid
  const int* skip;  // if set and any of skip[0..2] is nonzero, write nothing
  // batched launch (bsc != 0): blockIdx.z is the batch index and problem z
  // reads A + z bsa, B + z bsb and writes C + z bsc (no reduction splits)
  int64_t bsa = 0, bsb = 0, bsc = 0;
};

// One GT x GK operand chunk, 16 bytes (two doubles) per thread per load, four
// loads per thread; out-of-range elements are zero.
//   KMAJOR:  X[k][idx] (row stride ld): load e covers k row 4e + tid/64,
//            idx pair 2*(tid%64): a wave reads one whole 1 KB row.
//   !KMAJOR: X[idx][k]: load e covers idx row 32e + tid/8, k pair 2*(tid%8):
//            eight lanes read one 128-byte row segment.
// VEC: ld even and X 16-byte aligned (pairs are single 16-byte loads).
template <bool KMAJOR, bool VEC>
__device__ __forceinline__ void load_chunk(const double* X, int64_t ld, int64_t idx0, int64_t lim,
                                           int64_t kc, int64_t kend, double2 (&r)[4]) {
  const int tid = threadIdx.x;
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    int64_t row, col, rlim, clim;   // row/col of X in memory
    if constexpr (KMAJOR) {
      row = kc + 4 * e + (tid >> 6);
      col = idx0 + 2 * (tid & 63);
      rlim = kend;
      clim = lim;
    } else {
      row = idx0 + 32 * e + (tid >> 3);
      col = kc + 2 * (tid & 7);
      rlim = lim;
      clim = kend;
    }
    double2 v = make_double2(0.0, 0.0);
    if (row < rlim) {
      const double* src = X + row * ld + col;
      if (VEC && col + 1 < clim) {
        v = *reinterpret_cast<const double2*>(src);
      } else {
        if (col < clim) v.x = src[0];
        if (col + 1 < clim) v.y = src[1];
      }
    }
    r[e] = v;
  }
}

template <bool KMAJOR>
__device__ __forceinline__ void store_chunk(double* S, const double2 (&r)[4]) {
  const int tid = threadIdx.x;
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    if constexpr (KMAJOR) {
      *reinterpret_cast<double2*>(S + (4 * e + (tid >> 6)) * LDK + 2 * (tid & 63)) = r[e];
    } else {
      double* d = S + (32 * e + (tid >> 3)) * LDI + 2 * (tid & 7);
      d[0] = r[e].x;
      d[1] = r[e].y;
    }
  }
}

// Unguarded operand pointers of this thread for the four loads of a chunk
// (fully interior tiles with 16-byte-aligned rows), advanced chunk by chunk.
template <bool KMAJOR>
struct FastPtr {
  const double* p[4];
  int64_t step;
  __device__ __forceinline__ void init(const double* X, int64_t ld, int64_t idx0, int64_t kc) {
    const int tid = threadIdx.x;
#pragma unroll
    for (int e = 0; e < 4; ++e)
      p[e] = KMAJOR ? X + (kc + 4 * e + (tid >> 6)) * ld + idx0 + 2 * (tid & 63)
                    : X + (idx0 + 32 * e + (tid >> 3)) * ld + kc + 2 * (tid & 7);
    step = KMAJOR ? GK * ld : GK;
  }
  __device__ __forceinline__ void load(int c, double2 (&r)[4]) const {
    const int64_t o = c * step;
#pragma unroll
    for (int e = 0; e < 4; ++e) r[e] = *reinterpret_cast<const double2*>(p[e] + o);
  }
};

// MFMA operand of lane l for reduction step kk (k = 4kk + l/16) and index
// base + l%16.
template <bool KMAJOR>
__device__ __forceinline__ double frag(const double* S, int kk, int base, int lane) {
  if constexpr (KMAJOR) return S[(4 * kk + (lane >> 4)) * LDK + base + (lane & 15)];
  return S[(base + (lane & 15)) * LDI + 4 * kk + (lane >> 4)];
}

// acc += op(A)[i0.., k] op(B)[k, j0..] over k in [kbeg, kend) for a 128 x 128
// tile; wave (wr, wc) owns rows 64wr..+63 and columns 64wc..+63 as 4 x 4
// sixteen-square fragments.  A is k-major (AK) or row-major; B is k-major (BK)
// or stored n x k (its rows are the output columns).  Interior tiles with
// aligned rows take unguarded loads for every full chunk; the LDS operands of
// reduction step kk+1 are read while the MFMAs of step kk run.
template <bool AK, bool BK, bool VEC>
__device__ __forceinline__ void tile_mma(const double* A, int64_t lda, const double* B, int64_t ldb,
                                         int64_t m, int64_t n, int64_t kbeg, int64_t kend, int64_t i0,
                                         int64_t j0, double* sA, double* sB, d4 (&acc)[4][4]) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int ib = (wave >> 1) * 64, jb = (wave & 1) * 64;
  const int nch = kend > kbeg ? static_cast<int>(ceil_div(kend - kbeg, GK)) : 0;
  const int nfull = kend > kbeg ? static_cast<int>((kend - kbeg) / GK) : 0;
  const bool fast = VEC && i0 + GT <= m && j0 + GT <= n;
  FastPtr<AK> pa;
  FastPtr<BK> pb;
  pa.init(A, lda, i0, kbeg);
  pb.init(B, ldb, j0, kbeg);
  double2 ra[4], rb[4];
  auto gload = [&](int c) {
    if (fast && c < nfull) {
      pa.load(c, ra);
      pb.load(c, rb);
    } else {
      const int64_t kc = kbeg + static_cast<int64_t>(c) * GK;
      load_chunk<AK, VEC>(A, lda, i0, m, kc, kend, ra);
      load_chunk<BK, VEC>(B, ldb, j0, n, kc, kend, rb);
    }
  };
  auto rd = [&](const double* SA, const double* SB, int kk, double (&av)[4], double (&bv)[4]) {
#pragma unroll
    for (int p = 0; p < 4; ++p) av[p] = frag<AK>(SA, kk, ib + 16 * p, lane);
#pragma unroll
    for (int q = 0; q < 4; ++q) bv[q] = frag<BK>(SB, kk, jb + 16 * q, lane);
  };
  auto mm = [&](const double (&av)[4], const double (&bv)[4]) {
#pragma unroll
    for (int p = 0; p < 4; ++p)
#pragma unroll
      for (int q = 0; q < 4; ++q) acc[p][q] = mma64(av[p], bv[q], acc[p][q]);
  };
  double a0[4], b0[4], a1[4], b1[4];
  if (nch > 0) {
    gload(0);
    store_chunk<AK>(sA, ra);
    store_chunk<BK>(sB, rb);
  }
  __syncthreads();
  if (nch > 0) rd(sA, sB, 0, a0, b0);
  // the last reduction step of a chunk runs after the barrier, behind the
  // LDS reads of the next chunk's first step
  for (int c = 0; c < nch; ++c) {
    const int buf = c & 1;
    if (c + 1 < nch) gload(c + 1);
    const double* SA = sA + buf * GBUF;
    const double* SB = sB + buf * GBUF;
    rd(SA, SB, 1, a1, b1);
    mm(a0, b0);
    rd(SA, SB, 2, a0, b0);
    mm(a1, b1);
    rd(SA, SB, 3, a1, b1);
    mm(a0, b0);
    if (c + 1 < nch) {
      store_chunk<AK>(sA + (buf ^ 1) * GBUF, ra);
      store_chunk<BK>(sB + (buf ^ 1) * GBUF, rb);
    }
    __syncthreads();
    if (c + 1 < nch) rd(sA + (buf ^ 1) * GBUF, sB + (buf ^ 1) * GBUF, 0, a0, b0);
    mm(a1, b1);
  }
}

// Output element v of fragment (p, q) of this lane: tile row / column.
__device__ __forceinline__ int out_row(int wave, int lane, int p, int v) {
  return (wave >> 1) * 64 + 16 * p + 4 * v + (lane >> 4);
}
__device__ __forceinline__ int out_col(int wave, int lane, int q) { return (wave & 1) * 64 + 16 * q + (lane & 15); }

// C tile (128 x 128) = sum_k op(A)[i][k] B[k][j] over this split's k range.
// A_KMAJOR: A stored k x m (TN form); otherwise m x k (NN form).  B is k x n.
template <bool A_KMAJOR, bool VEC>
__global__ __launch_bounds__(GNT, 2) void gemm_kernel(GemmArgs g) {
  int ti, tj, split;
  if (g.upper_only) {
    // 1-D grid over the upper-triangle tiles only (split-major), so that no
    // work-group idles and consecutive work-groups -- which the hardware
    // deals out to the XCDs in turn -- carry equal work
    const int ntiles = g.tri_tiles;
    split = blockIdx.x / ntiles;
    int t = blockIdx.x - split * ntiles;
    ti = 0;
    int rowlen = g.tn_tiles;
    while (t >= rowlen) {
      t -= rowlen;
      ++ti;
      --rowlen;
    }
    tj = ti + t;
  } else {
    // skew the column tile by the row tile: work-group b runs on XCD b % 8, and
    // without the skew one XCD would receive every tile of one column residue
    // (uneven work when B is triangular)
    ti = blockIdx.y;
    tj = (blockIdx.x + blockIdx.y) % gridDim.x;
    split = blockIdx.z;
  }
  if (g.upper_only && ti > tj) return;
  if (g.skip != nullptr && (g.skip[0] | g.skip[1] | g.skip[2]) != 0) return;
  const double* gA = g.A;
  const double* gB = g.B;
  double* gC = g.C;
  if (g.bsc != 0) {
    gA += split * g.bsa;
    gB += split * g.bsb;
    gC += split * g.bsc;
    split = 0;
  }
  __shared__ __attribute__((aligned(16))) double sA[2 * GBUF];
  __shared__ __attribute__((aligned(16))) double sB[2 * GBUF];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t i0 = static_cast<int64_t>(ti) * GT, j0 = static_cast<int64_t>(tj) * GT;
  const int64_t kbeg = static_cast<int64_t>(split) * g.kper;
  int64_t kend = kbeg + g.kper;
  if (kend > g.k) kend = g.k;
  if (g.b_upper && kend > j0 + GT) kend = j0 + GT;
  d4 acc[4][4];
#pragma unroll
  for (int p = 0; p < 4; ++p)
#pragma unroll
    for (int q = 0; q < 4; ++q) acc[p][q] = d4{0.0, 0.0, 0.0, 0.0};
  tile_mma<A_KMAJOR, true, VEC>(gA, g.lda, gB, g.ldb, g.m, g.n, kbeg, kend, i0, j0, sA, sB, acc);
#pragma unroll
  for (int p = 0; p < 4; ++p)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int64_t i = i0 + out_row(wave, lane, p, v);
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int64_t j = j0 + out_col(wave, lane, q);
        if (i < g.m && j < g.n) {
          if (g.part != nullptr) {
            g.part[(static_cast<int64_t>(split) * g.m + i) * g.n + j] = acc[p][q][v];
          } else {
            double val = g.alpha * acc[p][q][v];
            if (g.beta != 0.0) val += g.beta * gC[i * g.ldc + j];
            gC[i * g.ldc + j] = val;
          }
        }
      }
    }
}

// Gradient onto the stored blocks (block-sparse "SDDMM"):
//   Hbar_{K;s} += alpha * A[rows of K] * B[rows of K'_s]^T,
// reduction over the ns columns; one work-group per 128 x 128 tile of a
// stored block (blocks of up to 256 x 256: blockIdx.y picks the tile).
struct SddmmArgs {
  const double* A;
  int64_t lda;
  const double* B;
  int64_t ldb;
  double* Hbar;
  const int64_t* hoff;
  const int32_t* nbr;
  const int32_t* J;
  const int64_t* rowoff;
  int S;
  int ns;
  double alpha;
  const double* alpha_dev;   // optional device factor (e.g. a recurrence coefficient)
};

template <bool VEC>
__global__ __launch_bounds__(GNT, 2) void sddmm_kernel(SddmmArgs g) {
  __shared__ __attribute__((aligned(16))) double sA[2 * GBUF];
  __shared__ __attribute__((aligned(16))) double sB[2 * GBUF];
  const int blk = blockIdx.x;
  const int K = blk / g.S;
  const int Kp = g.nbr[blk];
  const int m = g.J[K], n = g.J[Kp];
  const int i0 = (blockIdx.y >> 1) * GT, j0 = (blockIdx.y & 1) * GT;
  if (i0 >= m || j0 >= n) return;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  d4 acc[4][4];
#pragma unroll
  for (int p = 0; p < 4; ++p)
#pragma unroll
    for (int q = 0; q < 4; ++q) acc[p][q] = d4{0.0, 0.0, 0.0, 0.0};
  tile_mma<false, false, VEC>(g.A + g.rowoff[K] * g.lda, g.lda, g.B + g.rowoff[Kp] * g.ldb, g.ldb, m, n, 0,
                              g.ns, i0, j0, sA, sB, acc);
  double* C = g.Hbar + g.hoff[blk];
  const double alpha = g.alpha * (g.alpha_dev ? *g.alpha_dev : 1.0);
#pragma unroll
  for (int p = 0; p < 4; ++p)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int i = i0 + out_row(wave, lane, p, v);
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int j = j0 + out_col(wave, lane, q);
        if (i < m && j < n) C[i * n + j] += alpha * acc[p][q][v];
      }
    }
}

// Symmetric rank-2k update of the upper triangle of a row-major n x n C:
//   C[i][j] += alpha * sum_l (A1[i][l] B1[j][l] + A2[i][l] B2[j][l]),  j >= i,
// all four operands n x k row-major with stride ld.  One work-group per
// upper-triangle tile; both products accumulate in the same registers, so C
// is read and written once.
struct Syr2kArgs {
  const double* A1;
  const double* B1;
  const double* A2;
  const double* B2;
  int64_t ld;
  double* C;
  int64_t ldc;
  int64_t n, k;
  double alpha;
  int tn_tiles;
};

template <bool VEC>
__global__ __launch_bounds__(GNT, 2) void syr2k_upper_kernel(Syr2kArgs g) {
  int t = blockIdx.x, ti = 0, rowlen = g.tn_tiles;
  while (t >= rowlen) {
    t -= rowlen;
    ++ti;
    --rowlen;
  }
  const int tj = ti + t;
  __shared__ __attribute__((aligned(16))) double sA[2 * GBUF];
  __shared__ __attribute__((aligned(16))) double sB[2 * GBUF];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t i0 = static_cast<int64_t>(ti) * GT, j0 = static_cast<int64_t>(tj) * GT;
  d4 acc[4][4];
#pragma unroll
  for (int p = 0; p < 4; ++p)
#pragma unroll
    for (int q = 0; q < 4; ++q) acc[p][q] = d4{0.0, 0.0, 0.0, 0.0};
  // every wave's last LDS read of the first product precedes its final
  // barrier, so the second product may refill the buffers at once
  tile_mma<false, false, VEC>(g.A1, g.ld, g.B1, g.ld, g.n, g.n, 0, g.k, i0, j0, sA, sB, acc);
  tile_mma<false, false, VEC>(g.A2, g.ld, g.B2, g.ld, g.n, g.n, 0, g.k, i0, j0, sA, sB, acc);
#pragma unroll
  for (int p = 0; p < 4; ++p)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int64_t i = i0 + out_row(wave, lane, p, v);
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int64_t j = j0 + out_col(wave, lane, q);
        if (j >= i && j < g.n) g.C[i * g.ldc + j] += g.alpha * acc[p][q][v];
      }
    }
}

__global__ void split_reduce_kernel(const double* part, int splits, int64_t m, int64_t n,
                                    double alpha, double beta, double* C, int64_t ldc,
                                    bool upper_only) {
  const int64_t total = m * n;
  const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
  for (int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; t < total; t += stride) {
    const int64_t i = t / n, j = t - (t / n) * n;
    if (upper_only && (i / GT) > (j / GT)) continue;
    double s = 0.0;
    for (int sp = 0; sp < splits; ++sp) s += part[sp * total + t];
    double v = alpha * s;
    if (beta != 0.0) v += beta * C[i * ldc + j];
    C[i * ldc + j] = v;
  }
}

// mode 0: (A + A^T)/2; 1: copy the upper triangle to the lower; 2: copy the
// lower triangle to the upper (tril(A) + tril(A,-1)^T).
__global__ void symmetrize_kernel(double* A, int64_t lda, int n, int mode) {
  const int64_t total = static_cast<int64_t>(n) * n;
  const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
  for (int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; t < total; t += stride) {
    const int64_t i = t / n, j = t - (t / n) * n;
    if (i >= j) continue;
    if (mode == 1) {
      A[j * lda + i] = A[i * lda + j];
    } else if (mode == 2) {
      A[i * lda + j] = A[j * lda + i];
    } else {
      const double v = 0.5 * (A[i * lda + j] + A[j * lda + i]);
      A[i * lda + j] = v;
      A[j * lda + i] = v;
    }
  }
}

// Lane l's value of a wave-uniform read (v_readlane), for a double.
__device__ __forceinline__ double rdlane(double v, int l) {
  const long long x = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane(static_cast<int>(x), l);
  const int hi = __builtin_amdgcn_readlane(static_cast<int>(x >> 32), l);
  return __longlong_as_double((static_cast<long long>(hi) << 32) | static_cast<unsigned int>(lo));
}

// Unblocked Cholesky of one w x w diagonal block (upper, in place) and the
// inverse of the factor, by one wave: lane t holds column t of the block
// (padded to HB with the identity) and, afterwards, column t of the inverse.
// Step j publishes row j of the factor in LDS, from where every lane reads
// the multipliers of its column's update; the inverse reads the rows of U
// back from LDS.  Only the upper triangle (a[r], r <= t) is meaningful: the
// updates run unmasked, and what they leave below the diagonal never enters
// an entry on or above it (entry (r, t) depends on entries (j, r) and (j, t)
// with j < r <= t only) and is not written out.  The factor is written back
// to S, its inverse to T (w x w, row stride w).
constexpr int CB = 64;   // diagonal blocks of the row-wise triangular solves
#ifndef CHEFSI_CHOL_CB
#define CHEFSI_CHOL_CB 64
#endif
constexpr int HB = CHEFSI_CHOL_CB;   // diagonal block of the blocked Cholesky (<= 64: one lane per column)
static_assert(HB >= 2 && HB <= 64 && HB % 2 == 0, "one lane per column, rows read in pairs");
__global__ __launch_bounds__(64) void potf2_inv_kernel(double* S, int64_t lds, int b0, int w, double* T,
                                                       int* status) {
  __shared__ __attribute__((aligned(16))) double sU[HB][HB];   // sU[j][t] = U[j][t] for t >= j
  __shared__ double sT[HB][HB];                                // sT[i][t] = U^{-1}[i][t]
  __shared__ double sR[HB];                                    // 1 / U[j][j]
  const int t = threadIdx.x;
  const bool col = t < w;
  const int tc = col ? t : w - 1;   // clamped column: every load is in bounds
  double a[HB];
#pragma unroll
  for (int r = 0; r < HB; ++r) {
    const int rc = r < w ? r : w - 1;
    const double v = S[static_cast<int64_t>(b0 + rc) * lds + b0 + tc];
    a[r] = (col && r < w) ? v : (r == t ? 1.0 : 0.0);
  }
  // status: 1 = a pivot not above zero, 2 = a pivot that is not finite.  A
  // failed pivot becomes NaN, which every later pivot inherits, so only the
  // first failure names the cause: within the block the first failing pivot,
  // across blocks (launched in order) the first block to fail.
  int bad = 0;
#pragma unroll
  for (int j = 0; j < HB; ++j) {
    const double d = rdlane(a[j], j);
    double piv = sqrt(d);
    if (!(d > 0.0) || !isfinite(d)) {
      if (bad == 0) bad = (d == d && !isinf(d)) ? 1 : 2;
      piv = __builtin_nan("");
    }
    const double rp = 1.0 / piv;
    a[j] = (t == j) ? piv : a[j] * rp;
    if (t < HB) sU[j][t] = a[j];
    if (t == 0) sR[j] = rp;
    __syncthreads();
    // a[r] -= U[j][r] U[j][t] for r > j, the multipliers read in pairs
#pragma unroll
    for (int r = (j + 1) & ~1; r < HB; r += 2) {
      const double2 u = *reinterpret_cast<const double2*>(&sU[j][r]);
      if (r > j) a[r] -= u.x * a[j];
      a[r + 1] -= u.y * a[j];
    }
    // the updates happen here: sunk to the steps that use them, they would
    // keep every multiplier read so far alive
#pragma unroll
    for (int r = j + 1; r < HB; ++r) asm volatile("" : "+v"(a[r]));
  }
  // column t of U^{-1}: T[i][t] = (delta_it - sum_{k>i} U[i][k] T[k][t]) / U[i][i]
  // (zero for i > t), the sum in four interleaved partial sums
  double ti[HB];
#pragma unroll
  for (int i = HB - 1; i >= 0; --i) {
    double p[4] = {(t == i) ? 1.0 : 0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int k = (i + 1) & ~1; k < HB; k += 2) {
      const double2 u = *reinterpret_cast<const double2*>(&sU[i][k]);
      if (k > i) p[(k - i - 1) & 3] -= u.x * ti[k];
      p[(k - i) & 3] -= u.y * ti[k + 1];
    }
    ti[i] = ((p[0] + p[1]) + (p[2] + p[3])) * sR[i];
    if (t < HB) sT[i][t] = ti[i];
    // keep each row's LDS reads in its own iteration (hoisted, they would
    // hold every row of U in registers at once)
    __builtin_amdgcn_sched_barrier(0);
  }
  __syncthreads();
  // both results leave through LDS, row by row (a rolled loop: per-row
  // addresses are not held in registers)
  for (int r = 0; r < w; ++r) {
    if (col) {
      S[static_cast<int64_t>(b0 + r) * lds + b0 + t] = (r <= t) ? sU[r][t] : 0.0;
      T[r * w + t] = sT[r][t];
    }
  }
  if (t == 0 && bad) atomicCAS(status, 0, bad);
}

__global__ void zero_lower_kernel(double* A, int64_t lda, int n) {
  const int64_t total = static_cast<int64_t>(n) * n;
  const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
  for (int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; t < total; t += stride) {
    const int64_t i = t / n, j = t - (t / n) * n;
    if (i > j) A[i * lda + j] = 0.0;
  }
}

// Y[:, b0:b0+w] <- Y[:, b0:b0+w] U_bb^{-1} row by row (forward substitution),
// 64 rows per work-group.
__global__ __launch_bounds__(64) void trsm_diag_kernel(double* Y, int64_t ldy, int64_t nrows,
                                                       const double* U, int64_t ldu, int b0, int w) {
  __shared__ double Ub[CB][CB + 1];
  __shared__ double Yb[CB][CB + 1];
  const int tid = threadIdx.x;
  const int64_t r0 = static_cast<int64_t>(blockIdx.x) * 64;
  for (int t = tid; t < w * w; t += 64) {
    const int r = t / w, c = t - (t / w) * w;
    Ub[r][c] = U[static_cast<int64_t>(b0 + r) * ldu + b0 + c];
  }
  for (int r = 0; r < 64; ++r) {
    const int64_t row = r0 + r;
    if (tid < w) Yb[r][tid] = (row < nrows) ? Y[row * ldy + b0 + tid] : 0.0;
  }
  __syncthreads();
  for (int c = 0; c < w; ++c) {
    double a0 = Yb[tid][c], a1 = 0.0;
    int q = 0;
    for (; q + 1 < c; q += 2) {
      a0 -= Yb[tid][q] * Ub[q][c];
      a1 -= Yb[tid][q + 1] * Ub[q + 1][c];
    }
    if (q < c) a0 -= Yb[tid][q] * Ub[q][c];
    Yb[tid][c] = (a0 + a1) / Ub[c][c];
  }
  __syncthreads();
  for (int r = 0; r < 64; ++r) {
    const int64_t row = r0 + r;
    if (tid < w && row < nrows) Y[row * ldy + b0 + tid] = Yb[r][tid];
  }
}

// Y[:, b0:b0+w] <- Y[:, b0:b0+w] L_bb^{-1} with L lower triangular (backward
// substitution over the block's columns), 64 rows per work-group.
__global__ __launch_bounds__(64) void trsm_diag_lower_kernel(double* Y, int64_t ldy, int64_t nrows,
                                                             const double* L, int64_t ldl, int b0, int w) {
  __shared__ double Lb[CB][CB + 1];
  __shared__ double Yb[CB][CB + 1];
  const int tid = threadIdx.x;
  const int64_t r0 = static_cast<int64_t>(blockIdx.x) * 64;
  for (int t = tid; t < w * w; t += 64) {
    const int r = t / w, c = t - (t / w) * w;
    Lb[r][c] = L[static_cast<int64_t>(b0 + r) * ldl + b0 + c];
  }
  for (int r = 0; r < 64; ++r) {
    const int64_t row = r0 + r;
    if (tid < w) Yb[r][tid] = (row < nrows) ? Y[row * ldy + b0 + tid] : 0.0;
  }
  __syncthreads();
  for (int c = w - 1; c >= 0; --c) {
    double acc = Yb[tid][c];
    for (int q = c + 1; q < w; ++q) acc -= Yb[tid][q] * Lb[q][c];
    Yb[tid][c] = acc / Lb[c][c];
  }
  __syncthreads();
  for (int r = 0; r < 64; ++r) {
    const int64_t row = r0 + r;
    if (tid < w && row < nrows) Y[row * ldy + b0 + tid] = Yb[r][tid];
  }
}

__global__ void fill_f64_kernel(double* d, int64_t count, double v) {
  const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
  for (int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; t < count; t += stride)
    d[t] = v;
}

__global__ void fill_int_kernel(int* d, int64_t count, int v) {
  const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
  for (int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; t < count; t += stride)
    d[t] = v;
}

// Sign of column j of a column-major eigenvector matrix: +1 if its
// largest-magnitude entry (lowest row index on ties) is positive.
__global__ __launch_bounds__(256) void colsign_kernel(const double* V, int64_t ldv, int n, double* sign) {
  __shared__ double sv[256];
  __shared__ int si[256];
  const int j = blockIdx.x, tid = threadIdx.x;
  const double* col = V + static_cast<int64_t>(j) * ldv;
  double best = -1.0;
  int bi = n;
  for (int i = tid; i < n; i += 256) {
    const double a = fabs(col[i]);
    if (a > best) {
      best = a;
      bi = i;
    }
  }
  sv[tid] = best;
  si[tid] = bi;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (tid < s) {
      const double o = sv[tid + s];
      const int oi = si[tid + s];
      if (o > sv[tid] || (o == sv[tid] && oi < si[tid])) {
        sv[tid] = o;
        si[tid] = oi;
      }
    }
    __syncthreads();
  }
  if (tid == 0) sign[j] = (si[0] < n && col[si[0]] < 0.0) ? -1.0 : 1.0;
}

// B[c][r] = A[r][c] * (scale ? scale[r] : 1), 32x32 LDS tiles.
__global__ __launch_bounds__(256) void transpose_kernel(const double* A, int64_t lda, double* B,
                                                        int64_t ldb, int rows, int cols,
                                                        const double* scale) {
  __shared__ double t[32][33];
  const int bx = blockIdx.x * 32, by = blockIdx.y * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  for (int yy = ty; yy < 32; yy += 8) {
    const int r = by + yy, c = bx + tx;
    t[yy][tx] = (r < rows && c < cols) ? A[static_cast<int64_t>(r) * lda + c] * (scale ? scale[r] : 1.0) : 0.0;
  }
  __syncthreads();
  for (int yy = ty; yy < 32; yy += 8) {
    const int c = bx + yy, r = by + tx;
    if (r < rows && c < cols) B[static_cast<int64_t>(c) * ldb + r] = t[tx][yy];
  }
}

unsigned grid1(int64_t total) {
  int64_t g = ceil_div(total, 256);
  if (g < 1) g = 1;
  if (g > 65536) g = 65536;
  return static_cast<unsigned>(g);
}

// operand rows can be read as aligned 16-byte pairs
bool vec_ok(const double* X, int64_t ld) { return (ld % 2) == 0 && (reinterpret_cast<uintptr_t>(X) & 15u) == 0; }

// Splits of the reduction for a launch of `tiles` output tiles: at least
// enough work-groups to fill the chip, then more until the last round of
// work-groups is nearly full (all work-groups carry equal work, so a round
// that is 1/8 full costs as much as a full one).  kGemmSlots = 256 CUs x 2
// resident work-groups of this kernel.
constexpr int64_t kGemmSlots = 512;
int choose_splits(int64_t tiles, int64_t k, int64_t kmin) {
  if (tiles < 1) tiles = 1;
  int64_t maxs = ceil_div(k, kmin);
  if (maxs > 64) maxs = 64;
  if (maxs < 1) maxs = 1;
  int64_t s = ceil_div(2048, tiles);
  if (s > maxs) s = maxs;
  if (s < 1) s = 1;
  for (; s < maxs; ++s) {
    const int64_t wgs = tiles * s;
    const int64_t rounds = ceil_div(wgs, kGemmSlots);
    if (wgs * 100 >= rounds * kGemmSlots * 97) break;   // last round at least ~3/4 full
  }
  return static_cast<int>(s);
}

}  // namespace

size_t gemm_tn_split_ws_elems(int64_t m, int64_t n, int64_t k, int64_t kmin) {
  // the upper-triangle-only launch has fewer tiles, hence the most splits
  const int64_t tm = ceil_div(m, GT);
  const int64_t tiles = (m == n) ? (tm * (tm + 1)) / 2 : tm * ceil_div(n, GT);
  const int s = choose_splits(tiles, k, kmin);
  return s > 1 ? static_cast<size_t>(s) * m * n : 0;
}

int gemm_tn(int64_t m, int64_t n, int64_t k, double alpha, const double* A, int64_t lda,
            const double* B, int64_t ldb, double beta, double* C, int64_t ldc, bool upper_only,
            double* d_split_ws, size_t split_ws_elems, hipStream_t st, int64_t kmin) {
  if (m <= 0 || n <= 0) return CHEFSI_OK;
  const int64_t tm = ceil_div(m, GT), tn = ceil_div(n, GT);
  int splits = choose_splits(upper_only ? (tm * (tm + 1)) / 2 : tm * tn, k, kmin);
  if (splits > 1 && (d_split_ws == nullptr || split_ws_elems < static_cast<size_t>(splits) * m * n))
    splits = 1;
  GemmArgs g{A, lda, B, ldb, C, ldc, m, n, k, alpha, beta, 0, nullptr, upper_only, false, 0, 0, nullptr};
  g.kper = round_up(ceil_div(k, splits), GK);
  if (k <= 0) g.kper = GK;
  if (splits > 1) g.part = d_split_ws;
  dim3 grid(static_cast<unsigned>(tn), static_cast<unsigned>(tm), static_cast<unsigned>(splits));
  if (upper_only) {
    if (tm != tn) return fail(CHEFSI_ERR_ARG, "gemm_tn: upper_only needs a square result");
    g.tn_tiles = static_cast<int>(tn);
    g.tri_tiles = static_cast<int>(tn * (tn + 1) / 2);
    grid = dim3(static_cast<unsigned>(g.tri_tiles * splits), 1, 1);
  }
  if (vec_ok(A, lda) && vec_ok(B, ldb))
    gemm_kernel<true, true><<<grid, GNT, 0, st>>>(g);
  else
    gemm_kernel<true, false><<<grid, GNT, 0, st>>>(g);
  CHEFSI_LAUNCHED("gemm_tn");
  if (splits > 1) {
    split_reduce_kernel<<<grid1(m * n), 256, 0, st>>>(d_split_ws, splits, m, n, alpha, beta, C, ldc, upper_only);
    CHEFSI_LAUNCHED("split_reduce");
  }
  return CHEFSI_OK;
}

int gemm_nn(int64_t m, int64_t n, int64_t k, double alpha, const double* A, int64_t lda,
            const double* B, int64_t ldb, double beta, double* C, int64_t ldc, hipStream_t st,
            bool b_upper, const int* skip_if) {
  if (m <= 0 || n <= 0) return CHEFSI_OK;
  const int64_t tm = ceil_div(m, GT), tn = ceil_div(n, GT);
  if (tm > 65535) return fail(CHEFSI_ERR_ARG, "gemm_nn: too many row tiles");
  GemmArgs g{A, lda, B, ldb, C, ldc, m, n, k, alpha, beta, round_up(k > 0 ? k : 1, GK), nullptr, false, b_upper,
             0, 0, skip_if};
  dim3 grid(static_cast<unsigned>(tn), static_cast<unsigned>(tm), 1);
  if (vec_ok(A, lda) && vec_ok(B, ldb))
    gemm_kernel<false, true><<<grid, GNT, 0, st>>>(g);
  else
    gemm_kernel<false, false><<<grid, GNT, 0, st>>>(g);
  CHEFSI_LAUNCHED("gemm_nn");
  return CHEFSI_OK;
}

int syr2k_upper(int64_t n, int64_t k, double alpha, const double* A1, const double* B1, const double* A2,
                const double* B2, int64_t ld, double* C, int64_t ldc, hipStream_t st) {
  if (n <= 0 || k <= 0) return CHEFSI_OK;
  const int64_t tn = ceil_div(n, GT);
  if (tn * (tn + 1) / 2 > 0x7fffffff) return fail(CHEFSI_ERR_ARG, "syr2k_upper: too many tiles");
  Syr2kArgs g{A1, B1, A2, B2, ld, C, ldc, n, k, alpha, static_cast<int>(tn)};
  const unsigned grid = static_cast<unsigned>(tn * (tn + 1) / 2);
  if (vec_ok(A1, ld) && vec_ok(B1, ld) && vec_ok(A2, ld) && vec_ok(B2, ld))
    syr2k_upper_kernel<true><<<grid, GNT, 0, st>>>(g);
  else
    syr2k_upper_kernel<false><<<grid, GNT, 0, st>>>(g);
  CHEFSI_LAUNCHED("syr2k_upper");
  return CHEFSI_OK;
}

// `count` products C_z = alpha A_z B_z + beta C_z of one shape, operand z at
// A + z sa, B + z sb, C + z sc, in one launch.
int gemm_nn_batched(int64_t m, int64_t n, int64_t k, double alpha, const double* A, int64_t lda, int64_t sa,
                    const double* B, int64_t ldb, int64_t sb, double beta, double* C, int64_t ldc, int64_t sc,
                    int64_t count, hipStream_t st, bool b_upper) {
  if (m <= 0 || n <= 0 || count <= 0) return CHEFSI_OK;
  if (count == 1) return gemm_nn(m, n, k, alpha, A, lda, B, ldb, beta, C, ldc, st, b_upper);
  const int64_t tm = ceil_div(m, GT), tn = ceil_div(n, GT);
  if (tm > 65535 || count > 65535) return fail(CHEFSI_ERR_ARG, "gemm_nn_batched: grid too large");
  if (sc == 0) return fail(CHEFSI_ERR_ARG, "gemm_nn_batched: the outputs must not overlap");
  GemmArgs g{A, lda, B, ldb, C, ldc, m, n, k, alpha, beta, round_up(k > 0 ? k : 1, GK), nullptr, false, b_upper,
             0, 0, nullptr};
  g.bsa = sa;
  g.bsb = sb;
  g.bsc = sc;
  dim3 grid(static_cast<unsigned>(tn), static_cast<unsigned>(tm), static_cast<unsigned>(count));
  // every operand pointer of the batch is aligned like the first when the strides are even
  const bool vec = vec_ok(A, lda) && vec_ok(B, ldb) && sa % 2 == 0 && sb % 2 == 0;
  if (vec)
    gemm_kernel<false, true><<<grid, GNT, 0, st>>>(g);
  else
    gemm_kernel<false, false><<<grid, GNT, 0, st>>>(g);
  CHEFSI_LAUNCHED("gemm_nn_batched");
  return CHEFSI_OK;
}

int launch_symmetrize(double* A, int64_t lda, int n, int mode, hipStream_t st) {
  symmetrize_kernel<<<grid1(static_cast<int64_t>(n) * n), 256, 0, st>>>(A, lda, n, mode);
  CHEFSI_LAUNCHED("symmetrize");
  return CHEFSI_OK;
}

int cholesky_upper(double* S, int64_t lds, int n, int* d_status, double* d_scr, hipStream_t st) {
  // blocked right-looking: factor and invert the diagonal block, panel
  // U12 = U11^{-T} S12 as one GEMM (in place: each work-group reads all of its
  // columns before it writes them), trailing update S22 -= U12^T U12 (upper)
  for (int b0 = 0; b0 < n; b0 += HB) {
    const int w = (n - b0) < HB ? (n - b0) : HB;
    potf2_inv_kernel<<<1, 64, 0, st>>>(S, lds, b0, w, d_scr, d_status);
    CHEFSI_LAUNCHED("potf2_inv");
    const int rest = n - b0 - w;
    if (rest > 0) {
      double* P = S + static_cast<int64_t>(b0) * lds + b0 + w;
      CHEFSI_TRY(gemm_tn(w, rest, w, 1.0, d_scr, w, P, lds, 0.0, P, lds, false, nullptr, 0, st));
      double* T = S + static_cast<int64_t>(b0 + w) * lds + b0 + w;
      CHEFSI_TRY(gemm_tn(rest, rest, w, -1.0, P, lds, P, lds, 1.0, T, lds, true, nullptr, 0, st));
    }
  }
  zero_lower_kernel<<<grid1(static_cast<int64_t>(n) * n), 256, 0, st>>>(S, lds, n);
  CHEFSI_LAUNCHED("zero_lower");
  return CHEFSI_OK;
}

int trsm_right_upper(double* Y, int64_t ldy, int64_t nrows, const double* U, int64_t ldu, int n,
                     hipStream_t st) {
  if (nrows <= 0) return CHEFSI_OK;
  for (int b0 = 0; b0 < n; b0 += CB) {
    const int w = (n - b0) < CB ? (n - b0) : CB;
    if (b0 > 0) {
      CHEFSI_TRY(gemm_nn(nrows, w, b0, -1.0, Y, ldy, U + b0, ldu, 1.0, Y + b0, ldy, st));
    }
    trsm_diag_kernel<<<static_cast<unsigned>(ceil_div(nrows, 64)), 64, 0, st>>>(Y, ldy, nrows, U, ldu, b0, w);
    CHEFSI_LAUNCHED("trsm_diag");
  }
  return CHEFSI_OK;
}

int trsm_right_lower(double* Y, int64_t ldy, int64_t nrows, const double* L, int64_t ldl, int n,
                     hipStream_t st) {
  if (nrows <= 0) return CHEFSI_OK;
  const int nblk = static_cast<int>(ceil_div(n, CB));
  for (int bi = nblk - 1; bi >= 0; --bi) {
    const int b0 = bi * CB;
    const int w = (n - b0) < CB ? (n - b0) : CB;
    const int rest = n - b0 - w;
    if (rest > 0) {
      CHEFSI_TRY(gemm_nn(nrows, w, rest, -1.0, Y + b0 + w, ldy, L + static_cast<int64_t>(b0 + w) * ldl + b0,
                         ldl, 1.0, Y + b0, ldy, st));
    }
    trsm_diag_lower_kernel<<<static_cast<unsigned>(ceil_div(nrows, 64)), 64, 0, st>>>(Y, ldy, nrows, L, ldl, b0, w);
    CHEFSI_LAUNCHED("trsm_diag_lower");
  }
  return CHEFSI_OK;
}

int sddmm_accumulate(const Plan& p, const double* A, int64_t lda, const double* B, int64_t ldb, int ns,
                     double alpha, const double* d_alpha, double* d_Hbar, hipStream_t st) {
  if (ns <= 0) return CHEFSI_OK;
  SddmmArgs g{A, lda, B, ldb, d_Hbar, p.d_hoff, p.d_nbr, p.d_J, p.d_rowoff, p.stencil, ns, alpha, d_alpha};
  const dim3 grid(static_cast<unsigned>(p.M * p.stencil), p.maxJ > GT ? 4u : 1u);
  if (vec_ok(A, lda) && vec_ok(B, ldb))
    sddmm_kernel<true><<<grid, GNT, 0, st>>>(g);
  else
    sddmm_kernel<false><<<grid, GNT, 0, st>>>(g);
  CHEFSI_LAUNCHED("sddmm");
  return CHEFSI_OK;
}

// Inverse of the upper triangular diagonal 64 x 64 blocks of U, one block per
// work-group of one wave: the block's rows go to LDS (a short last block is
// padded with the identity), lane t keeps column t of the inverse in
// registers, T[i][t] = (delta_it - sum_{k>i} U[i][k] T[k][t]) / U[i][i] from
// the last row up (four interleaved partial sums), and the result leaves
// through LDS row by row.  Only the upper triangle of U is read.
__global__ __launch_bounds__(64) void trtri_diag_kernel(const double* U, int64_t ldu, double* T, int64_t ldt,
                                                        int n) {
  __shared__ __attribute__((aligned(16))) double Us[CB][CB];
  __shared__ double Ts[CB][CB + 1];
  const int r0 = blockIdx.x * CB;
  const int w = (n - r0) < CB ? (n - r0) : CB;
  const int t = threadIdx.x;
  for (int r = 0; r < CB; ++r)
    Us[r][t] = (r < w && t < w) ? U[static_cast<int64_t>(r0 + r) * ldu + r0 + t] : (r == t ? 1.0 : 0.0);
  __syncthreads();
  double ti[CB];
#pragma unroll
  for (int i = CB - 1; i >= 0; --i) {
    double p[4] = {(t == i) ? 1.0 : 0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int k = (i + 1) & ~1; k < CB; k += 2) {
      const double2 u = *reinterpret_cast<const double2*>(&Us[i][k]);
      if (k > i) p[(k - i - 1) & 3] -= u.x * ti[k];
      p[(k - i) & 3] -= u.y * ti[k + 1];
    }
    ti[i] = ((p[0] + p[1]) + (p[2] + p[3])) / Us[i][i];
    Ts[i][t] = ti[i];
    // keep each row's LDS reads in its own iteration
    __builtin_amdgcn_sched_barrier(0);
  }
  __syncthreads();
  for (int r = 0; r < w; ++r)
    if (t < w) T[static_cast<int64_t>(r0 + r) * ldt + r0 + t] = Ts[r][t];
}

// Off-diagonal blocks of T = U^{-1}, bottom up: once the diagonal blocks of
// order b are inverted, each aligned pair of them, [r0, r0+b) and
// [r0+b, r0+b+m2) with m2 <= b, is joined by
//   [U11 U12; 0 U22]^{-1} = [T11, -T11 U12 T22; 0, T22]
// (W = U12 T22, then T12 = -T11 W).  The full pairs of one order run as one
// batched launch per product, a ragged last pair on its own; then b doubles.
// W holds at most n^2/4 doubles: pairs * b^2 <= n b / 2 with 2b <= n, and
// b * m2 <= b (n - b) for the ragged pair.
int trtri_offdiag(const double* U, int64_t ldu, double* T, int64_t ldt, int n, double* W, hipStream_t st) {
  for (int64_t b = CB; b < n; b *= 2) {
    const int64_t pairs = n / (2 * b);
    if (pairs > 0) {
      const int64_t su = 2 * b * ldu + 2 * b, stt = 2 * b * ldt + 2 * b;
      CHEFSI_TRY(gemm_nn_batched(b, b, b, 1.0, U + b, ldu, su, T + b * ldt + b, ldt, stt, 0.0, W, b, b * b, pairs, st,
                                 true));
      CHEFSI_TRY(gemm_nn_batched(b, b, b, -1.0, T, ldt, stt, W, b, b * b, 0.0, T + b, ldt, stt, pairs, st, false));
    }
    const int64_t r0 = pairs * 2 * b, m2 = n - r0 - b;
    if (m2 > 0) {
      CHEFSI_TRY(gemm_nn(b, m2, m2, 1.0, U + r0 * ldu + r0 + b, ldu, T + (r0 + b) * ldt + r0 + b, ldt, 0.0, W, m2,
                         st, true));
      CHEFSI_TRY(gemm_nn(b, m2, b, -1.0, T + r0 * ldt + r0, ldt, W, m2, 0.0, T + r0 * ldt + r0 + b, ldt, st));
    }
  }
  return CHEFSI_OK;
}

// T = U^{-1} (n x n, upper triangular, row-major); W is scratch of n*n/4
// doubles (rounded up).
int upper_inverse(const double* U, int n, double* T, double* W, hipStream_t st) {
  CHEFSI_TRY(launch_fill(T, static_cast<int64_t>(n) * n, 0.0, st));
  trtri_diag_kernel<<<static_cast<unsigned>(ceil_div(n, CB)), 64, 0, st>>>(U, n, T, n, n);
  CHEFSI_LAUNCHED("trtri_diag");
  return trtri_offdiag(U, n, T, n, n, W, st);
}

int launch_fill(double* d, int64_t count, double v, hipStream_t st) {
  if (count <= 0) return CHEFSI_OK;
  fill_f64_kernel<<<grid1(count), 256, 0, st>>>(d, count, v);
  CHEFSI_LAUNCHED("fill");
  return CHEFSI_OK;
}

int launch_fill_int(int* d, int64_t count, int v, hipStream_t st) {
  if (count <= 0) return CHEFSI_OK;
  fill_int_kernel<<<grid1(count), 256, 0, st>>>(d, count, v);
  CHEFSI_LAUNCHED("fill_int");
  return CHEFSI_OK;
}

int trmm_upper_upper(const double* A, const double* B, double* C, int n, hipStream_t st) {
  return gemm_nn(n, n, n, 1.0, A, n, B, n, 0.0, C, n, st);
}

int launch_transpose(const double* A, int64_t lda, double* B, int64_t ldb, int rows, int cols,
                     hipStream_t st, const double* row_scale) {
  dim3 grid(static_cast<unsigned>(ceil_div(cols, 32)), static_cast<unsigned>(ceil_div(rows, 32)));
  transpose_kernel<<<grid, 256, 0, st>>>(A, lda, B, ldb, rows, cols, row_scale);
  CHEFSI_LAUNCHED("transpose");
  return CHEFSI_OK;
}

// ------------------------------------------- Cholesky-QR condition bound
// With U the upper Cholesky factor of Y^T Y and T = U^{-1} (both upper, row
// major; entries below the diagonal are ignored), D_j = ||U[:, j]|| = ||y_j||,
// U_e = U D^{-1} and T_e = U_e^{-1} = D T:
//   bound = sqrt(||U_e||_1 ||T_e||_1 ||U_e||_inf ||T_e||_inf) >= kappa_2(Y D^{-1}).

namespace {

// Column sums over row stripes of kCondStripe rows: work-group s adds up rows
// [s*kCondStripe, (s+1)*kCondStripe) for every column (threads walk the
// columns, so each row is read coalesced) and writes one partial per column;
// cond_stripe_reduce_kernel sums the stripes in order.
//   mode 0: part = sum U[k][j]^2                      (k <= j)
//   mode 1: part = sum |U[k][j]|, part2 = sum d_k |T[k][j]|  (k <= j)
constexpr int kCondStripe = 16;

__global__ __launch_bounds__(256) void cond_stripe_kernel(const double* __restrict__ U, const double* __restrict__ T,
                                                          int n, const double* __restrict__ d, int mode,
                                                          double* __restrict__ part, double* __restrict__ part2) {
  const int s = blockIdx.x;
  const int r0 = s * kCondStripe;
  const int r1 = min(n, r0 + kCondStripe);
  for (int j = threadIdx.x; j < n; j += blockDim.x) {
    double a = 0.0, b = 0.0;
    const int kend = min(r1, j + 1);
    for (int k = r0; k < kend; ++k) {
      const int64_t o = static_cast<int64_t>(k) * n + j;
      const double u = U[o];
      if (mode == 0) {
        a += u * u;
      } else {
        a += fabs(u);
        b += d[k] * fabs(T[o]);
      }
    }
    part[static_cast<int64_t>(s) * n + j] = a;
    if (mode == 1) part2[static_cast<int64_t>(s) * n + j] = b;
  }
}

// Stripe sums in stripe order; mode 0: d_j = sqrt(sum); mode 1: cu_j = sum/d_j
// and ct_j = sum2.
__global__ __launch_bounds__(256) void cond_stripe_reduce_kernel(const double* __restrict__ part,
                                                                 const double* __restrict__ part2, int nstripe,
                                                                 int n, int mode, double* __restrict__ d,
                                                                 double* __restrict__ cu, double* __restrict__ ct) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  double a = 0.0, b = 0.0;
  for (int s = 0; s < nstripe; ++s) {
    a += part[static_cast<int64_t>(s) * n + j];
    if (mode == 1) b += part2[static_cast<int64_t>(s) * n + j];
  }
  if (mode == 0) {
    d[j] = sqrt(a);
  } else {
    cu[j] = a / d[j];
    ct[j] = b;
  }
}

__device__ __forceinline__ double block_sum256(double v, double* red) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  const double r = red[0] + red[1] + red[2] + red[3];
  __syncthreads();
  return r;
}

// row sums of |U_e| and |T_e| (work-group per row)
__global__ __launch_bounds__(256) void cond_rowsum_kernel(const double* __restrict__ U, const double* __restrict__ T,
                                                          int n, const double* __restrict__ d,
                                                          double* __restrict__ ru, double* __restrict__ rt) {
  __shared__ double red[4];
  const int i = blockIdx.x;
  const int64_t o = static_cast<int64_t>(i) * n;
  double su = 0.0, stt = 0.0;
  for (int j = i + threadIdx.x; j < n; j += blockDim.x) {
    su += fabs(U[o + j]) / d[j];
    stt += fabs(T[o + j]);
  }
  su = block_sum256(su, red);
  stt = block_sum256(stt, red);
  if (threadIdx.x == 0) {
    ru[i] = su;
    rt[i] = d[i] * stt;
  }
}

__global__ __launch_bounds__(256) void cond_final_kernel(const double* __restrict__ v, int n,
                                                         double* __restrict__ out) {
  __shared__ double red[4][4];
  double m[4] = {0.0, 0.0, 0.0, 0.0};
  for (int j = threadIdx.x; j < n; j += blockDim.x)
    for (int q = 0; q < 4; ++q) m[q] = fmax(m[q], v[static_cast<int64_t>(q) * n + j]);
  for (int q = 0; q < 4; ++q) {
    for (int o = 32; o > 0; o >>= 1) m[q] = fmax(m[q], __shfl_xor(m[q], o));
    if ((threadIdx.x & 63) == 0) red[q][threadIdx.x >> 6] = m[q];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double p = 1.0;
    for (int q = 0; q < 4; ++q) p *= fmax(fmax(red[q][0], red[q][1]), fmax(red[q][2], red[q][3]));
    out[0] = sqrt(p);
  }
}

}  // namespace

size_t cholqr_cond_scratch_elems(int n) {
  const size_t ns = static_cast<size_t>(ceil_div(n, kCondStripe));
  return 5 * static_cast<size_t>(n) + 2 * ns * static_cast<size_t>(n);
}

int cholqr_cond_bound(const double* U, const double* T, int n, double* d_scr, double* d_out, hipStream_t st) {
  if (n <= 0) return CHEFSI_OK;
  double* d = d_scr;
  double* v = d_scr + n;   // cu, ct, ru, rt
  const int nstripe = static_cast<int>(ceil_div(n, kCondStripe));
  double* part = d_scr + 5 * static_cast<int64_t>(n);
  double* part2 = part + static_cast<int64_t>(nstripe) * n;
  const unsigned g = static_cast<unsigned>(ceil_div(n, 256));
  cond_stripe_kernel<<<static_cast<unsigned>(nstripe), 256, 0, st>>>(U, T, n, d, 0, part, part2);
  CHEFSI_LAUNCHED("cond_stripe");
  cond_stripe_reduce_kernel<<<g, 256, 0, st>>>(part, part2, nstripe, n, 0, d, v, v + n);
  CHEFSI_LAUNCHED("cond_stripe_reduce");
  cond_stripe_kernel<<<static_cast<unsigned>(nstripe), 256, 0, st>>>(U, T, n, d, 1, part, part2);
  CHEFSI_LAUNCHED("cond_stripe");
  cond_stripe_reduce_kernel<<<g, 256, 0, st>>>(part, part2, nstripe, n, 1, d, v, v + n);
  CHEFSI_LAUNCHED("cond_stripe_reduce");
  cond_rowsum_kernel<<<static_cast<unsigned>(n), 256, 0, st>>>(U, T, n, d, v + 2 * static_cast<int64_t>(n),
                                                                 v + 3 * static_cast<int64_t>(n));
  CHEFSI_LAUNCHED("cond_rowsum");
  cond_final_kernel<<<1, 256, 0, st>>>(v, n, d_out);
  CHEFSI_LAUNCHED("cond_final");
  return CHEFSI_OK;
}

// Vcm: n x n eigenvectors in column-major order (column j = eigenvector j);
// Q (row-major) gets Q[i][j] = sign_j * Vcm[j*ldv + i].  Q[n..] holds scratch
// for the n signs: the caller passes Q with room for n*ldq + n doubles.
int launch_eigvec_fix(const double* Vcm, int64_t ldv, int n, double* Q, int64_t ldq, hipStream_t st) {
  double* sign = Q + static_cast<int64_t>(n) * ldq;
  colsign_kernel<<<static_cast<unsigned>(n), 256, 0, st>>>(Vcm, ldv, n, sign);
  CHEFSI_LAUNCHED("colsign");
  // Vcm viewed row-major is V^T (row j = eigenvector j): transpose with row scale.
  dim3 grid(static_cast<unsigned>(ceil_div(n, 32)), static_cast<unsigned>(ceil_div(n, 32)));
  transpose_kernel<<<grid, 256, 0, st>>>(Vcm, ldv, Q, ldq, n, n, sign);
  CHEFSI_LAUNCHED("eigvec_transpose");
  return CHEFSI_OK;
}

}  // namespace chefsi
