// Householder reduction of the projected matrix Hhat to symmetric tridiagonal
// form (the first stage of the dense eigensolve of Algorithm 1 step 4), FP64,
// in LAPACK's lower-triangle format (rocSOLVER's tridiagonal
// divide-and-conquer takes D and E unchanged; backtr.hip applies the
// reflectors as stored here):
//   Q = H(0) H(1) ... H(n-2),  H(i) = I - tau_i v_i v_i^T,
//   v_i = 0 above row i+1, v_i(i+1) = 1, v_i(i+2:n) stored in A(i+2:n, i),
//   D(i) = T(i, i), E(i) = T(i+1, i).
// The method is the classic blocked one: panels of kNB columns are reduced
// with delayed updates (the trailing matrix stays at its panel-start values,
// each new column is corrected by the panel's reflectors V and the vectors W),
// and the trailing matrix is updated once per panel, A -= V W^T + W V^T, as a
// rank-2k product.
//
// What differs from the usual sequence of small library kernels is the
// dependency chain per column, cut to two launches:
//   symv kernel   one work-group per 64 x 64 tile of the trailing lower
//                 triangle.  Each work-group first finishes the reflector of the
//                 column (the squared norm comes as per-row-block partial sums,
//                 reduced in the same order by every work-group), then computes
//                 both the row sums A_IJ v_J and, off the diagonal, the column
//                 sums A_IJ^T v_I of its tile, and its share of v^T A v.
//                 Diagonal tiles also form the panel products V^T v and W^T v
//                 of their rows.
//   update kernel one work-group per 64-row block.  Every work-group reduces
//                 the small partial sums (the same order everywhere), finishes
//                 w = tau (A v - V (W^T v) - W (V^T v)) - (tau/2)(w^T v) v for
//                 its rows (w^T v comes from v^T A v and the panel products, no
//                 extra reduction over rows), stores the reflector in LAPACK
//                 form, applies the panel's corrections to the next column and
//                 leaves that column's squared-norm partial sums.
// Every partial sum has a fixed owner and a fixed reduction order, so the
// result does not depend on scheduling.  Column-major storage, A(r, c) at
// A[r + c * lda]; only the lower triangle is read or written.
#include "common.h"

namespace chefsi {
namespace {

constexpr int kTB = 64;    // tile edge of the symmetric product
constexpr int kNB = 64;    // panel width (reflectors per rank-2k update)
constexpr int kTdThreads = 256;

struct TdArgs {
  double* A;
  int64_t lda;
  int n, nT;
  double* Vp;    // n x kNB row-major: panel reflectors, v(i+1) = 1 explicit
  double* Wp;    // n x kNB row-major: panel vectors w
  double* P;     // nT x nT x 64: P[(I nT + K) 64 + r] = part of (A v)(64 I + r) from tile column/row K
  double* S;     // per tile: its share of v^T A v
  double* VV;    // nT x kNB: per row block, part of V^T v
  double* WV;    // nT x kNB: per row block, part of W^T v
  double* nrm;   // nT: per row block, part of the squared norm below the subdiagonal
  double* D;
  double* E;
  double* tau;
};

__device__ __forceinline__ double wave_sum(double v) {
  // xor butterfly: every lane ends with the same value (addition is commutative)
  for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, 64);
  return v;
}

// Householder reflector of column i (LAPACK's dlarfg without its rescaling
// of tiny norms): sigma2 = squared norm of x(2:), alpha = x(1).  Returns tau;
// beta = the new subdiagonal entry, scal = the factor that turns x(2:) into v(2:).
__device__ __forceinline__ double reflector(double sigma2, double alpha, double* beta, double* scal) {
  if (sigma2 == 0.0) {
    *beta = alpha;
    *scal = 0.0;
    return 0.0;
  }
  const double b = -copysign(sqrt(alpha * alpha + sigma2), alpha);
  *beta = b;
  *scal = 1.0 / (alpha - b);
  return (b - alpha) / b;
}

constexpr int kSyWaves = kTdThreads / 64;   // waves per tile
constexpr int kSyCols = kTB / kSyWaves;     // tile columns per wave (16)

__device__ __forceinline__ double wave_part_sum(const double (*red)[kTB], int x) {
  double s = 0.0;
#pragma unroll
  for (int q = 0; q < kSyWaves; ++q) s += red[q][x];
  return s;
}

// Sums of 16 values per lane over the 64 lanes of a wave, all at once: each
// exchange step halves the values a lane holds, then two butterfly steps
// finish.  Lane l ends with the total of value l >> 2 (lanes l, l^1, l^2, l^3
// hold the same total).
__device__ __forceinline__ double wave_sum16(const double (&p)[16], int lane) {
  double q8[8], q4[4], q2[2];
  bool hi = (lane & 32) != 0;
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    const double send = hi ? p[k] : p[k + 8];
    q8[k] = (hi ? p[k + 8] : p[k]) + __shfl_xor(send, 32, 64);
  }
  hi = (lane & 16) != 0;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const double send = hi ? q8[k] : q8[k + 4];
    q4[k] = (hi ? q8[k + 4] : q8[k]) + __shfl_xor(send, 16, 64);
  }
  hi = (lane & 8) != 0;
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    const double send = hi ? q4[k] : q4[k + 2];
    q2[k] = (hi ? q4[k + 2] : q4[k]) + __shfl_xor(send, 8, 64);
  }
  hi = (lane & 4) != 0;
  double q1 = (hi ? q2[1] : q2[0]) + __shfl_xor(hi ? q2[0] : q2[1], 4, 64);
  q1 += __shfl_xor(q1, 2, 64);
  q1 += __shfl_xor(q1, 1, 64);
  return q1;
}

// One work-group per 64 x 64 tile (I, J), I >= J, of the trailing lower
// triangle; wave q holds columns 16q .. 16q+15 of the tile in registers, lane
// = row.  Off the diagonal the tile gives the row sums A_IJ v_J (combined over
// the waves in LDS) and the column sums A_IJ^T v_I (one multi-value wave
// reduction); a diagonal tile splits into its lower part with the diagonal
// (row sums) and its strictly lower part (column sums).
__global__ __launch_bounds__(kTdThreads) void td_symv_kernel(TdArgs a, int i, int j) {
  __shared__ double vI[kTB], vJ[kTB];
  __shared__ double red[kSyWaves][kTB];
  __shared__ double red2[kSyWaves][kTB];
  __shared__ double cs[kTB];
  const int t = threadIdx.x, r = t & 63, q = t >> 6;
  const int T0 = (i + 1) / kTB;
  const int64_t tile = blockIdx.x;
  int Ir = static_cast<int>((sqrt(8.0 * static_cast<double>(tile) + 1.0) - 1.0) * 0.5);
  while (static_cast<int64_t>(Ir) * (Ir + 1) / 2 > tile) --Ir;
  while (static_cast<int64_t>(Ir + 1) * (Ir + 2) / 2 <= tile) ++Ir;
  const int Jr = static_cast<int>(tile - static_cast<int64_t>(Ir) * (Ir + 1) / 2);
  const int I = T0 + Ir, J = T0 + Jr;
  const int r0 = I * kTB, c0 = J * kTB;
  const bool diag = (I == J);
  const int gr = r0 + r;

  // every global load is issued before the first use: the tile, the raw
  // column entries behind v_I and v_J, the norm partials
  double ld[kSyCols];
#pragma unroll
  for (int k = 0; k < kSyCols; ++k) {
    const int gc = c0 + q * kSyCols + k;
    const bool ok = gr < a.n && gc < a.n && gr > i && gc > i && (!diag || gr >= gc);
    ld[k] = ok ? a.A[gr + static_cast<int64_t>(gc) * a.lda] : 0.0;
  }
  const int gv = (t < 64) ? r0 + t : c0 + t - 64;
  const double xraw = (t < 128 && gv >= i + 2 && gv < a.n) ? a.A[gv + static_cast<int64_t>(i) * a.lda] : 0.0;
  const double alpha = a.A[(i + 1) + static_cast<int64_t>(i) * a.lda];
  const int nb0 = (i + 2 < a.n) ? (i + 2) / kTB : a.nT;   // row blocks holding x(2:)
  const double s0 = (nb0 + r < a.nT) ? a.nrm[nb0 + r] : 0.0;
  const double s1 = (nb0 + r + 64 < a.nT) ? a.nrm[nb0 + r + 64] : 0.0;

  double s = s0 + s1;
  for (int b = nb0 + r + 128; b < a.nT; b += 64) s += a.nrm[b];
  double beta, scal;
  const double tau = reflector(wave_sum(s), alpha, &beta, &scal);
  if (blockIdx.x == 0 && t == 0) {
    a.tau[i] = tau;
    a.E[i] = beta;
  }
  if (t < 128) {
    const double v = (gv == i + 1) ? 1.0 : xraw * scal;
    if (t < 64) vI[t] = v;
    else vJ[t - 64] = v;
  }
  __syncthreads();

  const double vr = vI[r];
  double acc = 0.0, p[kSyCols];
#pragma unroll
  for (int k = 0; k < kSyCols; ++k) {
    const int c = q * kSyCols + k;
    acc += ld[k] * vJ[c];
    p[k] = (!diag || r > c) ? ld[k] * vr : 0.0;
  }
  red[q][r] = acc;
  const double col = wave_sum16(p, r);
  const int cl = q * kSyCols + (r >> 2);
  if ((r & 3) == 0) {
    if (diag) cs[cl] = col;
    else a.P[(static_cast<int64_t>(J) * a.nT + I) * kTB + cl] = col;
  }
  __syncthreads();
  if (t < 64) {
    double y = wave_part_sum(red, t);
    if (diag) y += cs[t];
    a.P[(static_cast<int64_t>(I) * a.nT + J) * kTB + t] = y;
    const double sy = wave_sum(y * vI[t]);
    if (t == 0) a.S[tile] = diag ? sy : 2.0 * sy;
  }
  if (!diag) return;

  // diagonal tile: this row block's v into the panel, and its parts of
  // V^T v and W^T v over the panel's earlier columns (thread: column r,
  // rows 16q .. 16q+15)
  if (q == 0 && gr < a.n) a.Vp[static_cast<int64_t>(gr) * kNB + j] = vI[r];
  if (j == 0) return;
  // loaded only here (diagonal tiles), so that the tile's registers are free
  double sv = 0.0, sw = 0.0;
  if (r < j) {
    double pv[kSyCols], pw[kSyCols];
#pragma unroll
    for (int k = 0; k < kSyCols; ++k) {
      const int g = r0 + q * kSyCols + k;
      const bool ok = g > i && g < a.n;
      pv[k] = ok ? a.Vp[static_cast<int64_t>(g) * kNB + r] : 0.0;
      pw[k] = ok ? a.Wp[static_cast<int64_t>(g) * kNB + r] : 0.0;
    }
#pragma unroll
    for (int k = 0; k < kSyCols; ++k) {
      sv += pv[k] * vI[q * kSyCols + k];
      sw += pw[k] * vI[q * kSyCols + k];
    }
  }
  __syncthreads();
  red[q][r] = sv;
  red2[q][r] = sw;
  __syncthreads();
  if (t < 64 && t < j) {
    a.VV[static_cast<int64_t>(I) * kNB + t] = wave_part_sum(red, t);
    a.WV[static_cast<int64_t>(I) * kNB + t] = wave_part_sum(red2, t);
  }
}

// Column c's diagonal entry and squared-norm partials below its subdiagonal,
// one work-group per row block from c / 64 on (after a panel's rank-2k update).
__global__ __launch_bounds__(64) void td_start_kernel(TdArgs a, int c) {
  const int I = c / kTB + blockIdx.x;
  const int t = threadIdx.x;
  double s = 0.0;
  const int g = I * kTB + t;
  if (g < a.n) {
    const double x = a.A[g + static_cast<int64_t>(c) * a.lda];
    if (g == c) a.D[c] = x;
    if (g >= c + 2) s = x * x;
  }
  s = wave_sum(s);
  if (t == 0) a.nrm[I] = s;
}

constexpr int kUpOct = 8;                      // threads per row (octants of the sums)
constexpr int kUpThreads = 64 * kUpOct + 64;   // + one wave for row i+1
constexpr int kUpChunk = 8;                    // row blocks per octant per load batch

// One work-group per 64-row block of column i's trailing rows.  Waves 0-7 own
// the block's rows (lane = row, wave = octant of every sum); wave 8 repeats the
// arithmetic of row i+1, whose w every work-group needs for the next column.
// Phases: (1) all loads; (2) a = W^T v, b = V^T v and v^T A v from their
// partials; (3) w for the block's rows, the reflector stored in LAPACK form;
// (4) unless column i is the last of its panel, the next column corrected by
// the panel and its squared-norm partial for the next reflector.
__global__ __launch_bounds__(kUpThreads) void td_update_kernel(TdArgs a, int i, int j, int update_next,
                                                               int64_t ntiles) {
  __shared__ double sa[kNB], sb[kNB], W1[kNB + 1], V1[kNB + 1];
  __shared__ double red[kUpOct][kTB], redB[kUpOct][kTB];
  __shared__ double redx[kUpOct], sw[kTB], shs[kUpThreads / 64];
  __shared__ double sc[1];
  const int t = threadIdx.x, wv = t >> 6, lane = t & 63;
  const int T0 = (i + 1) / kTB;
  const int I = T0 + blockIdx.x;
  // waves 0-7: rows of block I, octant = wave; wave 8, lanes 0-7: row i+1
  const bool extra = (wv == kUpOct);
  const int o = extra ? (lane & (kUpOct - 1)) : wv;
  const int g = extra ? i + 1 : I * kTB + lane;
  const bool live = (extra ? (lane < kUpOct && update_next != 0) : true) && g > i && g < a.n;
  const double tau = a.tau[i];
  const double beta = a.E[i];

  // ---- loads: panel-product partials, v^T A v partials, this row's products
  // with every tile column, its panel row and its entry of the next column.
  // The first batch of every sum is loaded in one go (one memory round trip
  // for up to 64 row blocks and 4608 tiles); larger cases loop afterwards.
  const bool pan = !extra && lane < j;
  const int Ig = g / kTB, rg = g - Ig * kTB;
  double pa[kUpChunk], pb[kUpChunk], pp[kUpChunk], ps[8], vr[8], wr[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    const int c = o * 8 + k;
    const bool ok = live && c < j;
    vr[k] = ok ? a.Vp[static_cast<int64_t>(g) * kNB + c] : 0.0;
    wr[k] = ok ? a.Wp[static_cast<int64_t>(g) * kNB + c] : 0.0;
  }
  const double vg = live ? a.Vp[static_cast<int64_t>(g) * kNB + j] : 0.0;
  const double anext = (live && update_next && !extra) ? a.A[g + static_cast<int64_t>(i + 1) * a.lda] : 0.0;
#pragma unroll
  for (int m = 0; m < kUpChunk; ++m) {
    const int b = T0 + o + kUpOct * m;
    const bool ok = pan && b < a.nT;
    pa[m] = ok ? a.WV[static_cast<int64_t>(b) * kNB + lane] : 0.0;
    pb[m] = ok ? a.VV[static_cast<int64_t>(b) * kNB + lane] : 0.0;
    pp[m] = (live && b < a.nT) ? a.P[(static_cast<int64_t>(Ig) * a.nT + b) * kTB + rg] : 0.0;
  }
#pragma unroll
  for (int u = 0; u < 8; ++u) {
    const int64_t k = t + static_cast<int64_t>(kUpThreads) * u;
    ps[u] = k < ntiles ? a.S[k] : 0.0;
  }
  double xa = 0.0, xb = 0.0, y = 0.0, xs = 0.0;
#pragma unroll
  for (int m = 0; m < kUpChunk; ++m) {
    xa += pa[m];
    xb += pb[m];
    y += pp[m];
  }
#pragma unroll
  for (int u = 0; u < 8; ++u) xs += ps[u];
  for (int b0 = T0 + kUpOct * kUpChunk; b0 < a.nT; b0 += kUpOct * kUpChunk) {
#pragma unroll
    for (int m = 0; m < kUpChunk; ++m) {
      const int b = b0 + o + kUpOct * m;
      const bool ok = pan && b < a.nT;
      pa[m] = ok ? a.WV[static_cast<int64_t>(b) * kNB + lane] : 0.0;
      pb[m] = ok ? a.VV[static_cast<int64_t>(b) * kNB + lane] : 0.0;
      pp[m] = (live && b < a.nT) ? a.P[(static_cast<int64_t>(Ig) * a.nT + b) * kTB + rg] : 0.0;
    }
#pragma unroll
    for (int m = 0; m < kUpChunk; ++m) {
      xa += pa[m];
      xb += pb[m];
      y += pp[m];
    }
  }
  for (int64_t k0 = t + static_cast<int64_t>(kUpThreads) * 8; k0 < ntiles; k0 += static_cast<int64_t>(kUpThreads) * 8) {
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int64_t k = k0 + static_cast<int64_t>(kUpThreads) * u;
      ps[u] = k < ntiles ? a.S[k] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) xs += ps[u];
  }

  // ---- a = W^T v, b = V^T v, v^T A v: fixed-order reductions, finished by
  // wave 0 (which also forms a^T b) so that one barrier publishes them
  if (!extra) {
    red[wv][lane] = xa;
    redB[wv][lane] = xb;
  }
  xs = wave_sum(xs);
  if (lane == 0) shs[wv] = xs;
  __syncthreads();
  if (t < 64) {
    double u = 0.0, v = 0.0;
    if (t < j) {
#pragma unroll
      for (int q = 0; q < kUpOct; ++q) {
        u += red[q][t];
        v += redB[q][t];
      }
      sa[t] = u;
      sb[t] = v;
    }
    const double ab = wave_sum(u * v);
    double vav = 0.0;
#pragma unroll
    for (int q = 0; q < kUpThreads / 64; ++q) vav += shs[q];
    if (t == 0) sc[0] = -0.5 * tau * tau * (vav - 2.0 * ab);
  }
  __syncthreads();   // sa, sb, alpha2 ready; red/redB read
  // ---- w = tau (A v - V a - W b) + alpha2 v
  double z = y;
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    const int c = o * 8 + k;
    if (c < j) z -= vr[k] * sa[c] + wr[k] * sb[c];
  }
  const double alpha2 = sc[0];
  if (!extra) red[wv][lane] = live ? z : 0.0;
  else if (lane < kUpOct) redx[lane] = z;
  __syncthreads();
  // w of row i+1, the same expression in every work-group (its owner stores it too)
  double w1 = 0.0;
  if (update_next) {
    double zz = 0.0;
#pragma unroll
    for (int q = 0; q < kUpOct; ++q) zz += redx[q];
    w1 = tau * zz + alpha2;
  }
  if (t < 64) {
    double zz = 0.0;
#pragma unroll
    for (int q = 0; q < kUpOct; ++q) zz += red[q][t];
    double w = live ? tau * zz + alpha2 * vg : 0.0;
    if (update_next && g == i + 1) w = w1;
    sw[t] = w;
    if (g < a.n) {
      a.Wp[static_cast<int64_t>(g) * kNB + j] = w;
      if (g == i + 1) a.A[g + static_cast<int64_t>(i) * a.lda] = beta;
      else if (g > i + 1) a.A[g + static_cast<int64_t>(i) * a.lda] = vg;
    }
  }
  if (!update_next) return;

  // ---- next column: A(g, i+1) -= sum_{c <= j} V(g, c) W(i+1, c) + W(g, c) V(i+1, c)
  if (extra && lane < kUpOct) {
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const int c = o * 8 + k;
      if (c < j) {
        W1[c] = wr[k];
        V1[c] = vr[k];
      }
    }
    if (lane == 0) {
      W1[j] = w1;
      V1[j] = vg;
    }
  }
  __syncthreads();
  double u = 0.0;
  if (!extra && live) {
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const int c = o * 8 + k;
      if (c < j) u += vr[k] * W1[c] + wr[k] * V1[c];
    }
    if (o == kUpOct - 1) u += vg * W1[j] + sw[lane] * V1[j];
  }
  if (!extra) redB[wv][lane] = u;   // redB was last read before the previous barrier
  __syncthreads();
  if (t < 64) {
    double x2 = 0.0;
    if (live) {
      double upd = 0.0;
#pragma unroll
      for (int q = 0; q < kUpOct; ++q) upd += redB[q][t];
      const double x = anext - upd;
      a.A[g + static_cast<int64_t>(i + 1) * a.lda] = x;
      if (g == i + 1) a.D[i + 1] = x;
      if (g >= i + 3) x2 = x * x;
    }
    x2 = wave_sum(x2);
    if (t == 0) a.nrm[I] = x2;
  }
}

}  // namespace

size_t tridiag_scratch_bytes(int n) {
  if (n <= 0) return 0;
  const int64_t nT = ceil_div(n, kTB);
  const int64_t elems = 2 * static_cast<int64_t>(n) * kNB + nT * nT * kTB + nT * (nT + 1) / 2 +
                        2 * nT * kNB + nT + n + 64;
  return static_cast<size_t>(elems) * sizeof(double);
}

int tridiag_lower(double* A, int64_t lda, int n, double* D, double* E, double* tau, void* scratch,
                  hipStream_t st) {
  if (n <= 0) return CHEFSI_OK;
  TdArgs a{};
  a.A = A;
  a.lda = lda;
  a.n = n;
  a.nT = static_cast<int>(ceil_div(n, kTB));
  double* s = static_cast<double*>(scratch);
  const int64_t nT = a.nT;
  a.Vp = s;
  s += static_cast<int64_t>(n) * kNB;
  a.Wp = s;
  s += static_cast<int64_t>(n) * kNB;
  a.P = s;
  s += nT * nT * kTB;
  a.S = s;
  s += nT * (nT + 1) / 2;
  a.VV = s;
  s += nT * kNB;
  a.WV = s;
  s += nT * kNB;
  a.nrm = s;
  a.D = D;
  a.E = E;
  a.tau = tau;

  td_start_kernel<<<static_cast<unsigned>(a.nT), 64, 0, st>>>(a, 0);
  CHEFSI_LAUNCHED("td_start");
  for (int p0 = 0; p0 < n - 1;) {
    const int p1 = (p0 + kNB < n - 1) ? p0 + kNB : n - 1;
    for (int i = p0; i < p1; ++i) {
      const int k = a.nT - (i + 1) / kTB;
      const int64_t ntiles = static_cast<int64_t>(k) * (k + 1) / 2;
      td_symv_kernel<<<static_cast<unsigned>(ntiles), kTdThreads, 0, st>>>(a, i, i - p0);
      CHEFSI_LAUNCHED("td_symv");
      td_update_kernel<<<static_cast<unsigned>(k), kUpThreads, 0, st>>>(a, i, i - p0, i + 1 < p1 ? 1 : 0,
                                                                         ntiles);
      CHEFSI_LAUNCHED("td_update");
    }
    const int n2 = n - p1;
    // A22 -= V W^T + W V^T on the lower triangle of the trailing block: in
    // the row-major view (A^T, row stride lda) that is the upper triangle
    // updated with W V^T + V W^T
    CHEFSI_TRY(syr2k_upper(n2, p1 - p0, -1.0, a.Wp + static_cast<int64_t>(p1) * kNB, a.Vp + static_cast<int64_t>(p1) * kNB,
                           a.Vp + static_cast<int64_t>(p1) * kNB, a.Wp + static_cast<int64_t>(p1) * kNB, kNB,
                           A + p1 + static_cast<int64_t>(p1) * lda, lda, st));
    td_start_kernel<<<static_cast<unsigned>(a.nT - p1 / kTB), 64, 0, st>>>(a, p1);
    CHEFSI_LAUNCHED("td_start");
    p0 = p1;
  }
  return CHEFSI_OK;
}

}  // namespace chefsi
