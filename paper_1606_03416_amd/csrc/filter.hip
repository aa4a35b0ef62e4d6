// Chebyshev filter hot path for gfx950: block-sparse H^DG x multivector with
// the three-term recurrence fused into the epilogue.
//
// One work-group computes the rows of one element K for a tile of columns.
// Its reduction runs over the concatenation of the stencil neighbours' rows
// (eq. matvec_3: y_K = sum_{K' in N(K)} H_{K;K'} x_{K'}): the packed panel of
// H (written once per call by the repack kernel) against the gathered
// neighbour rows of the input block, on MFMA.  The recurrence
// Y_{k+1} = alpha_k (H Y_k - c Y_k) - beta_k Y_{k-1} is applied in the
// epilogue, so a step reads Y_k, Y_{k-1} and writes Y_{k+1} once.  FP64 and
// FP32 stage both operands through LDS; BF16 keeps its multivectors in 8-row
// tiles and loads MFMA operands directly.  The split-BF16 variant (BF16X3)
// stores every value as a pair of bf16 numbers hi + lo (hi = bf16(v),
// lo = bf16(v - hi): about 16 significant bits) in two arrays of that layout,
// H - cI likewise, and forms each product from three BF16 MFMAs,
// A_hi B_hi + A_hi B_lo + A_lo B_hi, accumulated in FP32 (the A_lo B_lo term is
// below the pair's own rounding).  Elements are launched in classes of equal
// row-block count (ceil(J_K/16)), one launch per class.
#include <type_traits>

#include "common.h"

namespace chefsi {

namespace {

constexpr int NT = 256;

struct StepArgs {
  const void* panel;
  const int64_t* poff;
  const int32_t* kpad;
  const int64_t* koff;
  const int32_t* kmap;
  const int32_t* J;
  const int32_t* rbv;
  const int64_t* rowoff;
  const int32_t* order;
  const double* coef;
  const void* in;
  int64_t ldi;
  const void* prev;
  int64_t ldp;
  void* out;
  int64_t ldo;
  const double* theta;
  double* part;
  int ns;
  int M;
};

// Work-group id -> linear work index, so that the work-groups one XCD runs
// (hardware id b goes to XCD b % 8) are consecutive work items.
__device__ __forceinline__ int xcd_linear(int b, int nwg) {
  const int q = nwg >> 3, r = nwg & 7;
  const int x = b & 7, i = b >> 3;
  return x * q + (x < r ? x : r) + i;
}

// Streamed data of the step kernels (the previous block, the output) carries
// the non-temporal hint, so that the L2 keeps the gathered neighbour rows,
// which several work-groups read.  (The same hint on the panels, which the
// work-groups of an element share, costs time.)
#ifndef CHEFSI_NT_STREAM
#define CHEFSI_NT_STREAM 1
#endif
template <typename T>
__device__ __forceinline__ T ld_stream(const T* p) {
  if constexpr (CHEFSI_NT_STREAM != 0) return __builtin_nontemporal_load(p);
  else return *p;
}
template <typename T>
__device__ __forceinline__ void st_stream(T* p, T v) {
  if constexpr (CHEFSI_NT_STREAM != 0) __builtin_nontemporal_store(v, p);
  else *p = v;
}
typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ uint2 ld_stream(const uint2* p) {
  const u32x2 v = ld_stream(reinterpret_cast<const u32x2*>(p));
  return make_uint2(v.x, v.y);
}
__device__ __forceinline__ void st_stream(uint2* p, uint2 v) {
  u32x2 w;
  w.x = v.x;
  w.y = v.y;
  st_stream(reinterpret_cast<u32x2*>(p), w);
}

// float <-> bf16 (round to nearest even; NaN stays NaN)
__device__ __forceinline__ uint16_t f2bf(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7fffffffu) > 0x7f800000u) return static_cast<uint16_t>(0x7fc0u);
  u += 0x7fffu + ((u >> 16) & 1u);
  return static_cast<uint16_t>(u >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float(static_cast<uint32_t>(h) << 16); }


// ---------------------------------------------------------------- BF16 path
// BF16 storage and MFMA operands (v_mfma_f32_16x16x32_bf16), FP32
// accumulation and epilogue.  Lane l supplies A[l%16][8(l/16)..+7] and
// B[8(l/16)..+7][l%16] and receives D[4(l/16)+q][l%16], q = 0..3.
//
// The recurrence is kept in 8-row tiles: rows padded per element to multiples
// of 8, and tile G stores its 8 rows state by state, element (G, j, e) at
// (G*ns + j)*8 + e.  Each element's panel is stored in 32-row chunks [JP][32],
// with -c folded into the diagonal of the self block, so the step is
// out = alpha*acc - beta*prev.  Both MFMA operands are single 16-byte loads
// straight from memory (a lane's eight reduction rows of one neighbour are
// contiguous, and 16 consecutive states are 256 contiguous bytes).  No LDS
// staging and no barriers in the main loop; each wave computes all of the
// element's rows for 16*BNC columns, and the four waves of a work-group share
// the element's panel through L1.
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
#ifndef CHEFSI_B16_NC
#define CHEFSI_B16_NC 4
#endif
#ifndef CHEFSI_B16_WAVES
#define CHEFSI_B16_WAVES 4
#endif
constexpr int BNT = 64 * CHEFSI_B16_WAVES;  // threads per work-group
// 16-column fragments per wave: CHEFSI_B16_NC (split: CHEFSI_B16X3_NC) for
// elements of <= 64 rows, 2 up to 128 rows and 1 above (register budget)
#ifndef CHEFSI_B16X3_NC
#define CHEFSI_B16X3_NC 4
#endif
template <int RB, bool X3 = false>
constexpr int b16_nc() {
  return X3 ? (RB <= 4 ? CHEFSI_B16X3_NC : (RB <= 8 ? 2 : 1)) : (RB <= 4 ? CHEFSI_B16_NC : (RB <= 8 ? 2 : 1));
}

struct StepArgsB {
  const uint16_t* panel;
  const int64_t* poff8;
  const int32_t* kpad8;
  const int64_t* kgoff;
  const int32_t* kg8;    // 8-row tile index of each reduction-row group (-1 pad)
  const int32_t* J;
  const int32_t* rbv;
  const int64_t* rowoff8;
  const int64_t* rowoff;
  const int32_t* order;
  const double* coef;
  const uint16_t* in;
  const uint16_t* prev;
  void* out;
  int64_t ldo;   // row stride of a float64 row-major output
  int ns;
  int M;
  int64_t panel_lo;   // split BF16: offset of the lo panel from panel (elements)
  int64_t mv_lo;      // split BF16: offset of the lo array from each multivector (elements)
};

// Row blocks [rb0, rb0 + RB) of element K (nrb row blocks in all; blocks at
// or beyond nrb are computed from a repeated valid block and not stored) for
// one tile of columns.  sG holds the element's gathered tile indices.
template <bool F64OUT, int RB, bool X3, int BNC>
__device__ __forceinline__ void step_body_b16(const StepArgsB& a, int K, int ct, const int32_t* sG, int nrb,
                                              int rb0) {
  constexpr int BTN = CHEFSI_B16_WAVES * 16 * BNC;
  const int JP = nrb * 16;   // panel rows of the element (chunk stride / 32)
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int q = lane >> 4, l16 = lane & 15;
  const int ngrp = a.kpad8[K] >> 3;
  const int nch = ngrp >> 2;
  const int ns = a.ns;
  const int jb = ct * BTN + wave * (16 * BNC) + l16;
  const uint16_t* pa = a.panel + a.poff8[K] + l16 * 32 + 8 * q;
  int rofs[RB];   // offset of row block rb0 + r in a chunk (a valid block for every r)
#pragma unroll
  for (int r = 0; r < RB; ++r) rofs[r] = min(rb0 + r, nrb - 1) * (16 * 32);
  const uint16_t* pb[BNC];
  bool vb[BNC];
#pragma unroll
  for (int n = 0; n < BNC; ++n) {
    const int j = jb + 16 * n;
    vb[n] = j < ns;
    pb[n] = a.in + static_cast<int64_t>(vb[n] ? j : 0) * 8;
  }
  const int64_t tstride = static_cast<int64_t>(ns) * 8;   // elements per 8-row tile
  f32x4 acc[RB][BNC];
#pragma unroll
  for (int r = 0; r < RB; ++r)
#pragma unroll
    for (int n = 0; n < BNC; ++n) acc[r][n] = f32x4{0.f, 0.f, 0.f, 0.f};

  // operand slots: [0, RB) hi panel, [RB, 2RB) lo panel (split only); the
  // same for the gathered rows with BNC
  constexpr int NA = X3 ? 2 * RB : RB, NB = X3 ? 2 * BNC : BNC;
  auto load = [&](int c, bf16x8* A, bf16x8* B) {
    const uint16_t* p = pa + static_cast<int64_t>(c) * (JP * 32);
#pragma unroll
    for (int r = 0; r < RB; ++r) A[r] = *reinterpret_cast<const bf16x8*>(p + rofs[r]);
    if constexpr (X3) {
#pragma unroll
      for (int r = 0; r < RB; ++r) A[RB + r] = *reinterpret_cast<const bf16x8*>(p + a.panel_lo + rofs[r]);
    }
    const int G = sG[c * 4 + q];
    const int64_t go = static_cast<int64_t>(G) * tstride;
#pragma unroll
    for (int n = 0; n < BNC; ++n) {
      bf16x8 v = {}, w = {};
      if (vb[n] && G >= 0) {
        v = *reinterpret_cast<const bf16x8*>(pb[n] + go);
        if constexpr (X3) w = *reinterpret_cast<const bf16x8*>(pb[n] + a.mv_lo + go);
      }
      B[n] = v;
      if constexpr (X3) B[BNC + n] = w;
    }
  };
  auto mma = [&](const bf16x8* A, const bf16x8* B) {
#pragma unroll
    for (int r = 0; r < RB; ++r)
#pragma unroll
      for (int n = 0; n < BNC; ++n) {
        if constexpr (X3) {
          acc[r][n] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A[RB + r], B[n], acc[r][n], 0, 0, 0);
          acc[r][n] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A[r], B[BNC + n], acc[r][n], 0, 0, 0);
        }
        acc[r][n] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A[r], B[n], acc[r][n], 0, 0, 0);
      }
  };
  bf16x8 A0[NA], B0[NB], A1[NA], B1[NB];
  load(0, A0, B0);
  int c = 0;
  for (; c + 2 <= nch; c += 2) {
    load(c + 1, A1, B1);
    mma(A0, B0);
    if (c + 2 < nch) load(c + 2, A0, B0);
    mma(A1, B1);
  }
  if (c < nch) mma(A0, B0);

  const int JK = a.J[K];
  const int J8 = round_up(JK, 8);
  const int64_t g8 = a.rowoff8[K];
  const float alpha = static_cast<float>(a.coef[0]);
  const float beta = static_cast<float>(a.coef[1]);
#pragma unroll
  for (int n = 0; n < BNC; ++n) {
    const int j = jb + 16 * n;
    if (!vb[n]) continue;
#pragma unroll
    for (int r = 0; r < RB; ++r) {
      const int i0 = (rb0 + r) * 16 + 4 * q;
      if (rb0 + r >= nrb || i0 >= J8) continue;
      const int64_t row = g8 + i0;   // multiple of 4: the 4 rows share one tile
      const int64_t o = (row >> 3) * tstride + static_cast<int64_t>(j) * 8 + (row & 7);
      uint2 xp = make_uint2(0, 0), xl = make_uint2(0, 0);
      if (a.prev != nullptr) {
        xp = ld_stream(reinterpret_cast<const uint2*>(a.prev + o));
        if constexpr (X3) xl = ld_stream(reinterpret_cast<const uint2*>(a.prev + a.mv_lo + o));
      }
      const uint32_t wp[2] = {xp.x, xp.y}, wl[2] = {xl.x, xl.y};
      float v[4];
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        float y = bf2f(static_cast<uint16_t>(wp[e >> 1] >> (16 * (e & 1))));
        if constexpr (X3) y += bf2f(static_cast<uint16_t>(wl[e >> 1] >> (16 * (e & 1))));
        v[e] = (i0 + e < JK) ? alpha * acc[r][n][e] - beta * y : 0.f;
      }
      if constexpr (F64OUT) {
        double* out = static_cast<double*>(a.out);
        const int64_t g0 = a.rowoff[K];
#pragma unroll
        for (int e = 0; e < 4; ++e)
          if (i0 + e < JK) out[(g0 + i0 + e) * a.ldo + j] = static_cast<double>(v[e]);
      } else {
        uint16_t* out = static_cast<uint16_t*>(a.out);
        uint16_t h[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) h[e] = f2bf(v[e]);
        st_stream(reinterpret_cast<uint2*>(out + o),
                  make_uint2(h[0] | (static_cast<uint32_t>(h[1]) << 16), h[2] | (static_cast<uint32_t>(h[3]) << 16)));
        if constexpr (X3) {
          uint16_t l[4];
#pragma unroll
          for (int e = 0; e < 4; ++e) l[e] = f2bf(v[e] - bf2f(h[e]));
          st_stream(reinterpret_cast<uint2*>(out + a.mv_lo + o),
                    make_uint2(l[0] | (static_cast<uint32_t>(l[1]) << 16), l[2] | (static_cast<uint32_t>(l[3]) << 16)));
        }
      }
    }
  }
}

#ifndef CHEFSI_B16_WPE
#define CHEFSI_B16_WPE 3
#endif
// RB row blocks per element; above 8 the rows are computed in two passes of
// RBS = ceil(RB / 2) blocks over the same gathered tiles (register budget).
template <int RB>
constexpr int b16_rbs() { return RB <= 8 ? RB : (RB + 1) / 2; }

template <bool F64OUT, int RB, bool X3>
__global__ __launch_bounds__(BNT) __attribute__((amdgpu_waves_per_eu(RB <= 4 && !X3 ? CHEFSI_B16_WPE : 2))) void step_kernel_b16(StepArgsB a) {
  __shared__ int32_t sG[7 * kMaxJ / 8];
  static_assert(RB * 16 <= kMaxJ, "row blocks beyond the largest ALB count");
  constexpr int RBS = b16_rbs<RB>();
  constexpr int BNC = b16_nc<RB, X3>();
  const int id = xcd_linear(blockIdx.x, gridDim.x);
#ifndef CHEFSI_B16_CG
#define CHEFSI_B16_CG 1
#endif
#ifndef CHEFSI_B16_CG8
#define CHEFSI_B16_CG8 8
#endif
  // groups of CG column tiles of one element run together (its panel is
  // reused from L2), the groups column-major; elements of more than 64 rows
  // have narrower column tiles and larger panels, so more tiles share one
  constexpr int CG = RB <= 4 ? CHEFSI_B16_CG : CHEFSI_B16_CG8;
  const int nct = (a.ns + CHEFSI_B16_WAVES * 16 * BNC - 1) / (CHEFSI_B16_WAVES * 16 * BNC);
  const int g = id / (a.M * CG);
  const int rem = id - g * (a.M * CG);
  const int cg = (CG * g + CG <= nct) ? CG : nct - CG * g;
  const int e = rem / cg;
  const int ct = CG * g + (rem - e * cg);
  const int K = a.order[e];
  {
    const int ngrp = a.kpad8[K] >> 3;
    const int32_t* kg = a.kg8 + a.kgoff[K];
    for (int t = threadIdx.x; t < ngrp; t += BNT) sG[t] = kg[t];
  }
  __syncthreads();
  for (int rb0 = 0; rb0 < RB; rb0 += RBS) step_body_b16<F64OUT, RBS, X3, BNC>(a, K, ct, sG, RB, rb0);
}

template <bool F64OUT, int RB, bool X3>
void launch_b16(const StepArgsB& a, int ns, hipStream_t st) {
  const int btn = CHEFSI_B16_WAVES * 16 * b16_nc<RB, X3>();
  dim3 grid(static_cast<unsigned>(ceil_div(ns, btn) * a.M));
  step_kernel_b16<F64OUT, RB, X3><<<grid, BNT, 0, st>>>(a);
}

template <bool F64OUT, bool X3>
void dispatch_step_b16(const Plan& p, StepArgsB a, int ns, hipStream_t st) {
  // one launch per row-block class of elements
  for (size_t gi = 0; gi < p.grp_rb.size(); ++gi) {
    a.order = p.d_order + p.grp_start[gi];
    a.M = p.grp_count[gi];
    switch (p.grp_rb[gi]) {
      case 1: launch_b16<F64OUT, 1, X3>(a, ns, st); break;
      case 2: launch_b16<F64OUT, 2, X3>(a, ns, st); break;
      case 3: launch_b16<F64OUT, 3, X3>(a, ns, st); break;
      case 4: launch_b16<F64OUT, 4, X3>(a, ns, st); break;
      case 5: launch_b16<F64OUT, 5, X3>(a, ns, st); break;
      case 6: launch_b16<F64OUT, 6, X3>(a, ns, st); break;
      case 7: launch_b16<F64OUT, 7, X3>(a, ns, st); break;
      case 8: launch_b16<F64OUT, 8, X3>(a, ns, st); break;
      case 9: launch_b16<F64OUT, 9, X3>(a, ns, st); break;
      case 10: launch_b16<F64OUT, 10, X3>(a, ns, st); break;
      case 11: launch_b16<F64OUT, 11, X3>(a, ns, st); break;
      case 12: launch_b16<F64OUT, 12, X3>(a, ns, st); break;
      case 13: launch_b16<F64OUT, 13, X3>(a, ns, st); break;
      case 14: launch_b16<F64OUT, 14, X3>(a, ns, st); break;
      case 15: launch_b16<F64OUT, 15, X3>(a, ns, st); break;
      default: launch_b16<F64OUT, 16, X3>(a, ns, st); break;
    }
  }
}

// X (float64 row-major) -> bf16 8-row tiles with zero padding rows, through a
// 64 x 64 LDS tile: reads along a row; each thread then writes the 8 rows of
// one (tile, state) pair as 16 contiguous bytes.
__global__ __launch_bounds__(256) void to_tiles_b16_kernel(const double* X, int64_t ldx, const int32_t* rowsrc8,
                                                           int64_t N8, int ns, uint16_t* out, uint16_t* out_lo) {
  __shared__ float tile[64][65];
  const int64_t r0 = static_cast<int64_t>(blockIdx.x) * 64;
  const int c0 = blockIdx.y * 64;
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  for (int rr = ty; rr < 64; rr += 4) {
    const int64_t r = r0 + rr;
    const int c = c0 + tx;
    float v = 0.f;
    if (r < N8 && c < ns) {
      const int32_t src = rowsrc8[r];
      if (src >= 0) v = static_cast<float>(X[static_cast<int64_t>(src) * ldx + c]);
    }
    tile[rr][tx] = v;
  }
  __syncthreads();
  // 8 row tiles x 64 states per block; thread t covers (tile t/64 and t/64+4, state t%64)
  for (int gg = ty; gg < 8; gg += 4) {
    const int c = c0 + tx;
    const int64_t G = (r0 >> 3) + gg;
    if (c < ns && G * 8 < N8) {
      uint32_t w[4], wl[4];
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const float x0 = tile[gg * 8 + 2 * e][tx], x1 = tile[gg * 8 + 2 * e + 1][tx];
        const uint16_t h0 = f2bf(x0), h1 = f2bf(x1);
        w[e] = h0 | (static_cast<uint32_t>(h1) << 16);
        wl[e] = f2bf(x0 - bf2f(h0)) | (static_cast<uint32_t>(f2bf(x1 - bf2f(h1))) << 16);
      }
      *reinterpret_cast<uint4*>(out + (G * ns + c) * 8) = make_uint4(w[0], w[1], w[2], w[3]);
      if (out_lo != nullptr)
        *reinterpret_cast<uint4*>(out_lo + (G * ns + c) * 8) = make_uint4(wl[0], wl[1], wl[2], wl[3]);
    }
  }
}

// ------------------------------------------------------- FP64 / FP32 paths
// v_mfma_f64_16x16x4f64 / v_mfma_f32_16x16x4f32: lane l supplies A[l%16][l/16]
// and B[l/16][l%16]; output v of lane l is D[4v + l/16][l%16] (FP64) or
// D[4(l/16) + v][l%16] (FP32).  A work-group takes one element and 64*NCF
// columns; wave w owns columns 16*NCF*w .. +16*NCF and all of the element's
// rows, as RB x NCF sixteen-square fragments.  Operands are staged through LDS
// in chunks of KC reduction rows with 16-byte loads; the k-major LDS rows are
// padded so that the k rows one wave reads fall on disjoint banks.  The last
// reduction step of a chunk runs after the barrier, behind the LDS reads of
// the next chunk's first step.
#ifndef CHEFSI_MF_KC64
#define CHEFSI_MF_KC64 8
#endif
#ifndef CHEFSI_MF_KC32
#define CHEFSI_MF_KC32 16
#endif
#ifndef CHEFSI_MF_EARLY
#define CHEFSI_MF_EARLY 1
#endif
#ifndef CHEFSI_MF_KC_RB
#define CHEFSI_MF_KC_RB 16
#endif
template <typename TC>
struct MT;

template <>
struct MT<double> {
  typedef double2 V;                     // one 16-byte load
  static constexpr int W = 2;            // elements per load
  // reduction rows per LDS chunk (elements of more than CHEFSI_MF_KC_RB row
  // blocks: 8, so that a thread stages at most four panel pieces)
  static constexpr int kc(int rb) { return rb <= CHEFSI_MF_KC_RB ? CHEFSI_MF_KC64 : 8; }
  typedef double acc_t __attribute__((ext_vector_type(4)));
  static __device__ __forceinline__ acc_t mma(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int lane, int v) { return 4 * v + (lane >> 4); }
  // row strides: 2*ld = 32 (mod 64) banks
  static constexpr int lda(int rb) { return rb * 16 + ((rb & 1) ? 0 : 16); }
  static constexpr int ldb(int tn) { return tn + 16; }
  static __device__ __forceinline__ V zero() { return make_double2(0.0, 0.0); }
  static __device__ __forceinline__ void set(V& x, int e, double v) { (e == 0 ? x.x : x.y) = v; }
};

template <>
struct MT<float> {
  typedef float4 V;
  static constexpr int W = 4;
  static constexpr int kc(int rb) { return rb <= CHEFSI_MF_KC_RB ? CHEFSI_MF_KC32 : 16; }
  typedef float acc_t __attribute__((ext_vector_type(4)));
  static __device__ __forceinline__ acc_t mma(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int lane, int v) { return 4 * (lane >> 4) + v; }
  // row strides: ld = 16 (mod 64) banks
  static constexpr int lda(int rb) { return rb * 16 + (((16 - rb * 16) % 64) + 64) % 64; }
  static constexpr int ldb(int tn) { return tn + 16; }
  static __device__ __forceinline__ V zero() { return make_float4(0.f, 0.f, 0.f, 0.f); }
  static __device__ __forceinline__ void set(V& x, int e, float v) {
    (e == 0 ? x.x : e == 1 ? x.y : e == 2 ? x.z : x.w) = v;
  }
};

// Epilogue shared by the FP64 / FP32 step kernels.  acc holds the wave's
// RB x NCF sixteen-square fragments of element K; the wave's columns start at
// jb.  EPI 0: Y_out = alpha (acc - c Y_in) - beta Y_prev; EPI 2: the panel
// already carries H - cI, Y_out = alpha acc - beta Y_prev; EPI 1: per-column
// partial sums of the squared residual rows.
template <typename TC, typename TOUT, int EPI, int RB, int NCF>
__device__ __forceinline__ void step_epilogue(const StepArgs& a, int K, int jb,
                                              const typename MT<TC>::acc_t (&acc)[RB][NCF]) {
  using T = MT<TC>;
  const int lane = threadIdx.x & 63;
  const int ns = a.ns;
  const TC* in = static_cast<const TC*>(a.in);
  const int64_t ldi = a.ldi;
  const int JK = a.J[K];
  const int64_t g0 = a.rowoff[K];
  // every load goes to a clamped, valid address and only the stores are
  // predicated, so that the loads of a row block issue together instead of
  // one branch (and one wait) per value
  int jc[NCF];
  bool jok[NCF];
#pragma unroll
  for (int q = 0; q < NCF; ++q) {
    const int j = jb + 16 * q + (lane & 15);
    jok[q] = j < ns;
    jc[q] = jok[q] ? j : ns - 1;
  }
  if constexpr (EPI == 0 || EPI == 2) {
    // EPI 2: the panel carries H - cI
    const TC alpha = static_cast<TC>(a.coef[0]), beta = static_cast<TC>(a.coef[1]);
    const TC cc = static_cast<TC>(a.coef[2]);
    const TC* prev = static_cast<const TC*>(a.prev);
    TOUT* out = static_cast<TOUT*>(a.out);
#pragma unroll
    for (int r = 0; r < RB; ++r) {
      TC pv[4][NCF], iv[4][NCF];
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t g = g0 + min(16 * r + T::row(lane, v), JK - 1);
#pragma unroll
        for (int q = 0; q < NCF; ++q) {
          pv[v][q] = (prev != nullptr) ? ld_stream(prev + g * a.ldp + jc[q]) : TC(0);
          if constexpr (EPI == 0) iv[v][q] = in[g * ldi + jc[q]];
        }
      }
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int i = 16 * r + T::row(lane, v);
        const int64_t g = g0 + i;
#pragma unroll
        for (int q = 0; q < NCF; ++q) {
          TC y = (EPI == 2) ? alpha * acc[r][q][v] : alpha * (acc[r][q][v] - cc * iv[v][q]);
          y -= beta * pv[v][q];
          if (i < JK && jok[q]) st_stream(out + g * a.ldo + jc[q], static_cast<TOUT>(y));
        }
      }
    }
  } else {
    // residual partial sums over the element's rows: sum_i (H x - theta x)_i^2;
    // each wave owns whole columns, so the sum needs no cross-wave step
    static_assert(std::is_same<TC, double>::value, "residual epilogue is FP64");
    double sum[NCF];
#pragma unroll
    for (int q = 0; q < NCF; ++q) sum[q] = 0.0;
#pragma unroll
    for (int r = 0; r < RB; ++r) {
      double iv[4][NCF];
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t g = g0 + min(16 * r + T::row(lane, v), JK - 1);
#pragma unroll
        for (int q = 0; q < NCF; ++q) iv[v][q] = in[g * ldi + jc[q]];
      }
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int i = 16 * r + T::row(lane, v);
#pragma unroll
        for (int q = 0; q < NCF; ++q) {
          const double th = a.theta[jc[q]];
          const double d = acc[r][q][v] - th * iv[v][q];
          if (i < JK) sum[q] += d * d;
        }
      }
    }
#pragma unroll
    for (int q = 0; q < NCF; ++q) {
      double t = sum[q];
      t += __shfl_xor(t, 16);
      t += __shfl_xor(t, 32);
      if (lane < 16 && jok[q]) a.part[static_cast<int64_t>(K) * ns + jc[q]] = t;
    }
  }
}

template <typename TC, typename TOUT, int EPI, int RB, int NCF, int NW>
__device__ __forceinline__ void step_body_mf(const StepArgs& a, int K, int ct, TC* sA, TC* sB, int32_t* sK) {
  using T = MT<TC>;
  using V = typename T::V;
  constexpr int NT = 64 * NW;                        // threads of the work-group
  constexpr int KC2 = T::kc(RB), W = T::W;
  constexpr int JP = RB * 16;
  constexpr int LDA = T::lda(RB);
  constexpr int TNF = 16 * NW * NCF;                 // columns of the work-group
  constexpr int LDB = T::ldb(TNF);
  constexpr int ASZ = KC2 * LDA, BSZ = KC2 * LDB;
  constexpr int APC = KC2 * JP / W;                  // 16-byte pieces of a panel chunk
  constexpr int AV = (APC + NT - 1) / NT;
  constexpr int BROWS = NT * W / TNF;                // gathered rows per load round
  constexpr int BV = KC2 / BROWS;
  constexpr int S = KC2 / 4;                         // reduction steps per chunk
  static_assert(AV >= 1 && AV <= 4 && BV >= 1 && S % 2 == 0, "chunk shape");
  static_assert(kStepKC % KC2 == 0, "element reduction rows are padded to whole chunks");
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int ns = a.ns;
  {
    const int32_t* km = a.kmap + a.koff[K];
    const int kp = a.kpad[K];
    for (int t = tid; t < kp; t += NT) sK[t] = km[t];
  }
  const TC* panel = static_cast<const TC*>(a.panel) + a.poff[K];
  const TC* in = static_cast<const TC*>(a.in);
  const int64_t ldi = a.ldi;
  const int j0 = ct * TNF;
  const int nch = a.kpad[K] / KC2;
  const bool vec = (ldi % W) == 0 && (reinterpret_cast<uintptr_t>(in) & 15u) == 0;
  const int bcp = tid % (TNF / W);
  const int brow = tid / (TNF / W);
  const int bcol = j0 + W * bcp;
  __syncthreads();

  // panel chunk: this thread's pieces tid + v NT, v < AV (clamped to a valid
  // address where the chunk has fewer pieces); named registers, not an array,
  // so that they never go to scratch memory
  V ra0, ra1, ra2, ra3, rb[BV];
  auto gload = [&](int c) {
    const TC* pa = panel + static_cast<int64_t>(c) * (KC2 * JP);
    ra0 = *reinterpret_cast<const V*>(pa + W * min(tid, APC - 1));
    if constexpr (AV > 1) ra1 = *reinterpret_cast<const V*>(pa + W * min(tid + NT, APC - 1));
    if constexpr (AV > 2) ra2 = *reinterpret_cast<const V*>(pa + W * min(tid + 2 * NT, APC - 1));
    if constexpr (AV > 3) ra3 = *reinterpret_cast<const V*>(pa + W * min(tid + 3 * NT, APC - 1));
#pragma unroll
    for (int v = 0; v < BV; ++v) {
      const int g = sK[c * KC2 + v * BROWS + brow];
      V x = T::zero();
      if (g >= 0) {
        const TC* src = in + static_cast<int64_t>(g) * ldi + bcol;
        if (vec && bcol + W - 1 < ns) {
          x = *reinterpret_cast<const V*>(src);
        } else {
#pragma unroll
          for (int e = 0; e < W; ++e)
            if (bcol + e < ns) T::set(x, e, src[e]);
        }
      }
      rb[v] = x;
    }
  };
  auto sstore = [&](TC* A, TC* B) {
    auto put = [&](int i1, const V& x) {
      if (i1 < APC) *reinterpret_cast<V*>(A + ((W * i1) / JP) * LDA + (W * i1) % JP) = x;
    };
    put(tid, ra0);
    if constexpr (AV > 1) put(tid + NT, ra1);
    if constexpr (AV > 2) put(tid + 2 * NT, ra2);
    if constexpr (AV > 3) put(tid + 3 * NT, ra3);
#pragma unroll
    for (int v = 0; v < BV; ++v) *reinterpret_cast<V*>(B + (v * BROWS + brow) * LDB + W * bcp) = rb[v];
  };

  using acc_t = typename T::acc_t;
  acc_t acc[RB][NCF];
#pragma unroll
  for (int r = 0; r < RB; ++r)
#pragma unroll
    for (int q = 0; q < NCF; ++q) acc[r][q] = acc_t{};
  const int cb = wave * (16 * NCF);
  TC fa[2][RB], fb[2][NCF];
  auto rd = [&](const TC* A, const TC* B, int kk, int slot) {
    const int kr = 4 * kk + (lane >> 4);
#pragma unroll
    for (int r = 0; r < RB; ++r) fa[slot][r] = A[kr * LDA + 16 * r + (lane & 15)];
#pragma unroll
    for (int q = 0; q < NCF; ++q) fb[slot][q] = B[kr * LDB + cb + 16 * q + (lane & 15)];
  };
  auto mm = [&](int slot) {
#pragma unroll
    for (int r = 0; r < RB; ++r)
#pragma unroll
      for (int q = 0; q < NCF; ++q) acc[r][q] = T::mma(fa[slot][r], fb[slot][q], acc[r][q]);
  };
  // The staging registers take chunk c + 2 as soon as chunk c + 1 has gone
  // to LDS, so a chunk's loads have a whole chunk of MFMA work to arrive in.
  gload(0);
  sstore(sA, sB);
#if CHEFSI_MF_EARLY
  if (nch > 1) gload(1);
#endif
  __syncthreads();
  if (nch > 0) rd(sA, sB, 0, 0);
  for (int c = 0; c < nch; ++c) {
    const int buf = c & 1;
#if !CHEFSI_MF_EARLY
    if (c + 1 < nch) gload(c + 1);
#endif
#pragma unroll
    for (int kk = 1; kk < S; ++kk) {
      rd(sA + buf * ASZ, sB + buf * BSZ, kk, kk & 1);
      mm((kk - 1) & 1);
    }
    if (c + 1 < nch) sstore(sA + (buf ^ 1) * ASZ, sB + (buf ^ 1) * BSZ);
#if CHEFSI_MF_EARLY
    if (c + 2 < nch) gload(c + 2);
#endif
    __syncthreads();
    if (c + 1 < nch) rd(sA + (buf ^ 1) * ASZ, sB + (buf ^ 1) * BSZ, 0, 0);
    mm((S - 1) & 1);
  }

  step_epilogue<TC, TOUT, EPI, RB, NCF>(a, K, j0 + cb, acc);
}

// Work-group id -> (element slot e, column tile ct): groups of CG column tiles
// of one element run together (its panel is reused from L2), the groups
// column-major.
#ifndef CHEFSI_MF_CG
#define CHEFSI_MF_CG 2
#endif
#ifndef CHEFSI_MF_CG8
#define CHEFSI_MF_CG8 8
#endif
template <int CG>
__device__ __forceinline__ void step_tile(int id, int M, int nct, int& e, int& ct) {
  const int g = id / (M * CG);
  const int rem = id - g * (M * CG);
  const int cg = (CG * g + CG <= nct) ? CG : nct - CG * g;
  e = rem / cg;
  ct = CG * g + (rem - e * cg);
}

#ifndef CHEFSI_MF_LB
#define CHEFSI_MF_LB 2
#endif
#ifndef CHEFSI_SK_LEN
#define CHEFSI_SK_LEN (7 * kMaxJ)
#endif
template <typename TC, typename TOUT, int EPI, int RB, int NCF, int NW>
__global__ __launch_bounds__(64 * NW, CHEFSI_MF_LB) void step_kernel_mf(StepArgs a) {
  using T = MT<TC>;
  __shared__ __attribute__((aligned(16))) TC sA[2 * T::kc(RB) * T::lda(RB)];
  __shared__ __attribute__((aligned(16))) TC sB[2 * T::kc(RB) * T::ldb(16 * NW * NCF)];
  __shared__ int32_t sK[CHEFSI_SK_LEN];
  static_assert(RB * 16 <= kMaxJ, "row blocks beyond the largest ALB count");
  const int id = xcd_linear(blockIdx.x, gridDim.x);
  int e, ct;
  step_tile<CHEFSI_MF_CG>(id, a.M, (a.ns + 16 * NW * NCF - 1) / (16 * NW * NCF), e, ct);
  step_body_mf<TC, TOUT, EPI, RB, NCF, NW>(a, a.order[e], ct, sA, sB, sK);
}

// ------------------------------------------ FP64 / FP32, direct MFMA operands
// Each wave loads its MFMA operands straight from memory in the MFMA lane
// layout -- lane l takes panel entry (k = 4s + l/16, row 16r + l%16) and the
// gathered entry (k = 4s + l/16, column 16q + l%16), so sixteen lanes read
// 16 consecutive values of one row -- into a ring of P reduction steps of
// registers.  No operand goes through LDS and the waves never wait for each
// other after the element's reduction-row map is in LDS; the waves of a
// work-group take neighbouring columns of the same element, so they share its
// panel rows through the L1 cache.  Padded reduction rows (kmap < 0) gather the
// element's first row, against the zero rows of the padded panel.
#ifndef CHEFSI_DL_P
#define CHEFSI_DL_P 2
#endif
template <typename TC, typename TOUT, int EPI, int RB, int NCF, int NW>
__device__ __forceinline__ void step_body_dl(const StepArgs& a, int K, int ct, int32_t* sK) {
  using T = MT<TC>;
  using acc_t = typename T::acc_t;
  constexpr int JP = RB * 16, TNF = 16 * NW * NCF, P = CHEFSI_DL_P;
  static_assert(P == 1 || P == 2 || P == 4, "the ring of P steps divides the steps of a padded element");
  static_assert(kStepKC % (4 * P) == 0, "element reduction rows are padded to whole rings");
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int ns = a.ns;
  const int kp = a.kpad[K];
  {
    const int32_t* km = a.kmap + a.koff[K];
    const int32_t self = static_cast<int32_t>(a.rowoff[K]);
    for (int t = tid; t < kp; t += 64 * NW) {
      const int32_t g = km[t];
      sK[t] = g >= 0 ? g : self;
    }
  }
  __syncthreads();
  const TC* panel = static_cast<const TC*>(a.panel) + a.poff[K] + (lane >> 4) * JP + (lane & 15);
  const TC* in = static_cast<const TC*>(a.in);
  const int64_t ldi = a.ldi;
  const int jb = ct * TNF + wave * (16 * NCF);
  int cofs[NCF];   // the wave's columns, clamped into the block (outputs beyond ns are not stored)
#pragma unroll
  for (int q = 0; q < NCF; ++q) cofs[q] = min(jb + 16 * q + (lane & 15), ns - 1);
  const int32_t* sk = sK + (lane >> 4);
  const int nk = kp >> 2;   // reduction steps of four rows
  TC fa[P][RB], fb[P][NCF];
  auto ld = [&](int st, int slot) {
    const TC* ps = panel + static_cast<int64_t>(st) * (4 * JP);
#pragma unroll
    for (int r = 0; r < RB; ++r) fa[slot][r] = ps[16 * r];
    const TC* xs = in + static_cast<int64_t>(sk[4 * st]) * ldi;
#pragma unroll
    for (int q = 0; q < NCF; ++q) fb[slot][q] = xs[cofs[q]];
  };
  acc_t acc[RB][NCF];
#pragma unroll
  for (int r = 0; r < RB; ++r)
#pragma unroll
    for (int q = 0; q < NCF; ++q) acc[r][q] = acc_t{};
#pragma unroll
  for (int t = 0; t < P; ++t) {
    ld(min(t, nk - 1), t);
    __builtin_amdgcn_sched_barrier(0);
  }
  for (int s0 = 0; s0 < nk; s0 += P) {
#pragma unroll
    for (int t = 0; t < P; ++t) {
#pragma unroll
      for (int r = 0; r < RB; ++r)
#pragma unroll
        for (int q = 0; q < NCF; ++q) acc[r][q] = T::mma(fa[t][r], fb[t][q], acc[r][q]);
      // the ring slot is refilled with step s0 + P + t (the last step again
      // past the end: loads stay in bounds, the values are not used); the
      // scheduling barriers keep the compiler from moving the loads next to
      // their use
      __builtin_amdgcn_sched_barrier(0);
      ld(min(s0 + P + t, nk - 1), t);
      __builtin_amdgcn_sched_barrier(0);
    }
  }
  step_epilogue<TC, TOUT, EPI, RB, NCF>(a, K, jb, acc);
}

#ifndef CHEFSI_DL_LB
#define CHEFSI_DL_LB 2
#endif
template <typename TC, typename TOUT, int EPI, int RB, int NCF, int NW>
__global__ __launch_bounds__(64 * NW, CHEFSI_DL_LB) void step_kernel_dl(StepArgs a) {
  __shared__ int32_t sK[CHEFSI_SK_LEN];
  static_assert(RB * 16 <= kMaxJ, "row blocks beyond the largest ALB count");
  const int id = xcd_linear(blockIdx.x, gridDim.x);
  int e, ct;
  // elements of more than 64 rows: narrower column tiles, larger panels
  step_tile<RB <= 4 ? CHEFSI_MF_CG : CHEFSI_MF_CG8>(id, a.M, (a.ns + 16 * NW * NCF - 1) / (16 * NW * NCF), e, ct);
  step_body_dl<TC, TOUT, EPI, RB, NCF, NW>(a, a.order[e], ct, sK);
}

#ifndef CHEFSI_MF_NCF
#define CHEFSI_MF_NCF 2
#endif
#ifndef CHEFSI_MF_WAVES
#define CHEFSI_MF_WAVES 4
#endif
#ifndef CHEFSI_MF_WAVES_RB
#define CHEFSI_MF_WAVES_RB 4
#endif
template <typename TC, typename TOUT, int EPI, int RB>
void launch_mf(const StepArgs& a, int ns, hipStream_t st) {
  // elements of more than 128 rows: 16 columns per wave (register budget);
  // elements of up to CHEFSI_MF_WAVES_RB row blocks: CHEFSI_MF_WAVES waves
  constexpr int NCF = RB <= 8 ? CHEFSI_MF_NCF : 1;
  constexpr int NW = RB <= CHEFSI_MF_WAVES_RB ? CHEFSI_MF_WAVES : 4;
  dim3 grid(static_cast<unsigned>(ceil_div(ns, 16 * NW * NCF) * a.M)), block(64 * NW);
  step_kernel_mf<TC, TOUT, EPI, RB, NCF, NW><<<grid, block, 0, st>>>(a);
}

#ifndef CHEFSI_DL_NCF
#define CHEFSI_DL_NCF 4
#endif
#ifndef CHEFSI_DL_NCF6
#define CHEFSI_DL_NCF6 2
#endif
#ifndef CHEFSI_DL_NCF8
#define CHEFSI_DL_NCF8 2
#endif
template <typename TC, typename TOUT, int EPI, int RB>
void launch_dl(const StepArgs& a, int ns, hipStream_t st) {
  // sixteen-column fragments per wave: CHEFSI_DL_NCF up to 64 rows,
  // CHEFSI_DL_NCF6 up to 96, CHEFSI_DL_NCF8 up to 128, one beyond (register
  // budget)
  constexpr int NCF = RB <= 4 ? CHEFSI_DL_NCF : (RB <= 6 ? CHEFSI_DL_NCF6 : (RB <= 8 ? CHEFSI_DL_NCF8 : 1));
  constexpr int NW = 4;
  dim3 grid(static_cast<unsigned>(ceil_div(ns, 16 * NW * NCF) * a.M)), block(64 * NW);
  step_kernel_dl<TC, TOUT, EPI, RB, NCF, NW><<<grid, block, 0, st>>>(a);
}

// FP64 steps take the direct-operand kernel, FP32 steps the LDS-staged one
// (at twice the MFMA rate, FP32 operands cannot come as 4-byte lane loads)
#ifndef CHEFSI_STEP_DL
#define CHEFSI_STEP_DL 1
#endif
template <typename TC, typename TOUT, int EPI, int RB>
void launch_step(const StepArgs& a, int ns, hipStream_t st) {
  if constexpr (CHEFSI_STEP_DL != 0 && std::is_same<TC, double>::value)
    launch_dl<TC, TOUT, EPI, RB>(a, ns, st);
  else
    launch_mf<TC, TOUT, EPI, RB>(a, ns, st);
}

template <typename TC, typename TOUT, int EPI>
int dispatch_step_mf(const Plan& p, StepArgs a, int ns, hipStream_t st) {
  // one launch per row-block class of elements
  for (size_t gi = 0; gi < p.grp_rb.size(); ++gi) {
    a.order = p.d_order + p.grp_start[gi];
    a.M = p.grp_count[gi];
    if (ceil_div(ns, 64) * a.M > 0x7fffffff) return fail(CHEFSI_ERR_ARG, "step: too many work-groups");
    switch (p.grp_rb[gi]) {
      case 1: launch_step<TC, TOUT, EPI, 1>(a, ns, st); break;
      case 2: launch_step<TC, TOUT, EPI, 2>(a, ns, st); break;
      case 3: launch_step<TC, TOUT, EPI, 3>(a, ns, st); break;
      case 4: launch_step<TC, TOUT, EPI, 4>(a, ns, st); break;
      case 5: launch_step<TC, TOUT, EPI, 5>(a, ns, st); break;
      case 6: launch_step<TC, TOUT, EPI, 6>(a, ns, st); break;
      case 7: launch_step<TC, TOUT, EPI, 7>(a, ns, st); break;
      case 8: launch_step<TC, TOUT, EPI, 8>(a, ns, st); break;
      case 9: launch_step<TC, TOUT, EPI, 9>(a, ns, st); break;
      case 10: launch_step<TC, TOUT, EPI, 10>(a, ns, st); break;
      case 11: launch_step<TC, TOUT, EPI, 11>(a, ns, st); break;
      case 12: launch_step<TC, TOUT, EPI, 12>(a, ns, st); break;
      case 13: launch_step<TC, TOUT, EPI, 13>(a, ns, st); break;
      case 14: launch_step<TC, TOUT, EPI, 14>(a, ns, st); break;
      case 15: launch_step<TC, TOUT, EPI, 15>(a, ns, st); break;
      case 16: launch_step<TC, TOUT, EPI, 16>(a, ns, st); break;
      default: return fail(CHEFSI_ERR_UNSUPPORTED, "step: more than 16 row blocks");
    }
  }
  CHEFSI_LAUNCHED("cheb_step");
  return CHEFSI_OK;
}

StepArgs base_args(const Plan& p, const void* panel, int ns) {
  StepArgs a{};
  a.panel = panel;
  a.poff = p.d_poff;
  a.kpad = p.d_kpad;
  a.koff = p.d_koff;
  a.kmap = p.d_kmap;
  a.J = p.d_J;
  a.rbv = p.d_rb;
  a.rowoff = p.d_rowoff;
  a.order = p.d_order;
  a.ns = ns;
  a.M = p.M;
  return a;
}

// ------------------------------------------------------------ small kernels
__global__ void set_bounds_kernel(double a, double b, double a0, double* d) {
  if (threadIdx.x == 0) {
    d[0] = a;
    d[1] = b;
    d[2] = a0;
  }
}

// coef[3k + {0,1,2}] = (alpha_k, beta_k, c) of the scaled recurrence.
__global__ void cheb_coef_kernel(const double* bounds, int m, double* coef) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const double a = bounds[0], b = bounds[1], a0 = bounds[2];
  const double e = 0.5 * (b - a);
  const double c = 0.5 * (b + a);
  const double s1 = e / (a0 - c);
  const double tau = 2.0 / s1;
  double s = s1;
  for (int k = 0; k < m; ++k) {
    if (k == 0) {
      coef[0] = s1 / e;
      coef[1] = 0.0;
    } else {
      const double sn = 1.0 / (tau - s);
      coef[3 * k + 0] = 2.0 * sn / e;
      coef[3 * k + 1] = s * sn;
      s = sn;
    }
    coef[3 * k + 2] = c;
  }
}

__global__ void rev_coef_kernel(const double* coef, int m, double* rcoef) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  for (int j = 0; j < m; ++j) {
    rcoef[3 * j + 0] = coef[3 * j + 0];
    rcoef[3 * j + 1] = (j + 1 < m) ? coef[3 * (j + 1) + 1] : 0.0;
    rcoef[3 * j + 2] = coef[3 * j + 2];
  }
}

__global__ void sum_first_kernel(const double* v, int k, double* out) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double s = 0.0;
  for (int i = 0; i < k; ++i) s += v[i];
  out[0] = s;
}

__global__ void const_coef_kernel(double alpha, double beta, double c, double* coef) {
  if (threadIdx.x == 0) {
    coef[0] = alpha;
    coef[1] = beta;
    coef[2] = c;
  }
}

template <typename T>
__device__ __forceinline__ T cvt(double v) {
  return static_cast<T>(v);
}
// bf16 values are stored as raw 16-bit patterns (uint16_t)
template <>
__device__ __forceinline__ uint16_t cvt<uint16_t>(double v) {
  return f2bf(static_cast<float>(v));
}

// lo: the low half of a split bf16 value (v - bf16(v), rounded to bf16)
template <typename T>
__device__ __forceinline__ T cvt_part(double v, bool lo) {
  return cvt<T>(v);
}
template <>
__device__ __forceinline__ uint16_t cvt_part<uint16_t>(double v, bool lo) {
  const uint16_t h = f2bf(static_cast<float>(v));
  return lo ? f2bf(static_cast<float>(v - static_cast<double>(bf2f(h)))) : h;
}

template <typename T>
__global__ void fill_kernel(T* d, int64_t count) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
  for (int64_t t = i; t < count; t += stride) d[t] = cvt<T>(0.0);
}

// Scatter the stored blocks into per-element panels:
//   panel_K[pre_s + r][i] = H_{K;K'_s}[i][r]    (or of H^T when transposing)
// with one 32x32 tile of one block per work-group (LDS transpose).
struct RepackArgs {
  const double* H;
  const int64_t* hoff;
  const int32_t* nbr;
  const int32_t* J;
  const int64_t* poff;
  const int32_t* rbv;
  int S;
  bool transpose_h;
  const double* shift;   // if set: the self block gets -shift on its diagonal
  bool lo_part;          // bf16 panels: store bf16(v - bf16(v)), the low half of a split value
};

// CHUNKED (bf16 path): within each 32-row chunk of the element's reduction
// rows the panel is stored row-of-H-major, [JP][32], so that one lane's eight
// consecutive reduction rows are contiguous.
template <typename T, bool CHUNKED>
__device__ __forceinline__ int64_t panel_index(int k, int i, int JP) {
  if constexpr (CHUNKED) return (static_cast<int64_t>(k >> 5) * JP + i) * 32 + (k & 31);
  return static_cast<int64_t>(k) * JP + i;
}

template <typename T, bool CHUNKED>
__global__ __launch_bounds__(256) void repack_kernel(RepackArgs ra, T* panel_base) {
  __shared__ double tile[32][33];
  const int blk = blockIdx.y;  // K * S + s
  const int K = blk / ra.S;
  const int s = blk - K * ra.S;
  const int Kp = ra.nbr[blk];
  const int JK = ra.J[K], JKp = ra.J[Kp];
  const int JP = ra.rbv[K] * 16;
  int pre = 0;
  for (int t = 0; t < s; ++t) {
    const int Jt = ra.J[ra.nbr[K * ra.S + t]];
    pre += CHUNKED ? round_up(Jt, 8) : Jt;   // BF16 panels: 8-padded neighbour segments
  }
  const int sopp = (s == 0) ? 0 : ((s & 1) ? s + 1 : s - 1);
  // panel row index k = pre + (column of H_{K;K'}), panel column = row of H_{K;K'}
  // Normal: source H_{K;s} (JK x JKp) -> panel[pre + c][r] (transpose).
  // H^T:    source H_{K';opp(s)} (JKp x JK), element [r][c] = (H^T)_{K;K'}[c][r]
  //         -> panel[pre + r][c] (copy).
  const double* src = ra.transpose_h ? ra.H + ra.hoff[Kp * ra.S + sopp] : ra.H + ra.hoff[blk];
  const int R = ra.transpose_h ? JKp : JK;
  const int C = ra.transpose_h ? JK : JKp;
  const int tilesC = (C + 31) / 32;
  const int tr = blockIdx.x / tilesC;
  const int tc = blockIdx.x - tr * tilesC;
  if (tr * 32 >= R) return;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  const double sh = (ra.shift != nullptr && s == 0) ? *ra.shift : 0.0;
  for (int yy = ty; yy < 32; yy += 8) {
    const int r = tr * 32 + yy, c = tc * 32 + tx;
    tile[yy][tx] = (r < R && c < C) ? src[static_cast<int64_t>(r) * C + c] - (r == c ? sh : 0.0) : 0.0;
  }
  __syncthreads();
  T* panel = panel_base + ra.poff[K];
  if (!ra.transpose_h) {
    // panel[pre + c][r] = tile[r][c]; write along r (panel columns) for coalescing
    for (int yy = ty; yy < 32; yy += 8) {
      const int c = tc * 32 + yy, r = tr * 32 + tx;
      if (c < C && r < R) panel[panel_index<T, CHUNKED>(pre + c, r, JP)] = cvt_part<T>(tile[tx][yy], ra.lo_part);
    }
  } else {
    for (int yy = ty; yy < 32; yy += 8) {
      const int r = tr * 32 + yy, c = tc * 32 + tx;
      if (r < R && c < C) panel[panel_index<T, CHUNKED>(pre + r, c, JP)] = cvt_part<T>(tile[yy][tx], ra.lo_part);
    }
  }
}

template <typename TS, typename TD>
__global__ void convert_kernel(const TS* src, int64_t lds, TD* dst, int64_t ldd, int64_t n, int ns) {
  const int64_t total = n * ns;
  const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
  for (int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; t < total; t += stride) {
    const int64_t r = t / ns;
    const int c = static_cast<int>(t - r * ns);
    dst[r * ldd + c] = cvt<TD>(static_cast<double>(src[r * lds + c]));
  }
}

// out[j] = sqrt(sum_r part[r][j]): 64 columns per work-group, 16 row groups
// per column (rows g, g+16, ...; four independent loads in flight), the group
// sums combined in a fixed order.
__global__ __launch_bounds__(1024) void colsum_sqrt_kernel(const double* part, int rows, int ns, double* out) {
  __shared__ double red[16][64];
  const int c = threadIdx.x & 63, g = threadIdx.x >> 6;
  const int j = blockIdx.x * 64 + c;
  double s = 0.0;
  if (j < ns) {
    int r = g;
    for (; r + 48 < rows; r += 64) {
      const double a0 = part[static_cast<int64_t>(r) * ns + j];
      const double a1 = part[static_cast<int64_t>(r + 16) * ns + j];
      const double a2 = part[static_cast<int64_t>(r + 32) * ns + j];
      const double a3 = part[static_cast<int64_t>(r + 48) * ns + j];
      s += a0;
      s += a1;
      s += a2;
      s += a3;
    }
    for (; r < rows; r += 16) s += part[static_cast<int64_t>(r) * ns + j];
  }
  red[g][c] = s;
  __syncthreads();
  if (g == 0 && j < ns) {
    double t = 0.0;
#pragma unroll
    for (int q = 0; q < 16; ++q) t += red[q][c];
    out[j] = sqrt(t);
  }
}

unsigned grid_for(int64_t total, int threads = 256) {
  int64_t g = ceil_div(total, threads);
  if (g < 1) g = 1;
  if (g > 65536) g = 65536;
  return static_cast<unsigned>(g);
}

}  // namespace

// ------------------------------------------------------------ launchers
int launch_set_bounds(double a, double b, double a0, double* d_bounds, hipStream_t st) {
  set_bounds_kernel<<<1, 64, 0, st>>>(a, b, a0, d_bounds);
  CHEFSI_LAUNCHED("set_bounds");
  return CHEFSI_OK;
}

int launch_cheb_coef(const double* d_bounds, int m, double* d_coef, hipStream_t st) {
  cheb_coef_kernel<<<1, 64, 0, st>>>(d_bounds, m, d_coef);
  CHEFSI_LAUNCHED("cheb_coef");
  return CHEFSI_OK;
}

int launch_rev_coef(const double* d_coef, int m, double* d_rcoef, hipStream_t st) {
  rev_coef_kernel<<<1, 64, 0, st>>>(d_coef, m, d_rcoef);
  CHEFSI_LAUNCHED("rev_coef");
  return CHEFSI_OK;
}

int launch_sum_first(const double* d_v, int k, double* d_out, hipStream_t st) {
  sum_first_kernel<<<1, 64, 0, st>>>(d_v, k, d_out);
  CHEFSI_LAUNCHED("sum_first");
  return CHEFSI_OK;
}

int launch_const_coef(double alpha, double c, double* d_coef, hipStream_t st) {
  const_coef_kernel<<<1, 64, 0, st>>>(alpha, 0.0, c, d_coef);
  CHEFSI_LAUNCHED("const_coef");
  return CHEFSI_OK;
}

int launch_const_coef3(double alpha, double beta, double c, double* d_coef, hipStream_t st) {
  const_coef_kernel<<<1, 64, 0, st>>>(alpha, beta, c, d_coef);
  CHEFSI_LAUNCHED("const_coef");
  return CHEFSI_OK;
}

int launch_repack(const Plan& p, const double* d_H, int dtype, bool transpose_h, void* d_panel,
                  hipStream_t st, const double* d_shift) {
  const unsigned fill_grid = grid_for(p.panel_elems);
  RepackArgs ra{d_H, p.d_hoff, p.d_nbr, p.d_J, p.d_poff, p.d_rb, p.stencil, transpose_h, d_shift, false};
  const int tiles = static_cast<int>(ceil_div(p.maxJ, 32) * ceil_div(p.maxJ, 32));
  dim3 grid(tiles, p.M * p.stencil);
  if (dtype == CHEFSI_F64) {
    fill_kernel<double><<<fill_grid, 256, 0, st>>>(static_cast<double*>(d_panel), p.panel_elems);
    repack_kernel<double, false><<<grid, 256, 0, st>>>(ra, static_cast<double*>(d_panel));
  } else if (dtype == CHEFSI_F32) {
    fill_kernel<float><<<fill_grid, 256, 0, st>>>(static_cast<float*>(d_panel), p.panel_elems);
    repack_kernel<float, false><<<grid, 256, 0, st>>>(ra, static_cast<float*>(d_panel));
  } else if (dtype == CHEFSI_BF16 || dtype == CHEFSI_BF16X3) {
    // split BF16: the hi panel, then the lo panel panel8_elems further on
    const int parts = (dtype == CHEFSI_BF16X3) ? 2 : 1;
    const unsigned fill8 = grid_for(parts * p.panel8_elems);
    RepackArgs rb = ra;
    rb.poff = p.d_poff8;
    fill_kernel<uint16_t><<<fill8, 256, 0, st>>>(static_cast<uint16_t*>(d_panel), parts * p.panel8_elems);
    repack_kernel<uint16_t, true><<<grid, 256, 0, st>>>(rb, static_cast<uint16_t*>(d_panel));
    if (parts == 2) {
      rb.lo_part = true;
      repack_kernel<uint16_t, true><<<grid, 256, 0, st>>>(rb, static_cast<uint16_t*>(d_panel) + p.panel8_elems);
    }
  } else {
    return fail(CHEFSI_ERR_UNSUPPORTED, "repack: dtype");
  }
  CHEFSI_LAUNCHED("repack");
  return CHEFSI_OK;
}

int launch_step(const Plan& p, const void* d_panel, int dtype, const double* d_coef,
                const StepIO& io, int ns, hipStream_t st) {
  if (ns <= 0) return CHEFSI_OK;
  StepArgs a = base_args(p, d_panel, ns);
  a.coef = d_coef;
  a.in = io.in;
  a.ldi = io.ldi;
  a.prev = io.prev;
  a.ldp = io.ldp;
  a.out = io.out;
  a.ldo = io.ldo;
  if (dtype == CHEFSI_F64) {
    if (!io.in_f64 || (io.prev && !io.prev_f64) || !io.out_f64)
      return fail(CHEFSI_ERR_ARG, "step: FP64 step needs FP64 operands");
    if (io.shifted) return dispatch_step_mf<double, double, 2>(p, a, ns, st);
    return dispatch_step_mf<double, double, 0>(p, a, ns, st);
  }
  if (dtype == CHEFSI_F32) {
    if (io.in_f64 || (io.prev && io.prev_f64))
      return fail(CHEFSI_ERR_ARG, "step: FP32 step needs FP32 inputs");
    if (io.shifted) {
      if (io.out_f64) return dispatch_step_mf<float, double, 2>(p, a, ns, st);
      return dispatch_step_mf<float, float, 2>(p, a, ns, st);
    }
    if (io.out_f64) return dispatch_step_mf<float, double, 0>(p, a, ns, st);
    return dispatch_step_mf<float, float, 0>(p, a, ns, st);
  }
  return fail(CHEFSI_ERR_UNSUPPORTED, "step: dtype");
}

int launch_step_b16(const Plan& p, const void* d_panel8, const double* d_coef, const void* in, const void* prev,
                    void* out, bool out_f64, int64_t ldo, int ns, hipStream_t st, bool split) {
  if (ns <= 0) return CHEFSI_OK;
  if (in == nullptr || out == nullptr) return fail(CHEFSI_ERR_ARG, "step: null buffer");
  if ((reinterpret_cast<uintptr_t>(in) | reinterpret_cast<uintptr_t>(prev) | reinterpret_cast<uintptr_t>(d_panel8)) & 15u)
    return fail(CHEFSI_ERR_ARG, "step: BF16 buffers must be 16-byte aligned");
  if (!out_f64 && (reinterpret_cast<uintptr_t>(out) & 7u)) return fail(CHEFSI_ERR_ARG, "step: BF16 output alignment");
  if (ceil_div(ns, 32) * p.M > 0x7fffffff) return fail(CHEFSI_ERR_ARG, "step: too many work-groups");
  StepArgsB a{};
  a.panel = static_cast<const uint16_t*>(d_panel8);
  a.poff8 = p.d_poff8;
  a.kpad8 = p.d_kpad8;
  a.kgoff = p.d_kgoff;
  a.kg8 = p.d_kg8;
  a.J = p.d_J;
  a.rbv = p.d_rb;
  a.rowoff8 = p.d_rowoff8;
  a.rowoff = p.d_rowoff;
  a.order = p.d_order;
  a.coef = d_coef;
  a.in = static_cast<const uint16_t*>(in);
  a.prev = static_cast<const uint16_t*>(prev);
  a.out = out;
  a.ldo = ldo;
  a.ns = ns;
  a.M = p.M;
  a.panel_lo = split ? p.panel8_elems : 0;
  a.mv_lo = split ? p.N8 * static_cast<int64_t>(ns) : 0;
  if (split) {
    if (out_f64)
      dispatch_step_b16<true, true>(p, a, ns, st);
    else
      dispatch_step_b16<false, true>(p, a, ns, st);
  } else if (out_f64) {
    dispatch_step_b16<true, false>(p, a, ns, st);
  } else {
    dispatch_step_b16<false, false>(p, a, ns, st);
  }
  CHEFSI_LAUNCHED("cheb_step_b16");
  return CHEFSI_OK;
}

int launch_to_tiles_b16(const Plan& p, const double* X, int64_t ldx, void* out, int ns, hipStream_t st, bool split) {
  if (ns <= 0) return CHEFSI_OK;
  dim3 grid(static_cast<unsigned>(ceil_div(p.N8, 64)), static_cast<unsigned>(ceil_div(ns, 64)));
  uint16_t* hi = static_cast<uint16_t*>(out);
  to_tiles_b16_kernel<<<grid, 256, 0, st>>>(X, ldx, p.d_rowsrc8, p.N8, ns, hi,
                                            split ? hi + p.N8 * static_cast<int64_t>(ns) : nullptr);
  CHEFSI_LAUNCHED("to_tiles_b16");
  return CHEFSI_OK;
}

int launch_resid_partial(const Plan& p, const void* d_panel, const double* d_X, int64_t ldx,
                         const double* d_theta, int ns, double* d_part, hipStream_t st) {
  if (ns <= 0) return CHEFSI_OK;
  StepArgs a = base_args(p, d_panel, ns);
  a.in = d_X;
  a.ldi = ldx;
  a.theta = d_theta;
  a.part = d_part;
  return dispatch_step_mf<double, double, 1>(p, a, ns, st);
}

int launch_colsum_sqrt(const double* d_part, int rows, int ns, double* d_out, hipStream_t st) {
  if (ns <= 0) return CHEFSI_OK;
  colsum_sqrt_kernel<<<static_cast<unsigned>(ceil_div(ns, 64)), 1024, 0, st>>>(d_part, rows, ns, d_out);
  CHEFSI_LAUNCHED("colsum_sqrt");
  return CHEFSI_OK;
}

int launch_convert(const double* src, int64_t lds, void* dst, int dst_dtype, int64_t ldd,
                   int64_t n, int ns, hipStream_t st) {
  const unsigned g = grid_for(n * ns);
  if (dst_dtype == CHEFSI_F64)
    convert_kernel<double, double><<<g, 256, 0, st>>>(src, lds, static_cast<double*>(dst), ldd, n, ns);
  else if (dst_dtype == CHEFSI_F32)
    convert_kernel<double, float><<<g, 256, 0, st>>>(src, lds, static_cast<float*>(dst), ldd, n, ns);
  else
    return fail(CHEFSI_ERR_UNSUPPORTED, "convert: dtype");
  CHEFSI_LAUNCHED("convert");
  return CHEFSI_OK;
}

int launch_copy_f64(const double* src, int64_t lds, double* dst, int64_t ldd, int64_t n, int ns,
                    hipStream_t st) {
  return launch_convert(src, lds, dst, CHEFSI_F64, ldd, n, ns, st);
}

}  // namespace chefsi
