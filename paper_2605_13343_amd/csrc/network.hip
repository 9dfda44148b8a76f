// Network forward of the hierarchical transformer preconditioner (paper
// Sec. 4.1-4.4 and Supplementary "Network Architecture Details"), every
// frame of a batch at once.
//
// Layout: diagonal-stream tokens are the batch's rows (Nd = ntot); off-
// diagonal tokens are (tile, t) pairs (No = mtot * L_s).  The residual streams
// stay FP32; GEMM inputs are BF16 (compute = HP_BF16, MFMA 32x32x16 with FP32
// accumulation) or FP32 (compute = HP_F32, MFMA 32x32x2 in FP32).
#include <math.h>
#include <string.h>

#include <array>
#include <type_traits>

#include "batch.h"

namespace hp {

typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x4_t __attribute__((ext_vector_type(4)));
typedef float f32x16_t __attribute__((ext_vector_type(16)));
typedef float f32x4_t __attribute__((ext_vector_type(4)));

__device__ inline float gelu_f(float x) { return 0.5f * x * (1.f + erff(x * 0.7071067811865476f)); }
__device__ inline float softplus_f(float x) { return fmaxf(x, 0.f) + log1pf(expf(-fabsf(x))); }

template <typename AT> __device__ inline AT to_act(float v);
template <> __device__ inline float to_act<float>(float v) { return v; }
template <> __device__ inline uint16_t to_act<uint16_t>(float v) { return f32_to_bf16(v); }

__device__ inline float wave_sum_f(float v) { return wave_total(v); }

// Four independent wave sums.
__device__ inline void wave_sum4(float (&v)[4]) {
#pragma unroll
  for (int r = 0; r < 4; ++r) v[r] = wave_total(v[r]);
}

// ------------------------------------------------------------------ GEMM
// Y[M, N] = act(X[M, K] W + b) (+ resid), with W given transposed as
// Wt[N][K] (K contiguous, K % 32 == 0).  64 x 64 block tile, four waves of
// 32 x 32, K staged through two LDS buffers in steps of 32.
struct GemmArgs {
  const void* X;
  int64_t ldx;
  const void* Wt;
  int K;
  const float* bias;
  const float* resid;
  int64_t ldr;
  float* Yf;
  int64_t ldf;
  void* Yb;
  int64_t ldb;
  float* pre;   // optional: value before the activation (after the bias)
  int64_t ldp;
  int M, N, act;
};

// GELU of the BF16 path from the complementary error function of
// Abramowitz & Stegun, Handbook of Mathematical Functions, formula 7.1.26:
// erfc(z) = t (a1 + t (a2 + t (a3 + t (a4 + t a5)))) exp(-z^2), t = 1 / (1 +
// p z), z >= 0, absolute error at most 1.5e-7.  With z = |x| / sqrt(2) and
// q = erfc(z) / 2, GELU(x) = x (1 + erf(x / sqrt 2)) / 2 = max(x, 0) - |x| q
// for either sign; the 1/2 is folded into a1..a5 and 1/sqrt 2 into p and the
// exponent.  14 operations (one reciprocal, one exp2), no branches, and no
// cancellation in 1 + erf for negative x; far below the BF16 rounding of the
// value that follows.  The FP32 path keeps the library erff.
__device__ inline float gelu_bf16path(float x) {
  const float ax = fabsf(x);
  const float t = __builtin_amdgcn_rcpf(fmaf(ax, 0.23164189758f, 1.f));  // p / sqrt 2
  const float poly =
      t * fmaf(t, fmaf(t, fmaf(t, fmaf(t, 0.5307027145f, -0.7265760135f), 0.7107068705f), -0.142248368f),
               0.127414796f);
  const float e2 = __builtin_amdgcn_exp2f(x * (x * -0.72134752044f));  // exp(-x^2 / 2) = 2^(-x^2 log2(e) / 2)
  float relu;  // max(x, 0) as one instruction (fmaxf adds a NaN-canonicalising max)
  asm("v_max_f32 %0, 0, %1" : "=v"(relu) : "v"(x));
  return fmaf(-ax, poly * e2, relu);
}

template <typename AT> __device__ inline float gemm_gelu(float v);
template <> __device__ inline float gemm_gelu<float>(float v) { return gelu_f(v); }
template <> __device__ inline float gemm_gelu<uint16_t>(float v) { return gelu_bf16path(v); }

// Epilogue of one 32 x 32 output fragment that the MFMA produced transposed
// (W as the first operand): the lane holds output row `row` and, for q = 0..3,
// the four consecutive columns cb + 8 q .. cb + 8 q + 3 in acc[4 q .. 4 q + 3]
// (cb = fragment column + 4 (lane / 32)).  Four-wide vector loads and stores
// where every operand's leading dimension and base allow them.
// Two floats to packed BF16, round to nearest even (the hardware conversion).
__device__ inline uint32_t pack_bf16x2(float lo, float hi) {
  typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));
  typedef float f32x2_t __attribute__((ext_vector_type(2)));
  const f32x2_t v = {lo, hi};
  return __builtin_bit_cast(uint32_t, __builtin_convertvector(v, bf16x2_t));
}

// Bias of the four column groups cb + 8q .. cb + 8q + 3 (q = 0..3) of a
// fragment, zero without a bias.
__device__ inline void gemm_bias16(const GemmArgs& a, int cb, float bv[16]) {
  if (a.bias) {
    if (((uintptr_t)a.bias & 15) == 0) {
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const float4 t = *(const float4*)(a.bias + cb + 8 * q);
        bv[4 * q] = t.x;
        bv[4 * q + 1] = t.y;
        bv[4 * q + 2] = t.z;
        bv[4 * q + 3] = t.w;
      }
    } else {
#pragma unroll
      for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int c = 0; c < 4; ++c) bv[4 * q + c] = a.bias[cb + 8 * q + c];
    }
  } else {
#pragma unroll
    for (int e = 0; e < 16; ++e) bv[e] = 0.f;
  }
}

template <typename AT, bool GELU>
__device__ inline void gemm_epilogue_t(const GemmArgs& a, const f32x16_t& acc, int row, int cb, bool vec) {
  if (row >= a.M) return;
  const int64_t r = row;
  // row bases formed once; the columns below are 32-bit offsets from them
  float* pre = a.pre ? a.pre + r * a.ldp : nullptr;
  const float* res = a.resid ? a.resid + r * a.ldr : nullptr;
  float* yf = a.Yf ? a.Yf + r * a.ldf : nullptr;
  AT* yb = a.Yb ? (AT*)a.Yb + r * a.ldb : nullptr;
  constexpr bool gelu = GELU;
  // presence tests on the (uniform) kernel arguments, not on the row pointers
  const bool has_pre = a.pre != nullptr, has_res = a.resid != nullptr, has_yf = a.Yf != nullptr,
             has_yb = a.Yb != nullptr;
  if (vec && cb + 27 < a.N) {
    // every column of the fragment in range: the bias and residual loads of
    // all four column groups are issued together, then one wait
    float bv[16], rv[16];
    gemm_bias16(a, cb, bv);
    if (has_res) {
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const float4 t = *(const float4*)(res + cb + 8 * q);
        rv[4 * q] = t.x;
        rv[4 * q + 1] = t.y;
        rv[4 * q + 2] = t.z;
        rv[4 * q + 3] = t.w;
      }
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int c0 = cb + 8 * q;
      float v[4];
#pragma unroll
      for (int c = 0; c < 4; ++c) v[c] = acc[4 * q + c] + bv[4 * q + c];
      if (has_pre) *(float4*)(pre + c0) = make_float4(v[0], v[1], v[2], v[3]);
      if (gelu) {
#pragma unroll
        for (int c = 0; c < 4; ++c) v[c] = gemm_gelu<AT>(v[c]);
      }
      if (has_res) {
#pragma unroll
        for (int c = 0; c < 4; ++c) v[c] += rv[4 * q + c];
      }
      if (has_yf) *(float4*)(yf + c0) = make_float4(v[0], v[1], v[2], v[3]);
      if (has_yb) {
        if constexpr (sizeof(AT) == 2)
          *(uint2*)(yb + c0) = make_uint2(pack_bf16x2(v[0], v[1]), pack_bf16x2(v[2], v[3]));
        else
          *(float4*)(yb + c0) = make_float4(v[0], v[1], v[2], v[3]);
      }
    }
    return;
  }
#pragma unroll
  for (int q = 0; q < 4; ++q) {
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const int col = cb + 8 * q + c;
      if (col >= a.N) break;
      float x = acc[4 * q + c] + (a.bias ? a.bias[col] : 0.f);
      if (has_pre) pre[col] = x;
      if (gelu) x = gemm_gelu<AT>(x);
      if (has_res) x += res[col];
      if (has_yf) yf[col] = x;
      if (has_yb) yb[col] = to_act<AT>(x);
    }
  }
}

// The activation is a template parameter so that the per-element code has no
// branches; the launch-wide choice is taken once here.
template <typename AT>
__device__ inline void gemm_epilogue(const GemmArgs& a, const f32x16_t& acc, int row, int cb, bool vec) {
  if (a.act == 1) gemm_epilogue_t<AT, true>(a, acc, row, cb, vec);
  else gemm_epilogue_t<AT, false>(a, acc, row, cb, vec);
}

// Whether every output and the residual admit the four-wide accesses of the
// epilogue (leading dimensions multiples of 4, 16-byte aligned bases).
__device__ inline bool gemm_vec_ok(const GemmArgs& a, int act_bytes) {
  auto ok = [](const void* p, int64_t ld, int eb) {
    return !p || ((ld & 3) == 0 && ((uintptr_t)p & (uintptr_t)(4 * eb - 1)) == 0);
  };
  return ok(a.resid, a.ldr, 4) && ok(a.Yf, a.ldf, 4) && ok(a.pre, a.ldp, 4) && ok(a.Yb, a.ldb, act_bytes);
}

template <typename AT>
__global__ __launch_bounds__(256) void k_gemm(GemmArgs a) {
  constexpr int BM = 64, BN = 64, BK = 32;
  constexpr int PAD = sizeof(AT) == 2 ? 8 : 4;
  constexpr int NV = sizeof(AT) == 2 ? 1 : 2;  // 16-byte loads per thread and operand
  __shared__ __attribute__((aligned(16))) AT sA[2][BM][BK + PAD];
  __shared__ __attribute__((aligned(16))) AT sB[2][BN][BK + PAD];
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  // 1-D grid, remapped so that one XCD receives consecutive (row tile,
  // column tile) pairs, column fastest: the column tiles of a row tile share
  // that XCD's L2 copy of the X rows instead of fetching them again
  const int tiles_n = (a.N + BN - 1) / BN, nblk = (int)gridDim.x, id = (int)blockIdx.x;
  const int lin = (nblk % 8 == 0) ? (id % 8) * (nblk / 8) + id / 8 : id;
  const int m0 = (lin / tiles_n) * BM, n0 = (lin % tiles_n) * BN;
  const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
  const AT* X = (const AT*)a.X;
  const AT* W = (const AT*)a.Wt;
  // two-stage pipeline: the next K step's global loads are issued before the
  // current step's MFMAs and stored to the other LDS buffer after them
  uint4 ra[NV], rb[NV];
  auto gload = [&](int k0) {
#pragma unroll
    for (int q = 0; q < NV; ++q) {
      const int idx = tid + q * 256;
      const int r = sizeof(AT) == 2 ? idx >> 2 : idx >> 3;
      const int c = sizeof(AT) == 2 ? (idx & 3) * 8 : (idx & 7) * 4;
      ra[q] = (m0 + r < a.M) ? *(const uint4*)(X + (int64_t)(m0 + r) * a.ldx + k0 + c) : make_uint4(0, 0, 0, 0);
      rb[q] = (n0 + r < a.N) ? *(const uint4*)(W + (int64_t)(n0 + r) * a.K + k0 + c) : make_uint4(0, 0, 0, 0);
    }
  };
  auto sstore = [&](int buf) {
#pragma unroll
    for (int q = 0; q < NV; ++q) {
      const int idx = tid + q * 256;
      const int r = sizeof(AT) == 2 ? idx >> 2 : idx >> 3;
      const int c = sizeof(AT) == 2 ? (idx & 3) * 8 : (idx & 7) * 4;
      *(uint4*)&sA[buf][r][c] = ra[q];
      *(uint4*)&sB[buf][r][c] = rb[q];
    }
  };
  f32x16_t acc;
#pragma unroll
  for (int i = 0; i < 16; ++i) acc[i] = 0.f;
  const int nk = a.K / BK;
  gload(0);
  sstore(0);
  __syncthreads();
  for (int kt = 0; kt < nk; ++kt) {
    const int buf = kt & 1;
    if (kt + 1 < nk) gload((kt + 1) * BK);
    if constexpr (sizeof(AT) == 2) {
#pragma unroll
      for (int kk = 0; kk < BK; kk += 16) {
        bf16x8_t av = __builtin_bit_cast(bf16x8_t, *(const uint4*)&sA[buf][wm + (lane & 31)][kk + (lane >> 5) * 8]);
        bf16x8_t bv = __builtin_bit_cast(bf16x8_t, *(const uint4*)&sB[buf][wn + (lane & 31)][kk + (lane >> 5) * 8]);
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(bv, av, acc, 0, 0, 0);
      }
    } else {
#pragma unroll
      for (int kk = 0; kk < BK; kk += 2) {
        float av = sA[buf][wm + (lane & 31)][kk + (lane >> 5)];
        float bv = sB[buf][wn + (lane & 31)][kk + (lane >> 5)];
        acc = __builtin_amdgcn_mfma_f32_32x32x2f32(bv, av, acc, 0, 0, 0);
      }
    }
    if (kt + 1 < nk) sstore(buf ^ 1);
    __syncthreads();
  }
  gemm_epilogue<AT>(a, acc, m0 + wm + (lane & 31), n0 + wn + 4 * (lane >> 5), gemm_vec_ok(a, (int)sizeof(AT)));
}

// BF16 tile-kernel family: a BM x BN block tile of (BM/WM) x (BN/WN) waves,
// each wave WM x WN in 32 x 32 MFMA fragments, K staged through two LDS
// buffers in steps of BK.  Global loads run PF steps ahead of the MFMAs (PF =
// 1: the next step's loads are issued before the current step's MFMAs; PF =
// 2: two register sets, so a step's loads have two steps of MFMAs to land
// before they are written to LDS).  Every member issues, per output element,
// the same MFMA sequence along K (k ascending in steps of 16) and the same
// epilogue, so all of them give bit-identical results; the autotuner picks
// one per shape.  1-D grid with the XCD-aware, column-fastest tile order.
template <int BM, int BN, int BK, int WM, int WN, int PF>
__global__ __launch_bounds__((BM / WM) * (BN / WN) * 64) void k_gemm_bt(GemmArgs a, int tiles_n) {
  constexpr int NWN = BN / WN, NT = (BM / WM) * NWN * 64, LDK = BK + 8, KC = BK / 8;
  // 16-byte chunks per thread and operand (the last round may leave threads idle)
  constexpr int CA = (BM * KC + NT - 1) / NT, CB = (BN * KC + NT - 1) / NT, FM = WM / 32, FN = WN / 32;
  static_assert(PF == 1 || PF == 2, "prefetch depth 1 or 2");
  __shared__ __attribute__((aligned(16))) uint16_t sA[2][BM][LDK];
  __shared__ __attribute__((aligned(16))) uint16_t sB[2][BN][LDK];
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int nblk = (int)gridDim.x, id = (int)blockIdx.x;
  const int lin = (nblk % 8 == 0) ? (id % 8) * (nblk / 8) + id / 8 : id;
  const int m0 = (lin / tiles_n) * BM, n0 = (lin % tiles_n) * BN;
  const int wm = (wave / NWN) * WM, wn = (wave % NWN) * WN;
  const uint16_t* X = (const uint16_t*)a.X;
  const uint16_t* W = (const uint16_t*)a.Wt;
  uint4 ra[PF][CA], rb[PF][CB];
  auto gload = [&](uint4(&xa)[CA], uint4(&xb)[CB], int k0) {
#pragma unroll
    for (int q = 0; q < CA; ++q) {
      const int idx = tid + q * NT, r = idx / KC, c = (idx % KC) * 8;
      if (BM * KC % NT != 0 && idx >= BM * KC) break;
      xa[q] = (m0 + r < a.M) ? *(const uint4*)(X + (int64_t)(m0 + r) * a.ldx + k0 + c) : make_uint4(0, 0, 0, 0);
    }
#pragma unroll
    for (int q = 0; q < CB; ++q) {
      const int idx = tid + q * NT, r = idx / KC, c = (idx % KC) * 8;
      if (BN * KC % NT != 0 && idx >= BN * KC) break;
      xb[q] = (n0 + r < a.N) ? *(const uint4*)(W + (int64_t)(n0 + r) * a.K + k0 + c) : make_uint4(0, 0, 0, 0);
    }
  };
  auto sstore = [&](const uint4(&xa)[CA], const uint4(&xb)[CB], int buf) {
#pragma unroll
    for (int q = 0; q < CA; ++q) {
      const int idx = tid + q * NT;
      if (BM * KC % NT != 0 && idx >= BM * KC) break;
      *(uint4*)&sA[buf][idx / KC][(idx % KC) * 8] = xa[q];
    }
#pragma unroll
    for (int q = 0; q < CB; ++q) {
      const int idx = tid + q * NT;
      if (BN * KC % NT != 0 && idx >= BN * KC) break;
      *(uint4*)&sB[buf][idx / KC][(idx % KC) * 8] = xb[q];
    }
  };
  f32x16_t acc[FM][FN];
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j)
#pragma unroll
      for (int q = 0; q < 16; ++q) acc[i][j][q] = 0.f;
  auto compute = [&](int buf) {
#pragma unroll
    for (int kk = 0; kk < BK; kk += 16) {
      bf16x8_t av[FM], bv[FN];
#pragma unroll
      for (int i = 0; i < FM; ++i)
        av[i] = __builtin_bit_cast(bf16x8_t, *(const uint4*)&sA[buf][wm + 32 * i + (lane & 31)][kk + (lane >> 5) * 8]);
#pragma unroll
      for (int j = 0; j < FN; ++j)
        bv[j] = __builtin_bit_cast(bf16x8_t, *(const uint4*)&sB[buf][wn + 32 * j + (lane & 31)][kk + (lane >> 5) * 8]);
#pragma unroll
      for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(bv[j], av[i], acc[i][j], 0, 0, 0);
    }
  };
  const int nk = a.K / BK;
  if constexpr (PF == 1) {
    gload(ra[0], rb[0], 0);
    sstore(ra[0], rb[0], 0);
    __syncthreads();
    for (int kt = 0; kt < nk; ++kt) {
      const int buf = kt & 1;
      if (kt + 1 < nk) gload(ra[0], rb[0], (kt + 1) * BK);
      compute(buf);
      if (kt + 1 < nk) sstore(ra[0], rb[0], buf ^ 1);
      __syncthreads();
    }
  } else {
    // step s lives in LDS buffer s & 1 and in register set s & 1
    gload(ra[0], rb[0], 0);
    if (nk > 1) gload(ra[1], rb[1], BK);
    sstore(ra[0], rb[0], 0);
    __syncthreads();
    for (int kt = 0; kt < nk; kt += 2) {
      if (kt + 2 < nk) gload(ra[0], rb[0], (kt + 2) * BK);
      compute(0);
      if (kt + 1 < nk) sstore(ra[1], rb[1], 1);
      __syncthreads();
      if (kt + 1 >= nk) break;
      if (kt + 3 < nk) gload(ra[1], rb[1], (kt + 3) * BK);
      compute(1);
      if (kt + 2 < nk) sstore(ra[0], rb[0], 0);
      __syncthreads();
    }
  }
  const bool vec = gemm_vec_ok(a, 2);
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j)
      gemm_epilogue<uint16_t>(a, acc[i][j], m0 + wm + 32 * i + (lane & 31), n0 + wn + 32 * j + 4 * (lane >> 5), vec);
}

// ------------------------------------------------------------------ fused FFN
// X += GELU(U W1 + b1) W2 + b2 for d = 128, hidden 4d = 512, BF16 operands and
// FP32 accumulation, without the hidden activations leaving the chip (the
// inference path).  Block: 128 rows, 4 waves; a wave owns 32 rows and all
// 128 outputs of them.  The hidden units run in 4 chunks of 128:
//   1. H^T chunk (128 hidden x the wave's 32 rows: four 32 x 32 fragments) =
//      W1c U^T along K = 512 in steps of 32; the block's U rows and W1c rows
//      pass through a 3-stage LDS ring filled straight from global memory,
//      which runs on across chunks (the next chunk's first steps load while
//      a chunk ends);
//   2. bias, GELU and BF16 rounding in registers;
//   3. Y^T += W2c H^T, with W2c (128 outputs x 128 hidden) staged in LDS
//      while step 1 runs.
// Every output element sees the MFMA sequence of the two-GEMM path (k steps
// of 16 in increasing order, one accumulator chain, W as the first operand),
// the same bias, GELU and rounding, and the same epilogue ((acc + b2) + X),
// so the results equal it bit for bit.  After step 1 a lane holds hidden
// units 8 q + 4 (lane / 32) + 0..3 (q = 0..3) of each fragment for its row;
// step 3 takes units 8 (lane / 32) + 0..7 of each 16-unit k step, so each
// lane swaps two of its four groups with the lane 32 away.
// The biases are read with wave-uniform (scalar) loads, so reading them
// never waits for the ring's vector loads in flight.  LDS: 80 KB (two blocks
// per CU); at most 256 registers per lane (two waves per SIMD).  Rows past M
// load row M - 1 and are not stored.
constexpr int FFN_BM = 128, FFN_HC = 128, FFN_ST = 3;
constexpr int FFN_RING = FFN_ST * 256 * 32;  // BF16 elements: per stage 128 U rows + 128 W1 rows, 32 k each
constexpr int FFN_W2 = 128 * 128;            // BF16 elements: 128 outputs x 128 hidden of one chunk

__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2)))
void k_ffn_fused(const uint16_t* __restrict__ U, const uint16_t* __restrict__ W1t, const float* __restrict__ b1,
                 const uint16_t* __restrict__ W2t, const float* __restrict__ b2, float* X, int M) {
  constexpr int K = 512, NO = 128, BK = 32, NCH = 512 / FFN_HC, KT = K / BK, NT = NCH * KT, LPW = 4;
  __shared__ __attribute__((aligned(1024))) uint16_t lds[FFN_RING + FFN_W2];
  uint16_t* const ring = lds;            // [stage][256 rows][32 k], 16-byte chunk c of row r at c ^ ((r / 4) % 4)
  uint16_t* const w2s = lds + FFN_RING;  // [128 outputs][128 hidden], 16-byte chunk c of row r at c ^ (r % 16)
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63, hh = lane >> 5, r32 = lane & 31;
  const int m0 = blockIdx.x * FFN_BM;
  // ring sources: stage rows 0..127 are U rows m0.., rows 128..255 the chunk's
  // W1 rows; one wave instruction fills one 1 KB block (16 rows of 64 bytes,
  // lane i -> row i / 4, position i % 4); waves 0-1 fill the U part, 2-3 the W1 part
  const uint16_t* src[LPW];
  bool w1part[LPW];
#pragma unroll
  for (int q = 0; q < LPW; ++q) {
    const int blk = wave * LPW + q, crow = 16 * blk + (lane >> 2);
    const int c = (lane & 3) ^ ((crow >> 2) & 3);
    w1part[q] = crow >= FFN_BM;
    src[q] = crow < FFN_BM ? U + (int64_t)min(m0 + crow, M - 1) * K + 8 * c : W1t + (int64_t)(crow - FFN_BM) * K + 8 * c;
  }
  auto issue = [&](int t) {
    const int slot = t % FFN_ST, ch = t / KT, k0 = (t % KT) * BK;
#pragma unroll
    for (int q = 0; q < LPW; ++q) {
      const int blk = wave * LPW + q;
      const uint16_t* p = src[q] + k0 + (w1part[q] ? (int64_t)ch * FFN_HC * K : 0);
      __builtin_amdgcn_global_load_lds((const __attribute__((address_space(1))) void*)p,
                                       (__attribute__((address_space(3))) void*)&ring[slot * 8192 + blk * 512], 16, 0,
                                       0);
    }
  };
  // W2 columns of chunk ch: 32 instructions of 4 rows x 256 bytes, 8 per wave
  auto issue_w2 = [&](int ch) {
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int j = wave * 8 + q, r = 4 * j + (lane >> 4), pos = lane & 15, c = pos ^ (r & 15);
      __builtin_amdgcn_global_load_lds(
          (const __attribute__((address_space(1))) void*)(W2t + (int64_t)r * 512 + ch * FFN_HC + 8 * c),
          (__attribute__((address_space(3))) void*)&w2s[j * 512], 16, 0, 0);
    }
  };
  // the eight biases of columns cb .. cb + 7 (cb wave-uniform), the lane's four of them
  auto bias4 = [&](const float* b, int cb) {
    float v[8];
#pragma unroll
    for (int e = 0; e < 8; ++e)
      v[e] = __builtin_bit_cast(float, __builtin_amdgcn_readfirstlane(__builtin_bit_cast(int, b[cb + e])));
    return hh ? make_float4(v[4], v[5], v[6], v[7]) : make_float4(v[0], v[1], v[2], v[3]);
  };
  auto opnd = [&](int slot, int row, int c) {
    return __builtin_bit_cast(bf16x8_t, *(const uint4*)&ring[slot * 8192 + row * 32 + 8 * (c ^ ((row >> 2) & 3))]);
  };
  f32x16_t acc1[4], acc2[4];
#pragma unroll
  for (int f = 0; f < 4; ++f)
#pragma unroll
    for (int q = 0; q < 16; ++q) acc1[f][q] = acc2[f][q] = 0.f;
#pragma unroll
  for (int t = 0; t < FFN_ST - 1; ++t) issue(t);
  for (int t = 0; t < NT; ++t) {
    // step t has landed once only the later steps' loads are outstanding
    // (waiting for more, such as a W2 chunk issued between them, is safe; the
    // last steps wait for everything)
    if (t + FFN_ST - 2 < NT) asm volatile("s_waitcnt vmcnt(%0)" ::"n"((FFN_ST - 2) * LPW) : "memory");
    else asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
    __builtin_amdgcn_s_barrier();  // every wave is past step t - 1 (and a chunk's W2 reads)
    asm volatile("" ::: "memory");
    const int kt = t % KT, ch = t / KT;
    if (kt == 0) issue_w2(ch);
    if (t + FFN_ST - 1 < NT) issue(t + FFN_ST - 1);
    const int slot = t % FFN_ST;
#pragma unroll
    for (int kk = 0; kk < BK; kk += 16) {
      const int c = kk / 8 + hh;
      const bf16x8_t ub = opnd(slot, 32 * wave + r32, c);
#pragma unroll
      for (int f = 0; f < 4; ++f)
        acc1[f] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(opnd(slot, FFN_BM + 32 * f + r32, c), ub, acc1[f], 0, 0, 0);
    }
    if (kt != KT - 1) continue;
    // the chunk's hidden values: bias, GELU, BF16 (as the first GEMM's
    // epilogue), regrouped into the k order of the second product
    uint4 hop[8];  // B operand of k step 2 f + e of this chunk
#pragma unroll
    for (int f = 0; f < 4; ++f) {
      uint32_t d[8];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const float4 bb = bias4(b1, ch * FFN_HC + 32 * f + 8 * q);
        const float v0 = gelu_bf16path(acc1[f][4 * q] + bb.x), v1 = gelu_bf16path(acc1[f][4 * q + 1] + bb.y);
        const float v2 = gelu_bf16path(acc1[f][4 * q + 2] + bb.z), v3 = gelu_bf16path(acc1[f][4 * q + 3] + bb.w);
        d[2 * q] = pack_bf16x2(v0, v1);
        d[2 * q + 1] = pack_bf16x2(v2, v3);
      }
      // lane half 0 keeps units 0-3 and 16-19 and needs 4-7, 20-23 from half 1;
      // half 1 keeps 12-15 and 28-31 and needs 8-11, 24-27 from half 0
      uint32_t x[4];
#pragma unroll
      for (int e = 0; e < 2; ++e) {
        x[2 * e] = (uint32_t)__shfl_xor((int)(hh ? d[4 * e] : d[4 * e + 2]), 32);
        x[2 * e + 1] = (uint32_t)__shfl_xor((int)(hh ? d[4 * e + 1] : d[4 * e + 3]), 32);
      }
#pragma unroll
      for (int e = 0; e < 2; ++e)
        hop[2 * f + e] = hh ? make_uint4(x[2 * e], x[2 * e + 1], d[4 * e + 2], d[4 * e + 3])
                            : make_uint4(d[4 * e], d[4 * e + 1], x[2 * e], x[2 * e + 1]);
      for (int q = 0; q < 16; ++q) acc1[f][q] = 0.f;
    }
    // second product over the chunk's 8 k steps (W2 landed and was published by
    // the barriers of the chunk's later steps)
#pragma unroll
    for (int s2 = 0; s2 < 8; ++s2)
#pragma unroll
      for (int o = 0; o < 4; ++o) {
        const int r = 32 * o + r32, pos = (2 * s2 + hh) ^ (r & 15);
        const bf16x8_t wa = __builtin_bit_cast(bf16x8_t, *(const uint4*)&w2s[r * 128 + 8 * pos]);
        acc2[o] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(wa, __builtin_bit_cast(bf16x8_t, hop[s2]), acc2[o], 0, 0, 0);
      }
  }
  // epilogue through LDS as FP32, 32 rows x 128 outputs per wave: (acc + b2) + X
  __syncthreads();  // every wave is done with the ring and the W2 chunk
  float* stg = (float*)lds + wave * (32 * NO);
  auto at = [&](int r, int col) {
    const int byte = 4 * (r * NO + col), line = byte >> 7;
    return ((line << 7) | (((byte >> 4) & 7) ^ (line & 7)) << 4 | (byte & 15)) >> 2;
  };
#pragma unroll
  for (int o = 0; o < 4; ++o) {
    const int cl = 32 * o + 4 * hh;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const float4 bb = bias4(b2, 32 * o + 8 * q);
      *(float4*)&stg[at(r32, cl + 8 * q)] = make_float4(acc2[o][4 * q] + bb.x, acc2[o][4 * q + 1] + bb.y,
                                                         acc2[o][4 * q + 2] + bb.z, acc2[o][4 * q + 3] + bb.w);
    }
  }
  asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");  // the wave reads back only its own rows
#pragma unroll
  for (int t = 0; t < 16; ++t) {
    const int r = 2 * t + (lane >> 5), col = 4 * (lane & 31);
    const int64_t row = (int64_t)m0 + 32 * wave + r;
    const float4 u = *(const float4*)&stg[at(r, col)];
    if (row < M) {
      float4 x = *(const float4*)(X + row * NO + col);
      x.x = u.x + x.x;
      x.y = u.y + x.y;
      x.z = u.z + x.z;
      x.w = u.w + x.w;
      *(float4*)(X + row * NO + col) = x;
    }
  }
}

__global__ void k_zero_f32(float* p, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0.f;
}

// ------------------------------------------------------------------ LayerNorm
// Eight consecutive values of a row: loaded with two 16-byte loads when the
// address allows, stored as one 16-byte BF16 pack (or two FP32 float4).
__device__ inline void load8(const float* p, float (&v)[8]) {
  if (((uintptr_t)p & 15) == 0) {
    const float4 a = ((const float4*)p)[0], b = ((const float4*)p)[1];
    v[0] = a.x, v[1] = a.y, v[2] = a.z, v[3] = a.w, v[4] = b.x, v[5] = b.y, v[6] = b.z, v[7] = b.w;
  } else {
#pragma unroll
    for (int i = 0; i < 8; ++i) v[i] = p[i];
  }
}
template <typename AT>
__device__ inline void store8(AT* y, const float (&v)[8]) {
  if constexpr (sizeof(AT) == 2) {
    if (((uintptr_t)y & 15) == 0) {
      *(uint4*)y = make_uint4(pack_bf16x2(v[0], v[1]), pack_bf16x2(v[2], v[3]), pack_bf16x2(v[4], v[5]),
                              pack_bf16x2(v[6], v[7]));
      return;
    }
  } else {
    if (((uintptr_t)y & 15) == 0) {
      ((float4*)y)[0] = make_float4(v[0], v[1], v[2], v[3]);
      ((float4*)y)[1] = make_float4(v[4], v[5], v[6], v[7]);
      return;
    }
  }
#pragma unroll
  for (int i = 0; i < 8; ++i) y[i] = to_act<AT>(v[i]);
}

// LayerNorm of rows of C = 128 (eps 1e-5), FP32 in, activation type out.  A
// wave takes four rows, one per 16-lane DPP row: lane l holds columns
// 8 (l % 16) .. + 7 of row l / 16 (two 16-byte loads, one 16-byte BF16
// store), and the row statistics are 16-lane DPP sums.
template <typename AT>
__global__ __launch_bounds__(256) void k_layernorm128(const float* X, const float* g, const float* b, AT* Y, int M) {
  const int lane = threadIdx.x & 63, row0 = (blockIdx.x * 4 + (threadIdx.x >> 6)) * 4;
  if (row0 >= M) return;  // wave-uniform: the reductions below need every lane
  const int row = row0 + (lane >> 4), c0 = 8 * (lane & 15);
  const bool live = row < M;
  float x[8];
  if (live) load8(X + (int64_t)row * 128 + c0, x);
  else {
#pragma unroll
    for (int q = 0; q < 8; ++q) x[q] = 0.f;
  }
  float mu = 0.f;
#pragma unroll
  for (int q = 0; q < 8; ++q) mu += x[q];
  mu = row16_sum(mu) * (1.f / 128.f);
  float var = 0.f;
#pragma unroll
  for (int q = 0; q < 8; ++q) var += (x[q] - mu) * (x[q] - mu);
  const float rs = rsqrtf(row16_sum(var) * (1.f / 128.f) + 1e-5f);
  float gm[8], bt[8], y[8];
  load8(g + c0, gm);
  load8(b + c0, bt);
#pragma unroll
  for (int q = 0; q < 8; ++q) y[q] = (x[q] - mu) * rs * gm[q] + bt[q];
  if (live) store8<AT>(Y + (int64_t)row * 128 + c0, y);
}

// LayerNorm over the 4d concat [x | a | c | g] (Sec. 4.3: each token joins its
// row, column and global highway context before the FFN).  Segment s of row
// r is read from S_s + r * ld_s (s < 3) or from G + frame * 128; with has_ctx
// = 0 the three context segments are zero.  A wave takes four rows at once
// (lane l: segment l / 16, 8 features of each row).
template <typename AT>
__global__ __launch_bounds__(256) void k_ln_concat(const float* S0, int64_t ld0, const float* S1, int64_t ld1,
                                                   const float* S2, int64_t ld2, const float* G, const int* row2f,
                                                   const float* gam, const float* bet, AT* Y, int M, int has_ctx) {
  const int row0 = (blockIdx.x * 4 + (threadIdx.x >> 6)) * 4, lane = threadIdx.x & 63;
  if (row0 >= M) return;
  const int seg = lane >> 4, c0 = (lane & 15) * 8;
  float v[4][8];
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int row = min(row0 + r, M - 1);  // rows past M repeat the last row and are not stored
    const float* src = nullptr;
    if (seg == 0) src = S0 + (int64_t)row * ld0;
    else if (has_ctx) {
      if (seg == 1) src = S1 + (int64_t)row * ld1;
      else if (seg == 2) src = S2 + (int64_t)row * ld2;
      else src = G + (int64_t)row2f[row] * 128;
    }
    if (src) {
      load8(src + c0, v[r]);
    } else {
#pragma unroll
      for (int i = 0; i < 8; ++i) v[r][i] = 0.f;
    }
  }
  float mu[4], var[4];
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    mu[r] = 0.f;
#pragma unroll
    for (int i = 0; i < 8; ++i) mu[r] += v[r][i];
  }
  wave_sum4(mu);
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    mu[r] *= (1.f / 512.f);
    var[r] = 0.f;
#pragma unroll
    for (int i = 0; i < 8; ++i) var[r] += (v[r][i] - mu[r]) * (v[r][i] - mu[r]);
  }
  wave_sum4(var);
  const int gc = seg * 128 + c0;
  float gm[8], bt[8];
  load8(gam + gc, gm);
  load8(bet + gc, bt);
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    if (row0 + r >= M) break;
    const float rs = rsqrtf(var[r] * (1.f / 512.f) + 1e-5f);
    float o[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) o[i] = (v[r][i] - mu[r]) * rs * gm[i] + bt[i];
    store8<AT>(Y + (int64_t)(row0 + r) * 512 + gc, o);
  }
}

// ------------------------------------------------------------------ features
// Per-frame summary (one block per frame), the definition used here of
// the 12 global features: log2(N)/16, log(rho_max/rho_min), mean and std of
// log rho, heavy fraction, mean/std/min/max of log A_ii, nx/32, ny/32, nz/32.
__global__ __launch_bounds__(1024) void k_frame_stats(const FrameDesc* fr, const float* rho, const float* sys,
                                                     int64_t ntot, float* glob) {
  constexpr int NW = 16;   // waves of the 1024-thread block
  constexpr int CAP = 16;  // nodes per thread whose logs stay in registers (frames up to 16384 nodes)
  __shared__ double red[NW][6];
  const FrameDesc F = fr[blockIdx.x];
  const double* dg8 = reinterpret_cast<const double*>(sys + 5 * ntot);
  const int t = threadIdx.x, w = t >> 6, lane = t & 63;
  // K wave reductions at once (sum, or min / max by op), then the waves'
  // results in wave order: one pair of barriers per batch of statistics
  auto reduce = [&](double (&v)[6], const int (&op)[6], int K) {
#pragma unroll
    for (int i = 0; i < 6; ++i) {
      if (i >= K) break;
      double x = v[i];
      auto comb = [&](double a, double b) { return op[i] == 0 ? a + b : op[i] < 0 ? fmin(a, b) : fmax(a, b); };
      x = comb(x, dpp_move_d<0xB1>(x));
      x = comb(x, dpp_move_d<0x4E>(x));
      x = comb(x, dpp_move_d<0x141>(x));
      x = comb(x, dpp_move_d<0x140>(x));
      // row broadcasts: the rows outside the mask keep their own value
      {
        const unsigned long long u = __builtin_bit_cast(unsigned long long, x);
        const unsigned lo = (unsigned)__builtin_amdgcn_update_dpp((int)(unsigned)u, (int)(unsigned)u, 0x142, 0xA, 0xF, false);
        const unsigned hi = (unsigned)__builtin_amdgcn_update_dpp((int)(unsigned)(u >> 32), (int)(unsigned)(u >> 32), 0x142, 0xA, 0xF, false);
        const double y = __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
        x = (lane >> 4) & 1 ? comb(x, y) : x;
      }
      {
        const unsigned long long u = __builtin_bit_cast(unsigned long long, x);
        const unsigned lo = (unsigned)__builtin_amdgcn_update_dpp((int)(unsigned)u, (int)(unsigned)u, 0x143, 0xC, 0xF, false);
        const unsigned hi = (unsigned)__builtin_amdgcn_update_dpp((int)(unsigned)(u >> 32), (int)(unsigned)(u >> 32), 0x143, 0xC, 0xF, false);
        const double y = __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
        x = (lane >> 5) & 1 ? comb(x, y) : x;
      }
      v[i] = x;  // lane 63 holds the wave's result
    }
    __syncthreads();
    if (lane == 63)
      for (int i = 0; i < K; ++i) red[w][i] = v[i];
    __syncthreads();
    for (int i = 0; i < K; ++i) {
      double r = red[0][i];
      for (int q = 1; q < NW; ++q) r = op[i] == 0 ? r + red[q][i] : op[i] < 0 ? fmin(r, red[q][i]) : fmax(r, red[q][i]);
      v[i] = r;
    }
  };
  double lrv[CAP], lav[CAP];
  const bool cached = F.n <= 1024 * CAP;
  double a1[6] = {0, 0, 1e300, -1e300, 1e300, -1e300};
#pragma unroll
  for (int u = 0; u < CAP; ++u) {
    const int c = t + 1024 * u;
    if (c < F.n) {
      lrv[u] = log((double)rho[F.n0 + c]);
      lav[u] = log(dg8[F.n0 + c]);
      a1[0] += lrv[u];
      a1[1] += lav[u];
      a1[2] = fmin(a1[2], lrv[u]);
      a1[3] = fmax(a1[3], lrv[u]);
      a1[4] = fmin(a1[4], lav[u]);
      a1[5] = fmax(a1[5], lav[u]);
    }
  }
  for (int c = t + 1024 * CAP; c < F.n; c += 1024) {  // frames beyond the register cache
    const double lr = log((double)rho[F.n0 + c]), la = log(dg8[F.n0 + c]);
    a1[0] += lr;
    a1[1] += la;
    a1[2] = fmin(a1[2], lr);
    a1[3] = fmax(a1[3], lr);
    a1[4] = fmin(a1[4], la);
    a1[5] = fmax(a1[5], la);
  }
  reduce(a1, {0, 0, -1, 1, -1, 1}, 6);
  const double n = F.n;
  const double mr = a1[0] / n, ma = a1[1] / n;
  const double lmin = a1[2], lmax = a1[3], amin = a1[4], amax = a1[5];
  const double mid = 0.5 * (lmin + lmax);
  double a2[6] = {0, 0, 0, 0, 0, 0};
  auto second = [&](double lr, double la) {
    a2[0] += (lr - mr) * (lr - mr);
    a2[1] += (la - ma) * (la - ma);
    a2[2] += lr > mid ? 1.0 : 0.0;
  };
  if (cached) {
#pragma unroll
    for (int u = 0; u < CAP; ++u)
      if (t + 1024 * u < F.n) second(lrv[u], lav[u]);
  } else {
    for (int c = t; c < F.n; c += 1024) second(log((double)rho[F.n0 + c]), log(dg8[F.n0 + c]));
  }
  reduce(a2, {0, 0, 0, 0, 0, 0}, 3);
  const double sdr = sqrt(a2[0] / n), sda = sqrt(a2[1] / n), heavy = lmax > lmin ? a2[2] / n : 0.0;
  if (t == 0) {
    float* g = glob + blockIdx.x * 12;
    g[0] = (float)(log2(n) / 16.0);
    g[1] = (float)(lmax - lmin);
    g[2] = (float)mr;
    g[3] = (float)sdr;
    g[4] = (float)heavy;
    g[5] = (float)ma;
    g[6] = (float)sda;
    g[7] = (float)amin;
    g[8] = (float)amax;
    g[9] = F.nx / 32.f;
    g[10] = F.ny / 32.f;
    g[11] = F.nz / 32.f;
  }
}

// Node features (8) + the frame summary (12), zero padded to 32 columns.
template <typename AT>
__global__ void k_features(const FrameDesc* fr, const int* blk2f, const float* rho, const float* sys, int64_t ntot,
                           const float* glob, AT* out) {
  const int f = blk2f[blockIdx.x];
  const FrameDesc F = fr[f];
  const int c = (blockIdx.x - F.b0) * NODE_BLOCK + threadIdx.x;
  if (c >= F.n) return;
  const int64_t i = F.n0 + c;
  const double* dg8 = reinterpret_cast<const double*>(sys + 5 * ntot);
  const int x = mcoord(c, F.xm), y = mcoord(c, F.ym), z = mcoord(c, F.zm);
  float v[32];
  v[0] = (float)log((double)rho[i]);
  v[1] = (x + 0.5f) / F.nx;
  v[2] = (y + 0.5f) / F.ny;
  v[3] = (z + 0.5f) / F.nz;
  v[4] = z == F.nz - 1 ? 1.f : 0.f;
  v[5] = (x == 0 || x == F.nx - 1 || y == 0 || y == F.ny - 1) ? 1.f : 0.f;
  v[6] = z == 0 ? 1.f : 0.f;
  v[7] = (float)log(dg8[i]);
  for (int j = 0; j < 12; ++j) v[8 + j] = glob[f * 12 + j];
  for (int j = 20; j < 32; ++j) v[j] = 0.f;
  for (int j = 0; j < 32; ++j) out[i * 32 + j] = to_act<AT>(v[j]);
}

// ------------------------------------------------------------------ encoder GCN
// Y = D^-1 A H: y_i = h_i - sum_j (w_ij / A_ii) h_j over the 6 faces.
// Eight rows per block of 256 threads, 32 threads a row with four features
// each (16-byte loads of the seven rows involved).
template <typename AT>
__global__ __launch_bounds__(256) void k_gcn_spmm(const FrameDesc* fr, const int* node2f, const float* sys,
                                                  int64_t ntot, const float* H, AT* Y) {
  const int64_t i = (int64_t)xcd_block(blockIdx.x, gridDim.x) * 8 + (threadIdx.x >> 5);
  if (i >= ntot) return;
  const int col = (threadIdx.x & 31) * 4;
  const FrameDesc F = fr[node2f[i]];
  const unsigned c = (unsigned)(i - F.n0);
  const float *dg = sys, *wx = sys + ntot, *wy = sys + 2 * ntot, *wz = sys + 3 * ntot;
  const float id = 1.f / dg[i];
  const int64_t nb[6] = {F.n0 + mstep_plus(c, F.xm), F.n0 + mstep_minus(c, F.xm), F.n0 + mstep_plus(c, F.ym),
                         F.n0 + mstep_minus(c, F.ym), F.n0 + mstep_plus(c, F.zm), F.n0 + mstep_minus(c, F.zm)};
  const float wv[6] = {wx[i], wx[nb[1]], wy[i], wy[nb[3]], wz[i], wz[nb[5]]};
  float4 hv[6];
#pragma unroll
  for (int q = 0; q < 6; ++q) hv[q] = *(const float4*)(H + nb[q] * 128 + col);
  const float4 hi = *(const float4*)(H + i * 128 + col);
  float y[4];
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    auto comp = [&](const float4& t) { return e == 0 ? t.x : e == 1 ? t.y : e == 2 ? t.z : t.w; };
    float sum = wv[0] * comp(hv[0]);
#pragma unroll
    for (int q = 1; q < 6; ++q) sum = fmaf(wv[q], comp(hv[q]), sum);
    y[e] = comp(hi) - sum * id;
  }
  if constexpr (sizeof(AT) == 2)
    *(uint2*)(Y + i * 128 + col) = make_uint2(pack_bf16x2(y[0], y[1]), pack_bf16x2(y[2], y[3]));
  else
    *(float4*)(Y + i * 128 + col) = make_float4(y[0], y[1], y[2], y[3]);
}

// ------------------------------------------------------------------ edge-bias MLPs
// MLP_e(e) = GELU(e W1 + b1) W2 + b2, e in R^4 (Sec. 4.2, Supplementary:
// per-head bias from the edge descriptor (dx, A_ij)); W1 [4][E], W2 [E][H].
struct EdgeW {
  const float *w1, *b1, *w2, *b2;
  int E, H;
};
// The edge MLPs of up to EDGE_LAYERS layers, layer blockIdx.y of a launch:
// the inference computes every layer's tables in one launch per kernel, each
// layer into its own buffer (outputs advance by a per-layer stride).
constexpr int EDGE_LAYERS = 8;
struct EdgeWs {
  EdgeW w[EDGE_LAYERS];
};

// The edge MLP's parameters [W1 (4E) | b1 (E) | W2 (E H) | b2 (H)] are
// contiguous in the weight vector; each block stages them in LDS once.
constexpr int EDGE_MAX_FLOATS = 5 * 64 + 64 * 8 + 8;

__device__ inline void edge_stage(const EdgeW& w, float* sw) {
  const int n = 5 * w.E + w.E * w.H + w.H;
  for (int q = threadIdx.x; q < n; q += blockDim.x) sw[q] = w.w1[q];
  __syncthreads();
}

// MLP_e(e) from the staged parameters; out[h] for h < H (8 slots).  The
// hidden units are folded into the output sums one at a time (no hidden
// array), in the same order as a hidden-then-output evaluation.
template <bool FAST>
__device__ inline float edge_gelu(float x) {
  if constexpr (FAST) return gelu_bf16path(x);
  else return gelu_f(x);
}

// FAST: the BF16 path's GELU (the MLP's outputs are attention biases added to
// logits of BF16 queries and keys); otherwise the library erff.
// HK, EK > 0 fix H and E at compile time (the per-head loop then has exactly
// H multiply-adds); 0 takes them from the arguments.
template <bool FAST, int HK = 0, int EK = 0>
__device__ inline void edge_mlp(const float* sw, int E_, int H_, const float e[4], float out[8]) {
  const int E = EK ? EK : E_, H = HK ? HK : H_;
  const float *w1 = sw, *b1 = sw + 4 * E, *w2 = sw + 5 * E, *b2 = sw + 5 * E + E * H;
#pragma unroll
  for (int h = 0; h < 8; ++h) out[h] = h < H ? b2[h] : 0.f;
#pragma unroll(EK ? 4 : 1)
  for (int k = 0; k < E; ++k) {
    float s = b1[k];
#pragma unroll
    for (int q = 0; q < 4; ++q) s = fmaf(e[q], w1[q * E + k], s);
    const float g = edge_gelu<FAST>(s);
#pragma unroll
    for (int h = 0; h < 8; ++h)
      if (h < H) out[h] = fmaf(g, w2[k * H + h], out[h]);
  }
}

// Stencil-slot constants of one layer's edge MLP, computed by one block: the
// first layer's partial sums b1 + dx_e W1[0..2] (cst[e][k], row stride 65)
// and MLP_e(dx_e, 0) (base[e][h]), for the 7 slots e.
constexpr int EDGE_CST = 7 * 65 + 7 * 8;

template <bool FAST>
__device__ inline void edge_slot_consts(const float* sw, int E, int H, float* out) {
  const float *w1 = sw, *b1 = sw + 4 * E;
  auto slot_dx = [](int e, float (&d)[3]) {
    d[0] = d[1] = d[2] = 0.f;
    if (e > 0) d[(e - 1) / 2] = ((e - 1) % 2 == 0) ? 0.25f : -0.25f;
  };
  for (int q = threadIdx.x; q < 7 * E; q += blockDim.x) {
    const int e = q / E, k = q % E;
    float d[3];
    slot_dx(e, d);
    float sv = b1[k];
#pragma unroll
    for (int c = 0; c < 3; ++c) sv = fmaf(d[c], w1[c * E + k], sv);
    out[e * 65 + k] = sv;
  }
  if (threadIdx.x < 7) {
    const int e = threadIdx.x;
    float d[3], o[8];
    slot_dx(e, d);
    const float e0[4] = {d[0], d[1], d[2], 0.f};
    edge_mlp<FAST>(sw, E, H, e0, o);
    for (int h = 0; h < 8; ++h) out[7 * 65 + e * 8 + h] = h < H ? o[h] : 0.f;
  }
}

// Within-leaf bias table with A_ij = 0: T0[h][i][j] = MLP_e((pos j - pos i)/4, 0).
// Every leaf has the same shape, so one table per layer serves all leaves.
// The block after the table's blocks writes the stencil-slot constants.
// Block bx of nbx (the last one writes the slot constants) of one layer.
template <bool FAST>
__device__ inline void edge_table_block(const EdgeW& w, int bx, int nbx, int L, unsigned xm, unsigned ym, unsigned zm,
                                        float* T0, float* slots) {
  __shared__ float sw[EDGE_MAX_FLOATS];
  edge_stage(w, sw);
  if (bx == nbx - 1) {
    edge_slot_consts<FAST>(sw, w.E, w.H, slots);
    return;
  }
  const int p = bx * blockDim.x + threadIdx.x;
  if (p >= L * L) return;
  const int i = p / L, j = p % L;
  float e[4] = {(mcoord(j, xm) - mcoord(i, xm)) * 0.25f, (mcoord(j, ym) - mcoord(i, ym)) * 0.25f,
                (mcoord(j, zm) - mcoord(i, zm)) * 0.25f, 0.f};
  float o[8];
  edge_mlp<FAST>(sw, w.E, w.H, e, o);
  for (int h = 0; h < w.H; ++h) T0[(h * L + i) * L + j] = o[h];
}

template <bool FAST>
__global__ __launch_bounds__(256) void k_edge_table(EdgeWs ws, int L, unsigned xm, unsigned ym, unsigned zm, float* T0,
                                                    float* slots, int64_t t0_stride, int slot_stride) {
  edge_table_block<FAST>(ws.w[blockIdx.y], blockIdx.x, gridDim.x, L, xm, ym, zm, T0 + blockIdx.y * t0_stride,
                         slots + blockIdx.y * slot_stride);
}

// Stencil entries of node i inside its own leaf (self and up to 6 faces):
// nbr[i][e] = local index of j in the leaf (255: none), ahat[i][e] =
// A_ij / sqrt(A_ii A_jj), delta code in dir[i][e] (0 self, 1..6 = +x,-x,+y,-y,+z,-z).
__device__ inline void leaf_stencil_node(int64_t i, const FrameDesc* fr, const int* node2f, const float* sys,
                                         int64_t ntot, int L, uint8_t* nbr, float* ahat) {
  if (i >= ntot) return;
  const FrameDesc F = fr[node2f[i]];
  const unsigned c = (unsigned)(i - F.n0);
  const double* d8 = reinterpret_cast<const double*>(sys + 5 * ntot);
  const double *wx8 = d8 + ntot, *wy8 = d8 + 2 * ntot, *wz8 = d8 + 3 * ntot;
  const unsigned leaf = c / (unsigned)L;
  nbr[i * 7] = (uint8_t)(c % L);
  ahat[i * 7] = 1.f;
  const unsigned masks[3] = {F.xm, F.ym, F.zm};
  const double* ws[3] = {wx8, wy8, wz8};
  for (int a = 0; a < 3; ++a) {
    for (int sgn = 0; sgn < 2; ++sgn) {
      const int e = 1 + 2 * a + sgn;
      const bool edge = sgn == 0 ? (c & masks[a]) == masks[a] : (c & masks[a]) == 0;
      const unsigned cj = sgn == 0 ? mstep_plus(c, masks[a]) : mstep_minus(c, masks[a]);
      nbr[i * 7 + e] = 255;
      ahat[i * 7 + e] = 0.f;
      if (edge || cj / (unsigned)L != leaf) continue;
      const double w = sgn == 0 ? ws[a][i] : ws[a][F.n0 + cj];
      nbr[i * 7 + e] = (uint8_t)(cj % L);
      ahat[i * 7 + e] = (float)(-w / sqrt(d8[i] * d8[F.n0 + cj]));
    }
  }
}

__global__ void k_leaf_stencil(const FrameDesc* fr, const int* node2f, const float* sys, int64_t ntot, int L,
                               uint8_t* nbr, float* ahat) {
  leaf_stencil_node((int64_t)blockIdx.x * blockDim.x + threadIdx.x, fr, node2f, sys, ntot, L, nbr, ahat);
}

// Per-layer corrections of the diagonal bias at the stencil entries:
// corr[i][e][h] = MLP_e(dx_ij/4, Ahat_ij) - MLP_e(dx_ij/4, 0).
// Stencil corrections MLP_e(dx_e, Ahat) - MLP_e(dx_e, 0) of every (node,
// slot) pair, the same operations as edge_mlp with the first three input
// terms taken from the slot constants; grid-stride over pairs.
template <bool FAST, int HK = 0, int EK = 0>
__global__ __launch_bounds__(256) void k_edge_corr(EdgeWs ws, const float* slots, const uint8_t* nbr, const float* ahat,
                                                   int64_t ntot, float* corr, int slot_stride, int64_t corr_stride) {
  __shared__ float cst[EDGE_CST];
  __shared__ float sw[EDGE_MAX_FLOATS];
  const EdgeW w = ws.w[blockIdx.y];
  slots += blockIdx.y * slot_stride;
  corr += blockIdx.y * corr_stride;
  for (int q = threadIdx.x; q < EDGE_CST; q += blockDim.x) cst[q] = slots[q];
  edge_stage(w, sw);  // ends with a barrier
  const int E = EK ? EK : w.E, H = HK ? HK : w.H;
  const float *w1 = sw, *w2 = sw + 5 * E, *b2 = sw + 5 * E + E * H;
  const float* base = cst + 7 * 65;
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < ntot * 7;
       p += (int64_t)gridDim.x * blockDim.x) {
    const int e = (int)(p % 7);
    float* o = corr + p * H;
    if (nbr[p] == 255) {
      for (int h = 0; h < H; ++h) o[h] = 0.f;
      continue;
    }
    const float a = ahat[p];
    float out[8];
#pragma unroll
    for (int h = 0; h < 8; ++h) out[h] = h < H ? b2[h] : 0.f;
#pragma unroll(EK ? 4 : 1)
    for (int k = 0; k < E; ++k) {
      const float g = edge_gelu<FAST>(fmaf(a, w1[3 * E + k], cst[e * 65 + k]));
#pragma unroll
      for (int h = 0; h < 8; ++h)
        if (h < H) out[h] = fmaf(g, w2[k * H + h], out[h]);
    }
#pragma unroll
    for (int h = 0; h < 8; ++h)
      if (h < H) o[h] = out[h] - base[e * 8 + h];
  }
}

// Off-diagonal pair descriptors (Supplementary "Off-diagonal attention
// stack"): for tile m, row token t, column token t':
//   (centroid(J_m^t') - centroid(I_m^t)) / 4,  mean of Ahat over I_m^t x J_m^t'.
// The strip pairs of a tile are split into chunks of at most DESC_CHUNK
// leaves a side (a big tile's serial loop would otherwise dominate): one
// block per chunk, FP64 partial sums per chunk (the Ahat sum of every token
// pair, the coordinate sums of every row and column token); a second kernel
// adds a tile's chunks in order.  Within a block,
// one thread per row-strip node first finds its stencil entries that land
// in the column strip (the group t' of each and its Ahat, once per entry);
// thread (t, t') then adds those of group t whose target is in group t', in
// the order node, axis, direction.
constexpr int DESC_CHUNK = 4;
constexpr int DESC_MAX_LEAF = 64;  // leaf sizes 32 and 64
struct DescChunk {
  int tile;   // global tile index
  int k0, k1; // leaf range [k0, k1) inside the strips
};

__device__ inline void off_desc_chunk(int bx, const FrameDesc* fr, const int* tile2f, const DescChunk* ch,
                                      const float* sys, int64_t ntot, int L, int LS, double* part) {
  __shared__ double sval[DESC_CHUNK * DESC_MAX_LEAF][6];
  __shared__ __align__(8) uint8_t sgrp[DESC_CHUNK * DESC_MAX_LEAF][8];  // 6 used: one 8-byte read a node
  __shared__ int scrd[2][DESC_CHUNK][DESC_MAX_LEAF / 4][3];  // token coordinate sums: row, column strip
  const DescChunk c = ch[bx];
  const FrameDesc F = fr[tile2f[c.tile]];
  const int m = c.tile - F.m0, K = F.K;
  int j = 0;
  while (m >= K - (K >> (j + 1))) ++j;
  const int i = m - (K - (K >> j)), S = 1 << j, r0 = 2 * i * S, c0 = r0 + S, p = L / LS;
  const double* d8 = reinterpret_cast<const double*>(sys + 5 * ntot);
  const double* w8[3] = {d8 + ntot, d8 + 2 * ntot, d8 + 3 * ntot};
  const unsigned masks[3] = {F.xm, F.ym, F.zm};
  const int nn = (c.k1 - c.k0) * L;  // row-strip nodes of the chunk (at most DESC_CHUNK * DESC_MAX_LEAF)
  for (int n = threadIdx.x; n < nn; n += blockDim.x) {
    const unsigned ci = (unsigned)((r0 + c.k0) * L + n);
    for (int a = 0; a < 3; ++a) {
      for (int sgn = 0; sgn < 2; ++sgn) {
        const int e = 2 * a + sgn;
        uint8_t g = 255;  // none
        double v = 0.0;
        const bool edge = sgn == 0 ? (ci & masks[a]) == masks[a] : (ci & masks[a]) == 0;
        if (!edge) {
          const unsigned cj = sgn == 0 ? mstep_plus(ci, masks[a]) : mstep_minus(ci, masks[a]);
          const int kj = cj / L;
          if (kj >= c0 && kj < c0 + S) {
            const double w = sgn == 0 ? w8[a][F.n0 + ci] : w8[a][F.n0 + cj];
            g = (uint8_t)((cj % L) / p);
            v = -w / sqrt(d8[F.n0 + ci] * d8[F.n0 + cj]);
          }
        }
        sgrp[n][e] = g;
        sval[n][e] = v;
      }
    }
  }
  // Coordinate sums of every token of the chunk, once per (strip, leaf,
  // token, axis).  A token's p cells are consecutive and its first is a
  // multiple of p, so they are first | i (i < p), and the sum over them is
  // p mcoord(first) + the sum of mcoord(i) (only the mask's bits below p
  // matter there).  The sums are integers: exact in FP64 in any order.
  const int nk = c.k1 - c.k0;
  for (int q = threadIdx.x; q < 2 * nk * LS * 3; q += blockDim.x) {
    const int a = q % 3, tok = (q / 3) % LS, kk = (q / (3 * LS)) % nk, side = q / (3 * LS * nk);
    const unsigned first = (unsigned)(((side ? c0 : r0) + c.k0 + kk) * L + tok * p);
    const unsigned lm = masks[a] & (unsigned)(p - 1);
    int lo = 0;
    for (int u = 0; u < p; ++u) lo += mcoord((unsigned)u, lm);
    scrd[side][kk][tok][a] = p * mcoord(first, masks[a]) + lo;
  }
  __syncthreads();
  const int t = threadIdx.x / LS, t2 = threadIdx.x % LS;
  if (t >= LS) return;
  double cI[3] = {0, 0, 0}, cJ[3] = {0, 0, 0}, acc = 0.0;
  for (int k = c.k0; k < c.k1; ++k) {
    const int kk = k - c.k0;
    for (int a = 0; a < 3; ++a) {
      cI[a] += (double)scrd[0][kk][t][a];
      cJ[a] += (double)scrd[1][kk][t2][a];
    }
    for (int l = t * p; l < (t + 1) * p; ++l) {
      const int n = (k - c.k0) * L + l;
      const uint2 gw = *reinterpret_cast<const uint2*>(&sgrp[n][0]);
#pragma unroll
      for (int e = 0; e < 6; ++e)
        if ((((e < 4 ? gw.x : gw.y) >> (8 * (e & 3))) & 0xffu) == (unsigned)t2) acc += sval[n][e];
    }
  }
  // chunk record: [Ahat sums, LS x LS | row-token coordinate sums, LS x 3 |
  // column-token coordinate sums, LS x 3] (a row token's sums do not depend on
  // t', nor a column token's on t)
  double* o = part + (int64_t)bx * (LS * LS + 6 * LS);
  o[t * LS + t2] = acc;
  if (t2 == 0)
    for (int a = 0; a < 3; ++a) o[LS * LS + t * 3 + a] = cI[a];
  if (t == 0)
    for (int a = 0; a < 3; ++a) o[LS * LS + 3 * LS + t2 * 3 + a] = cJ[a];
}

__global__ __launch_bounds__(256) void k_off_desc_part(const FrameDesc* fr, const int* tile2f, const DescChunk* ch,
                                                       const float* sys, int64_t ntot, int L, int LS, double* part) {
  off_desc_chunk(blockIdx.x, fr, tile2f, ch, sys, ntot, L, LS, part);
}

// The head of the inference's side chain in one launch, three independent
// parts as block ranges: [0, nd) descriptor chunks (k_off_desc_part), the
// next ns blocks the leaf stencils (k_leaf_stencil), then nl layers of nt
// blocks of edge tables (k_edge_table).  One launch instead of three keeps
// the chain that runs ahead of the encoder short.
template <bool FAST>
__global__ __launch_bounds__(256) void k_side_head(const FrameDesc* fr, const int* tile2f, const DescChunk* ch,
                                                   const float* sys, int64_t ntot, int L, int LS, double* part, int nd,
                                                   const int* node2f, uint8_t* nbr, float* ahat, int ns, EdgeWs ws,
                                                   unsigned xm, unsigned ym, unsigned zm, float* T0, float* slots,
                                                   int64_t t0_stride, int slot_stride, int nt) {
  int bx = blockIdx.x;
  if (bx < nd) {
    off_desc_chunk(bx, fr, tile2f, ch, sys, ntot, L, LS, part);
    return;
  }
  bx -= nd;
  if (bx < ns) {
    leaf_stencil_node((int64_t)bx * blockDim.x + threadIdx.x, fr, node2f, sys, ntot, L, nbr, ahat);
    return;
  }
  bx -= ns;
  const int l = bx / nt;
  bx -= l * nt;
  edge_table_block<FAST>(ws.w[l], bx, nt, L, xm, ym, zm, T0 + l * t0_stride, slots + l * slot_stride);
}

// desc of tile (block) mg from its chunks [chunk0[mg], chunk0[mg + 1]).
__global__ __launch_bounds__(256) void k_off_desc_final(const FrameDesc* fr, const int* tile2f, const int* chunk0,
                                                        const double* part, int L, int LS, float* desc) {
  const int mg = blockIdx.x;
  const FrameDesc F = fr[tile2f[mg]];
  const int m = mg - F.m0, K = F.K;
  int j = 0;
  while (m >= K - (K >> (j + 1))) ++j;
  const int S = 1 << j, p = L / LS;
  const int t = threadIdx.x / LS, t2 = threadIdx.x % LS;
  if (t >= LS) return;
  double v[7] = {0, 0, 0, 0, 0, 0, 0};
  for (int c = chunk0[mg]; c < chunk0[mg + 1]; ++c) {
    const double* o = part + (int64_t)c * (LS * LS + 6 * LS);
    for (int a = 0; a < 3; ++a) {
      v[a] += o[LS * LS + t * 3 + a];
      v[3 + a] += o[LS * LS + 3 * LS + t2 * 3 + a];
    }
    v[6] += o[t * LS + t2];
  }
  const double inv = 1.0 / (double)(S * p);
  float* out = desc + (((int64_t)mg * LS + t) * LS + t2) * 4;
  for (int a = 0; a < 3; ++a) out[a] = (float)((v[3 + a] - v[a]) * inv * 0.25);
  out[3] = (float)(v[6] * inv * inv);
}

// Off-diagonal bias per layer: bias[m][h][t][t'] = MLP_e(desc[m][t][t']).
template <bool FAST, int HK = 0, int EK = 0>
__global__ __launch_bounds__(256) void k_edge_off(EdgeWs ws, const float* desc, int64_t npairs, int LS, float* bias,
                                                  int64_t bias_stride) {
  __shared__ float sw[EDGE_MAX_FLOATS];
  const EdgeW w = ws.w[blockIdx.y];
  bias += blockIdx.y * bias_stride;
  edge_stage(w, sw);
  const int H = HK ? HK : w.H;
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < npairs; p += (int64_t)gridDim.x * blockDim.x) {
    const int64_t m = p / (LS * LS);
    const int tt = (int)(p % (LS * LS));
    const float4 dv = *(const float4*)(desc + p * 4);
    const float e[4] = {dv.x, dv.y, dv.z, dv.w};
    float o[8];
    edge_mlp<FAST, HK, EK>(sw, w.E, w.H, e, o);
#pragma unroll
    for (int h = 0; h < 8; ++h)
      if (h < H) bias[(m * H + h) * LS * LS + tt] = o[h];
  }
}

// ------------------------------------------------------------------ attention
// One wave per (group, head): T tokens (a leaf, T = L, or a tile, T = L_s),
// head dim 32.  S = Q K^T / sqrt(32) + bias, softmax over keys, O = P V.
// Diagonal groups read the shared table T0[h] plus the stencil corrections
// of their own row; tiles read a dense per-tile bias.
template <typename AT, int T, bool DIAG>
__global__ __launch_bounds__(64) void k_attention(const AT* qkv, AT* out, const float* bias, const float* corr,
                                                  const uint8_t* nbr, int H) {
  constexpr int DH = 32;
  __shared__ float sK[T][DH + 1], sV[T][DH + 1], sB[T][T + 1];
  const int grp = blockIdx.x, h = blockIdx.y, lane = threadIdx.x;
  const int d = H * DH;
  const int64_t row0 = (int64_t)grp * T;
  for (int idx = lane; idx < T * DH; idx += 64) {
    const int r = idx / DH, c = idx % DH;
    const AT* q = qkv + (row0 + r) * 3 * d + h * DH + c;
    sK[r][c] = ldf(q, d);
    sV[r][c] = ldf(q, 2 * d);
  }
  const float* bt = DIAG ? bias + (int64_t)h * T * T : bias + ((int64_t)grp * H + h) * T * T;
  for (int idx = lane; idx < T * T; idx += 64) sB[idx / T][idx % T] = bt[idx];
  __syncthreads();
  if (lane >= T) return;
  const int64_t row = row0 + lane;
  if (DIAG) {
    for (int e = 0; e < 7; ++e) {
      const int lj = nbr[row * 7 + e];
      if (lj != 255) sB[lane][lj] += corr[(row * 7 + e) * H + h];
    }
  }
  float q[DH];
  const float scale = 0.17677669529663687f;  // 1/sqrt(32)
#pragma unroll
  for (int c = 0; c < DH; ++c) q[c] = ldf(qkv, row * 3 * d + h * DH + c) * scale;
  float s[T];
  float mx = -3.4e38f;
#pragma unroll
  for (int j = 0; j < T; ++j) {
    float a = sB[lane][j];
#pragma unroll
    for (int c = 0; c < DH; ++c) a = fmaf(q[c], sK[j][c], a);
    s[j] = a;
    mx = fmaxf(mx, a);
  }
  float sum = 0.f;
#pragma unroll
  for (int j = 0; j < T; ++j) {
    s[j] = expf(s[j] - mx);
    sum += s[j];
  }
  const float inv = 1.f / sum;
  float o[DH];
#pragma unroll
  for (int c = 0; c < DH; ++c) o[c] = 0.f;
#pragma unroll
  for (int j = 0; j < T; ++j) {
#pragma unroll
    for (int c = 0; c < DH; ++c) o[c] = fmaf(s[j], sV[j][c], o[c]);
  }
#pragma unroll
  for (int c = 0; c < DH; ++c) out[row * d + h * DH + c] = to_act<AT>(o[c] * inv);
}

// Within-leaf attention on the matrix cores (BF16 operands, FP32
// accumulation): one wave per (leaf, head), the four heads of a leaf in one
// block.  The wave forms S^T = K Q^T (keys as rows, queries as columns, so a
// lane owns one query and half of its keys), adds scale and bias, takes the
// softmax with one cross-lane step (lane l and l ^ 32 share a query), and
// forms O^T = V^T P^T.  The key order inside each 16-wide MFMA step is
// permuted so that the B operand of the second product is exactly the P
// values a lane already holds: step (a, s), slot e of half hh is key
// 32a + 16s + 8(e/4) + 4hh + e%4, and V^T is read from LDS in that order.
template <int T>
__global__ __launch_bounds__(256) void k_attention_mfma(const uint16_t* qkv, uint16_t* out, const float* T0,
                                                       const float* corr, const uint8_t* nbr) {
  constexpr int DH = 32, H = 4, D = H * DH, NT = T / 32, VP = T + 8;
  __shared__ __attribute__((aligned(16))) uint16_t sVt[H][DH][VP];
  // stencil corrections of the current query tile as a dense row per query
  __shared__ __attribute__((aligned(16))) float sC[H][32][T + 4];
  const int h = threadIdx.x >> 6, lane = threadIdx.x & 63, hh = lane >> 5, c32 = lane & 31;
  const int64_t row0 = (int64_t)blockIdx.x * T;
  const uint16_t* base = qkv + row0 * 3 * D + h * DH;
  // Each LDS region (sVt[h], sC[h]) is written and read by the wave of head
  // h only, and one wave's LDS accesses complete in order: the waves never
  // wait for each other, a wait for the wave's own LDS operations and a
  // compiler fence stand in for block barriers.
  auto wave_lds_fence = [] { asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory"); };
  // the block's global operands are requested together: V rows (key ->
  // 16-byte chunks) and the K operands of both key tiles and both 16-wide
  // steps, which stay in registers
  constexpr int NV = T * 4 / 64;
  uint4 vch[NV];
#pragma unroll
  for (int u = 0; u < NV; ++u) {
    const int idx = lane + 64 * u, key = idx >> 2, c0 = (idx & 3) * 8;
    vch[u] = *(const uint4*)(base + (int64_t)key * 3 * D + 2 * D + c0);
  }
  bf16x8_t kop[2][NT];
#pragma unroll
  for (int s = 0; s < 2; ++s)
#pragma unroll
    for (int t = 0; t < NT; ++t)
      kop[s][t] = __builtin_bit_cast(bf16x8_t,
                                     *(const uint4*)(base + (int64_t)(32 * t + c32) * 3 * D + D + 16 * s + 8 * hh));
  // V^T into LDS
#pragma unroll
  for (int u = 0; u < NV; ++u) {
    const int idx = lane + 64 * u, key = idx >> 2, c0 = (idx & 3) * 8;
    const uint16_t* pv = (const uint16_t*)&vch[u];
#pragma unroll
    for (int e = 0; e < 8; ++e) sVt[h][c0 + e][key] = pv[e];
  }
  wave_lds_fence();
  const float scale = 0.17677669529663687f;  // 1/sqrt(32)
#pragma unroll 1
  for (int b = 0; b < NT; ++b) {
    const int q = 32 * b + c32;
    const int64_t row = row0 + q;
    // this query tile's global operands together: Q, the query's stencil
    // entries held by this half (slots e = 4 hh .. 4 hh + 3 of 7) and its
    // row of the bias table
    bf16x8_t qop[2];
#pragma unroll
    for (int s = 0; s < 2; ++s)
      qop[s] = __builtin_bit_cast(bf16x8_t, *(const uint4*)(base + (int64_t)(32 * b + c32) * 3 * D + 16 * s + 8 * hh));
    int lj[4];
    float cv[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int e = 4 * hh + u;
      lj[u] = 255;
      cv[u] = 0.f;
      if (e < 7) {
        lj[u] = nbr[row * 7 + e];
        cv[u] = corr[(row * 7 + e) * H + h];
      }
    }
    const float* bt = T0 + ((int64_t)h * T + q) * T;
    float4 bvv[NT][4];
#pragma unroll
    for (int a = 0; a < NT; ++a)
#pragma unroll
      for (int i = 0; i < 4; ++i) bvv[a][i] = *(const float4*)(bt + 32 * a + 8 * i + 4 * hh);
    // S^T tiles of this query tile: S[a] = K[32a..][:] Q[32b..][:]^T
    f32x16_t S[NT];
#pragma unroll
    for (int a = 0; a < NT; ++a)
#pragma unroll
      for (int q2 = 0; q2 < 16; ++q2) S[a][q2] = 0.f;
#pragma unroll
    for (int s = 0; s < 2; ++s)
#pragma unroll
      for (int a = 0; a < NT; ++a) S[a] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(kop[s][a], qop[s], S[a], 0, 0, 0);
    // the query's row of corrections: zero its half, then the half-wave hh
    // writes its neighbours (distinct neighbours have distinct keys)
#pragma unroll
    for (int z = 0; z < T / 8; ++z) *(float4*)&sC[h][c32][hh * (T / 2) + 4 * z] = make_float4(0.f, 0.f, 0.f, 0.f);
    wave_lds_fence();
#pragma unroll
    for (int u = 0; u < 4; ++u)
      if (lj[u] != 255) sC[h][c32][lj[u]] = cv[u];
    wave_lds_fence();
    float mx = -3.4e38f;
#pragma unroll
    for (int a = 0; a < NT; ++a)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int k0 = 32 * a + 8 * i + 4 * hh;
        const float4 bv = bvv[a][i];
        const float4 cw = *(const float4*)&sC[h][c32][k0];
        const float bj[4] = {bv.x + cw.x, bv.y + cw.y, bv.z + cw.z, bv.w + cw.w};
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const float v = fmaf(S[a][4 * i + j], scale, bj[j]);
          S[a][4 * i + j] = v;
          mx = fmaxf(mx, v);
        }
      }
    mx = fmaxf(mx, __shfl_xor(mx, 32, 64));
    float sum = 0.f;
#pragma unroll
    for (int a = 0; a < NT; ++a)
#pragma unroll
      for (int q2 = 0; q2 < 16; ++q2) {
        const float p = __expf(S[a][q2] - mx);  // P is rounded to BF16 for the product below
        S[a][q2] = p;
        sum += p;
      }
    sum += __shfl_xor(sum, 32, 64);
    f32x16_t O;
#pragma unroll
    for (int q2 = 0; q2 < 16; ++q2) O[q2] = 0.f;
#pragma unroll
    for (int a = 0; a < NT; ++a)
#pragma unroll
      for (int s = 0; s < 2; ++s) {
        bf16x8_t pb, vb;
        const int kb = 32 * a + 16 * s + 4 * hh;
        uint16_t vv[8];
        *(uint2*)&vv[0] = *(const uint2*)&sVt[h][c32][kb];
        *(uint2*)&vv[4] = *(const uint2*)&sVt[h][c32][kb + 8];
        vb = __builtin_bit_cast(bf16x8_t, *(const uint4*)vv);
        const uint4 pw = make_uint4(pack_bf16x2(S[a][8 * s], S[a][8 * s + 1]), pack_bf16x2(S[a][8 * s + 2], S[a][8 * s + 3]),
                                    pack_bf16x2(S[a][8 * s + 4], S[a][8 * s + 5]),
                                    pack_bf16x2(S[a][8 * s + 6], S[a][8 * s + 7]));
        pb = __builtin_bit_cast(bf16x8_t, pw);
        O = __builtin_amdgcn_mfma_f32_32x32x16_bf16(vb, pb, O, 0, 0, 0);
      }
    const float inv = 1.f / sum;
    uint16_t* orow = out + row * D + h * DH;
#pragma unroll
    for (int i = 0; i < 4; ++i)
      *(uint2*)(orow + 8 * i + 4 * hh) =
          make_uint2(pack_bf16x2(O[4 * i] * inv, O[4 * i + 1] * inv), pack_bf16x2(O[4 * i + 2] * inv, O[4 * i + 3] * inv));
  }
}

// The diagonal attention sublayer of one leaf in one block (BF16 inference,
// L = 64 tokens, 4 heads of 32, d = 128): X += O Wo^T + bo with
// O = MHA(LN1(X)) and the edge-biased attention of k_attention_mfma, so that
// neither the normalised tokens nor Q, K, V nor O leave the chip.  Four waves:
//   1. LN1 of the leaf's 64 rows (each wave 16, four at a time, the lanes and
//      DPP sums of k_layernorm128) into a BF16 tile in LDS;
//   2. wave h forms head h's Q, K and V (two 32 x 32 fragments each, W as the
//      first MFMA operand, k steps of 16 in order, bias then BF16 rounding:
//      the QKV GEMM's chain and epilogue).  Q and K become the attention's
//      MFMA operands in registers (each lane swaps two of its four groups with
//      the lane 32 away); V goes to LDS transposed;
//   3. the attention of k_attention_mfma, its BF16 output into the LDS tile;
//   4. the output projection (wave h: features 32 h .. + 31 of all 64 tokens),
//      epilogue (acc + bo) + X, as the O GEMM.
// Each value sees the arithmetic of the four separate launches, so the results
// equal them bit for bit.  The stencil corrections of the attention logits are
// selected in registers (each lane compares its keys with its query's seven
// neighbours) instead of going through a dense LDS row: 35 KB of LDS, no
// register spills at two waves per SIMD.
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2)))
void k_attn_sublayer64(float* X, const float* __restrict__ g1, const float* __restrict__ be1,
                       const uint16_t* __restrict__ Wqkv, const float* __restrict__ bqkv,
                       const uint16_t* __restrict__ Wo, const float* __restrict__ bo, const float* T0,
                       const float* corr, const uint8_t* nbr) {
  constexpr int T = 64, DH = 32, H = 4, D = H * DH, NT = T / 32, VP = T + 8, AP = D + 8;
  __shared__ __attribute__((aligned(16))) uint16_t sA[T][AP];  // LN1(X), later O
  __shared__ __attribute__((aligned(16))) uint16_t sVt[H][DH][VP];
  const int h = threadIdx.x >> 6, lane = threadIdx.x & 63, hh = lane >> 5, c32 = lane & 31;
  const int64_t row0 = (int64_t)blockIdx.x * T;
  // 1. LN1 (the wave's 16 rows requested together)
  {
    const int c0 = 8 * (lane & 15);
    float4 xv[4][2];
#pragma unroll
    for (int it = 0; it < 4; ++it) {
      const float* xr = X + (row0 + 16 * h + 4 * it + (lane >> 4)) * D + c0;
      xv[it][0] = ((const float4*)xr)[0];
      xv[it][1] = ((const float4*)xr)[1];
    }
    float gm[8], bt[8];
    load8(g1 + c0, gm);
    load8(be1 + c0, bt);
#pragma unroll
    for (int it = 0; it < 4; ++it) {
      const int r = 16 * h + 4 * it + (lane >> 4);
      const float x[8] = {xv[it][0].x, xv[it][0].y, xv[it][0].z, xv[it][0].w,
                          xv[it][1].x, xv[it][1].y, xv[it][1].z, xv[it][1].w};
      float mu = 0.f;
#pragma unroll
      for (int q = 0; q < 8; ++q) mu += x[q];
      mu = row16_sum(mu) * (1.f / 128.f);
      float var = 0.f;
#pragma unroll
      for (int q = 0; q < 8; ++q) var += (x[q] - mu) * (x[q] - mu);
      const float rs = rsqrtf(row16_sum(var) * (1.f / 128.f) + 1e-5f);
      float y[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) y[q] = (x[q] - mu) * rs * gm[q] + bt[q];
      store8<uint16_t>(&sA[r][c0], y);
    }
  }
  // this wave's operands of part j's weight rows (j D + 32 h + c32, k 8 hh
  // of every k step), shared by both token blocks
  auto load_w = [&](const uint16_t* Wt, int wrow, bf16x8_t* w) {
    const uint16_t* src = Wt + (int64_t)wrow * D + 8 * hh;
#pragma unroll
    for (int s = 0; s < D / 16; ++s) w[s] = __builtin_bit_cast(bf16x8_t, *(const uint4*)(src + 16 * s));
  };
  bf16x8_t wcur[D / 16], wnext[D / 16];
  load_w(Wqkv, 32 * h + c32, wcur);
  __syncthreads();
  // 2. head h's Q, K, V: fragment (token block rb, part j) over features
  // j D + 32 h .. + 31; the regrouping of a fragment's BF16 values into the
  // MFMA operand layout of k steps 0 and 1 (features 16 s + 8 hh .. + 7)
  auto frag = [&](int j, int rb, const bf16x8_t* w) {
    f32x16_t acc;
#pragma unroll
    for (int q = 0; q < 16; ++q) acc[q] = 0.f;
#pragma unroll
    for (int s = 0; s < D / 16; ++s) {
      const bf16x8_t xb = __builtin_bit_cast(bf16x8_t, *(const uint4*)&sA[32 * rb + c32][16 * s + 8 * hh]);
      acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(w[s], xb, acc, 0, 0, 0);
    }
    const int cb = j * D + 32 * h + 4 * hh;
    uint32_t d[8];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      // biases by scalar loads: a bias's offset in the weight vector need not be 16-byte aligned
      const float* bq = bqkv + cb + 8 * q;
      d[2 * q] = pack_bf16x2(acc[4 * q] + bq[0], acc[4 * q + 1] + bq[1]);
      d[2 * q + 1] = pack_bf16x2(acc[4 * q + 2] + bq[2], acc[4 * q + 3] + bq[3]);
    }
    return std::array<uint32_t, 8>{d[0], d[1], d[2], d[3], d[4], d[5], d[6], d[7]};
  };
  auto regroup = [&](const std::array<uint32_t, 8>& d, bf16x8_t* op) {
    uint32_t x[4];
#pragma unroll
    for (int e = 0; e < 2; ++e) {
      x[2 * e] = (uint32_t)__shfl_xor((int)(hh ? d[4 * e] : d[4 * e + 2]), 32);
      x[2 * e + 1] = (uint32_t)__shfl_xor((int)(hh ? d[4 * e + 1] : d[4 * e + 3]), 32);
    }
#pragma unroll
    for (int e = 0; e < 2; ++e)
      op[e] = __builtin_bit_cast(bf16x8_t, hh ? make_uint4(x[2 * e], x[2 * e + 1], d[4 * e + 2], d[4 * e + 3])
                                               : make_uint4(d[4 * e], d[4 * e + 1], x[2 * e], x[2 * e + 1]));
  };
  bf16x8_t qop[NT][2], kopT[NT][2];  // [token block][k step]
  // Q (the K rows load meanwhile)
  load_w(Wqkv, D + 32 * h + c32, wnext);
#pragma unroll
  for (int rb = 0; rb < NT; ++rb) regroup(frag(0, rb, wcur), qop[rb]);
  // K (the V rows load meanwhile)
  load_w(Wqkv, 2 * D + 32 * h + c32, wcur);
#pragma unroll
  for (int rb = 0; rb < NT; ++rb) regroup(frag(1, rb, wnext), kopT[rb]);
  // V, transposed into LDS: this lane's key 32 rb + c32, head features
  // 8 q + 4 hh + 0..3
#pragma unroll
  for (int rb = 0; rb < NT; ++rb) {
    const std::array<uint32_t, 8> v = frag(2, rb, wcur);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int f0 = 8 * q + 4 * hh;
      sVt[h][f0][32 * rb + c32] = (uint16_t)(v[2 * q] & 0xffff);
      sVt[h][f0 + 1][32 * rb + c32] = (uint16_t)(v[2 * q] >> 16);
      sVt[h][f0 + 2][32 * rb + c32] = (uint16_t)(v[2 * q + 1] & 0xffff);
      sVt[h][f0 + 3][32 * rb + c32] = (uint16_t)(v[2 * q + 1] >> 16);
    }
  }
  __syncthreads();  // every wave is done reading LN1(X): the tile takes O next; V^T is in place
  // 3. attention (k_attention_mfma's arithmetic)
  const float scale = 0.17677669529663687f;  // 1/sqrt(32)
#pragma unroll
  for (int b = 0; b < NT; ++b) {
    if (b > 0) __builtin_amdgcn_sched_barrier(0);  // keep the tiles' register lifetimes apart
    const int q = 32 * b + c32;
    const int64_t row = row0 + q;
    // the query's 7 stencil neighbours (key, correction); 255: none
    int lj[7];
    float cv[7];
#pragma unroll
    for (int e = 0; e < 7; ++e) {
      lj[e] = nbr[row * 7 + e];
      cv[e] = corr[(row * 7 + e) * H + h];
    }
    const float* bt = T0 + ((int64_t)h * T + q) * T;
    float4 bvv[NT][4];
#pragma unroll
    for (int a = 0; a < NT; ++a)
#pragma unroll
      for (int i = 0; i < 4; ++i) bvv[a][i] = *(const float4*)(bt + 32 * a + 8 * i + 4 * hh);
    f32x16_t S[NT];
#pragma unroll
    for (int a = 0; a < NT; ++a)
#pragma unroll
      for (int q2 = 0; q2 < 16; ++q2) S[a][q2] = 0.f;
#pragma unroll
    for (int s = 0; s < 2; ++s)
#pragma unroll
      for (int a = 0; a < NT; ++a) S[a] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(kopT[a][s], qop[b][s], S[a], 0, 0, 0);
    // k_attention_mfma adds a dense row of corrections (the neighbour's value
    // at its key, 0 elsewhere); here each lane selects it for its keys
    float mx = -3.4e38f;
#pragma unroll
    for (int a = 0; a < NT; ++a)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int k0 = 32 * a + 8 * i + 4 * hh;
        const float4 bv = bvv[a][i];
        float cw[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int jj = 0; jj < 4; ++jj)
#pragma unroll
          for (int e = 0; e < 7; ++e) cw[jj] = lj[e] == k0 + jj ? cv[e] : cw[jj];
        const float bj[4] = {bv.x + cw[0], bv.y + cw[1], bv.z + cw[2], bv.w + cw[3]};
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const float v = fmaf(S[a][4 * i + j], scale, bj[j]);
          S[a][4 * i + j] = v;
          mx = fmaxf(mx, v);
        }
      }
    mx = fmaxf(mx, __shfl_xor(mx, 32, 64));
    float sum = 0.f;
#pragma unroll
    for (int a = 0; a < NT; ++a)
#pragma unroll
      for (int q2 = 0; q2 < 16; ++q2) {
        const float p = __expf(S[a][q2] - mx);  // P is rounded to BF16 for the product below
        S[a][q2] = p;
        sum += p;
      }
    sum += __shfl_xor(sum, 32, 64);
    f32x16_t O;
#pragma unroll
    for (int q2 = 0; q2 < 16; ++q2) O[q2] = 0.f;
#pragma unroll
    for (int a = 0; a < NT; ++a)
#pragma unroll
      for (int s = 0; s < 2; ++s) {
        bf16x8_t pb, vb;
        const int kb = 32 * a + 16 * s + 4 * hh;
        uint16_t vv[8];
        *(uint2*)&vv[0] = *(const uint2*)&sVt[h][c32][kb];
        *(uint2*)&vv[4] = *(const uint2*)&sVt[h][c32][kb + 8];
        vb = __builtin_bit_cast(bf16x8_t, *(const uint4*)vv);
        const uint4 pw = make_uint4(pack_bf16x2(S[a][8 * s], S[a][8 * s + 1]), pack_bf16x2(S[a][8 * s + 2], S[a][8 * s + 3]),
                                    pack_bf16x2(S[a][8 * s + 4], S[a][8 * s + 5]),
                                    pack_bf16x2(S[a][8 * s + 6], S[a][8 * s + 7]));
        pb = __builtin_bit_cast(bf16x8_t, pw);
        O = __builtin_amdgcn_mfma_f32_32x32x16_bf16(vb, pb, O, 0, 0, 0);
      }
    const float inv = 1.f / sum;
#pragma unroll
    for (int i = 0; i < 4; ++i)
      *(uint2*)&sA[q][h * DH + 8 * i + 4 * hh] =
          make_uint2(pack_bf16x2(O[4 * i] * inv, O[4 * i + 1] * inv), pack_bf16x2(O[4 * i + 2] * inv, O[4 * i + 3] * inv));
  }
  load_w(Wo, 32 * h + c32, wnext);  // the output projection's rows, while the other waves finish
  __syncthreads();  // O of every head in the tile
  // 4. X += O Wo^T + bo: wave h, output features 32 h .. + 31, token blocks 0, 1
#pragma unroll
  for (int tb = 0; tb < NT; ++tb) {
    f32x16_t acc;
#pragma unroll
    for (int q = 0; q < 16; ++q) acc[q] = 0.f;
#pragma unroll
    for (int s = 0; s < D / 16; ++s) {
      const bf16x8_t ob = __builtin_bit_cast(bf16x8_t, *(const uint4*)&sA[32 * tb + c32][16 * s + 8 * hh]);
      acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(wnext[s], ob, acc, 0, 0, 0);
    }
    const int cb = 32 * h + 4 * hh;
    float* xr = X + (row0 + 32 * tb + c32) * D;
    float4 rv[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) rv[q] = *(const float4*)(xr + cb + 8 * q);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const float* bq = bo + cb + 8 * q;
      *(float4*)(xr + cb + 8 * q) = make_float4((acc[4 * q] + bq[0]) + rv[q].x, (acc[4 * q + 1] + bq[1]) + rv[q].y,
                                                (acc[4 * q + 2] + bq[2]) + rv[q].z, (acc[4 * q + 3] + bq[3]) + rv[q].w);
    }
  }
}

// Off-diagonal tile attention on the matrix cores (T = 16 tokens, BF16
// operands, FP32 accumulation): one wave per (tile, head), the four heads of
// a tile in one block.  S^T = K Q^T is one 16x16x32 MFMA (keys as rows: lane
// l owns query l % 16 and keys 4 (l / 16) .. + 3, so the softmax reduces over
// the four lanes l % 16 + 16 g); O^T = V^T P^T is two 16x16x16 MFMAs whose B
// operand is exactly the four P values each lane holds.
__global__ __launch_bounds__(256) void k_attention_tile_mfma(const uint16_t* qkv, uint16_t* out, const float* bias) {
  constexpr int T = 16, DH = 32, H = 4, D = H * DH;
  __shared__ __attribute__((aligned(16))) uint16_t sVt[H][DH][T + 8];
  const int h = threadIdx.x >> 6, lane = threadIdx.x & 63, q4 = lane >> 4, c16 = lane & 15;
  const int64_t row0 = (int64_t)blockIdx.x * T;
  const uint16_t* base = qkv + row0 * 3 * D + h * DH;
  {  // V^T into LDS: lane -> (key lane / 4, 8 head features)
    const int key = lane >> 2, c0 = (lane & 3) * 8;
    const uint4 v = *(const uint4*)(base + (int64_t)key * 3 * D + 2 * D + c0);
    const uint16_t* pv = (const uint16_t*)&v;
#pragma unroll
    for (int e = 0; e < 8; ++e) sVt[h][c0 + e][key] = pv[e];
  }
  __syncthreads();
  const bf16x8_t ka = __builtin_bit_cast(bf16x8_t, *(const uint4*)(base + (int64_t)c16 * 3 * D + D + 8 * q4));
  const bf16x8_t qb = __builtin_bit_cast(bf16x8_t, *(const uint4*)(base + (int64_t)c16 * 3 * D + 8 * q4));
  f32x4_t S = {0.f, 0.f, 0.f, 0.f};
  S = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ka, qb, S, 0, 0, 0);
  const float scale = 0.17677669529663687f;  // 1/sqrt(32)
  const float4 bv = *(const float4*)(bias + ((int64_t)blockIdx.x * H + h) * T * T + c16 * T + 4 * q4);
  float v[4] = {fmaf(S[0], scale, bv.x), fmaf(S[1], scale, bv.y), fmaf(S[2], scale, bv.z), fmaf(S[3], scale, bv.w)};
  float mx = fmaxf(fmaxf(v[0], v[1]), fmaxf(v[2], v[3]));
  mx = fmaxf(mx, __shfl_xor(mx, 16, 64));
  mx = fmaxf(mx, __shfl_xor(mx, 32, 64));
  float sum = 0.f;
  uint16_t pp[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    v[j] = expf(v[j] - mx);
    sum += v[j];
    pp[j] = f32_to_bf16(v[j]);
  }
  sum += __shfl_xor(sum, 16, 64);
  sum += __shfl_xor(sum, 32, 64);
  const float inv = 1.f / sum;
  const bf16x4_t pb = __builtin_bit_cast(bf16x4_t, *(const uint2*)pp);
  uint16_t* orow = out + (row0 + c16) * D + h * DH;
#pragma unroll
  for (int half = 0; half < 2; ++half) {
    const bf16x4_t va = __builtin_bit_cast(bf16x4_t, *(const uint2*)&sVt[h][16 * half + c16][4 * q4]);
    f32x4_t O = {0.f, 0.f, 0.f, 0.f};
    O = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(va, pb, O, 0, 0, 0);
    uint16_t o4[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) o4[j] = f32_to_bf16(O[j] * inv);
    *(uint2*)(orow + 16 * half + 4 * q4) = *(const uint2*)o4;
  }
}

// ------------------------------------------------------------------ strips and highways
// Leaves per chunk of the highway trees (levels below the chunk size are
// handled in registers).
constexpr int STRIP_CHUNK = 16;

// Highway buffers of the diagonal tokens (Sec. 4.3): r_i (c_i) is the mean of
// the diagonal token i and of every off-diagonal token whose row (column)
// sub-strip contains i.  Leaf k sits at level j in tile K - K/2^j + (k >> (j+1))
// on side (k >> j) & 1; its position l maps to sub-strip token l / p.
// The highway buffers by (leaf k, sub-strip t) groups.  The off-diagonal
// tokens a node reads depend only on its leaf and its sub-strip t = l / p, so
// per group:  rs (cs) = sum over the levels where the leaf is on the row
// (column) side of token t of that level's tile.  Then r_i = (x_i + rs) / n_r
// and c_i = (x_i + cs) / n_c, with n_r (n_c) = 1 + the number of row (column)
// levels of the leaf; the group sums of r and c feed the off-diagonal
// tokens' context.
// rs is a root-to-leaf path sum: with u = k >> j the level-j ancestor of
// leaf k, R_j(u) = R_{j+1}(u >> 1) + [u even] Xo(tile (j, u >> 1), t), R_J =
// 0, rs = R_0 (cs alike with [u odd]).  Upper levels (2^j >= C = min(16, K)):
// per (frame, t), R at each aligned chunk of C leaves; lower levels: per
// (chunk, t), down to the leaves in registers.  Levels are added top-down.
__device__ inline void leaf_sides(int k, int J, int& nr, int& nc) {
  nr = 1;
  nc = 1;
  for (int j = 0; j < J; ++j) {
    if (((k >> j) & 1) == 0) ++nr;
    else ++nc;
  }
}

__global__ __launch_bounds__(256) void k_hw_levels_hi(const FrameDesc* fr, const int* chunk0, const float* Xo,
                                                      int LS, float* top) {
  const int f = blockIdx.x, t = blockIdx.y, side = threadIdx.x >> 7, col = threadIdx.x & 127;
  const FrameDesc F = fr[f];
  const int K = F.K, C = min(STRIP_CHUNK, K);
  int jc = 0;
  while ((1 << jc) < C) ++jc;  // C = 2^jc
  for (int q = 0; q < K / C; ++q) {
    float R = 0.f;
    for (int j = F.J - 1; j >= jc; --j) {
      const int u = q >> (j - jc);
      if ((u & 1) == side) R += Xo[((int64_t)(F.m0 + K - (K >> j) + (u >> 1)) * LS + t) * 128 + col];
    }
    top[(((int64_t)chunk0[f] + q) * LS + t) * 256 + 128 * side + col] = R;
  }
}

__global__ __launch_bounds__(256) void k_hw_levels_lo(const FrameDesc* fr, const int2* tab, const float* top,
                                                      const float* Xo, int LS, float* rs, float* cs) {
  const int2 e = tab[blockIdx.x];
  const int t = blockIdx.y, side = threadIdx.x >> 7, col = threadIdx.x & 127;
  const FrameDesc F = fr[e.x];
  const int K = F.K, C = min(STRIP_CHUNK, K), leaf0 = e.y * C;
  float v[STRIP_CHUNK];
  v[0] = top[(((int64_t)blockIdx.x) * LS + t) * 256 + 128 * side + col];
  // every level's token is loaded first (branch-free, so the loads issue
  // together: a load behind a branch was waited for before the next one),
  // then added where the leaf is on this side.  Entries past the chunk's
  // levels load a valid row of the frame's tiles and are not used.
  float xo[2 * STRIP_CHUNK - 2];  // level j at offset (16 >> j) - 2
  if (F.MH > 0) {
    const int mlast = F.m0 + F.MH - 1;
#pragma unroll
    for (int j = 3; j >= 0; --j)
#pragma unroll
      for (int i = 0; i < (STRIP_CHUNK >> j); ++i) {
        const int u = (leaf0 >> j) + i, m = min(F.m0 + K - (K >> j) + (u >> 1), mlast);
        xo[(STRIP_CHUNK >> j) - 2 + i] = Xo[((int64_t)m * LS + t) * 128 + col];
      }
  }
  // level j: node i (local, descending so the parent v[i >> 1] is still the level-(j+1) value)
#pragma unroll
  for (int j = 3; j >= 0; --j) {
    if ((C >> j) < 2) continue;  // level j lies above the chunk
#pragma unroll
    for (int i = (STRIP_CHUNK >> j) - 1; i >= 0; --i) {
      if (i >= (C >> j)) continue;
      const int u = (leaf0 >> j) + i;
      const float x = v[i >> 1];
      v[i] = (u & 1) == side ? x + xo[(STRIP_CHUNK >> j) - 2 + i] : x;
    }
  }
  float* out = side ? cs : rs;
#pragma unroll
  for (int q = 0; q < STRIP_CHUNK; ++q)
    if (q < C) out[(((int64_t)F.k0 + leaf0 + q) * LS + t) * 128 + col] = v[q];
}

// Off-diagonal token context (the mean of r over I_m^t and of c over J_m^t)
// from the group sums hr, hc of r and c: tile (j, i) of a frame has the row
// strip of leaves [2 i S, 2 i S + S) and the column strip [2 i S + S, 2 i S +
// 2 S), S = 2^j, so its strip sums are the dyadic block sums D_j[2 i] of hr and
// D_j[2 i + 1] of hc, with D_0 the leaves and D_{j+1}[q] = D_j[2 q] + D_j[2 q +
// 1].  Lower levels: one block per (aligned chunk of C = min(16, K) leaves,
// t), threads (side, feature); the block builds D_0 .. D_log2(C) of its chunk
// in registers, writes the context of every tile that lies inside the chunk,
// and the chunk total.  Upper levels (2 S > C): per (frame, t), strip sums
// of the chunk totals in chunk order.  Each context entry is divided by S p.

// One level of the chunk tree: the context of the level's tiles inside the
// chunk (v holds the blocks of size S), then the fold to blocks of size 2 S.
template <int S, typename OT>
__device__ inline void strip_level(float (&v)[STRIP_CHUNK], int C, int leaf0, int j, const FrameDesc& F, int t,
                                   int LS, int side, int col, int p, OT* out) {
#pragma unroll
  for (int il = 0; il < STRIP_CHUNK / (2 * S); ++il) {
    if (il < C / (2 * S)) {
      const int m = F.K - (F.K >> j) + leaf0 / (2 * S) + il;
      out[((int64_t)(F.m0 + m) * LS + t) * 256 + 128 * side + col] = to_act<OT>(v[2 * il + side] / (float)(S * p));
    }
  }
#pragma unroll
  for (int q = 0; q < STRIP_CHUNK / (2 * S); ++q) v[q] = v[2 * q] + v[2 * q + 1];
}

// Sums over the p rows of each (leaf, sub-strip) group of a node stream:
// out[(leaf, t)][128] (one block per leaf, 4 sub-strip groups x 128
// features; rows added in order).  With hr = hc = these sums, the strip tree
// below yields the pooling means of the off-diagonal tokens.
__global__ __launch_bounds__(512) void k_group_sums(const FrameDesc* fr, const int* leaf2f, const float* X, int L,
                                                    int LS, float* out) {
  const int64_t kg = blockIdx.x;
  const FrameDesc F = fr[leaf2f[kg]];
  const int p = L / LS, col = threadIdx.x & 127;
  const float* base = X + ((int64_t)F.n0 + (kg - F.k0) * L) * 128 + col;
  for (int t = threadIdx.x >> 7; t < LS; t += 4) {
    float a = 0.f;
    for (int q = 0; q < p; ++q) a += base[(int64_t)(t * p + q) * 128];
    out[(kg * LS + t) * 128 + col] = a;
  }
}

template <typename OT>
__global__ __launch_bounds__(256) void k_hw_strips_lo(const FrameDesc* fr, const int2* tab, const float* hr,
                                                      const float* hc, int L, int LS, OT* out, float* tot) {
  const int2 e = tab[blockIdx.x];
  const int t = blockIdx.y, side = threadIdx.x >> 7, col = threadIdx.x & 127, p = L / LS;
  const FrameDesc F = fr[e.x];
  const int C = min(STRIP_CHUNK, F.K), leaf0 = e.y * C;
  const float* H = side ? hc : hr;
  float v[STRIP_CHUNK];
#pragma unroll
  for (int q = 0; q < STRIP_CHUNK; ++q)
    v[q] = q < C ? H[(((int64_t)F.k0 + leaf0 + q) * LS + t) * 128 + col] : 0.f;
  static_assert(STRIP_CHUNK == 16, "four tree levels per chunk");
  if (2 <= C) strip_level<1>(v, C, leaf0, 0, F, t, LS, side, col, p, out);
  if (4 <= C) strip_level<2>(v, C, leaf0, 1, F, t, LS, side, col, p, out);
  if (8 <= C) strip_level<4>(v, C, leaf0, 2, F, t, LS, side, col, p, out);
  if (16 <= C) strip_level<8>(v, C, leaf0, 3, F, t, LS, side, col, p, out);
  tot[(((int64_t)blockIdx.x) * LS + t) * 256 + 128 * side + col] = v[0];
}

template <typename OT>
__global__ __launch_bounds__(256) void k_hw_strips_hi(const FrameDesc* fr, const int* chunk0, const float* tot,
                                                      int L, int LS, OT* out) {
  const int f = blockIdx.x, t = blockIdx.y, side = threadIdx.x >> 7, col = threadIdx.x & 127, p = L / LS;
  const FrameDesc F = fr[f];
  const int K = F.K, C = min(STRIP_CHUNK, K);
  const float* T = tot + ((int64_t)chunk0[f] * LS + t) * 256 + 128 * side + col;
  int j = 0;
  while ((2 << j) <= C) ++j;  // first level whose tiles span more than one chunk
  for (; j < F.J; ++j) {
    const int S = 1 << j, nc = S / C;
    for (int i = 0; i < (K >> (j + 1)); ++i) {
      const int c0 = (2 * i * S + side * S) / C;
      float sum = 0.f;
      for (int q = 0; q < nc; ++q) sum += T[(int64_t)(c0 + q) * LS * 256];
      const int m = K - (K >> j) + i;
      out[((int64_t)(F.m0 + m) * LS + t) * 256 + 128 * side + col] = to_act<OT>(sum / (float)(S * p));
    }
  }
}

// r, c of the diagonal tokens written out (the reverse pass reads them).
__global__ __launch_bounds__(256) void k_hw_materialize(const FrameDesc* fr, const int* node2f, const float* Xd,
                                                        const float* rs, const float* cs, int L, int LS,
                                                        int64_t ntot, float* R, float* Cc) {
  const int64_t i = (int64_t)blockIdx.x * 2 + (threadIdx.x >> 7);
  if (i >= ntot) return;
  const int col = threadIdx.x & 127;
  const FrameDesc F = fr[node2f[i]];
  const int c = (int)(i - F.n0), k = c / L, l = c % L, p = L / LS;
  int nr, nc;
  leaf_sides(k, F.J, nr, nc);
  const int64_t gi = (((int64_t)F.k0 + k) * LS + l / p) * 128 + col;
  const float x = Xd[i * 128 + col];
  // r = (x + rs) / n_r as a product with the reciprocal, as the diagonal LayerNorm forms it
  R[i * 128 + col] = (x + rs[gi]) * (1.f / (float)nr);
  Cc[i * 128 + col] = (x + cs[gi]) * (1.f / (float)nc);
}

// LN([x | r | c | g]) of the diagonal tokens with r, c formed on the fly from
// the level sums.  One wave per (leaf, sub-strip) group: its p = 4 rows share
// the level sums, so the wave loads them once, keeps the four rows in flight
// together (lane l: segment l / 16 of the concat, 8 features), and also
// writes the group's sums of r and of c (rows added in order), which the
// off-diagonal context is built from.

template <typename AT>
__global__ __launch_bounds__(256) void k_ln_hw_diag(const FrameDesc* fr, const int* node2f, const float* X,
                                                    const float* rs, const float* cs, const float* G, int L, int LS,
                                                    const float* gam, const float* bet, AT* Y, float* hr, float* hc,
                                                    int M) {
  const int row0 = (blockIdx.x * 4 + (threadIdx.x >> 6)) * 4, lane = threadIdx.x & 63;
  if (row0 >= M) return;
  const int f = node2f[row0];
  const FrameDesc F = fr[f];
  const int c = row0 - F.n0, k = c / L, l = c % L, p = L / LS;
  const int seg = lane >> 4, c0 = (lane & 15) * 8;
  const int64_t grp = ((int64_t)F.k0 + k) * LS + l / p;
  float v[4][8];
  if (seg == 3) {
    load8(G + (int64_t)f * 128 + c0, v[0]);
#pragma unroll
    for (int r = 1; r < 4; ++r)
#pragma unroll
      for (int q = 0; q < 8; ++q) v[r][q] = v[0][q];
  } else {
#pragma unroll
    for (int r = 0; r < 4; ++r) load8(X + (int64_t)(row0 + r) * 128 + c0, v[r]);
    if (seg > 0) {
      int nr, nc;
      leaf_sides(k, F.J, nr, nc);
      const float inv = 1.f / (float)(seg == 1 ? nr : nc);
      float h[8], o[8];
      load8((seg == 1 ? rs : cs) + grp * 128 + c0, h);
#pragma unroll
      for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int q = 0; q < 8; ++q) v[r][q] = (v[r][q] + h[q]) * inv;
#pragma unroll
      for (int q = 0; q < 8; ++q) o[q] = ((v[0][q] + v[1][q]) + v[2][q]) + v[3][q];
      float* dst = (seg == 1 ? hr : hc) + grp * 128 + c0;
      ((float4*)dst)[0] = make_float4(o[0], o[1], o[2], o[3]);
      ((float4*)dst)[1] = make_float4(o[4], o[5], o[6], o[7]);
    }
  }
  float mu[4], rsd[4];
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    mu[r] = 0.f;
#pragma unroll
    for (int q = 0; q < 8; ++q) mu[r] += v[r][q];
  }
  wave_sum4(mu);
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    mu[r] *= (1.f / 512.f);
    rsd[r] = 0.f;
#pragma unroll
    for (int q = 0; q < 8; ++q) rsd[r] += (v[r][q] - mu[r]) * (v[r][q] - mu[r]);
  }
  wave_sum4(rsd);
  const int gc = seg * 128 + c0;
  float gm[8], bt[8];
  load8(gam + gc, gm);
  load8(bet + gc, bt);
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const float sd = rsqrtf(rsd[r] * (1.f / 512.f) + 1e-5f);
    float o[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) o[q] = (v[r][q] - mu[r]) * sd * gm[q] + bt[q];
    store8<AT>(Y + (int64_t)(row0 + r) * 512 + gc, o);
  }
}

// Column sums of 128-wide rows over chunks of at most SUM_CHUNK rows (first
// stage of the per-frame global token g = mean of all tokens of the frame).
// 512 threads: row group g (4 of them) adds rows g, g + 4, ... of the chunk,
// then the groups are added in order.
constexpr int SUM_CHUNK = 64;
struct SumChunk {
  int frame, kind;  // kind 0: diagonal rows, 1: off-diagonal rows
  int64_t row0;
  int rows;
};

__global__ __launch_bounds__(512) void k_chunk_sums(const SumChunk* ch, const float* Xd, const float* Xo,
                                                    float* part) {
  __shared__ float red[4][128];
  const SumChunk c = ch[blockIdx.x];
  const float* X = (c.kind ? Xo : Xd) + c.row0 * 128;
  const int col = threadIdx.x & 127, g = threadIdx.x >> 7;
  float s = 0.f;
#pragma unroll 4
  for (int r = g; r < c.rows; r += 4) s += X[(int64_t)r * 128 + col];
  red[g][col] = s;
  __syncthreads();
  if (g == 0) part[(int64_t)blockIdx.x * 128 + col] = ((red[0][col] + red[1][col]) + red[2][col]) + red[3][col];
}

// Per-frame mean from the chunk sums: 8 groups of 128 features, group g adds
// chunks g, g + 8, ... in order, then the groups are added in order.
__global__ __launch_bounds__(1024) void k_frame_mean(const int* chunk0, const float* part, const float* count,
                                                     float* G) {
  __shared__ float red[8][128];
  const int f = blockIdx.x, col = threadIdx.x & 127, g = threadIdx.x >> 7;
  float s = 0.f;
  for (int c = chunk0[f] + g; c < chunk0[f + 1]; c += 8) s += part[(int64_t)c * 128 + col];
  red[g][col] = s;
  __syncthreads();
  if (g == 0) {
    float t = red[0][col];
#pragma unroll
    for (int q = 1; q < 8; ++q) t += red[q][col];
    G[f * 128 + col] = t / count[f];
  }
}

// ------------------------------------------------------------------ heads and packing
// G_k = F_k F_k^T (one block per leaf).  Thread (bi, bj) forms the 4 x 4
// block of rows 4 bi.., columns 4 bj.. (8 LDS reads per 16 FMAs); each entry is
// its own FMA chain over c in order, and entries (i, j) and (j, i) multiply the
// same pairs, so G_k is exactly symmetric.
template <typename FT, int L>
__global__ __launch_bounds__(256) void k_gram(const float* Frows, FT* G) {
  constexpr int NB = L / 4, LP = L + 4;
  __shared__ __attribute__((aligned(16))) float sF[L][LP];
  const int64_t kg = blockIdx.x;
  for (int idx = threadIdx.x; idx < L * L / 4; idx += 256) {
    const int i = (4 * idx) / L, c = (4 * idx) % L;
    *(float4*)&sF[i][c] = *(const float4*)(Frows + kg * L * L + 4 * idx);
  }
  __syncthreads();
  if (threadIdx.x >= NB * NB) return;
  const int bi = threadIdx.x / NB, bj = threadIdx.x % NB;
  float acc[4][4];
#pragma unroll
  for (int r = 0; r < 4; ++r)
#pragma unroll
    for (int q = 0; q < 4; ++q) acc[r][q] = 0.f;
#pragma unroll 4
  for (int c = 0; c < L; ++c) {
    float fi[4], fj[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      fi[r] = sF[4 * bi + r][c];
      fj[r] = sF[4 * bj + r][c];
    }
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
      for (int q = 0; q < 4; ++q) acc[r][q] = fmaf(fi[r], fj[q], acc[r][q]);
  }
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    FT* g = G + kg * L * L + (int64_t)(4 * bi + r) * L + 4 * bj;
    if constexpr (sizeof(FT) == 2)
      *(uint2*)g = make_uint2(pack_bf16x2(acc[r][0], acc[r][1]), pack_bf16x2(acc[r][2], acc[r][3]));
    else
      *(float4*)g = make_float4(acc[r][0], acc[r][1], acc[r][2], acc[r][3]);
  }
}

// G_k = F_k F_k^T for L = 64 on the matrix cores (FP32 MFMA 32x32x2, FP32
// accumulation; one block per leaf, wave (I, J) forms the 32 x 32 block
// (I, J) along c in steps of 2).  Entries (i, j) and (j, i) multiply the same
// pairs in the same order, so G_k stays exactly symmetric, and each wave
// writes its block transposed (block (J, I)): a lane then holds four
// consecutive columns of one row.
typedef float f32x16v_t __attribute__((ext_vector_type(16)));
template <typename FT>
__global__ __launch_bounds__(256) void k_gram_mfma(const float* Frows, FT* G) {
  constexpr int L = 64, LP = L + 1;  // odd pitch: a column read touches 32 banks
  __shared__ float sF[L][LP];
  const int64_t kg = blockIdx.x;
  const float* src = Frows + kg * L * L;
  for (int idx = threadIdx.x; idx < L * L; idx += 256) sF[idx / L][idx % L] = src[idx];
  __syncthreads();
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int I = wave >> 1, J = wave & 1, r = lane & 31, h = lane >> 5;
  f32x16v_t acc;
#pragma unroll
  for (int v = 0; v < 16; ++v) acc[v] = 0.f;
#pragma unroll 8
  for (int k = 0; k < L; k += 2)
    acc = __builtin_amdgcn_mfma_f32_32x32x2f32(sF[32 * I + r][k + h], sF[32 * J + r][k + h], acc, 0, 0, 0);
  // acc[4 i + j] = G[32 I + 8 i + 4 h + j][32 J + r] = G[32 J + r][32 I + 8 i + 4 h + j]
  FT* g = G + kg * L * L + (int64_t)(32 * J + r) * L + 32 * I + 4 * h;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    if constexpr (sizeof(FT) == 2)
      *(uint2*)(g + 8 * i) = make_uint2(pack_bf16x2(acc[4 * i], acc[4 * i + 1]), pack_bf16x2(acc[4 * i + 2], acc[4 * i + 3]));
    else
      *(float4*)(g + 8 * i) = make_float4(acc[4 * i], acc[4 * i + 1], acc[4 * i + 2], acc[4 * i + 3]);
  }
}

// B_m = U_m V_m^T (one block per tile); UV rows = [U row | V row].
template <typename FT, int LS>
__global__ void k_uvt(const float* UV, FT* B) {
  const int64_t m = blockIdx.x;
  const int t = threadIdx.x / LS, t2 = threadIdx.x % LS;
  if (t >= LS) return;
  const float* u = UV + (m * LS + t) * (2 * LS);
  const float* v = UV + (m * LS + t2) * (2 * LS) + LS;
  float a = 0.f;
  for (int s = 0; s < LS; ++s) a = fmaf(u[s], v[s], a);
  B[(m * LS + t) * LS + t2] = to_act<FT>(a);
}

// Node heads [Ut | Vt | lam-logit] -> factor sections; lam = softplus.
// The row (36 floats, 16-byte aligned) is read whole before any store: with
// loads and stores interleaved, each load waited for the store before it.
template <typename FT, int LS>
__global__ void k_pack_nodes(const float* __restrict__ NH, int64_t ntot, FT* __restrict__ Ut, FT* __restrict__ Vt,
                             float* __restrict__ lam) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= ntot) return;
  constexpr int NQ = (2 * LS + 1 + 3) / 4;  // float4s covering [Ut | Vt | lam-logit] (<= 9 of the 36)
  float r[4 * NQ];
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    const float4 t = *(const float4*)(NH + i * 36 + 4 * q);
    r[4 * q] = t.x;
    r[4 * q + 1] = t.y;
    r[4 * q + 2] = t.z;
    r[4 * q + 3] = t.w;
  }
#pragma unroll
  for (int s = 0; s < LS; ++s) {
    Ut[i * LS + s] = to_act<FT>(r[s]);
    Vt[i * LS + s] = to_act<FT>(r[LS + s]);
  }
  lam[i] = softplus_f(r[2 * LS]);
}

// Weight conversion: dst[(n_off + n) * ld + k_off + k] = src[k * ncols + n].
struct ConvDesc {
  int64_t src, dst;
  int rows, cols, ld, n_off, k_off, pad;
};

// pad == 0 (transposed, forward):  dst[(n_off + n) * ld + k_off + k] = src[k * cols + n]
// pad == 1 (plain, backward dX):   dst[(k_off + k) * ld + n_off + n] = src[k * cols + n]
// One block per 64 x 64 tile (desc, k0, n0) of a source matrix, staged in LDS
// so that both the FP32 reads and the compute-type writes are row-contiguous.
template <typename AT>
__global__ __launch_bounds__(256) void k_convert(const ConvDesc* d, const int4* tiles, const float* W, AT* out) {
  __shared__ float t[64][65];
  const int4 tl = tiles[blockIdx.x];
  const ConvDesc c = d[tl.x];
  const int k0 = tl.y, n0 = tl.z;
  for (int e = threadIdx.x; e < 4096; e += 256) {
    const int kk = e >> 6, nn = e & 63, k = k0 + kk, n = n0 + nn;
    t[kk][nn] = (k < c.rows && n < c.cols) ? W[c.src + (int64_t)k * c.cols + n] : 0.f;
  }
  __syncthreads();
  for (int e = threadIdx.x; e < 4096; e += 256) {
    const int hi = e >> 6, lo = e & 63;
    // pad 0: rows of the output are n (hi), k (lo) contiguous; pad 1: rows k, n contiguous
    const int kk = c.pad ? hi : lo, nn = c.pad ? lo : hi, k = k0 + kk, n = n0 + nn;
    if (k >= c.rows || n >= c.cols) continue;
    const int64_t o = c.pad ? (int64_t)(c.k_off + k) * c.ld + c.n_off + n : (int64_t)(c.n_off + n) * c.ld + c.k_off + k;
    out[c.dst + o] = to_act<AT>(t[kk][nn]);
  }
}

// ------------------------------------------------------------------ host side

struct GemmW {
  int64_t off;  // element offset in the converted-weight arena
  int N, K;
};

struct NetPlan {
  std::vector<WeightEntry> lay;
  std::vector<ConvDesc> conv;
  int64_t arena = 0;
  std::vector<int4> tiles;  // (descriptor, k0, n0) conversion tiles, forward copies first
  int ntiles_fwd = 0;
  GemmW enc1, enc2, gcn[4], pool, hleaf1, hleaf2, hnode, huv;
  GemmW qkv[2][16], o[2][16], f1[2][16], f2[2][16];
  // plain copies W[in][out] for the input-gradient GEMMs dX = dY W^T
  // (N = in features, K = out features padded to 32)
  GemmW b_enc2, b_gcn[4], b_pool, b_hleaf1, b_hleaf2, b_hnode, b_huv;
  GemmW b_qkv[2][16], b_o[2][16], b_f1[2][16], b_f2[2][16];
};

static int64_t woff(const NetPlan& P, const std::string& n) {
  const WeightEntry* e = find_weight(P.lay, n);
  return e ? e->offset : -1;
}

static NetPlan make_plan(const hp_model_config& c) {
  NetPlan P;
  P.lay = weight_layout(c);
  auto gemm = [&](int N, int K) {
    GemmW g{P.arena, N, K};
    P.arena += (int64_t)N * K;
    return g;
  };
  auto conv = [&](const GemmW& g, const std::string& name, int n_off, int k_off) {
    const WeightEntry* e = find_weight(P.lay, name);
    P.conv.push_back(ConvDesc{e->offset, g.off, e->rows, e->cols, g.K, n_off, k_off, 0});
  };
  const int d = c.d, LS = c.rank;
  P.enc1 = gemm(d, 32);
  conv(P.enc1, "enc1.w", 0, 0);
  P.enc2 = gemm(d, d);
  conv(P.enc2, "enc2.w", 0, 0);
  for (int g = 0; g < c.gcn; ++g) {
    P.gcn[g] = gemm(d, d);
    conv(P.gcn[g], "gcn" + std::to_string(g) + ".w", 0, 0);
  }
  P.pool = gemm(d, 2 * d);
  conv(P.pool, "pool.wr", 0, 0);
  conv(P.pool, "pool.wc", 0, d);
  for (int s = 0; s < 2; ++s)
    for (int l = 0; l < c.layers; ++l) {
      std::string p = std::string(s ? "off" : "diag") + std::to_string(l) + ".";
      P.qkv[s][l] = gemm(3 * d, d);
      conv(P.qkv[s][l], p + "qkv.w", 0, 0);
      P.o[s][l] = gemm(d, d);
      conv(P.o[s][l], p + "o.w", 0, 0);
      P.f1[s][l] = gemm(4 * d, 4 * d);
      conv(P.f1[s][l], p + "f1.w", 0, 0);
      P.f2[s][l] = gemm(d, 4 * d);
      conv(P.f2[s][l], p + "f2.w", 0, 0);
    }
  P.hleaf1 = gemm(d, d);
  conv(P.hleaf1, "hleaf1.w", 0, 0);
  P.hleaf2 = gemm(c.leaf, d);
  conv(P.hleaf2, "hleaf2.w", 0, 0);
  P.hnode = gemm(2 * LS + 1, d);
  conv(P.hnode, "hut.w", 0, 0);
  conv(P.hnode, "hvt.w", LS, 0);
  conv(P.hnode, "hlam.w", 2 * LS, 0);
  P.huv = gemm(2 * LS, d);
  conv(P.huv, "hu.w", 0, 0);
  conv(P.huv, "hv.w", LS, 0);
  // backward copies
  auto bconv = [&](const GemmW& g, const std::string& name, int n_off, int k_off) {
    const WeightEntry* e = find_weight(P.lay, name);
    P.conv.push_back(ConvDesc{e->offset, g.off, e->rows, e->cols, g.K, n_off, k_off, 1});
  };
  auto pad32 = [](int v) { return (v + 31) / 32 * 32; };
  P.b_enc2 = gemm(d, d);
  bconv(P.b_enc2, "enc2.w", 0, 0);
  for (int g = 0; g < c.gcn; ++g) {
    P.b_gcn[g] = gemm(d, d);
    bconv(P.b_gcn[g], "gcn" + std::to_string(g) + ".w", 0, 0);
  }
  P.b_pool = gemm(2 * d, d);
  bconv(P.b_pool, "pool.wr", 0, 0);
  bconv(P.b_pool, "pool.wc", 0, d);
  for (int s = 0; s < 2; ++s)
    for (int l = 0; l < c.layers; ++l) {
      std::string p = std::string(s ? "off" : "diag") + std::to_string(l) + ".";
      P.b_qkv[s][l] = gemm(d, 3 * d);
      bconv(P.b_qkv[s][l], p + "qkv.w", 0, 0);
      P.b_o[s][l] = gemm(d, d);
      bconv(P.b_o[s][l], p + "o.w", 0, 0);
      P.b_f1[s][l] = gemm(4 * d, 4 * d);
      bconv(P.b_f1[s][l], p + "f1.w", 0, 0);
      P.b_f2[s][l] = gemm(4 * d, d);
      bconv(P.b_f2[s][l], p + "f2.w", 0, 0);
    }
  P.b_hleaf1 = gemm(d, d);
  bconv(P.b_hleaf1, "hleaf1.w", 0, 0);
  P.b_hleaf2 = gemm(d, pad32(c.leaf));
  bconv(P.b_hleaf2, "hleaf2.w", 0, 0);
  P.b_hnode = gemm(d, 64);
  bconv(P.b_hnode, "hut.w", 0, 0);
  bconv(P.b_hnode, "hvt.w", LS, 0);
  bconv(P.b_hnode, "hlam.w", 2 * LS, 0);
  P.b_huv = gemm(d, pad32(2 * LS));
  bconv(P.b_huv, "hu.w", 0, 0);
  bconv(P.b_huv, "hv.w", LS, 0);
  for (int i = 0; i < (int)P.conv.size(); ++i) {
    const ConvDesc& cd = P.conv[i];
    for (int k0 = 0; k0 < cd.rows; k0 += 64)
      for (int n0 = 0; n0 < cd.cols; n0 += 64) P.tiles.push_back(make_int4(i, k0, n0, 0));
    if (cd.pad == 0) P.ntiles_fwd = (int)P.tiles.size();
  }
  return P;
}

// Workspace of one batch (every buffer sized at creation, 4-byte activations
// so one arena serves both precisions).
struct NetBufs {
  NetPlan plan;
  int64_t Nd = 0, No = 0;
  void* feats = nullptr;
  float *H = nullptr, *Henc = nullptr, *R = nullptr, *C = nullptr, *Xo = nullptr, *Xo0 = nullptr;
  void *a128 = nullptr, *b128 = nullptr, *qkv = nullptr, *u512 = nullptr, *h512 = nullptr;
  void *ctx = nullptr, *ao128 = nullptr, *bo128 = nullptr, *qkvo = nullptr, *uo512 = nullptr, *ho512 = nullptr;
  float *ctxf = nullptr;
  float *hrs = nullptr, *hcs = nullptr, *hhr = nullptr, *hhc = nullptr;  // highway group sums [ktot L_s][128]
  float* eslots = nullptr;     // edge-MLP stencil-slot constants of the current layer [EDGE_CST]
  int2* lvl_tab = nullptr;     // (frame, chunk) of every frame's leaves, for the level sums
  int nlvl = 0;
  int* lvl0 = nullptr;         // first chunk of each frame [nframes]
  float* lvl_top = nullptr;    // level sums above each chunk [nlvl][L_s][2][128]
  int2* strip_tab = nullptr;   // (frame, chunk) of the context tree's lower levels
  int nstrip = 0;
  int* strip0 = nullptr;       // first chunk of each frame [nframes]
  float* strip_tot = nullptr;  // chunk totals [nstrip][L_s][2][128]
  float *Frows = nullptr, *NH = nullptr, *UV = nullptr;
  float *T0 = nullptr, *corr = nullptr, *ahat = nullptr, *desc = nullptr, *boff = nullptr;
  uint8_t* nbr = nullptr;
  // the inference's per-layer copies of T0, eslots, corr and boff (computed
  // ahead of the layers); pre: layer_fwd reads them, pre_side: they come
  // from the side stream (layer l waits for side_ev[l])
  float *T0l = nullptr, *eslotsl = nullptr, *corrl = nullptr, *boffl = nullptr;
  int pre = 0, pre_side = 0;
  int par = 0;  // the off-diagonal stack runs on the batch's off stream
  float *gpart = nullptr, *G = nullptr, *gcount = nullptr, *glob = nullptr, *bias_node = nullptr, *bias_uv = nullptr;
  void* warena = nullptr;
  ConvDesc* d_conv = nullptr;
  int4* d_tiles = nullptr;
  int *node2f = nullptr, *tok2f = nullptr, *tile2f = nullptr, *chunk0 = nullptr;
  SumChunk* chunks = nullptr;
  int nchunks = 0;
  DescChunk* desc_chunks = nullptr;
  int* desc_chunk0 = nullptr;
  double* desc_part = nullptr;
  int ndesc_chunks = 0;
};

static NetBufs* nb_of(Batch& b) { return reinterpret_cast<NetBufs*>(b.net.ws); }

hp_status network_supported(const hp_model_config& c) {
  if (c.d != 128 || c.edge_hidden > 64 || c.heads * 32 != c.d || c.node_feats + c.glob_feats > 32 ||
      c.gcn > 4 || c.layers > 16)
    return set_error(HP_E_SHAPE, "network: supported d = 128, heads = 4 (head dim 32), edge_hidden <= 64, "
                                 "gcn <= 4, layers <= 16, node_feats + glob_feats <= 32");
  return HP_OK;
}

static hp_status network_alloc_impl(Batch& b);

// The network workspace (about 12 KB per node) is allocated by the first
// call that runs the network, so a batch used only for solves and applies
// holds the solver's workspace alone.  A failed allocation leaves no
// half-built workspace behind (its buffers are released with the batch).
hp_status network_alloc(Batch& b) {
  if (b.net.ws) return HP_OK;
  HP_TRY(network_supported(b.cfg));
  const hp_status s = network_alloc_impl(b);
  if (s != HP_OK && b.net.ws) {
    b.net_free(b.net.ws);
    b.net.ws = nullptr;
  }
  return s;
}

static hp_status network_alloc_impl(Batch& b) {
  auto* N = new NetBufs();
  b.net.ws = N;
  b.net_free = [](void* p) { delete reinterpret_cast<NetBufs*>(p); };
  const hp_model_config& c = b.cfg;
  N->plan = make_plan(c);
  const int64_t Nd = b.ntot, No = std::max<int64_t>(b.mtot, 1) * c.rank, d = c.d;
  N->Nd = Nd;
  N->No = No;
  hp_status s = HP_OK;
  auto A = [&](auto** p, size_t bytes) {
    if (s == HP_OK) s = b.alloc((void**)p, bytes);
  };
  A(&N->feats, Nd * 32 * 4);
  A(&N->H, Nd * d * 4);
  A(&N->Henc, Nd * d * 4);
  A(&N->R, Nd * d * 4);
  A(&N->C, Nd * d * 4);
  A(&N->a128, Nd * d * 4);
  A(&N->b128, Nd * d * 4);
  A(&N->qkv, Nd * 3 * d * 4);
  A(&N->u512, Nd * 4 * d * 4);
  A(&N->h512, Nd * 4 * d * 4);
  A(&N->Xo, No * d * 4);
  A(&N->Xo0, No * d * 4);
  A(&N->ctx, No * 2 * d * 4);
  A(&N->ctxf, No * 2 * d * 4);
  A(&N->hrs, b.ktot * c.rank * d * 4);
  A(&N->hcs, b.ktot * c.rank * d * 4);
  A(&N->hhr, b.ktot * c.rank * d * 4);
  A(&N->hhc, b.ktot * c.rank * d * 4);
  std::vector<int2> stab;
  std::vector<int> strip0(b.nframes, 0);
  for (int f = 0; f < b.nframes; ++f) {
    strip0[f] = (int)stab.size();
    if (b.fr[f].MH == 0) continue;
    const int C = std::min(STRIP_CHUNK, b.fr[f].K);
    for (int q = 0; q < b.fr[f].K / C; ++q) stab.push_back(make_int2(f, q));
  }
  N->nstrip = (int)stab.size();
  A(&N->eslots, EDGE_CST * 4);
  std::vector<int2> ltab;
  std::vector<int> lvl0(b.nframes, 0);
  for (int f = 0; f < b.nframes; ++f) {
    lvl0[f] = (int)ltab.size();
    const int C = std::min(STRIP_CHUNK, b.fr[f].K);
    for (int q = 0; q < b.fr[f].K / C; ++q) ltab.push_back(make_int2(f, q));
  }
  N->nlvl = (int)ltab.size();
  A(&N->lvl_tab, std::max<size_t>(ltab.size(), 1) * sizeof(int2));
  A(&N->lvl0, std::max(b.nframes, 1) * 4);
  A(&N->lvl_top, std::max<size_t>(ltab.size(), 1) * c.rank * 2 * d * 4);
  A(&N->strip_tab, std::max<size_t>(stab.size(), 1) * sizeof(int2));
  A(&N->strip0, std::max(b.nframes, 1) * 4);
  A(&N->strip_tot, std::max<size_t>(stab.size(), 1) * c.rank * 2 * d * 4);
  A(&N->ao128, No * d * 4);
  A(&N->bo128, No * d * 4);
  A(&N->qkvo, No * 3 * d * 4);
  A(&N->uo512, No * 4 * d * 4);
  A(&N->ho512, No * 4 * d * 4);
  A(&N->Frows, Nd * c.leaf * 4);
  A(&N->NH, Nd * 36 * 4);
  A(&N->UV, No * 2 * c.rank * 4);
  A(&N->T0, (size_t)c.heads * c.leaf * c.leaf * 4);
  A(&N->corr, Nd * 7 * c.heads * 4);
  A(&N->ahat, Nd * 7 * 4);
  A(&N->nbr, Nd * 7);
  A(&N->desc, std::max<int64_t>(b.mtot, 1) * c.rank * c.rank * 4 * 4);
  A(&N->boff, std::max<int64_t>(b.mtot, 1) * c.heads * c.rank * c.rank * 4);
  {
    const size_t nl = (size_t)std::max(c.layers, 1);
    A(&N->T0l, nl * c.heads * c.leaf * c.leaf * 4);
    A(&N->eslotsl, nl * EDGE_CST * 4);
    A(&N->corrl, nl * Nd * 7 * c.heads * 4);
    A(&N->boffl, nl * std::max<int64_t>(b.mtot, 1) * c.heads * c.rank * c.rank * 4);
  }
  A(&N->G, b.nframes * d * 4);
  A(&N->gcount, b.nframes * 4);
  A(&N->glob, b.nframes * 12 * 4);
  A(&N->bias_node, 64 * 4);
  A(&N->bias_uv, 64 * 4);
  A(&N->warena, N->plan.arena * 4);
  A(&N->d_conv, N->plan.conv.size() * sizeof(ConvDesc));
  A(&N->d_tiles, N->plan.tiles.size() * sizeof(int4));
  A(&N->node2f, Nd * 4);
  A(&N->tok2f, No * 4);
  A(&N->tile2f, std::max<int64_t>(b.mtot, 1) * 4);
  A(&N->chunk0, (b.nframes + 1) * 4);
  if (s != HP_OK) return s;
  // maps and chunk tables
  std::vector<int> node2f(Nd), tok2f(No, 0), tile2f(std::max<int64_t>(b.mtot, 1), 0), chunk0(b.nframes + 1);
  std::vector<SumChunk> ch;
  std::vector<float> cnt(b.nframes);
  for (int f = 0; f < b.nframes; ++f) {
    const FrameDesc& F = b.fr[f];
    for (int i = 0; i < F.n; ++i) node2f[F.n0 + i] = f;
    for (int m = 0; m < F.MH; ++m) {
      tile2f[F.m0 + m] = f;
      for (int t = 0; t < c.rank; ++t) tok2f[(int64_t)(F.m0 + m) * c.rank + t] = f;
    }
    chunk0[f] = (int)ch.size();
    for (int r = 0; r < F.n; r += SUM_CHUNK)
      ch.push_back(SumChunk{f, 0, (int64_t)F.n0 + r, std::min(SUM_CHUNK, F.n - r)});
    if (c.offdiag)
      for (int r = 0; r < F.MH * c.rank; r += SUM_CHUNK)
        ch.push_back(SumChunk{f, 1, (int64_t)F.m0 * c.rank + r, std::min(SUM_CHUNK, F.MH * c.rank - r)});
    cnt[f] = (float)(F.n + (c.offdiag ? F.MH * c.rank : 0));
  }
  chunk0[b.nframes] = (int)ch.size();
  N->nchunks = (int)ch.size();
  std::vector<DescChunk> dch;
  std::vector<int> dch0(std::max<int64_t>(b.mtot, 1) + 1, 0);
  for (int f = 0; f < b.nframes; ++f) {
    const FrameDesc& F = b.fr[f];
    for (int m = 0; m < F.MH; ++m) {
      int j = 0;
      while (m >= F.K - (F.K >> (j + 1))) ++j;
      dch0[F.m0 + m] = (int)dch.size();
      for (int k = 0; k < (1 << j); k += DESC_CHUNK)
        dch.push_back(DescChunk{F.m0 + m, k, std::min(1 << j, k + DESC_CHUNK)});
    }
  }
  dch0[b.mtot] = (int)dch.size();
  N->ndesc_chunks = (int)dch.size();
  A(&N->desc_chunks, std::max<size_t>(dch.size(), 1) * sizeof(DescChunk));
  A(&N->desc_chunk0, dch0.size() * sizeof(int));
  A(&N->desc_part, std::max<size_t>(dch.size(), 1) * (c.rank * c.rank + 6 * c.rank) * sizeof(double));
  A(&N->chunks, ch.size() * sizeof(SumChunk));
  A(&N->gpart, ch.size() * 128 * 4);
  if (s != HP_OK) return s;
  auto up = [&](void* dst, const void* src, size_t n) {
    if (s == HP_OK && hipMemcpy(dst, src, n, hipMemcpyHostToDevice) != hipSuccess)
      s = set_error(HP_E_HIP, "network_alloc: upload failed");
  };
  up(N->node2f, node2f.data(), Nd * 4);
  up(N->tok2f, tok2f.data(), No * 4);
  up(N->tile2f, tile2f.data(), tile2f.size() * 4);
  up(N->chunk0, chunk0.data(), chunk0.size() * 4);
  up(N->chunks, ch.data(), ch.size() * sizeof(SumChunk));
  if (!stab.empty()) up(N->strip_tab, stab.data(), stab.size() * sizeof(int2));
  if (b.nframes > 0) up(N->strip0, strip0.data(), strip0.size() * 4);
  if (!ltab.empty()) up(N->lvl_tab, ltab.data(), ltab.size() * sizeof(int2));
  if (b.nframes > 0) up(N->lvl0, lvl0.data(), lvl0.size() * 4);
  if (!dch.empty()) up(N->desc_chunks, dch.data(), dch.size() * sizeof(DescChunk));
  up(N->desc_chunk0, dch0.data(), dch0.size() * sizeof(int));
  up(N->gcount, cnt.data(), cnt.size() * 4);
  up(N->d_conv, N->plan.conv.data(), N->plan.conv.size() * sizeof(ConvDesc));
  up(N->d_tiles, N->plan.tiles.data(), N->plan.tiles.size() * sizeof(int4));
  if (s == HP_OK && hipMemset(N->warena, 0, N->plan.arena * 4) != hipSuccess)
    s = set_error(HP_E_HIP, "network_alloc: memset failed");
  return s;
}

// BF16 tile kernel with a deeper K pipeline: K steps of 32 pass through an
// LDS ring of ST stages filled straight from global memory
// (global_load_lds_dwordx4: one wave instruction writes 1 KB = 16 rows of 64
// bytes, lane i -> row i / 4, 16-byte position i % 4), so ST - 1 steps of
// loads are in flight while a step is multiplied.  Rows are unpadded; the
// 16-byte chunk c of row r sits at position c ^ ((r / 4) % 4), which keeps
// the 16-byte operand reads of 16 consecutive rows on distinct banks.  Rows
// past M (or N) load the last row; they only feed outputs that are not
// stored.  Same MFMA sequence along K and same epilogue as k_gemm_bt, so the
// results are bit-identical to it.
// Two blocks per CU (their rings fit the LDS together) need at most 128 VGPRs
// per lane: four waves per SIMD.
template <int BM, int BN, int WM, int WN, int ST>
__global__ __launch_bounds__((BM / WM) * (BN / WN) * 64) __attribute__((amdgpu_waves_per_eu(4)))
void k_gemm_dl(GemmArgs a, int tiles_n) {
  constexpr int NWN = BN / WN, NW = (BM / WM) * NWN, BK = 32, FM = WM / 32, FN = WN / 32;
  constexpr int BLK = (BM + BN) / 16, LPW = BLK / NW;  // 1 KB blocks per stage, per wave
  static_assert(BLK % NW == 0, "stage blocks do not split over the waves");
  static_assert(ST >= 3, "at least three stages");
  __shared__ __attribute__((aligned(1024))) uint16_t ring[ST][(BM + BN) * BK];
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int nblk = (int)gridDim.x, id = (int)blockIdx.x;
  const int lin = (nblk % 8 == 0) ? (id % 8) * (nblk / 8) + id / 8 : id;
  const int m0 = (lin / tiles_n) * BM, n0 = (lin % tiles_n) * BN;
  const int wm = (wave / NWN) * WM, wn = (wave % NWN) * WN;
  const uint16_t* X = (const uint16_t*)a.X;
  const uint16_t* W = (const uint16_t*)a.Wt;
  // this lane's source row and chunk for each of the wave's blocks (k offset added per step)
  const uint16_t* src[LPW];
#pragma unroll
  for (int q = 0; q < LPW; ++q) {
    const int blk = wave * LPW + q, crow = 16 * blk + (lane >> 2);  // row of the combined [A | B] stage
    const int c = (lane & 3) ^ ((crow >> 2) & 3);                   // the chunk that lands at position lane % 4
    src[q] = crow < BM ? X + (int64_t)min(m0 + crow, a.M - 1) * a.ldx + 8 * c
                       : W + (int64_t)min(n0 + crow - BM, a.N - 1) * a.K + 8 * c;
  }
  auto issue = [&](int slot, int k0) {
#pragma unroll
    for (int q = 0; q < LPW; ++q) {
      const int blk = wave * LPW + q;
      __builtin_amdgcn_global_load_lds((const __attribute__((address_space(1))) void*)(src[q] + k0),
                                       (__attribute__((address_space(3))) void*)&ring[slot][blk * 512], 16, 0, 0);
    }
  };
  // 16-byte operand of row r (of the A part, or of the B part at row BM + r), k chunk c
  auto opnd = [&](int slot, int row, int c) {
    return __builtin_bit_cast(bf16x8_t, *(const uint4*)&ring[slot][row * BK + 8 * (c ^ ((row >> 2) & 3))]);
  };
  f32x16_t acc[FM][FN];
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j)
#pragma unroll
      for (int q = 0; q < 16; ++q) acc[i][j][q] = 0.f;
  const int nk = a.K / BK;
#pragma unroll
  for (int s2 = 0; s2 < ST - 1; ++s2)
    if (s2 < nk) issue(s2, s2 * BK);
  for (int kt = 0; kt < nk; ++kt) {
    // step kt has landed once only the later steps' loads are outstanding
    if (kt + ST - 2 < nk) asm volatile("s_waitcnt vmcnt(%0)" ::"n"((ST - 2) * LPW) : "memory");
    else asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    // a bare barrier (__syncthreads' fence would wait for every load in
    // flight): this wave's reads of step kt - 1 are done, its part of step kt
    // has landed, so after the barrier every part of step kt is in LDS and
    // step kt - 1's slot may be refilled
    asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
    __builtin_amdgcn_s_barrier();
    asm volatile("" ::: "memory");
    if (kt + ST - 1 < nk) issue((kt + ST - 1) % ST, (kt + ST - 1) * BK);
    const int slot = kt % ST;
#pragma unroll
    for (int kk = 0; kk < BK; kk += 16) {
      const int c = kk / 8 + (lane >> 5);
      bf16x8_t av[FM], bv[FN];
#pragma unroll
      for (int i = 0; i < FM; ++i) av[i] = opnd(slot, wm + 32 * i + (lane & 31), c);
#pragma unroll
      for (int j = 0; j < FN; ++j) bv[j] = opnd(slot, BM + wn + 32 * j + (lane & 31), c);
#pragma unroll
      for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(bv[j], av[i], acc[i][j], 0, 0, 0);
    }
  }
  // A full block tile whose only output is the BF16 one leaves through LDS:
  // from the fragments a lane holds 8 bytes of each of 4 column groups of one
  // row, so a direct store sends 32 rows' pieces per instruction; restaged,
  // 8 lanes write one row's 128 contiguous bytes.  The values are those of
  // the direct epilogue (bias, activation, BF16 rounding).
  static_assert(NW * WM * WN <= ST * (BM + BN) * BK, "staging tiles exceed the ring");
  if (a.Yb && !a.Yf && !a.resid && !a.pre && m0 + BM <= a.M && n0 + BN <= a.N &&
      (((uintptr_t)a.Yb | (uintptr_t)(2 * a.ldb)) & 15) == 0) {
    __syncthreads();  // every wave is done with the ring's operands
    uint16_t* stg = &ring[0][0] + wave * (WM * WN);
    // element (r, col) of the wave's WM x WN tile; the 16-byte chunks of each
    // 128-byte LDS line are XOR-swizzled by the line index, so the fragment
    // writes (32 rows at once) and the row reads both spread over all banks
    auto at = [&](int r, int col) {
      const int byte = 2 * (r * WN + col), line = byte >> 7;
      return ((line << 7) | (((byte >> 4) & 7) ^ (line & 7)) << 4 | (byte & 15)) >> 1;
    };
    // the activation as a compile-time choice: branch-free per-element code
    auto fill = [&](auto gelu_tag) {
      constexpr bool GELU = decltype(gelu_tag)::value;
#pragma unroll
      for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j) {
          const int cl = 32 * j + 4 * (lane >> 5);
          float bv[16];
          gemm_bias16(a, n0 + wn + cl, bv);
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            float v[4];
#pragma unroll
            for (int c = 0; c < 4; ++c) {
              v[c] = acc[i][j][4 * q + c] + bv[4 * q + c];
              if constexpr (GELU) v[c] = gelu_bf16path(v[c]);
            }
            *(uint2*)&stg[at(32 * i + (lane & 31), cl + 8 * q)] =
                make_uint2(pack_bf16x2(v[0], v[1]), pack_bf16x2(v[2], v[3]));
          }
        }
    };
    if (a.act == 1) fill(std::true_type{});
    else fill(std::false_type{});
    // the wave reads back only its own tile, and one wave's LDS accesses
    // complete in order
    asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
    constexpr int LPR = WN / 8, RPI = 64 / LPR;  // lanes per row, rows per store
    uint16_t* yb = (uint16_t*)a.Yb + (int64_t)(m0 + wm) * a.ldb + n0 + wn;
#pragma unroll
    for (int t = 0; t < WM / RPI; ++t) {
      const int r = t * RPI + lane / LPR, col = 8 * (lane % LPR);
      *(uint4*)(yb + (int64_t)r * a.ldb + col) = *(const uint4*)&stg[at(r, col)];
    }
    return;
  }
  // With an FP32 output or a residual (and no pre-activation copy) a full
  // tile goes through LDS as FP32 in passes of 32 rows: a lane then reads
  // and writes 16 contiguous bytes and a row's columns leave together; the
  // residual is read the same way.  Same values as the direct epilogue.
  static_assert(NW * 32 * WN * 4 <= ST * (BM + BN) * BK * 2, "FP32 staging tiles exceed the ring");
  if (!a.pre && (a.Yf || a.resid) && m0 + BM <= a.M && n0 + BN <= a.N && gemm_vec_ok(a, 2)) {
    __syncthreads();  // every wave is done with the ring's operands
    float* stg = (float*)&ring[0][0] + wave * (32 * WN);
    auto at = [&](int r, int col) {
      const int byte = 4 * (r * WN + col), line = byte >> 7;
      return ((line << 7) | (((byte >> 4) & 7) ^ (line & 7)) << 4 | (byte & 15)) >> 2;
    };
    constexpr int LPR = WN / 4, RPI = 64 / LPR;  // lanes per row, rows per access
    auto fill = [&](int i, auto gelu_tag) {
      constexpr bool GELU = decltype(gelu_tag)::value;
#pragma unroll
      for (int j = 0; j < FN; ++j) {
        const int cl = 32 * j + 4 * (lane >> 5);
        float bv[16];
        gemm_bias16(a, n0 + wn + cl, bv);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          float v[4];
#pragma unroll
          for (int c = 0; c < 4; ++c) {
            v[c] = acc[i][j][4 * q + c] + bv[4 * q + c];
            if constexpr (GELU) v[c] = gelu_bf16path(v[c]);
          }
          *(float4*)&stg[at(lane & 31, cl + 8 * q)] = make_float4(v[0], v[1], v[2], v[3]);
        }
      }
    };
#pragma unroll
    for (int i = 0; i < FM; ++i) {
      if (a.act == 1) fill(i, std::true_type{});
      else fill(i, std::false_type{});
      // the wave reads back only its own rows, and one wave's LDS accesses
      // complete in order (so the next pass may overwrite them after these reads)
      asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
#pragma unroll
      for (int t = 0; t < 32 / RPI; ++t) {
        const int r = t * RPI + lane / LPR, col = 4 * (lane % LPR);
        const float4 u = *(const float4*)&stg[at(r, col)];
        const int64_t row = m0 + wm + 32 * i + r;
        const int gc = n0 + wn + col;
        float v[4] = {u.x, u.y, u.z, u.w};
        if (a.resid) {
          const float4 rr = *(const float4*)(a.resid + row * a.ldr + gc);
          v[0] += rr.x;
          v[1] += rr.y;
          v[2] += rr.z;
          v[3] += rr.w;
        }
        if (a.Yf) *(float4*)(a.Yf + row * a.ldf + gc) = make_float4(v[0], v[1], v[2], v[3]);
        if (a.Yb)
          *(uint2*)((uint16_t*)a.Yb + row * a.ldb + gc) = make_uint2(pack_bf16x2(v[0], v[1]), pack_bf16x2(v[2], v[3]));
      }
      asm volatile("" ::: "memory");
    }
    return;
  }
  const bool vec = gemm_vec_ok(a, 2);
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j)
      gemm_epilogue<uint16_t>(a, acc[i][j], m0 + wm + 32 * i + (lane & 31), n0 + wn + 32 * j + 4 * (lane >> 5), vec);
}

// BF16 GEMM variants, indexed by the autotuner's "kind": block tile BM x BN,
// K step BK (K must be a multiple of it), waves.
struct GemmVar {
  const char* name;
  int bk;
};
static const GemmVar kGemmVars[] = {
    {"64x64x32", 32},       {"128x128x32", 32},      {"64x64x64", 64},          {"128x64x64", 64},
    {"128x128x32w8", 32},   {"256x128x32w8", 32},    {"128x128x32w8pf2", 32},   {"256x128x32w8pf2", 32},
    {"64x64x64pf2", 64},    {"128x128x64w8", 64},    {"128x256x32w8", 32},
    {"dl128x128x32s4", 32}, {"dl256x128x32s3", 32},  {"dl128x256x32s3", 32},
};
constexpr int kNumGemmVars = (int)(sizeof(kGemmVars) / sizeof(kGemmVars[0]));
int gemm_variant_count() { return kNumGemmVars; }
const char* gemm_variant_name(int v) { return v >= 0 && v < kNumGemmVars ? kGemmVars[v].name : "?"; }
static bool gemm_variant_fits(int v, int K) { return v >= 0 && v < kNumGemmVars && K % kGemmVars[v].bk == 0; }

template <int BM, int BN, int BK, int WM, int WN, int PF = 1>
static void launch_bt(const GemmArgs& a, hipStream_t st) {
  const int tn = (a.N + BN - 1) / BN, tm = (a.M + BM - 1) / BM;
  hipLaunchKernelGGL((k_gemm_bt<BM, BN, BK, WM, WN, PF>), dim3((unsigned)(tm * tn)), dim3((BM / WM) * (BN / WN) * 64),
                     0, st, a, tn);
}

template <int BM, int BN, int WM, int WN, int ST>
static void launch_dl(const GemmArgs& a, hipStream_t st) {
  const int tn = (a.N + BN - 1) / BN, tm = (a.M + BM - 1) / BM;
  hipLaunchKernelGGL((k_gemm_dl<BM, BN, WM, WN, ST>), dim3((unsigned)(tm * tn)), dim3((BM / WM) * (BN / WN) * 64), 0,
                     st, a, tn);
}

static void launch_gemm(int kind, const GemmArgs& a, bool bf16, hipStream_t st) {
  if (!bf16) {
    const unsigned nb = (unsigned)(((a.M + 63) / 64) * ((a.N + 63) / 64));
    hipLaunchKernelGGL(k_gemm<float>, dim3(nb), dim3(256), 0, st, a);
    return;
  }
  switch (kind) {
    case 1: launch_bt<128, 128, 32, 64, 64>(a, st); break;
    case 2: launch_bt<64, 64, 64, 32, 32>(a, st); break;
    case 3: launch_bt<128, 64, 64, 64, 32>(a, st); break;
    case 4: launch_bt<128, 128, 32, 64, 32>(a, st); break;
    case 5: launch_bt<256, 128, 32, 64, 64>(a, st); break;
    case 6: launch_bt<128, 128, 32, 64, 32, 2>(a, st); break;
    case 7: launch_bt<256, 128, 32, 64, 64, 2>(a, st); break;
    case 8: launch_bt<64, 64, 64, 32, 32, 2>(a, st); break;
    case 9: launch_bt<128, 128, 64, 64, 32>(a, st); break;
    case 10: launch_bt<128, 256, 32, 64, 64>(a, st); break;
    case 11: launch_dl<128, 128, 64, 32, 4>(a, st); break;
    case 12: launch_dl<256, 128, 64, 64, 3>(a, st); break;
    case 13: launch_dl<128, 256, 64, 64, 3>(a, st); break;
    default: {
      const unsigned nb = (unsigned)(((a.M + 63) / 64) * ((a.N + 63) / 64));
      hipLaunchKernelGGL(k_gemm<uint16_t>, dim3(nb), dim3(256), 0, st, a);
    }
  }
}

// GEMM tile autotuner (BF16, N > 64): the first call of a shape (N, K, M) on
// a batch times every variant whose K step divides K (one warm launch each,
// then three rounds over the variants of two launches timed one by one, the
// fastest kept) with the call's outputs redirected to a scratch
// buffer, so tuning never touches the call's own outputs (in-place residual
// calls included); the call then runs once with the fastest.  All variants
// compute bit-identical results.  Under stream capture, with tuning off, or if
// the scratch buffer cannot be had, a shape takes the choice recorded for the
// same (N, M) at the nearest K, else the 128 x 128 kernel.
static int gemm_choice(Batch& b, const GemmArgs& a, hipStream_t st) {
  const auto key = std::make_tuple(a.N, a.K, (int64_t)a.M);
  auto it = b.gemm_pick.find(key);
  if (it != b.gemm_pick.end()) return it->second.pick;
  auto fallback = [&]() {
    int best = 1, dk = 1 << 30;
    for (const auto& kv : b.gemm_pick)
      if (std::get<0>(kv.first) == a.N && std::get<2>(kv.first) == (int64_t)a.M &&
          std::abs(std::get<1>(kv.first) - a.K) < dk && gemm_variant_fits(kv.second.pick, a.K)) {
        dk = std::abs(std::get<1>(kv.first) - a.K);
        best = kv.second.pick;
      }
    return best;
  };
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  hipStreamIsCapturing(st, &cs);
  if (!b.gemm_autotune || cs != hipStreamCaptureStatusNone) return fallback();
  size_t need = 0;
  if (a.Yf) need = std::max(need, (size_t)a.M * (size_t)a.ldf * 4);
  if (a.Yb) need = std::max(need, (size_t)a.M * (size_t)a.ldb * 2);
  if (a.pre) need = std::max(need, (size_t)a.M * (size_t)a.ldp * 4);
  void* scratch = nullptr;
  if (need == 0 || hipMalloc(&scratch, need) != hipSuccess) {
    (void)hipGetLastError();
    return fallback();
  }
  // the inference's other streams would share the GPU with the timed launches
  hipDeviceSynchronize();
  GemmArgs t = a;
  if (t.Yf) t.Yf = (float*)scratch;
  if (t.Yb) t.Yb = scratch;
  if (t.pre) t.pre = (float*)scratch;
  // rounds over all variants (so drifting clocks affect every variant alike),
  // each variant's fastest timed launch kept
  constexpr int ROUNDS = 3, REPS = 2;
  hipEvent_t ev[REPS + 1];
  for (auto& e : ev) hipEventCreate(&e);
  GemmPick g;
  g.pick = 1;
  g.us.assign(kNumGemmVars, -1.f);
  for (int kind = 0; kind < kNumGemmVars; ++kind)
    if (gemm_variant_fits(kind, a.K)) launch_gemm(kind, t, true, st);  // warm
  for (int round = 0; round < ROUNDS; ++round) {
    for (int kind = 0; kind < kNumGemmVars; ++kind) {
      if (!gemm_variant_fits(kind, a.K)) continue;
      hipEventRecord(ev[0], st);
      for (int r = 0; r < REPS; ++r) {
        launch_gemm(kind, t, true, st);
        hipEventRecord(ev[r + 1], st);
      }
      hipEventSynchronize(ev[REPS]);
      for (int r = 0; r < REPS; ++r) {
        float ms = 0.f;
        hipEventElapsedTime(&ms, ev[r], ev[r + 1]);
        if (g.us[kind] < 0.f || ms * 1e3f < g.us[kind]) g.us[kind] = ms * 1e3f;
      }
    }
  }
  for (int kind = 0; kind < kNumGemmVars; ++kind)
    if (g.us[kind] >= 0.f && (g.us[kind] < g.us[g.pick] || g.us[g.pick] < 0.f)) g.pick = kind;
  for (auto& e : ev) hipEventDestroy(e);
  hipFree(scratch);
  b.gemm_pick[key] = g;
  return g.pick;
}

template <typename AT>
static void gemm(Batch& b, const void* X, int64_t ldx, const NetBufs& NB, const GemmW& w, const float* bias,
                 const float* resid, int64_t ldr, float* Yf, int64_t ldf, void* Yb, int64_t ldb, int64_t M, int act,
                 float* pre = nullptr, int64_t ldp = 0) {
  if (M <= 0) return;
  hipStream_t st = b.stream;
  GemmArgs a;
  a.X = X;
  a.ldx = ldx;
  a.Wt = (const AT*)NB.warena + w.off;
  a.K = w.K;
  a.bias = bias;
  a.resid = resid;
  a.ldr = ldr;
  a.Yf = Yf;
  a.ldf = ldf;
  a.Yb = Yb;
  a.ldb = ldb;
  a.pre = pre;
  a.ldp = ldp;
  a.M = (int)M;
  a.N = w.N;
  a.act = act;
  const bool bf16 = sizeof(AT) == 2;
  int kind = 0;
  if (bf16 && w.N > 64)
    kind = gemm_variant_fits(b.gemm_variant, a.K) ? b.gemm_variant : b.gemm_variant >= 0 ? 0 : gemm_choice(b, a, st);
  const bool timed = (b.prof.kind == PROF_GEMM || b.prof.kind == PROF_GEMM_BYTES) &&
                     2 * (b.prof.used + 1) <= (int)b.prof.ev.size();
  if (timed) hipEventRecord(b.prof.ev[2 * b.prof.used], st);
  launch_gemm(kind, a, bf16, st);
  if (timed) {
    hipEventRecord(b.prof.ev[2 * b.prof.used + 1], st);
    b.prof.used++;
    if (b.prof.kind == PROF_GEMM) {
      b.prof.work += 2.0 * (double)M * w.N * w.K;
    } else {
      // algorithmic HBM bytes: X and W once, bias, and each output / residual once
      const double s = (double)sizeof(AT), mn = (double)M * w.N;
      b.prof.work += s * ((double)M * w.K + (double)w.N * w.K) + (bias ? 4.0 * w.N : 0.0) + (resid ? 4.0 * mn : 0.0) +
                     (Yf ? 4.0 * mn : 0.0) + (Yb ? s * mn : 0.0) + (pre ? 4.0 * mn : 0.0);
    }
  }
}

// The fused FFN (BF16 inference): X += GELU(U W1 + b1) W2 + b2, timed with
// the GEMMs when GEMM timing is on (work: the two products' flops, or the
// algorithmic bytes U, W1, W2, biases, X read and written).
// Launches the fused FFN where its layout assumptions hold (d = 128, hidden
// 512, 16-byte aligned biases); returns false to leave the FFN to the two GEMMs.
static bool ffn_fused(Batch& b, const void* U, const NetBufs& NB, const GemmW& w1, const float* b1, const GemmW& w2,
                      const float* b2, float* X, int64_t M) {
  if (w1.N != 512 || w1.K != 512 || w2.N != 128 || w2.K != 512 || ((uintptr_t)b1 & 15) || ((uintptr_t)b2 & 15) ||
      ((uintptr_t)X & 15) || ((uintptr_t)U & 15))
    return false;
  if (M <= 0) return true;
  hipStream_t st = b.stream;
  const int pk = b.prof.kind;
  const bool timed = (pk == PROF_GEMM || pk == PROF_GEMM_BYTES || pk == PROF_FFN || pk == PROF_FFN_BYTES) &&
                     2 * (b.prof.used + 1) <= (int)b.prof.ev.size();
  if (timed) hipEventRecord(b.prof.ev[2 * b.prof.used], st);
  hipLaunchKernelGGL(k_ffn_fused, dim3((unsigned)((M + 127) / 128)), dim3(256), 0, st, (const uint16_t*)U,
                     (const uint16_t*)NB.warena + w1.off, b1, (const uint16_t*)NB.warena + w2.off, b2, X, (int)M);
  if (timed) {
    hipEventRecord(b.prof.ev[2 * b.prof.used + 1], st);
    b.prof.used++;
    const double m = (double)M;
    if (pk == PROF_GEMM || pk == PROF_FFN)
      b.prof.work += 2.0 * m * w1.N * w1.K + 2.0 * m * w2.N * w2.K;
    else
      b.prof.work += 2.0 * (m * w1.K + (double)w1.N * w1.K + (double)w2.N * w2.K) + 4.0 * (w1.N + w2.N) +
                     8.0 * m * w2.N;
  }
  return true;
}

// Training saves of the forward pass (FP32).
struct TrainSave {
  float* Hg[5];                      // encoder: input of each GCN layer, then the encoder output
  float* xin_d[17];                  // residual streams entering each layer (and after the last)
  float* xin_o[17];
};
struct LayerSave {
  float *xmid_d, *xmid_o;            // FFN residual inputs
  float *pre_d, *pre_o;              // FFN hidden pre-activations [M][4d]
};

// The heads' biases gathered for their GEMMs: [hut | hvt | hlam] and
// [hu | hv] (one launch instead of five small copies).
__global__ __launch_bounds__(64) void k_head_biases(const float* hut, const float* hvt, const float* hlam,
                                                    const float* hu, const float* hv, int LS, float* bias_node,
                                                    float* bias_uv) {
  const int t = threadIdx.x;
  if (t < LS) {
    bias_node[t] = hut[t];
    bias_uv[t] = hu[t];
  } else if (t < 2 * LS) {
    bias_node[t] = hvt[t - LS];
    bias_uv[t] = hv[t - LS];
  } else if (t == 2 * LS) {
    bias_node[t] = hlam[0];
  }
}

// Stencil slots (neighbour index and Ahat) of every node and the
// off-diagonal pair descriptors: functions of the system alone.
static void stencil_desc(Batch& b, const float* sys, hipStream_t st) {
  NetBufs& N = *nb_of(b);
  const hp_model_config& c = b.cfg;
  const int64_t Nd = N.Nd, L = c.leaf, LS = c.rank;
  const FrameDesc* fr = b.d_fr;
  if (c.offdiag && b.mtot > 0) {
    hipLaunchKernelGGL(k_off_desc_part, dim3((unsigned)N.ndesc_chunks), dim3(256), 0, st, fr, N.tile2f,
                       (const DescChunk*)N.desc_chunks, sys, b.ntot, (int)L, (int)LS, N.desc_part);
    hipLaunchKernelGGL(k_off_desc_final, dim3((unsigned)b.mtot), dim3(256), 0, st, fr, N.tile2f,
                       (const int*)N.desc_chunk0, (const double*)N.desc_part, (int)L, (int)LS, N.desc);
  }
  hipLaunchKernelGGL(k_leaf_stencil, dim3((unsigned)((Nd + 255) / 256)), dim3(256), 0, st, fr, N.node2f, sys, b.ntot,
                     (int)L, N.nbr, N.ahat);
}

// Where layer l's edge-bias tables live: the shared buffers, or the
// inference's per-layer copies.
struct EdgeTabs {
  float *T0, *eslots, *corr, *boff;
};
static EdgeTabs edge_tabs(const Batch& b, const NetBufs& N, int l) {
  if (!N.pre) return {N.T0, N.eslots, N.corr, N.boff};
  const hp_model_config& c = b.cfg;
  return {N.T0l + (size_t)l * c.heads * c.leaf * c.leaf, N.eslotsl + (size_t)l * EDGE_CST,
          N.corrl + (size_t)l * N.Nd * 7 * c.heads,
          N.boffl + (size_t)l * std::max<int64_t>(b.mtot, 1) * c.heads * c.rank * c.rank};
}

// Edge-bias tables of layers [l0, l0 + nl) of one stack (sidx 0: the
// within-leaf table T0, the slot constants and the stencil corrections; 1:
// the off-diagonal pair biases), from the edge MLP's FP32 weights, one launch
// per kernel with the layer as blockIdx.y.  Several layers at once need the
// inference's per-layer buffers (N.pre), whose layers lie a fixed stride apart.
static EdgeWs edge_ws(Batch& b, const float* W, int l0, int nl, int sidx) {
  const NetPlan& P = nb_of(b)->plan;
  auto wp = [&](const std::string& n) { return W + woff(P, n); };
  EdgeWs ws{};
  for (int q = 0; q < nl; ++q) {
    const std::string p = std::string(sidx ? "off" : "diag") + std::to_string(l0 + q) + ".";
    ws.w[q] = EdgeW{wp(p + "e1.w"), wp(p + "e1.b"), wp(p + "e2.w"), wp(p + "e2.b"), b.cfg.edge_hidden, b.cfg.heads};
  }
  return ws;
}

// with_table false: the within-leaf tables and slot constants were written
// already (by k_side_head).
template <typename AT>
static void edge_tables(Batch& b, const float* W, int l0, int nl, int sidx, hipStream_t st, bool with_table = true) {
  NetBufs& N = *nb_of(b);
  const hp_model_config& c = b.cfg;
  const int64_t Nd = N.Nd, L = c.leaf, LS = c.rank, H = c.heads;
  const EdgeWs ws = edge_ws(b, W, l0, nl, sidx);
  const EdgeTabs t = edge_tabs(b, N, l0), t1 = nl > 1 ? edge_tabs(b, N, l0 + 1) : t;
  const int64_t t0_stride = t1.T0 - t.T0, corr_stride = t1.corr - t.corr, boff_stride = t1.boff - t.boff;
  const int slot_stride = (int)(t1.eslots - t.eslots);
  if (sidx == 0) {
    const unsigned lowmask = (unsigned)(L - 1);
    const FrameDesc& F0 = b.fr[0];
    if (with_table)
      hipLaunchKernelGGL(k_edge_table<sizeof(AT) == 2>, dim3((unsigned)((L * L + 255) / 256 + 1), (unsigned)nl),
                         dim3(256), 0, st, ws, (int)L, F0.xm & lowmask, F0.ym & lowmask, F0.zm & lowmask, t.T0,
                         t.eslots, t0_stride, slot_stride);
    if (H == 4 && c.edge_hidden == 32)  // the paper's widths: compile-time loops
      hipLaunchKernelGGL((k_edge_corr<sizeof(AT) == 2, 4, 32>), dim3((unsigned)((Nd * 7 + 255) / 256), (unsigned)nl),
                         dim3(256), 0, st, ws, (const float*)t.eslots, (const uint8_t*)N.nbr, (const float*)N.ahat,
                         Nd, t.corr, slot_stride, corr_stride);
    else
      hipLaunchKernelGGL(k_edge_corr<sizeof(AT) == 2>, dim3((unsigned)((Nd * 7 + 255) / 256), (unsigned)nl),
                         dim3(256), 0, st, ws, (const float*)t.eslots, (const uint8_t*)N.nbr, (const float*)N.ahat,
                         Nd, t.corr, slot_stride, corr_stride);
  } else {
    const int64_t npairs = b.mtot * LS * LS;
    if (H == 4 && c.edge_hidden == 32)
      hipLaunchKernelGGL((k_edge_off<sizeof(AT) == 2, 4, 32>), dim3((unsigned)((npairs + 255) / 256), (unsigned)nl),
                         dim3(256), 0, st, ws, (const float*)N.desc, npairs, (int)LS, t.boff, boff_stride);
    else
      hipLaunchKernelGGL(k_edge_off<sizeof(AT) == 2>, dim3((unsigned)((npairs + 255) / 256), (unsigned)nl),
                         dim3(256), 0, st, ws, (const float*)N.desc, npairs, (int)LS, t.boff, boff_stride);
  }
}

// Features, encoder, pooled off-diagonal tokens, descriptors and stencils.
// With sv, the encoder's intermediate H values are saved for training.
template <typename AT>
static hp_status fwd_prologue(Batch& b, const float* W, const float* rho, const float* sys, TrainSave* sv) {
  NetBufs& N = *nb_of(b);
  const NetPlan& P = N.plan;
  const hp_model_config& c = b.cfg;
  hipStream_t st = b.stream;
  const int64_t Nd = N.Nd, d = c.d, L = c.leaf, LS = c.rank, H = c.heads;
  const int64_t No = b.mtot * LS;
  const bool use_off = c.offdiag && b.mtot > 0;
  const FrameDesc* fr = b.d_fr;
  auto wp = [&](const std::string& n) { return W + woff(P, n); };
  (void)fr; (void)use_off; (void)H; (void)No; (void)L; (void)LS;
  // weights -> transposed arena in the compute type
  // (training also converts the plain copies its input-gradient GEMMs read)
  const int ntiles = sv ? (int)P.tiles.size() : P.ntiles_fwd;
  hipLaunchKernelGGL(k_convert<AT>, dim3((unsigned)ntiles), dim3(256), 0, st, N.d_conv, (const int4*)N.d_tiles, W,
                     (AT*)N.warena);
  hipLaunchKernelGGL(k_head_biases, dim3(1), dim3(64), 0, st, wp("hut.b"), wp("hvt.b"), wp("hlam.b"), wp("hu.b"),
                     wp("hv.b"), (int)LS, N.bias_node, N.bias_uv);
  // features and encoder (Sec. 4.1)
  hipLaunchKernelGGL(k_frame_stats, dim3(b.nframes), dim3(1024), 0, st, fr, rho, sys, b.ntot, N.glob);
  hipLaunchKernelGGL(k_features<AT>, dim3(b.nblk), dim3(NODE_BLOCK), 0, st, fr, b.d_blk2f, rho, sys, b.ntot, N.glob,
                     (AT*)N.feats);
  gemm<AT>(b, N.feats, 32, N, P.enc1, wp("enc1.b"), nullptr, 0, nullptr, 0, N.a128, d, Nd, 1);
  gemm<AT>(b, N.a128, d, N, P.enc2, wp("enc2.b"), nullptr, 0, N.H, d, N.b128, d, Nd, 0);
  for (int g = 0; g < c.gcn; ++g) {
    if (sv) HP_HIP(hipMemcpyAsync(sv->Hg[g], N.H, Nd * d * 4, hipMemcpyDeviceToDevice, st));
    hipLaunchKernelGGL(k_gcn_spmm<AT>, dim3((unsigned)((Nd + 7) / 8)), dim3(256), 0, st, fr, N.node2f, sys, b.ntot,
                       (const float*)N.H, (AT*)N.a128);
    gemm<AT>(b, N.a128, d, N, P.gcn[g], wp("gcn" + std::to_string(g) + ".b"), N.H, d, N.H, d, N.b128, d, Nd, 1);
  }
  if (b.keep_stages) HP_HIP(hipMemcpyAsync(N.Henc, N.H, Nd * d * 4, hipMemcpyDeviceToDevice, st));
  if (sv) HP_HIP(hipMemcpyAsync(sv->Hg[c.gcn], N.H, Nd * d * 4, hipMemcpyDeviceToDevice, st));
  // off-diagonal tokens: pooled strip means through [W_r; W_c] (Sec. 4.2)
  if (use_off) {
    // strip means of the encoder output: group sums, then the dyadic strip tree
    // (both strips from the same sums; N.hhr is free until the first layer)
    hipLaunchKernelGGL(k_group_sums, dim3((unsigned)b.ktot), dim3(512), 0, st, fr, b.d_leaf2f, (const float*)N.H,
                       (int)L, (int)LS, N.hhr);
    hipLaunchKernelGGL(k_hw_strips_lo<AT>, dim3((unsigned)N.nstrip, (unsigned)LS), dim3(256), 0, st, fr,
                       (const int2*)N.strip_tab, (const float*)N.hhr, (const float*)N.hhr, (int)L, (int)LS, (AT*)N.ctx,
                       N.strip_tot);
    hipLaunchKernelGGL(k_hw_strips_hi<AT>, dim3((unsigned)b.nframes, (unsigned)LS), dim3(256), 0, st, fr,
                       (const int*)N.strip0, (const float*)N.strip_tot, (int)L, (int)LS, (AT*)N.ctx);
    gemm<AT>(b, N.ctx, 2 * d, N, P.pool, wp("pool.b"), nullptr, 0, N.Xo, d, nullptr, 0, No, 0);
    if (b.keep_stages) HP_HIP(hipMemcpyAsync(N.Xo0, N.Xo, No * d * 4, hipMemcpyDeviceToDevice, st));
  }
  if (!N.pre) stencil_desc(b, sys, st);  // else computed ahead with the per-layer tables
  HP_HIP(hipGetLastError());
  return HP_OK;
}

// One transformer block of both stacks (Sec. 4.2-4.3), in place on the
// residual streams N.H / N.Xo.  With ls, the FFN residual inputs and the
// FFN pre-activations are saved for the reverse pass.
template <typename AT>
static hp_status layer_fwd(Batch& b, const float* W, const float* sys, int l, LayerSave* ls) {
  NetBufs& N = *nb_of(b);
  const NetPlan& P = N.plan;
  const hp_model_config& c = b.cfg;
  // with N.par the off-diagonal sublayers go to the off stream (b.stream is
  // pointed there around them, so the GEMM helper launches there too)
  hipStream_t const main_st = b.stream;
  hipStream_t st = main_st;
  struct StreamRestore {
    Batch& b;
    hipStream_t s;
    ~StreamRestore() { b.stream = s; }
  } restore{b, main_st};
  auto stack_stream = [&](int sidx) {
    b.stream = (N.par && sidx == 1) ? b.offs : main_st;
    return b.stream;
  };
  const int64_t Nd = N.Nd, d = c.d, L = c.leaf, LS = c.rank, H = c.heads;
  const int64_t No = b.mtot * LS;
  const bool use_off = c.offdiag && b.mtot > 0;
  const FrameDesc* fr = b.d_fr;
  auto wp = [&](const std::string& n) { return W + woff(P, n); };
  (void)fr; (void)use_off; (void)H; (void)No; (void)L; (void)LS;
  const EdgeTabs tabs = edge_tabs(b, N, l);
  for (int sidx = 0; sidx < 2; ++sidx) {
    if (sidx == 1 && !use_off) continue;
    st = stack_stream(sidx);
    const std::string p = std::string(sidx ? "off" : "diag") + std::to_string(l) + ".";
    float* X = sidx ? N.Xo : N.H;
    const int64_t M = sidx ? No : Nd;
    void* a = sidx ? N.ao128 : N.a128;
    void* q = sidx ? N.qkvo : N.qkv;
    void* o = sidx ? N.bo128 : N.b128;
    if (sidx == 0 && sizeof(AT) == 2 && b.attn_fused && !b.attn_valu && !ls && L == 64 && H == 4 && d == 128 &&
        P.qkv[0][l].N == 384 && P.qkv[0][l].K == 128 && P.o[0][l].N == 128 && P.o[0][l].K == 128) {
      // the whole sublayer in one launch (LN1, QKV, attention, output projection)
      if (!N.pre) edge_tables<AT>(b, W, l, 1, sidx, st);
      else if (N.pre_side) HP_HIP(hipStreamWaitEvent(st, b.side_ev[l], 0));
      const uint16_t* wa = (const uint16_t*)N.warena;
      hipLaunchKernelGGL(k_attn_sublayer64, dim3((unsigned)b.ktot), dim3(256), 0, st, X, wp(p + "ln1.g"),
                         wp(p + "ln1.b"), wa + P.qkv[0][l].off, wp(p + "qkv.b"), wa + P.o[0][l].off, wp(p + "o.b"),
                         (const float*)tabs.T0, (const float*)tabs.corr, (const uint8_t*)N.nbr);
      continue;
    }
    hipLaunchKernelGGL(k_layernorm128<AT>, dim3((unsigned)((M + 15) / 16)), dim3(256), 0, st, (const float*)X,
                       wp(p + "ln1.g"), wp(p + "ln1.b"), (AT*)a, (int)M);
    gemm<AT>(b, a, d, N, P.qkv[sidx][l], wp(p + "qkv.b"), nullptr, 0, nullptr, 0, q, 3 * d, M, 0);
    if (!N.pre) edge_tables<AT>(b, W, l, 1, sidx, st);
    else if (N.pre_side && (sidx == 0 || N.par)) HP_HIP(hipStreamWaitEvent(st, b.side_ev[l], 0));
    if (sidx == 0) {
      if (sizeof(AT) == 2 && !b.attn_valu) {
        if (L == 64)
          hipLaunchKernelGGL(k_attention_mfma<64>, dim3((unsigned)b.ktot), dim3(256), 0, st, (const uint16_t*)q,
                             (uint16_t*)o, (const float*)tabs.T0, (const float*)tabs.corr, (const uint8_t*)N.nbr);
        else
          hipLaunchKernelGGL(k_attention_mfma<32>, dim3((unsigned)b.ktot), dim3(256), 0, st, (const uint16_t*)q,
                             (uint16_t*)o, (const float*)tabs.T0, (const float*)tabs.corr, (const uint8_t*)N.nbr);
      } else if (L == 64) {
        hipLaunchKernelGGL((k_attention<AT, 64, true>), dim3((unsigned)b.ktot, (unsigned)H), dim3(64), 0, st,
                           (const AT*)q, (AT*)o, (const float*)tabs.T0, (const float*)tabs.corr,
                           (const uint8_t*)N.nbr, (int)H);
      } else {
        hipLaunchKernelGGL((k_attention<AT, 32, true>), dim3((unsigned)b.ktot, (unsigned)H), dim3(64), 0, st,
                           (const AT*)q, (AT*)o, (const float*)tabs.T0, (const float*)tabs.corr,
                           (const uint8_t*)N.nbr, (int)H);
      }
    } else {
      if (sizeof(AT) == 2 && LS == 16 && !b.attn_valu)
        hipLaunchKernelGGL(k_attention_tile_mfma, dim3((unsigned)b.mtot), dim3(256), 0, st, (const uint16_t*)q,
                           (uint16_t*)o, (const float*)tabs.boff);
      else if (LS == 16)
        hipLaunchKernelGGL((k_attention<AT, 16, false>), dim3((unsigned)b.mtot, (unsigned)H), dim3(64), 0, st,
                           (const AT*)q, (AT*)o, (const float*)tabs.boff, nullptr, nullptr, (int)H);
      else
        hipLaunchKernelGGL((k_attention<AT, 8, false>), dim3((unsigned)b.mtot, (unsigned)H), dim3(64), 0, st,
                           (const AT*)q, (AT*)o, (const float*)tabs.boff, nullptr, nullptr, (int)H);
    }
    gemm<AT>(b, o, d, N, P.o[sidx][l], wp(p + "o.b"), X, d, X, d, nullptr, 0, M, 0);
    if (N.par && sidx == 1) HP_HIP(hipEventRecord(b.off_ev[2 + 2 * l], st));
  }
  st = stack_stream(0);
  // the highways read both stacks' attention outputs
  if (N.par) HP_HIP(hipStreamWaitEvent(st, b.off_ev[2 + 2 * l], 0));
  // highways (Sec. 4.3)
  if (c.highways) {
    if (use_off) {
      hipLaunchKernelGGL(k_hw_levels_hi, dim3((unsigned)b.nframes, (unsigned)LS), dim3(256), 0, st, fr,
                         (const int*)N.lvl0, (const float*)N.Xo, (int)LS, N.lvl_top);
      hipLaunchKernelGGL(k_hw_levels_lo, dim3((unsigned)N.nlvl, (unsigned)LS), dim3(256), 0, st, fr,
                         (const int2*)N.lvl_tab, (const float*)N.lvl_top, (const float*)N.Xo, (int)LS, N.hrs, N.hcs);
      if (ls)  // the reverse pass reads r and c
        hipLaunchKernelGGL(k_hw_materialize, dim3((unsigned)((Nd + 1) / 2)), dim3(256), 0, st, fr, N.node2f,
                           (const float*)N.H, (const float*)N.hrs, (const float*)N.hcs, (int)L, (int)LS, Nd, N.R,
                           N.C);
    } else {
      HP_HIP(hipMemcpyAsync(N.R, N.H, Nd * d * 4, hipMemcpyDeviceToDevice, st));
      HP_HIP(hipMemcpyAsync(N.C, N.H, Nd * d * 4, hipMemcpyDeviceToDevice, st));
    }
    hipLaunchKernelGGL(k_chunk_sums, dim3((unsigned)N.nchunks), dim3(512), 0, st, (const SumChunk*)N.chunks,
                       (const float*)N.H, (const float*)N.Xo, N.gpart);
    hipLaunchKernelGGL(k_frame_mean, dim3(b.nframes), dim3(1024), 0, st, (const int*)N.chunk0,
                       (const float*)N.gpart, (const float*)N.gcount, N.G);
  }
  for (int sidx = 0; sidx < 2; ++sidx) {
    if (sidx == 1 && !use_off) continue;
    st = stack_stream(sidx);
    // the off-diagonal FFN's context comes from the group sums of the
    // diagonal LayerNorm (and its frame means from the highway step)
    if (N.par && sidx == 1) HP_HIP(hipStreamWaitEvent(st, b.off_ev[3 + 2 * l], 0));
    const std::string p = std::string(sidx ? "off" : "diag") + std::to_string(l) + ".";
    float* X = sidx ? N.Xo : N.H;
    const int64_t M = sidx ? No : Nd;
    void* u = sidx ? N.uo512 : N.u512;
    void* h = sidx ? N.ho512 : N.h512;
    if (sidx == 1 && c.highways && N.nstrip > 0) {
      // context of the off-diagonal tokens from the group sums the diagonal
      // LayerNorm wrote (taken before the diagonal FFN)
      hipLaunchKernelGGL(k_hw_strips_lo<float>, dim3((unsigned)N.nstrip, (unsigned)LS), dim3(256), 0, st, fr,
                         (const int2*)N.strip_tab, (const float*)N.hhr, (const float*)N.hhc, (int)L, (int)LS, N.ctxf,
                         N.strip_tot);
      hipLaunchKernelGGL(k_hw_strips_hi<float>, dim3((unsigned)b.nframes, (unsigned)LS), dim3(256), 0, st, fr,
                         (const int*)N.strip0, (const float*)N.strip_tot, (int)L, (int)LS, N.ctxf);
    }
    if (sidx == 0 && c.highways && use_off)
      hipLaunchKernelGGL(k_ln_hw_diag<AT>, dim3((unsigned)((M + 15) / 16)), dim3(256), 0, st, fr, N.node2f,
                         (const float*)X, (const float*)N.hrs, (const float*)N.hcs, (const float*)N.G, (int)L,
                         (int)LS, wp(p + "ln2.g"), wp(p + "ln2.b"), (AT*)u, N.hhr, N.hhc, (int)M);
    else if (sidx == 0)
      hipLaunchKernelGGL(k_ln_concat<AT>, dim3((unsigned)((M + 15) / 16)), dim3(256), 0, st, (const float*)X, d,
                         (const float*)N.R, d, (const float*)N.C, d, (const float*)N.G, (const int*)N.node2f,
                         wp(p + "ln2.g"), wp(p + "ln2.b"), (AT*)u, (int)M, c.highways);
    else
      hipLaunchKernelGGL(k_ln_concat<AT>, dim3((unsigned)((M + 15) / 16)), dim3(256), 0, st, (const float*)X, d,
                         (const float*)N.ctxf, 2 * d, (const float*)(N.ctxf + d), 2 * d, (const float*)N.G,
                         (const int*)N.tok2f, wp(p + "ln2.g"), wp(p + "ln2.b"), (AT*)u, (int)M, c.highways);
    if (N.par && sidx == 0) HP_HIP(hipEventRecord(b.off_ev[3 + 2 * l], st));
    if (ls) HP_HIP(hipMemcpyAsync(sidx ? ls->xmid_o : ls->xmid_d, X, M * d * 4, hipMemcpyDeviceToDevice, st));
    if (sizeof(AT) == 2 && !ls && b.ffn_fused &&
        ffn_fused(b, u, N, P.f1[sidx][l], wp(p + "f1.b"), P.f2[sidx][l], wp(p + "f2.b"), X, M)) {
    } else {
      gemm<AT>(b, u, 4 * d, N, P.f1[sidx][l], wp(p + "f1.b"), nullptr, 0, nullptr, 0, h, 4 * d, M, 1,
               ls ? (sidx ? ls->pre_o : ls->pre_d) : nullptr, 4 * d);
      gemm<AT>(b, h, 4 * d, N, P.f2[sidx][l], wp(p + "f2.b"), X, d, X, d, nullptr, 0, M, 0);
    }
  }
  HP_HIP(hipGetLastError());
  return HP_OK;
}

// The stencil slots, descriptors and every layer's edge-bias tables depend
// on the system and the weights only.  They are computed first, into
// per-layer buffers: on the side stream, beside the encoder and the early
// layers (layer l waits for its tables' event), or in order on the batch
// stream while a graph is being captured or kernels are being timed.
template <typename AT>
static hp_status tables_ahead(Batch& b, const float* W, const float* sys) {
  NetBufs& N = *nb_of(b);
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  HP_HIP(hipStreamIsCapturing(b.stream, &cs));
  N.pre = 1;
  // under a solve-step capture the side streams fork from and join back into
  // the capturing stream through events, so the graph keeps the overlap; they
  // exist from the eager inference that preceded the capture
  const bool fork_in_capture = b.capture_forks && b.side && b.side_start && b.side_done &&
                               (int)b.side_ev.size() >= b.cfg.layers &&
                               (!(b.cfg.offdiag && b.mtot > 0) ||
                                (b.offs && (int)b.off_ev.size() >= 2 + 2 * b.cfg.layers));
  N.pre_side = (cs == hipStreamCaptureStatusNone || fork_in_capture) && b.prof.kind == PROF_NONE;
  hipStream_t st = b.stream;
  if (N.pre_side) {
    if (!b.side) HP_HIP(hipStreamCreateWithFlags(&b.side, hipStreamNonBlocking));
    if (!b.side_start) HP_HIP(hipEventCreateWithFlags(&b.side_start, hipEventDisableTiming));
    if (!b.side_done) HP_HIP(hipEventCreateWithFlags(&b.side_done, hipEventDisableTiming));
    while ((int)b.side_ev.size() < b.cfg.layers) {
      hipEvent_t e;
      HP_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
      b.side_ev.push_back(e);
    }
    // after everything enqueued so far (an earlier inference's readers of
    // these buffers included)
    HP_HIP(hipEventRecord(b.side_start, b.stream));
    HP_HIP(hipStreamWaitEvent(b.side, b.side_start, 0));
    st = b.side;
  }
  const bool use_off = b.cfg.offdiag && b.mtot > 0;
  N.par = N.pre_side && use_off;
  if (N.par) {
    if (!b.offs) HP_HIP(hipStreamCreateWithFlags(&b.offs, hipStreamNonBlocking));
    while ((int)b.off_ev.size() < 2 + 2 * b.cfg.layers) {
      hipEvent_t e;
      HP_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
      b.off_ev.push_back(e);
    }
  }
  if (b.cfg.layers <= EDGE_LAYERS) {
    // descriptor chunks, leaf stencils and every layer's within-leaf table in
    // one launch, then the descriptors, then every layer's stencil
    // corrections and pair biases (one launch each)
    const hp_model_config& c = b.cfg;
    const int64_t L = c.leaf, LS = c.rank, Nd = N.Nd;
    const int nl = c.layers, nd = use_off ? (int)N.ndesc_chunks : 0, ns = (int)((Nd + 255) / 256);
    const int nt = (int)((L * L + 255) / 256 + 1);
    const EdgeTabs t = edge_tabs(b, N, 0), t1 = nl > 1 ? edge_tabs(b, N, 1) : t;
    const unsigned lowmask = (unsigned)(L - 1);
    const FrameDesc& F0 = b.fr[0];
    hipLaunchKernelGGL(k_side_head<sizeof(AT) == 2>, dim3((unsigned)(nd + ns + nl * nt)), dim3(256), 0, st, b.d_fr,
                       N.tile2f, (const DescChunk*)N.desc_chunks, sys, b.ntot, (int)L, (int)LS, N.desc_part, nd,
                       N.node2f, N.nbr, N.ahat, ns, edge_ws(b, W, 0, nl, 0), F0.xm & lowmask, F0.ym & lowmask,
                       F0.zm & lowmask, t.T0, t.eslots, (int64_t)(t1.T0 - t.T0), (int)(t1.eslots - t.eslots), nt);
    if (use_off)
      hipLaunchKernelGGL(k_off_desc_final, dim3((unsigned)b.mtot), dim3(256), 0, st, b.d_fr, N.tile2f,
                         (const int*)N.desc_chunk0, (const double*)N.desc_part, (int)L, (int)LS, N.desc);
    edge_tables<AT>(b, W, 0, nl, 0, st, false);
    if (use_off) edge_tables<AT>(b, W, 0, nl, 1, st);
    if (N.pre_side)
      for (int l = 0; l < nl; ++l) HP_HIP(hipEventRecord(b.side_ev[l], st));
    if (N.pre_side) HP_HIP(hipEventRecord(b.side_done, st));
    HP_HIP(hipGetLastError());
    return HP_OK;
  }
  stencil_desc(b, sys, st);
  // every layer's tables in one launch per kernel (fewer, fuller launches on
  // the side stream, whose chain runs ahead of the encoder)
  for (int l0 = 0; l0 < b.cfg.layers; l0 += EDGE_LAYERS) {
    const int nl = std::min(EDGE_LAYERS, b.cfg.layers - l0);
    edge_tables<AT>(b, W, l0, nl, 0, st);
    if (use_off) edge_tables<AT>(b, W, l0, nl, 1, st);
    if (N.pre_side)
      for (int l = l0; l < l0 + nl; ++l) HP_HIP(hipEventRecord(b.side_ev[l], st));
  }
  if (N.pre_side) HP_HIP(hipEventRecord(b.side_done, st));
  HP_HIP(hipGetLastError());
  return HP_OK;
}

template <typename AT, typename FT>
static hp_status forward(Batch& b, const float* W, const float* rho, const float* sys, void* fac) {
  struct PreReset {
    NetBufs& N;
    ~PreReset() { N.pre = N.pre_side = N.par = 0; }
  } pre_reset{*nb_of(b)};
  HP_TRY(launch_tick(b.d_ticks, b.stream));  // start of the step, for per-frame latencies
  HP_TRY(tables_ahead<AT>(b, W, sys));
  HP_TRY(fwd_prologue<AT>(b, W, rho, sys, nullptr));
  NetBufs& N = *nb_of(b);
  if (N.par) {  // the off stack starts from the pooled tokens
    HP_HIP(hipEventRecord(b.off_ev[0], b.stream));
    HP_HIP(hipStreamWaitEvent(b.offs, b.off_ev[0], 0));
  }
  for (int l = 0; l < b.cfg.layers; ++l) HP_TRY(layer_fwd<AT>(b, W, sys, l, nullptr));
  const NetPlan& P = N.plan;
  const hp_model_config& c = b.cfg;
  hipStream_t st = b.stream;
  const int64_t Nd = N.Nd, d = c.d, L = c.leaf, LS = c.rank, H = c.heads;
  const int64_t No = b.mtot * LS;
  const bool use_off = c.offdiag && b.mtot > 0;
  const FrameDesc* fr = b.d_fr;
  auto wp = [&](const std::string& n) { return W + woff(P, n); };
  (void)fr; (void)use_off; (void)H; (void)No; (void)L; (void)LS;
  // heads (Sec. 4.4)
  const char* base = (const char*)fac;
  int64_t offs[5], tot;
  factor_offsets(b, sizeof(FT) == 2 ? HP_BF16 : HP_F32, offs, &tot);
  hipLaunchKernelGGL(k_layernorm128<AT>, dim3((unsigned)((Nd + 15) / 16)), dim3(256), 0, st, (const float*)N.H,
                     wp("diaglnf.g"), wp("diaglnf.b"), (AT*)N.a128, (int)Nd);
  gemm<AT>(b, N.a128, d, N, P.hleaf1, wp("hleaf1.b"), nullptr, 0, nullptr, 0, N.b128, d, Nd, 1);
  gemm<AT>(b, N.b128, d, N, P.hleaf2, wp("hleaf2.b"), nullptr, 0, N.Frows, L, nullptr, 0, Nd, 0);
  if (L == 64)
    hipLaunchKernelGGL((k_gram_mfma<FT>), dim3((unsigned)b.ktot), dim3(256), 0, st, (const float*)N.Frows,
                       (FT*)(base + offs[0]));
  else
    hipLaunchKernelGGL((k_gram<FT, 32>), dim3((unsigned)b.ktot), dim3(256), 0, st, (const float*)N.Frows,
                       (FT*)(base + offs[0]));
  gemm<AT>(b, N.a128, d, N, P.hnode, N.bias_node, nullptr, 0, N.NH, 36, nullptr, 0, Nd, 0);
  if (LS == 16)
    hipLaunchKernelGGL((k_pack_nodes<FT, 16>), dim3((unsigned)((Nd + 255) / 256)), dim3(256), 0, st,
                       (const float*)N.NH, Nd, (FT*)(base + offs[2]), (FT*)(base + offs[3]), (float*)(base + offs[4]));
  else
    hipLaunchKernelGGL((k_pack_nodes<FT, 8>), dim3((unsigned)((Nd + 255) / 256)), dim3(256), 0, st,
                       (const float*)N.NH, Nd, (FT*)(base + offs[2]), (FT*)(base + offs[3]), (float*)(base + offs[4]));
  // the diagonal tokens' heads above need only this stream's work; the
  // off-diagonal head reads the off stack's last output, so the streams join
  // here (the off stack's last layer ran beside the heads above)
  if (N.par) {
    HP_HIP(hipEventRecord(b.off_ev[1], b.offs));
    HP_HIP(hipStreamWaitEvent(b.stream, b.off_ev[1], 0));
  }
  if (N.pre_side) HP_HIP(hipStreamWaitEvent(b.stream, b.side_done, 0));  // every side launch joined
  if (b.mtot > 0) {
    if (use_off) {
      hipLaunchKernelGGL(k_layernorm128<AT>, dim3((unsigned)((No + 15) / 16)), dim3(256), 0, st, (const float*)N.Xo,
                         wp("offlnf.g"), wp("offlnf.b"), (AT*)N.ao128, (int)No);
      gemm<AT>(b, N.ao128, d, N, P.huv, N.bias_uv, nullptr, 0, N.UV, 2 * LS, nullptr, 0, No, 0);
    } else {
      hipLaunchKernelGGL(k_zero_f32, dim3((unsigned)((No * 2 * LS + 255) / 256)), dim3(256), 0, st, N.UV,
                         (int64_t)(No * 2 * LS));  // a kernel, not a memset: the inference may be captured
    }
    if (LS == 16)
      hipLaunchKernelGGL((k_uvt<FT, 16>), dim3((unsigned)b.mtot), dim3(256), 0, st, (const float*)N.UV,
                         (FT*)(base + offs[1]));
    else
      hipLaunchKernelGGL((k_uvt<FT, 8>), dim3((unsigned)b.mtot), dim3(64), 0, st, (const float*)N.UV,
                         (FT*)(base + offs[1]));
  }
  HP_HIP(hipGetLastError());
  return HP_OK;
}

int infer_signature(const Batch& B) {
  return B.keep_stages | (B.ffn_fused << 1) | (B.attn_valu << 2) | (B.gemm_autotune << 3) |
         ((B.gemm_variant + 1) << 4);
}

bool infer_ready_for_capture(const Batch& B, int compute) {
  return B.net.ws && B.infer_warm.count(std::make_pair(compute, infer_signature(B))) > 0;
}

}  // namespace hp

using namespace hp;

// One inference is ~120 launches.  With the "infer_graph" switch on, after a
// first eager call per (compute, switches) (the GEMM autotuner times there,
// and buffers are allocated), an inference is captured once per (weights,
// rho, sys, factors) buffers and replayed as a hipGraph; under capture the
// GEMMs take the recorded tile choices.  Calls with live kernel timing on run
// eagerly.  The graph reads the buffers' current contents at each replay.
// Off by default: at the precision workload the eager launches already run
// back to back (4.03 ms per inference eager, 4.10 ms replayed).
extern "C" hp_status hp_infer_factors(hp_batch b, const float* d_weights, const float* d_rho, const float* d_sys,
                                      void* d_factors, int32_t compute) {
  if (!b || !d_weights || !d_rho || !d_sys || !d_factors)
    return set_error(HP_E_INVALID, "hp_infer_factors: NULL argument");
  if (compute != HP_BF16 && compute != HP_F32)
    return set_error(HP_E_INVALID, "hp_infer_factors: compute must be HP_F32 or HP_BF16");
  Batch& B = *b;
  HP_TRY(network_alloc(B));
  auto run = [&]() -> hp_status {
    if (compute == HP_BF16) return forward<uint16_t, uint16_t>(B, d_weights, d_rho, d_sys, d_factors);
    return forward<float, float>(B, d_weights, d_rho, d_sys, d_factors);
  };
  const int sig = infer_signature(B);
  const auto warm = std::make_pair((int)compute, sig);
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  HP_HIP(hipStreamIsCapturing(B.stream, &cs));
  // inside a caller's capture (a captured solve step) the launches join it
  if (!B.infer_graph || B.prof.kind != PROF_NONE || !B.infer_warm.count(warm) || cs != hipStreamCaptureStatusNone) {
    HP_TRY(run());
    B.infer_warm.insert(warm);
    return HP_OK;
  }
  const auto key = std::make_tuple((int)compute, (const void*)d_weights, (const void*)d_rho, (const void*)d_sys,
                                   (const void*)d_factors, sig);
  auto it = B.infer_graphs.find(key);
  hipGraphExec_t exec = nullptr;
  if (it != B.infer_graphs.end()) {
    exec = it->second;
  } else {
    if (B.infer_graphs.size() >= 8) {  // callers cycling through buffers: keep the cache small
      for (auto& kv : B.infer_graphs) hipGraphExecDestroy(kv.second);
      B.infer_graphs.clear();
    }
    if (!B.cap_stream) HP_HIP(hipStreamCreateWithFlags(&B.cap_stream, hipStreamNonBlocking));
    std::swap(B.stream, B.cap_stream);  // the forward launches on B.stream
    hipGraph_t graph = nullptr;
    hipError_t e = hipStreamBeginCapture(B.stream, hipStreamCaptureModeThreadLocal);
    hp_status s = e == hipSuccess ? run() : HP_E_HIP;
    if (e == hipSuccess) e = hipStreamEndCapture(B.stream, &graph);
    std::swap(B.stream, B.cap_stream);
    if (s != HP_OK) {
      if (graph) hipGraphDestroy(graph);
      return s;
    }
    if (e != hipSuccess) return set_error(HP_E_HIP, "inference capture: %s", hipGetErrorString(e));
    e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    hipGraphDestroy(graph);
    if (e != hipSuccess) return set_error(HP_E_HIP, "hipGraphInstantiate: %s", hipGetErrorString(e));
    B.infer_graphs[key] = exec;
  }
  HP_HIP(hipGraphLaunch(exec, B.stream));
  return HP_OK;
}

extern "C" hp_status hp_debug_copy(hp_batch b, const char* name, void* d_dst, int64_t bytes) {
  if (!b || !name || !d_dst || bytes < 0) return set_error(HP_E_INVALID, "hp_debug_copy: bad arguments");
  if (!b->net.ws) return set_error(HP_E_STATE, "hp_debug_copy: no inference has run on this batch");
  NetBufs& N = *nb_of(*b);
  const void* src = nullptr;
  int64_t cap = 0;
  const std::string n = name;
  const int64_t d = b->cfg.d;
  if (n == "feats") src = N.feats, cap = N.Nd * 32 * 4;
  else if ((n == "enc" || n == "xo0") && !b->keep_stages)
    return set_error(HP_E_INVALID, "hp_debug_copy: '%s' is kept only with hp_debug_set(\"keep_stages\", 1)",
                     n.c_str());
  else if (n == "enc") src = N.Henc, cap = N.Nd * d * 4;
  else if (n == "xo0") src = N.Xo0, cap = N.No * d * 4;
  else if (n == "xd") src = N.H, cap = N.Nd * d * 4;
  else if (n == "xo") src = N.Xo, cap = N.No * d * 4;
  else if (n == "frows") src = N.Frows, cap = N.Nd * b->cfg.leaf * 4;
  else if (n == "nodeh") src = N.NH, cap = N.Nd * 36 * 4;
  else if (n == "uv") src = N.UV, cap = N.No * 2 * b->cfg.rank * 4;
  else if (n == "desc") src = N.desc, cap = std::max<int64_t>(b->mtot, 1) * b->cfg.rank * b->cfg.rank * 16;
  else if (n == "glob") src = N.glob, cap = b->nframes * 12 * 4;
  if (!src) return set_error(HP_E_INVALID, "hp_debug_copy: unknown buffer '%s'", name);
  if (bytes > cap) return set_error(HP_E_INVALID, "hp_debug_copy: %lld bytes requested, buffer holds %lld",
                                    (long long)bytes, (long long)cap);
  HP_HIP(hipMemcpyAsync(d_dst, src, bytes, hipMemcpyDeviceToDevice, b->stream));
  return HP_OK;
}

// Reverse pass and training step.
#include "net_backward.h"
#include "net_train.h"
