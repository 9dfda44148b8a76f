// Reverse-mode kernels of the network (included by network.hip after the
// forward kernels).  Reductions over rows are split into fixed chunks whose
// partials are summed in a fixed order, so gradients are bit-reproducible.
#pragma once

namespace hp {

__device__ inline float gelu_grad(float x) {
  const float cdf = 0.5f * (1.f + erff(x * 0.7071067811865476f));
  const float pdf = 0.3989422804014327f * expf(-0.5f * x * x);
  return cdf + x * pdf;
}

// ------------------------------------------------------------------ weight-gradient GEMM
// part[chunk][i][o] = sum over rows r of the chunk of X[r][i] * D[r][o]
// (X: activations [M][ldx], D: output gradients [M][ldd], both in AT).
// 64 x 64 tile of (i, o), four waves of 32 x 32, rows staged 32 at a time
// and transposed into LDS so that the MFMA operands are row-contiguous.
struct GemmTNArgs {
  const void* X;
  int64_t ldx;
  const void* D;
  int64_t ldd;
  int M, NI, NO, rows_per_chunk;
  float* part;  // [nchunks][NI][NO]
};

template <typename AT>
__global__ __launch_bounds__(256) void k_gemm_tn(GemmTNArgs a) {
  constexpr int BK = 32, PAD = sizeof(AT) == 2 ? 8 : 4;
  __shared__ __attribute__((aligned(16))) AT sA[64][BK + PAD];
  __shared__ __attribute__((aligned(16))) AT sB[64][BK + PAD];
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int i0 = blockIdx.x * 64, o0 = blockIdx.y * 64, chunk = blockIdx.z;
  const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
  const int r_begin = chunk * a.rows_per_chunk, r_end = min(a.M, r_begin + a.rows_per_chunk);
  const AT* X = (const AT*)a.X;
  const AT* D = (const AT*)a.D;
  f32x16_t acc;
#pragma unroll
  for (int q = 0; q < 16; ++q) acc[q] = 0.f;
  for (int r0 = r_begin; r0 < r_end; r0 += BK) {
    // 32 rows x 64 columns of X and of D; thread -> (row tid/8, 8 columns)
    const int rr = tid >> 3, cc = (tid & 7) * 8;
    const int r = r0 + rr;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      AT xv = (AT)0, dv = (AT)0;
      if (r < r_end && i0 + cc + e < a.NI) xv = X[(int64_t)r * a.ldx + i0 + cc + e];
      if (r < r_end && o0 + cc + e < a.NO) dv = D[(int64_t)r * a.ldd + o0 + cc + e];
      sA[cc + e][rr] = xv;
      sB[cc + e][rr] = dv;
    }
    __syncthreads();
    if constexpr (sizeof(AT) == 2) {
#pragma unroll
      for (int kk = 0; kk < BK; kk += 16) {
        bf16x8_t av = __builtin_bit_cast(bf16x8_t, *(const uint4*)&sA[wm + (lane & 31)][kk + (lane >> 5) * 8]);
        bf16x8_t bv = __builtin_bit_cast(bf16x8_t, *(const uint4*)&sB[wn + (lane & 31)][kk + (lane >> 5) * 8]);
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av, bv, acc, 0, 0, 0);
      }
    } else {
#pragma unroll
      for (int kk = 0; kk < BK; kk += 2) {
        acc = __builtin_amdgcn_mfma_f32_32x32x2f32(sA[wm + (lane & 31)][kk + (lane >> 5)],
                                                   sB[wn + (lane & 31)][kk + (lane >> 5)], acc, 0, 0, 0);
      }
    }
    __syncthreads();
  }
  const int o = o0 + wn + (lane & 31);
  if (o >= a.NO) return;
  float* P = a.part + (int64_t)chunk * a.NI * a.NO;
#pragma unroll
  for (int q = 0; q < 4; ++q)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int i = i0 + wm + q * 8 + (lane >> 5) * 4 + j;
      if (i < a.NI) P[(int64_t)i * a.NO + o] = acc[q * 4 + j];
    }
}

// out[i * ldo + (o - o_begin)] (+)= sum over chunks of part[c][i][o], for
// i < ni_store and o in [o_begin, o_begin + o_count) (splits one product into
// the weight tensors that share it).
__global__ void k_reduce_chunks(const float* part, int nchunks, int NI, int NO, int o_begin, int o_count,
                                int ni_store, float* out, int ldo, int accumulate) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)ni_store * o_count) return;
  const int i = (int)(e / o_count), oc = (int)(e % o_count), o = o_begin + oc;
  const int64_t src = (int64_t)i * NO + o;
  float s = 0.f;
  for (int c = 0; c < nchunks; ++c) s += part[(int64_t)c * NI * NO + src];
  float* dst = out + (int64_t)i * ldo + oc;
  *dst = accumulate ? *dst + s : s;
}

// Column sums over rows in chunks: part[chunk][col] (bias gradients).
__global__ __launch_bounds__(256) void k_colsum_chunks(const float* D, int64_t ldd, int M, int N, int rows_per_chunk,
                                                       float* part) {
  const int col = blockIdx.x * 256 + threadIdx.x;
  if (col >= N) return;
  const int r0 = blockIdx.y * rows_per_chunk, r1 = min(M, r0 + rows_per_chunk);
  float s = 0.f;
  for (int r = r0; r < r1; ++r) s += D[(int64_t)r * ldd + col];
  part[(int64_t)blockIdx.y * N + col] = s;
}

// ------------------------------------------------------------------ elementwise
// g_pre = g ⊙ GELU'(pre); writes FP32 and the compute-type copy.
template <typename AT>
__global__ void k_gelu_bwd(const float* g, const float* pre, int64_t n, float* out, AT* outb) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  const float v = g[e] * gelu_grad(pre[e]);
  out[e] = v;
  if (outb) outb[e] = to_act<AT>(v);
}

template <typename AT>
__global__ void k_to_act(const float* x, int64_t rows, int cols, int64_t ldx, AT* y, int64_t ldy) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= rows * cols) return;
  const int64_t r = e / cols;
  const int c = (int)(e % cols);
  y[r * ldy + c] = to_act<AT>(x[r * ldx + c]);
}

__global__ void k_add_inplace(float* y, const float* x, int64_t n) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < n) y[e] += x[e];
}

// ------------------------------------------------------------------ LayerNorm backward
// Rows of width C (128 or 512) given by up to 4 segments of 128 (as in the
// forward concat); dY [M][C] FP32.  dX segments written (segment 0 may be
// accumulated into); gamma/beta partials per block of 16 rows.
struct LnSeg {
  const float* p[4];
  int64_t ld[4];
  const int* row2f;  // segment 3 indexed by frame when set
};

template <int C>
__global__ __launch_bounds__(256) void k_ln_bwd(LnSeg in, const float* gam, const float* dY, int M, float* dX0,
                                                int acc0, float* dX1, float* dX2, float* dX3, float* gpart) {
  constexpr int PER = C / 64;
  __shared__ float sg[4][2 * C];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  float pg[PER], pb[PER];
#pragma unroll
  for (int q = 0; q < PER; ++q) pg[q] = pb[q] = 0.f;
  for (int rr = 0; rr < 4; ++rr) {
    const int row = blockIdx.x * 16 + wave * 4 + rr;
    if (row >= M) break;
    float x[PER], dy[PER];
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int col = lane + 64 * q, seg = col >> 7, cc = col & 127;
      const float* base = in.p[seg];
      float v = 0.f;
      if (base) {
        const int64_t r = (seg == 3 && in.row2f) ? in.row2f[row] : row;
        v = base[r * in.ld[seg] + cc];
      }
      x[q] = v;
      dy[q] = dY[(int64_t)row * C + col];
    }
    float s = 0.f;
#pragma unroll
    for (int q = 0; q < PER; ++q) s += x[q];
    const float mu = wave_sum_f(s) * (1.f / C);
    float v2 = 0.f;
#pragma unroll
    for (int q = 0; q < PER; ++q) v2 += (x[q] - mu) * (x[q] - mu);
    const float rs = rsqrtf(wave_sum_f(v2) * (1.f / C) + 1e-5f);
    float a = 0.f, b = 0.f;
    float xh[PER], gx[PER];
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int col = lane + 64 * q;
      xh[q] = (x[q] - mu) * rs;
      gx[q] = dy[q] * gam[col];
      a += gx[q];
      b += gx[q] * xh[q];
      pg[q] += dy[q] * xh[q];
      pb[q] += dy[q];
    }
    const float ma = wave_sum_f(a) * (1.f / C), mb = wave_sum_f(b) * (1.f / C);
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int col = lane + 64 * q, seg = col >> 7, cc = col & 127;
      const float d = rs * (gx[q] - ma - xh[q] * mb);
      float* out = seg == 0 ? dX0 : seg == 1 ? dX1 : seg == 2 ? dX2 : dX3;
      if (seg == 0 && C == 128) {
        float* o = dX0 + (int64_t)row * 128 + cc;
        *o = acc0 ? *o + d : d;
      } else if (out) {
        float* o = out + (int64_t)row * 128 + cc;
        *o = (seg == 0 && acc0) ? *o + d : d;
      }
    }
  }
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    sg[wave][lane + 64 * q] = pg[q];
    sg[wave][C + lane + 64 * q] = pb[q];
  }
  __syncthreads();
  for (int e = threadIdx.x; e < 2 * C; e += 256)
    gpart[(int64_t)blockIdx.x * 2 * C + e] = sg[0][e] + sg[1][e] + sg[2][e] + sg[3][e];
}

// ------------------------------------------------------------------ attention backward
// One wave per (group, head), lane = query row.  Recomputes S, P from Q, K and
// the bias, then dV = P^T dO, dS = P ⊙ (dO V^T - rowdot(dO, O)), dQ = s dS K,
// dK = s dS^T Q (s = 1/sqrt(32)).  dqkv [rows][3d] FP32.  The bias gradient
// dS goes to dsb (diagonal: [group][h][T][T], for the shared-table
// reduction; tiles: dense per tile) and, for diagonal groups, to dcorr at the
// row's stencil entries.
template <typename AT, int T, bool DIAG>
__global__ __launch_bounds__(64) void k_attention_bwd(const AT* qkv, const float* dO, const float* bias,
                                                      const float* corr, const uint8_t* nbr, int H, float* dqkv,
                                                      float* dsb, float* dcorr) {
  constexpr int DH = 32;
  __shared__ float sQ[T][DH + 1], sK[T][DH + 1], sV[T][DH + 1], sdO[T][DH + 1];
  __shared__ float sP[T][T + 1], sS[T][T + 1];
  const int grp = blockIdx.x, h = blockIdx.y, lane = threadIdx.x;
  const int d = H * DH;
  const int64_t row0 = (int64_t)grp * T;
  const float scale = 0.17677669529663687f;
  for (int idx = lane; idx < T * DH; idx += 64) {
    const int r = idx / DH, c = idx % DH;
    const AT* q = qkv + (row0 + r) * 3 * d + h * DH + c;
    sQ[r][c] = ldf(q, 0);
    sK[r][c] = ldf(q, d);
    sV[r][c] = ldf(q, 2 * d);
    sdO[r][c] = dO[(row0 + r) * d + h * DH + c];
  }
  const float* bt = DIAG ? bias + (int64_t)h * T * T : bias + ((int64_t)grp * H + h) * T * T;
  for (int idx = lane; idx < T * T; idx += 64) sS[idx / T][idx % T] = bt[idx];
  __syncthreads();
  if (lane < T) {
    const int64_t row = row0 + lane;
    if (DIAG) {
      for (int e = 0; e < 7; ++e) {
        const int lj = nbr[row * 7 + e];
        if (lj != 255) sS[lane][lj] += corr[(row * 7 + e) * H + h];
      }
    }
    float s[T];
    float mx = -3.4e38f;
    for (int j = 0; j < T; ++j) {
      float a = sS[lane][j];
      for (int c = 0; c < DH; ++c) a = fmaf(sQ[lane][c] * scale, sK[j][c], a);
      s[j] = a;
      mx = fmaxf(mx, a);
    }
    float sum = 0.f;
    for (int j = 0; j < T; ++j) {
      s[j] = expf(s[j] - mx);
      sum += s[j];
    }
    const float inv = 1.f / sum;
    float Dv = 0.f;  // rowdot(dO, O) with O = P V
    for (int c = 0; c < DH; ++c) {
      float o = 0.f;
      for (int j = 0; j < T; ++j) o = fmaf(s[j], sV[j][c], o);
      Dv = fmaf(sdO[lane][c], o * inv, Dv);
    }
    for (int j = 0; j < T; ++j) {
      const float p = s[j] * inv;
      float dp = 0.f;
      for (int c = 0; c < DH; ++c) dp = fmaf(sdO[lane][c], sV[j][c], dp);
      sP[lane][j] = p;
      s[j] = p * (dp - Dv);  // dS
    }
    float dq[DH];
    for (int c = 0; c < DH; ++c) dq[c] = 0.f;
    for (int j = 0; j < T; ++j)
      for (int c = 0; c < DH; ++c) dq[c] = fmaf(s[j], sK[j][c], dq[c]);
    for (int c = 0; c < DH; ++c) dqkv[row * 3 * d + h * DH + c] = dq[c] * scale;
    float* ds_out = dsb + ((int64_t)grp * H + h) * T * T + (int64_t)lane * T;
    for (int j = 0; j < T; ++j) ds_out[j] = s[j];
    if (DIAG) {
      for (int e = 0; e < 7; ++e) {
        const int lj = nbr[row * 7 + e];
        dcorr[(row * 7 + e) * H + h] = lj != 255 ? s[lj] : 0.f;
      }
    }
    for (int j = 0; j < T; ++j) sS[lane][j] = s[j];
  }
  __syncthreads();
  if (lane < T) {  // lane = key j: dK_j = s sum_i dS_ij q_i, dV_j = sum_i P_ij dO_i
    const int64_t row = row0 + lane;
    float dk[DH], dv[DH];
    for (int c = 0; c < DH; ++c) dk[c] = dv[c] = 0.f;
    for (int i = 0; i < T; ++i) {
      const float ds = sS[i][lane], p = sP[i][lane];
      for (int c = 0; c < DH; ++c) {
        dk[c] = fmaf(ds, sQ[i][c], dk[c]);
        dv[c] = fmaf(p, sdO[i][c], dv[c]);
      }
    }
    for (int c = 0; c < DH; ++c) {
      dqkv[row * 3 * d + d + h * DH + c] = dk[c] * scale;
      dqkv[row * 3 * d + 2 * d + h * DH + c] = dv[c];
    }
  }
}

// dT0[h][i][j] = sum over leaves of dS[leaf][h][i][j] (fixed order).
__global__ void k_reduce_leaves(const float* dsb, int64_t ngroups, int HTT, float* out) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= HTT) return;
  float s = 0.f;
  for (int64_t g = 0; g < ngroups; ++g) s += dsb[g * HTT + e];
  out[e] = s;
}

// ------------------------------------------------------------------ edge-MLP backward
// Gradients of MLP_e = GELU(e W1 + b1) W2 + b2 summed over a list of
// (descriptor e, output gradient) pairs.  Thread = (hidden unit k, pair lane
// sub of 8); each block sums its range of pairs in a fixed order and writes a
// partial [W1 (4E) | b1 (E) | W2 (E H) | b2 (H)].  Sources: kind 0 = the
// shared diagonal table (pair = i L + j, gradient dT0[h][i][j]); kind 1 =
// stencil corrections (pair = node 7 + e: +dcorr at (dx, Ahat), -dcorr at
// (dx, 0)); kind 2 = off-diagonal descriptors with a dense per-tile gradient.
struct EdgeBwdSrc {
  int kind;
  int64_t npairs;
  int L;
  unsigned xm, ym, zm;      // kind 0: within-leaf coordinate masks
  const float* dT0;         // kind 0: [H][L][L]
  const uint8_t* nbr;       // kind 1
  const float* ahat;        // kind 1
  const float* dcorr;       // kind 1: [pairs][H]
  const float* desc;        // kind 2: [pairs][4]
  const float* dbias;       // kind 2: [tile][H][LS][LS]
  int LS;
};

constexpr int EDGE_NP_MAX = 4 * 32 + 32 + 32 * 8 + 8;

__global__ __launch_bounds__(256) void k_edge_bwd(EdgeW w, EdgeBwdSrc src, int64_t pairs_per_block, float* part) {
  __shared__ float red[8][EDGE_NP_MAX];
  const int E = w.E, H = w.H, NP = 5 * E + E * H + H;
  const int k = threadIdx.x & 31, sub = threadIdx.x >> 5;
  float aw1[4] = {0.f, 0.f, 0.f, 0.f}, ab1 = 0.f, aw2[8], ab2[8];
  for (int h = 0; h < 8; ++h) aw2[h] = ab2[h] = 0.f;
  auto one = [&](const float e[4], const float* dout) {
    if (k >= E) return;
    float pre = w.b1[k];
    for (int q = 0; q < 4; ++q) pre = fmaf(e[q], w.w1[q * E + k], pre);
    const float hid = gelu_f(pre);
    float dh = 0.f;
    for (int h = 0; h < H; ++h) {
      aw2[h] = fmaf(hid, dout[h], aw2[h]);
      dh = fmaf(dout[h], w.w2[k * H + h], dh);
      if (k == 0) ab2[h] += dout[h];
    }
    const float dp = dh * gelu_grad(pre);
    ab1 += dp;
    for (int q = 0; q < 4; ++q) aw1[q] = fmaf(e[q], dp, aw1[q]);
  };
  const int64_t p0 = (int64_t)blockIdx.x * pairs_per_block, p1 = min(src.npairs, p0 + pairs_per_block);
  for (int64_t p = p0 + sub; p < p1; p += 8) {
    float dout[8];
    if (src.kind == 0) {
      const int i = (int)(p / src.L), j = (int)(p % src.L);
      float e[4] = {(mcoord(j, src.xm) - mcoord(i, src.xm)) * 0.25f, (mcoord(j, src.ym) - mcoord(i, src.ym)) * 0.25f,
                    (mcoord(j, src.zm) - mcoord(i, src.zm)) * 0.25f, 0.f};
      for (int h = 0; h < H; ++h) dout[h] = src.dT0[((int64_t)h * src.L + i) * src.L + j];
      one(e, dout);
    } else if (src.kind == 1) {
      if (src.nbr[p] == 255) continue;
      const int ee = (int)(p % 7);
      float dd[3] = {0.f, 0.f, 0.f};
      if (ee > 0) dd[(ee - 1) / 2] = ((ee - 1) % 2 == 0) ? 0.25f : -0.25f;
      float e1[4] = {dd[0], dd[1], dd[2], src.ahat[p]}, e0[4] = {dd[0], dd[1], dd[2], 0.f};
      for (int h = 0; h < H; ++h) dout[h] = src.dcorr[p * H + h];
      one(e1, dout);
      for (int h = 0; h < H; ++h) dout[h] = -dout[h];
      one(e0, dout);
    } else {
      const int64_t m = p / (src.LS * src.LS);
      const int tt = (int)(p % (src.LS * src.LS));
      float e[4] = {src.desc[p * 4], src.desc[p * 4 + 1], src.desc[p * 4 + 2], src.desc[p * 4 + 3]};
      for (int h = 0; h < H; ++h) dout[h] = src.dbias[(m * H + h) * src.LS * src.LS + tt];
      one(e, dout);
    }
  }
  if (k < E) {
    for (int q = 0; q < 4; ++q) red[sub][q * E + k] = aw1[q];
    red[sub][4 * E + k] = ab1;
    for (int h = 0; h < H; ++h) red[sub][5 * E + k * H + h] = aw2[h];
    if (k == 0)
      for (int h = 0; h < H; ++h) red[sub][5 * E + E * H + h] = ab2[h];
  }
  __syncthreads();
  for (int q = threadIdx.x; q < NP; q += 256) {
    float s = 0.f;
    for (int t = 0; t < 8; ++t) s += red[t][q];
    part[(int64_t)blockIdx.x * NP + q] = s;
  }
}

// ------------------------------------------------------------------ strips, highways, pooling
// Adjoint of the strip means (pooling and highway context) for node rows: dA_i (+)= sum over the tokens whose
// row sub-strip holds i of dout[tok][0:128] * s_tok, and likewise dBsrc_i over
// column sub-strips with dout[tok][128:256]; s_tok = 1 / (S p) (means).
__global__ __launch_bounds__(256) void k_strip_means_bwd(const FrameDesc* fr, const int* node2f, const float* dout,
                                                         int L, int LS, int64_t ntot, float* dA, float* dB,
                                                         int accumulate) {
  const int64_t i = (int64_t)blockIdx.x * 2 + (threadIdx.x >> 7);
  if (i >= ntot) return;
  const int col = threadIdx.x & 127;
  const FrameDesc F = fr[node2f[i]];
  const int c = (int)(i - F.n0), k = c / L, l = c % L, p = L / LS, K = F.K;
  float ra = 0.f, rb = 0.f;
  for (int j = 0; j < F.J; ++j) {
    const int m = K - (K >> j) + (k >> (j + 1));
    const float inv = 1.f / (float)((1 << j) * p);
    const float* row = dout + ((int64_t)(F.m0 + m) * LS + l / p) * 256;
    if (((k >> j) & 1) == 0) ra += row[col] * inv;
    else rb += row[128 + col] * inv;
  }
  if (dB == dA) {
    dA[i * 128 + col] = accumulate ? dA[i * 128 + col] + ra + rb : ra + rb;
  } else {
    dA[i * 128 + col] = accumulate ? dA[i * 128 + col] + ra : ra;
    dB[i * 128 + col] = accumulate ? dB[i * 128 + col] + rb : rb;
  }
}

// Highway adjoint at the nodes: given dr_i, dc_i (diagonal FFN inputs plus the
// off-diagonal readers' share) the normalised contributions wr_i = dr_i / n_r,
// wc_i = dc_i / n_c; dXd_i += wr_i + wc_i + dg_f / count_f.  Without
// off-diagonal tokens r_i = c_i = x_i (n_r = n_c = 1).
__global__ __launch_bounds__(256) void k_highway_bwd_nodes(const FrameDesc* fr, const int* node2f, const float* dR,
                                                           const float* dC, const float* dG, const float* count,
                                                           int L, int64_t ntot, int with_off, float* WR, float* WC,
                                                           float* dXd) {
  const int64_t i = (int64_t)blockIdx.x * 2 + (threadIdx.x >> 7);
  if (i >= ntot) return;
  const int col = threadIdx.x & 127;
  const int f = node2f[i];
  const FrameDesc F = fr[f];
  const int k = (int)(i - F.n0) / L;
  int nr = 1, nc = 1;
  for (int j = 0; with_off && j < F.J; ++j) {
    if (((k >> j) & 1) == 0) ++nr;
    else ++nc;
  }
  const float wr = dR[i * 128 + col] / nr, wc = dC[i * 128 + col] / nc;
  WR[i * 128 + col] = wr;
  WC[i * 128 + col] = wc;
  dXd[i * 128 + col] += wr + wc + dG[f * 128 + col] / count[f];
}

// Off-diagonal tokens of the highway adjoint: dXo[tok] += sum of WR over the
// row sub-strip + sum of WC over the column sub-strip + dg_f / count_f.
__global__ __launch_bounds__(128) void k_highway_bwd_tokens(const FrameDesc* fr, const int* tile2f, const float* WR,
                                                            const float* WC, const float* dG, const float* count,
                                                            int L, int LS, float* dXo) {
  const int64_t tok = blockIdx.x;
  const int mg = (int)(tok / LS), t = (int)(tok % LS);
  const int f = tile2f[mg];
  const FrameDesc F = fr[f];
  const int m = mg - F.m0, K = F.K;
  int j = 0;
  while (m >= K - (K >> (j + 1))) ++j;
  const int i = m - (K - (K >> j)), S = 1 << j, r0 = 2 * i * S, c0 = r0 + S, p = L / LS;
  const int col = threadIdx.x;
  float s = 0.f;
  for (int k = 0; k < S; ++k)
    for (int l = t * p; l < (t + 1) * p; ++l) {
      s += WR[((int64_t)F.n0 + (int64_t)(r0 + k) * L + l) * 128 + col];
      s += WC[((int64_t)F.n0 + (int64_t)(c0 + k) * L + l) * 128 + col];
    }
  dXo[tok * 128 + col] += s + dG[f * 128 + col] / count[f];
}

// (D^-1 A)^T g: entry j = g_j - sum over faces (w_ij / A_ii) g_i.
__global__ __launch_bounds__(256) void k_gcn_spmm_t(const FrameDesc* fr, const int* node2f, const float* sys,
                                                    int64_t ntot, const float* G, float* out, int accumulate) {
  const int64_t i = (int64_t)blockIdx.x * 2 + (threadIdx.x >> 7);
  if (i >= ntot) return;
  const int col = threadIdx.x & 127;
  const FrameDesc F = fr[node2f[i]];
  const unsigned c = (unsigned)(i - F.n0);
  const float *dg = sys, *wx = sys + ntot, *wy = sys + 2 * ntot, *wz = sys + 3 * ntot;
  const int64_t xp = F.n0 + mstep_plus(c, F.xm), xn = F.n0 + mstep_minus(c, F.xm);
  const int64_t yp = F.n0 + mstep_plus(c, F.ym), yn = F.n0 + mstep_minus(c, F.ym);
  const int64_t zp = F.n0 + mstep_plus(c, F.zm), zn = F.n0 + mstep_minus(c, F.zm);
  float s = wx[i] / dg[xp] * G[xp * 128 + col];
  s = fmaf(wx[xn] / dg[xn], G[xn * 128 + col], s);
  s = fmaf(wy[i] / dg[yp], G[yp * 128 + col], s);
  s = fmaf(wy[yn] / dg[yn], G[yn * 128 + col], s);
  s = fmaf(wz[i] / dg[zp], G[zp * 128 + col], s);
  s = fmaf(wz[zn] / dg[zn], G[zn * 128 + col], s);
  const float v = G[i * 128 + col] - s;
  out[i * 128 + col] = accumulate ? out[i * 128 + col] + v : v;
}

// ------------------------------------------------------------------ heads: split and join
// NH [N][36] = (Ut | Vt | lam-logit); lam = softplus(logit).
template <int LS>
__global__ void k_split_nodeheads(const float* NH, int64_t ntot, float* Ut, float* Vt, float* lam) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= ntot) return;
  for (int s = 0; s < LS; ++s) {
    Ut[i * LS + s] = NH[i * 36 + s];
    Vt[i * LS + s] = NH[i * 36 + LS + s];
  }
  lam[i] = softplus_f(NH[i * 36 + 2 * LS]);
}

// dNH [N][64] (zero padded beyond 2 LS + 1) from dUt, dVt, dlam.
template <int LS>
__global__ void k_join_nodeheads(const float* NH, const float* dUt, const float* dVt, const float* dlam, int64_t ntot,
                                 float* dNH) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= ntot) return;
  for (int s = 0; s < LS; ++s) {
    dNH[i * 64 + s] = dUt[i * LS + s];
    dNH[i * 64 + LS + s] = dVt[i * LS + s];
  }
  const float x = NH[i * 36 + 2 * LS];
  dNH[i * 64 + 2 * LS] = dlam[i] / (1.f + expf(-x));
  for (int s = 2 * LS + 1; s < 64; ++s) dNH[i * 64 + s] = 0.f;
}

// UV [No][2 LS] <-> U, V [mtot][LS][LS].
template <int LS>
__global__ void k_split_uv(const float* UV, int64_t ntok, float* U, float* V) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= ntok * LS) return;
  const int64_t tok = e / LS;
  const int s = (int)(e % LS);
  U[e] = UV[tok * 2 * LS + s];
  V[e] = UV[tok * 2 * LS + LS + s];
}

template <int LS>
__global__ void k_join_uv(const float* dU, const float* dV, int64_t ntok, float* dUV) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= ntok * LS) return;
  const int64_t tok = e / LS;
  const int s = (int)(e % LS);
  dUV[tok * 2 * LS + s] = dU[e];
  dUV[tok * 2 * LS + LS + s] = dV[e];
}

// ------------------------------------------------------------------ optimiser
// Sum of squares of the gradient in chunks (FP64 partials).
__global__ __launch_bounds__(256) void k_sumsq_chunks(const float* g, int64_t n, int64_t per, double* part) {
  __shared__ double red[4];
  const int64_t b0 = (int64_t)blockIdx.x * per, b1 = min(n, b0 + per);
  double s = 0.0;
  for (int64_t e = b0 + threadIdx.x; e < b1; e += 256) s += (double)g[e] * (double)g[e];
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) part[blockIdx.x] = red[0] + red[1] + red[2] + red[3];
}

// AdamW with the global-norm clip (PyTorch semantics): clip factor
// min(1, clip / (||g|| + 1e-6)); p *= 1 - lr wd; m, v moments; bias corrections.
struct AdamArgs {
  double lr, b1, b2, eps, wd, clip;
  int step, nparts;
  int64_t n;
};

__global__ void k_adamw(AdamArgs a, const double* part, const float* g, float* p, float* m, float* v, double* gnorm) {
  __shared__ double gn;
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int i = 0; i < a.nparts; ++i) s += part[i];
    gn = sqrt(s);
    if (blockIdx.x == 0) *gnorm = gn;
  }
  __syncthreads();
  const double sc = a.clip > 0 ? fmin(1.0, a.clip / (gn + 1e-6)) : 1.0;
  const double bc1 = 1.0 - pow(a.b1, a.step), bc2 = 1.0 - pow(a.b2, a.step);
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < a.n; e += (int64_t)gridDim.x * blockDim.x) {
    const double gg = (double)g[e] * sc;
    double pp = (double)p[e] * (1.0 - a.lr * a.wd);
    const double mm = a.b1 * (double)m[e] + (1.0 - a.b1) * gg;
    const double vv = a.b2 * (double)v[e] + (1.0 - a.b2) * gg * gg;
    pp -= a.lr * (mm / bc1) / (sqrt(vv / bc2) + a.eps);
    p[e] = (float)pp;
    m[e] = (float)mm;
    v[e] = (float)vv;
  }
}

}  // namespace hp
