// Assembly, 7-point SpMV, the H-matrix apply and the fused PCG pipeline.
//
// PCG (paper Sec. 3 and Sec. 5; Saad 2003 Alg. 9.1) runs as four kernels per
// iteration for the learned preconditioner and two for Jacobi / identity:
//
//   k_spmv_p      node blocks: rho' = r.z, beta, p = z + beta p_old (on the fly
//                 at the 7 stencil points, p ping-pongs), q = A p, partials of
//                 p.q.  Jacobi / identity: also the stop checks of the last update.
//   k_update_hmat leaf blocks: alpha, x += alpha p (FP64, x ping-pongs),
//                 r -= alpha q or the FP64 residual replacement r = b - A x,
//                 the leaf stage of M (G_k r_k + lam r / A_ii, restriction
//                 Ut^T r, Vt^T r), partials of ||r||^2.
//   k_coarse_check coarse blocks (one per tile): stop checks (redundant in
//                 every block of the frame), then the tile's coupling: strip
//                 sums s^r, s^c, t^r = B s^c, t^c = B^T s^r.
//   k_prolong     leaf blocks: gather T^r, T^c down the levels,
//                 z += Ut T^r + Vt T^c, partials of r.z.
//
// All reductions run in a fixed order (FP64), so a solve is bit-reproducible
// and independent of how frames are batched.  Frames that stopped are skipped
// by every kernel, which makes a fixed chunk of iterations safe to replay
// from a hipGraph.
#include <float.h>
#include <math.h>

#include <mutex>

#include "batch.h"

namespace hp {

// ------------------------------------------------------------------ helpers

__device__ inline double warp_sum(double v) { return wave_total_d(v); }

// A frame stops (run by its lead thread once): one fewer active frame, and
// the device clock at the stop for per-frame latencies.
__device__ inline void frame_stopped(const PcgBufs& B_, int f) {
  atomicSub(B_.n_active, 1);
  B_.ticks[2 + f] = (int64_t)wall_clock64();
}

__global__ void k_tick(int64_t* p) { *p = (int64_t)wall_clock64(); }

hp_status launch_tick(int64_t* p, hipStream_t s) {
  hipLaunchKernelGGL(k_tick, dim3(1), dim3(1), 0, s, p);
  HP_HIP(hipGetLastError());
  return HP_OK;
}

// Fixed-order block sum of one double per thread (blockDim multiple of 64).
__device__ inline double block_sum(double v, double* red) {
  v = warp_sum(v);
  int w = threadIdx.x >> 6, nw = blockDim.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[w] = v;
  __syncthreads();
  double s = 0.0;
  for (int i = 0; i < nw; ++i) s += red[i];
  return s;
}

// Fixed-order sum of `count` partials (written by an earlier kernel) by the
// whole block: thread t adds entries t, t + nt, ... in order, then the
// fixed-order block reduction.  Every block gets the same bits.
__device__ inline double frame_sum(const double* part, int count, double* red) {
  double a = 0.0;
  for (int j = threadIdx.x; j < count; j += blockDim.x) a += part[j];
  return block_sum(a, red);
}

// Assembled system: FP32 [diag | wx | wy | wz | 1/diag] (5 ntot floats) for
// the SpMV and Jacobi, then FP64 [diag | wx | wy | wz] (4 ntot doubles) for the
// FP64 residual replacement.
struct SysPtr {
  const float *dg, *wx, *wy, *wz, *idg;
  const double *dg8, *wx8, *wy8, *wz8;
  __device__ SysPtr(const float* sys, int64_t ntot)
      : dg(sys), wx(sys + ntot), wy(sys + 2 * ntot), wz(sys + 3 * ntot), idg(sys + 4 * ntot),
        dg8(reinterpret_cast<const double*>(sys + 5 * ntot)), wx8(dg8 + ntot), wy8(dg8 + 2 * ntot),
        wz8(dg8 + 3 * ntot) {}
};

// b_i - (A v)_i in FP64 with the FP64 coefficients (v is FP32, exact in FP64).
template <typename V>
__device__ inline double resid_f64(const SysPtr& s, const FrameDesc& F, unsigned c, double bi, V v) {
  int64_t i = F.n0 + c;
  int64_t xp = F.n0 + mstep_plus(c, F.xm), xn = F.n0 + mstep_minus(c, F.xm);
  int64_t yp = F.n0 + mstep_plus(c, F.ym), yn = F.n0 + mstep_minus(c, F.ym);
  int64_t zp = F.n0 + mstep_plus(c, F.zm), zn = F.n0 + mstep_minus(c, F.zm);
  double a = bi - s.dg8[i] * (double)v(i);
  a += s.wx8[i] * (double)v(xp);
  a += s.wx8[xn] * (double)v(xn);
  a += s.wy8[i] * (double)v(yp);
  a += s.wy8[yn] * (double)v(yn);
  a += s.wz8[i] * (double)v(zp);
  a += s.wz8[zn] * (double)v(zn);
  return a;
}

// ------------------------------------------------------------------ assembly

// ops: HP_ASM_NEUMANN drops the Dirichlet term of the top layer (zero flux on
// every face); HP_ASM_RHO_CONDUCTANCE takes the harmonic mean of rho as face
// conductance, 2 rho_i rho_j / (rho_i + rho_j), instead of that of 1/rho.
__global__ void k_assemble(const FrameDesc* fr, const int* blk2f, const float* rho, float* sys, int64_t ntot,
                           int ops) {
  const FrameDesc F = fr[blk2f[blockIdx.x]];
  int c = (blockIdx.x - F.b0) * NODE_BLOCK + threadIdx.x;
  if (c >= F.n) return;
  int64_t i = F.n0 + c;
  double ri = rho[i];
  // a padded frame: padding cells get identity rows and no faces, a face
  // towards padding is a zero-flux face, the Dirichlet layer is the top of
  // the frame's grid
  const bool pad = F.padded != 0;
  const bool own = !pad || in_region(F, (unsigned)c);
  const bool rho_cond = (ops & HP_ASM_RHO_CONDUCTANCE) != 0;
  auto face = [&](double rj) -> double { return rho_cond ? 2.0 * ri * rj / (ri + rj) : 2.0 / (ri + rj); };
  auto wplus = [&](unsigned m) -> double {
    if (!own || (c & m) == m) return 0.0;
    const unsigned j = mstep_plus(c, m);
    if (pad && !in_region(F, j)) return 0.0;
    return face((double)rho[F.n0 + j]);
  };
  auto wminus = [&](unsigned m) -> double {
    if (!own || (c & m) == 0) return 0.0;
    const unsigned j = mstep_minus(c, m);
    if (pad && !in_region(F, j)) return 0.0;
    return face((double)rho[F.n0 + j]);
  };
  double wpx = wplus(F.xm), wpy = wplus(F.ym), wpz = wplus(F.zm);
  double d = wpx + wminus(F.xm) + wpy + wminus(F.ym) + wpz + wminus(F.zm);
  const bool top = pad ? mcoord((unsigned)c, F.zm) == F.rz - 1 : (c & F.zm) == F.zm;
  if (!(ops & HP_ASM_NEUMANN) && own && top) d += 1.0 / ri;
  if (!own) d = 1.0;
  sys[i] = (float)d;
  sys[ntot + i] = (float)wpx;
  sys[2 * ntot + i] = (float)wpy;
  sys[3 * ntot + i] = (float)wpz;
  sys[4 * ntot + i] = (float)(1.0 / d);
  double* s8 = reinterpret_cast<double*>(sys + 5 * ntot);
  s8[i] = d;
  s8[ntot + i] = wpx;
  s8[2 * ntot + i] = wpy;
  s8[3 * ntot + i] = wpz;
}

__global__ __launch_bounds__(NODE_BLOCK) void k_spmv(const FrameDesc* fr, const int* blk2f, const float* sys,
                                                      int64_t ntot, const float* p, float* q) {
  const int bid = xcd_block(blockIdx.x, gridDim.x);  // stencil neighbours in one L2
  const FrameDesc F = fr[blk2f[bid]];
  int c = (bid - F.b0) * NODE_BLOCK + threadIdx.x;
  if (c >= F.n) return;
  // (A p)_i in FP32: the diagonal term, then the faces +x, -x, +y, -y, +z, -z
  // as FMAs in that order.  The node's own coefficients are read once and q
  // written once: streaming (non-temporal) accesses keep them from evicting
  // the p values that the neighbours read again
  SysPtr s(sys, ntot);
  const int64_t i = F.n0 + c;
  const int64_t xp = F.n0 + mstep_plus(c, F.xm), xn = F.n0 + mstep_minus(c, F.xm);
  const int64_t yp = F.n0 + mstep_plus(c, F.ym), yn = F.n0 + mstep_minus(c, F.ym);
  const int64_t zp = F.n0 + mstep_plus(c, F.zm), zn = F.n0 + mstep_minus(c, F.zm);
  const float dgi = __builtin_nontemporal_load(s.dg + i), wxi = __builtin_nontemporal_load(s.wx + i);
  const float wyi = __builtin_nontemporal_load(s.wy + i), wzi = __builtin_nontemporal_load(s.wz + i);
  float a = dgi * p[i];
  a = fmaf(-wxi, p[xp], a);
  a = fmaf(-s.wx[xn], p[xn], a);
  a = fmaf(-wyi, p[yp], a);
  a = fmaf(-s.wy[yn], p[yn], a);
  a = fmaf(-wzi, p[zp], a);
  a = fmaf(-s.wz[zn], p[zn], a);
  __builtin_nontemporal_store(a, q + i);
}

// ------------------------------------------------------------------ H-matrix stages

template <typename FT>
struct Factors {
  const FT* G;      // [ktot][L][L]
  const FT* B;      // [mtot][LS][LS]
  const FT* Ut;     // [ntot][LS]
  const FT* Vt;     // [ntot][LS]
  const float* lam; // [ntot]
};

// Load n consecutive factor values as floats (vectorised).
template <typename FT, int N>
__device__ inline void load_vec(const FT* p, float* out) {
  if constexpr (sizeof(FT) == 2 && N % 8 == 0) {
    // 16-byte loads (every caller's range starts on a multiple of 8 elements)
    const uint4* q = reinterpret_cast<const uint4*>(p);
#pragma unroll
    for (int i = 0; i < N / 8; ++i) {
      const uint4 u = q[i];
      const uint32_t w[4] = {u.x, u.y, u.z, u.w};
#pragma unroll
      for (int h = 0; h < 4; ++h) {
        out[8 * i + 2 * h] = bf16_to_f32((uint16_t)(w[h] & 0xffff));
        out[8 * i + 2 * h + 1] = bf16_to_f32((uint16_t)(w[h] >> 16));
      }
    }
  } else if constexpr (sizeof(FT) == 2) {
    static_assert(N % 4 == 0, "bf16 vector loads come in fours");
    const uint2* q = reinterpret_cast<const uint2*>(p);
#pragma unroll
    for (int i = 0; i < N / 4; ++i) {
      uint2 u = q[i];
      out[4 * i + 0] = bf16_to_f32((uint16_t)(u.x & 0xffff));
      out[4 * i + 1] = bf16_to_f32((uint16_t)(u.x >> 16));
      out[4 * i + 2] = bf16_to_f32((uint16_t)(u.y & 0xffff));
      out[4 * i + 3] = bf16_to_f32((uint16_t)(u.y >> 16));
    }
  } else {
    static_assert(N % 4 == 0, "f32 vector loads come in fours");
    const float4* q = reinterpret_cast<const float4*>(p);
#pragma unroll
    for (int i = 0; i < N / 4; ++i) {
      float4 u = q[i];
      out[4 * i + 0] = u.x;
      out[4 * i + 1] = u.y;
      out[4 * i + 2] = u.z;
      out[4 * i + 3] = u.w;
    }
  }
}

// Leaf stage of y = M r for leaf kg (global index) whose rows start at row0:
//   y = G_k r_k + lam r / A_ii        -> y[row0 .. row0+L)
//   u = Ut_k^T r_k,  v = Vt_k^T r_k   -> uh[kg], vh[kg]
// split into load() (this thread's slice of G, Ut, Vt and the Jacobi gate,
// independent of r, so kernels issue it before their reductions) and
// apply() (rs: r_k in LDS; all threads take part).
template <int L, int LS, typename FT>
struct LeafPre {
  static constexpr int TPR = LEAF_THREADS / L;   // threads per row (G product)
  static constexpr int CPT = L / TPR;            // columns per thread
  static constexpr int GR = LEAF_THREADS / LS;   // row groups (restriction)
  static constexpr int RPG = L / GR;             // rows per group
  static_assert(RPG >= 1, "leaf too small for the restriction layout");
  float g[CPT], u[RPG], v[RPG], lamv, idgv;  // the gate lam / A_ii is formed in apply(): no wait in load()

  __device__ inline void load(int64_t kg, int64_t row0, const Factors<FT>& fac, const float* idg) {
    const int t = threadIdx.x, row = t / TPR, c0 = (t % TPR) * CPT;
    load_vec<FT, CPT>(fac.G + (kg * L + row) * L + c0, g);
    const int s = t % LS, grp = t / LS;
#pragma unroll
    for (int j = 0; j < RPG; ++j) {
      const int64_t l = row0 + grp * RPG + j;
      u[j] = ldf(fac.Ut, l * LS + s);
      v[j] = ldf(fac.Vt, l * LS + s);
    }
    lamv = fac.lam[row0 + row];  // every lane (no divergent branch); only the row's lead uses them
    idgv = idg[row0 + row];
  }

  __device__ inline void apply(int64_t kg, int64_t row0, const float* rs, float* y, float* uh, float* vh,
                               float* red) const {
    const int t = threadIdx.x;
    {
      const int row = t / TPR, c0 = (t % TPR) * CPT;
      float a = 0.f;
#pragma unroll
      for (int c = 0; c < CPT; ++c) a = fmaf(g[c], rs[c0 + c], a);
      a = group_sum<TPR>(a);
      const float gate = lamv * idgv;
      if (t % TPR == 0) y[row0 + row] = fmaf(gate, rs[row], a);
    }
    const int s = t % LS, grp = t / LS;
    float au = 0.f, av = 0.f;
#pragma unroll
    for (int j = 0; j < RPG; ++j) {
      const float rl = rs[grp * RPG + j];
      au = fmaf(u[j], rl, au);
      av = fmaf(v[j], rl, av);
    }
    // reduce the groups held inside one wave (lanes s + LS*q)
#pragma unroll
    for (int o = 32; o >= LS; o >>= 1) {
      au += __shfl_xor(au, o, 64);
      av += __shfl_xor(av, o, 64);
    }
    const int w = t >> 6;
    if ((t & 63) < LS) {
      red[w * 2 * LS + s] = au;
      red[w * 2 * LS + LS + s] = av;
    }
    __syncthreads();
    if (t < 2 * LS) {
      float acc = 0.f;
      for (int q = 0; q < LEAF_THREADS / 64; ++q) acc += red[q * 2 * LS + t];
      if (t < LS) uh[kg * LS + t] = acc;
      else vh[kg * LS + t - LS] = acc;
    }
  }
};

template <int L, int LS, typename FT>
__device__ inline void leaf_stage(int64_t kg, int64_t row0, const float* rs, const Factors<FT>& fac,
                                  const float* idg, float* y, float* uh, float* vh, float* red) {
  LeafPre<L, LS, FT> pre;
  pre.load(kg, row0, fac, idg);
  pre.apply(kg, row0, rs, y, uh, vh, red);
}

// Prolongation for leaf kg: y[rows] += Ut_k T^r + Vt_k T^c.  load() reads
// this thread's Ut, Vt entries (row t / TPR, entries s0 ..), apply() returns
// the updated value of the row in the lane with t % TPR == 0, else 0; the
// caller passes the row's current y value in yrow (lane t % TPR == 0).
template <int L, int LS, typename FT>
struct ProlongPre {
  static constexpr int TPR = LEAF_THREADS / L;
  static constexpr int SPT = LS / TPR;  // coarse entries per thread
  float u[SPT], v[SPT];

  __device__ inline void load(int64_t row0, const Factors<FT>& fac) {
    const int t = threadIdx.x, row = t / TPR, s0 = (t % TPR) * SPT;
    if constexpr (SPT >= 4) {
      load_vec<FT, SPT>(fac.Ut + (row0 + row) * LS + s0, u);
      load_vec<FT, SPT>(fac.Vt + (row0 + row) * LS + s0, v);
    } else {
#pragma unroll
      for (int s = 0; s < SPT; ++s) {
        u[s] = ldf(fac.Ut, (row0 + row) * LS + s0 + s);
        v[s] = ldf(fac.Vt, (row0 + row) * LS + s0 + s);
      }
    }
  }

  __device__ inline float apply(const float* trs, const float* tcs, float yrow) const {
    const int s0 = (threadIdx.x % TPR) * SPT;
    float a = 0.f;
#pragma unroll
    for (int s = 0; s < SPT; ++s) {
      if constexpr (SPT >= 4) {
        a = fmaf(u[s], trs[s0 + s], fmaf(v[s], tcs[s0 + s], a));
      } else {
        a = fmaf(u[s], trs[s0 + s], a);
        a = fmaf(v[s], tcs[s0 + s], a);
      }
    }
    a = group_sum<TPR>(a);
    return yrow + a;
  }
};

// Coarse coupling of one tile (paper Sec. 5 strip aggregation and coarse
// coupling), run by one whole block.  Tile m = (j, i), S = 2^j leaves a side:
//   s^r = sum of u over the row strip (leaves [2iS, 2iS+S)),
//   s^c = sum of v over the column strip (leaves [2iS+S, 2iS+2S)),
//   t^r = B_m s^c,  t^c = B_m^T s^r,
// written to tr / tc [tile][LS].  The strip sums run in a fixed order
// (NCH interleaved chunks of leaves, then the chunks in order).  load() takes
// the per-thread chunk sums and the B entries (no barrier, so a kernel can
// issue it ahead of its reductions); finish() reduces and multiplies.
template <int LS, typename FT>
struct TilePre {
  static constexpr int NCH = LEAF_THREADS / LS;
  float a, c, b[LS];
  int64_t mg;

  __device__ inline void load(const FrameDesc& F, int m, const float* uh, const float* vh, const FT* B) {
    const int K = F.K, t = threadIdx.x;
    int j = 0;
    while (m >= K - (K >> (j + 1))) ++j;
    const int i = m - (K - (K >> j)), S = 1 << j;
    const int s = t % LS, ch = t / LS;
    const int64_t lr = (int64_t)F.k0 + 2 * i * S, lc = lr + S;
    a = 0.f;
    c = 0.f;
    // the chunk's loads are issued U at a time before their (in-order) sums:
    // a load-add chain would expose one memory latency per leaf
    constexpr int U = 8;
    for (int k0 = ch; k0 < S; k0 += U * NCH) {
      float ua[U], va[U];
#pragma unroll
      for (int q = 0; q < U; ++q) {
        const int k = k0 + q * NCH;
        ua[q] = k < S ? uh[(lr + k) * LS + s] : 0.f;
        va[q] = k < S ? vh[(lc + k) * LS + s] : 0.f;
      }
#pragma unroll
      for (int q = 0; q < U; ++q)
        if (k0 + q * NCH < S) {
          a += ua[q];
          c += va[q];
        }
    }
    mg = (int64_t)F.m0 + m;
    const FT* Bm = B + mg * LS * LS;
    if (t < LS) {
#pragma unroll
      for (int u = 0; u < LS; ++u) b[u] = ldf(Bm, t * LS + u);   // row t of B
    } else if (t < 2 * LS) {
#pragma unroll
      for (int u = 0; u < LS; ++u) b[u] = ldf(Bm, u * LS + (t - LS));   // column of B
    }
  }

  __device__ inline void finish(float* tr, float* tc) const {
    __shared__ float pr[NCH][LS], pc[NCH][LS], sr[LS], sc[LS];
    const int t = threadIdx.x, s = t % LS, ch = t / LS;
    pr[ch][s] = a;
    pc[ch][s] = c;
    __syncthreads();
    if (t < LS) {
      float x = 0.f;
      for (int q = 0; q < NCH; ++q) x += pr[q][t];
      sr[t] = x;
    } else if (t < 2 * LS) {
      float x = 0.f;
      for (int q = 0; q < NCH; ++q) x += pc[q][t - LS];
      sc[t - LS] = x;
    }
    __syncthreads();
    if (t < LS) {
      float x = 0.f;
#pragma unroll
      for (int u = 0; u < LS; ++u) x = fmaf(b[u], sc[u], x);
      tr[mg * LS + t] = x;
    } else if (t < 2 * LS) {
      float x = 0.f;
#pragma unroll
      for (int u = 0; u < LS; ++u) x = fmaf(b[u], sr[u], x);
      tc[mg * LS + t - LS] = x;
    }
  }
};

// Gather of leaf kg (global index) for entry s < LS: T^r = sum of t^r over the
// tiles where the leaf is on the row side, T^c over those where it is on the
// column side, levels in increasing order.
template <int LS>
__device__ inline void gather_leaf(const FrameDesc& F, int64_t kg, int s, const float* tr, const float* tc,
                                   float& Tr, float& Tc) {
  const int k = (int)(kg - F.k0), K = F.K;
  float a = 0.f, c = 0.f;
  constexpr int JMAX = 16;  // every level's load in flight at once (up to 2^16 leaves)
  if (F.J <= JMAX) {
    float tv[JMAX];
#pragma unroll
    for (int j = 0; j < JMAX; ++j) {
      tv[j] = 0.f;
      if (j < F.J) {
        const int64_t m = (int64_t)F.m0 + K - (K >> j) + (k >> (j + 1));
        tv[j] = ((k >> j) & 1) == 0 ? tr[m * LS + s] : tc[m * LS + s];
      }
    }
#pragma unroll
    for (int j = 0; j < JMAX; ++j)
      if (j < F.J) {
        if (((k >> j) & 1) == 0) a += tv[j];
        else c += tv[j];
      }
  } else {
    for (int j = 0; j < F.J; ++j) {
      const int64_t m = (int64_t)F.m0 + K - (K >> j) + (k >> (j + 1));
      if (((k >> j) & 1) == 0) a += tr[m * LS + s];
      else c += tc[m * LS + s];
    }
  }
  Tr = a;
  Tc = c;
}

// ------------------------------------------------------------------ standalone apply

template <int L, int LS, typename FT>
__global__ __launch_bounds__(LEAF_THREADS) void k_apply_leaf(const FrameDesc* fr, const int* leaf2f,
                                                             const float* sys, int64_t ntot, Factors<FT> fac,
                                                             const float* r, float* y, float* uh, float* vh) {
  __shared__ float rs[L];
  __shared__ float red[(LEAF_THREADS / 64) * 2 * LS];
  const int64_t kg = blockIdx.x;
  const FrameDesc F = fr[leaf2f[kg]];
  const int64_t row0 = F.n0 + (kg - F.k0) * L;
  LeafPre<L, LS, FT> pre;
  pre.load(kg, row0, fac, sys + 4 * ntot);  // G, Ut, Vt and the gate ahead of the barrier
  for (int l = threadIdx.x; l < L; l += blockDim.x) rs[l] = r[row0 + l];
  __syncthreads();
  pre.apply(kg, row0, rs, y, uh, vh, red);
}

// One block per coarse block (a tile, or a placeholder for a frame without
// tiles).
template <int LS, typename FT>
__global__ __launch_bounds__(LEAF_THREADS) void k_apply_coarse(const FrameDesc* fr, const int2* cblk,
                                                               Factors<FT> fac, const float* uh, const float* vh,
                                                               float* tr, float* tc) {
  const int2 cb = cblk[blockIdx.x];
  if (cb.y < 0) return;
  const FrameDesc F = fr[cb.x];
  TilePre<LS, FT> pre;
  pre.load(F, cb.y, uh, vh, fac.B);
  pre.finish(tr, tc);
}

template <int L, int LS, typename FT>
__global__ __launch_bounds__(LEAF_THREADS) void k_apply_prolong(const FrameDesc* fr, const int* leaf2f,
                                                                Factors<FT> fac, const float* tr,
                                                                const float* tc, float* y) {
  __shared__ float trs[LS], tcs[LS];
  const int64_t kg = blockIdx.x;
  const FrameDesc F = fr[leaf2f[kg]];
  const int64_t row0 = F.n0 + (kg - F.k0) * L;
  ProlongPre<L, LS, FT> pre;
  pre.load(row0, fac);
  constexpr int TPR = LEAF_THREADS / L;
  const int row = threadIdx.x / TPR;
  const float yr = (threadIdx.x % TPR == 0) ? y[row0 + row] : 0.f;
  if (threadIdx.x < LS) gather_leaf<LS>(F, kg, threadIdx.x, tr, tc, trs[threadIdx.x], tcs[threadIdx.x]);
  __syncthreads();
  const float v = pre.apply(trs, tcs, yr);
  if (threadIdx.x % TPR == 0) y[row0 + row] = v;
}

// ------------------------------------------------------------------ PCG kernels
//
// Synchronisation is by kernel boundaries only: no kernel reads data that
// another block of the same kernel writes.  Every block of a kernel reduces
// the partials that the previous kernel wrote for its frame, in the same fixed
// order, so all blocks of a frame reach bit-identical scalars and decisions;
// the frame's lead block writes the frame state, always to the slot that no
// block of that kernel reads.  Jacobi / identity: an iteration at parity par
// reads st[2f + par] in its first kernel and leaves its result in
// st[2f + (par ^ 1)].  Learned preconditioner: k_spmv_p reads slot 0 and
// writes slot 1, k_update_hmat reads slot 1, k_coarse_check reads slot 1 and
// writes slot 0, k_prolong reads slot 0.


__device__ inline bool is_replacement(const FrameState& s, const SolveParams& prm, int u) {
  return s.force_rc || (prm.recompute_every > 0 && u % prm.recompute_every == 0);
}

// Stop decisions after update u with ||r||^2 = rr.  A residual that passes the
// tolerance stops the frame only when it is a true (replaced) residual; a
// passing recurrence residual forces a replacement on the next update.
__device__ inline bool stop_checks(FrameState& s, const SolveParams& prm, int u, double rr, bool replaced) {
  s.it = u;
  s.rr = rr;
  s.force_rc = 0;
  if (rr <= s.target) {
    if (replaced) {
      s.flags |= HP_CONVERGED;
      return true;
    }
    s.force_rc = 1;
  }
  double rn = sqrt(rr);
  if (prm.stagnation && u % 100 == 0) {
    if (rn > 0.5 * s.rwin) {
      s.flags |= HP_STAGNATED;
      return true;
    }
    s.rwin = rn;
  }
  if (u >= prm.max_iter) {
    s.flags |= HP_MAXITER;
    return true;
  }
  return false;
}

// First kernel of an iteration (node blocks): [Jacobi / identity: stop checks
// of the previous update], positivity of rho' = r.z, beta = rho'/rho,
// p = z + beta p_old at the 7 stencil points, q = A p, partials of p.q.
template <bool SIMPLE>
__global__ __launch_bounds__(NODE_BLOCK) void k_spmv_p(const FrameDesc* fr, const int* blk2f, PcgBufs B_, int rd,
                                                       int wr, const float* pold, float* pnew) {
  __shared__ double red[NODE_BLOCK / 64];
  const int bid = xcd_block(blockIdx.x, gridDim.x);  // stencil neighbours in one L2
  const int f = blk2f[bid];
  const FrameDesc F = fr[f];
  FrameState S = load_state(B_.st + 2 * f + rd);
  FrameState* out = B_.st + 2 * f + wr;
  const bool lead = bid == F.b0 && threadIdx.x == 0;
  if (S.done) {
    if (lead) store_state(out, S);
    return;
  }
  const SolveParams prm = *B_.prm;
  // stencil operands (independent of beta) before the reductions
  const int c = (bid - F.b0) * NODE_BLOCK + threadIdx.x;
  const bool own = c < F.n;
  float zv[7], pv[7], cf[7];
  if (own) {
    const unsigned cu = (unsigned)c;
    const int64_t nb[7] = {F.n0 + c,
                           F.n0 + mstep_plus(cu, F.xm), F.n0 + mstep_minus(cu, F.xm),
                           F.n0 + mstep_plus(cu, F.ym), F.n0 + mstep_minus(cu, F.ym),
                           F.n0 + mstep_plus(cu, F.zm), F.n0 + mstep_minus(cu, F.zm)};
    SysPtr sp(B_.sys, B_.ntot);
    cf[0] = sp.dg[nb[0]];
    cf[1] = -sp.wx[nb[0]];
    cf[2] = -sp.wx[nb[2]];
    cf[3] = -sp.wy[nb[0]];
    cf[4] = -sp.wy[nb[4]];
    cf[5] = -sp.wz[nb[0]];
    cf[6] = -sp.wz[nb[6]];
#pragma unroll
    for (int e = 0; e < 7; ++e) {
      zv[e] = B_.z[nb[e]];
      pv[e] = pold[nb[e]];
    }
  }
  if (SIMPLE && !S.fresh) {
    const int u = S.it + 1;
    const bool rep = is_replacement(S, prm, u);
    const double rr = frame_sum(B_.part_rr + F.b0, F.nb, red);
    if (stop_checks(S, prm, u, rr, rep)) {
      if (lead) {
        S.done = 1;
        store_state(out, S);
        frame_stopped(B_, f);
      }
      return;
    }
  }
  S.fresh = 0;
  const double rz = SIMPLE ? frame_sum(B_.part_rz + F.b0, F.nb, red) : frame_sum(B_.part_rz + F.k0, F.K, red);
  if (!(rz > 0.0) || !isfinite(rz)) {
    if (lead) {
      S.flags |= HP_NOT_SPD;
      S.done = 1;
      store_state(out, S);
      frame_stopped(B_, f);
    }
    return;
  }
  S.beta = rz / S.rho;
  S.rho = rz;
  const float beta = (float)S.beta;
  double pq = 0.0;
  if (own) {
    // the same operation order as k_spmv (diagonal, then +x, -x, +y, -y, +z,
    // -z) with p = z + beta p_old
    float P[7];
#pragma unroll
    for (int e = 0; e < 7; ++e) P[e] = fmaf(beta, pv[e], zv[e]);
    float qi = cf[0] * P[0];
#pragma unroll
    for (int e = 1; e < 7; ++e) qi = fmaf(cf[e], P[e], qi);
    pnew[F.n0 + c] = P[0];
    B_.q[F.n0 + c] = qi;
    pq = (double)P[0] * (double)qi;
  }
  double bs = block_sum(pq, red);
  if (threadIdx.x == 0) B_.part_pq[bid] = bs;
  if (lead) store_state(out, S);
}

// x accumulates in FP64 (x += alpha p with alpha in FP64); r, p, q are FP32.
// NodePre holds thread l's p, q, r, x (l < L), loaded before the reductions.
struct NodePre {
  float p, q, r;
  double x;
};

template <int L>
__device__ inline NodePre xr_load(int64_t row0, const PcgBufs& B_, const double* xold, const float* p) {
  NodePre n{0.f, 0.f, 0.f, 0.0};
  if (threadIdx.x < L) {
    const int64_t i = row0 + threadIdx.x;
    n.p = p[i];
    n.q = B_.q[i];
    n.r = B_.r[i];
    n.x = xold[i];
  }
  return n;
}

template <int L>
__device__ inline double xr_update(const FrameDesc& F, int64_t row0, const PcgBufs& B_, const NodePre& n,
                                   const double* xold, double* xnew, const float* p, double alpha, bool recompute,
                                   float* rs) {
  static_assert(L <= LEAF_THREADS, "one row per thread");
  double rr = 0.0;
  const int l = threadIdx.x;
  if (l < L) {
    const int64_t i = row0 + l;
    xnew[i] = fma(alpha, (double)n.p, n.x);
    float ri;
    if (recompute) {
      SysPtr s(B_.sys, B_.ntot);
      const unsigned c = (unsigned)(i - F.n0);
      ri = (float)resid_f64(s, F, c, (double)B_.b[i], [&](int64_t j) { return fma(alpha, (double)p[j], xold[j]); });
    } else {
      ri = fmaf(-(float)alpha, n.q, n.r);
    }
    B_.r[i] = ri;
    rs[l] = ri;
    rr = (double)ri * (double)ri;
  }
  return rr;
}

// Second kernel (leaf blocks): alpha = rho / p.q, x and r update (or FP64
// residual replacement), leaf stage of z = M r, partials of ||r||^2.
template <int L, int LS, typename FT>
__global__ __launch_bounds__(LEAF_THREADS) void k_update_hmat(const FrameDesc* fr, const int* leaf2f, PcgBufs B_,
                                                              Factors<FT> fac, const double* xold, double* xnew,
                                                              const float* p) {
  __shared__ float rs[L];
  __shared__ float red[(LEAF_THREADS / 64) * 2 * LS];
  __shared__ double dred[LEAF_THREADS / 64];
  const int64_t kg = blockIdx.x;
  // every frame holds K L rows in leaf order (n0 = k0 L), so the leaf's rows
  // and factors are known before its frame: everything that does not depend
  // on alpha is requested beside the frame's descriptor and state
  const int64_t row0 = kg * L;
  const int f = leaf2f[kg];
  LeafPre<L, LS, FT> pre;
  pre.load(kg, row0, fac, B_.sys + 4 * B_.ntot);
  const NodePre np = xr_load<L>(row0, B_, xold, p);
  const FrameDesc F = fr[f];
  const FrameState S = load_state(B_.st + 2 * f + 1);
  if (S.done) return;
  const SolveParams prm = *B_.prm;
  const bool rep = is_replacement(S, prm, S.it + 1);
  const double alpha = S.rho / frame_sum(B_.part_pq + F.b0, F.nb, dred);
  double rr = xr_update<L>(F, row0, B_, np, xold, xnew, p, alpha, rep, rs);
  __syncthreads();
  pre.apply(kg, row0, rs, B_.z, B_.uh, B_.vh, red);
  double bs = block_sum(rr, dred);
  if (threadIdx.x == 0) B_.part_rr[kg] = bs;
}

// Setup check for Jacobi / identity (one block per frame): ||b||, the target
// and the check of r0 from the node-block partials.
__global__ __launch_bounds__(LEAF_THREADS) void k_frame_setup(const FrameDesc* fr, PcgBufs B_) {
  __shared__ double dred[LEAF_THREADS / 64];
  const int f = blockIdx.x;
  const FrameDesc F = fr[f];
  FrameState* sp = B_.st + 2 * f;
  FrameState S = load_state(sp);
  if (S.done) return;
  const SolveParams prm = *B_.prm;
  const double rr = frame_sum(B_.part_rr + F.b0, F.nb, dred);
  const double bb = frame_sum(B_.part_pq + F.b0, F.nb, dred);
  S.bnorm = sqrt(bb);
  S.target = (prm.tol * S.bnorm) * (prm.tol * S.bnorm);
  S.rr = rr;
  S.rwin = sqrt(rr);
  S.it = 0;
  S.fresh = 1;
  bool stop = true;
  if (rr <= S.target) S.flags |= HP_CONVERGED;
  else if (prm.max_iter <= 0) S.flags |= HP_MAXITER;
  else stop = false;
  if (threadIdx.x == 0) {
    if (stop) {
      S.done = 1;
      frame_stopped(B_, f);
    }
    store_state(sp, S);
  }
}

// Third kernel of the learned preconditioner (coarse blocks: one per tile,
// a placeholder block for a frame without tiles): the stop checks of the
// update (or, at setup, ||b||, the target and the check of r0) from the
// per-leaf partials, computed by every block of the frame; the frame's lead
// block (its first) writes the state.  A frame that goes on then couples the
// block's tile.
template <int LS, typename FT>
__global__ __launch_bounds__(LEAF_THREADS) void k_coarse_check(const FrameDesc* fr, const int2* cblk, PcgBufs B_,
                                                               Factors<FT> fac, int setup) {
  __shared__ double dred[LEAF_THREADS / 64];
  const int2 cb = cblk[blockIdx.x];
  const int f = cb.x;
  const bool lead = cb.y <= 0 && threadIdx.x == 0;
  const FrameDesc F = fr[f];
  FrameState S = load_state(B_.st + 2 * f + 1);
  if (S.done) {
    if (lead) store_state(B_.st + 2 * f, S);
    return;
  }
  TilePre<LS, FT> pre;
  if (cb.y >= 0) pre.load(F, cb.y, B_.uh, B_.vh, fac.B);  // ahead of the reductions
  const SolveParams prm = *B_.prm;
  const double rr = frame_sum(B_.part_rr + F.k0, F.K, dred);
  bool stop;
  if (setup) {
    const double bb = frame_sum(B_.part_pq + F.k0, F.K, dred);
    S.bnorm = sqrt(bb);
    S.target = (prm.tol * S.bnorm) * (prm.tol * S.bnorm);
    S.rr = rr;
    S.rwin = sqrt(rr);
    S.it = 0;
    S.fresh = 1;
    stop = true;
    if (rr <= S.target) S.flags |= HP_CONVERGED;
    else if (prm.max_iter <= 0) S.flags |= HP_MAXITER;
    else stop = false;
  } else {
    const int u = S.it + 1;
    stop = stop_checks(S, prm, u, rr, is_replacement(S, prm, u));
  }
  if (stop) S.done = 1;
  if (lead) {
    store_state(B_.st + 2 * f, S);
    if (stop) frame_stopped(B_, f);
  }
  if (stop || cb.y < 0) return;
  pre.finish(B_.Tr, B_.Tc);
}

// Last kernel (leaf blocks): gather T^r, T^c, z += Ut T^r + Vt T^c,
// partials of r.z.
template <int L, int LS, typename FT>
__global__ __launch_bounds__(LEAF_THREADS) void k_prolong(const FrameDesc* fr, const int* leaf2f, PcgBufs B_,
                                                          Factors<FT> fac) {
  __shared__ float trs[LS], tcs[LS];
  __shared__ double dred[LEAF_THREADS / 64];
  const int64_t kg = blockIdx.x;
  const int f = leaf2f[kg];
  const FrameDesc F = fr[f];
  if (B_.st[2 * f].done) return;
  const int64_t row0 = F.n0 + (kg - F.k0) * L;
  constexpr int TPR = LEAF_THREADS / L;
  const int row = threadIdx.x / TPR;
  const bool lead = threadIdx.x % TPR == 0;
  ProlongPre<L, LS, FT> pre;
  pre.load(row0, fac);
  float zr = lead ? B_.z[row0 + row] : 0.f;
  const float rr = lead ? B_.r[row0 + row] : 0.f;
  if (threadIdx.x < LS) gather_leaf<LS>(F, kg, threadIdx.x, B_.Tr, B_.Tc, trs[threadIdx.x], tcs[threadIdx.x]);
  __syncthreads();
  zr = pre.apply(trs, tcs, zr);
  double rz = 0.0;
  if (lead) {
    B_.z[row0 + row] = zr;
    rz = (double)rr * (double)zr;
  }
  double bs = block_sum(rz, dred);
  if (threadIdx.x == 0) B_.part_rz[kg] = bs;
}

// Setup for the learned preconditioner (leaf blocks): r = b - A x0 in FP64,
// p0 = 0, the leaf stage of z = M r, partials of ||r||^2 and ||b||^2.
template <int L, int LS, typename FT>
__global__ __launch_bounds__(LEAF_THREADS) void k_setup_hmat(const FrameDesc* fr, const int* leaf2f, PcgBufs B_,
                                                             Factors<FT> fac) {
  __shared__ float rs[L];
  __shared__ float red[(LEAF_THREADS / 64) * 2 * LS];
  __shared__ double dred[LEAF_THREADS / 64];
  const int64_t kg = blockIdx.x;
  const int f = leaf2f[kg];
  const FrameDesc F = fr[f];
  if (B_.st[2 * f].done) return;
  const int64_t row0 = F.n0 + (kg - F.k0) * L;
  SysPtr s(B_.sys, B_.ntot);
  double rr = 0.0, bb = 0.0;
  for (int l = threadIdx.x; l < L; l += blockDim.x) {
    int64_t i = row0 + l;
    float ri = (float)resid_f64(s, F, (unsigned)(i - F.n0), (double)B_.b[i], [&](int64_t j) { return B_.x0[j]; });
    B_.r[i] = ri;
    B_.p0[i] = 0.f;
    rs[l] = ri;
    rr += (double)ri * (double)ri;
    bb += (double)B_.b[i] * (double)B_.b[i];
  }
  __syncthreads();
  leaf_stage<L, LS, FT>(kg, row0, rs, fac, B_.sys + 4 * B_.ntot, B_.z, B_.uh, B_.vh, red);
  double rsum = block_sum(rr, dred);
  double bsum = block_sum(bb, dred);
  if (threadIdx.x == 0) {
    B_.part_rr[kg] = rsum;
    B_.part_pq[kg] = bsum;
  }
}

// Setup for Jacobi / identity (node blocks): r = b - A x0, z, p0 = 0 and the
// partials of ||r||^2, r.z and ||b||^2.
template <bool JAC>
__global__ __launch_bounds__(NODE_BLOCK) void k_setup_simple(const FrameDesc* fr, const int* blk2f, PcgBufs B_) {
  __shared__ double red[NODE_BLOCK / 64];
  const int f = blk2f[blockIdx.x];
  const FrameDesc F = fr[f];
  if (B_.st[2 * f].done) return;
  SysPtr s(B_.sys, B_.ntot);
  int c = (blockIdx.x - F.b0) * NODE_BLOCK + threadIdx.x;
  double rr = 0.0, bb = 0.0, rz = 0.0;
  if (c < F.n) {
    int64_t i = F.n0 + c;
    float ri = (float)resid_f64(s, F, c, (double)B_.b[i], [&](int64_t j) { return B_.x0[j]; });
    float zi = JAC ? ri * s.idg[i] : ri;
    B_.r[i] = ri;
    B_.z[i] = zi;
    B_.p0[i] = 0.f;
    rr = (double)ri * (double)ri;
    rz = (double)ri * (double)zi;
    bb = (double)B_.b[i] * (double)B_.b[i];
  }
  double a = block_sum(rr, red), b = block_sum(bb, red), cz = block_sum(rz, red);
  if (threadIdx.x == 0) {
    B_.part_rr[blockIdx.x] = a;
    B_.part_rz[blockIdx.x] = cz;
    B_.part_pq[blockIdx.x] = b;
  }
}

// Second kernel for Jacobi / identity (node blocks): alpha, x, r (or FP64
// replacement), z = D^-1 r or r, partials of ||r||^2 and r.z.
template <bool JAC>
__global__ __launch_bounds__(NODE_BLOCK) void k_update_simple(const FrameDesc* fr, const int* blk2f, PcgBufs B_,
                                                              int par, const double* xold, double* xnew,
                                                              const float* p) {
  __shared__ double red[NODE_BLOCK / 64];
  const int f = blk2f[blockIdx.x];
  const FrameDesc F = fr[f];
  const FrameState S = load_state(B_.st + 2 * f + (par ^ 1));
  if (S.done) return;
  const SolveParams prm = *B_.prm;
  const bool rep = is_replacement(S, prm, S.it + 1);
  const double alpha = S.rho / frame_sum(B_.part_pq + F.b0, F.nb, red);
  const float af = (float)alpha;
  SysPtr s(B_.sys, B_.ntot);
  int c = (blockIdx.x - F.b0) * NODE_BLOCK + threadIdx.x;
  double rr = 0.0, rz = 0.0;
  if (c < F.n) {
    int64_t i = F.n0 + c;
    xnew[i] = fma(alpha, (double)p[i], xold[i]);
    float ri;
    if (rep)
      ri = (float)resid_f64(s, F, c, (double)B_.b[i], [&](int64_t j) { return fma(alpha, (double)p[j], xold[j]); });
    else
      ri = fmaf(-af, B_.q[i], B_.r[i]);
    float zi = JAC ? ri * s.idg[i] : ri;
    B_.r[i] = ri;
    B_.z[i] = zi;
    rr = (double)ri * (double)ri;
    rz = (double)ri * (double)zi;
  }
  double a = block_sum(rr, red), cz = block_sum(rz, red);
  if (threadIdx.x == 0) {
    B_.part_rr[blockIdx.x] = a;
    B_.part_rz[blockIdx.x] = cz;
  }
}

// After a pass: a frame that did an odd number of updates holds x in x1.
// With stopped_only, frames still iterating are left alone (x0 is the other
// half of their iterate pair).
__global__ void k_finalize_x(const FrameDesc* fr, const int* blk2f, const FrameState* st, const double* x1,
                             double* x0, int stopped_only) {
  const int f = blk2f[blockIdx.x];
  const FrameDesc F = fr[f];
  const FrameState S = load_state(st + 2 * f);
  if (!S.active || (S.it & 1) == 0 || (stopped_only && !S.done)) return;
  int c = (blockIdx.x - F.b0) * NODE_BLOCK + threadIdx.x;
  if (c < F.n) x0[F.n0 + c] = x1[F.n0 + c];
}

// ------------------------------------------------------------------ host launchers




hp_status launch_assemble(const LaunchGeom& g, const float* rho, float* sys, int ops) {
  hipLaunchKernelGGL(k_assemble, dim3(g.nblk), dim3(NODE_BLOCK), 0, g.stream, g.fr, g.blk2f, rho, sys, g.ntot, ops);
  HP_HIP(hipGetLastError());
  return HP_OK;
}

hp_status launch_spmv(const LaunchGeom& g, const float* sys, const float* p, float* q) {
  hipLaunchKernelGGL(k_spmv, dim3(g.nblk), dim3(NODE_BLOCK), 0, g.stream, g.fr, g.blk2f, sys, g.ntot, p, q);
  HP_HIP(hipGetLastError());
  return HP_OK;
}

template <int L, int LS, typename FT>
static hp_status apply_t(const LaunchGeom& g, const float* sys, const void* fbase, const int64_t* offs,
                         const float* r, float* y, float* uh, float* vh, float* Tr, float* Tc) {
  const char* base = (const char*)fbase;
  Factors<FT> fac{(const FT*)(base + offs[0]), (const FT*)(base + offs[1]), (const FT*)(base + offs[2]),
                  (const FT*)(base + offs[3]), (const float*)(base + offs[4])};
  hipLaunchKernelGGL((k_apply_leaf<L, LS, FT>), dim3(g.ktot), dim3(LEAF_THREADS), 0, g.stream, g.fr, g.leaf2f, sys,
                     g.ntot, fac, r, y, uh, vh);
  hipLaunchKernelGGL((k_apply_coarse<LS, FT>), dim3(g.ncblk), dim3(LEAF_THREADS), 0, g.stream, g.fr, g.cblk, fac,
                     uh, vh, Tr, Tc);
  hipLaunchKernelGGL((k_apply_prolong<L, LS, FT>), dim3(g.ktot), dim3(LEAF_THREADS), 0, g.stream, g.fr, g.leaf2f,
                     fac, Tr, Tc, y);
  HP_HIP(hipGetLastError());
  return HP_OK;
}

hp_status launch_apply(const LaunchGeom& g, int L, int LS, int fdtype, const float* sys, const void* fac,
                       const int64_t* offs, const float* r, float* y, float* uh, float* vh, float* Tr, float* Tc) {
  if (L == 64 && LS == 16) {
    return fdtype == HP_BF16 ? apply_t<64, 16, uint16_t>(g, sys, fac, offs, r, y, uh, vh, Tr, Tc)
                             : apply_t<64, 16, float>(g, sys, fac, offs, r, y, uh, vh, Tr, Tc);
  }
  if (L == 32 && LS == 8) {
    return fdtype == HP_BF16 ? apply_t<32, 8, uint16_t>(g, sys, fac, offs, r, y, uh, vh, Tr, Tc)
                             : apply_t<32, 8, float>(g, sys, fac, offs, r, y, uh, vh, Tr, Tc);
  }
  return set_error(HP_E_SHAPE, "apply: unsupported (L, L_s) = (%d, %d); supported (64, 16), (32, 8)", L, LS);
}

// ------------------------------------------------------------------ one-frame apply without allocation
//
// hp_apply_static runs the apply kernels above on one frame without a batch.
// Its workspace (the one-frame table, leaf -> frame map and coarse-block list
// the kernels index, and the coarse vectors u, v, t^r, t^c) lives in
// `scratch`, a fixed array of this translation unit's device code.  In host
// code the array's name is only a stand-in: its device address is obtained
// once per device with hipGetSymbolAddress and every launch passes that
// address.  Every call on a device shares that device's array.

constexpr size_t kScratchBytes = 4718592;  // 4.5 MiB: N up to 2^20 at (L, L_s) = (32, 8) or (64, 16)
constexpr int64_t kStaticMaxN = int64_t(1) << 20;
__device__ __align__(256) unsigned char scratch[kScratchBytes];

static int64_t round256(int64_t v) { return (v + 255) & ~(int64_t)255; }

// Byte layout of the workspace of one frame with K leaves, rank LS.
struct StaticLayout {
  int64_t leaf2f, cblk, uh, vh, tr, tc, end;
  StaticLayout(int64_t K, int64_t LS) {
    const int64_t ncb = std::max<int64_t>(K - 1, 1);
    leaf2f = round256((int64_t)sizeof(FrameDesc));
    cblk = leaf2f + round256(4 * K);
    uh = cblk + round256(8 * ncb);
    vh = uh + round256(4 * K * LS);
    tr = vh + round256(4 * K * LS);
    tc = tr + round256(4 * K * LS);
    end = tc + round256(4 * K * LS);
  }
};

// The frame table of a one-frame batch: frame 0 at row 0, every leaf in
// frame 0, one coarse block per tile (a placeholder when there is none).
__global__ void k_single_frame_tables(FrameDesc F, FrameDesc* fr, int* leaf2f, int2* cblk) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i == 0) fr[0] = F;
  if (i < F.K) leaf2f[i] = 0;
  if (i < max(F.MH, 1)) cblk[i] = F.MH > 0 ? make_int2(0, i) : make_int2(0, -1);
}

static std::mutex g_scratch_mu;
static void* g_scratch_dev[256];  // device address of `scratch`, per device ordinal

// Device address of `scratch` on the current device (looked up on the first
// call on each device, with that device current).
static hp_status scratch_address(char** out) {
  int dev = -1;
  HP_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= 256) return set_error(HP_E_HIP, "hp_apply_static: device ordinal %d out of range", dev);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return set_error(HP_E_HIP, "hp_apply_static: hipGetSymbolAddress(scratch) on device %d failed: %s", dev,
                       hipGetErrorString(e));
    g_scratch_dev[dev] = p;
  }
  *out = (char*)g_scratch_dev[dev];
  return HP_OK;
}

}  // namespace hp

extern "C" hp_status hp_apply_static(int32_t nx, int32_t ny, int32_t nz, int32_t leaf, int32_t rank,
                                     const float* d_sys, const void* d_factors, int32_t fdtype, const float* d_r,
                                     float* d_y, int32_t ncols, void* hip_stream) {
  using namespace hp;
  if (!d_sys || !d_factors || !d_r || !d_y) return set_error(HP_E_INVALID, "hp_apply_static: NULL argument");
  if (ncols < 1) return set_error(HP_E_INVALID, "hp_apply_static: ncols must be >= 1");
  if (fdtype != HP_F32 && fdtype != HP_BF16) return set_error(HP_E_INVALID, "hp_apply_static: bad fdtype");
  if ((uintptr_t)d_factors & 15) return set_error(HP_E_INVALID, "hp_apply_static: factors must be 16-byte aligned");
  if (!((leaf == 64 && rank == 16) || (leaf == 32 && rank == 8)))
    return set_error(HP_E_SHAPE, "hp_apply_static: supported (leaf, rank): (64, 16), (32, 8)");
  if (nx <= 0 || ny <= 0 || nz <= 0 || !admissible_grid(nx, ny, nz, nullptr))
    return set_error(HP_E_SHAPE, "hp_apply_static: grid %d x %d x %d is not admissible", nx, ny, nz);
  const int64_t n = (int64_t)nx * ny * nz;
  if (n > kStaticMaxN)
    return set_error(HP_E_SHAPE, "hp_apply_static: N = %lld exceeds the static workspace's maximum %lld",
                     (long long)n, (long long)kStaticMaxN);
  hp_partition_info pi;
  HP_TRY(hp_build_partition((int32_t)n, leaf, rank, &pi, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr));
  const StaticLayout lay(pi.K, rank);
  if (lay.end > (int64_t)kScratchBytes)
    return set_error(HP_E_SHAPE, "hp_apply_static: workspace of %lld bytes exceeds the static %zu",
                     (long long)lay.end, kScratchBytes);
  const uintptr_t r0 = (uintptr_t)d_r, y0 = (uintptr_t)d_y, len = (uintptr_t)(4 * n * (int64_t)ncols);
  if (r0 < y0 + len && y0 < r0 + len) return set_error(HP_E_INVALID, "hp_apply_static: r and y must not overlap");
  char* ws = nullptr;
  HP_TRY(scratch_address(&ws));

  FrameDesc F{};
  F.n = (int)n;
  F.K = pi.K;
  F.MH = pi.MH;
  F.J = pi.J;
  F.nz = nz;
  F.nx = nx;
  F.ny = ny;
  morton_masks(nx, ny, nz, &F.xm, &F.ym, &F.zm);
  F.nb = (int)((n + NODE_BLOCK - 1) / NODE_BLOCK);
  LaunchGeom g{};
  g.fr = (const FrameDesc*)ws;
  g.blk2f = nullptr;  // the apply kernels index leaves and tiles only
  g.leaf2f = (const int*)(ws + lay.leaf2f);
  g.cblk = (const int2*)(ws + lay.cblk);
  g.nframes = 1;
  g.nblk = F.nb;
  g.ncblk = std::max(pi.MH, 1);
  g.ktot = pi.K;
  g.ntot = n;
  g.kmax = pi.K;
  g.stream = (hipStream_t)hip_stream;
  hipLaunchKernelGGL(k_single_frame_tables, dim3((pi.K + 255) / 256), dim3(256), 0, g.stream, F, (FrameDesc*)ws,
                     (int*)(ws + lay.leaf2f), (int2*)(ws + lay.cblk));
  HP_HIP(hipGetLastError());
  int64_t offs[5], tot;
  factor_offsets_n(pi.K, pi.MH, n, leaf, rank, fdtype, offs, &tot);
  float* uh = (float*)(ws + lay.uh);
  float* vh = (float*)(ws + lay.vh);
  float* tr = (float*)(ws + lay.tr);
  float* tc = (float*)(ws + lay.tc);
  for (int32_t c = 0; c < ncols; ++c)
    HP_TRY(launch_apply(g, leaf, rank, fdtype, d_sys, d_factors, offs, d_r + c * n, d_y + c * n, uh, vh, tr, tc));
  return HP_OK;
}

namespace hp {



template <int L, int LS, typename FT>
static Factors<FT> make_factors(const PcgLaunch& P) {
  const char* base = (const char*)P.fbase;
  return Factors<FT>{(const FT*)(base + P.offs[0]), (const FT*)(base + P.offs[1]), (const FT*)(base + P.offs[2]),
                     (const FT*)(base + P.offs[3]), (const float*)(base + P.offs[4])};
}

template <int L, int LS, typename FT>
static void hmat_setup(const PcgLaunch& P) {
  auto fac = make_factors<L, LS, FT>(P);
  const LaunchGeom& g = P.g;
  hipLaunchKernelGGL((k_setup_hmat<L, LS, FT>), dim3(g.ktot), dim3(LEAF_THREADS), 0, g.stream, g.fr, g.leaf2f, P.B,
                     fac);
  hipLaunchKernelGGL((k_coarse_check<LS, FT>), dim3(g.ncblk), dim3(LEAF_THREADS), 0, g.stream, g.fr, g.cblk, P.B,
                     fac, 1);
  hipLaunchKernelGGL((k_prolong<L, LS, FT>), dim3(g.ktot), dim3(LEAF_THREADS), 0, g.stream, g.fr, g.leaf2f, P.B, fac);
}

template <int L, int LS, typename FT>
static void hmat_iter(const PcgLaunch& P, int par) {
  auto fac = make_factors<L, LS, FT>(P);
  const LaunchGeom& g = P.g;
  const float* pold = par ? P.B.p1 : P.B.p0;
  float* pnew = par ? P.B.p0 : P.B.p1;
  const double* xold = par ? P.B.x1 : P.B.x0;
  double* xnew = par ? P.B.x0 : P.B.x1;
  // live timing (eager only): algorithmic bytes of an iteration without
  // residual replacement, every frame active
  auto timed = [&](int kind) {
    Prof* pr = P.prof;
    if (!pr || pr->kind != kind || 2 * (pr->used + 1) > (int)pr->ev.size()) return false;
    hipEventRecord(pr->ev[2 * pr->used], g.stream);
    return true;
  };
  auto done = [&](double bytes) {
    Prof* pr = P.prof;
    hipEventRecord(pr->ev[2 * pr->used + 1], g.stream);
    pr->used++;
    pr->work += bytes;
  };
  bool t = timed(PROF_SPMV);
  hipLaunchKernelGGL(k_spmv_p<false>, dim3(g.nblk), dim3(NODE_BLOCK), 0, g.stream, g.fr, g.blk2f, P.B, 0, 1, pold,
                     pnew);
  if (t) done(32.0 * (double)g.ntot);  // z, p_old, 4 coefficients in; p, q out
  t = timed(PROF_UPDATE);
  hipLaunchKernelGGL((k_update_hmat<L, LS, FT>), dim3(g.ktot), dim3(LEAF_THREADS), 0, g.stream, g.fr, g.leaf2f, P.B,
                     fac, xold, xnew, (const float*)pnew);
  // per node p, q, r, x, lam, 1/diag in, x, r, z out (44 B); per leaf G, Ut, Vt in, u, v out
  if (t) done((double)g.ktot * (44.0 * L + (double)sizeof(FT) * (L * L + 2 * L * LS) + 8.0 * LS));
  hipLaunchKernelGGL((k_coarse_check<LS, FT>), dim3(g.ncblk), dim3(LEAF_THREADS), 0, g.stream, g.fr, g.cblk, P.B,
                     fac, 0);
  hipLaunchKernelGGL((k_prolong<L, LS, FT>), dim3(g.ktot), dim3(LEAF_THREADS), 0, g.stream, g.fr, g.leaf2f, P.B, fac);
}

__global__ void k_pcg_init(FrameState* st, int nframes, int* n_active, SolveParams* prm, SolveParams p) {
  const int f = blockIdx.x * blockDim.x + threadIdx.x;
  if (f < nframes) {
    FrameState s;
    s.rho = 1.0;
    s.alpha = s.beta = s.rr = s.target = s.bnorm = s.rwin = 0.0;
    s.it = s.flags = s.done = s.force_rc = s.fresh = 0;
    s.active = 1;
    store_state(st + 2 * f, s);
    store_state(st + 2 * f + 1, s);
  }
  if (f == 0) {
    *n_active = nframes;
    prm->tol = p.tol;
    prm->max_iter = p.max_iter;
    prm->recompute_every = p.recompute_every;
    prm->stagnation = p.stagnation;
    prm->pad = 0;
  }
}

hp_status pcg_init_states(FrameState* st, int nframes, int* n_active, SolveParams* prm, const SolveParams& p,
                          hipStream_t s) {
  hipLaunchKernelGGL(k_pcg_init, dim3((unsigned)((nframes + 63) / 64)), dim3(64), 0, s, st, nframes, n_active, prm, p);
  HP_HIP(hipGetLastError());
  return HP_OK;
}

hp_status pcg_setup(const PcgLaunch& P) {
  const LaunchGeom& g = P.g;
  if (P.mode == HP_PRECOND_HMAT) {
    if (P.L == 64 && P.LS == 16) {
      if (P.fdtype == HP_BF16) hmat_setup<64, 16, uint16_t>(P);
      else hmat_setup<64, 16, float>(P);
    } else if (P.L == 32 && P.LS == 8) {
      if (P.fdtype == HP_BF16) hmat_setup<32, 8, uint16_t>(P);
      else hmat_setup<32, 8, float>(P);
    } else {
      return set_error(HP_E_SHAPE, "pcg: unsupported (L, L_s) = (%d, %d)", P.L, P.LS);
    }
  } else {
    if (P.mode == HP_PRECOND_JACOBI)
      hipLaunchKernelGGL(k_setup_simple<true>, dim3(g.nblk), dim3(NODE_BLOCK), 0, g.stream, g.fr, g.blk2f, P.B);
    else
      hipLaunchKernelGGL(k_setup_simple<false>, dim3(g.nblk), dim3(NODE_BLOCK), 0, g.stream, g.fr, g.blk2f, P.B);
    hipLaunchKernelGGL(k_frame_setup, dim3(g.nframes), dim3(LEAF_THREADS), 0, g.stream, g.fr, P.B);
  }
  HP_HIP(hipGetLastError());
  return HP_OK;
}

// Enqueue `count` iterations (count even), the first at parity 0.
hp_status pcg_iterations(const PcgLaunch& P, int count) {
  const LaunchGeom& g = P.g;
  for (int it = 0; it < count; ++it) {
    int par = it & 1;
    if (P.mode == HP_PRECOND_HMAT) {
      if (P.L == 64 && P.LS == 16) {
        if (P.fdtype == HP_BF16) hmat_iter<64, 16, uint16_t>(P, par);
        else hmat_iter<64, 16, float>(P, par);
      } else if (P.L == 32 && P.LS == 8) {
        if (P.fdtype == HP_BF16) hmat_iter<32, 8, uint16_t>(P, par);
        else hmat_iter<32, 8, float>(P, par);
      } else {
        return set_error(HP_E_SHAPE, "pcg: unsupported (L, L_s) = (%d, %d)", P.L, P.LS);
      }
    } else {
      const float* pold = par ? P.B.p1 : P.B.p0;
      float* pnew = par ? P.B.p0 : P.B.p1;
      const double* xold = par ? P.B.x1 : P.B.x0;
      double* xnew = par ? P.B.x0 : P.B.x1;
      hipLaunchKernelGGL(k_spmv_p<true>, dim3(g.nblk), dim3(NODE_BLOCK), 0, g.stream, g.fr, g.blk2f, P.B, par,
                         par ^ 1, pold, pnew);
      if (P.mode == HP_PRECOND_JACOBI)
        hipLaunchKernelGGL(k_update_simple<true>, dim3(g.nblk), dim3(NODE_BLOCK), 0, g.stream, g.fr, g.blk2f, P.B,
                           par, xold, xnew, (const float*)pnew);
      else
        hipLaunchKernelGGL(k_update_simple<false>, dim3(g.nblk), dim3(NODE_BLOCK), 0, g.stream, g.fr, g.blk2f, P.B,
                           par, xold, xnew, (const float*)pnew);
    }
  }
  HP_HIP(hipGetLastError());
  return HP_OK;
}

hp_status pcg_finalize(const PcgLaunch& P, bool stopped_only) {
  const LaunchGeom& g = P.g;
  hipLaunchKernelGGL(k_finalize_x, dim3(g.nblk), dim3(NODE_BLOCK), 0, g.stream, g.fr, g.blk2f,
                     (const FrameState*)P.B.st, (const double*)P.B.x1, P.B.x0, (int)stopped_only);
  HP_HIP(hipGetLastError());
  return HP_OK;
}

}  // namespace hp
