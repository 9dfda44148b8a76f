// Assembly, 7-point SpMV, the H-matrix apply and the fused PCG pipeline.
//
// PCG (paper Sec. 3 and Sec. 5; Saad 2003 Alg. 9.1) runs as three kernels per
// iteration for the learned preconditioner and two for Jacobi / identity:
//
//   k_spmv_p      node blocks: p = z + beta p_old (on the fly at the 7 stencil
//                 points, p ping-pongs), q = A p, FP64 partials of p.q; the last
//                 block of a frame reduces them in a fixed order -> alpha.
//   k_update_hmat leaf blocks: x += alpha p (x ping-pongs), r -= alpha q or the
//                 FP64 residual replacement r = b - A x, the leaf stage of M
//                 (G_k r_k + lam r / A_ii, restriction Ut^T r, Vt^T r), FP64
//                 partials of ||r||^2; the last block of a frame takes the
//                 stop decisions and runs the frame's coarse stage (strip sums,
//                 B / B^T coupling, accumulation down the levels).
//   k_prolong     leaf blocks: z += Ut T^r + Vt T^c, FP64 partials of r.z; the
//                 last block -> positivity check, beta = rho'/rho.
//
// Per-frame scalars live in FrameState and are written only by the last
// block to arrive (atomic ticket per frame and kernel), so every reduction
// has a fixed order and the solve is bit-reproducible.  Frames that stopped
// are skipped by every kernel, which makes a fixed chunk of iterations safe
// to replay from a hipGraph.
#include <float.h>
#include <math.h>

#include "batch.h"

namespace hp {

// ------------------------------------------------------------------ helpers

__device__ inline double warp_sum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
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

// Ticket: returns true in every thread of the last block (of `count`) to
// arrive for this counter; resets the counter for the next use.
__device__ inline bool last_arrival(unsigned* ticket, unsigned count) {
  __shared__ int is_last;
  __syncthreads();
  if (threadIdx.x == 0) {
    __threadfence();
    unsigned t = atomicAdd(ticket, 1u);
    is_last = (t == count - 1);
    if (is_last) {
      *ticket = 0;
      __threadfence();
    }
  }
  __syncthreads();
  return is_last != 0;
}

__device__ inline double vload(const double* p) { return *(const volatile double*)p; }

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

// (A v)_i in FP32 with v read through a functor (7-point stencil, Morton).
template <typename V>
__device__ inline float stencil_f32(const SysPtr& s, const FrameDesc& F, unsigned c, V v) {
  int64_t i = F.n0 + c;
  int64_t xp = F.n0 + mstep_plus(c, F.xm), xn = F.n0 + mstep_minus(c, F.xm);
  int64_t yp = F.n0 + mstep_plus(c, F.ym), yn = F.n0 + mstep_minus(c, F.ym);
  int64_t zp = F.n0 + mstep_plus(c, F.zm), zn = F.n0 + mstep_minus(c, F.zm);
  float a = s.dg[i] * v(i);
  a = fmaf(-s.wx[i], v(xp), a);
  a = fmaf(-s.wx[xn], v(xn), a);
  a = fmaf(-s.wy[i], v(yp), a);
  a = fmaf(-s.wy[yn], v(yn), a);
  a = fmaf(-s.wz[i], v(zp), a);
  a = fmaf(-s.wz[zn], v(zn), a);
  return a;
}

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

__global__ void k_assemble(const FrameDesc* fr, const int* blk2f, const float* rho, float* sys, int64_t ntot) {
  const FrameDesc F = fr[blk2f[blockIdx.x]];
  int c = (blockIdx.x - F.b0) * NODE_BLOCK + threadIdx.x;
  if (c >= F.n) return;
  int64_t i = F.n0 + c;
  double ri = rho[i];
  auto wplus = [&](unsigned m) -> double {
    if ((c & m) == m) return 0.0;
    return 2.0 / (ri + (double)rho[F.n0 + mstep_plus(c, m)]);
  };
  auto wminus = [&](unsigned m) -> double {
    if ((c & m) == 0) return 0.0;
    return 2.0 / (ri + (double)rho[F.n0 + mstep_minus(c, m)]);
  };
  double wpx = wplus(F.xm), wpy = wplus(F.ym), wpz = wplus(F.zm);
  double d = wpx + wminus(F.xm) + wpy + wminus(F.ym) + wpz + wminus(F.zm);
  if ((c & F.zm) == F.zm) d += 1.0 / ri;
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

__global__ void k_spmv(const FrameDesc* fr, const int* blk2f, const float* sys, int64_t ntot,
                       const float* p, float* q) {
  const FrameDesc F = fr[blk2f[blockIdx.x]];
  int c = (blockIdx.x - F.b0) * NODE_BLOCK + threadIdx.x;
  if (c >= F.n) return;
  SysPtr s(sys, ntot);
  q[F.n0 + c] = stencil_f32(s, F, c, [&](int64_t j) { return p[j]; });
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
  if constexpr (sizeof(FT) == 2) {
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
// rs: r_k in LDS (L floats).  Returns nothing; all threads take part.
template <int L, int LS, typename FT>
__device__ inline void leaf_stage(int64_t kg, int64_t row0, const float* rs, const Factors<FT>& fac,
                                  const float* idg, float* y, float* uh, float* vh, float* red) {
  constexpr int TPR = LEAF_THREADS / L;  // threads per row
  constexpr int CPT = L / TPR;           // columns per thread
  const int t = threadIdx.x;
  {
    int row = t / TPR, c0 = (t % TPR) * CPT;
    float g[CPT];
    load_vec<FT, CPT>(fac.G + (kg * L + row) * L + c0, g);
    float a = 0.f;
#pragma unroll
    for (int c = 0; c < CPT; ++c) a = fmaf(g[c], rs[c0 + c], a);
#pragma unroll
    for (int o = TPR / 2; o > 0; o >>= 1) a += __shfl_xor(a, o, 64);
    if (t % TPR == 0) {
      int64_t i = row0 + row;
      y[i] = fmaf(fac.lam[i] * idg[i], rs[row], a);
    }
  }
  // restriction: thread -> (s, row group)
  {
    constexpr int G = LEAF_THREADS / LS;     // row groups
    constexpr int RPG = L / G;               // rows per group
    static_assert(RPG >= 1, "leaf too small for the restriction layout");
    int s = t % LS, g = t / LS;
    float au = 0.f, av = 0.f;
#pragma unroll
    for (int j = 0; j < RPG; ++j) {
      int l = g * RPG + j;
      float rl = rs[l];
      au = fmaf(ldf(fac.Ut, (row0 + l) * LS + s), rl, au);
      av = fmaf(ldf(fac.Vt, (row0 + l) * LS + s), rl, av);
    }
    // reduce the groups held inside one wave (lanes s + LS*q)
#pragma unroll
    for (int o = 32; o >= LS; o >>= 1) {
      au += __shfl_xor(au, o, 64);
      av += __shfl_xor(av, o, 64);
    }
    int w = t >> 6;
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
}

// Prolongation for leaf kg: y[rows] += Ut_k T^r + Vt_k T^c.  Returns the
// updated value of row (t / TPR) in the lane with t % TPR == 0, else 0; the
// caller passes the row's current y value in yrow (lane t % TPR == 0).
template <int L, int LS, typename FT>
__device__ inline float prolong_row(int64_t row0, const float* trs, const float* tcs, const Factors<FT>& fac,
                                    float yrow) {
  constexpr int TPR = LEAF_THREADS / L;
  constexpr int SPT = LS / TPR;  // coarse entries per thread
  const int t = threadIdx.x;
  int row = t / TPR, s0 = (t % TPR) * SPT;
  float a = 0.f;
  if constexpr (SPT >= 4) {
    float u[SPT], v[SPT];
    load_vec<FT, SPT>(fac.Ut + (row0 + row) * LS + s0, u);
    load_vec<FT, SPT>(fac.Vt + (row0 + row) * LS + s0, v);
#pragma unroll
    for (int s = 0; s < SPT; ++s) a = fmaf(u[s], trs[s0 + s], fmaf(v[s], tcs[s0 + s], a));
  } else {
#pragma unroll
    for (int s = 0; s < SPT; ++s) {
      a = fmaf(ldf(fac.Ut, (row0 + row) * LS + s0 + s), trs[s0 + s], a);
      a = fmaf(ldf(fac.Vt, (row0 + row) * LS + s0 + s), tcs[s0 + s], a);
    }
  }
#pragma unroll
  for (int o = TPR / 2; o > 0; o >>= 1) a += __shfl_xor(a, o, 64);
  return yrow + a;
}

// Coarse stage of one frame, run by one whole block (paper Sec. 5 strip
// aggregation and coarse coupling): level sums of u and v up the dyadic
// tree; per tile m = (j, i): t^r = B_m s^c with s^c the level-j sum of the
// column strip, t^c = B_m^T s^r with s^r the row-strip sum; leaf k adds t^r
// of the tile where it is on the row side and t^c where it is on the column
// side, at every level.  lds holds 2.5 K LS floats.
template <int LS, typename FT>
__device__ void coarse_stage(const FrameDesc& F, const float* uh, const float* vh, const FT* B, float* Tr,
                             float* Tc, float* lds) {
  const int K = F.K, J = F.J, nt = blockDim.x, t = threadIdx.x;
  const int64_t kb = (int64_t)F.k0 * LS;
  for (int e = t; e < K * LS; e += nt) {
    Tr[kb + e] = 0.f;
    Tc[kb + e] = 0.f;
  }
  if (J == 0) return;
  float* Pu = lds;
  float* Pv = Pu + (K / 2) * LS;
  float* Qu = Pv + (K / 2) * LS;
  float* Qv = Qu + (K / 4) * LS;
  float* tb = Qv + (K / 4) * LS;  // [0, K/2 LS): t^r, [K/2 LS, K LS): t^c
  const float* su = uh + kb;
  const float* sv = vh + kb;
  const FT* Bf = B + (int64_t)F.m0 * LS * LS;
  for (int j = 0; j < J; ++j) {
    const int nj = K >> (j + 1);
    const int mb = K - (K >> j);
    for (int o = t; o < 2 * nj * LS; o += nt) {
      int which = o / (nj * LS), rem = o % (nj * LS), i = rem / LS, s = rem % LS;
      const FT* Bm = Bf + (int64_t)(mb + i) * LS * LS;
      float a = 0.f;
      if (which == 0) {
        const float* sc = sv + (2 * i + 1) * LS;
#pragma unroll
        for (int u = 0; u < LS; ++u) a = fmaf(ldf(Bm, s * LS + u), sc[u], a);
        tb[i * LS + s] = a;
      } else {
        const float* sr = su + (2 * i) * LS;
#pragma unroll
        for (int u = 0; u < LS; ++u) a = fmaf(ldf(Bm, u * LS + s), sr[u], a);
        tb[(K / 2) * LS + i * LS + s] = a;
      }
    }
    __syncthreads();
    for (int e = t; e < K * LS; e += nt) {
      int k = e / LS, s = e % LS, i = k >> (j + 1);
      if (((k >> j) & 1) == 0) Tr[kb + e] += tb[i * LS + s];
      else Tc[kb + e] += tb[(K / 2) * LS + i * LS + s];
    }
    if (j + 1 < J) {
      float* du = (j % 2 == 0) ? Pu : Qu;
      float* dv = (j % 2 == 0) ? Pv : Qv;
      for (int e = t; e < nj * LS; e += nt) {
        int bb = e / LS, s = e % LS;
        du[e] = su[(2 * bb) * LS + s] + su[(2 * bb + 1) * LS + s];
        dv[e] = sv[(2 * bb) * LS + s] + sv[(2 * bb + 1) * LS + s];
      }
      su = du;
      sv = dv;
    }
    __syncthreads();
  }
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
  for (int l = threadIdx.x; l < L; l += blockDim.x) rs[l] = r[row0 + l];
  __syncthreads();
  leaf_stage<L, LS, FT>(kg, row0, rs, fac, sys + 4 * ntot, y, uh, vh, red);
}

template <int LS, typename FT>
__global__ __launch_bounds__(LEAF_THREADS) void k_apply_coarse(const FrameDesc* fr, Factors<FT> fac,
                                                               const float* uh, const float* vh, float* Tr,
                                                               float* Tc) {
  extern __shared__ float lds[];
  const FrameDesc F = fr[blockIdx.x];
  coarse_stage<LS, FT>(F, uh, vh, fac.B, Tr, Tc, lds);
}

template <int L, int LS, typename FT>
__global__ __launch_bounds__(LEAF_THREADS) void k_apply_prolong(const FrameDesc* fr, const int* leaf2f,
                                                                Factors<FT> fac, const float* Tr,
                                                                const float* Tc, float* y) {
  __shared__ float trs[LS], tcs[LS];
  const int64_t kg = blockIdx.x;
  const FrameDesc F = fr[leaf2f[kg]];
  const int64_t row0 = F.n0 + (kg - F.k0) * L;
  if (threadIdx.x < LS) {
    trs[threadIdx.x] = Tr[kg * LS + threadIdx.x];
    tcs[threadIdx.x] = Tc[kg * LS + threadIdx.x];
  }
  __syncthreads();
  constexpr int TPR = LEAF_THREADS / L;
  int row = threadIdx.x / TPR;
  float yr = (threadIdx.x % TPR == 0) ? y[row0 + row] : 0.f;
  float v = prolong_row<L, LS, FT>(row0, trs, tcs, fac, yr);
  if (threadIdx.x % TPR == 0) y[row0 + row] = v;
}

// ------------------------------------------------------------------ PCG kernels



enum { TK_SPMV = 0, TK_UPD = 1, TK_PRO = 2, TK_SETUP = 3 };

// Stop decisions after the x / r update of iteration k (rr = ||r||^2).
// Called by one thread; returns true when the frame stops.
// A residual that passes the tolerance stops the frame only when it is a
// true (replaced) residual; a recurrence residual that passes forces a
// replacement on the next iteration instead.
__device__ inline bool stop_checks(FrameState& s, const SolveParams& prm, int k, double rr, bool replaced) {
  s.k = k;
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
  if (prm.stagnation && k % 100 == 0) {
    if (rn > 0.5 * s.rwin) {
      s.flags |= HP_STAGNATED;
      return true;
    }
    s.rwin = rn;
  }
  if (k >= prm.max_iter) {
    s.flags |= HP_MAXITER;
    return true;
  }
  return false;
}

__device__ inline void finish_frame(FrameState& s, int* n_active) {
  s.done = 1;
  atomicSub(n_active, 1);
}

// p = z + beta p_old; q = A p; partial p.q -> alpha in the last block.
__global__ __launch_bounds__(NODE_BLOCK) void k_spmv_p(const FrameDesc* fr, const int* blk2f, PcgBufs B_,
                                                       const float* pold, float* pnew) {
  __shared__ double red[NODE_BLOCK / 64];
  const int f = blk2f[blockIdx.x];
  const FrameDesc F = fr[f];
  FrameState* st = B_.st + f;
  if (st->done) return;
  const float beta = (float)st->beta;
  const float* z = B_.z;
  SysPtr s(B_.sys, B_.ntot);
  int c = (blockIdx.x - F.b0) * NODE_BLOCK + threadIdx.x;
  double pq = 0.0;
  if (c < F.n) {
    auto P = [&](int64_t j) { return fmaf(beta, pold[j], z[j]); };
    float qi = stencil_f32(s, F, c, P);
    float pi = P(F.n0 + c);
    pnew[F.n0 + c] = pi;
    B_.q[F.n0 + c] = qi;
    pq = (double)pi * (double)qi;
  }
  double bs = block_sum(pq, red);
  if (threadIdx.x == 0) B_.part_pq[blockIdx.x] = bs;
  if (last_arrival(B_.ticket + 4 * f + TK_SPMV, F.nb)) {
    if (threadIdx.x == 0) {
      double tot = 0.0;
      for (int j = 0; j < F.nb; ++j) tot += vload(B_.part_pq + F.b0 + j);
      st->alpha = st->rho / tot;
    }
  }
}

// Shared per-leaf x / r update.  Writes x_new, r; fills rs (LDS); returns the
// thread's share of ||r||^2.
// x accumulates in FP64 (x += alpha p with alpha in FP64); r, p, q are FP32.
template <int L>
__device__ inline double xr_update(const FrameDesc& F, int64_t row0, const PcgBufs& B_, const double* xold,
                                   double* xnew, const float* p, double alpha, bool recompute, float* rs) {
  SysPtr s(B_.sys, B_.ntot);
  const float af = (float)alpha;
  double rr = 0.0;
  for (int l = threadIdx.x; l < L; l += blockDim.x) {
    int64_t i = row0 + l;
    xnew[i] = fma(alpha, (double)p[i], xold[i]);
    float ri;
    if (recompute) {
      unsigned c = (unsigned)(i - F.n0);
      ri = (float)resid_f64(s, F, c, (double)B_.b[i], [&](int64_t j) { return fma(alpha, (double)p[j], xold[j]); });
    } else {
      ri = fmaf(-af, B_.q[i], B_.r[i]);
    }
    B_.r[i] = ri;
    rs[l] = ri;
    rr += (double)ri * (double)ri;
  }
  return rr;
}

template <int L, int LS, typename FT>
__global__ __launch_bounds__(LEAF_THREADS) void k_update_hmat(const FrameDesc* fr, const int* leaf2f, PcgBufs B_,
                                                              Factors<FT> fac, const double* xold, double* xnew,
                                                              const float* p) {
  extern __shared__ float lds[];
  __shared__ float rs[L];
  __shared__ float red[(LEAF_THREADS / 64) * 2 * LS];
  __shared__ double dred[LEAF_THREADS / 64];
  __shared__ int stop;
  const int64_t kg = blockIdx.x;
  const int f = leaf2f[kg];
  const FrameDesc F = fr[f];
  FrameState* st = B_.st + f;
  if (st->done) return;
  const SolveParams prm = *B_.prm;
  const int64_t row0 = F.n0 + (kg - F.k0) * L;
  const double alpha = st->alpha;
  const int knext = st->k + 1;
  const bool recompute = st->force_rc || (prm.recompute_every > 0 && knext % prm.recompute_every == 0);
  double rr = xr_update<L>(F, row0, B_, xold, xnew, p, alpha, recompute, rs);
  __syncthreads();
  leaf_stage<L, LS, FT>(kg, row0, rs, fac, B_.sys + 4 * B_.ntot, B_.z, B_.uh, B_.vh, red);
  double bs = block_sum(rr, dred);
  if (threadIdx.x == 0) B_.part_rr[kg] = bs;
  if (last_arrival(B_.ticket + 4 * f + TK_UPD, F.K)) {
    if (threadIdx.x == 0) {
      double tot = 0.0;
      for (int j = 0; j < F.K; ++j) tot += vload(B_.part_rr + F.k0 + j);
      stop = stop_checks(*st, prm, knext, tot, recompute);
      if (stop) finish_frame(*st, B_.n_active);
    }
    __syncthreads();
    if (!stop) {
      __threadfence();
      coarse_stage<LS, FT>(F, B_.uh, B_.vh, fac.B, B_.Tr, B_.Tc, lds);
    }
  }
}

// z += Ut T^r + Vt T^c; partial r.z -> positivity, beta in the last block.
template <int L, int LS, typename FT>
__global__ __launch_bounds__(LEAF_THREADS) void k_prolong(const FrameDesc* fr, const int* leaf2f, PcgBufs B_,
                                                          Factors<FT> fac, int setup) {
  __shared__ float trs[LS], tcs[LS];
  __shared__ double dred[LEAF_THREADS / 64];
  const int64_t kg = blockIdx.x;
  const int f = leaf2f[kg];
  const FrameDesc F = fr[f];
  FrameState* st = B_.st + f;
  if (st->done) return;
  const int64_t row0 = F.n0 + (kg - F.k0) * L;
  if (threadIdx.x < LS) {
    trs[threadIdx.x] = B_.Tr[kg * LS + threadIdx.x];
    tcs[threadIdx.x] = B_.Tc[kg * LS + threadIdx.x];
  }
  __syncthreads();
  constexpr int TPR = LEAF_THREADS / L;
  const int row = threadIdx.x / TPR;
  const bool lead = threadIdx.x % TPR == 0;
  float zr = lead ? B_.z[row0 + row] : 0.f;
  zr = prolong_row<L, LS, FT>(row0, trs, tcs, fac, zr);
  double rz = 0.0;
  if (lead) {
    B_.z[row0 + row] = zr;
    rz = (double)B_.r[row0 + row] * (double)zr;
  }
  double bs = block_sum(rz, dred);
  if (threadIdx.x == 0) B_.part_rz[kg] = bs;
  if (last_arrival(B_.ticket + 4 * f + TK_PRO, F.K)) {
    if (threadIdx.x == 0) {
      double tot = 0.0;
      for (int j = 0; j < F.K; ++j) tot += vload(B_.part_rz + F.k0 + j);
      if (!(tot > 0.0) || !isfinite(tot)) {
        st->flags |= HP_NOT_SPD;
        finish_frame(*st, B_.n_active);
      } else {
        st->beta = setup ? 0.0 : tot / st->rho;
        st->rho = tot;
      }
    }
  }
}

// Setup for the learned preconditioner: r = b - A x0 (FP64), ||b||, ||r||,
// the leaf stage of z = M r and, in the last block, the coarse stage.  p0 = 0.
template <int L, int LS, typename FT>
__global__ __launch_bounds__(LEAF_THREADS) void k_setup_hmat(const FrameDesc* fr, const int* leaf2f, PcgBufs B_,
                                                             Factors<FT> fac) {
  extern __shared__ float lds[];
  __shared__ float rs[L];
  __shared__ float red[(LEAF_THREADS / 64) * 2 * LS];
  __shared__ double dred[LEAF_THREADS / 64];
  __shared__ int stop;
  const int64_t kg = blockIdx.x;
  const int f = leaf2f[kg];
  const FrameDesc F = fr[f];
  FrameState* st = B_.st + f;
  if (st->done) return;
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
    B_.part_rz[kg] = bsum;
  }
  if (last_arrival(B_.ticket + 4 * f + TK_SETUP, F.K)) {
    if (threadIdx.x == 0) {
      double rt = 0.0, bt = 0.0;
      for (int j = 0; j < F.K; ++j) {
        rt += vload(B_.part_rr + F.k0 + j);
        bt += vload(B_.part_rz + F.k0 + j);
      }
      const SolveParams prm = *B_.prm;
      st->bnorm = sqrt(bt);
      st->target = (prm.tol * st->bnorm) * (prm.tol * st->bnorm);
      st->rr = rt;
      st->rwin = sqrt(rt);
      st->k = 0;
      stop = rt <= st->target;
      if (stop) {
        st->flags |= HP_CONVERGED;
        finish_frame(*st, B_.n_active);
      }
    }
    __syncthreads();
    if (!stop) {
      __threadfence();
      coarse_stage<LS, FT>(F, B_.uh, B_.vh, fac.B, B_.Tr, B_.Tc, lds);
    }
  }
}

// Jacobi / identity: setup over node blocks.
template <bool JAC>
__global__ __launch_bounds__(NODE_BLOCK) void k_setup_simple(const FrameDesc* fr, const int* blk2f, PcgBufs B_) {
  __shared__ double red[NODE_BLOCK / 64];
  const int f = blk2f[blockIdx.x];
  const FrameDesc F = fr[f];
  FrameState* st = B_.st + f;
  if (st->done) return;
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
  if (last_arrival(B_.ticket + 4 * f + TK_SETUP, F.nb)) {
    if (threadIdx.x == 0) {
      double rt = 0.0, bt = 0.0, zt = 0.0;
      for (int j = 0; j < F.nb; ++j) {
        rt += vload(B_.part_rr + F.b0 + j);
        zt += vload(B_.part_rz + F.b0 + j);
        bt += vload(B_.part_pq + F.b0 + j);
      }
      const SolveParams prm = *B_.prm;
      st->bnorm = sqrt(bt);
      st->target = (prm.tol * st->bnorm) * (prm.tol * st->bnorm);
      st->rr = rt;
      st->rwin = sqrt(rt);
      st->k = 0;
      if (rt <= st->target) {
        st->flags |= HP_CONVERGED;
        finish_frame(*st, B_.n_active);
      } else if (!(zt > 0.0) || !isfinite(zt)) {
        st->flags |= HP_NOT_SPD;
        finish_frame(*st, B_.n_active);
      } else {
        st->rho = zt;
        st->beta = 0.0;
      }
    }
  }
}

// Jacobi / identity iteration update over node blocks: x, r, z, ||r||^2, r.z.
template <bool JAC>
__global__ __launch_bounds__(NODE_BLOCK) void k_update_simple(const FrameDesc* fr, const int* blk2f, PcgBufs B_,
                                                              const double* xold, double* xnew, const float* p) {
  __shared__ double red[NODE_BLOCK / 64];
  const int f = blk2f[blockIdx.x];
  const FrameDesc F = fr[f];
  FrameState* st = B_.st + f;
  if (st->done) return;
  const SolveParams prm = *B_.prm;
  const double alpha = st->alpha;
  const float af = (float)alpha;
  const int knext = st->k + 1;
  const bool recompute = st->force_rc || (prm.recompute_every > 0 && knext % prm.recompute_every == 0);
  SysPtr s(B_.sys, B_.ntot);
  int c = (blockIdx.x - F.b0) * NODE_BLOCK + threadIdx.x;
  double rr = 0.0, rz = 0.0;
  if (c < F.n) {
    int64_t i = F.n0 + c;
    xnew[i] = fma(alpha, (double)p[i], xold[i]);
    float ri;
    if (recompute)
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
  if (last_arrival(B_.ticket + 4 * f + TK_UPD, F.nb)) {
    if (threadIdx.x == 0) {
      double rt = 0.0, zt = 0.0;
      for (int j = 0; j < F.nb; ++j) {
        rt += vload(B_.part_rr + F.b0 + j);
        zt += vload(B_.part_rz + F.b0 + j);
      }
      if (stop_checks(*st, prm, knext, rt, recompute)) {
        finish_frame(*st, B_.n_active);
      } else if (!(zt > 0.0) || !isfinite(zt)) {
        st->flags |= HP_NOT_SPD;
        finish_frame(*st, B_.n_active);
      } else {
        st->beta = zt / st->rho;
        st->rho = zt;
      }
    }
  }
}

// After a pass: frames that ended on an odd iteration hold x in x1.
__global__ void k_finalize_x(const FrameDesc* fr, const int* blk2f, const FrameState* st, const double* x1,
                             double* x0) {
  const int f = blk2f[blockIdx.x];
  const FrameDesc F = fr[f];
  if (!st[f].active || (st[f].k & 1) == 0) return;
  int c = (blockIdx.x - F.b0) * NODE_BLOCK + threadIdx.x;
  if (c < F.n) x0[F.n0 + c] = x1[F.n0 + c];
}

// ------------------------------------------------------------------ host launchers



static size_t coarse_lds_bytes(int kmax, int ls) { return (size_t)(5 * kmax * ls / 2 + ls) * sizeof(float); }

hp_status launch_assemble(const LaunchGeom& g, const float* rho, float* sys) {
  hipLaunchKernelGGL(k_assemble, dim3(g.nblk), dim3(NODE_BLOCK), 0, g.stream, g.fr, g.blk2f, rho, sys, g.ntot);
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
  hipLaunchKernelGGL((k_apply_coarse<LS, FT>), dim3(g.nframes), dim3(LEAF_THREADS), coarse_lds_bytes(g.kmax, LS),
                     g.stream, g.fr, fac, uh, vh, Tr, Tc);
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
  hipLaunchKernelGGL((k_setup_hmat<L, LS, FT>), dim3(g.ktot), dim3(LEAF_THREADS), coarse_lds_bytes(g.kmax, LS),
                     g.stream, g.fr, g.leaf2f, P.B, fac);
  hipLaunchKernelGGL((k_prolong<L, LS, FT>), dim3(g.ktot), dim3(LEAF_THREADS), 0, g.stream, g.fr, g.leaf2f, P.B, fac,
                     1);
}

template <int L, int LS, typename FT>
static void hmat_iter(const PcgLaunch& P, int parity) {
  auto fac = make_factors<L, LS, FT>(P);
  const LaunchGeom& g = P.g;
  const float* pold = parity ? P.B.p1 : P.B.p0;
  float* pnew = parity ? P.B.p0 : P.B.p1;
  const double* xold = parity ? P.B.x1 : P.B.x0;
  double* xnew = parity ? P.B.x0 : P.B.x1;
  hipLaunchKernelGGL(k_spmv_p, dim3(g.nblk), dim3(NODE_BLOCK), 0, g.stream, g.fr, g.blk2f, P.B, pold, pnew);
  hipLaunchKernelGGL((k_update_hmat<L, LS, FT>), dim3(g.ktot), dim3(LEAF_THREADS), coarse_lds_bytes(g.kmax, LS),
                     g.stream, g.fr, g.leaf2f, P.B, fac, xold, xnew, (const float*)pnew);
  hipLaunchKernelGGL((k_prolong<L, LS, FT>), dim3(g.ktot), dim3(LEAF_THREADS), 0, g.stream, g.fr, g.leaf2f, P.B, fac,
                     0);
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
  } else if (P.mode == HP_PRECOND_JACOBI) {
    hipLaunchKernelGGL(k_setup_simple<true>, dim3(g.nblk), dim3(NODE_BLOCK), 0, g.stream, g.fr, g.blk2f, P.B);
  } else {
    hipLaunchKernelGGL(k_setup_simple<false>, dim3(g.nblk), dim3(NODE_BLOCK), 0, g.stream, g.fr, g.blk2f, P.B);
  }
  HP_HIP(hipGetLastError());
  return HP_OK;
}

// Enqueue `count` iterations (count even) starting at parity 0.
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
      hipLaunchKernelGGL(k_spmv_p, dim3(g.nblk), dim3(NODE_BLOCK), 0, g.stream, g.fr, g.blk2f, P.B, pold, pnew);
      if (P.mode == HP_PRECOND_JACOBI)
        hipLaunchKernelGGL(k_update_simple<true>, dim3(g.nblk), dim3(NODE_BLOCK), 0, g.stream, g.fr, g.blk2f, P.B,
                           xold, xnew, (const float*)pnew);
      else
        hipLaunchKernelGGL(k_update_simple<false>, dim3(g.nblk), dim3(NODE_BLOCK), 0, g.stream, g.fr, g.blk2f,
                           P.B, xold, xnew, (const float*)pnew);
    }
  }
  HP_HIP(hipGetLastError());
  return HP_OK;
}

hp_status pcg_finalize(const PcgLaunch& P) {
  const LaunchGeom& g = P.g;
  hipLaunchKernelGGL(k_finalize_x, dim3(g.nblk), dim3(NODE_BLOCK), 0, g.stream, g.fr, g.blk2f,
                     (const FrameState*)P.B.st, (const double*)P.B.x1, P.B.x0);
  HP_HIP(hipGetLastError());
  return HP_OK;
}

}  // namespace hp
