// Cosine-Hutchinson training objective on the GPU (paper Sec. 6.1-6.2):
// spectrally smoothed probes, X = A Z, the multi-column apply Y = M X, the
// loss 1 - <Z, Y>_F / (||Z||_F ||Y||_F) per system and its reverse pass to the
// factor set (F, U, V, Ut, Vt, lam) of Sec. 4.4.  Every reduction has a fixed
// order.  Columns: KZ = 16 probes, stored [rows][KZ].
#include <math.h>

#include "batch.h"

namespace hp {

constexpr int KZ = 16;

__device__ inline double bsum_d(double v, double* red) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  double s = 0.0;
  for (int i = 0; i < (int)(blockDim.x >> 6); ++i) s += red[i];
  return s;
}

// ------------------------------------------------------------------ probes
// One damped-Jacobi sweep z <- z - omega D^-1 A z (Eq. 8), or (omega < 0)
// out = A z.  16 rows x 16 columns per block.
__global__ __launch_bounds__(256) void k_probe_step(const FrameDesc* fr, const int* node2f, const float* sys,
                                                   int64_t ntot, const float* Z, float* out, float omega) {
  const int64_t i = (int64_t)blockIdx.x * 16 + (threadIdx.x >> 4);
  if (i >= ntot) return;
  const int col = threadIdx.x & 15;
  const FrameDesc F = fr[node2f[i]];
  const unsigned c = (unsigned)(i - F.n0);
  const float *dg = sys, *wx = sys + ntot, *wy = sys + 2 * ntot, *wz = sys + 3 * ntot;
  auto v = [&](int64_t j) { return Z[j * KZ + col]; };
  const int64_t xp = F.n0 + mstep_plus(c, F.xm), xn = F.n0 + mstep_minus(c, F.xm);
  const int64_t yp = F.n0 + mstep_plus(c, F.ym), yn = F.n0 + mstep_minus(c, F.ym);
  const int64_t zp = F.n0 + mstep_plus(c, F.zm), zn = F.n0 + mstep_minus(c, F.zm);
  float a = dg[i] * v(i);
  a = fmaf(-wx[i], v(xp), a);
  a = fmaf(-wx[xn], v(xn), a);
  a = fmaf(-wy[i], v(yp), a);
  a = fmaf(-wy[yn], v(yn), a);
  a = fmaf(-wz[i], v(zp), a);
  a = fmaf(-wz[zn], v(zn), a);
  out[i * KZ + col] = omega < 0.f ? a : v(i) - omega * a / dg[i];
}

// ------------------------------------------------------------------ factor products
// G_k = F_k F_k^T (FP32; entries (i, j) and (j, i) run the same FMA sequence).
template <int L>
__global__ __launch_bounds__(256) void k_gram_f32(const float* F, float* G) {
  __shared__ float sF[L][L + 1];
  const int64_t kg = blockIdx.x;
  for (int idx = threadIdx.x; idx < L * L; idx += 256) sF[idx / L][idx % L] = F[kg * L * L + idx];
  __syncthreads();
  for (int idx = threadIdx.x; idx < L * L; idx += 256) {
    const int i = idx / L, j = idx % L;
    float a = 0.f;
    for (int c = 0; c < L; ++c) a = fmaf(sF[i][c], sF[j][c], a);
    G[kg * L * L + idx] = a;
  }
}

// B_m = U_m V_m^T.
template <int LS>
__global__ void k_uvt_f32(const float* U, const float* V, float* B) {
  const int64_t m = blockIdx.x;
  const int t = threadIdx.x / LS, t2 = threadIdx.x % LS;
  if (t >= LS) return;
  float a = 0.f;
  for (int s = 0; s < LS; ++s) a = fmaf(U[(m * LS + t) * LS + s], V[(m * LS + t2) * LS + s], a);
  B[(m * LS + t) * LS + t2] = a;
}

// ------------------------------------------------------------------ multi-column apply
// Leaf stage for KZ columns (one block per leaf): with_g: Y_k = G_k X_k +
// (lam / A_ii) X_k; always: restriction u_k = Ut_k^T X_k, v_k = Vt_k^T X_k.
template <int L, int LS>
__global__ __launch_bounds__(256) void k_m_leaf(const FrameDesc* fr, const int* leaf2f, const float* sys, int64_t ntot,
                                                const float* G, const float* Ut, const float* Vt, const float* lam,
                                                const float* X, float* Y, float* uh, float* vh, int with_g) {
  __shared__ float sX[L][KZ + 1];
  const int64_t kg = blockIdx.x;
  const FrameDesc F = fr[leaf2f[kg]];
  const int64_t row0 = F.n0 + (kg - F.k0) * L;
  for (int idx = threadIdx.x; idx < L * KZ; idx += 256) sX[idx / KZ][idx % KZ] = X[row0 * KZ + idx];
  __syncthreads();
  if (with_g) {
    for (int idx = threadIdx.x; idx < L * KZ; idx += 256) {
      const int l = idx / KZ, c = idx % KZ;
      const float* g = G + (kg * L + l) * L;
      float a = 0.f;
      for (int q = 0; q < L; ++q) a = fmaf(g[q], sX[q][c], a);
      const int64_t i = row0 + l;
      Y[i * KZ + c] = fmaf(lam[i] / sys[i], sX[l][c], a);
    }
  }
  for (int idx = threadIdx.x; idx < LS * KZ; idx += 256) {
    const int s = idx / KZ, c = idx % KZ;
    float a = 0.f, b = 0.f;
    for (int l = 0; l < L; ++l) {
      a = fmaf(Ut[(row0 + l) * LS + s], sX[l][c], a);
      b = fmaf(Vt[(row0 + l) * LS + s], sX[l][c], b);
    }
    uh[(kg * LS + s) * KZ + c] = a;
    vh[(kg * LS + s) * KZ + c] = b;
  }
}

// Coarse stage for KZ columns (one block per frame): per tile SR = sum of u
// over the row strip, SC = sum of v over the column strip; t^r = B SC,
// t^c = B^T SR; per leaf TR = sum of t^r over the tiles where it is on the
// row side, TC = sum of t^c where it is on the column side.  Phases are
// separated by block barriers; tmp holds t^r | t^c.
template <int LS>
__global__ __launch_bounds__(256) void k_m_coarse(const FrameDesc* fr, const float* uh, const float* vh,
                                                  const float* B, float* SR, float* SC, float* TR, float* TC,
                                                  float* tmp) {
  const FrameDesc F = fr[blockIdx.x];
  const int K = F.K, J = F.J, MH = F.MH, t = threadIdx.x, nt = blockDim.x;
  const int64_t kb = (int64_t)F.k0 * LS * KZ, mb = (int64_t)F.m0 * LS * KZ;
  const int per = LS * KZ;
  for (int e = t; e < MH * per; e += nt) {
    const int m = e / per, r = e % per;
    int j = 0;
    while (m >= K - (K >> (j + 1))) ++j;
    const int i = m - (K - (K >> j)), S = 1 << j;
    float a = 0.f, c = 0.f;
    for (int k = 2 * i * S; k < 2 * i * S + S; ++k) a += uh[kb + (int64_t)k * per + r];
    for (int k = 2 * i * S + S; k < 2 * i * S + 2 * S; ++k) c += vh[kb + (int64_t)k * per + r];
    SR[mb + e] = a;
    SC[mb + e] = c;
  }
  __syncthreads();
  float* tr = tmp + 2 * mb;
  float* tc = tr + (int64_t)MH * per;
  for (int e = t; e < MH * per; e += nt) {
    const int m = e / per, s = (e % per) / KZ, col = e % KZ;
    const float* Bm = B + ((int64_t)F.m0 + m) * LS * LS;
    float a = 0.f, c = 0.f;
    for (int u = 0; u < LS; ++u) {
      a = fmaf(Bm[s * LS + u], SC[mb + (int64_t)m * per + u * KZ + col], a);
      c = fmaf(Bm[u * LS + s], SR[mb + (int64_t)m * per + u * KZ + col], c);
    }
    tr[e] = a;
    tc[e] = c;
  }
  __syncthreads();
  for (int e = t; e < K * per; e += nt) {
    const int k = e / per, r = e % per;
    float a = 0.f, c = 0.f;
    for (int j = 0; j < J; ++j) {
      const int m = K - (K >> j) + (k >> (j + 1));
      if (((k >> j) & 1) == 0) a += tr[(int64_t)m * per + r];
      else c += tc[(int64_t)m * per + r];
    }
    TR[kb + e] = a;
    TC[kb + e] = c;
  }
}

// Prolongation for KZ columns: Y_k += Ut_k TR_k + Vt_k TC_k.
template <int L, int LS>
__global__ __launch_bounds__(256) void k_m_prolong(const FrameDesc* fr, const int* leaf2f, const float* Ut,
                                                   const float* Vt, const float* TR, const float* TC, float* Y) {
  const int64_t kg = blockIdx.x;
  const FrameDesc F = fr[leaf2f[kg]];
  const int64_t row0 = F.n0 + (kg - F.k0) * L;
  for (int idx = threadIdx.x; idx < L * KZ; idx += 256) {
    const int l = idx / KZ, c = idx % KZ;
    float a = 0.f;
    for (int s = 0; s < LS; ++s) {
      a = fmaf(Ut[(row0 + l) * LS + s], TR[(kg * LS + s) * KZ + c], a);
      a = fmaf(Vt[(row0 + l) * LS + s], TC[(kg * LS + s) * KZ + c], a);
    }
    Y[(row0 + l) * KZ + c] += a;
  }
}

// ------------------------------------------------------------------ loss
// Partials per node block of <Z,Y>, ||Z||^2, ||Y||^2 (FP64).
__global__ __launch_bounds__(256) void k_loss_partials(const FrameDesc* fr, const int* blk2f, const float* Z,
                                                       const float* Y, double* part) {
  __shared__ double red[4];
  const FrameDesc F = fr[blk2f[blockIdx.x]];
  const int c = (blockIdx.x - F.b0) * NODE_BLOCK + threadIdx.x;
  double zy = 0, zz = 0, yy = 0;
  if (c < F.n) {
    const int64_t i = F.n0 + c;
    for (int q = 0; q < KZ; ++q) {
      const double z = Z[i * KZ + q], y = Y[i * KZ + q];
      zy += z * y;
      zz += z * z;
      yy += y * y;
    }
  }
  zy = bsum_d(zy, red);
  zz = bsum_d(zz, red);
  yy = bsum_d(yy, red);
  if (threadIdx.x == 0) {
    part[3 * blockIdx.x] = zy;
    part[3 * blockIdx.x + 1] = zz;
    part[3 * blockIdx.x + 2] = yy;
  }
}

// Per frame: loss = 1 - zy / (|z||y|); coefficients of dY = c1 Z + c2 Y for
// the objective scale * sum_f loss_f: c1 = -scale / (|z||y|),
// c2 = scale zy / (|z| |y|^3).
__global__ void k_loss_frame(const FrameDesc* fr, const double* part, double scale, double* lossf, double* coef) {
  const FrameDesc F = fr[blockIdx.x];
  if (threadIdx.x != 0) return;
  double zy = 0, zz = 0, yy = 0;
  for (int b = 0; b < F.nb; ++b) {
    zy += part[3 * (F.b0 + b)];
    zz += part[3 * (F.b0 + b) + 1];
    yy += part[3 * (F.b0 + b) + 2];
  }
  const double nz = sqrt(zz), ny = sqrt(yy);
  lossf[blockIdx.x] = 1.0 - zy / (nz * ny);
  coef[2 * blockIdx.x] = -scale / (nz * ny);
  coef[2 * blockIdx.x + 1] = scale * zy / (nz * ny * ny * ny);
}

__global__ void k_loss_dy(const int* node2f, const double* coef, const float* Z, const float* Y, int64_t ntot,
                          float* dY) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= ntot * KZ) return;
  const int f = node2f[e / KZ];
  dY[e] = (float)(coef[2 * f] * (double)Z[e] + coef[2 * f + 1] * (double)Y[e]);
}

// ------------------------------------------------------------------ SAI-style loss (the loss ablation)
// L_f = || A Y / s_f - Z ||_F^2 with Y = M Z (Prop. 1(3)); s_f = ||A_f||
// read as the largest absolute row sum, from the FP64 coefficients, one
// block per frame.
__global__ __launch_bounds__(256) void k_sai_scale(const FrameDesc* fr, const float* sys, int64_t ntot, double* s) {
  __shared__ double red[4];
  const FrameDesc F = fr[blockIdx.x];
  const double* d64 = (const double*)(sys + 5 * ntot);
  const double *dg = d64, *wx = d64 + ntot, *wy = d64 + 2 * ntot, *wz = d64 + 3 * ntot;
  double m = 0.0;
  for (int c = threadIdx.x; c < F.n; c += blockDim.x) {
    const int64_t i = F.n0 + c;
    const unsigned cu = (unsigned)c;
    const int64_t xn = F.n0 + mstep_minus(cu, F.xm), yn = F.n0 + mstep_minus(cu, F.ym),
                  zn = F.n0 + mstep_minus(cu, F.zm);
    m = fmax(m, dg[i] + wx[i] + wx[xn] + wy[i] + wy[yn] + wz[i] + wz[zn]);
  }
  for (int o = 32; o > 0; o >>= 1) m = fmax(m, __shfl_xor(m, o, 64));
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    double r = red[0];
    for (int w = 1; w < (int)(blockDim.x >> 6); ++w) r = fmax(r, red[w]);
    s[blockIdx.x] = r;
  }
}

// Partials per node block of sum (W / s - Z)^2 with W = A Y (FP64).
__global__ __launch_bounds__(256) void k_sai_partials(const FrameDesc* fr, const int* blk2f, const float* Z,
                                                      const float* W, const double* s, double* part) {
  __shared__ double red[4];
  const int f = blk2f[blockIdx.x];
  const FrameDesc F = fr[f];
  const int c = (blockIdx.x - F.b0) * NODE_BLOCK + threadIdx.x;
  const double inv = 1.0 / s[f];
  double acc = 0;
  if (c < F.n) {
    const int64_t i = F.n0 + c;
    for (int q = 0; q < KZ; ++q) {
      const double r = (double)W[i * KZ + q] * inv - (double)Z[i * KZ + q];
      acc += r * r;
    }
  }
  acc = bsum_d(acc, red);
  if (threadIdx.x == 0) part[3 * blockIdx.x] = acc;
}

// Per frame: the loss and the coefficients of dW = c1 (W c2 - Z) for the
// objective scale * sum_f L_f: c1 = 2 scale / s_f, c2 = 1 / s_f.
__global__ void k_sai_frame(const FrameDesc* fr, const double* part, const double* s, double scale, double* lossf,
                            double* coef) {
  const FrameDesc F = fr[blockIdx.x];
  if (threadIdx.x != 0) return;
  double l = 0;
  for (int b = 0; b < F.nb; ++b) l += part[3 * (F.b0 + b)];
  lossf[blockIdx.x] = l;
  coef[2 * blockIdx.x] = 2.0 * scale / s[blockIdx.x];
  coef[2 * blockIdx.x + 1] = 1.0 / s[blockIdx.x];
}

// dW = c1 (W c2 - Z), in place of W; dY = A dW follows (A symmetric).
__global__ void k_sai_dw(const int* node2f, const double* coef, const float* Z, float* W, int64_t ntot) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= ntot * KZ) return;
  const int f = node2f[e / KZ];
  W[e] = (float)(coef[2 * f] * ((double)W[e] * coef[2 * f + 1] - (double)Z[e]));
}

// ------------------------------------------------------------------ reverse pass to the factors
// Per leaf: dG = dY_k X_k^T, dF_k = (dG + dG^T) F_k, dlam_i = sum_q dY X / A_ii,
// dUt_k = dY_k TR_k^T + X_k TR2_k^T, dVt_k = dY_k TC_k^T + X_k TC2_k^T.
template <int L, int LS>
__global__ __launch_bounds__(256) void k_grad_leaf(const FrameDesc* fr, const int* leaf2f, const float* sys,
                                                   const float* F, const float* X, const float* dY, const float* TR,
                                                   const float* TC, const float* TR2, const float* TC2, float* dF,
                                                   float* dUt, float* dVt, float* dlam) {
  __shared__ float sX[L][KZ + 1], sD[L][KZ + 1];
  __shared__ float sG[L][L + 1];
  const int64_t kg = blockIdx.x;
  const FrameDesc Fd = fr[leaf2f[kg]];
  const int64_t row0 = Fd.n0 + (kg - Fd.k0) * L;
  for (int idx = threadIdx.x; idx < L * KZ; idx += 256) {
    sX[idx / KZ][idx % KZ] = X[row0 * KZ + idx];
    sD[idx / KZ][idx % KZ] = dY[row0 * KZ + idx];
  }
  __syncthreads();
  for (int idx = threadIdx.x; idx < L * L; idx += 256) {
    const int i = idx / L, j = idx % L;
    float a = 0.f;
    for (int q = 0; q < KZ; ++q) a = fmaf(sD[i][q], sX[j][q], a);
    sG[i][j] = a;
  }
  __syncthreads();
  for (int idx = threadIdx.x; idx < L * L; idx += 256) {
    const int i = idx / L, c = idx % L;
    const float* Fk = F + kg * L * L;
    float a = 0.f;
    for (int j = 0; j < L; ++j) a = fmaf(sG[i][j] + sG[j][i], Fk[j * L + c], a);
    dF[kg * L * L + idx] = a;
  }
  for (int l = threadIdx.x; l < L; l += 256) {
    float a = 0.f;
    for (int q = 0; q < KZ; ++q) a = fmaf(sD[l][q], sX[l][q], a);
    dlam[row0 + l] = a / sys[row0 + l];
  }
  for (int idx = threadIdx.x; idx < L * LS; idx += 256) {
    const int l = idx / LS, s = idx % LS;
    float a = 0.f, b = 0.f;
    for (int q = 0; q < KZ; ++q) {
      a = fmaf(sD[l][q], TR[(kg * LS + s) * KZ + q], a);
      a = fmaf(sX[l][q], TR2[(kg * LS + s) * KZ + q], a);
      b = fmaf(sD[l][q], TC[(kg * LS + s) * KZ + q], b);
      b = fmaf(sX[l][q], TC2[(kg * LS + s) * KZ + q], b);
    }
    dUt[(row0 + l) * LS + s] = a;
    dVt[(row0 + l) * LS + s] = b;
  }
}

// Per tile: dB = SR2 SC^T + SR SC2^T, dU = dB V, dV = dB^T U.
template <int LS>
__global__ __launch_bounds__(256) void k_grad_tile(const float* U, const float* V, const float* SR, const float* SC,
                                                   const float* SR2, const float* SC2, float* dU, float* dV) {
  __shared__ float sB[LS][LS + 1];
  const int64_t m = blockIdx.x;
  const int64_t base = m * LS * KZ;
  for (int idx = threadIdx.x; idx < LS * LS; idx += 256) {
    const int s = idx / LS, u = idx % LS;
    float a = 0.f;
    for (int q = 0; q < KZ; ++q) {
      a = fmaf(SR2[base + s * KZ + q], SC[base + u * KZ + q], a);
      a = fmaf(SR[base + s * KZ + q], SC2[base + u * KZ + q], a);
    }
    sB[s][u] = a;
  }
  __syncthreads();
  for (int idx = threadIdx.x; idx < LS * LS; idx += 256) {
    const int t = idx / LS, s = idx % LS;
    float a = 0.f, b = 0.f;
    for (int u = 0; u < LS; ++u) {
      a = fmaf(sB[t][u], V[(m * LS + u) * LS + s], a);
      b = fmaf(sB[u][t], U[(m * LS + u) * LS + s], b);
    }
    dU[(m * LS + t) * LS + s] = a;
    dV[(m * LS + t) * LS + s] = b;
  }
}

// ------------------------------------------------------------------ workspace and drivers

struct TrainWS {
  int kz = 0;
  float *G = nullptr, *B = nullptr, *Y = nullptr, *dY = nullptr;
  float* W = nullptr;          // SAI loss: A Y, then its adjoint dW
  double* sai_s = nullptr;     // SAI loss: ||A|| per frame
  float *uh = nullptr, *vh = nullptr, *gu = nullptr, *gv = nullptr;
  float *SR = nullptr, *SC = nullptr, *SR2 = nullptr, *SC2 = nullptr;
  float *TR = nullptr, *TC = nullptr, *TR2 = nullptr, *TC2 = nullptr, *tmp = nullptr, *scratch = nullptr;
  double *part = nullptr, *lossf = nullptr, *coef = nullptr;
  int* node2f = nullptr;
};

static TrainWS* tws(Batch& b) { return reinterpret_cast<TrainWS*>(b.train_ws); }

hp_status train_ws_alloc(Batch& b) {
  if (b.train_ws) return HP_OK;
  auto* T = new TrainWS();
  b.train_ws = T;
  b.train_free = [](void* p) { delete reinterpret_cast<TrainWS*>(p); };
  const int L = b.cfg.leaf, LS = b.cfg.rank;
  const int64_t nt = b.ntot, kt = b.ktot, mt = std::max<int64_t>(b.mtot, 1);
  hp_status s = HP_OK;
  auto A = [&](auto** p, size_t bytes) {
    if (s == HP_OK) s = b.alloc((void**)p, bytes);
  };
  A(&T->G, kt * L * L * 4);
  A(&T->B, mt * LS * LS * 4);
  A(&T->Y, nt * KZ * 4);
  A(&T->dY, nt * KZ * 4);
  A(&T->W, nt * KZ * 4);
  A(&T->sai_s, std::max(b.nframes, 1) * 8);
  for (float** p : {&T->uh, &T->vh, &T->gu, &T->gv, &T->TR, &T->TC, &T->TR2, &T->TC2}) A(p, kt * LS * KZ * 4);
  for (float** p : {&T->SR, &T->SC, &T->SR2, &T->SC2}) A(p, mt * LS * KZ * 4);
  A(&T->tmp, 2 * mt * LS * KZ * 4);
  A(&T->part, (size_t)3 * b.nblk * 8);
  A(&T->lossf, b.nframes * 8);
  A(&T->coef, 2 * b.nframes * 8);
  A(&T->node2f, nt * 4);
  if (s != HP_OK) return s;
  std::vector<int> n2f(nt);
  for (int f = 0; f < b.nframes; ++f)
    for (int i = 0; i < b.fr[f].n; ++i) n2f[b.fr[f].n0 + i] = f;
  HP_HIP(hipMemcpy(T->node2f, n2f.data(), nt * 4, hipMemcpyHostToDevice));
  T->kz = KZ;
  return HP_OK;
}

template <int L, int LS>
static hp_status loss_fwd_t(Batch& b, const float* sys, const hp_factor_set& f, const float* X, const float* Z,
                            double scale) {
  TrainWS& T = *tws(b);
  hipStream_t st = b.stream;
  const int64_t nt = b.ntot;
  hipLaunchKernelGGL((k_gram_f32<L>), dim3((unsigned)b.ktot), dim3(256), 0, st, (const float*)f.F, T.G);
  if (b.mtot > 0)
    hipLaunchKernelGGL((k_uvt_f32<LS>), dim3((unsigned)b.mtot), dim3(LS * LS), 0, st, (const float*)f.U,
                       (const float*)f.V, T.B);
  hipLaunchKernelGGL((k_m_leaf<L, LS>), dim3((unsigned)b.ktot), dim3(256), 0, st, b.d_fr, b.d_leaf2f, sys, nt,
                     (const float*)T.G, (const float*)f.Ut, (const float*)f.Vt, (const float*)f.lam, X, T.Y, T.uh,
                     T.vh, 1);
  hipLaunchKernelGGL((k_m_coarse<LS>), dim3(b.nframes), dim3(256), 0, st, b.d_fr, (const float*)T.uh,
                     (const float*)T.vh, (const float*)T.B, T.SR, T.SC, T.TR, T.TC, T.tmp);
  hipLaunchKernelGGL((k_m_prolong<L, LS>), dim3((unsigned)b.ktot), dim3(256), 0, st, b.d_fr, b.d_leaf2f,
                     (const float*)f.Ut, (const float*)f.Vt, (const float*)T.TR, (const float*)T.TC, T.Y);
  if (b.loss_kind == 1) {  // SAI: W = A Y, || W / s - Z ||^2
    hipLaunchKernelGGL(k_probe_step, dim3((unsigned)((nt + 15) / 16)), dim3(256), 0, st, b.d_fr,
                       (const int*)T.node2f, sys, nt, (const float*)T.Y, T.W, -1.f);
    hipLaunchKernelGGL(k_sai_scale, dim3(b.nframes), dim3(256), 0, st, b.d_fr, sys, nt, T.sai_s);
    hipLaunchKernelGGL(k_sai_partials, dim3(b.nblk), dim3(NODE_BLOCK), 0, st, b.d_fr, b.d_blk2f, Z,
                       (const float*)T.W, (const double*)T.sai_s, T.part);
    hipLaunchKernelGGL(k_sai_frame, dim3(b.nframes), dim3(64), 0, st, b.d_fr, (const double*)T.part,
                       (const double*)T.sai_s, scale, T.lossf, T.coef);
  } else {
    hipLaunchKernelGGL(k_loss_partials, dim3(b.nblk), dim3(NODE_BLOCK), 0, st, b.d_fr, b.d_blk2f, Z,
                       (const float*)T.Y, T.part);
    hipLaunchKernelGGL(k_loss_frame, dim3(b.nframes), dim3(64), 0, st, b.d_fr, (const double*)T.part, scale,
                       T.lossf, T.coef);
  }
  HP_HIP(hipGetLastError());
  return HP_OK;
}

template <int L, int LS>
static hp_status loss_bwd_t(Batch& b, const float* sys, const hp_factor_set& f, const float* X, const float* Z,
                            const hp_factor_set& g) {
  TrainWS& T = *tws(b);
  hipStream_t st = b.stream;
  const int64_t nt = b.ntot;
  if (b.loss_kind == 1) {  // SAI: dW = c1 (W c2 - Z), dY = A dW
    hipLaunchKernelGGL(k_sai_dw, dim3((unsigned)((nt * KZ + 255) / 256)), dim3(256), 0, st, (const int*)T.node2f,
                       (const double*)T.coef, Z, T.W, nt);
    hipLaunchKernelGGL(k_probe_step, dim3((unsigned)((nt + 15) / 16)), dim3(256), 0, st, b.d_fr,
                       (const int*)T.node2f, sys, nt, (const float*)T.W, T.dY, -1.f);
  } else {
    hipLaunchKernelGGL(k_loss_dy, dim3((unsigned)((nt * KZ + 255) / 256)), dim3(256), 0, st,
                       (const int*)T.node2f, (const double*)T.coef, Z, (const float*)T.Y, nt, T.dY);
  }
  hipLaunchKernelGGL((k_m_leaf<L, LS>), dim3((unsigned)b.ktot), dim3(256), 0, st, b.d_fr, b.d_leaf2f, sys, nt,
                     (const float*)T.G, (const float*)f.Ut, (const float*)f.Vt, (const float*)f.lam,
                     (const float*)T.dY, T.Y /* unused */, T.gu, T.gv, 0);
  hipLaunchKernelGGL((k_m_coarse<LS>), dim3(b.nframes), dim3(256), 0, st, b.d_fr, (const float*)T.gu,
                     (const float*)T.gv, (const float*)T.B, T.SR2, T.SC2, T.TR2, T.TC2, T.tmp);
  hipLaunchKernelGGL((k_grad_leaf<L, LS>), dim3((unsigned)b.ktot), dim3(256), 0, st, b.d_fr, b.d_leaf2f, sys,
                     (const float*)f.F, X, (const float*)T.dY, (const float*)T.TR, (const float*)T.TC,
                     (const float*)T.TR2, (const float*)T.TC2, g.F, g.Ut, g.Vt, g.lam);
  if (b.mtot > 0)
    hipLaunchKernelGGL((k_grad_tile<LS>), dim3((unsigned)b.mtot), dim3(256), 0, st, (const float*)f.U,
                       (const float*)f.V, (const float*)T.SR, (const float*)T.SC, (const float*)T.SR2,
                       (const float*)T.SC2, g.U, g.V);
  HP_HIP(hipGetLastError());
  return HP_OK;
}

// With the SAI loss the apply's input is Z itself (Y = M Z), not X = A Z.
hp_status loss_fwd(Batch& b, const float* sys, const hp_factor_set& f, const float* X, const float* Z, double scale) {
  const float* Xa = b.loss_kind == 1 ? Z : X;
  if (b.cfg.leaf == 64) return loss_fwd_t<64, 16>(b, sys, f, Xa, Z, scale);
  return loss_fwd_t<32, 8>(b, sys, f, Xa, Z, scale);
}

hp_status loss_bwd(Batch& b, const float* sys, const hp_factor_set& f, const float* X, const float* Z,
                   const hp_factor_set& g) {
  const float* Xa = b.loss_kind == 1 ? Z : X;
  if (b.cfg.leaf == 64) return loss_bwd_t<64, 16>(b, sys, f, Xa, Z, g);
  return loss_bwd_t<32, 8>(b, sys, f, Xa, Z, g);
}

hp_status probes(Batch& b, const float* sys, const float* zraw, float* z, float* x, int sweeps, float omega) {
  TrainWS& T = *tws(b);
  hipStream_t st = b.stream;
  const unsigned grid = (unsigned)((b.ntot + 15) / 16);
  const float* src = zraw;
  for (int s = 0; s < sweeps; ++s) {
    // ping-pong between z and dY, chosen by the parity of the sweeps left so
    // that the last sweep lands in z and no sweep reads its own output
    float* dst = ((sweeps - 1 - s) % 2 == 0) ? z : T.dY;
    hipLaunchKernelGGL(k_probe_step, dim3(grid), dim3(256), 0, st, b.d_fr, (const int*)T.node2f, sys, b.ntot, src,
                       dst, omega);
    src = dst;
  }
  if (sweeps == 0) HP_HIP(hipMemcpyAsync(z, zraw, b.ntot * KZ * 4, hipMemcpyDeviceToDevice, st));
  hipLaunchKernelGGL(k_probe_step, dim3(grid), dim3(256), 0, st, b.d_fr, (const int*)T.node2f, sys, b.ntot,
                     (const float*)z, x, -1.f);
  HP_HIP(hipGetLastError());
  return HP_OK;
}

const double* train_lossf(Batch& b) { return tws(b)->lossf; }

}  // namespace hp

using namespace hp;

extern "C" hp_status hp_train_init(hp_batch b, int32_t kz) {
  if (!b) return set_error(HP_E_INVALID, "hp_train_init: NULL batch");
  if (kz != KZ) return set_error(HP_E_INVALID, "hp_train_init: kz must be %d", KZ);
  return train_ws_alloc(*b);
}

extern "C" hp_status hp_probes(hp_batch b, const float* d_sys, const float* d_zraw, float* d_z, float* d_x,
                               int32_t sweeps, float omega) {
  if (!b || !d_sys || !d_zraw || !d_z || !d_x || sweeps < 0) return set_error(HP_E_INVALID, "hp_probes: bad arguments");
  if (!b->train_ws) return set_error(HP_E_STATE, "hp_probes: call hp_train_init first");
  if (d_zraw == d_z) return set_error(HP_E_INVALID, "hp_probes: zraw and z must not alias");
  return probes(*b, d_sys, d_zraw, d_z, d_x, sweeps, omega);
}

extern "C" hp_status hp_loss_fwd(hp_batch b, const float* d_sys, const hp_factor_set* f, const float* d_x,
                                 const float* d_z, double scale, double* h_loss) {
  if (!b || !d_sys || !f || !d_x || !d_z || !h_loss) return set_error(HP_E_INVALID, "hp_loss_fwd: NULL argument");
  if (!b->train_ws) return set_error(HP_E_STATE, "hp_loss_fwd: call hp_train_init first");
  HP_TRY(loss_fwd(*b, d_sys, *f, d_x, d_z, scale));
  HP_HIP(hipMemcpyAsync(h_loss, tws(*b)->lossf, b->nframes * 8, hipMemcpyDeviceToHost, b->stream));
  HP_HIP(hipStreamSynchronize(b->stream));
  return HP_OK;
}

extern "C" hp_status hp_loss_bwd(hp_batch b, const float* d_sys, const hp_factor_set* f, const float* d_x,
                                 const float* d_z, const hp_factor_set* grad) {
  if (!b || !d_sys || !f || !d_x || !d_z || !grad) return set_error(HP_E_INVALID, "hp_loss_bwd: NULL argument");
  if (!b->train_ws) return set_error(HP_E_STATE, "hp_loss_bwd: call hp_train_init first");
  return loss_bwd(*b, d_sys, *f, d_x, d_z, *grad);
}
