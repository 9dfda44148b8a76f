// Training of the network on the GPU (included at the end of network.hip):
// the forward pass with saves, the cosine-Hutchinson loss and its adjoint
// with respect to the factors (train.hip), then the reverse pass through the
// heads, every transformer block (recomputed from its saved input), the
// pooling and the encoder; and the AdamW update with a global-norm clip
// (Sec. 6.3; Supplementary "Optimizer and schedule").
#pragma once

namespace hp {

struct NetTrainBufs {
  TrainSave sv{};
  LayerSave ls{};
  float *Zs = nullptr, *X = nullptr;                  // smoothed probes, A Zs  [Nd][16]
  float *ones = nullptr, *preh = nullptr, *preg = nullptr;
  float *dXd = nullptr, *dXo = nullptr, *da = nullptr, *dao = nullptr, *dO = nullptr, *dh = nullptr;
  float *d512 = nullptr, *dqkv = nullptr, *dR = nullptr, *dC = nullptr, *dGd = nullptr, *dGo = nullptr;
  float *dctx = nullptr, *WR = nullptr, *WC = nullptr, *dgf = nullptr;
  float *dsb = nullptr, *dsbo = nullptr, *dcorr = nullptr, *dT0 = nullptr;
  void *t128b = nullptr, *t512b = nullptr, *t384b = nullptr, *t64b = nullptr;
  float *U = nullptr, *V = nullptr, *Ut = nullptr, *Vt = nullptr, *lam = nullptr;
  float *gF = nullptr, *gU = nullptr, *gV = nullptr, *gUt = nullptr, *gVt = nullptr, *glam = nullptr;
  float *dNH = nullptr, *dUV = nullptr;
  float* part = nullptr;  // chunk partials of the row reductions
  int64_t part_cap = 0;
  double *gnpart = nullptr, *gnorm = nullptr;
  int ngn = 0;
  int64_t nw = 0;
};

static NetTrainBufs* ntb_of(Batch& b) { return reinterpret_cast<NetTrainBufs*>(b.net_train); }

constexpr int64_t GN_CHUNK = 65536;

hp_status network_train_alloc(Batch& b) {
  if (b.net_train) return HP_OK;
  const hp_model_config& c = b.cfg;
  if (c.edge_hidden > 32 || c.heads > 8)
    return set_error(HP_E_SHAPE, "training: supported edge_hidden <= 32 and heads <= 8");
  HP_TRY(network_alloc(b));
  HP_TRY(train_ws_alloc(b));
  auto* T = new NetTrainBufs();
  b.net_train = T;
  b.net_train_free = [](void* p) { delete reinterpret_cast<NetTrainBufs*>(p); };
  NetBufs& N = *nb_of(b);
  const int64_t Nd = N.Nd, No = N.No, d = c.d, H = c.heads, L = c.leaf, LS = c.rank;
  const int64_t mt = std::max<int64_t>(b.mtot, 1), R = std::max(Nd, No);
  int32_t cnt;
  hp_weight_count(&c, &cnt, &T->nw);
  hp_status s = HP_OK;
  auto A = [&](auto** p, size_t bytes) {
    if (s == HP_OK) s = b.alloc((void**)p, bytes);
  };
  for (int g = 0; g <= c.gcn; ++g) A(&T->sv.Hg[g], Nd * d * 4);
  for (int l = 0; l <= c.layers; ++l) {
    A(&T->sv.xin_d[l], Nd * d * 4);
    A(&T->sv.xin_o[l], No * d * 4);
  }
  A(&T->ls.xmid_d, Nd * d * 4);
  A(&T->ls.xmid_o, No * d * 4);
  A(&T->ls.pre_d, Nd * 4 * d * 4);
  A(&T->ls.pre_o, No * 4 * d * 4);
  A(&T->Zs, Nd * 16 * 4);
  A(&T->X, Nd * 16 * 4);
  A(&T->ones, b.nframes * 4);
  A(&T->preh, Nd * d * 4);
  A(&T->preg, Nd * d * 4);
  for (float** p : {&T->dXd, &T->da, &T->dO, &T->dh, &T->dR, &T->dC, &T->dGd, &T->WR, &T->WC}) A(p, R * d * 4);
  for (float** p : {&T->dXo, &T->dao, &T->dGo}) A(p, No * d * 4);
  A(&T->dctx, No * 2 * d * 4);
  A(&T->d512, R * 4 * d * 4);
  A(&T->dqkv, R * 3 * d * 4);
  A(&T->t128b, R * d * 4);
  A(&T->t512b, R * 4 * d * 4);
  A(&T->t384b, R * 3 * d * 4);
  A(&T->t64b, R * 64 * 4);
  A(&T->dgf, b.nframes * d * 4);
  A(&T->dsb, b.ktot * H * L * L * 4);
  A(&T->dsbo, mt * H * LS * LS * 4);
  A(&T->dcorr, Nd * 7 * H * 4);
  A(&T->dT0, H * L * L * 4);
  A(&T->U, mt * LS * LS * 4);
  A(&T->V, mt * LS * LS * 4);
  A(&T->Ut, Nd * LS * 4);
  A(&T->Vt, Nd * LS * 4);
  A(&T->lam, Nd * 4);
  A(&T->gF, Nd * L * 4);
  A(&T->gU, mt * LS * LS * 4);
  A(&T->gV, mt * LS * LS * 4);
  A(&T->gUt, Nd * LS * 4);
  A(&T->gVt, Nd * LS * 4);
  A(&T->glam, Nd * 4);
  A(&T->dNH, Nd * 64 * 4);
  A(&T->dUV, No * 2 * LS * 4);
  // LayerNorm partials are the largest user: one 2C row per 16 rows
  T->part_cap = std::max<int64_t>(16ll << 20, (R / 16 + 64) * 2 * 4 * d);
  A(&T->part, T->part_cap * 4);
  T->ngn = (int)((T->nw + GN_CHUNK - 1) / GN_CHUNK);
  A(&T->gnpart, T->ngn * 8);
  A(&T->gnorm, 8);
  if (s != HP_OK) return s;
  std::vector<float> ones(b.nframes, 1.f);
  HP_HIP(hipMemcpy(T->ones, ones.data(), b.nframes * 4, hipMemcpyHostToDevice));
  return HP_OK;
}

__global__ void k_fill(float* p, int64_t n, float v) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < n) p[e] = v;
}

// y[r][c] = x[r][c] for c < cols, 0 for cols <= c < ycols (compute type).
template <typename AT>
__global__ void k_to_act_pad(const float* x, int64_t rows, int cols, int64_t ldx, AT* y, int ycols) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= rows * ycols) return;
  const int64_t r = e / ycols;
  const int c = (int)(e % ycols);
  y[e] = to_act<AT>(c < cols ? x[r * ldx + c] : 0.f);
}

// dctx[tok] = (dA[tok] | dB[tok]): the two context segments of the
// off-diagonal LayerNorm adjoint, packed as the strip-mean adjoint reads them.
__global__ void k_pack_ctx(const float* dA, const float* dB, int64_t ntok, float* dctx) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= ntok * 128) return;
  const int64_t t = e >> 7;
  const int c = (int)(e & 127);
  dctx[t * 256 + c] = dA[e];
  dctx[t * 256 + 128 + c] = dB[e];
}

static unsigned gsz(int64_t n, int bs = 256) { return (unsigned)((n + bs - 1) / bs); }

template <typename AT>
struct TrainCtx {
  Batch& b;
  NetTrainBufs& T;
  const NetPlan& P;
  hipStream_t st;
  const float* W;
  float* G;  // flat weight gradient (accumulated)

  int64_t off(const std::string& n) const { return woff(P, n); }
  const float* wp(const std::string& n) const { return W + woff(P, n); }

  // G[dst + i ldo + (o - o_begin)] += sum_r X[r][i] D[r][o] for i < ni_store,
  // o in [o_begin, o_begin + o_count); X [M][ldx] and D [M][ldd] in AT.
  void dW(const void* X, int64_t ldx, int NI, const void* D, int64_t ldd, int NO, int64_t M, const std::string& dst,
          int ldo, int o_begin, int o_count, int ni_store) {
    if (M <= 0) return;
    const int tiles = ((NI + 63) / 64) * ((NO + 63) / 64);
    int64_t nch = std::max<int64_t>(1, std::min<int64_t>(512 / tiles + 1, (M + 1023) / 1024));
    nch = std::max<int64_t>(1, std::min<int64_t>(nch, T.part_cap / ((int64_t)NI * NO)));
    int64_t rpc = (M + nch - 1) / nch;
    rpc = (rpc + 31) / 32 * 32;
    nch = (M + rpc - 1) / rpc;
    GemmTNArgs a{X, ldx, D, ldd, (int)M, NI, NO, (int)rpc, T.part};
    hipLaunchKernelGGL(k_gemm_tn<AT>, dim3((unsigned)((NI + 63) / 64), (unsigned)((NO + 63) / 64), (unsigned)nch),
                       dim3(256), 0, st, a);
    hipLaunchKernelGGL(k_reduce_chunks, dim3(gsz((int64_t)ni_store * o_count)), dim3(256), 0, st,
                       (const float*)T.part, (int)nch, NI, NO, o_begin, o_count, ni_store, G + off(dst), ldo, 1);
  }
  // G[dst + (o - o_begin)] += column sums of D[:, o] (FP32 [M][ldd]).
  void dB(const float* D, int64_t ldd, int NO, int64_t M, const std::string& dst, int o_begin, int o_count) {
    if (M <= 0) return;
    const int64_t rpc = 1024, nch = (M + rpc - 1) / rpc;
    hipLaunchKernelGGL(k_colsum_chunks, dim3((unsigned)((NO + 255) / 256), (unsigned)nch), dim3(256), 0, st, D, ldd,
                       (int)M, NO, (int)rpc, T.part);
    hipLaunchKernelGGL(k_reduce_chunks, dim3(gsz(o_count)), dim3(256), 0, st, (const float*)T.part, (int)nch, 1, NO,
                       o_begin, o_count, 1, G + off(dst), 0, 1);
  }
  void toact(const float* x, int64_t rows, int cols, int64_t ldx, void* y, int ycols) {
    if (rows <= 0) return;
    hipLaunchKernelGGL(k_to_act_pad<AT>, dim3(gsz(rows * ycols)), dim3(256), 0, st, x, rows, cols, ldx, (AT*)y,
                       ycols);
  }
  // LayerNorm adjoint; gamma then beta gradients land in the contiguous
  // name.g / name.b slots.
  template <int C>
  void ln_bwd(const LnSeg& in, const std::string& name, const float* dY, int64_t M, float* dX0, int acc0, float* dX1,
              float* dX2, float* dX3) {
    if (M <= 0) return;
    const int64_t nblk = (M + 15) / 16;
    hipLaunchKernelGGL(k_ln_bwd<C>, dim3((unsigned)nblk), dim3(256), 0, st, in, wp(name + ".g"), dY, (int)M, dX0,
                       acc0, dX1, dX2, dX3, T.part);
    hipLaunchKernelGGL(k_reduce_chunks, dim3(gsz(2 * C)), dim3(256), 0, st, (const float*)T.part, (int)nblk, 1, 2 * C,
                       0, 2 * C, 1, G + off(name + ".g"), 0, 1);
  }
  // Edge-MLP parameters (e1.w, e1.b, e2.w, e2.b are contiguous).
  void edge_bwd(const std::string& pre, const EdgeBwdSrc& src) {
    if (src.npairs <= 0) return;
    EdgeW ew{wp(pre + "e1.w"), wp(pre + "e1.b"), wp(pre + "e2.w"), wp(pre + "e2.b"), b.cfg.edge_hidden, b.cfg.heads};
    const int NP = 5 * ew.E + ew.E * ew.H + ew.H;
    const int64_t ppb = 2048, nblk = (src.npairs + ppb - 1) / ppb;
    hipLaunchKernelGGL(k_edge_bwd, dim3((unsigned)nblk), dim3(256), 0, st, ew, src, ppb, T.part);
    hipLaunchKernelGGL(k_reduce_chunks, dim3(gsz(NP)), dim3(256), 0, st, (const float*)T.part, (int)nblk, 1, NP, 0,
                       NP, 1, G + off(pre + "e1.w"), 0, 1);
  }
};

// Gradient of the batch-mean loss with respect to the flat weights W
// (written to grad); the mean loss is returned through h_loss when set.
template <typename AT>
static hp_status train_grad_t(Batch& b, const float* W, const float* rho, const float* sys, const float* zraw,
                              int sweeps, float omega, float* grad, double* h_loss) {
  NetBufs& N = *nb_of(b);
  NetTrainBufs& T = *ntb_of(b);
  const NetPlan& P = N.plan;
  const hp_model_config& c = b.cfg;
  hipStream_t st = b.stream;
  TrainCtx<AT> X{b, T, P, st, W, grad};
  const int64_t Nd = N.Nd, d = c.d, L = c.leaf, LS = c.rank, H = c.heads;
  const int64_t No = b.mtot * LS, mt = std::max<int64_t>(b.mtot, 1);
  const bool use_off = c.offdiag && b.mtot > 0;
  const FrameDesc* fr = b.d_fr;
  hipLaunchKernelGGL(k_fill, dim3(gsz(T.nw)), dim3(256), 0, st, grad, T.nw, 0.f);
  // the forward pass runs the FFNs as the two GEMMs its per-layer
  // recomputation differentiates (never the fused inference kernel)
  struct FfnGuard {
    Batch& b;
    int saved;
    ~FfnGuard() { b.ffn_fused = saved; }
  } ffn_guard{b, b.ffn_fused};
  b.ffn_fused = 0;

  // ---- probes (Sec. 6.3) and the forward pass with saves
  HP_TRY(probes(b, sys, zraw, T.Zs, T.X, sweeps, omega));
  HP_TRY(fwd_prologue<AT>(b, W, rho, sys, &T.sv));
  for (int l = 0; l < c.layers; ++l) {
    HP_HIP(hipMemcpyAsync(T.sv.xin_d[l], N.H, Nd * d * 4, hipMemcpyDeviceToDevice, st));
    if (use_off) HP_HIP(hipMemcpyAsync(T.sv.xin_o[l], N.Xo, No * d * 4, hipMemcpyDeviceToDevice, st));
    HP_TRY(layer_fwd<AT>(b, W, sys, l, nullptr));
  }
  // heads (Sec. 4.4) into an FP32 factor set
  hipLaunchKernelGGL(k_layernorm128<AT>, dim3(gsz(Nd, 16)), dim3(256), 0, st, (const float*)N.H, X.wp("diaglnf.g"),
                     X.wp("diaglnf.b"), (AT*)N.a128, (int)Nd);
  gemm<AT>(b, N.a128, d, N, P.hleaf1, X.wp("hleaf1.b"), nullptr, 0, nullptr, 0, N.b128, d, Nd, 1, T.preh, d);
  gemm<AT>(b, N.b128, d, N, P.hleaf2, X.wp("hleaf2.b"), nullptr, 0, N.Frows, L, nullptr, 0, Nd, 0);
  gemm<AT>(b, N.a128, d, N, P.hnode, N.bias_node, nullptr, 0, N.NH, 36, nullptr, 0, Nd, 0);
  if (LS == 16)
    hipLaunchKernelGGL(k_split_nodeheads<16>, dim3(gsz(Nd)), dim3(256), 0, st, (const float*)N.NH, Nd, T.Ut, T.Vt,
                       T.lam);
  else
    hipLaunchKernelGGL(k_split_nodeheads<8>, dim3(gsz(Nd)), dim3(256), 0, st, (const float*)N.NH, Nd, T.Ut, T.Vt,
                       T.lam);
  if (use_off) {
    hipLaunchKernelGGL(k_layernorm128<AT>, dim3(gsz(No, 16)), dim3(256), 0, st, (const float*)N.Xo, X.wp("offlnf.g"),
                       X.wp("offlnf.b"), (AT*)N.ao128, (int)No);
    gemm<AT>(b, N.ao128, d, N, P.huv, N.bias_uv, nullptr, 0, N.UV, 2 * LS, nullptr, 0, No, 0);
    if (LS == 16)
      hipLaunchKernelGGL(k_split_uv<16>, dim3(gsz(No * LS)), dim3(256), 0, st, (const float*)N.UV, No, T.U, T.V);
    else
      hipLaunchKernelGGL(k_split_uv<8>, dim3(gsz(No * LS)), dim3(256), 0, st, (const float*)N.UV, No, T.U, T.V);
  } else {
    hipLaunchKernelGGL(k_fill, dim3(gsz(mt * LS * LS)), dim3(256), 0, st, T.U, mt * LS * LS, 0.f);
    hipLaunchKernelGGL(k_fill, dim3(gsz(mt * LS * LS)), dim3(256), 0, st, T.V, mt * LS * LS, 0.f);
  }

  // ---- loss (Sec. 3.2) and its adjoint with respect to the factors
  const hp_factor_set fs{N.Frows, T.U, T.V, T.Ut, T.Vt, T.lam};
  const hp_factor_set gs{T.gF, T.gU, T.gV, T.gUt, T.gVt, T.glam};
  HP_TRY(loss_fwd(b, sys, fs, T.X, T.Zs, 1.0 / b.nframes));
  HP_TRY(loss_bwd(b, sys, fs, T.X, T.Zs, gs));

  // ---- heads
  if (LS == 16)
    hipLaunchKernelGGL(k_join_nodeheads<16>, dim3(gsz(Nd)), dim3(256), 0, st, (const float*)N.NH,
                       (const float*)T.gUt, (const float*)T.gVt, (const float*)T.glam, Nd, T.dNH);
  else
    hipLaunchKernelGGL(k_join_nodeheads<8>, dim3(gsz(Nd)), dim3(256), 0, st, (const float*)N.NH, (const float*)T.gUt,
                       (const float*)T.gVt, (const float*)T.glam, Nd, T.dNH);
  const int nh = (int)(2 * LS + 1);
  X.toact(T.dNH, Nd, 64, 64, T.t64b, 64);
  X.dW(N.a128, d, (int)d, T.t64b, 64, nh, Nd, "hut.w", (int)LS, 0, (int)LS, (int)d);
  X.dW(N.a128, d, (int)d, T.t64b, 64, nh, Nd, "hvt.w", (int)LS, (int)LS, (int)LS, (int)d);
  X.dW(N.a128, d, (int)d, T.t64b, 64, nh, Nd, "hlam.w", 1, (int)(2 * LS), 1, (int)d);
  X.dB(T.dNH, 64, nh, Nd, "hut.b", 0, (int)LS);
  X.dB(T.dNH, 64, nh, Nd, "hvt.b", (int)LS, (int)LS);
  X.dB(T.dNH, 64, nh, Nd, "hlam.b", (int)(2 * LS), 1);
  gemm<AT>(b, T.t64b, 64, N, P.b_hnode, nullptr, nullptr, 0, T.da, d, nullptr, 0, Nd, 0);
  const int Lp = (int)((L + 31) / 32 * 32);
  X.toact(T.gF, Nd, (int)L, L, T.t64b, Lp);
  X.dW(N.b128, d, (int)d, T.t64b, Lp, (int)L, Nd, "hleaf2.w", (int)L, 0, (int)L, (int)d);
  X.dB(T.gF, L, (int)L, Nd, "hleaf2.b", 0, (int)L);
  gemm<AT>(b, T.t64b, Lp, N, P.b_hleaf2, nullptr, nullptr, 0, T.dh, d, nullptr, 0, Nd, 0);
  hipLaunchKernelGGL(k_gelu_bwd<AT>, dim3(gsz(Nd * d)), dim3(256), 0, st, (const float*)T.dh, (const float*)T.preh,
                     Nd * d, T.dh, (AT*)T.t128b);
  X.dW(N.a128, d, (int)d, T.t128b, d, (int)d, Nd, "hleaf1.w", (int)d, 0, (int)d, (int)d);
  X.dB(T.dh, d, (int)d, Nd, "hleaf1.b", 0, (int)d);
  gemm<AT>(b, T.t128b, d, N, P.b_hleaf1, nullptr, T.da, d, T.da, d, nullptr, 0, Nd, 0);
  {
    const LnSeg in{{N.H, nullptr, nullptr, nullptr}, {d, 0, 0, 0}, nullptr};
    X.template ln_bwd<128>(in, "diaglnf", T.da, Nd, T.dXd, 0, nullptr, nullptr, nullptr);
  }
  if (use_off) {
    if (LS == 16)
      hipLaunchKernelGGL(k_join_uv<16>, dim3(gsz(No * LS)), dim3(256), 0, st, (const float*)T.gU, (const float*)T.gV,
                         No, T.dUV);
    else
      hipLaunchKernelGGL(k_join_uv<8>, dim3(gsz(No * LS)), dim3(256), 0, st, (const float*)T.gU, (const float*)T.gV,
                         No, T.dUV);
    const int nuv = (int)(2 * LS), Kuv = (nuv + 31) / 32 * 32;
    X.toact(T.dUV, No, nuv, nuv, T.t64b, Kuv);
    X.dW(N.ao128, d, (int)d, T.t64b, Kuv, nuv, No, "hu.w", (int)LS, 0, (int)LS, (int)d);
    X.dW(N.ao128, d, (int)d, T.t64b, Kuv, nuv, No, "hv.w", (int)LS, (int)LS, (int)LS, (int)d);
    X.dB(T.dUV, nuv, nuv, No, "hu.b", 0, (int)LS);
    X.dB(T.dUV, nuv, nuv, No, "hv.b", (int)LS, (int)LS);
    gemm<AT>(b, T.t64b, Kuv, N, P.b_huv, nullptr, nullptr, 0, T.dao, d, nullptr, 0, No, 0);
    const LnSeg in{{N.Xo, nullptr, nullptr, nullptr}, {d, 0, 0, 0}, nullptr};
    X.template ln_bwd<128>(in, "offlnf", T.dao, No, T.dXo, 0, nullptr, nullptr, nullptr);
  }

  // ---- transformer blocks in reverse, each recomputed from its saved input
  const unsigned lowmask = (unsigned)(L - 1);
  const FrameDesc& F0 = b.fr[0];
  for (int l = c.layers - 1; l >= 0; --l) {
    HP_HIP(hipMemcpyAsync(N.H, T.sv.xin_d[l], Nd * d * 4, hipMemcpyDeviceToDevice, st));
    if (use_off) HP_HIP(hipMemcpyAsync(N.Xo, T.sv.xin_o[l], No * d * 4, hipMemcpyDeviceToDevice, st));
    HP_TRY(layer_fwd<AT>(b, W, sys, l, &T.ls));
    // FFN sublayers: X += f2(GELU(f1(LN2([X | r | c | g]))))
    for (int sidx = 0; sidx < 2; ++sidx) {
      if (sidx == 1 && !use_off) continue;
      const std::string p = std::string(sidx ? "off" : "diag") + std::to_string(l) + ".";
      const int64_t M = sidx ? No : Nd;
      float* dXs = sidx ? T.dXo : T.dXd;
      void* u = sidx ? N.uo512 : N.u512;
      void* h = sidx ? N.ho512 : N.h512;
      float* pre = sidx ? T.ls.pre_o : T.ls.pre_d;
      X.toact(dXs, M, (int)d, d, T.t128b, (int)d);
      X.dW(h, 4 * d, (int)(4 * d), T.t128b, d, (int)d, M, p + "f2.w", (int)d, 0, (int)d, (int)(4 * d));
      X.dB(dXs, d, (int)d, M, p + "f2.b", 0, (int)d);
      gemm<AT>(b, T.t128b, d, N, P.b_f2[sidx][l], nullptr, nullptr, 0, T.d512, 4 * d, nullptr, 0, M, 0);
      hipLaunchKernelGGL(k_gelu_bwd<AT>, dim3(gsz(M * 4 * d)), dim3(256), 0, st, (const float*)T.d512,
                         (const float*)pre, M * 4 * d, T.d512, (AT*)T.t512b);
      X.dW(u, 4 * d, (int)(4 * d), T.t512b, 4 * d, (int)(4 * d), M, p + "f1.w", (int)(4 * d), 0, (int)(4 * d),
           (int)(4 * d));
      X.dB(T.d512, 4 * d, (int)(4 * d), M, p + "f1.b", 0, (int)(4 * d));
      gemm<AT>(b, T.t512b, 4 * d, N, P.b_f1[sidx][l], nullptr, nullptr, 0, T.d512, 4 * d, nullptr, 0, M, 0);
      const bool hw = c.highways != 0;
      if (sidx == 0) {
        const LnSeg in{{T.ls.xmid_d, hw ? N.R : nullptr, hw ? N.C : nullptr, hw ? N.G : nullptr},
                       {d, d, d, d}, N.node2f};
        X.template ln_bwd<512>(in, p + "ln2", T.d512, M, T.dXd, 1, T.dR, T.dC, T.dGd);
      } else {
        const LnSeg in{{T.ls.xmid_o, hw ? N.ctxf : nullptr, hw ? N.ctxf + d : nullptr, hw ? N.G : nullptr},
                       {d, 2 * d, 2 * d, d}, N.tok2f};
        X.template ln_bwd<512>(in, p + "ln2", T.d512, M, T.dXo, 1, T.dao, T.dh, T.dGo);
      }
    }
    // highway adjoint (Sec. 4.3): r, c, g are means of the streams
    if (c.highways) {
      hipLaunchKernelGGL(k_chunk_sums, dim3((unsigned)N.nchunks), dim3(512), 0, st, (const SumChunk*)N.chunks,
                         (const float*)T.dGd, (const float*)T.dGo, N.gpart);
      hipLaunchKernelGGL(k_frame_mean, dim3(b.nframes), dim3(1024), 0, st, (const int*)N.chunk0,
                         (const float*)N.gpart, (const float*)T.ones, T.dgf);
      if (use_off) {
        hipLaunchKernelGGL(k_pack_ctx, dim3(gsz(No * d)), dim3(256), 0, st, (const float*)T.dao,
                           (const float*)T.dh, No, T.dctx);
        hipLaunchKernelGGL(k_strip_means_bwd, dim3((unsigned)((Nd + 1) / 2)), dim3(256), 0, st, fr, N.node2f,
                           (const float*)T.dctx, (int)L, (int)LS, Nd, T.dR, T.dC, 1);
      }
      hipLaunchKernelGGL(k_highway_bwd_nodes, dim3((unsigned)((Nd + 1) / 2)), dim3(256), 0, st, fr, N.node2f,
                         (const float*)T.dR, (const float*)T.dC, (const float*)T.dgf, (const float*)N.gcount, (int)L,
                         Nd, (int)use_off, T.WR, T.WC, T.dXd);
      if (use_off)
        hipLaunchKernelGGL(k_highway_bwd_tokens, dim3((unsigned)No), dim3(128), 0, st, fr, N.tile2f,
                           (const float*)T.WR, (const float*)T.WC, (const float*)T.dgf, (const float*)N.gcount,
                           (int)L, (int)LS, T.dXo);
    }
    // attention sublayers: X += MHA(LN1(X)) W_o + b_o
    for (int sidx = 0; sidx < 2; ++sidx) {
      if (sidx == 1 && !use_off) continue;
      const std::string p = std::string(sidx ? "off" : "diag") + std::to_string(l) + ".";
      const int64_t M = sidx ? No : Nd;
      float* dXs = sidx ? T.dXo : T.dXd;
      void* a = sidx ? N.ao128 : N.a128;
      void* q = sidx ? N.qkvo : N.qkv;
      void* o = sidx ? N.bo128 : N.b128;
      X.toact(dXs, M, (int)d, d, T.t128b, (int)d);
      X.dW(o, d, (int)d, T.t128b, d, (int)d, M, p + "o.w", (int)d, 0, (int)d, (int)d);
      X.dB(dXs, d, (int)d, M, p + "o.b", 0, (int)d);
      gemm<AT>(b, T.t128b, d, N, P.b_o[sidx][l], nullptr, nullptr, 0, T.dO, d, nullptr, 0, M, 0);
      if (sidx == 0) {
        if (L == 64)
          hipLaunchKernelGGL((k_attention_bwd<AT, 64, true>), dim3((unsigned)b.ktot, (unsigned)H), dim3(64), 0, st,
                             (const AT*)q, (const float*)T.dO, (const float*)N.T0, (const float*)N.corr,
                             (const uint8_t*)N.nbr, (int)H, T.dqkv, T.dsb, T.dcorr);
        else
          hipLaunchKernelGGL((k_attention_bwd<AT, 32, true>), dim3((unsigned)b.ktot, (unsigned)H), dim3(64), 0, st,
                             (const AT*)q, (const float*)T.dO, (const float*)N.T0, (const float*)N.corr,
                             (const uint8_t*)N.nbr, (int)H, T.dqkv, T.dsb, T.dcorr);
      } else {
        if (LS == 16)
          hipLaunchKernelGGL((k_attention_bwd<AT, 16, false>), dim3((unsigned)b.mtot, (unsigned)H), dim3(64), 0, st,
                             (const AT*)q, (const float*)T.dO, (const float*)N.boff, nullptr, nullptr, (int)H,
                             T.dqkv, T.dsbo, nullptr);
        else
          hipLaunchKernelGGL((k_attention_bwd<AT, 8, false>), dim3((unsigned)b.mtot, (unsigned)H), dim3(64), 0, st,
                             (const AT*)q, (const float*)T.dO, (const float*)N.boff, nullptr, nullptr, (int)H,
                             T.dqkv, T.dsbo, nullptr);
      }
      X.toact(T.dqkv, M, (int)(3 * d), 3 * d, T.t384b, (int)(3 * d));
      X.dW(a, d, (int)d, T.t384b, 3 * d, (int)(3 * d), M, p + "qkv.w", (int)(3 * d), 0, (int)(3 * d), (int)d);
      X.dB(T.dqkv, 3 * d, (int)(3 * d), M, p + "qkv.b", 0, (int)(3 * d));
      gemm<AT>(b, T.t384b, 3 * d, N, P.b_qkv[sidx][l], nullptr, nullptr, 0, T.da, d, nullptr, 0, M, 0);
      const LnSeg in{{sidx ? T.sv.xin_o[l] : T.sv.xin_d[l], nullptr, nullptr, nullptr}, {d, 0, 0, 0}, nullptr};
      X.template ln_bwd<128>(in, p + "ln1", T.da, M, dXs, 1, nullptr, nullptr, nullptr);
      // edge-bias MLPs: the shared within-leaf table, the stencil corrections,
      // the off-diagonal pair descriptors
      if (sidx == 0) {
        hipLaunchKernelGGL(k_reduce_leaves, dim3(gsz(H * L * L)), dim3(256), 0, st, (const float*)T.dsb, b.ktot,
                           (int)(H * L * L), T.dT0);
        EdgeBwdSrc s0{};
        s0.kind = 0;
        s0.npairs = L * L;
        s0.L = (int)L;
        s0.xm = F0.xm & lowmask;
        s0.ym = F0.ym & lowmask;
        s0.zm = F0.zm & lowmask;
        s0.dT0 = T.dT0;
        X.edge_bwd(p, s0);
        EdgeBwdSrc s1{};
        s1.kind = 1;
        s1.npairs = Nd * 7;
        s1.nbr = N.nbr;
        s1.ahat = N.ahat;
        s1.dcorr = T.dcorr;
        X.edge_bwd(p, s1);
      } else {
        EdgeBwdSrc s2{};
        s2.kind = 2;
        s2.npairs = b.mtot * LS * LS;
        s2.desc = N.desc;
        s2.dbias = T.dsbo;
        s2.LS = (int)LS;
        X.edge_bwd(p, s2);
      }
    }
  }

  // ---- pooled off-diagonal tokens: Xo0 = [mean_I h | mean_J h] [W_r; W_c] + b
  if (use_off) {
    X.toact(T.dXo, No, (int)d, d, T.t128b, (int)d);
    X.dW(N.ctx, 2 * d, (int)(2 * d), T.t128b, d, (int)d, No, "pool.wr", (int)d, 0, (int)d, (int)(2 * d));
    X.dB(T.dXo, d, (int)d, No, "pool.b", 0, (int)d);
    gemm<AT>(b, T.t128b, d, N, P.b_pool, nullptr, nullptr, 0, T.dctx, 2 * d, nullptr, 0, No, 0);
    hipLaunchKernelGGL(k_strip_means_bwd, dim3((unsigned)((Nd + 1) / 2)), dim3(256), 0, st, fr, N.node2f,
                       (const float*)T.dctx, (int)L, (int)LS, Nd, T.dXd, T.dXd, 1);
  }

  // ---- encoder: GCN layers H += GELU((D^-1 A) H W + b) in reverse, then the MLP
  for (int g = c.gcn - 1; g >= 0; --g) {
    const std::string p = "gcn" + std::to_string(g);
    hipLaunchKernelGGL(k_gcn_spmm<AT>, dim3((unsigned)((Nd + 7) / 8)), dim3(256), 0, st, fr, N.node2f, sys, b.ntot,
                       (const float*)T.sv.Hg[g], (AT*)N.a128);
    gemm<AT>(b, N.a128, d, N, P.gcn[g], X.wp(p + ".b"), nullptr, 0, nullptr, 0, N.b128, d, Nd, 1, T.preg, d);
    hipLaunchKernelGGL(k_gelu_bwd<AT>, dim3(gsz(Nd * d)), dim3(256), 0, st, (const float*)T.dXd,
                       (const float*)T.preg, Nd * d, T.dh, (AT*)T.t128b);
    X.dW(N.a128, d, (int)d, T.t128b, d, (int)d, Nd, p + ".w", (int)d, 0, (int)d, (int)d);
    X.dB(T.dh, d, (int)d, Nd, p + ".b", 0, (int)d);
    gemm<AT>(b, T.t128b, d, N, P.b_gcn[g], nullptr, nullptr, 0, T.dO, d, nullptr, 0, Nd, 0);
    hipLaunchKernelGGL(k_gcn_spmm_t, dim3((unsigned)((Nd + 1) / 2)), dim3(256), 0, st, fr, N.node2f, sys, b.ntot,
                       (const float*)T.dO, T.dXd, 1);
  }
  gemm<AT>(b, N.feats, 32, N, P.enc1, X.wp("enc1.b"), nullptr, 0, nullptr, 0, N.a128, d, Nd, 1, T.preg, d);
  X.toact(T.dXd, Nd, (int)d, d, T.t128b, (int)d);
  X.dW(N.a128, d, (int)d, T.t128b, d, (int)d, Nd, "enc2.w", (int)d, 0, (int)d, (int)d);
  X.dB(T.dXd, d, (int)d, Nd, "enc2.b", 0, (int)d);
  gemm<AT>(b, T.t128b, d, N, P.b_enc2, nullptr, nullptr, 0, T.dO, d, nullptr, 0, Nd, 0);
  hipLaunchKernelGGL(k_gelu_bwd<AT>, dim3(gsz(Nd * d)), dim3(256), 0, st, (const float*)T.dO, (const float*)T.preg,
                     Nd * d, T.dh, (AT*)T.t128b);
  X.dW(N.feats, 32, 32, T.t128b, d, (int)d, Nd, "enc1.w", (int)d, 0, (int)d, c.node_feats + c.glob_feats);
  X.dB(T.dh, d, (int)d, Nd, "enc1.b", 0, (int)d);
  HP_HIP(hipGetLastError());
  if (h_loss) {
    std::vector<double> lf(b.nframes);
    HP_HIP(hipMemcpyAsync(lf.data(), train_lossf(b), b.nframes * 8, hipMemcpyDeviceToHost, st));
    HP_HIP(hipStreamSynchronize(st));
    double s = 0;
    for (double v : lf) s += v;
    *h_loss = s / b.nframes;
  }
  return HP_OK;
}

}  // namespace hp

extern "C" hp_status hp_train_grad(hp_batch b, const float* d_weights, const float* d_rho, const float* d_sys,
                                   const float* d_zraw, int32_t sweeps, float omega, int32_t compute, float* d_grad,
                                   double* h_loss) {
  using namespace hp;
  if (!b || !d_weights || !d_rho || !d_sys || !d_zraw || !d_grad || sweeps < 0)
    return set_error(HP_E_INVALID, "hp_train_grad: bad arguments");
  HP_TRY(network_train_alloc(*b));
  if (compute == HP_BF16)
    return train_grad_t<uint16_t>(*b, d_weights, d_rho, d_sys, d_zraw, sweeps, omega, d_grad, h_loss);
  if (compute == HP_F32) return train_grad_t<float>(*b, d_weights, d_rho, d_sys, d_zraw, sweeps, omega, d_grad, h_loss);
  return set_error(HP_E_INVALID, "hp_train_grad: compute must be HP_F32 or HP_BF16");
}

extern "C" hp_status hp_adamw_step(hp_batch b, float* d_weights, const float* d_grad, float* d_m, float* d_v,
                                   int64_t n, const hp_adamw_opts* opt, double* h_gnorm) {
  using namespace hp;
  if (!b || !d_weights || !d_grad || !d_m || !d_v || !opt || n <= 0 || opt->step < 1)
    return set_error(HP_E_INVALID, "hp_adamw_step: bad arguments");
  HP_TRY(network_train_alloc(*b));
  NetTrainBufs& T = *ntb_of(*b);
  if (n != T.nw)
    return set_error(HP_E_SHAPE, "hp_adamw_step: n = %lld, the model has %lld weights", (long long)n,
                     (long long)T.nw);
  hipStream_t st = b->stream;
  hipLaunchKernelGGL(k_sumsq_chunks, dim3((unsigned)T.ngn), dim3(256), 0, st, d_grad, n, GN_CHUNK, T.gnpart);
  AdamArgs a{opt->lr, opt->beta1, opt->beta2, opt->eps, opt->weight_decay, opt->clip, opt->step, T.ngn, n};
  const unsigned grid = (unsigned)std::min<int64_t>(1024, (n + 255) / 256);
  hipLaunchKernelGGL(k_adamw, dim3(grid), dim3(256), 0, st, a, (const double*)T.gnpart, d_grad, d_weights, d_m, d_v,
                     T.gnorm);
  HP_HIP(hipGetLastError());
  if (h_gnorm) {
    HP_HIP(hipMemcpyAsync(h_gnorm, T.gnorm, 8, hipMemcpyDeviceToHost, st));
    HP_HIP(hipStreamSynchronize(st));
  }
  return HP_OK;
}

extern "C" hp_status hp_train_step(hp_batch b, float* d_weights, float* d_grad, float* d_m, float* d_v,
                                   const float* d_rho, const float* d_sys, const float* d_zraw, int32_t sweeps,
                                   float omega, int32_t compute, const hp_adamw_opts* opt, double* h_loss,
                                   double* h_gnorm) {
  using namespace hp;
  if (!b || !opt) return set_error(HP_E_INVALID, "hp_train_step: NULL argument");
  HP_TRY(hp_train_grad(b, d_weights, d_rho, d_sys, d_zraw, sweeps, omega, compute, d_grad, nullptr));
  NetTrainBufs& T = *ntb_of(*b);
  HP_TRY(hp_adamw_step(b, d_weights, d_grad, d_m, d_v, T.nw, opt, h_gnorm));
  if (h_loss) {
    std::vector<double> lf(b->nframes);
    HP_HIP(hipMemcpyAsync(lf.data(), train_lossf(*b), b->nframes * 8, hipMemcpyDeviceToHost, b->stream));
    HP_HIP(hipStreamSynchronize(b->stream));
    double s = 0;
    for (double v : lf) s += v;
    *h_loss = s / b->nframes;
  }
  return HP_OK;
}
