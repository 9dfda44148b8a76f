// The batch object behind hp_batch and the launch interfaces between the
// host driver and the kernel translation units.
#pragma once

#include <algorithm>
#include <array>
#include <map>
#include <set>
#include <tuple>
#include <vector>

#include "common.h"

namespace hp {

struct LaunchGeom {
  const FrameDesc* fr;
  const int* blk2f;
  const int* leaf2f;
  const int2* cblk;  // coarse blocks: (frame, tile), tile -1 for a frame without tiles
  int nframes, nblk, ncblk;
  int64_t ktot, ntot;
  int kmax;
  hipStream_t stream;
};

struct PcgBufs {
  const float* sys;
  int64_t ntot;
  const float* b;
  double *x0, *x1;   // FP64 solution, ping-pong
  float *p0, *p1;
  float *r, *z, *q;
  float *uh, *vh, *Tr, *Tc;
  double *part_pq, *part_rr, *part_rz;
  int* n_active;
  FrameState* st;
  const SolveParams* prm;
  int64_t* ticks;    // device clock: [0] inference start, [1] solve start, [2 + f] frame f's stop
};

// Live kernel timing: every launch of one kernel family is bracketed by HIP
// events on the batch stream (eager launches only, never inside a capture).
enum { PROF_NONE = 0, PROF_GEMM = 1, PROF_UPDATE = 2, PROF_SPMV = 3, PROF_GEMM_BYTES = 4, PROF_FFN = 5,
       PROF_FFN_BYTES = 6 };
struct Prof {
  int kind = PROF_NONE;
  std::vector<hipEvent_t> ev;  // 2 per launch
  int used = 0;
  double work = 0.0;           // algorithmic flops (GEMM) or bytes (others)
};

struct PcgLaunch {
  LaunchGeom g;
  PcgBufs B;
  int mode, L, LS, fdtype;
  const void* fbase;
  const int64_t* offs;
  Prof* prof = nullptr;  // eager launches only (never set while capturing)
};

// Device workspace of the network forward (sized at batch creation).
struct NetWork {
  int64_t tokens_d = 0, tokens_o = 0;  // diagonal and off-diagonal token counts
  float* feats = nullptr;              // [ntot][32] node features, zero padded
  void* ws = nullptr;                  // one arena for every activation buffer
  size_t ws_bytes = 0;
};

// Autotuner record of one GEMM shape: the chosen tile kernel (0: 64 x 64,
// 1: 128 x 128) and the measured average launch time of each.
struct GemmPick {
  int pick = 1;
  std::vector<float> us;  // per variant, -1 where the variant's K step does not divide K
};
int gemm_variant_count();
const char* gemm_variant_name(int v);

struct Batch {
  hp_model_config cfg{};
  Prof prof;
  int nframes = 0;
  std::vector<FrameDesc> fr;
  std::vector<std::array<int, 3>> dims;
  int64_t ntot = 0, ktot = 0, mtot = 0;
  int nblk = 0, kmax = 0, nmax = 0;
  hipStream_t stream = nullptr;
  hipStream_t cap_stream = nullptr;
  // inference side stream: the per-layer edge-bias tables (they depend on the
  // system and the weights only) run there beside the encoder; side_ev[l]
  // marks layer l's tables
  hipStream_t side = nullptr;
  hipEvent_t side_start = nullptr, side_done = nullptr;
  std::vector<hipEvent_t> side_ev;
  // the off-diagonal stack's stream: its attention and FFN sublayers run
  // beside the diagonal ones, joined where the highways couple the stacks
  // (off_ev: [0] prologue done, [1] off stack done, then two per layer)
  hipStream_t offs = nullptr;
  std::vector<hipEvent_t> off_ev;
  FrameDesc* d_fr = nullptr;
  int* d_blk2f = nullptr;
  int* d_leaf2f = nullptr;
  int2* d_cblk = nullptr;
  int ncblk = 0;
  // solver workspace
  double* x1 = nullptr;
  float *p0 = nullptr, *p1 = nullptr, *r = nullptr, *z = nullptr, *q = nullptr;
  float *uh = nullptr, *vh = nullptr, *Tr = nullptr, *Tc = nullptr;
  double *part_pq = nullptr, *part_rr = nullptr, *part_rz = nullptr;
  int* n_active = nullptr;
  int64_t* d_ticks = nullptr;  // [nframes + 2] device clock stamps (PcgBufs::ticks)
  // pinned host staging: [0] active count read back, [1] active count upload,
  // then SolveParams, then nframes FrameState
  char* h_pin = nullptr;
  FrameState* st = nullptr;
  SolveParams* prm = nullptr;
  NetWork net;
  void (*net_free)(void*) = nullptr;  // releases net.ws
  void* train_ws = nullptr;             // training workspace (hp_train_init)
  void (*train_free)(void*) = nullptr;
  int attn_valu = 0;                    // diagnostics: BF16 leaf attention on the vector ALUs
  int gemm_variant = -1;                // diagnostics: BF16 GEMMs forced onto one tile variant (-1: autotuned)
  int ffn_fused = 1;                    // BF16 inference: the FFN as one fused kernel (0: two GEMMs; same results)
  int attn_fused = 1;                   // BF16 inference, L = 64: the diagonal attention sublayer as one kernel (same results)
  int keep_stages = 0;                  // diagnostics: keep the encoder output and pooled tokens for hp_debug_copy
  int gemm_autotune = 1;                // time both tile kernels on a shape's first call
  std::map<std::tuple<int, int, int64_t>, GemmPick> gemm_pick;
  void* net_train = nullptr;            // network training workspace (first hp_train_grad)
  void (*net_train_free)(void*) = nullptr;
  std::map<std::tuple<int, int, const void*, const void*, const void*, const void*, int>, hipGraphExec_t> graphs;
  // inference graphs by (compute, weights, rho, sys, factors, switches); the
  // (compute, switches) pairs that have run eagerly once (GEMM shapes tuned)
  std::map<std::tuple<int, const void*, const void*, const void*, const void*, int>, hipGraphExec_t> infer_graphs;
  std::set<std::pair<int, int>> infer_warm;
  int infer_graph = 0;                  // replay inferences from a captured hipGraph after the first (opt-in)
  int capture_forks = 0;                // set while a solve step is captured: the inference keeps its side streams
  int loss_kind = 0;                    // training objective: 0 cosine-Hutchinson, 1 SAI-style (the loss ablation)
  int last_iters[3] = {0, 0, 0};        // iterations the last solve needed, per preconditioner (first chunk length)
  // captured solve steps (inference + PCG setup + first chunk) by (compute,
  // weights, rho, sys, factors, b, x, first chunk, tol, max_iter,
  // recompute_every, stagnation)
  std::map<std::tuple<int, const void*, const void*, const void*, const void*, const void*, const void*, int, double,
                      int, int, int>,
           hipGraphExec_t>
      step_graphs;
  std::vector<void*> allocs;

  ~Batch();
  hp_status alloc(void** p, size_t bytes);
  LaunchGeom geom() const;
};

void factor_offsets(const Batch& b, int dtype, int64_t offs[5], int64_t* total);
// The same section offsets for explicit sizes (ktot leaves, mtot tiles, ntot nodes).
void factor_offsets_n(int64_t ktot, int64_t mtot, int64_t ntot, int L, int LS, int dtype, int64_t offs[5],
                      int64_t* total);

// solver.hip
hp_status launch_assemble(const LaunchGeom& g, const float* rho, float* sys, int ops);
hp_status launch_spmv(const LaunchGeom& g, const float* sys, const float* p, float* q);
hp_status launch_apply(const LaunchGeom& g, int L, int LS, int fdtype, const float* sys, const void* fac,
                       const int64_t* offs, const float* r, float* y, float* uh, float* vh, float* Tr, float* Tc);
hp_status pcg_setup(const PcgLaunch& P);
// Every frame of the batch active from the standard initial state, the
// active count and the solve parameters, written by a kernel on stream s
// (no host copy, so no wait for earlier work on the stream).
hp_status pcg_init_states(FrameState* st, int nframes, int* n_active, SolveParams* prm, const SolveParams& p,
                          hipStream_t s);
hp_status pcg_iterations(const PcgLaunch& P, int count);
hp_status pcg_finalize(const PcgLaunch& P, bool stopped_only = false);
// One device-clock stamp (wall_clock64) into *p, on stream s.
hp_status launch_tick(int64_t* p, hipStream_t s);

// network.hip
hp_status network_supported(const hp_model_config& c);
// The switches that select an inference's kernels, and whether an inference
// of this compute type may be captured (workspace allocated, GEMM tiles tuned).
int infer_signature(const Batch& B);
bool infer_ready_for_capture(const Batch& B, int compute);
// The network workspace, allocated on the first call that needs it (no-op after).
hp_status network_alloc(Batch& b);

// train.hip
hp_status train_ws_alloc(Batch& b);
hp_status loss_fwd(Batch& b, const float* sys, const hp_factor_set& f, const float* X, const float* Z, double scale);
hp_status loss_bwd(Batch& b, const float* sys, const hp_factor_set& f, const float* X, const float* Z,
                   const hp_factor_set& g);
hp_status probes(Batch& b, const float* sys, const float* zraw, float* z, float* x, int sweeps, float omega);
const double* train_lossf(Batch& b);

}  // namespace hp

struct hp_batch_s : hp::Batch {};
