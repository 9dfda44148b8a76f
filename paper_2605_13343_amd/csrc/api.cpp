// Batch object and the C entry points of the solver path.
#include <string.h>

#include <map>
#include <tuple>

#include "batch.h"

namespace hp {

static int64_t align256(int64_t v) { return (v + 255) & ~(int64_t)255; }

void factor_offsets_n(int64_t ktot, int64_t mtot, int64_t ntot, int L, int LS, int dtype, int64_t offs[5],
                      int64_t* total) {
  const int64_t es = dtype == HP_BF16 ? 2 : 4;
  int64_t o = 0;
  offs[0] = o;
  o = align256(o + ktot * L * L * es);
  offs[1] = o;
  o = align256(o + std::max<int64_t>(mtot, 1) * LS * LS * es);
  offs[2] = o;
  o = align256(o + ntot * LS * es);
  offs[3] = o;
  o = align256(o + ntot * LS * es);
  offs[4] = o;
  o = align256(o + ntot * 4);
  *total = o;
}

void factor_offsets(const Batch& b, int dtype, int64_t offs[5], int64_t* total) {
  factor_offsets_n(b.ktot, b.mtot, b.ntot, b.cfg.leaf, b.cfg.rank, dtype, offs, total);
}

Batch::~Batch() {
  if (side) hipStreamSynchronize(side);
  if (offs) hipStreamSynchronize(offs);
  for (hipEvent_t e : prof.ev) hipEventDestroy(e);
  if (net_free && net.ws) net_free(net.ws);
  if (train_free && train_ws) train_free(train_ws);
  if (net_train_free && net_train) net_train_free(net_train);
  for (auto& kv : graphs) hipGraphExecDestroy(kv.second);
  for (auto& kv : infer_graphs) hipGraphExecDestroy(kv.second);
  for (auto& kv : step_graphs) hipGraphExecDestroy(kv.second);
  for (void* p : allocs) hipFree(p);
  if (h_pin) hipHostFree(h_pin);
  if (cap_stream) hipStreamDestroy(cap_stream);
  for (hipEvent_t e : side_ev) hipEventDestroy(e);
  if (side_start) hipEventDestroy(side_start);
  if (side_done) hipEventDestroy(side_done);
  if (side) hipStreamDestroy(side);
  for (hipEvent_t e : off_ev) hipEventDestroy(e);
  if (offs) hipStreamDestroy(offs);
}

hp_status Batch::alloc(void** p, size_t bytes) {
  hipError_t e = hipMalloc(p, std::max<size_t>(bytes, 256));
  if (e != hipSuccess) return set_error(HP_E_NOMEM, "hipMalloc(%zu) failed: %s", bytes, hipGetErrorString(e));
  allocs.push_back(*p);
  return HP_OK;
}

LaunchGeom Batch::geom() const {
  LaunchGeom g;
  g.fr = d_fr;
  g.blk2f = d_blk2f;
  g.leaf2f = d_leaf2f;
  g.cblk = d_cblk;
  g.ncblk = ncblk;
  g.nframes = nframes;
  g.nblk = nblk;
  g.ktot = ktot;
  g.ntot = ntot;
  g.kmax = kmax;
  g.stream = stream;
  return g;
}

}  // namespace hp

using namespace hp;

static bool supported_cfg(const hp_model_config& c, std::string* why) {
  if (!((c.leaf == 64 && c.rank == 16) || (c.leaf == 32 && c.rank == 8))) {
    *why = "supported (leaf, rank): (64, 16), (32, 8)";
    return false;
  }
  return true;
}

extern "C" hp_status hp_batch_create(const hp_model_config* cfg, int32_t nframes, const int32_t* dims,
                                     void* hip_stream, hp_batch* out) {
  if (!cfg || !dims || !out || nframes <= 0) return set_error(HP_E_INVALID, "hp_batch_create: bad arguments");
  std::string why;
  if (!supported_cfg(*cfg, &why)) return set_error(HP_E_SHAPE, "hp_batch_create: %s", why.c_str());
  HP_TRY(network_supported(*cfg));
  auto* b = new hp_batch_s();
  b->cfg = *cfg;
  b->nframes = nframes;
  b->stream = (hipStream_t)hip_stream;
  const int L = cfg->leaf, LS = cfg->rank;
  int64_t n0 = 0, k0 = 0, m0 = 0;
  int nb0 = 0;
  for (int f = 0; f < nframes; ++f) {
    int nx = dims[3 * f], ny = dims[3 * f + 1], nz = dims[3 * f + 2];
    if (!admissible_grid(nx, ny, nz, &why)) {
      delete b;
      return set_error(HP_E_SHAPE, "hp_batch_create: frame %d (%d x %d x %d): %s", f, nx, ny, nz, why.c_str());
    }
    int n = nx * ny * nz;
    hp_partition_info pi;
    hp_status s = hp_build_partition(n, L, LS, &pi, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr);
    if (s != HP_OK) {
      delete b;
      return s;
    }
    FrameDesc F{};
    F.n = n;
    F.n0 = (int)n0;
    F.K = pi.K;
    F.k0 = (int)k0;
    F.MH = pi.MH;
    F.m0 = (int)m0;
    F.J = pi.J;
    F.nz = nz;
    F.nx = nx;
    F.ny = ny;
    F.rx = nx;
    F.ry = ny;
    F.rz = nz;
    F.rthr = (unsigned)n;
    morton_masks(nx, ny, nz, &F.xm, &F.ym, &F.zm);
    F.nb = (n + NODE_BLOCK - 1) / NODE_BLOCK;
    F.b0 = nb0;
    // the leaf kernels take a leaf's first row as (global leaf) x L
    if ((int64_t)F.n0 != (int64_t)F.k0 * L || (int64_t)F.n != (int64_t)F.K * L) {
      delete b;
      return set_error(HP_E_SHAPE, "hp_batch_create: frame %d is not a whole number of leaves", f);
    }
    b->fr.push_back(F);
    b->dims.push_back({nx, ny, nz});
    n0 += n;
    k0 += pi.K;
    m0 += pi.MH;
    nb0 += F.nb;
    b->kmax = std::max(b->kmax, pi.K);
    b->nmax = std::max(b->nmax, n);
  }
  if (n0 >= (1ll << 31)) {
    delete b;
    return set_error(HP_E_SHAPE, "hp_batch_create: more than 2^31 unknowns");
  }
  b->ntot = n0;
  b->ktot = k0;
  b->mtot = m0;
  b->nblk = nb0;
  std::vector<int> blk2f(nb0), leaf2f(k0);
  std::vector<int2> cblk;
  for (int f = 0; f < nframes; ++f) {
    for (int j = 0; j < b->fr[f].nb; ++j) blk2f[b->fr[f].b0 + j] = f;
    for (int j = 0; j < b->fr[f].K; ++j) leaf2f[b->fr[f].k0 + j] = f;
    if (b->fr[f].MH == 0) cblk.push_back(make_int2(f, -1));
    for (int m = 0; m < b->fr[f].MH; ++m) cblk.push_back(make_int2(f, m));
  }
  b->ncblk = (int)cblk.size();
  hp_status s = HP_OK;
  auto A = [&](void** p, size_t bytes) {
    if (s == HP_OK) s = b->alloc(p, bytes);
  };
  A((void**)&b->d_fr, sizeof(FrameDesc) * nframes);
  A((void**)&b->d_blk2f, sizeof(int) * nb0);
  A((void**)&b->d_leaf2f, sizeof(int) * k0);
  A((void**)&b->d_cblk, sizeof(int2) * cblk.size());
  const size_t nf = sizeof(float) * n0;
  A((void**)&b->x1, 2 * nf);
  A((void**)&b->p0, nf);
  A((void**)&b->p1, nf);
  A((void**)&b->r, nf);
  A((void**)&b->z, nf);
  A((void**)&b->q, nf);
  const size_t kf = sizeof(float) * k0 * LS;
  A((void**)&b->uh, kf);
  A((void**)&b->vh, kf);
  A((void**)&b->Tr, kf);
  A((void**)&b->Tc, kf);
  const size_t np = sizeof(double) * std::max<int64_t>(nb0, k0);
  A((void**)&b->part_pq, np);
  A((void**)&b->part_rr, np);
  A((void**)&b->part_rz, np);
  A((void**)&b->n_active, sizeof(int));
  A((void**)&b->d_ticks, sizeof(int64_t) * (nframes + 2));
  A((void**)&b->st, sizeof(FrameState) * 2 * nframes);
  A((void**)&b->prm, sizeof(SolveParams));
  if (s != HP_OK) {
    delete b;
    return s;
  }
  if (hipHostMalloc((void**)&b->h_pin, 256 + sizeof(FrameState) * 2 * nframes) != hipSuccess) {
    delete b;
    return set_error(HP_E_NOMEM, "hipHostMalloc failed");
  }
  auto cp = [&](void* dst, const void* src, size_t n) {
    if (s == HP_OK && hipMemcpy(dst, src, n, hipMemcpyHostToDevice) != hipSuccess)
      s = set_error(HP_E_HIP, "hp_batch_create: upload failed");
  };
  cp(b->d_fr, b->fr.data(), sizeof(FrameDesc) * nframes);
  cp(b->d_blk2f, blk2f.data(), sizeof(int) * nb0);
  cp(b->d_leaf2f, leaf2f.data(), sizeof(int) * k0);
  cp(b->d_cblk, cblk.data(), sizeof(int2) * cblk.size());
  if (s == HP_OK && hipMemset(b->d_ticks, 0, sizeof(int64_t) * (nframes + 2)) != hipSuccess)
    s = set_error(HP_E_HIP, "hp_batch_create: memset failed");
  if (s != HP_OK) {
    delete b;
    return s;
  }
  *out = b;
  return HP_OK;
}

extern "C" hp_status hp_batch_set_regions(hp_batch b, const int32_t* regions) {
  if (!b) return set_error(HP_E_INVALID, "hp_batch_set_regions: bad arguments");
  std::vector<FrameDesc> fr = b->fr;
  std::string why;
  for (int f = 0; f < b->nframes; ++f) {
    FrameDesc& F = fr[f];
    const int nx = F.nx, ny = F.ny, nz = F.nz;
    const int32_t whole[4] = {nx, ny, nz, F.n};
    const int32_t* reg = regions ? regions + 4 * f : whole;
    unsigned thr;
    if (!region_threshold(nx, ny, nz, reg, &thr, &why))
      return set_error(HP_E_SHAPE, "hp_batch_set_regions: frame %d (%d x %d x %d box): %s", f, nx, ny, nz, why.c_str());
    F.rx = reg[0];
    F.ry = reg[1];
    F.rz = reg[2];
    F.rthr = thr;
    F.padded = !(reg[0] == nx && reg[1] == ny && reg[2] == nz && reg[3] == F.n);
  }
  // the stream's work may still read the descriptors
  if (hipStreamSynchronize(b->stream) != hipSuccess ||
      hipMemcpy(b->d_fr, fr.data(), sizeof(FrameDesc) * b->nframes, hipMemcpyHostToDevice) != hipSuccess)
    return set_error(HP_E_HIP, "hp_batch_set_regions: upload failed");
  b->fr = fr;
  return HP_OK;
}

extern "C" hp_status hp_batch_destroy(hp_batch b) {
  delete b;
  return HP_OK;
}

extern "C" hp_status hp_batch_info(hp_batch b, int32_t dtype, hp_batch_info_t* info) {
  if (!b || !info) return set_error(HP_E_INVALID, "hp_batch_info: NULL argument");
  info->nframes = b->nframes;
  info->ntot = b->ntot;
  info->ktot = b->ktot;
  info->mtot = b->mtot;
  info->sys_floats = 13 * b->ntot;
  int64_t offs[5], tot;
  factor_offsets(*b, HP_F32, offs, &tot);
  info->factor_bytes[0] = tot;
  factor_offsets(*b, HP_BF16, offs, &tot);
  info->factor_bytes[1] = tot;
  factor_offsets(*b, dtype == HP_BF16 ? HP_BF16 : HP_F32, offs, &tot);
  info->off_G = offs[0];
  info->off_B = offs[1];
  info->off_Ut = offs[2];
  info->off_Vt = offs[3];
  info->off_lam = offs[4];
  int32_t cnt;
  int64_t wf;
  hp_weight_count(&b->cfg, &cnt, &wf);
  info->weight_floats = wf;
  return HP_OK;
}

extern "C" hp_status hp_batch_offsets(hp_batch b, int64_t* n0, int64_t* k0, int64_t* m0) {
  if (!b) return set_error(HP_E_INVALID, "hp_batch_offsets: NULL batch");
  for (int f = 0; f < b->nframes; ++f) {
    if (n0) n0[f] = b->fr[f].n0;
    if (k0) k0[f] = b->fr[f].k0;
    if (m0) m0[f] = b->fr[f].m0;
  }
  return HP_OK;
}

extern "C" hp_status hp_assemble(hp_batch b, const float* d_rho, float* d_sys) {
  if (!b || !d_rho || !d_sys) return set_error(HP_E_INVALID, "hp_assemble: NULL argument");
  return launch_assemble(b->geom(), d_rho, d_sys, 0);
}

extern "C" hp_status hp_assemble_ops(hp_batch b, const float* d_rho, float* d_sys, int32_t ops) {
  if (!b || !d_rho || !d_sys) return set_error(HP_E_INVALID, "hp_assemble_ops: NULL argument");
  if (ops & ~(HP_ASM_NEUMANN | HP_ASM_RHO_CONDUCTANCE))
    return set_error(HP_E_INVALID, "hp_assemble_ops: unknown bits in ops=%d", ops);
  return launch_assemble(b->geom(), d_rho, d_sys, ops);
}

extern "C" hp_status hp_spmv(hp_batch b, const float* d_sys, const float* d_p, float* d_q) {
  if (!b || !d_sys || !d_p || !d_q) return set_error(HP_E_INVALID, "hp_spmv: NULL argument");
  return launch_spmv(b->geom(), d_sys, d_p, d_q);
}

// Shared checks of the apply entry points; fills offs for fdtype.
static hp_status apply_args(hp_batch b, const float* d_sys, const void* d_factors, int32_t fdtype, const float* d_r,
                            float* d_y, int32_t ncols, const char* who, int64_t offs[5]) {
  if (!b || !d_sys || !d_factors || !d_r || !d_y) return set_error(HP_E_INVALID, "%s: NULL argument", who);
  if (ncols < 1) return set_error(HP_E_INVALID, "%s: ncols must be >= 1", who);
  if (fdtype != HP_F32 && fdtype != HP_BF16) return set_error(HP_E_INVALID, "%s: bad fdtype", who);
  if ((uintptr_t)d_factors & 15) return set_error(HP_E_INVALID, "%s: factors must be 16-byte aligned", who);
  const uintptr_t r0 = (uintptr_t)d_r, y0 = (uintptr_t)d_y, len = (uintptr_t)(4 * b->ntot * (int64_t)ncols);
  if (r0 < y0 + len && y0 < r0 + len) return set_error(HP_E_INVALID, "%s: r and y must not overlap", who);
  int64_t tot;
  factor_offsets(*b, fdtype, offs, &tot);
  return HP_OK;
}

extern "C" hp_status hp_apply(hp_batch b, const float* d_sys, const void* d_factors, int32_t fdtype,
                              const float* d_r, float* d_y, int32_t ncols) {
  int64_t offs[5];
  HP_TRY(apply_args(b, d_sys, d_factors, fdtype, d_r, d_y, ncols, "hp_apply", offs));
  // column c is r[c ntot .. (c+1) ntot); the columns share the batch's
  // coarse workspace and run one after another on the batch stream
  for (int32_t c = 0; c < ncols; ++c)
    HP_TRY(launch_apply(b->geom(), b->cfg.leaf, b->cfg.rank, fdtype, d_sys, d_factors, offs, d_r + c * b->ntot,
                        d_y + c * b->ntot, b->uh, b->vh, b->Tr, b->Tc));
  return HP_OK;
}

// ------------------------------------------------------------------ PCG driver

// Iterations per host check, and the first chunk's length: as many iterations
// as the batch's previous solve with this preconditioner needed, rounded up to
// a multiple of 4 (even, as every chunk) and kept between one chunk and 256
// iterations (so at most 64 more graph lengths are ever captured): for a
// batch solved again and again, one active-count readback instead of
// several.  Frames stop at their own iteration either way; only trailing
// no-op iterations of stopped frames differ.  It never exceeds max_iter
// (rounded up to even): every frame has stopped by then, so further
// iterations would only be no-ops.
static int chunk_len(const hp_solve_opts& o) { return std::max(2, o.chunk + (o.chunk & 1)); }
static int first_chunk_len(const Batch* b, int mode, const hp_solve_opts& o) {
  const int chunk = chunk_len(o);
  int first = chunk;
  const int64_t prev = std::min<int64_t>(b->last_iters[mode], 256);
  const int64_t cap = std::max<int64_t>(2, (int64_t)o.max_iter + (o.max_iter & 1));
  if (prev > chunk) first = (int)std::min<int64_t>((prev + 3) / 4 * 4, cap);
  return first;
}

// The pinned staging area is rewritten only after the stream has drained
// (every pass ends with a synchronisation), so the async uploads never race.
// With begun, the pass's setup and first chunk are already enqueued (as part
// of a captured step graph, every frame active from the standard state).
static hp_status run_pass(Batch* b, PcgLaunch& P, const hp_solve_opts& o, const std::vector<FrameState>& init,
                          int nact, std::vector<FrameState>& out, bool begun = false) {
  out.clear();
  int* h_active = (int*)b->h_pin;
  int* h_nact = (int*)(b->h_pin + 64);
  SolveParams* h_prm = (SolveParams*)(b->h_pin + 128);
  FrameState* h_st = (FrameState*)(b->h_pin + 256);
  const SolveParams prm{o.tol, o.max_iter, o.recompute_every, o.stagnation, 0};
  // every frame active from the standard state: written on the device, so
  // the host does not wait for the work already on the stream (the inference)
  bool standard = nact == b->nframes;
  for (int f = 0; f < b->nframes && standard; ++f)
    standard = init[f].active == 1 && init[f].done == 0 && init[f].rho == 1.0 && init[f].it == 0 &&
               init[f].flags == 0 && init[f].force_rc == 0 && init[f].fresh == 0 && init[f].alpha == 0.0 &&
               init[f].beta == 0.0 && init[f].rr == 0.0 && init[f].target == 0.0 && init[f].bnorm == 0.0 &&
               init[f].rwin == 0.0;
  if (begun) {
    if (!standard) return set_error(HP_E_STATE, "pcg: a begun pass must start from the standard state");
  } else if (standard) {
    HP_TRY(pcg_init_states(b->st, b->nframes, b->n_active, b->prm, prm, b->stream));
  } else {
    HP_HIP(hipStreamSynchronize(b->stream));  // the pinned staging may still feed an earlier copy
    for (int f = 0; f < b->nframes; ++f) h_st[2 * f] = h_st[2 * f + 1] = init[f];
    *h_nact = nact;
    *h_prm = prm;
    HP_HIP(hipMemcpyAsync(b->st, h_st, sizeof(FrameState) * 2 * b->nframes, hipMemcpyHostToDevice, b->stream));
    HP_HIP(hipMemcpyAsync(b->n_active, h_nact, sizeof(int), hipMemcpyHostToDevice, b->stream));
    HP_HIP(hipMemcpyAsync(b->prm, h_prm, sizeof(SolveParams), hipMemcpyHostToDevice, b->stream));
  }
  if (!begun) HP_TRY(pcg_setup(P));
  const int chunk = chunk_len(o);
  const int first = first_chunk_len(b, P.mode, o);
  // Graphs are keyed by the caller's buffers: a caller that cycles through
  // many buffer sets would grow the cache without bound, so it is emptied
  // once it holds kMaxPcgGraphs executables (every earlier pass has ended
  // with a synchronisation, so none of them is still running).
  constexpr size_t kMaxPcgGraphs = 48;
  if (o.use_graph && b->graphs.size() >= kMaxPcgGraphs) {
    HP_HIP(hipStreamSynchronize(b->stream));
    for (auto& kv : b->graphs) hipGraphExecDestroy(kv.second);
    b->graphs.clear();
  }
  // one captured graph per chunk length
  auto graph_for = [&](int n, hipGraphExec_t* out) -> hp_status {
    auto key = std::make_tuple(P.mode, P.fdtype, (const void*)P.B.sys, P.fbase, (const void*)P.B.b,
                               (const void*)P.B.x0, n);
    auto it = b->graphs.find(key);
    if (it != b->graphs.end()) {
      *out = it->second;
      return HP_OK;
    }
    if (!b->cap_stream) HP_HIP(hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking));
    PcgLaunch C = P;
    C.g.stream = b->cap_stream;
    C.prof = nullptr;
    hipGraph_t graph;
    HP_HIP(hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeThreadLocal));
    hp_status s = pcg_iterations(C, n);
    hipError_t e = hipStreamEndCapture(b->cap_stream, &graph);
    if (s != HP_OK) return s;
    if (e != hipSuccess) return set_error(HP_E_HIP, "hipStreamEndCapture: %s", hipGetErrorString(e));
    hipGraphExec_t exec = nullptr;
    e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    hipGraphDestroy(graph);
    if (e != hipSuccess) return set_error(HP_E_HIP, "hipGraphInstantiate: %s", hipGetErrorString(e));
    b->graphs[key] = exec;
    *out = exec;
    return HP_OK;
  };
  hipGraphExec_t exec = nullptr, exec_first = nullptr;
  if (o.use_graph) {
    HP_TRY(graph_for(chunk, &exec));
    exec_first = exec;
    if (first != chunk && !begun) HP_TRY(graph_for(first, &exec_first));
  }
  const int64_t max_chunks = (int64_t)o.max_iter / chunk + 2;
  for (int64_t c = 0; c < max_chunks; ++c) {
    // the first chunk goes straight after the setup (a frame the setup
    // stopped is skipped by every kernel); later ones after a look at the
    // active count
    if (c == 1 && first > chunk) {
      // a warm first chunk has most likely stopped every frame: the stopped
      // frames' x, the active count and the states come back in one wait
      HP_TRY(pcg_finalize(P, true));
      HP_HIP(hipMemcpyAsync(h_active, b->n_active, sizeof(int), hipMemcpyDeviceToHost, b->stream));
      HP_HIP(hipMemcpyAsync(h_st, b->st, sizeof(FrameState) * 2 * b->nframes, hipMemcpyDeviceToHost, b->stream));
      HP_HIP(hipStreamSynchronize(b->stream));
      if (*h_active <= 0) {
        out.resize(b->nframes);
        for (int f = 0; f < b->nframes; ++f) out[f] = h_st[2 * f];
        return HP_OK;
      }
    } else if (c > 0) {
      HP_HIP(hipMemcpyAsync(h_active, b->n_active, sizeof(int), hipMemcpyDeviceToHost, b->stream));
      HP_HIP(hipStreamSynchronize(b->stream));
      if (*h_active <= 0) break;
    }
    if (c == 0 && begun) continue;  // the first chunk is in the step graph
    if (exec) HP_HIP(hipGraphLaunch(c == 0 ? exec_first : exec, b->stream));
    else HP_TRY(pcg_iterations(P, c == 0 ? first : chunk));
  }
  HP_TRY(pcg_finalize(P));
  return HP_OK;
}

// Final per-frame states (slot 0 of each frame).
static hp_status read_states(Batch* b, std::vector<FrameState>& out) {
  std::vector<FrameState> both(2 * b->nframes);
  HP_HIP(hipMemcpyAsync(both.data(), b->st, sizeof(FrameState) * 2 * b->nframes, hipMemcpyDeviceToHost, b->stream));
  HP_HIP(hipStreamSynchronize(b->stream));
  out.resize(b->nframes);
  for (int f = 0; f < b->nframes; ++f) out[f] = both[2 * f];
  return HP_OK;
}

static hp_status check_solve(hp_batch b, const float* d_sys, const void* d_factors, const hp_solve_opts* opts,
                             const float* d_b, const double* d_x, const hp_solve_result* res, const char* who) {
  if (!b || !d_sys || !opts || !d_b || !d_x || !res) return set_error(HP_E_INVALID, "%s: NULL argument", who);
  const hp_solve_opts& o = *opts;
  if (o.precond < 0 || o.precond > 2) return set_error(HP_E_INVALID, "%s: bad precond", who);
  if (o.precond == HP_PRECOND_HMAT && !d_factors) return set_error(HP_E_INVALID, "%s: factors required for HMAT", who);
  if (o.precond == HP_PRECOND_HMAT && ((uintptr_t)d_factors & 15))
    return set_error(HP_E_INVALID, "%s: factors must be 16-byte aligned", who);
  if (o.precond == HP_PRECOND_HMAT && o.fdtype != HP_F32 && o.fdtype != HP_BF16)
    return set_error(HP_E_INVALID, "%s: bad fdtype", who);
  if (!(o.tol >= 0) || o.max_iter < 0 || o.recompute_every < 0)
    return set_error(HP_E_INVALID, "%s: bad tolerance or limits", who);
  if ((const void*)d_b == (const void*)d_x) return set_error(HP_E_INVALID, "%s: b and x must not alias", who);
  return HP_OK;
}

// The launch description of a solve on the batch's stream (offs: factor
// section offsets, kept alive by the caller).
static PcgLaunch make_launch(Batch* b, const float* d_sys, const void* d_factors, const hp_solve_opts& o,
                             const float* d_b, double* d_x, int64_t offs[5]) {
  int64_t tot;
  factor_offsets(*b, o.precond == HP_PRECOND_HMAT ? o.fdtype : HP_F32, offs, &tot);
  PcgLaunch P;
  P.g = b->geom();
  P.mode = o.precond;
  P.L = b->cfg.leaf;
  P.LS = b->cfg.rank;
  P.fdtype = o.fdtype;
  P.fbase = d_factors;
  P.offs = offs;
  if (!o.use_graph) P.prof = &b->prof;
  PcgBufs& B = P.B;
  B.sys = d_sys;
  B.ntot = b->ntot;
  B.b = d_b;
  B.x0 = d_x;
  B.x1 = b->x1;
  B.p0 = b->p0;
  B.p1 = b->p1;
  B.r = b->r;
  B.z = b->z;
  B.q = b->q;
  B.uh = b->uh;
  B.vh = b->vh;
  B.Tr = b->Tr;
  B.Tc = b->Tc;
  B.part_pq = b->part_pq;
  B.part_rr = b->part_rr;
  B.part_rz = b->part_rz;
  B.n_active = b->n_active;
  B.st = b->st;
  B.prm = b->prm;
  B.ticks = b->d_ticks;
  return P;
}

// Every frame active from the standard initial state.
static std::vector<FrameState> standard_states(int nframes) {
  std::vector<FrameState> init(nframes);
  for (auto& s : init) {
    memset(&s, 0, sizeof s);
    s.rho = 1.0;
    s.active = 1;
  }
  return init;
}

// A solve after its checks: the first pass (begun: its setup and first chunk
// already enqueued), the per-frame results, and the Jacobi-PCG restart of
// every frame that did not converge.
static hp_status solve_body(Batch* b, const hp_solve_opts& o, PcgLaunch& P, hp_solve_result* res, bool begun) {
  std::vector<FrameState> init = standard_states(b->nframes);
  std::vector<FrameState> out;
  HP_TRY(run_pass(b, P, o, init, b->nframes, out, begun));
  if (out.empty()) HP_TRY(read_states(b, out));
  {
    int mx = 0;
    for (int f = 0; f < b->nframes; ++f) mx = std::max(mx, out[f].it);
    b->last_iters[o.precond] = mx;
  }
  bool any_fail = false;
  for (int f = 0; f < b->nframes; ++f) {
    res[f].iters = out[f].it;
    res[f].flags = out[f].flags;
    res[f].relres = out[f].bnorm > 0 ? sqrt(out[f].rr) / out[f].bnorm : 0.0;
    if (!(out[f].flags & HP_CONVERGED)) any_fail = true;
  }
  if (any_fail && o.fallback && o.precond == HP_PRECOND_HMAT) {
    std::vector<FrameState> init2(b->nframes);
    int nact = 0;
    for (int f = 0; f < b->nframes; ++f) {
      memset(&init2[f], 0, sizeof(FrameState));
      init2[f].rho = 1.0;
      bool redo = !(out[f].flags & HP_CONVERGED);
      init2[f].active = redo;
      init2[f].done = !redo;
      nact += redo;
    }
    hp_solve_opts o2 = o;
    o2.precond = HP_PRECOND_JACOBI;
    o2.stagnation = 0;
    PcgLaunch P2 = P;
    P2.mode = HP_PRECOND_JACOBI;
    std::vector<FrameState> out2;
    HP_TRY(run_pass(b, P2, o2, init2, nact, out2));
    if (out2.empty()) HP_TRY(read_states(b, out2));
    any_fail = false;
    for (int f = 0; f < b->nframes; ++f) {
      if (!init2[f].active) continue;
      res[f].iters += out2[f].it;
      res[f].flags |= out2[f].flags | HP_FELL_BACK;
      res[f].relres = out2[f].bnorm > 0 ? sqrt(out2[f].rr) / out2[f].bnorm : 0.0;
      if (!(out2[f].flags & HP_CONVERGED)) any_fail = true;
    }
  }
  if (any_fail && !o.fallback) {
    for (int f = 0; f < b->nframes; ++f)
      if (res[f].flags & HP_NOT_SPD) return set_error(HP_E_NOT_SPD, "hp_pcg_solve: frame %d lost positivity", f);
    return set_error(HP_E_NOCONV, "hp_pcg_solve: tolerance not reached");
  }
  return HP_OK;
}

extern "C" hp_status hp_pcg_solve(hp_batch b, const float* d_sys, const void* d_factors, const hp_solve_opts* opts,
                                  const float* d_b, double* d_x, hp_solve_result* res) {
  HP_TRY(check_solve(b, d_sys, d_factors, opts, d_b, d_x, res, "hp_pcg_solve"));
  const hp_solve_opts o = *opts;
  int64_t offs[5];
  PcgLaunch P = make_launch(b, d_sys, d_factors, o, d_b, d_x, offs);
  HP_TRY(launch_tick(b->d_ticks + 1, b->stream));
  return solve_body(b, o, P, res, false);
}

// One step of the method: inference, then PCG with the learned preconditioner.
// With use_graph (and the inference's GEMM tiles already tuned by an earlier
// eager inference of this compute type), the inference, the PCG setup and the
// first chunk of iterations are one captured hipGraph, kept per buffer set and
// first-chunk length; the rest of the solve (further chunks when a frame is
// still iterating, the fallback) follows as in hp_pcg_solve.
extern "C" hp_status hp_solve_step(hp_batch b, const float* d_weights, const float* d_rho, const float* d_sys,
                                   void* d_factors, int32_t compute, const hp_solve_opts* opts, const float* d_b,
                                   double* d_x, hp_solve_result* res) {
  HP_TRY(check_solve(b, d_sys, d_factors, opts, d_b, d_x, res, "hp_solve_step"));
  if (!d_weights || !d_rho) return set_error(HP_E_INVALID, "hp_solve_step: NULL argument");
  if (opts->precond != HP_PRECOND_HMAT || opts->fdtype != compute)
    return set_error(HP_E_INVALID, "hp_solve_step: precond must be HMAT with fdtype equal to the compute type");
  const hp_solve_opts o = *opts;
  const bool graph = o.use_graph && b->prof.kind == PROF_NONE && infer_ready_for_capture(*b, compute);
  int64_t offs[5];
  PcgLaunch P = make_launch(b, d_sys, d_factors, o, d_b, d_x, offs);
  if (!graph) {
    HP_TRY(hp_infer_factors(b, d_weights, d_rho, d_sys, d_factors, compute));
    HP_TRY(launch_tick(b->d_ticks + 1, b->stream));
    return solve_body(b, o, P, res, false);
  }
  const int first = first_chunk_len(b, HP_PRECOND_HMAT, o);
  const auto key = std::make_tuple((int)compute, (const void*)d_weights, (const void*)d_rho, (const void*)d_sys,
                                   (const void*)d_factors, (const void*)d_b, (const void*)d_x, first, o.tol, o.max_iter,
                                   o.recompute_every, o.stagnation);
  auto it = b->step_graphs.find(key);
  hipGraphExec_t exec = nullptr;
  if (it != b->step_graphs.end()) {
    exec = it->second;
  } else {
    if (b->step_graphs.size() >= 8) {  // callers cycling through buffers: keep the cache small
      HP_HIP(hipStreamSynchronize(b->stream));
      for (auto& kv : b->step_graphs) hipGraphExecDestroy(kv.second);
      b->step_graphs.clear();
    }
    if (!b->cap_stream) HP_HIP(hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking));
    const SolveParams prm{o.tol, o.max_iter, o.recompute_every, o.stagnation, 0};
    std::swap(b->stream, b->cap_stream);  // every launch below goes to the capturing stream
    PcgLaunch C = P;
    C.g.stream = b->stream;
    C.prof = nullptr;
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal);
    hp_status s = e == hipSuccess ? HP_OK : set_error(HP_E_HIP, "hipStreamBeginCapture: %s", hipGetErrorString(e));
    b->capture_forks = 1;
    if (s == HP_OK) s = hp_infer_factors(b, d_weights, d_rho, d_sys, d_factors, compute);
    b->capture_forks = 0;
    if (s == HP_OK) s = launch_tick(b->d_ticks + 1, b->stream);
    if (s == HP_OK) s = pcg_init_states(b->st, b->nframes, b->n_active, b->prm, prm, b->stream);
    if (s == HP_OK) s = pcg_setup(C);
    if (s == HP_OK) s = pcg_iterations(C, first);
    if (e == hipSuccess) e = hipStreamEndCapture(b->stream, &g);
    std::swap(b->stream, b->cap_stream);
    if (s != HP_OK) {
      if (g) hipGraphDestroy(g);
      return s;
    }
    if (e != hipSuccess) return set_error(HP_E_HIP, "step capture: %s", hipGetErrorString(e));
    e = hipGraphInstantiate(&exec, g, nullptr, nullptr, 0);
    hipGraphDestroy(g);
    if (e != hipSuccess) return set_error(HP_E_HIP, "hipGraphInstantiate: %s", hipGetErrorString(e));
    b->step_graphs[key] = exec;
  }
  HP_HIP(hipGraphLaunch(exec, b->stream));
  return solve_body(b, o, P, res, true);
}

extern "C" hp_status hp_frame_times(hp_batch b, double* h_stop_ms, double* h_solve_start_ms) {
  if (!b || !h_stop_ms) return set_error(HP_E_INVALID, "hp_frame_times: NULL argument");
  std::vector<int64_t> t(b->nframes + 2);
  HP_HIP(hipMemcpyAsync(t.data(), b->d_ticks, sizeof(int64_t) * t.size(), hipMemcpyDeviceToHost, b->stream));
  HP_HIP(hipStreamSynchronize(b->stream));
  if (t[1] == 0) return set_error(HP_E_STATE, "hp_frame_times: no solve has run on this batch");
  int dev = 0, khz = 0;
  HP_HIP(hipGetDevice(&dev));
  HP_HIP(hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev));
  if (khz <= 0) return set_error(HP_E_HIP, "hp_frame_times: device clock rate unknown");
  // the reference is the last inference's start if it began before the last
  // solve (an inference-plus-solve step), else the solve's start
  const int64_t ref = (t[0] != 0 && t[0] <= t[1]) ? t[0] : t[1];
  const double ms_per_tick = 1.0 / (double)khz;
  for (int f = 0; f < b->nframes; ++f) h_stop_ms[f] = (double)(t[2 + f] - ref) * ms_per_tick;
  if (h_solve_start_ms) *h_solve_start_ms = (double)(t[1] - ref) * ms_per_tick;
  return HP_OK;
}

extern "C" hp_status hp_debug_set(hp_batch b, const char* name, int32_t value) {
  if (!b || !name) return set_error(HP_E_INVALID, "hp_debug_set: NULL argument");
  const std::string n = name;
  // captured inference and solve-step graphs hold the kernels the switches
  // chose when they were captured: drop them, so the next call recaptures
  if (!b->infer_graphs.empty() || !b->step_graphs.empty()) {
    HP_HIP(hipStreamSynchronize(b->stream));
    for (auto& kv : b->infer_graphs) hipGraphExecDestroy(kv.second);
    for (auto& kv : b->step_graphs) hipGraphExecDestroy(kv.second);
    b->infer_graphs.clear();
    b->step_graphs.clear();
  }
  if (n == "attention_valu") {
    b->attn_valu = value != 0;
    return HP_OK;
  }
  if (n == "infer_graph") {
    b->infer_graph = value != 0;
    return HP_OK;
  }
  if (n == "keep_stages") {
    b->keep_stages = value != 0;
    return HP_OK;
  }
  if (n == "attn_fused") {
    b->attn_fused = value != 0;
    return HP_OK;
  }
  if (n == "ffn_fused") {
    b->ffn_fused = value != 0;
    return HP_OK;
  }
  if (n == "gemm_small_tiles") {
    b->gemm_variant = value != 0 ? 0 : -1;
    return HP_OK;
  }
  if (n == "gemm_variant") {
    if (value < -1 || value >= gemm_variant_count())
      return set_error(HP_E_INVALID, "hp_debug_set: gemm_variant %d outside [-1, %d)", (int)value,
                       gemm_variant_count());
    b->gemm_variant = value;
    return HP_OK;
  }
  if (n == "sai_loss") {
    b->loss_kind = value != 0;
    return HP_OK;
  }
  if (n == "gemm_autotune") {
    b->gemm_autotune = value != 0;
    return HP_OK;
  }
  return set_error(HP_E_INVALID, "hp_debug_set: unknown option '%s'", name);
}

extern "C" hp_status hp_autotune_report(hp_batch b, char* buf, int64_t len, int32_t* entries) {
  if (!b || (!buf && len > 0) || len < 0) return set_error(HP_E_INVALID, "hp_autotune_report: bad arguments");
  std::string out;
  char line[160];
  for (const auto& kv : b->gemm_pick) {
    snprintf(line, sizeof line, "gemm N=%d K=%d M=%lld tile=%s us=", std::get<0>(kv.first), std::get<1>(kv.first),
             (long long)std::get<2>(kv.first), gemm_variant_name(kv.second.pick));
    out += line;
    for (size_t v = 0; v < kv.second.us.size(); ++v) {
      if (kv.second.us[v] < 0.f) continue;
      snprintf(line, sizeof line, "%s%s:%.2f", out.back() == '=' ? "" : ",", gemm_variant_name((int)v),
               kv.second.us[v]);
      out += line;
    }
    out += "\n";
  }
  if (entries) *entries = (int32_t)b->gemm_pick.size();
  if (len > 0) {
    const size_t n = std::min<size_t>(out.size(), (size_t)len - 1);
    memcpy(buf, out.data(), n);
    buf[n] = 0;
  }
  return HP_OK;
}

extern "C" hp_status hp_profile_enable(hp_batch b, const char* kernel) {
  if (!b || !kernel) return set_error(HP_E_INVALID, "hp_profile_enable: NULL argument");
  const std::string k = kernel;
  int kind = k == "gemm"         ? PROF_GEMM
             : k == "gemm_bytes" ? PROF_GEMM_BYTES
             : k == "update"     ? PROF_UPDATE
             : k == "spmv"       ? PROF_SPMV
             : k == "ffn"        ? PROF_FFN
             : k == "ffn_bytes"  ? PROF_FFN_BYTES
             : k == "none"       ? PROF_NONE
                                 : -1;
  if (kind < 0) return set_error(HP_E_INVALID, "hp_profile_enable: unknown kernel family '%s'", kernel);
  if (kind != PROF_NONE && b->prof.ev.empty()) {
    b->prof.ev.resize(2 * 4096);
    for (auto& e : b->prof.ev) HP_HIP(hipEventCreate(&e));
  }
  b->prof.kind = kind;
  b->prof.used = 0;
  b->prof.work = 0.0;
  return HP_OK;
}

extern "C" hp_status hp_profile_read(hp_batch b, int32_t* launches, double* total_ms, double* work) {
  if (!b || !launches || !total_ms || !work) return set_error(HP_E_INVALID, "hp_profile_read: NULL argument");
  double ms = 0.0;
  if (b->prof.used > 0) HP_HIP(hipEventSynchronize(b->prof.ev[2 * b->prof.used - 1]));
  for (int i = 0; i < b->prof.used; ++i) {
    float t = 0.f;
    HP_HIP(hipEventElapsedTime(&t, b->prof.ev[2 * i], b->prof.ev[2 * i + 1]));
    ms += t;
  }
  *launches = b->prof.used;
  *total_ms = ms;
  *work = b->prof.work;
  b->prof.used = 0;
  b->prof.work = 0.0;
  return HP_OK;
}
