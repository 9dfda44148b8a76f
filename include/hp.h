/*
 * hp.h -- C ABI of the MI355X (gfx950) library for hierarchical transformer
 * preconditioning of multiphase Poisson systems (Osborne et al., arxiv
 * 2605.13343, "Hierarchical Transformer Preconditioning for Interactive
 * Physics Simulation").
 *
 * Problem statement (paper Sec. 4 "Notation and pipeline", Sec. 5, Sec. 6.1):
 * given a sparse SPD system A x = b whose unknowns are laid out along a
 * space-filling curve, a network reads per-node features and the partition
 * and emits factors of M ~ A^-1 on a weak-admissibility H-matrix partition;
 * PCG then solves A x = b with M.  Training minimises the cosine-Hutchinson
 * probe loss 1 - <Z, M A Z>_F / (||Z||_F ||M A Z||_F).
 *
 * Conventions
 *  - Status codes, never exceptions.  hp_last_error() returns a thread-local
 *    message for the last non-OK status of the calling thread.
 *  - "d_" pointers are device pointers (hipMalloc'd or torch CUDA tensors on
 *    the batch's device); "h_" / plain pointers are host memory.  The caller
 *    owns every buffer it passes and the library never frees them.  A batch
 *    owns only the workspaces it allocates in hp_batch_create.
 *  - Work is enqueued on the batch's stream (the caller's hipStream_t, may be
 *    NULL for the default stream) and calls return after enqueueing, except
 *    where a host output is requested (hp_pcg_solve results, hp_train_step
 *    loss): those synchronise the stream.
 *  - Shape errors are reported before anything is enqueued.
 *
 * Grids and order.  Frame f is a cell-centred nx x ny x nz grid, z vertical,
 * with N = nx ny nz unknowns in Morton order (bit b of x, y, z at bits 3b,
 * 3b+1, 3b+2).  The library requires power-of-two dims whose Morton codes are
 * exactly 0..N-1 (log2 nx, log2 ny in {log2 nz, log2 nz + 1}, nx >= ny), so a
 * cell's Morton code is its row index.  A one-layer grid (nz = 1, the
 * paper's 2D benchmark) interleaves x and y only (bit b of x, y at bits 2b,
 * 2b+1; ny <= nx <= 2 ny); its z faces are all boundary faces, so the 7-point
 * stencil is the 5-point one.  Leaves are the K = N / L contiguous index
 * ranges of length L (paper Sec. 4); K must be a power of two.
 *
 * Batch layout.  The frames of a batch are concatenated: frame f's nodes are
 * rows [n0_f, n0_f + N_f) of every per-node array, its leaves [k0_f, ...),
 * its tiles [m0_f, ...).  hp_batch_info reports all sizes.
 */
#ifndef HP_H
#define HP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t hp_status;
enum {
  HP_OK = 0,
  HP_E_INVALID = 1,  /* bad argument (NULL where required, negative size, ...) */
  HP_E_SHAPE = 2,    /* grid not admissible, N % L != 0, K not a power of two, L % L_s != 0 */
  HP_E_HIP = 3,      /* a HIP runtime call failed; message names it */
  HP_E_NOMEM = 4,    /* device allocation failed in hp_batch_create */
  HP_E_NOT_SPD = 5,  /* solve: M lost positivity and fallback is off */
  HP_E_NOCONV = 6,   /* solve: tolerance not reached and fallback is off */
  HP_E_STATE = 7     /* call out of order (e.g. no weights uploaded) */
};

enum { HP_F32 = 0, HP_BF16 = 1 };                  /* factor / compute precision */
enum { HP_PRECOND_NONE = 0, HP_PRECOND_JACOBI = 1, HP_PRECOND_HMAT = 2 };
enum {                                             /* hp_assemble_ops bits */
  HP_ASM_NEUMANN = 1,         /* zero flux on every face (no Dirichlet top layer) */
  HP_ASM_RHO_CONDUCTANCE = 2  /* face weight: harmonic mean of rho (else of 1/rho) */
};
enum {                                             /* per-frame solve flags */
  HP_CONVERGED = 1, HP_NOT_SPD = 2, HP_STAGNATED = 4, HP_MAXITER = 8, HP_FELL_BACK = 16
};

const char* hp_last_error(void);

/* Network shape (paper Sec. 4, Supplementary "Network Architecture Details").
 * The library supports d = 128, heads in {2, 4, 8}, leaf in {32, 64},
 * rank = leaf / 4, edge_hidden = 32, node_feats = 8, glob_feats = 12. */
typedef struct {
  int32_t d, heads, layers, leaf, rank, edge_hidden, gcn, node_feats, glob_feats;
  int32_t highways; /* 1: row/column/global highway buffers on (Sec. 4.3) */
  int32_t offdiag;  /* 1: off-diagonal stack on (Sec. 4.2) */
} hp_model_config;

/* ------------------------------------------------------------------ host only */

/* Morton order of an nx x ny x nz grid: perm[i] = x + nx (y + ny z) of the
 * i-th cell along the curve (paper Supplementary "Grid and ordering").
 * perm has N entries, host memory.  Any positive dims are accepted. */
hp_status hp_morton_order(int32_t nx, int32_t ny, int32_t nz, int32_t* perm);

/* Padded frames (paper Sec. 8: the partition is sized to a maximum N, and a
 * smaller frame is padded to it; Supplementary "Grid and ordering": the
 * benchmark's W x H grid, close to square with W H >= N, is cut to the first
 * N cells in Morton order).  A frame keeps the power-of-two box nx x ny x nz
 * that hp_batch_create admits, and region = (W, H, D, n) names its own cells:
 * the first n cells, in Morton order, of the W x H x D grid at the box origin
 * (1 <= W <= nx, 1 <= H <= ny, 1 <= D <= nz, 1 <= n <= W H D).  Every other
 * cell of the box is padding.
 * hp_region_mask: mask[c] = 1 if the box's c-th cell in Morton order is one
 * of the frame's cells, else 0; N = nx ny nz entries, host memory.  Host only,
 * bit-exact.  HP_E_SHAPE for a box hp_batch_create rejects or a region that
 * does not fit it. */
hp_status hp_region_mask(int32_t nx, int32_t ny, int32_t nz, const int32_t* region, uint8_t* mask);

typedef struct {
  int32_t n, leaf, rank;   /* N, L, L_s */
  int32_t K, J, MH;        /* leaves, levels (log2 K), unique off-diagonal tiles (K - 1) */
  int64_t P;               /* packed width K L^2 + M_H L_s^2 + 2 N L_s + N (Sec. 4.4) */
  int64_t off_diag, off_B, off_Ut, off_Vt, off_lam;  /* section offsets in elements */
} hp_partition_info;

/* Weak-admissibility partition at eta = 1 (paper Sec. 4, Sec. 4.2 and
 * Supplementary "H-matrix partition"): K = N / L leaves; tile m at level j
 * (S = 2^j leaves per side), index i within the level, m = K - K/2^j + i,
 * rows = leaves [2iS, 2iS+S), columns = leaves [2iS+S, 2iS+2S).  Two-call
 * idiom: with every array NULL only *info is filled.  Otherwise (host memory)
 * tile_* have M_H entries, leaf_tile and leaf_side have K*J entries
 * (leaf-major): leaf k at level j sits in tile leaf_tile[k*J+j] on side
 * leaf_side[k*J+j] (0 row strip, 1 column strip).  Pure integer, bit-exact. */
hp_status hp_build_partition(int32_t n, int32_t leaf, int32_t rank, hp_partition_info* info,
                             int32_t* tile_level, int32_t* tile_row0, int32_t* tile_col0,
                             int32_t* tile_span, int32_t* leaf_tile, int8_t* leaf_side);

/* ------------------------------------------------------------------ batches */

typedef struct hp_batch_s* hp_batch;

typedef struct {
  int32_t nframes;
  int64_t ntot, ktot, mtot;       /* nodes, leaves, tiles over all frames */
  int64_t sys_floats;             /* floats of the assembled-system buffer: 13 * ntot */
  int64_t factor_bytes[2];        /* factor buffer bytes for HP_F32, HP_BF16 */
  int64_t off_G, off_B, off_Ut, off_Vt, off_lam;   /* byte offsets, per dtype below */
  int64_t weight_floats;          /* flat FP32 weight vector length */
} hp_batch_info_t;

/* Create a batch of nframes frames with dims[3f..3f+2] = (nx, ny, nz) (host).
 * All frames share cfg (one leaf size L and rank L_s).  hip_stream is the
 * caller's hipStream_t (borrowed; NULL = default stream).  Allocates the
 * workspaces of the solver calls (assembly, SpMV, apply, PCG; about 130 bytes
 * per node).  The network's workspace (about 12 KB per node) is allocated by
 * the first hp_infer_factors, hp_train_grad or hp_adamw_step call on the batch
 * and kept; later calls allocate nothing. */
hp_status hp_batch_create(const hp_model_config* cfg, int32_t nframes, const int32_t* dims,
                          void* hip_stream, hp_batch* out);
hp_status hp_batch_destroy(hp_batch b);
/* Sets every frame's region (see hp_region_mask): regions[4f .. 4f+3] =
 * (W, H, D, n) for frame f (host), NULL = every frame is its whole box (the
 * state after hp_batch_create).  From the next hp_assemble / hp_assemble_ops
 * on, a padding cell's row of A is the identity row with no faces, a face
 * between a frame cell and padding is a zero-flux boundary face, and the
 * Dirichlet term of hp_assemble sits on the top layer of the frame's grid
 * (z = D-1).  A is then the frame's operator on its own cells, direct-summed
 * with I on the padding; with a right-hand side that is zero on the padding
 * the solution is zero there and the frame's own solution elsewhere.  The
 * network and the solver run on the whole box, padding included (the
 * partition is the box's).  Waits for the batch stream; HP_E_SHAPE (nothing
 * changed) if a region does not fit its frame's box. */
hp_status hp_batch_set_regions(hp_batch b, const int32_t* regions);
/* Sizes; factor offsets are given for dtype (HP_F32 or HP_BF16). */
hp_status hp_batch_info(hp_batch b, int32_t dtype, hp_batch_info_t* info);
/* Per-frame offsets (host arrays of nframes entries, any may be NULL). */
hp_status hp_batch_offsets(hp_batch b, int64_t* n0, int64_t* k0, int64_t* m0);

/* Assemble A for every frame (paper Sec. 7.1 and Supplementary "Operator
 * assembly", in 3D): face weight w_ij = 2 / (rho_i + rho_j) (harmonic mean of
 * 1/rho), A_ij = -w_ij, A_ii = sum_j w_ij, plus 1/rho_i on the top layer
 * (Dirichlet p = 0 one spacing above), zero flux elsewhere.
 *   d_rho [ntot]  FP32 density per node, Morton order.
 *   d_sys [13 ntot floats] output, 8-byte aligned: FP32 [diag | wx | wy | wz |
 *                 1/diag] (5 ntot floats; the SpMV and Jacobi read these) then
 *                 FP64 [diag | wx | wy | wz] (4 ntot doubles; the FP64
 *                 residual replacement reads these).  wx_i is the weight of
 *                 the face between i and its +x neighbour (0 on the +x
 *                 boundary), likewise wy, wz.  Computed in FP64; the FP32
 *                 copies are rounded once. */
hp_status hp_assemble(hp_batch b, const float* d_rho, float* d_sys);

/* hp_assemble with the operator chosen by ops (HP_ASM_* bits; 0 is
 * hp_assemble).  The paper's benchmark operator (Sec. 7.1 "Benchmark",
 * Supplementary "Operator assembly") is HP_ASM_NEUMANN | HP_ASM_RHO_CONDUCTANCE:
 * w_ij = 2 rho_i rho_j / (rho_i + rho_j) and zero flux on every boundary face,
 * so A 1 = 0 and A is singular; PCG needs a right-hand side with zero sum
 * (the paper leaves the constant mode to CG).  Same output layout;
 * HP_E_INVALID for unknown bits. */
hp_status hp_assemble_ops(hp_batch b, const float* d_rho, float* d_sys, int32_t ops);

/* q = A p for every frame (FP32, 7-point stencil in Morton order). */
hp_status hp_spmv(hp_batch b, const float* d_sys, const float* d_p, float* d_q);

/* Packed factors of M, per batch (paper Sec. 4.4 "All factors pack into a
 * single tensor"): byte sections [G: ktot L L][B: mtot Ls Ls][Ut: ntot Ls]
 * [Vt: ntot Ls] in the factor dtype, then [lam: ntot] FP32, each section
 * 256-byte aligned at the offsets hp_batch_info reports.  The buffer itself
 * must be 16-byte aligned (the kernels read it in 16-byte loads); the calls
 * that read it return HP_E_INVALID otherwise.  G_k = F_k F_k^T is
 * stored (the diagonal block of M, Sec. 4.2), B_m = U_m V_m^T.  Within a
 * section frames follow each other, so a one-frame batch holds exactly the
 * paper's per-frame packing [K L^2][M_H L_s^2][N L_s][N L_s][N].
 *
 * M r = blockdiag(G_k) r + diag(lam / A_ii) r + the FMM-style far field of
 * Sec. 5 (restriction u = Ut^T r, v = Vt^T r; strip sums; t^c = B^T s^r,
 * t^r = B s^c; prolongation Ut sum t^r + Vt sum t^c).
 *
 * hp_apply: y = M r for every frame and each of ncols >= 1 right-hand
 * sides.  d_r, d_y: [ncols][ntot] FP32, column-major (column c is
 * d_r[c ntot .. (c+1) ntot)); the two ranges must not overlap.  The columns
 * run one after another through the single-column kernels, so every column
 * equals a one-column call bit for bit.  fdtype HP_F32 or HP_BF16 selects how
 * d_factors is read; accumulation is FP32.  Asynchronous on the batch
 * stream; errors (HP_E_INVALID) before anything is enqueued. */
hp_status hp_apply(hp_batch b, const float* d_sys, const void* d_factors, int32_t fdtype,
                   const float* d_r, float* d_y, int32_t ncols);

/* ------------------------------------------------------------------ without allocation */

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): y = M r as
 * hp_apply computes it, for ONE frame and without an hp_batch.
 *   nx, ny, nz   the frame's grid (the admissible grids of hp_batch_create);
 *   leaf, rank   (64, 16) or (32, 8);
 *   d_sys        the frame's hp_assemble output (13 N floats);
 *   d_factors    the one-frame packing [G K L^2][B M_H L_s^2][Ut N L_s]
 *                [Vt N L_s] in fdtype, then [lam N] FP32, each section
 *                256-byte aligned (the offsets hp_batch_info reports for a
 *                one-frame batch);
 *   d_r, d_y     [ncols][N] FP32, column-major, not overlapping;
 *   hip_stream   a stream of the current device (NULL: its default stream).
 * Results equal hp_apply on a one-frame batch bit for bit (same kernels).
 * Workspace: one fixed 4.5 MiB device array inside the library per device,
 * held until the process ends, which limits N to 2^20 (HP_E_SHAPE beyond).
 * The call allocates nothing (no hipMalloc, hipFree or allocating library
 * routine); its first call on a device looks up that device's array.
 * Every call on a device uses the same array and rewrites it completely
 * before reading it: calls that overlap in time on one device (two streams,
 * or two host threads) race and give wrong results; serialise them.
 * Asynchronous on hip_stream; argument errors are returned before anything
 * is enqueued. */
hp_status hp_apply_static(int32_t nx, int32_t ny, int32_t nz, int32_t leaf, int32_t rank, const float* d_sys,
                          const void* d_factors, int32_t fdtype, const float* d_r, float* d_y, int32_t ncols,
                          void* hip_stream);

typedef struct {
  int32_t precond;          /* HP_PRECOND_* */
  int32_t fdtype;           /* factor dtype for HP_PRECOND_HMAT */
  double tol;               /* stop when ||r|| <= tol ||b|| */
  int32_t max_iter;         /* per frame, counted in SpMVs */
  int32_t recompute_every;  /* r = b - A x in FP64 every this many iterations (0 = never) */
  int32_t fallback;         /* 1: NOT_SPD/STAGNATED/MAXITER frames restart with Jacobi-PCG from x */
  int32_t use_graph;        /* 1: replay a captured hipGraph per chunk of iterations */
  int32_t chunk;            /* iterations per host check (even, >= 2); the first check comes
                               after as many iterations as the batch's previous solve with
                               the same precond needed (multiple of 4, at most 256 and at
                               most max_iter rounded up to even), if more */
  int32_t stagnation;       /* 1: STAGNATED when ||r_k|| > 0.5 ||r_{k-100}|| at k % 100 == 0 */
} hp_solve_opts;

typedef struct {
  int32_t iters;            /* SpMVs of this frame, fallback included */
  int32_t flags;            /* HP_CONVERGED | HP_NOT_SPD | ... */
  double relres;            /* last recurrence ||r|| / ||b|| (FP64) */
} hp_solve_result;

/* PCG on every frame (paper Sec. 3, Sec. 5 "Single-graph capture", Sec. 6.3
 * precision split): x0 = d_x on entry, r = b - A x0, z = M r, p = z; per
 * iteration q = A p, alpha = rho / p.q, x += alpha p, r -= alpha q, residual
 * replacement every recompute_every, stop at ||r|| <= tol ||b||,
 * z = M r, rho' = r.z (flag NOT_SPD unless > 0 and finite), beta = rho'/rho,
 * p = z + beta p.  r, z, p, q are FP32; the solution x accumulates in FP64
 * (an FP32 x cannot hold a 1e-6 true residual on the stiffer frames); inner
 * products, norms, alpha, beta are FP64 (products of FP32 values formed
 * exactly in FP64, summed in a fixed order).  A residual that passes tol
 * stops a frame only if it is a true residual b - A x (FP64, with the FP64
 * coefficients); a passing recurrence residual forces a replacement on the
 * next iteration.  d_b: [ntot] FP32; d_x: [ntot] FP64.  d_factors may be NULL unless precond == HMAT.
 * res (host, nframes entries) receives per-frame results; the call
 * synchronises the stream.  Returns HP_OK even when frames fell back; with
 * fallback off, HP_E_NOT_SPD / HP_E_NOCONV if any frame failed. */
hp_status hp_pcg_solve(hp_batch b, const float* d_sys, const void* d_factors,
                       const hp_solve_opts* opts, const float* d_b, double* d_x,
                       hp_solve_result* res);

/* One step of the method (paper Sec. 5 "Single-graph capture"): network
 * inference into d_factors (as hp_infer_factors with compute), then PCG with
 * the learned preconditioner (as hp_pcg_solve; opts->precond must be
 * HP_PRECOND_HMAT and opts->fdtype equal compute).  With opts->use_graph and
 * an earlier eager hp_infer_factors of this compute type on the batch (which
 * tuned its GEMM tiles), the whole inference, the PCG setup and the first
 * chunk of iterations (as many as the batch's previous solve needed, see
 * hp_solve_opts.chunk) are one captured hipGraph, kept per (buffers, first
 * chunk length, tol, max_iter, recompute_every, stagnation; at most 8) and
 * replayed; a frame still iterating after it continues in chunk graphs, and
 * the fallback runs as in hp_pcg_solve.  Otherwise the two calls run one
 * after the other.  Results equal hp_infer_factors followed by hp_pcg_solve
 * bit for bit.  Synchronises the stream (host results). */
hp_status hp_solve_step(hp_batch b, const float* d_weights, const float* d_rho, const float* d_sys,
                        void* d_factors, int32_t compute, const hp_solve_opts* opts, const float* d_b, double* d_x,
                        hp_solve_result* res);

/* Per-frame latency of the last hp_pcg_solve from device-clock stamps: the
 * lead thread of each frame stamps the clock when the frame stops (its last
 * stop, fallback included), and the library stamps the start of every
 * hp_infer_factors and hp_pcg_solve call.  h_stop_ms [nframes] (host)
 * receives each frame's stop time in ms after the last inference's start
 * when that inference began before the solve (a step of inference plus
 * solve), else after the solve's start; h_solve_start_ms (host, optional)
 * the solve's start on the same scale.  Synchronises the batch stream.
 * HP_E_STATE if no solve has run on the batch. */
hp_status hp_frame_times(hp_batch b, double* h_stop_ms, double* h_solve_start_ms);

/* ------------------------------------------------------------------ network */

/* Weight vector: every tensor of the network in the order hp_weight_info
 * reports, FP32, row-major, linear maps stored [in, out] (y = x W + b). */
hp_status hp_weight_count(const hp_model_config* cfg, int32_t* count, int64_t* floats);
/* name (<= 63 chars + NUL), rank-1 or rank-2 shape, offset in floats. */
hp_status hp_weight_info(const hp_model_config* cfg, int32_t index, char* name, int32_t* rows,
                         int32_t* cols, int64_t* offset);

/* Network forward for every frame (paper Sec. 4.1-4.4): features from
 * (rho, A), encoder MLP + GCN, diagonal and off-diagonal attention stacks
 * with highways, decoder heads, then the packed factors (G = F F^T,
 * B = U V^T, Ut, Vt, lam).  compute = HP_BF16 runs the GEMMs on MFMA in
 * BF16 with FP32 accumulation and writes BF16 factors (lam FP32);
 * HP_F32 runs everything in FP32 and writes FP32 factors.
 *   d_weights [weight_floats] FP32; d_rho [ntot] FP32 (Morton);
 *   d_sys from hp_assemble; d_factors per hp_batch_info(compute).
 * Asynchronous on the batch stream.  Internally an eager call also uses two
 * streams of the batch's own (the edge-bias tables, the off-diagonal stack),
 * forked from and joined back into the batch stream, so later work on the
 * batch stream is ordered after the whole inference; they stay unused under
 * graph capture and live kernel timing.  The first call per compute type
 * tunes the GEMM tiles (it synchronises the device and allocates).  With the "infer_graph"
 * switch of hp_debug_set on (default off), later calls replay an inference
 * captured once per (d_weights, d_rho, d_sys, d_factors) buffer set as a
 * hipGraph (it reads the buffers' contents at each replay; at most 8 such
 * sets are kept), with results equal to the eager path's bit for bit. */
hp_status hp_infer_factors(hp_batch b, const float* d_weights, const float* d_rho,
                           const float* d_sys, void* d_factors, int32_t compute);

/* ------------------------------------------------------------------ training */

/* The paper's factor set of one batch (Sec. 4.4), FP32 device arrays:
 * F [ktot][L][L] leaf factors (diagonal block F_k F_k^T), U, V
 * [mtot][L_s][L_s] tile factors (B_m = U_m V_m^T), Ut, Vt [ntot][L_s] node
 * bridges, lam [ntot] Jacobi gate (M adds diag(lam) diag(A)^-1). */
typedef struct {
  float *F, *U, *V, *Ut, *Vt, *lam;
} hp_factor_set;

/* Allocate the training workspace of the batch (the only allocating call
 * besides hp_batch_create).  kz = probes per system, must be 16. */
hp_status hp_train_init(hp_batch b, int32_t kz);

/* Spectrally biased probes (Sec. 6.2, Eq. 8): z = (I - omega D^-1 A)^sweeps zraw,
 * then x = A z (the loss treats x as fixed input).  zraw, z, x: [ntot][16] FP32,
 * row-major; zraw and z must not alias. */
hp_status hp_probes(hp_batch b, const float* d_sys, const float* d_zraw, float* d_z, float* d_x, int32_t sweeps,
                    float omega);

/* Cosine-Hutchinson loss (Sec. 6.1, Eq. loss) of every frame f:
 * loss_f = 1 - <Z_f, Y_f>_F / (||Z_f||_F ||Y_f||_F) with Y = M X, M from the
 * factor set f.  h_loss [nframes] (host) receives loss_f; the call
 * synchronises.  scale weights the objective scale * sum_f loss_f whose
 * gradient hp_loss_bwd returns (1/nframes gives the batch mean).  Sums of
 * <Z,Y>, ||Z||^2, ||Y||^2 are FP64 in a fixed order. */
hp_status hp_loss_fwd(hp_batch b, const float* d_sys, const hp_factor_set* f, const float* d_x, const float* d_z,
                      double scale, double* h_loss);

/* Gradient of scale * sum_f loss_f with respect to every array of the factor
 * set, written to grad (overwritten, FP32).  Must follow hp_loss_fwd with the
 * same arguments on the same batch (it reuses that call's saved state). */
hp_status hp_loss_bwd(hp_batch b, const float* d_sys, const hp_factor_set* f, const float* d_x, const float* d_z,
                      const hp_factor_set* grad);

/* Gradient of the batch-mean cosine-Hutchinson loss with respect to every
 * network weight (Sec. 6.1-6.3): probes from zraw as hp_probes, the forward
 * pass of hp_infer_factors in the compute type (HP_F32 or HP_BF16; the heads
 * emit an FP32 factor set), the loss, and the reverse pass through heads,
 * transformer blocks (each recomputed from its saved input), pooling and
 * encoder.  d_weights: flat FP32 weights in hp_weight_info order; d_rho,
 * d_sys as for hp_infer_factors; d_zraw [ntot][16] FP32; d_grad (device,
 * caller-owned, overwritten) the FP32 gradient in the weight layout.
 * h_loss (host, optional) receives the batch-mean loss and the call then
 * synchronises.  The first call allocates the training workspace (saved
 * activations of every layer; about 5 KB per node at d = 128).  Reductions
 * over rows use fixed chunking, so the result is bit-reproducible.
 * Errors: HP_E_SHAPE for models with edge_hidden > 32 or heads > 8. */
hp_status hp_train_grad(hp_batch b, const float* d_weights, const float* d_rho, const float* d_sys,
                        const float* d_zraw, int32_t sweeps, float omega, int32_t compute, float* d_grad,
                        double* h_loss);

/* AdamW with decoupled weight decay after a global l2-norm clip (Supplementary
 * "Optimizer and schedule"; PyTorch semantics: clip factor
 * min(1, clip / (||g|| + 1e-6)), bias-corrected moments, step counts from 1).
 * Updates d_weights, d_m, d_v (FP32, n = hp_weight_count total) in place on
 * the batch's stream; h_gnorm (host, optional) receives the pre-clip norm and
 * the call then synchronises.  clip <= 0 disables clipping. */
typedef struct {
  double lr, beta1, beta2, eps, weight_decay, clip;
  int32_t step;
} hp_adamw_opts;
hp_status hp_adamw_step(hp_batch b, float* d_weights, const float* d_grad, float* d_m, float* d_v, int64_t n,
                        const hp_adamw_opts* opt, double* h_gnorm);

/* One training step (Sec. 6.3): hp_train_grad into d_grad (caller-owned
 * scratch of hp_batch_info weight_floats floats, overwritten) followed by
 * hp_adamw_step on d_weights / d_m / d_v.  h_loss and h_gnorm (host,
 * optional) receive the batch-mean loss at the weights before the update and
 * the pre-clip gradient norm; requesting either synchronises the stream. */
hp_status hp_train_step(hp_batch b, float* d_weights, float* d_grad, float* d_m, float* d_v, const float* d_rho,
                        const float* d_sys, const float* d_zraw, int32_t sweeps, float omega, int32_t compute,
                        const hp_adamw_opts* opt, double* h_loss, double* h_gnorm);

/* ------------------------------------------------------------------ diagnostics */

/* Copy `bytes` of a named internal buffer of the last hp_infer_factors call
 * into d_dst (device, caller-owned), on the batch's stream.  Names: "feats"
 * [ntot][32] encoder input (compute type), "glob" [nframes][12] FP32 frame
 * summaries, "enc" [ntot][d] FP32 encoder output, "xo0" [mtot L_s][d] FP32
 * pooled off-diagonal tokens (these two only when the "keep_stages" switch of
 * hp_debug_set was on during the inference), "xd" / "xo" [..][d] FP32 residual streams after
 * the last layer, "desc" [mtot][L_s][L_s][4] FP32 off-diagonal pair
 * descriptors, "frows" [ntot][L] FP32 leaf-head rows (F), "nodeh" [ntot][36]
 * FP32 node heads (Ut | Vt | lam logit), "uv" [mtot L_s][2 L_s] FP32 (U | V).
 * For tests; HP_E_INVALID on an unknown name or a size beyond the buffer. */
hp_status hp_debug_copy(hp_batch b, const char* name, void* d_dst, int64_t bytes);

/* Test switches of one batch.  Every call synchronises the batch stream and
 * drops the batch's captured inference and solve-step graphs (they hold the
 * kernels chosen when they were captured); the next call recaptures.
 * "infer_graph" (0/1, default 0): replay
 * inferences from a captured hipGraph after the first (see
 * hp_infer_factors); "keep_stages" (0/1, default 0): keep the
 * encoder output and the pooled off-diagonal tokens of each inference for
 * hp_debug_copy ("enc", "xo0"; two device copies per inference);
 * "attention_valu" (0/1): with BF16 compute, run
 * the within-leaf attention on the vector ALUs instead of the matrix cores;
 * "sai_loss" (0/1, default 0): train with the SAI-style loss of the paper's
 * loss ablation (Sec. 6.1 Prop. 1(3)) instead of the cosine-Hutchinson loss:
 * per system || A Y / ||A|| - Z ||_F^2 with Y = M Z (the apply then takes Z,
 * and the X argument of hp_loss_fwd / hp_loss_bwd is unused) and ||A|| the
 * largest absolute row sum of A; hp_loss_fwd, hp_loss_bwd, hp_train_grad and
 * hp_train_step follow the switch;
 * "gemm_variant" (-1 or 0..13, default -1): run every BF16 GEMM whose K the
 * variant's K step divides on that tile variant (block tile x K step, "w8":
 * 8 waves, "pf2": loads two K steps ahead; 0: 64x64x32, 1: 128x128x32, 2:
 * 64x64x64, 3: 128x64x64, 4: 128x128x32w8, 5: 256x128x32w8, 6:
 * 128x128x32w8pf2, 7: 256x128x32w8pf2, 8: 64x64x64pf2, 9: 128x128x64w8,
 * 10: 128x256x32w8; "dl", 11-13: K through an LDS ring of 4 or 3 stages
 * filled straight from global memory: 11: dl128x128x32s4, 12:
 * dl256x128x32s3, 13: dl128x256x32s3;
 * other GEMMs on variant 0), -1 lets the autotuner choose (the tests
 * compare the variants); "gemm_small_tiles" (0/1): the same as gemm_variant
 * 0 / -1; "attn_fused" (0/1, default 1): with BF16 compute outside
 * training, L = 64 and 4 heads, run the diagonal stack's attention sublayer
 * (LN1, QKV, the edge-biased leaf attention, the output projection and the
 * residual) as one kernel per leaf, with the same arithmetic per value, so
 * the results equal the separate launches bit for bit; "ffn_fused" (0/1, default 1): with BF16 compute outside training,
 * run each FFN as one fused kernel (hidden activations kept on chip; the
 * same MFMA sequence, GELU and rounding per element, so the results equal
 * the two-GEMM FFN bit for bit) instead of two GEMMs; "gemm_autotune" (0/1, default 1): time every variant on the first
 * call of each BF16 GEMM shape, writing to a scratch buffer, and keep the
 * fastest (off: the 128 x 128 x 32 kernel).  HP_E_INVALID on an unknown name
 * or a variant out of range. */
hp_status hp_debug_set(hp_batch b, const char* name, int32_t value);

/* The GEMM autotuner's records of this batch, one text line per shape
 * ("gemm N=.. K=.. M=.. tile=<chosen> us=<variant>:<us>,..", the fastest of six
 * timed launches of each variant, in three interleaved rounds, in microseconds), written into buf
 * (host, len bytes, always NUL-terminated when len > 0; truncated if short).
 * *entries (optional) receives the number of shapes. */
hp_status hp_autotune_report(hp_batch b, char* buf, int64_t len, int32_t* entries);

/* Live kernel timing for roofline figures.  After hp_profile_enable(b,
 * family), every eager launch of that kernel family on the batch stream is
 * bracketed by HIP events (at most 4096 launches are recorded): "gemm" (the
 * network's GEMMs; work = 2 M N K flops per launch), "gemm_bytes" (the same
 * launches; work = their algorithmic HBM bytes: X, W, the bias and every
 * output and residual operand once; the fused FFN kernels are part of this
 * family), "ffn" / "ffn_bytes" (the fused FFN kernels alone: flops
 * 2 M (512 * 512 + 512 * 128), or U, the weights, the biases and X read and
 * written once), "update" (the PCG
 * x/r/leaf-stage kernel of the learned preconditioner; work = its algorithmic
 * HBM bytes with every frame active: 44 B per node plus G, Ut, Vt per leaf)
 * and "spmv" (the PCG SpMV kernel; 32 B per node).  PCG launches are timed
 * only in solves with use_graph = 0.  "none" turns timing off.
 * hp_profile_read synchronises on the last event and returns the launch
 * count, the summed kernel time in ms and the summed work, then resets the
 * counters. */
hp_status hp_profile_enable(hp_batch b, const char* kernel);
hp_status hp_profile_read(hp_batch b, int32_t* launches, double* total_ms, double* work);

#ifdef __cplusplus
}
#endif
#endif /* HP_H */
