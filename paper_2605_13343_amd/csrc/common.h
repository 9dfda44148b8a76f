// Internal definitions shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/hp.h"

namespace hp {

// ---------------------------------------------------------------- errors
hp_status set_error(hp_status code, const char* fmt, ...);

#define HP_HIP(call)                                                                  \
  do {                                                                                \
    hipError_t e_ = (call);                                                           \
    if (e_ != hipSuccess)                                                             \
      return ::hp::set_error(HP_E_HIP, "%s failed: %s (%s:%d)", #call,                \
                             hipGetErrorString(e_), __FILE__, __LINE__);              \
  } while (0)

#define HP_TRY(expr)                 \
  do {                               \
    hp_status s_ = (expr);           \
    if (s_ != HP_OK) return s_;      \
  } while (0)

// ---------------------------------------------------------------- frames
// One frame of a batch as the kernels see it.  Morton code == local row.
struct FrameDesc {
  int n, n0;        // unknowns, first row in the batch
  int K, k0;        // leaves, first leaf
  int MH, m0;       // tiles, first tile
  int J;            // levels = log2 K
  int nz;           // grid height (top layer z = nz-1)
  unsigned xm, ym, zm;  // Morton bit masks of x, y, z within the code
  int nb, b0;       // node blocks (of NODE_BLOCK rows) and first node block
  int nx, ny;       // grid width and depth
  // The frame's own cells when its grid is smaller than the box (padded):
  // cell c belongs to the frame iff its coordinates lie in rx x ry x rz and
  // c < rthr; every other cell of the box is padding (an identity row).
  int rx, ry, rz, padded;
  unsigned rthr;
};

constexpr int NODE_BLOCK = 128;   // rows per node block
constexpr int LEAF_THREADS = 128; // threads per leaf block

// Per-frame PCG scalars (device), double-buffered by iteration parity.
struct FrameState {
  double rho;     // r.z of the current residual
  double alpha;   // last step length (record)
  double beta;    // last rho'/rho (record)
  double rr;      // ||r||^2 at the last check
  double target;  // (tol ||b||)^2
  double bnorm;   // ||b||
  double rwin;    // ||r|| at the last stagnation checkpoint
  int it;         // updates done and checked
  int flags;      // HP_* flags
  int done;       // 1: frame stopped (converged or failed)
  int active;     // 1: frame takes part in this solve
  int force_rc;   // 1: next update replaces r by b - A x (confirmation)
  int fresh;      // 1: set up, no update yet
};

// Field-wise copies of a frame state between global memory and registers.
// (A whole-struct copy keeps the kernel's local copy in memory, which the
// compiler then places per thread in LDS; field by field it stays in
// registers.)
__device__ inline FrameState load_state(const FrameState* p) {
  FrameState s;
  s.rho = p->rho;
  s.alpha = p->alpha;
  s.beta = p->beta;
  s.rr = p->rr;
  s.target = p->target;
  s.bnorm = p->bnorm;
  s.rwin = p->rwin;
  s.it = p->it;
  s.flags = p->flags;
  s.done = p->done;
  s.active = p->active;
  s.force_rc = p->force_rc;
  s.fresh = p->fresh;
  return s;
}

__device__ inline void store_state(FrameState* p, const FrameState& s) {
  p->rho = s.rho;
  p->alpha = s.alpha;
  p->beta = s.beta;
  p->rr = s.rr;
  p->target = s.target;
  p->bnorm = s.bnorm;
  p->rwin = s.rwin;
  p->it = s.it;
  p->flags = s.flags;
  p->done = s.done;
  p->active = s.active;
  p->force_rc = s.force_rc;
  p->fresh = s.fresh;
}

struct SolveParams {
  double tol;
  int max_iter, recompute_every, stagnation, pad;
};

// ---------------------------------------------------------------- bf16
__host__ __device__ inline float bf16_to_f32(uint16_t h) {
  union { uint32_t u; float f; } c;
  c.u = (uint32_t)h << 16;
  return c.f;
}
__host__ __device__ inline uint16_t f32_to_bf16(float f) {  // round to nearest even
  union { uint32_t u; float f; } c;
  c.f = f;
  if ((c.u & 0x7f800000u) == 0x7f800000u && (c.u & 0x007fffffu)) return 0x7fc0;  // NaN
  c.u += 0x7fffu + ((c.u >> 16) & 1u);
  return (uint16_t)(c.u >> 16);
}

// Block index remapped so that each of the 8 XCDs (the dispatcher deals the
// blocks of a launch out to them round-robin) runs one contiguous range of
// the logical blocks: the neighbouring rows a stencil reads then sit in the
// same L2.  A bijection of [0, n) for any n.
__device__ inline int xcd_block(int id, int n) {
  const int q = n >> 3, r = n & 7, x = id & 7, k = id >> 3;
  return x * q + min(x, r) + k;
}

// Cross-lane sums on the VALU's data-parallel-primitive (DPP) lane paths
// instead of LDS permutes.  row16_sum: the sum over each aligned group of 16
// lanes, with the same bits in every lane of the group (partners by quad
// permutations, then the half-row and row mirrors).  wave_total: the sum over
// all 64 lanes (row broadcasts fold the four rows into lane 63), returned as
// a wave-uniform value.  Every lane of the wave must be active.
template <int CTRL>
__device__ inline float dpp_move(float v) {
  return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, v), CTRL, 0xF, 0xF, false));
}
// sum over each aligned group of W lanes (W = 1, 2, 4, 8 or 16)
template <int W>
__device__ inline float group_sum(float v) {
  static_assert(W == 1 || W == 2 || W == 4 || W == 8 || W == 16, "DPP groups are 1 to 16 lanes");
  if constexpr (W >= 2) v += dpp_move<0xB1>(v);   // quad_perm [1, 0, 3, 2]
  if constexpr (W >= 4) v += dpp_move<0x4E>(v);   // quad_perm [2, 3, 0, 1]
  if constexpr (W >= 8) v += dpp_move<0x141>(v);  // row_half_mirror
  if constexpr (W >= 16) v += dpp_move<0x140>(v); // row_mirror
  return v;
}
__device__ inline float row16_sum(float v) { return group_sum<16>(v); }
__device__ inline float wave_total(float v) {
  v = row16_sum(v);
  // row_bcast:15 into rows 1 and 3, then row_bcast:31 into rows 2 and 3
  v += __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0x142, 0xA, 0xF, false));
  v += __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0x143, 0xC, 0xF, false));
  return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), 63));
}

// The same for FP64 (each move takes the two 32-bit halves); rows outside
// ROWS receive zero in the broadcast steps.
template <int CTRL, int ROWS = 0xF>
__device__ inline double dpp_move_d(double v) {
  const unsigned long long u = __builtin_bit_cast(unsigned long long, v);
  const unsigned lo = (unsigned)__builtin_amdgcn_update_dpp(0, (int)(unsigned)u, CTRL, ROWS, 0xF, false);
  const unsigned hi = (unsigned)__builtin_amdgcn_update_dpp(0, (int)(unsigned)(u >> 32), CTRL, ROWS, 0xF, false);
  return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}
__device__ inline double wave_total_d(double v) {
  v += dpp_move_d<0xB1>(v);
  v += dpp_move_d<0x4E>(v);
  v += dpp_move_d<0x141>(v);
  v += dpp_move_d<0x140>(v);
  v += dpp_move_d<0x142, 0xA>(v);
  v += dpp_move_d<0x143, 0xC>(v);
  const unsigned long long u = __builtin_bit_cast(unsigned long long, v);
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)u, 63);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(u >> 32), 63);
  return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}

template <typename T> __device__ inline float ldf(const T* p, int64_t i);
template <> __device__ inline float ldf<float>(const float* p, int64_t i) { return p[i]; }
template <> __device__ inline float ldf<uint16_t>(const uint16_t* p, int64_t i) { return bf16_to_f32(p[i]); }

// ---------------------------------------------------------------- Morton neighbours
// Neighbour of code c one step along the axis whose bits are mask; the
// boundary wraps to the far side, where the face weight is zero.
__device__ inline unsigned mstep_plus(unsigned c, unsigned mask) {
  return (((c | ~mask) + 1u) & mask) | (c & ~mask);
}
__device__ inline unsigned mstep_minus(unsigned c, unsigned mask) {
  return (((c & mask) - 1u) & mask) | (c & ~mask);
}
// Whether cell c (box rank) is one of the frame's own cells (see FrameDesc).
__device__ inline int mcoord(unsigned c, unsigned mask);
__device__ inline bool in_region(const FrameDesc& F, unsigned c) {
  return c < F.rthr && mcoord(c, F.xm) < F.rx && mcoord(c, F.ym) < F.ry && mcoord(c, F.zm) < F.rz;
}
__device__ inline int mcoord(unsigned c, unsigned mask) {
  int v = 0, b = 0;
  while (mask) {
    unsigned low = mask & (~mask + 1u);
    if (c & low) v |= 1 << b;
    ++b;
    mask &= mask - 1u;
  }
  return v;
}

// ---------------------------------------------------------------- host helpers
bool admissible_grid(int nx, int ny, int nz, std::string* why);
void morton_masks(int nx, int ny, int nz, unsigned* xm, unsigned* ym, unsigned* zm);
// Region (W, H, D, n) of a frame inside its nx x ny x nz box: checks it and
// returns the rank threshold of FrameDesc::rthr.
bool region_threshold(int nx, int ny, int nz, const int32_t* reg, unsigned* thr, std::string* why);

struct WeightEntry {
  std::string name;
  int rows, cols;   // cols == 0 for rank-1
  int64_t offset;
};
std::vector<WeightEntry> weight_layout(const hp_model_config& c);
const WeightEntry* find_weight(const std::vector<WeightEntry>& w, const std::string& name);

}  // namespace hp
