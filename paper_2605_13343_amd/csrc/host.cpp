// Host-only parts of the library: errors, Morton order, the H-matrix
// partition and the weight layout.  Pure integer, no device code.
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <numeric>

#include "common.h"

namespace hp {

static thread_local std::string g_err;

hp_status set_error(hp_status code, const char* fmt, ...) {
  char buf[1024];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

static int ilog2_exact(int v) {
  if (v <= 0 || (v & (v - 1))) return -1;
  int l = 0;
  while ((1 << l) < v) ++l;
  return l;
}

// Morton codes of the grid are exactly 0..N-1 iff the interleave x,y,z,x,y,z,...
// fills the low bits without gaps: log2 nx, log2 ny in {lz, lz+1}, ly <= lx.
// A 2D grid (nz = 1) interleaves x,y,x,y,...: ly <= lx <= ly + 1.
bool admissible_grid(int nx, int ny, int nz, std::string* why) {
  int lx = ilog2_exact(nx), ly = ilog2_exact(ny), lz = ilog2_exact(nz);
  if (lx < 0 || ly < 0 || lz < 0) {
    if (why) *why = "grid dims must be powers of two";
    return false;
  }
  if (nz == 1) {
    if (!(ly <= lx && lx <= ly + 1)) {
      if (why) *why = "2D grid dims must satisfy ny <= nx <= 2 ny";
      return false;
    }
    return true;
  }
  if (!(ly <= lx && lx <= lz + 1 && ly >= lz)) {
    if (why) *why = "grid dims must satisfy nz <= ny <= nx <= 2 nz with ny in {nz, 2 nz}";
    return false;
  }
  return true;
}

static uint64_t spread3(uint64_t v) {
  uint64_t r = 0;
  for (int b = 0; b < 21; ++b) r |= ((v >> b) & 1ull) << (3 * b);
  return r;
}

static uint64_t spread2(uint64_t v) {
  uint64_t r = 0;
  for (int b = 0; b < 32; ++b) r |= ((v >> b) & 1ull) << (2 * b);
  return r;
}

// Bits of the Morton rank that hold each coordinate.  Sorting the 3D codes of
// a one-layer grid gives the 2D interleave, so there z has no bits (mask 0:
// every z face is a boundary face).
void morton_masks(int nx, int ny, int nz, unsigned* xm, unsigned* ym, unsigned* zm) {
  if (nz == 1) {
    *xm = (unsigned)spread2((uint64_t)nx - 1);
    *ym = (unsigned)(spread2((uint64_t)ny - 1) << 1);
    *zm = 0u;
    return;
  }
  *xm = (unsigned)spread3((uint64_t)nx - 1);
  *ym = (unsigned)(spread3((uint64_t)ny - 1) << 1);
  *zm = (unsigned)(spread3((uint64_t)nz - 1) << 2);
}

// Box rank of a coordinate: its bits deposited, lowest first, into the bits of mask.
static unsigned deposit_bits(unsigned v, unsigned mask) {
  unsigned r = 0;
  for (unsigned m = mask; m; m &= m - 1u, v >>= 1)
    if (v & 1u) r |= m & (~m + 1u);
  return r;
}

// The frame's cells are the first n cells of the W x H x D grid in Morton
// order.  Box ranks follow the same order, so they are the grid cells whose
// rank lies below that of the grid's (n+1)-th cell (every grid cell when n is
// all of them: then the threshold is the box size).
bool region_threshold(int nx, int ny, int nz, const int32_t* reg, unsigned* thr, std::string* why) {
  const int W = reg[0], H = reg[1], D = reg[2], n = reg[3];
  if (W < 1 || W > nx || H < 1 || H > ny || D < 1 || D > nz) {
    if (why) *why = "the region's grid must fit the box";
    return false;
  }
  const int64_t cells = (int64_t)W * H * D;
  if (n < 1 || n > cells) {
    if (why) *why = "the region's cell count must lie in [1, W H D]";
    return false;
  }
  if (n == cells) {
    *thr = (unsigned)((int64_t)nx * ny * nz);
    return true;
  }
  unsigned xm, ym, zm;
  morton_masks(nx, ny, nz, &xm, &ym, &zm);
  std::vector<unsigned> r;
  r.reserve((size_t)cells);
  for (int z = 0; z < D; ++z)
    for (int y = 0; y < H; ++y)
      for (int x = 0; x < W; ++x) r.push_back(deposit_bits(x, xm) | deposit_bits(y, ym) | deposit_bits(z, zm));
  std::nth_element(r.begin(), r.begin() + n, r.end());
  *thr = r[n];
  return true;
}

// ------------------------------------------------------------------ weights
// Order and shapes of every tensor of the network; see hp_weight_info.
std::vector<WeightEntry> weight_layout(const hp_model_config& c) {
  std::vector<WeightEntry> w;
  int64_t off = 0;
  auto add = [&](const std::string& n, int r, int cc) {
    w.push_back({n, r, cc, off});
    off += (int64_t)r * (cc ? cc : 1);
  };
  auto lin = [&](const std::string& n, int in, int out) {
    add(n + ".w", in, out);
    add(n + ".b", out, 0);
  };
  auto ln = [&](const std::string& n, int width) {
    add(n + ".g", width, 0);
    add(n + ".b", width, 0);
  };
  const int d = c.d, F = c.node_feats + c.glob_feats, E = c.edge_hidden, H = c.heads;
  lin("enc1", F, d);
  lin("enc2", d, d);
  for (int g = 0; g < c.gcn; ++g) lin("gcn" + std::to_string(g), d, d);
  add("pool.wr", d, d);
  add("pool.wc", d, d);
  add("pool.b", d, 0);
  for (const char* st : {"diag", "off"}) {
    for (int l = 0; l < c.layers; ++l) {
      std::string p = std::string(st) + std::to_string(l) + ".";
      ln(p + "ln1", d);
      lin(p + "qkv", d, 3 * d);
      lin(p + "o", d, d);
      lin(p + "e1", 4, E);
      lin(p + "e2", E, H);
      ln(p + "ln2", 4 * d);
      lin(p + "f1", 4 * d, 4 * d);
      lin(p + "f2", 4 * d, d);
    }
    ln(std::string(st) + "lnf", d);
  }
  lin("hleaf1", d, d);
  lin("hleaf2", d, c.leaf);
  lin("hu", d, c.rank);
  lin("hv", d, c.rank);
  lin("hut", d, c.rank);
  lin("hvt", d, c.rank);
  lin("hlam", d, 1);
  return w;
}

const WeightEntry* find_weight(const std::vector<WeightEntry>& w, const std::string& name) {
  for (auto& e : w)
    if (e.name == name) return &e;
  return nullptr;
}

}  // namespace hp

using namespace hp;

extern "C" const char* hp_last_error(void) { return g_err.c_str(); }

extern "C" hp_status hp_morton_order(int32_t nx, int32_t ny, int32_t nz, int32_t* perm) {
  if (nx <= 0 || ny <= 0 || nz <= 0 || !perm) return set_error(HP_E_INVALID, "hp_morton_order: bad arguments");
  int64_t n = (int64_t)nx * ny * nz;
  if (n > (1ll << 30)) return set_error(HP_E_INVALID, "hp_morton_order: grid too large");
  std::vector<uint64_t> code(n);
  for (int z = 0; z < nz; ++z)
    for (int y = 0; y < ny; ++y)
      for (int x = 0; x < nx; ++x)
        code[x + (int64_t)nx * (y + (int64_t)ny * z)] = spread3(x) | (spread3(y) << 1) | (spread3(z) << 2);
  std::vector<int32_t> idx(n);
  std::iota(idx.begin(), idx.end(), 0);
  std::sort(idx.begin(), idx.end(), [&](int32_t a, int32_t b) { return code[a] < code[b]; });
  memcpy(perm, idx.data(), n * sizeof(int32_t));
  return HP_OK;
}

extern "C" hp_status hp_region_mask(int32_t nx, int32_t ny, int32_t nz, const int32_t* region, uint8_t* mask) {
  if (!region || !mask) return set_error(HP_E_INVALID, "hp_region_mask: bad arguments");
  std::string why;
  if (!admissible_grid(nx, ny, nz, &why)) return set_error(HP_E_SHAPE, "hp_region_mask: %s", why.c_str());
  unsigned thr;
  if (!region_threshold(nx, ny, nz, region, &thr, &why)) return set_error(HP_E_SHAPE, "hp_region_mask: %s", why.c_str());
  unsigned xm, ym, zm;
  morton_masks(nx, ny, nz, &xm, &ym, &zm);
  auto coord = [](unsigned c, unsigned m) {
    int v = 0, b = 0;
    for (; m; m &= m - 1u, ++b)
      if (c & m & (~m + 1u)) v |= 1 << b;
    return v;
  };
  const int64_t n = (int64_t)nx * ny * nz;
  for (int64_t c = 0; c < n; ++c) {
    const unsigned u = (unsigned)c;
    mask[c] = (uint8_t)(u < thr && coord(u, xm) < region[0] && coord(u, ym) < region[1] && coord(u, zm) < region[2]);
  }
  return HP_OK;
}

extern "C" hp_status hp_build_partition(int32_t n, int32_t leaf, int32_t rank, hp_partition_info* info,
                                        int32_t* tile_level, int32_t* tile_row0, int32_t* tile_col0,
                                        int32_t* tile_span, int32_t* leaf_tile, int8_t* leaf_side) {
  if (n <= 0 || leaf <= 0 || rank <= 0 || !info) return set_error(HP_E_INVALID, "hp_build_partition: bad arguments");
  if (n % leaf) return set_error(HP_E_SHAPE, "hp_build_partition: N=%d is not a multiple of L=%d", n, leaf);
  if (leaf % rank) return set_error(HP_E_SHAPE, "hp_build_partition: L=%d not a multiple of L_s=%d", leaf, rank);
  int K = n / leaf;
  int J = ilog2_exact(K);
  if (J < 0) return set_error(HP_E_SHAPE, "hp_build_partition: leaf count K=%d is not a power of two", K);
  info->n = n;
  info->leaf = leaf;
  info->rank = rank;
  info->K = K;
  info->J = J;
  info->MH = K - 1;
  info->off_diag = 0;
  info->off_B = (int64_t)K * leaf * leaf;
  info->off_Ut = info->off_B + (int64_t)(K - 1) * rank * rank;
  info->off_Vt = info->off_Ut + (int64_t)n * rank;
  info->off_lam = info->off_Vt + (int64_t)n * rank;
  info->P = info->off_lam + n;
  bool want = tile_level || tile_row0 || tile_col0 || tile_span || leaf_tile || leaf_side;
  if (!want) return HP_OK;
  if (!(tile_level && tile_row0 && tile_col0 && tile_span && leaf_tile && leaf_side))
    return set_error(HP_E_INVALID, "hp_build_partition: pass all output arrays or none");
  for (int j = 0; j < J; ++j) {
    int S = 1 << j;
    for (int i = 0; i < (K >> (j + 1)); ++i) {
      int m = K - (K >> j) + i;
      tile_level[m] = j;
      tile_row0[m] = 2 * i * S;
      tile_col0[m] = 2 * i * S + S;
      tile_span[m] = S;
    }
  }
  for (int k = 0; k < K; ++k)
    for (int j = 0; j < J; ++j) {
      leaf_tile[k * J + j] = K - (K >> j) + (k >> (j + 1));
      leaf_side[k * J + j] = (int8_t)((k >> j) & 1);
    }
  return HP_OK;
}

extern "C" hp_status hp_weight_count(const hp_model_config* cfg, int32_t* count, int64_t* floats) {
  if (!cfg || !count || !floats) return set_error(HP_E_INVALID, "hp_weight_count: NULL argument");
  auto w = weight_layout(*cfg);
  *count = (int32_t)w.size();
  *floats = w.back().offset + (int64_t)w.back().rows * (w.back().cols ? w.back().cols : 1);
  return HP_OK;
}

extern "C" hp_status hp_weight_info(const hp_model_config* cfg, int32_t index, char* name, int32_t* rows,
                                    int32_t* cols, int64_t* offset) {
  if (!cfg || !name || !rows || !cols || !offset) return set_error(HP_E_INVALID, "hp_weight_info: NULL argument");
  auto w = weight_layout(*cfg);
  if (index < 0 || index >= (int)w.size()) return set_error(HP_E_INVALID, "hp_weight_info: index out of range");
  snprintf(name, 64, "%s", w[index].name.c_str());
  *rows = w[index].rows;
  *cols = w[index].cols;
  *offset = w[index].offset;
  return HP_OK;
}
