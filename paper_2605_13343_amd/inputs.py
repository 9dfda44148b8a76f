"""Seeded synthetic inputs shared by the GPU path and by the CPU oracle.

This module holds random draws and array shapes only.  It holds none of the
method's arithmetic: no ordering, no assembly, no network evaluation, no
preconditioner and no solver.  Everything the method computes is done on one
side by the HIP library and on the other side by the oracle, each from these
same arrays.

Frames follow the multiphase pressure-Poisson setting of the paper
(Supplementary "Multiphase Poisson Benchmark Generation") moved to a 3D
cell-centred grid: a light background density rho=1 with heavy inclusions
(seeded spheres, optionally a heavy bottom layer) and a uniform right-hand
side.  All grid arrays are in lexicographic cell order, id = x + nx*(y + ny*z),
with z the vertical axis (z = nz-1 is the top layer).

The paper's own benchmark (Sec. 7.1 "Benchmark"; Supplementary "Multiphase
Poisson Benchmark Generation") is drawn by the "paper2d_<N>" recipes: a 2D grid
(nz = 1) whose heavy cells are 1-3 rectangular barriers with gaps, density
noise, zero flux on every face and a mean-zero Gaussian right-hand side.
"""
from __future__ import annotations

import dataclasses
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np


# ----------------------------------------------------------------------------
# workloads
# ----------------------------------------------------------------------------

@dataclasses.dataclass(frozen=True)
class FrameRecipe:
    """How one family of frames is drawn."""
    grids: Tuple[Tuple[int, int, int], ...]   # candidate (nx, ny, nz); one is drawn per frame
    spheres: Tuple[int, int]                  # inclusive range of the sphere count
    contrast: Tuple[float, float]             # heavy density range (rho_light = 1)
    radius: Tuple[float, float] = (2.0, 4.0)  # sphere radius range, in cells
    heavy_bottom_layer: bool = False          # rho_heavy for z < nz/2 (stratified two-phase)


GRID_OF_N = {
    1024: (16, 8, 8),
    2048: (16, 16, 8),
    4096: (16, 16, 16),
    8192: (32, 16, 16),
    16384: (32, 32, 16),
}

RECIPES: Dict[str, "FrameRecipe | BarrierRecipe"] = {
    # N=1,024, 3 spheres at 100:1
    "plain1024": FrameRecipe(grids=(GRID_OF_N[1024],), spheres=(3, 3), contrast=(100.0, 100.0)),
    # N=8,192, 8 spheres at 100:1
    "precision8192": FrameRecipe(grids=(GRID_OF_N[8192],), spheres=(8, 8), contrast=(100.0, 100.0)),
    # N=4,096 training systems: 2-8 spheres, contrast uniform in [10, 100]
    "train4096": FrameRecipe(grids=(GRID_OF_N[4096],), spheres=(2, 8), contrast=(10.0, 100.0)),
    # the same law on the two smaller grids of the mixed batches
    "train1024": FrameRecipe(grids=(GRID_OF_N[1024],), spheres=(2, 8), contrast=(10.0, 100.0)),
    "train2048": FrameRecipe(grids=(GRID_OF_N[2048],), spheres=(2, 8), contrast=(10.0, 100.0)),
    # batching: N drawn uniformly from {1,024, 2,048, 4,096, 8,192}
    "batch_mixed": FrameRecipe(grids=tuple(GRID_OF_N[n] for n in (1024, 2048, 4096, 8192)),
                               spheres=(2, 8), contrast=(10.0, 100.0)),
    # N=16,384: heavy bottom half plus 16 spheres at 100:1
    "largest16384": FrameRecipe(grids=(GRID_OF_N[16384],), spheres=(16, 16), contrast=(100.0, 100.0),
                                heavy_bottom_layer=True),
}


@dataclasses.dataclass(frozen=True)
class BarrierRecipe:
    """The paper's 2D frames (Supplementary "Multiphase Poisson Benchmark
    Generation"): rho_heavy log-uniform in `contrast`, rho_light = 1, 1-3
    barriers, each a band across the whole domain (vertical or horizontal,
    equally likely) with its centre uniform in [0.2, 0.8] and its thickness
    uniform in [0.05, 0.20] along the cross axis (unit-square coordinates),
    and one of four gap topologies: a gap at the high end of the band ("top"),
    at the low end ("bottom"), in its middle ("middle_hole"), or none
    ("closed").  A cell is heavy if any band covers it.  Every density is
    then multiplied by 1 + N(0, 0.05^2).  b ~ N(0, I) minus its mean."""
    grid: Tuple[int, int]                     # (W, H) = (nx, ny); nz = 1
    contrast: Tuple[float, float] = (5.0, 100.0)
    box: Optional[Tuple[int, int]] = None     # padded frames: the power-of-two box holding the W x H grid
    cells: Optional[int] = None               # padded frames: N, the grid cut to its first N cells in Morton order
    barriers: Tuple[int, int] = (1, 3)
    centre: Tuple[float, float] = (0.2, 0.8)
    thickness: Tuple[float, float] = (0.05, 0.20)
    gap: float = 0.2                          # gap length, fraction of the band's length
    noise: float = 0.05


GAP_TOPOLOGIES = ("top", "bottom", "middle_hole", "closed")

# W x H: powers of two, as close to square as powers of two allow, so that
# W * H = N and the Morton truncation to the first N cells keeps every cell.
GRID2D_OF_N = {1024: (32, 32), 2048: (64, 32), 4096: (64, 64), 8192: (128, 64), 16384: (128, 128)}

for _n, _wh in GRID2D_OF_N.items():
    RECIPES[f"paper2d_{_n}"] = BarrierRecipe(grid=_wh)

# The paper's own grid choice for N that is not a product of two close powers
# of two: W x H as close to square as possible with W H >= N (W = ceil(sqrt N),
# H = ceil(N / W)), cut to the first N cells in Morton order.  Such a frame is
# padded to the smallest power-of-two box the library's partition accepts.
TRUNC2D_OF_N = {2048: ((46, 45), (64, 64)), 8192: ((91, 91), (128, 128))}

for _n, (_wh, _box) in TRUNC2D_OF_N.items():
    RECIPES[f"paper2d_trunc_{_n}"] = BarrierRecipe(grid=_wh, box=_box, cells=_n)


@dataclasses.dataclass
class Frame:
    nx: int
    ny: int
    nz: int
    rho: np.ndarray   # float64 [N], lexicographic
    b: np.ndarray     # float64 [N], lexicographic, uniform in [-1, 1) (mean-zero Gaussian for 2D barriers)
    seed: int
    neumann: bool = False   # zero flux on every face, conductance the harmonic mean of rho (the paper's operator)
    # Padded frames: (W, H, D, cells), the frame's own cells are the first
    # `cells` cells, in Morton order, of the W x H x D grid at the origin of
    # the nx x ny x nz box; the rest of the box is padding.  b is then the raw
    # draw over the box: the right-hand side is b on the frame's cells (minus
    # its mean there for the zero-flux operator) and 0 on the padding, which
    # each side forms from its own cell mask.
    region: Optional[Tuple[int, int, int, int]] = None

    @property
    def n(self) -> int:
        """Unknowns of the box (the partition's N)."""
        return self.nx * self.ny * self.nz

    @property
    def cells(self) -> int:
        """The frame's own cells."""
        return self.n if self.region is None else int(self.region[3])


def _make_barrier_frame(rc: BarrierRecipe, seed: int) -> Frame:
    """Draw order: rho_heavy, barrier count, per barrier (orientation, centre,
    thickness, gap topology), the density noise cell by cell, then b."""
    rng = np.random.default_rng(seed)
    W, H = rc.grid
    nx, ny = rc.box if rc.box is not None else rc.grid
    heavy = float(np.exp(rng.uniform(np.log(rc.contrast[0]), np.log(rc.contrast[1]))))
    nb = int(rng.integers(rc.barriers[0], rc.barriers[1] + 1))
    y, x = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
    u, v = (x.ravel() + 0.5) / W, (y.ravel() + 0.5) / H        # unit-square centres of the W x H grid
    in_grid = (x.ravel() < W) & (y.ravel() < H)
    inside = np.zeros(nx * ny, dtype=bool)
    for _ in range(nb):
        vertical = bool(rng.integers(2))
        c = float(rng.uniform(*rc.centre))
        t = float(rng.uniform(*rc.thickness))
        topo = GAP_TOPOLOGIES[int(rng.integers(len(GAP_TOPOLOGIES)))]
        across, along = (u, v) if vertical else (v, u)
        band = np.abs(across - c) <= 0.5 * t
        if topo == "top":
            band &= along < 1.0 - rc.gap
        elif topo == "bottom":
            band &= along >= rc.gap
        elif topo == "middle_hole":
            band &= np.abs(along - 0.5) >= 0.5 * rc.gap
        inside |= band & in_grid
    rho = np.where(inside, heavy, 1.0) * (1.0 + rc.noise * rng.standard_normal(nx * ny))
    b = rng.standard_normal(nx * ny)
    if rc.box is None:
        b -= b.mean()
        return Frame(nx=nx, ny=ny, nz=1, rho=rho.astype(np.float64), b=b, seed=seed, neumann=True)
    rho = np.where(in_grid, rho, 1.0)       # the box outside the grid: light, noise-free
    cells = rc.cells if rc.cells is not None else W * H
    return Frame(nx=nx, ny=ny, nz=1, rho=rho.astype(np.float64), b=b, seed=seed, neumann=True,
                 region=(W, H, 1, cells))


def make_frame(recipe: str | FrameRecipe | BarrierRecipe, seed: int) -> Frame:
    """Draw one frame.  Sphere recipes draw, in order: grid, sphere count,
    contrast, spheres (cx, cy, cz, r each), then b cell by cell."""
    rc = RECIPES[recipe] if isinstance(recipe, str) else recipe
    if isinstance(rc, BarrierRecipe):
        return _make_barrier_frame(rc, seed)
    rng = np.random.default_rng(seed)
    nx, ny, nz = rc.grids[int(rng.integers(len(rc.grids)))] if len(rc.grids) > 1 else rc.grids[0]
    ns = int(rng.integers(rc.spheres[0], rc.spheres[1] + 1))
    heavy = float(rng.uniform(rc.contrast[0], rc.contrast[1])) if rc.contrast[1] > rc.contrast[0] \
        else float(rc.contrast[0])
    sph = []
    for _ in range(ns):
        cx, cy, cz = rng.uniform(0.0, 1.0, size=3) * np.array([nx, ny, nz], dtype=np.float64)
        r = rng.uniform(rc.radius[0], rc.radius[1])
        sph.append((cx, cy, cz, r))
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    px, py, pz = (x.ravel() + 0.5), (y.ravel() + 0.5), (z.ravel() + 0.5)
    inside = np.zeros(nx * ny * nz, dtype=bool)
    for (cx, cy, cz, r) in sph:
        inside |= (px - cx) ** 2 + (py - cy) ** 2 + (pz - cz) ** 2 <= r * r
    if rc.heavy_bottom_layer:
        inside |= z.ravel() < nz // 2
    rho = np.where(inside, heavy, 1.0).astype(np.float64)
    b = rng.uniform(-1.0, 1.0, size=nx * ny * nz).astype(np.float64)
    return Frame(nx=nx, ny=ny, nz=nz, rho=rho, b=b, seed=seed)


def make_frame_grid(nx: int, ny: int, nz: int, seed: int, spheres: int = 3,
                    contrast: float = 100.0) -> Frame:
    """A frame on an arbitrary grid with the plain recipe's inclusion law."""
    return make_frame(FrameRecipe(grids=((nx, ny, nz),), spheres=(spheres, spheres),
                                  contrast=(contrast, contrast)), seed)


def make_padded_frame(box: Tuple[int, int, int], region: Tuple[int, int, int, int], seed: int,
                      spheres: int = 3, contrast: float = 100.0) -> Frame:
    """A 3D frame of the plain recipe's inclusion law on the box, whose own
    cells are `region` (W, H, D, cells); b stays the raw draw (see Frame)."""
    fr = make_frame_grid(*box, seed, spheres=spheres, contrast=contrast)
    fr.region = tuple(int(t) for t in region)
    return fr


# ----------------------------------------------------------------------------
# network shapes and seeded initial weights
# ----------------------------------------------------------------------------

@dataclasses.dataclass(frozen=True)
class ModelConfig:
    d: int = 128          # token width
    heads: int = 4        # attention heads (head dim d/heads)
    layers: int = 4       # transformer blocks per stack
    leaf: int = 64        # L, unknowns per dense leaf
    rank: int = 16        # L_s, coarse tokens per off-diagonal tile
    edge_hidden: int = 32 # hidden width of the edge-bias MLP
    gcn: int = 2          # residual graph-convolution layers in the encoder
    node_feats: int = 8   # per-node features
    glob_feats: int = 12  # per-frame global features broadcast to every node
    highways: bool = True
    offdiag: bool = True

    @property
    def feats(self) -> int:
        return self.node_feats + self.glob_feats


MODEL_PLAIN = ModelConfig(leaf=32, rank=8)
MODEL_DEFAULT = ModelConfig(leaf=64, rank=16)


def weight_spec(cfg: ModelConfig) -> List[Tuple[str, Tuple[int, ...], str]]:
    """Ordered (name, shape, init) list.  Linear maps are stored [in, out] and
    act as y = x @ W + b.  init is 'normal', 'zeros' or 'ones'."""
    d, F, E, H, L, R = cfg.d, cfg.feats, cfg.edge_hidden, cfg.heads, cfg.leaf, cfg.rank
    s: List[Tuple[str, Tuple[int, ...], str]] = []
    lin = lambda n, i, o, w="normal": s.extend([(n + ".w", (i, o), w), (n + ".b", (o,), "zeros")])
    ln = lambda n, w: s.extend([(n + ".g", (w,), "ones"), (n + ".b", (w,), "zeros")])
    lin("enc1", F, d)
    lin("enc2", d, d)
    for g in range(cfg.gcn):
        lin(f"gcn{g}", d, d)
    s.append(("pool.wr", (d, d), "normal"))
    s.append(("pool.wc", (d, d), "normal"))
    s.append(("pool.b", (d,), "zeros"))
    for st in ("diag", "off"):
        for l in range(cfg.layers):
            p = f"{st}{l}."
            ln(p + "ln1", d)
            lin(p + "qkv", d, 3 * d)
            lin(p + "o", d, d)
            lin(p + "e1", 4, E)
            lin(p + "e2", E, H)
            ln(p + "ln2", 4 * d)
            lin(p + "f1", 4 * d, 4 * d)
            lin(p + "f2", 4 * d, d)
        ln(st + "lnf", d)
    lin("hleaf1", d, d)
    lin("hleaf2", d, L)
    lin("hu", d, R)
    lin("hv", d, R, "zeros")       # zero V head: B_m = U_m V_m^T starts at 0
    lin("hut", d, R)
    lin("hvt", d, R)
    lin("hlam", d, 1)
    return s


def init_weights(cfg: ModelConfig, seed: int, std: float = 0.02) -> Dict[str, np.ndarray]:
    rng = np.random.default_rng(seed)
    out: Dict[str, np.ndarray] = {}
    for name, shape, init in weight_spec(cfg):
        if init == "normal":
            out[name] = (rng.standard_normal(shape) * std).astype(np.float32)
        elif init == "ones":
            out[name] = np.ones(shape, dtype=np.float32)
        else:
            out[name] = np.zeros(shape, dtype=np.float32)
    return out


def param_count(cfg: ModelConfig) -> int:
    return int(sum(int(np.prod(sh)) for _, sh, _ in weight_spec(cfg)))


# ----------------------------------------------------------------------------
# probes
# ----------------------------------------------------------------------------

def rademacher(n: int, kz: int, seed: int) -> np.ndarray:
    """[n, kz] matrix of independent +-1 entries (float32)."""
    rng = np.random.default_rng(seed)
    return (rng.integers(0, 2, size=(n, kz)) * 2 - 1).astype(np.float32)
