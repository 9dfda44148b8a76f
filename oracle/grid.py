"""Grid ordering, operator assembly and node features (oracle, float64).

TEST INFRASTRUCTURE ONLY -- see oracle/__init__.py.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.sparse as sp


def morton_code(x: int, y: int, z: int, bits: int = 16) -> int:
    """Z-order code of cell (x, y, z): bit b of x goes to bit 3b, of y to
    3b+1, of z to 3b+2 (paper, Supplementary "Grid and ordering": cells are
    sorted by Morton code; the 3D interleave is this build's reading)."""
    c = 0
    for b in range(bits):
        c |= ((x >> b) & 1) << (3 * b)
        c |= ((y >> b) & 1) << (3 * b + 1)
        c |= ((z >> b) & 1) << (3 * b + 2)
    return c


def morton_perm(nx: int, ny: int, nz: int) -> np.ndarray:
    """perm[i] = lexicographic id (x + nx*(y + ny*z)) of the i-th cell in
    Morton order.  Codes are unique, so the sort needs no tie-break."""
    ids, codes = [], []
    for z in range(nz):
        for y in range(ny):
            for x in range(nx):
                ids.append(x + nx * (y + ny * z))
                codes.append(morton_code(x, y, z))
    order = sorted(range(len(ids)), key=lambda t: codes[t])
    return np.array([ids[t] for t in order], dtype=np.int64)


def cell_xyz(nx: int, ny: int, nz: int, lex: np.ndarray) -> np.ndarray:
    lex = np.asarray(lex)
    return np.stack([lex % nx, (lex // nx) % ny, lex // (nx * ny)], axis=-1)


def region_mask_lex(nx: int, ny: int, nz: int, region=None) -> np.ndarray:
    """Which cells of the nx x ny x nz box belong to the frame, lexicographic
    boolean [nx ny nz].

    A frame whose grid is not a power-of-two box (paper Sec. 8: the partition
    is sized to a maximum N; Supplementary "Grid and ordering": a W x H grid,
    close to square, with W H >= N, whose cells are sorted by Morton code and
    cut to the first N) sits in the smallest box the partition accepts.
    region = (W, H, D, n): the frame's cells are the first n cells, in Morton
    order, of the W x H x D grid at the box origin; every other cell of the
    box is padding.  region None: every cell is the frame's.
    """
    mask = np.zeros(nx * ny * nz, dtype=bool)
    if region is None:
        mask[:] = True
        return mask
    W, H, D, n = (int(t) for t in region)
    if not (1 <= W <= nx and 1 <= H <= ny and 1 <= D <= nz and 1 <= n <= W * H * D):
        raise ValueError(f"region {region} does not fit the {nx} x {ny} x {nz} box")
    cells = sorted((morton_code(x, y, z), x + nx * (y + ny * z))
                   for z in range(D) for y in range(H) for x in range(W))
    for _, lid in cells[:n]:
        mask[lid] = True
    return mask


def region_rhs(nx: int, ny: int, nz: int, b_lex: np.ndarray, region=None, neumann: bool = False) -> np.ndarray:
    """Right-hand side of a padded frame, lexicographic: b on the frame's
    cells and 0 on the padding (so the solution is 0 there); for the
    zero-flux operator also minus its mean over the frame's cells, which
    makes it orthogonal to the null space of the frame's block (the constant
    on its cells; connected frames).  region None: b unchanged."""
    b_lex = np.asarray(b_lex, dtype=np.float64)
    if region is None:
        return b_lex.copy()
    real = region_mask_lex(nx, ny, nz, region)
    out = np.where(real, b_lex, 0.0)
    if neumann:
        out[real] -= out[real].mean()
    return out


def region_top(nz: int, region=None) -> int:
    """The layer that carries the Dirichlet condition: the top layer of the
    frame's grid (z = D-1), the box's top (z = nz-1) without a region."""
    return nz - 1 if region is None else int(region[2]) - 1


def assemble_lex(nx: int, ny: int, nz: int, rho: np.ndarray, neumann: bool = False,
                 region=None) -> sp.csr_matrix:
    """Cell-centred variable-coefficient Poisson operator (7-point; 5-point
    when nz = 1) in lexicographic order, spacing h = 1.

    Paper, Sec. 7.1 / Supplementary "Operator assembly": A_ii = sum_j w_ij,
    A_ij = -w_ij over cell-cell faces.

    neumann=False (the 3D workload): face weight w_ij = 2/(rho_i+rho_j), the
    harmonic mean of 1/rho; zero flux on every face except the top (z = nz-1),
    which carries p = 0 through a ghost cell one spacing away: A_ii += 1/rho_i.

    neumann=True (the paper's benchmark operator as printed): face weight
    w_ij = 2 rho_i rho_j/(rho_i+rho_j), the harmonic mean of rho, and zero
    flux on every boundary face, so A 1 = 0 (A is singular; the paper leaves
    the constant mode to CG with a consistent right-hand side).

    region (see region_mask_lex): faces join two cells of the frame only, a
    face towards padding is a zero-flux boundary face, the Dirichlet term
    sits on the frame grid's top layer, and a padding cell's row is the
    identity row (A_ii = 1, decoupled), so the frame's block is the operator
    of its own cells and the padding block is I.
    """
    n = nx * ny * nz
    real = region_mask_lex(nx, ny, nz, region)
    ztop = region_top(nz, region)
    rows, cols, vals = [], [], []
    diag = np.zeros(n)

    def lid(x, y, z):
        return x + nx * (y + ny * z)

    for z in range(nz):
        for y in range(ny):
            for x in range(nx):
                i = lid(x, y, z)
                if not real[i]:
                    diag[i] = 1.0
                    continue
                for (dx, dy, dz) in ((1, 0, 0), (0, 1, 0), (0, 0, 1)):
                    xx, yy, zz = x + dx, y + dy, z + dz
                    if xx >= nx or yy >= ny or zz >= nz:
                        continue
                    j = lid(xx, yy, zz)
                    if not real[j]:
                        continue
                    if neumann:
                        w = 2.0 * rho[i] * rho[j] / (rho[i] + rho[j])
                    else:
                        w = 2.0 / (rho[i] + rho[j])
                    rows += [i, j]
                    cols += [j, i]
                    vals += [-w, -w]
                    diag[i] += w
                    diag[j] += w
                if z == ztop and not neumann:
                    diag[i] += 1.0 / rho[i]
    rows += list(range(n))
    cols += list(range(n))
    vals += list(diag)
    return sp.csr_matrix((np.array(vals), (np.array(rows), np.array(cols))), shape=(n, n))


def assemble(nx: int, ny: int, nz: int, rho_lex: np.ndarray, neumann: bool = False,
             region=None) -> sp.csr_matrix:
    """The operator in Morton order: A_m = P A P^T with P the Morton perm."""
    perm = morton_perm(nx, ny, nz)
    A = assemble_lex(nx, ny, nz, rho_lex, neumann, region)
    Am = A[perm][:, perm].tocsr()
    Am.sort_indices()
    return Am


def features(nx: int, ny: int, nz: int, rho_lex: np.ndarray, neumann: bool = False,
             region=None) -> np.ndarray:
    """Per-node encoder input [N, 20] in Morton order.

    The paper (Sec. 4.1, Supplementary "Encoder") lists density, position and
    boundary indicators per node and a 12-value per-frame summary of the
    assembled system.  This build's definition:
      node:   log rho, (x+1/2)/nx, (y+1/2)/ny, (z+1/2)/nz, top flag (z=nz-1),
              side flag (x or y on the domain boundary), bottom flag (z=0),
              log A_ii
      global: log2(N)/16, log(rho_max/rho_min), mean and std of log rho,
              heavy fraction (log rho above the mid-point of its range),
              mean/std/min/max of log A_ii, nx/32, ny/32, nz/32
    Standard deviations are population (divide by N).  Pressure is absent:
    the frames have no previous time step.  The flags are geometric: on a 2D
    grid (nz = 1) every cell is both top and bottom layer.  A_ii comes from
    the operator the frame uses (neumann, region, as in assemble_lex).  With a
    region the network sees the whole box: positions, flags and the summary
    are those of the box, padding cells included (A_ii = 1 there).
    """
    n = nx * ny * nz
    perm = morton_perm(nx, ny, nz)
    A = assemble_lex(nx, ny, nz, rho_lex, neumann, region)
    dA = A.diagonal()
    xyz = cell_xyz(nx, ny, nz, np.arange(n))
    x, y, z = xyz[:, 0], xyz[:, 1], xyz[:, 2]
    lr = np.log(rho_lex)
    la = np.log(dA)
    node = np.stack([
        lr,
        (x + 0.5) / nx, (y + 0.5) / ny, (z + 0.5) / nz,
        (z == nz - 1).astype(np.float64),
        ((x == 0) | (x == nx - 1) | (y == 0) | (y == ny - 1)).astype(np.float64),
        (z == 0).astype(np.float64),
        la,
    ], axis=1)
    lmin, lmax = lr.min(), lr.max()
    heavy = float(np.mean(lr > 0.5 * (lmin + lmax))) if lmax > lmin else 0.0
    glob = np.array([
        math.log2(n) / 16.0,
        lmax - lmin,
        lr.mean(), lr.std(),
        heavy,
        la.mean(), la.std(), la.min(), la.max(),
        nx / 32.0, ny / 32.0, nz / 32.0,
    ])
    f = np.concatenate([node, np.broadcast_to(glob, (n, 12))], axis=1)
    return f[perm]


def positions(nx: int, ny: int, nz: int) -> np.ndarray:
    """Integer (x, y, z) of every cell, Morton order, [N, 3] float64."""
    perm = morton_perm(nx, ny, nz)
    return cell_xyz(nx, ny, nz, perm).astype(np.float64)
