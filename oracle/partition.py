"""Weak-admissibility H-matrix partition and packed factor layout (oracle).

TEST INFRASTRUCTURE ONLY -- see oracle/__init__.py.

Paper, Sec. 4 (notation and pipeline), Sec. 4.2 and Supplementary
"Apply-path tensor layout" / "H-matrix partition": N indices in K = N/L
contiguous leaves; off-diagonal tiles span S x S leaves with S = 2^j; at
eta = 1 the strict upper triangle holds M_H = K - 1 unique tiles (K/2 + K/4 +
... + 1); the partition is static per N and independent of A.

This build's reading of the tile order: level j = 0 (S = 1, finest) first;
within a level, tile i has row leaves [2iS, 2iS+S) and column leaves
[2iS+S, 2iS+2S), i.e. the row strip is the left sibling.  Tile index
m = K - K/2^j + i.
"""
from __future__ import annotations

from typing import Dict, List

import numpy as np


def build(n: int, leaf: int, rank: int) -> Dict:
    if n % leaf:
        raise ValueError("N must be a multiple of the leaf size")
    K = n // leaf
    if K & (K - 1):
        raise ValueError("leaf count must be a power of two")
    J = K.bit_length() - 1
    tiles: List[tuple] = []      # (level, row0, col0, span) in leaves
    for j in range(J):
        S = 1 << j
        for i in range(K // (2 * S)):
            tiles.append((j, 2 * i * S, 2 * i * S + S, S))
    MH = len(tiles)
    # membership by brute force over the tile list
    leaf_tile = np.full((K, J), -1, dtype=np.int64)
    leaf_side = np.full((K, J), -1, dtype=np.int64)
    for m, (j, r0, c0, S) in enumerate(tiles):
        for k in range(r0, r0 + S):
            assert leaf_tile[k, j] == -1
            leaf_tile[k, j], leaf_side[k, j] = m, 0
        for k in range(c0, c0 + S):
            assert leaf_tile[k, j] == -1
            leaf_tile[k, j], leaf_side[k, j] = m, 1
    sizes = {
        "diag": K * leaf * leaf,
        "B": MH * rank * rank,
        "Ut": n * rank,
        "Vt": n * rank,
        "lam": n,
    }
    off, acc = {}, 0
    for key in ("diag", "B", "Ut", "Vt", "lam"):
        off[key] = acc
        acc += sizes[key]
    return dict(n=n, L=leaf, Ls=rank, K=K, J=J, MH=MH, tiles=tiles,
                leaf_tile=leaf_tile, leaf_side=leaf_side,
                sizes=sizes, offsets=off, P=acc)


def packed_width(n: int, leaf: int, rank: int) -> int:
    """P = K L^2 + M_H L_s^2 + 2 N L_s + N (Sec. 4.4, Supplementary Table
    'supp_memory')."""
    K = n // leaf
    return K * leaf * leaf + (K - 1) * rank * rank + 2 * n * rank + n


def strip_nodes(part: Dict, m: int, t: int, side: int) -> np.ndarray:
    """Node ids of sub-strip t of tile m: positions [t p, (t+1) p) of every
    leaf on the row side (side 0) or column side (side 1); p = L / L_s."""
    j, r0, c0, S = part["tiles"][m]
    L, Ls = part["L"], part["Ls"]
    p = L // Ls
    k0 = r0 if side == 0 else c0
    return np.array([k * L + l for k in range(k0, k0 + S) for l in range(t * p, (t + 1) * p)],
                    dtype=np.int64)
