"""Pins of the oracle's ordering, assembly and partition (CPU only)."""
import math

import numpy as np
import pytest
import scipy.linalg

from oracle import grid, partition
from paper_2605_13343_amd import inputs

CONFIG_GRIDS = [(16, 8, 8), (16, 16, 8), (16, 16, 16), (32, 16, 16), (32, 32, 16)]


def _spread3(v):
    """Bit spread by the classic magic-mask method (independent of the
    oracle's bit-by-bit loop)."""
    v &= 0x3FF
    v = (v | (v << 16)) & 0x030000FF
    v = (v | (v << 8)) & 0x0300F00F
    v = (v | (v << 4)) & 0x030C30C3
    v = (v | (v << 2)) & 0x09249249
    return v


def test_morton_code_matches_magic_masks():
    rng = np.random.default_rng(0)
    for _ in range(200):
        x, y, z = (int(a) for a in rng.integers(0, 1024, 3))
        assert grid.morton_code(x, y, z) == _spread3(x) | (_spread3(y) << 1) | (_spread3(z) << 2)


@pytest.mark.parametrize("dims", CONFIG_GRIDS[:3])
def test_morton_perm_bijection_and_contiguous_codes(dims):
    nx, ny, nz = dims
    n = nx * ny * nz
    perm = grid.morton_perm(nx, ny, nz)
    assert sorted(perm.tolist()) == list(range(n))
    xyz = grid.cell_xyz(nx, ny, nz, perm)
    codes = [grid.morton_code(*map(int, c)) for c in xyz]
    # codes are exactly 0..N-1 on the workload grids, so rank == code
    assert codes == list(range(n))


def test_morton_leaves_are_blocks():
    nx, ny, nz = 32, 16, 16
    xyz = grid.cell_xyz(nx, ny, nz, grid.morton_perm(nx, ny, nz))
    for k in range(0, nx * ny * nz, 64):            # 64-leaf = 4x4x4 block
        blk = xyz[k:k + 64]
        assert all(len(set(blk[:, a] // 4)) == 1 for a in range(3))
        assert all(len(set(blk[:, a])) == 4 for a in range(3))
    xyz = grid.cell_xyz(16, 8, 8, grid.morton_perm(16, 8, 8))
    for k in range(0, 1024, 32):                    # 32-leaf = 4x4x2 block
        blk = xyz[k:k + 32]
        assert [len(set(blk[:, a])) for a in range(3)] == [4, 4, 2]


def test_assembly_hand_values():
    # 2x1x2 grid: cells (x,z) = (0,0),(1,0),(0,1),(1,1); rho 1, 3, 1, 1
    rho = np.array([1.0, 3.0, 1.0, 1.0])
    A = grid.assemble_lex(2, 1, 2, rho).toarray()
    w01 = 2 / (1 + 3)          # x-face between cells 0 and 1
    w02 = 2 / (1 + 1)
    w13 = 2 / (3 + 1)
    w23 = 2 / (1 + 1)
    assert A[0, 1] == -w01 and A[1, 0] == -w01
    assert A[0, 2] == -w02 and A[1, 3] == -w13 and A[2, 3] == -w23
    assert A[0, 3] == 0 and A[1, 2] == 0
    assert math.isclose(A[0, 0], w01 + w02)
    assert math.isclose(A[1, 1], w01 + w13)
    assert math.isclose(A[2, 2], w02 + w23 + 1.0)        # top row: ghost Dirichlet 1/rho
    assert math.isclose(A[3, 3], w13 + w23 + 1.0)


def test_assembly_symmetry_rowsums_and_spd():
    fr = inputs.make_frame("plain1024", 1000)
    A = grid.assemble(fr.nx, fr.ny, fr.nz, fr.rho)
    assert (A != A.T).nnz == 0
    rho_m = fr.rho[grid.morton_perm(fr.nx, fr.ny, fr.nz)]
    top = grid.positions(fr.nx, fr.ny, fr.nz)[:, 2] == fr.nz - 1
    rs = np.asarray(A.sum(axis=1)).ravel()
    assert np.allclose(rs[~top], 0.0, atol=1e-13)
    assert np.allclose(rs[top], 1.0 / rho_m[top], rtol=1e-13)
    assert A.nnz == fr.n + 2 * (15 * 8 * 8 + 16 * 7 * 8 + 16 * 8 * 7)
    scipy.linalg.cholesky(A.toarray())              # raises unless SPD


def test_assembly_constant_density_closed_form():
    nx, ny, nz = 8, 4, 4
    A = grid.assemble(nx, ny, nz, np.ones(nx * ny * nz)).toarray()
    ev = np.sort(np.linalg.eigvalsh(A))
    cf = sorted((2 - 2 * math.cos(math.pi * a / nx)) + (2 - 2 * math.cos(math.pi * b / ny))
                + (2 - 2 * math.cos((2 * c + 1) * math.pi / (2 * nz + 1)))
                for a in range(nx) for b in range(ny) for c in range(nz))
    assert np.allclose(ev, cf, atol=1e-12)
    A5 = grid.assemble(nx, ny, nz, 5.0 * np.ones(nx * ny * nz)).toarray()
    assert np.allclose(A5, A / 5.0, rtol=1e-14, atol=0)


def test_features_shape_and_globals():
    fr = inputs.make_frame("plain1024", 1001)
    f = grid.features(fr.nx, fr.ny, fr.nz, fr.rho)
    assert f.shape == (1024, 20)
    assert np.all(f[:, 8:] == f[0, 8:])
    assert math.isclose(f[0, 8], 10 / 16)
    assert math.isclose(f[0, 9], math.log(100.0))
    assert set(np.unique(f[:, 0])) <= {0.0, math.log(100.0)}


# ---------------------------------------------------------------- partition

def test_partition_counts_and_pairs():
    for n, L in [(1024, 32), (8192, 64), (4096, 64), (64, 64), (256, 32)]:
        p = partition.build(n, L, L // 4)
        K = n // L
        assert p["MH"] == K - 1
        # each leaf pair k < k' lies in exactly one tile, at the level of the
        # highest differing bit; k on the row side
        for k in range(K):
            for k2 in range(k + 1, K):
                hits = [m for m, (j, r0, c0, S) in enumerate(p["tiles"])
                        if r0 <= k < r0 + S and c0 <= k2 < c0 + S]
                assert len(hits) == 1
                assert p["tiles"][hits[0]][0] == (k ^ k2).bit_length() - 1
                assert not any(r0 <= k2 < r0 + S and c0 <= k < c0 + S for (j, r0, c0, S) in p["tiles"])
        assert (p["leaf_tile"] >= 0).all() and p["leaf_tile"].shape == (K, max(K.bit_length() - 1, 0))


def test_partition_reproduces_paper_memory_table():
    rows = [l.split() for l in open(__file__.replace("test_oracle_grid.py", "golden/supp_memory.txt"))
            if l.strip() and not l.startswith("#")]
    for N, K, MH, KL2, P, MB in rows:
        p = partition.build(int(N), 128, 32)
        assert p["K"] == int(K) and p["MH"] == int(MH)
        assert round(p["sizes"]["diag"] / 1e6, 3) == float(KL2)
        assert round(p["P"] / 1e6, 2) == float(P)
        assert round(4 * p["P"] / 1e6, 2 if float(MB) < 10 else 1) == float(MB)
        assert p["P"] == partition.packed_width(int(N), 128, 32)


def test_partition_workload_sizes():
    assert partition.packed_width(1024, 32, 8) == 52160
    assert partition.packed_width(8192, 64, 16) == 827136
    assert partition.packed_width(16384, 64, 16) == 1654528
