"""Pins of the oracle on the paper's own 2D benchmark (Sec. 7.1 "Benchmark";
Supplementary "Multiphase Poisson Benchmark Generation", "Operator
assembly"): the 2D Morton order, the zero-flux operator with the harmonic mean
of rho as face conductance, its null space, the generator's stated
properties, and PCG on the singular system (CPU only)."""
import math

import numpy as np
import pytest

from oracle import grid, network, pcg
from paper_2605_13343_amd import inputs


def _spread2(v):
    """2-way bit spread by magic masks (independent of the oracle's loop)."""
    v &= 0xFFFF
    v = (v | (v << 8)) & 0x00FF00FF
    v = (v | (v << 4)) & 0x0F0F0F0F
    v = (v | (v << 2)) & 0x33333333
    v = (v | (v << 1)) & 0x55555555
    return v


def test_morton_2d_order_by_hand():
    # 4 x 2 grid: x0 y0 x1 interleave -> (0,0) (1,0) (0,1) (1,1) (2,0) (3,0) (2,1) (3,1)
    assert grid.morton_perm(4, 2, 1).tolist() == [0, 1, 4, 5, 2, 3, 6, 7]


@pytest.mark.parametrize("wh", list(inputs.GRID2D_OF_N.values()))
def test_morton_2d_rank_is_the_2d_interleave(wh):
    """On the benchmark grids the Morton rank of a cell is its 2D interleaved
    code (x at even bits, y at odd bits), so leaves are square-ish blocks."""
    nx, ny = wh
    xyz = grid.cell_xyz(nx, ny, 1, grid.morton_perm(nx, ny, 1))
    assert (xyz[:, 2] == 0).all()
    codes = [_spread2(int(x)) | (_spread2(int(y)) << 1) for x, y, _ in xyz]
    assert codes == list(range(nx * ny))
    for k in range(0, nx * ny, 64):               # a 64-leaf is an 8 x 8 block
        blk = xyz[k:k + 64]
        assert len(set(blk[:, 0])) == 8 and len(set(blk[:, 1])) == 8


def test_neumann_assembly_hand_values():
    # 2 x 2 grid, lexicographic cells (0,0) (1,0) (0,1) (1,1), rho 1, 4, 2, 8;
    # w = 2 rho_i rho_j / (rho_i + rho_j): x faces 8/5, 16/5; y faces 4/3, 16/3;
    # no boundary term
    A = grid.assemble_lex(2, 2, 1, np.array([1.0, 4.0, 2.0, 8.0]), neumann=True).toarray()
    a, b, c, d = 8 / 5, 16 / 5, 4 / 3, 16 / 3
    ref = np.array([[a + c, -a, -c, 0.0],
                    [-a, a + d, 0.0, -d],
                    [-c, 0.0, c + b, -b],
                    [0.0, -d, -b, d + b]])
    assert np.allclose(A, ref, rtol=1e-15, atol=0)


def test_neumann_constant_density_closed_form():
    """rho = 3 everywhere: 3 times the zero-flux 5-point Laplacian, whose
    eigenvalues on a W x H cell grid are (2 - 2 cos(pi p / W)) +
    (2 - 2 cos(pi q / H)) (cosine modes)."""
    nx, ny = 8, 4
    A = grid.assemble(nx, ny, 1, 3.0 * np.ones(nx * ny), neumann=True).toarray()
    ev = np.sort(np.linalg.eigvalsh(A))
    cf = sorted(3.0 * ((2 - 2 * math.cos(math.pi * p / nx)) + (2 - 2 * math.cos(math.pi * q / ny)))
                for p in range(nx) for q in range(ny))
    assert np.allclose(ev, cf, atol=1e-12)
    # the Dirichlet-top operator of the 3D workload differs on the same grid
    Ad = grid.assemble(nx, ny, 1, 3.0 * np.ones(nx * ny)).toarray()
    assert np.abs(Ad - A).max() > 1.0


@pytest.mark.parametrize("seed", [9000, 9001, 9002])
def test_paper2d_operator_is_singular_psd_with_constant_null_space(seed):
    fr = inputs.make_frame("paper2d_1024", seed)
    A = grid.assemble(fr.nx, fr.ny, fr.nz, fr.rho, neumann=True)
    dA = A.diagonal()
    assert np.abs(A @ np.ones(fr.n)).max() <= 1e-12 * dA.max()
    Ad = A.toarray()
    assert np.array_equal(Ad, Ad.T)
    ev = np.linalg.eigvalsh(Ad)
    assert abs(ev[0]) <= 1e-11 * ev[-1]
    assert ev[1] > 1e-6 * ev[-1]          # connected grid: one zero eigenvalue


def test_paper2d_generator_properties():
    for n, (w, h) in inputs.GRID2D_OF_N.items():
        for seed in range(4):
            fr = inputs.make_frame(f"paper2d_{n}", seed)
            assert (fr.nx, fr.ny, fr.nz, fr.neumann) == (w, h, 1, True)
            assert abs(fr.b.mean()) <= 1e-14
            assert 0.5 < fr.b.std() < 1.5
            heavy = fr.rho > 2.5                  # rho_heavy >= 5, noise 5 %
            assert heavy.any() and (~heavy).any()
            assert np.abs(fr.rho[~heavy] - 1.0).max() < 0.3
            assert fr.rho[heavy].max() < 100 * 1.3
    # the same seed draws the same frame
    a, b = inputs.make_frame("paper2d_2048", 7), inputs.make_frame("paper2d_2048", 7)
    assert np.array_equal(a.rho, b.rho) and np.array_equal(a.b, b.b)


def test_paper2d_features_use_the_neumann_diagonal():
    fr = inputs.make_frame("paper2d_1024", 9000)
    f = grid.features(fr.nx, fr.ny, fr.nz, fr.rho, neumann=True)
    A = grid.assemble(fr.nx, fr.ny, fr.nz, fr.rho, neumann=True)
    assert np.allclose(f[:, 7], np.log(A.diagonal()), rtol=0, atol=1e-14)
    assert (f[:, 4] == 1).all() and (f[:, 6] == 1).all()     # one layer: top and bottom
    xyz = grid.positions(fr.nx, fr.ny, fr.nz)
    side = (xyz[:, 0] == 0) | (xyz[:, 0] == fr.nx - 1) | (xyz[:, 1] == 0) | (xyz[:, 1] == fr.ny - 1)
    assert np.array_equal(f[:, 5] == 1, side)
    fs = network.FrameSys(fr.nx, fr.ny, fr.nz, fr.rho, 64, 16, neumann=True)
    assert np.array_equal(fs.A.toarray(), A.toarray())


@pytest.mark.parametrize("precond", ["none", "jacobi"])
def test_pcg_on_the_singular_system_reaches_the_min_norm_solution(precond):
    """b is mean-zero, hence in the range of A: PCG reaches rtol 1e-8 and x
    minus its mean is the minimum-norm solution A^+ b (dense least squares),
    within kappa * rtol of the restricted operator."""
    fr = inputs.make_frame("paper2d_1024", 9003)
    A = grid.assemble(fr.nx, fr.ny, fr.nz, fr.rho, neumann=True)
    b = fr.b[grid.morton_perm(fr.nx, fr.ny, fr.nz)]
    M = None if precond == "none" else pcg.jacobi(A)
    x, k, flags, hist = pcg.pcg(A, b, M, tol=1e-8, max_iter=20000, stagnation=False)
    assert flags == pcg.CONVERGED
    assert np.linalg.norm(b - A @ x) <= 1e-8 * np.linalg.norm(b)
    Ad = A.toarray()
    xmn = np.linalg.lstsq(Ad, b, rcond=None)[0]
    assert abs(xmn.mean()) <= 1e-10 * np.abs(xmn).max()
    ev = np.linalg.eigvalsh(Ad)
    kappa = ev[-1] / ev[1]
    err = np.linalg.norm((x - x.mean()) - xmn) / np.linalg.norm(xmn)
    print(f"{precond}: {k} iterations, kappa {kappa:.3g}, error vs A^+ b {err:.2e}")
    assert err <= kappa * 1e-8
    if precond == "none":
        # CG from 0 stays in the range of A: x keeps mean zero
        assert abs(x.mean()) <= 1e-10 * np.abs(x).max()
