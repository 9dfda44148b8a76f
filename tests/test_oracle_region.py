"""Pins of the oracle's padded frames (paper Sec. 8: the partition is sized
to a maximum N and smaller frames are padded to it; Supplementary "Grid and
ordering": a W x H grid with W H >= N cut to its first N cells in Morton
order).  A frame keeps a power-of-two box; its own cells are the first n
cells of a W x H x D grid in Morton order; every other cell of the box is an
identity row.  Checked against what fixes these objects independently of the
oracle's code: a Morton code written here by magic-mask bit spreading, an
assembly by brute force over the cell set, the operator of the sub-grid on
its own (the pinned plain assembly), and direct solves (CPU only)."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle import grid, network, pcg
from paper_2605_13343_amd import hp, inputs


def _spread3(v):
    v &= 0x3FF
    v = (v | (v << 16)) & 0x030000FF
    v = (v | (v << 8)) & 0x0300F00F
    v = (v | (v << 4)) & 0x030C30C3
    v = (v | (v << 2)) & 0x09249249
    return v


def _code(x, y, z):
    return _spread3(x) | (_spread3(y) << 1) | (_spread3(z) << 2)


def _own_cells(W, H, D, n):
    """The first n cells of the W x H x D grid by this file's Morton code."""
    cells = sorted(((x, y, z) for z in range(D) for y in range(H) for x in range(W)), key=lambda c: _code(*c))
    return set(cells[:n])


CASES = [((4, 2, 1), (3, 2, 1, 5)), ((16, 16, 1), (11, 9, 1, 90)), ((16, 16, 1), (16, 13, 1, 208)),
         ((32, 32, 1), (25, 24, 1, 600)), ((8, 8, 4), (7, 5, 3, 100)), ((16, 16, 8), (12, 10, 6, 720)),
         ((16, 8, 8), (9, 8, 8, 576)), ((64, 64, 1), (46, 45, 1, 2048))]


@pytest.mark.parametrize("box,region", CASES)
def test_region_mask_is_the_first_cells_in_morton_order(box, region):
    nx, ny, nz = box
    own = _own_cells(*region)
    mask = grid.region_mask_lex(nx, ny, nz, region)
    exp = np.zeros(nx * ny * nz, dtype=bool)
    for (x, y, z) in own:
        exp[x + nx * (y + ny * z)] = True
    assert np.array_equal(mask, exp)
    assert mask.sum() == region[3]
    # the library's host mask (Morton order of the box) is the same set
    perm = grid.morton_perm(nx, ny, nz)
    assert np.array_equal(hp.region_mask(nx, ny, nz, region), mask[perm])


def test_region_mask_rejects_what_does_not_fit():
    with pytest.raises(ValueError):
        grid.region_mask_lex(8, 8, 1, (9, 8, 1, 10))
    with pytest.raises(ValueError):
        grid.region_mask_lex(8, 8, 1, (4, 4, 1, 17))
    for reg in ((9, 8, 1, 10), (4, 4, 1, 17), (4, 4, 1, 0), (4, 4, 2, 8)):
        with pytest.raises(RuntimeError):
            hp.region_mask(8, 8, 1, reg)
    with pytest.raises(RuntimeError):           # the box itself must be one the library admits
        hp.region_mask(12, 8, 1, (4, 4, 1, 8))


def test_region_assembly_hand_values():
    """3 x 2 grid in a 4 x 2 box cut to 5 cells: Morton codes of the grid are
    (0,0) 0, (1,0) 1, (0,1) 2, (1,1) 3, (2,0) 8, (2,1) 10, so (2,1) is cut.
    Lexicographic ids 0..7 = (0,0) (1,0) (2,0) (3,0) (0,1) (1,1) (2,1) (3,1);
    rho = 1, 2, 4, 9, 3, 6, 7, 5.  Zero-flux operator, w = 2 ri rj / (ri + rj)."""
    rho = np.array([1.0, 2.0, 4.0, 9.0, 3.0, 6.0, 7.0, 5.0])
    A = grid.assemble_lex(4, 2, 1, rho, neumann=True, region=(3, 2, 1, 5)).toarray()
    h = lambda a, b: 2 * a * b / (a + b)
    w01, w12, w04, w15, w45 = h(1, 2), h(2, 4), h(1, 3), h(2, 6), h(3, 6)
    ref = np.eye(8)
    ref[0, 0], ref[0, 1], ref[0, 4] = w01 + w04, -w01, -w04
    ref[1, 0], ref[1, 1], ref[1, 2], ref[1, 5] = -w01, w01 + w12 + w15, -w12, -w15
    ref[2, 1], ref[2, 2] = -w12, w12
    ref[4, 0], ref[4, 4], ref[4, 5] = -w04, w04 + w45, -w45
    ref[5, 1], ref[5, 4], ref[5, 5] = -w15, -w45, w15 + w45
    assert np.allclose(A, ref, rtol=1e-15, atol=0)
    # the Dirichlet operator: w = 2 / (ri + rj), + 1/rho on the grid's top
    # layer (one layer: every own cell), padding rows still identity rows
    Ad = grid.assemble_lex(4, 2, 1, rho, neumann=False, region=(3, 2, 1, 5)).toarray()
    g = lambda a, b: 2 / (a + b)
    faces = {(0, 1): g(1, 2), (1, 2): g(2, 4), (0, 4): g(1, 3), (1, 5): g(2, 6), (4, 5): g(3, 6)}
    refd = np.eye(8)
    for i in (0, 1, 2, 4, 5):
        refd[i, i] = 1 / rho[i]
    for (i, j), w in faces.items():
        refd[i, j] = refd[j, i] = -w
        refd[i, i] += w
        refd[j, j] += w
    assert np.allclose(Ad, refd, rtol=1e-15, atol=0)


@pytest.mark.parametrize("box,neumann", [((8, 8, 4), False), ((16, 16, 1), True), ((16, 8, 8), False)])
def test_whole_box_region_is_the_plain_operator(box, neumann):
    nx, ny, nz = box
    rho = np.random.default_rng(3).uniform(0.5, 50.0, nx * ny * nz)
    A0 = grid.assemble(nx, ny, nz, rho, neumann)
    A1 = grid.assemble(nx, ny, nz, rho, neumann, region=(nx, ny, nz, nx * ny * nz))
    assert (A0 != A1).nnz == 0


def _embed(box, W, H, D):
    """Lexicographic id in the box of each lexicographic cell of the W x H x D grid."""
    nx, ny, _ = box
    return np.array([x + nx * (y + ny * z) for z in range(D) for y in range(H) for x in range(W)])


@pytest.mark.parametrize("box,region,neumann", [((16, 16, 8), (12, 10, 6, 720), False),
                                                ((8, 8, 4), (5, 7, 4, 140), False),
                                                ((32, 32, 1), (25, 24, 1, 600), True)])
def test_untruncated_region_block_is_the_subgrid_operator(box, region, neumann):
    """With every grid cell kept, the frame's block is the plain operator of
    the W x H x D grid on its own (Dirichlet layer on its top z = D-1), the
    padding block is I and nothing couples the two."""
    nx, ny, nz = box
    W, H, D, n = region
    rho = np.random.default_rng(5).uniform(0.5, 100.0, nx * ny * nz)
    A = grid.assemble_lex(nx, ny, nz, rho, neumann, region).toarray()
    ids = _embed(box, W, H, D)
    sub = grid.assemble_lex(W, H, D, rho[ids], neumann).toarray()
    assert np.array_equal(A[np.ix_(ids, ids)], sub)
    pad = np.setdiff1d(np.arange(nx * ny * nz), ids)
    assert np.array_equal(A[np.ix_(pad, pad)], np.eye(len(pad)))
    assert not A[np.ix_(ids, pad)].any() and not A[np.ix_(pad, ids)].any()


@pytest.mark.parametrize("box,region,neumann", [((16, 16, 1), (11, 9, 1, 90), True),
                                                ((16, 16, 1), (11, 9, 1, 90), False),
                                                ((8, 8, 4), (7, 5, 3, 100), False),
                                                ((32, 32, 1), (25, 24, 1, 600), True)])
def test_truncated_region_matches_brute_force_assembly(box, region, neumann):
    """Faces only between two own cells, the Dirichlet term on the grid's top
    layer, identity rows elsewhere, by a loop over the cell set."""
    nx, ny, nz = box
    W, H, D, n = region
    rho = np.random.default_rng(7).uniform(0.5, 100.0, nx * ny * nz)
    own = _own_cells(*region)
    lid = lambda c: c[0] + nx * (c[1] + ny * c[2])
    N = nx * ny * nz
    ref = np.eye(N)
    for c in own:
        i = lid(c)
        ref[i, i] = 0.0
    for c in own:
        i = lid(c)
        for d in ((1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1)):
            q = (c[0] + d[0], c[1] + d[1], c[2] + d[2])
            if q in own:
                j = lid(q)
                w = 2 * rho[i] * rho[j] / (rho[i] + rho[j]) if neumann else 2 / (rho[i] + rho[j])
                ref[i, j] = -w
                ref[i, i] += w
        if not neumann and c[2] == D - 1:
            ref[i, i] += 1 / rho[i]
    A = grid.assemble_lex(nx, ny, nz, rho, neumann, region).toarray()
    assert np.allclose(A, ref, rtol=1e-14, atol=0)


def test_padded_dirichlet_solve_is_the_subgrid_solve():
    """PCG (Jacobi) on the padded system: x on the frame's cells solves the
    sub-grid system (direct sparse solve of its own plain operator), x on the
    padding stays 0 (b is 0 there and Jacobi never mixes cells)."""
    box, region = (16, 16, 8), (12, 10, 6, 720)
    fr = inputs.make_padded_frame(box, region, seed=11)
    nx, ny, nz = box
    A = grid.assemble_lex(nx, ny, nz, fr.rho, False, region).tocsr()
    b = grid.region_rhs(nx, ny, nz, fr.b, region, False)
    x, k, flags, _ = pcg.pcg(A, b, pcg.jacobi(A), tol=1e-10, max_iter=5000)
    assert flags == pcg.CONVERGED
    ids = _embed(box, *region[:3])
    sub = grid.assemble_lex(*region[:3], fr.rho[ids], False).tocsc()
    xs = spla.spsolve(sub, fr.b[ids])
    assert np.linalg.norm(x[ids] - xs) <= 1e-8 * np.linalg.norm(xs)
    pad = np.setdiff1d(np.arange(nx * ny * nz), ids)
    assert not x[pad].any()


def test_padded_neumann_solve_on_the_truncated_paper_grid():
    """The paper's 2048-cell grid (46 x 45 cut to 2,048 cells, in a 64 x 64
    box), zero-flux operator: the frame's block is singular with the constant
    on its cells as null space; b is consistent (mean-zero there); PCG
    reaches rtol 1e-8 and its mean-free part on the frame's cells is the
    minimum-norm solution of the frame's block (dense least squares)."""
    fr = inputs.make_frame("paper2d_trunc_2048", 9003)
    assert (fr.nx, fr.ny, fr.region) == (64, 64, (46, 45, 1, 2048))
    A = grid.assemble_lex(fr.nx, fr.ny, 1, fr.rho, True, fr.region).tocsr()
    b = grid.region_rhs(fr.nx, fr.ny, 1, fr.b, fr.region, True)
    real = grid.region_mask_lex(fr.nx, fr.ny, 1, fr.region)
    assert np.abs(A @ real.astype(float)).max() <= 1e-12 * A.diagonal().max()
    assert abs(b[real].sum()) <= 1e-12 * np.abs(b).sum() and not b[~real].any()
    x, k, flags, _ = pcg.pcg(A, b, pcg.jacobi(A), tol=1e-8, max_iter=20000, stagnation=False)
    assert flags == pcg.CONVERGED
    Ar = A[real][:, real].toarray()
    ev = np.linalg.eigvalsh(Ar)
    assert abs(ev[0]) <= 1e-11 * ev[-1] and ev[1] > 1e-8 * ev[-1]    # connected: one zero eigenvalue
    xmn = np.linalg.lstsq(Ar, b[real], rcond=None)[0]
    xr = x[real]
    err = np.linalg.norm((xr - xr.mean()) - xmn) / np.linalg.norm(xmn)
    assert err <= (ev[-1] / ev[1]) * 1e-8
    assert not x[~real].any()


def test_truncated_generator_and_features():
    """The generator's padded frames: heavy cells only inside the W x H grid,
    the box outside it light; the oracle's features of a padded frame are
    those of the whole box with the padded operator's diagonal (1 on the
    padding)."""
    for n, ((W, H), box) in inputs.TRUNC2D_OF_N.items():
        assert W * H >= n and W - 1 <= H <= W and (W - 1) * H < n
        fr = inputs.make_frame(f"paper2d_trunc_{n}", 1)
        rho = fr.rho.reshape(box[1], box[0])
        assert (rho[H:, :] == 1.0).all() and (rho[:, W:] == 1.0).all()
        assert (rho[:H, :W] > 2.5).any()
    fr = inputs.make_frame("paper2d_trunc_2048", 9001)
    f = grid.features(fr.nx, fr.ny, 1, fr.rho, True, fr.region)
    A = grid.assemble(fr.nx, fr.ny, 1, fr.rho, True, fr.region)
    assert np.allclose(f[:, 7], np.log(A.diagonal()), rtol=0, atol=1e-14)
    real = hp.region_mask(fr.nx, fr.ny, 1, fr.region)
    assert (f[~real, 7] == 0).all()
    fs = network.FrameSys(fr.nx, fr.ny, 1, fr.rho, 64, 16, True, fr.region)
    assert (fs.A != A).nnz == 0 and fs.n == 4096
