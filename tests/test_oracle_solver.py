"""Pins of the oracle's H-matrix apply and PCG (CPU only)."""
import math

import numpy as np
import pytest
import scipy.linalg
import scipy.sparse.linalg as spla

from oracle import grid, hmatrix, partition, pcg
from paper_2605_13343_amd import inputs


def _rand_factors(part, seed, scale_B=1.0):
    rng = np.random.default_rng(seed)
    K, L, Ls, n, MH = part["K"], part["L"], part["Ls"], part["n"], part["MH"]
    F = rng.standard_normal((K, L, L)) / math.sqrt(L)
    B = rng.standard_normal((MH, Ls, Ls)) * scale_B
    Ut = rng.standard_normal((n, Ls)) / math.sqrt(L)
    Vt = rng.standard_normal((n, Ls)) / math.sqrt(L)
    lam = rng.uniform(0.1, 1.0, n)
    dA = rng.uniform(0.5, 5.0, n)
    return hmatrix.gram(F), B, Ut, Vt, lam, dA


def _bruteforce_M(part, G, B, Ut, Vt, lam, dA):
    """Entry-by-entry M: leaf pair (k, k') with k < k' sits in the tile at
    level j = highest differing bit, index i = k >> (j+1) within the level."""
    n, L, K = part["n"], part["L"], part["K"]
    M = np.zeros((n, n))
    for k in range(K):
        for k2 in range(K):
            if k == k2:
                M[k * L:(k + 1) * L, k * L:(k + 1) * L] = G[k]
                continue
            lo, hi = min(k, k2), max(k, k2)
            j = (lo ^ hi).bit_length() - 1
            m = K - K // (1 << j) + (lo >> (j + 1))
            blk = Ut[lo * L:(lo + 1) * L] @ B[m] @ Vt[hi * L:(hi + 1) * L].T
            if k < k2:
                M[k * L:(k + 1) * L, k2 * L:(k2 + 1) * L] = blk
            else:
                M[k * L:(k + 1) * L, k2 * L:(k2 + 1) * L] = blk.T
    M[np.arange(n), np.arange(n)] += lam / dA
    return M


@pytest.mark.parametrize("n,L,Ls", [(256, 32, 8), (512, 64, 16), (64, 64, 16), (128, 32, 8)])
def test_apply_equals_explicit_and_bruteforce(n, L, Ls):
    part = partition.build(n, L, Ls)
    G, B, Ut, Vt, lam, dA = _rand_factors(part, n)
    M = hmatrix.explicit_M(part, G, B, Ut, Vt, lam, dA)
    Mb = _bruteforce_M(part, G, B, Ut, Vt, lam, dA)
    assert np.allclose(M, Mb, rtol=0, atol=1e-12)
    assert np.allclose(M, M.T, rtol=0, atol=1e-12)
    R = np.random.default_rng(1).standard_normal((n, 3))
    Y = hmatrix.apply(part, G, B, Ut, Vt, lam, dA, R)
    assert np.abs(Y - M @ R).max() <= 1e-12 * np.abs(M @ R).max()
    y0 = hmatrix.apply(part, G, B, Ut, Vt, lam, dA, R[:, 0])
    assert np.allclose(y0, Y[:, 0], rtol=0, atol=1e-13)


def test_apply_special_cases():
    part = partition.build(64, 64, 16)            # K = 1: no tiles
    G, B, Ut, Vt, lam, dA = _rand_factors(part, 3)
    assert part["MH"] == 0
    M = hmatrix.explicit_M(part, G, B, Ut, Vt, lam, dA)
    assert np.allclose(M, G[0] + np.diag(lam / dA))
    part = partition.build(512, 64, 16)           # zero coupling -> block diagonal
    G, B, Ut, Vt, lam, dA = _rand_factors(part, 4, scale_B=0.0)
    M = hmatrix.explicit_M(part, G, B, Ut, Vt, lam, dA)
    assert np.allclose(M, scipy.linalg.block_diag(*G) + np.diag(lam / dA))


def _c1_system():
    fr = inputs.make_frame("plain1024", 1000)
    A = grid.assemble(fr.nx, fr.ny, fr.nz, fr.rho)
    b = fr.b[grid.morton_perm(fr.nx, fr.ny, fr.nz)]
    return A, b


def test_cg_matches_scipy_iterates():
    A, b = _c1_system()
    ref = []
    spla.cg(A, b, rtol=1e-30, maxiter=20, callback=lambda xk: ref.append(xk.copy()))
    for k in range(1, 21):
        x, it, fl, _ = pcg.pcg(A, b, None, tol=1e-30, max_iter=k, recompute_every=0)
        assert it == k
        assert np.linalg.norm(x - ref[k - 1]) <= 1e-10 * np.linalg.norm(ref[k - 1])


def test_pcg_exact_inverse_one_iteration():
    fr = inputs.make_frame_grid(8, 4, 4, 5)
    A = grid.assemble(fr.nx, fr.ny, fr.nz, fr.rho)
    Ainv = np.linalg.inv(A.toarray())
    # every iteration replaces r by b - A x, so the first residual is a true one
    x, it, fl, h = pcg.pcg(A, fr.b, lambda r: Ainv @ r, tol=1e-10, recompute_every=1)
    assert it == 1 and fl == pcg.CONVERGED and h[1] < 1e-13


def test_jacobi_is_cg_on_scaled_system():
    A, b = _c1_system()
    d = A.diagonal()
    s = 1.0 / np.sqrt(d)
    As = (A.multiply(s[:, None]).multiply(s[None, :])).tocsr()
    for k in (1, 5, 17):
        xj, _, _, _ = pcg.pcg(A, b, pcg.jacobi(A), tol=1e-30, max_iter=k, recompute_every=0)
        y, _, _, _ = pcg.pcg(As, s * b, None, tol=1e-30, max_iter=k, recompute_every=0)
        assert np.linalg.norm(xj - s * y) <= 1e-10 * np.linalg.norm(xj)


def test_pcg_error_monotone_and_bound():
    A, b = _c1_system()
    Ad = A.toarray()
    xs = scipy.linalg.cho_solve(scipy.linalg.cho_factor(Ad), b)
    ev = np.linalg.eigvalsh(Ad)
    kappa = ev[-1] / ev[0]
    errs = []
    for k in range(1, 60, 3):
        x, _, _, _ = pcg.pcg(A, b, pcg.jacobi(A), tol=1e-30, max_iter=k, recompute_every=25)
        e = x - xs
        errs.append(math.sqrt(e @ Ad @ e))
    assert all(errs[i + 1] <= errs[i] * (1 + 1e-9) for i in range(len(errs) - 1))
    x, it, fl, h = pcg.pcg(A, b, pcg.jacobi(A), tol=1e-6)
    assert fl == pcg.CONVERGED
    assert np.linalg.norm(b - A @ x) / np.linalg.norm(b) <= 1e-6
    e = x - xs
    assert math.sqrt(e @ Ad @ e) / math.sqrt(xs @ Ad @ xs) <= math.sqrt(kappa) * 1e-6


def test_pcg_flags():
    A, b = _c1_system()
    x, it, fl, _ = pcg.pcg(A, b, lambda r: -r, tol=1e-6)
    assert fl == pcg.NOT_SPD and it == 0
    x, it, fl, _ = pcg.pcg(A, b, None, tol=1e-30, max_iter=5000)
    assert fl == pcg.STAGNATED and it % 100 == 0
    x, it, fl, _ = pcg.pcg(A, b, None, tol=1e-6, max_iter=7)
    assert fl == pcg.MAXITER and it == 7
    # fallback: an indefinite "preconditioner" hands over to Jacobi-PCG
    x, it, fl, _ = pcg.solve_with_fallback(A, b, lambda r: -r, tol=1e-6)
    assert fl & pcg.FELL_BACK and fl & pcg.CONVERGED and fl & pcg.NOT_SPD
    assert np.linalg.norm(b - A @ x) / np.linalg.norm(b) <= 1e-6


def _weak_diagonal_M(n, spread=4.0, seed=7):
    """An SPD preconditioner that preconditions badly: a diagonal with
    entries spread over 2 * spread decades."""
    d = 10.0 ** np.random.default_rng(seed).uniform(-spread, spread, n)
    return lambda r: d * r


def test_fallback_on_stagnation_and_iteration_cap():
    A, b = _c1_system()
    M = _weak_diagonal_M(A.shape[0])
    # less than a 2x drop over the first 100 iterations: STAGNATED at 100
    _, k, fl, h = pcg.pcg(A, b, M, tol=1e-6)
    assert fl == pcg.STAGNATED and k == 100 and h[100] > 0.5 * h[0]
    x, it, fl, _ = pcg.solve_with_fallback(A, b, M, tol=1e-6)
    assert fl == pcg.STAGNATED | pcg.FELL_BACK | pcg.CONVERGED and it > 100
    assert np.linalg.norm(b - A @ x) / np.linalg.norm(b) <= 1e-6
    # the warm start counts: Jacobi from x needs fewer iterations than from 0
    _, kj, _, _ = pcg.pcg(A, b, pcg.jacobi(A), tol=1e-6)
    assert it - 100 <= kj
    # the cap: MAXITER hands over as well, to a Jacobi pass with the same cap
    x, it, fl, _ = pcg.solve_with_fallback(A, b, M, tol=1e-6, max_iter=120, stagnation=False)
    assert fl == pcg.MAXITER | pcg.FELL_BACK | pcg.CONVERGED and 120 < it <= 240
    assert np.linalg.norm(b - A @ x) / np.linalg.norm(b) <= 1e-6


@pytest.mark.parametrize("scale", [1e-3, 1.0, 1e3])
def test_pcg_is_invariant_to_the_scale_of_b(scale):
    """PCG is linear in b: scaling b by c scales every iterate and residual by
    c, so iterations and flags (convergence, the stagnation windows, which
    compare ||r_k|| with ||r_(k-100)||) do not depend on c.  A frame of the
    paper's 2D benchmark with Jacobi to 1e-8 crosses the k = 100 window."""
    fr = inputs.make_frame("paper2d_1024", 9100)
    A = grid.assemble(fr.nx, fr.ny, fr.nz, fr.rho, neumann=True)
    b = fr.b[grid.morton_perm(fr.nx, fr.ny, fr.nz)]
    x1, k1, f1, _ = pcg.pcg(A, b, pcg.jacobi(A), tol=1e-8)
    xs, ks, fs, _ = pcg.pcg(A, scale * b, pcg.jacobi(A), tol=1e-8)
    assert k1 > 100 and f1 == pcg.CONVERGED
    assert (ks, fs) == (k1, f1)
    assert np.allclose(xs, scale * x1, rtol=1e-9, atol=1e-12 * scale * np.abs(x1).max())


def test_fp32_vector_pcg_tracks_fp64_then_still_meets_the_true_residual():
    """The precision split (float32 r, z, p, q; float64 x and scalars): the
    first iterates equal the float64 ones to float32 accuracy (no residual
    replacement), and a full solve still stops on a float64 true residual
    below the target, in at most a few more iterations."""
    fr = inputs.make_frame("paper2d_1024", 9100)
    A = grid.assemble(fr.nx, fr.ny, fr.nz, fr.rho, neumann=True)
    b = fr.b[grid.morton_perm(fr.nx, fr.ny, fr.nz)]
    M = pcg.jacobi(A)
    for k in (1, 3, 10):
        x64, _, _, _ = pcg.pcg(A, b, M, tol=0.0, max_iter=k, recompute_every=0, stagnation=False)
        x32, _, _, _ = pcg.pcg(A, b, M, tol=0.0, max_iter=k, recompute_every=0, stagnation=False,
                               fp32_iteration=True)
        assert np.linalg.norm(x32 - x64) / np.linalg.norm(x64) <= 4 * k * 2.0 ** -24, k
        assert not np.array_equal(x32, x64)        # the rounding does act
    x64, k64, f64, _ = pcg.pcg(A, b, None, tol=1e-8, max_iter=5000, stagnation=False)
    x32, k32, f32_, _ = pcg.pcg(A, b, None, tol=1e-8, max_iter=5000, stagnation=False, fp32_iteration=True)
    assert f64 == f32_ == pcg.CONVERGED
    assert np.linalg.norm(b - A @ x32) <= 1e-8 * np.linalg.norm(b)
    assert k64 <= k32 <= 1.2 * k64
