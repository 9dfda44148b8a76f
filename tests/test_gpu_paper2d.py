"""GPU parity on the paper's own 2D benchmark (Sec. 7.1 "Benchmark";
Supplementary "Multiphase Poisson Benchmark Generation", "Operator assembly",
"Convergence criterion"): the zero-flux 5-point operator with the harmonic
mean of rho as conductance (hp_assemble_ops), its SpMV, and PCG to the
paper's relative residual 1e-8 on the singular system, against the float64
oracle."""
import numpy as np
import pytest

from oracle import hmatrix, pcg as opcg
from paper_2605_13343_amd import hp, inputs
from tests.gpu_helpers import Side, relerr

pytestmark = pytest.mark.gpu

DEF = inputs.MODEL_DEFAULT
RTOL = 1e-8


def _frames():
    return ([inputs.make_frame("paper2d_1024", 9100 + i) for i in range(2)]
            + [inputs.make_frame("paper2d_2048", 9110), inputs.make_frame("paper2d_4096", 9120)])


def test_paper2d_assemble_matches_oracle():
    import torch
    s = Side(DEF, _frames())
    assert s.ops == hp.ASM_PAPER
    nt = s.B.ntot
    sys = s.sys[:5 * nt].double().cpu().numpy().reshape(5, -1)
    sys8 = s.sys[5 * nt:].view(torch.float64).cpu().numpy().reshape(4, -1)
    for f, fr in enumerate(s.frames):
        A = s.A[f].tocsr()
        rows = s.rows(f)
        d = A.diagonal()
        assert relerr(sys[0, rows], d) <= 2e-7
        assert relerr(sys[4, rows], 1.0 / d) <= 2e-7
        assert relerr(sys8[0, rows], d) <= 1e-15
        # FP64 row sums of the device operator vanish: A 1 = 0
        wx, wy = sys8[1, rows], sys8[2, rows]
        assert not sys8[3, rows].any()                       # no z faces on one layer
        from oracle import grid
        pos = grid.positions(fr.nx, fr.ny, fr.nz).astype(int)
        inv = {tuple(p): i for i, p in enumerate(pos)}
        for ax, step, w in ((1, (1, 0, 0), wx), (2, (0, 1, 0), wy)):
            exp = np.zeros(fr.n)
            for i, p in enumerate(pos):
                q = tuple(p + np.array(step))
                if q in inv:
                    exp[i] = -A[i, inv[q]]
            assert relerr(sys[ax, rows], exp) <= 2e-7
            assert relerr(w, exp) <= 1e-15
        assert np.abs(A @ np.ones(fr.n)).max() <= 1e-12 * d.max()


def test_paper2d_spmv_matches_oracle():
    import torch
    s = Side(DEF, _frames())
    rng = np.random.default_rng(0)
    p = rng.standard_normal(s.B.ntot).astype(np.float32)
    q = torch.zeros_like(s.b)
    s.B.spmv(s.sys, torch.tensor(p, device="cuda"), q)
    for f, qf in enumerate(s.split(q)):
        assert relerr(qf, s.A[f] @ p[s.rows(f)].astype(np.float64)) <= 1e-6
    # the constant vector is in the null space on the device too
    ones = torch.ones_like(s.b)
    s.B.spmv(s.sys, ones, q)
    for f, qf in enumerate(s.split(q)):
        assert np.abs(qf).max() <= 1e-5 * float(s.A[f].diagonal().max())


def _solve(s, precond, fac=None, **kw):
    import torch
    x = torch.zeros(s.B.ntot, dtype=torch.float64, device="cuda")
    res = s.B.pcg_solve(s.sys, fac, s.b, x, precond, tol=RTOL, **kw)
    return x, res


def _centred_err(x, xo):
    """Solutions of the singular system differ by constants: compare the
    mean-free parts."""
    a, b = x - x.mean(), xo - xo.mean()
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _kappa(A):
    ev = np.linalg.eigvalsh(A.toarray())
    return ev[-1] / ev[1]            # on the range of A (ev[0] = 0)


# Iteration counts at rtol 1e-8: the device iterates with the FP32 copy of A
# and FP32 vectors (the paper's precision split) and judges the stop on the
# FP64 true residual, which costs iterations against a float64 PCG (54 -> 60
# on one frame here, almost all from the rounded operator).  The oracle's PCG
# with fp32_iteration follows the same split; the device matches it within
# 2 % (at least 3), and the float64 oracle within `frac`.
def _iters_ok(it, k32, ko, frac):
    return abs(it - k32) <= max(3, int(0.02 * k32)) and abs(it - ko) <= max(3, int(frac * ko))


@pytest.mark.parametrize("precond,frac", [(hp.PRECOND_JACOBI, 0.05), (hp.PRECOND_NONE, 0.15)])
def test_paper2d_pcg_classic_matches_oracle(precond, frac):
    s = Side(DEF, _frames())
    x, res = _solve(s, precond, stagnation=False, max_iter=20000)
    rows = []
    for f, xf in enumerate(s.split(x)):
        A, b = s.A[f], s.bo[f]
        M = opcg.jacobi(A) if precond == hp.PRECOND_JACOBI else None
        xo, ko, flo, _ = opcg.pcg(A, b, M, tol=RTOL, max_iter=20000, stagnation=False)
        _, k32, fl32, _ = opcg.pcg(A, b, M, tol=RTOL, max_iter=20000, stagnation=False, fp32_iteration=True)
        it, fl, rr = res[f]
        true = np.linalg.norm(b - A @ xf) / np.linalg.norm(b)
        kap = _kappa(A) if s.frames[f].n <= 2048 else None
        xe = _centred_err(xf, xo)
        print(f"precond {precond} frame {f} N={s.frames[f].n} gpu {it} oracle fp32-iteration {k32} fp64 {ko} "
              f"true relres {true:.3e} x err {xe:.2e} kappa {kap}")
        rows.append((f, it, fl, k32, fl32, ko, flo, true, xe, kap))
    for f, it, fl, k32, fl32, ko, flo, true, xe, kap in rows:
        assert fl & hp.CONVERGED and flo == fl32 == opcg.CONVERGED, (f, fl, flo, fl32)
        assert _iters_ok(it, k32, ko, frac), (f, it, k32, ko)
        assert true <= RTOL, (f, true)
        if kap is not None:
            # both stop within rtol of the range solution: error <= 2 kappa rtol
            assert xe <= 2 * kap * RTOL, (f, xe, kap)


def _block_jacobi_factors(part, A, seed):
    """Leaf blocks G_k = A_kk^-1 (SPD: a proper principal block of the
    singular, irreducible M-matrix A is nonsingular), a small random
    coupling and Jacobi gate: an SPD M that cuts iterations well below
    Jacobi's, so no stagnation window comes near its threshold."""
    rng = np.random.default_rng(seed)
    K, L, Ls, n, MH = part["K"], part["L"], part["Ls"], part["n"], part["MH"]
    Ad = A.toarray()
    G = np.stack([np.linalg.inv(Ad[k * L:(k + 1) * L, k * L:(k + 1) * L]) for k in range(K)])
    Bm = rng.standard_normal((MH, Ls, Ls)) * 2e-4 / float(np.median(A.diagonal()))
    Ut = rng.standard_normal((n, Ls)) / np.sqrt(L)
    Vt = rng.standard_normal((n, Ls)) / np.sqrt(L)
    lam = rng.uniform(0.0, 0.2, n)
    return G, Bm, Ut, Vt, lam


def test_paper2d_hmat_pcg_matches_oracle():
    """PCG with held H-matrix factors (FP32) to rtol 1e-8 on the singular
    systems: flags, iterations, true residual and the mean-free solution
    against the oracle's float64 PCG with the same factors."""
    s = Side(DEF, _frames())
    facs = [_block_jacobi_factors(p, A, 40 + i) for i, (p, A) in enumerate(zip(s.parts, s.A))]
    fac, held = s.upload_factors(facs, hp.HP_F32)
    x, res = _solve(s, hp.PRECOND_HMAT, fac, fdtype=hp.HP_F32, max_iter=20000)
    rows = []
    for f, xf in enumerate(s.split(x)):
        A, b = s.A[f], s.bo[f]
        G, Bm, Ut, Vt, lam = held[f]
        dA = A.diagonal()
        Mf = lambda v: hmatrix.apply(s.parts[f], G, Bm, Ut, Vt, lam, dA, v)
        xo, ko, flo, _ = opcg.solve_with_fallback(A, b, Mf, tol=RTOL, max_iter=20000)
        _, k32, fl32, _ = opcg.solve_with_fallback(A, b, Mf, tol=RTOL, max_iter=20000, fp32_iteration=True)
        it, fl, rr = res[f]
        true = np.linalg.norm(b - A @ xf) / np.linalg.norm(b)
        xe = _centred_err(xf, xo)
        print(f"hmat frame {f} N={s.frames[f].n} gpu {it} flags {fl} oracle fp32-iteration {k32} fp64 {ko} "
              f"flags {flo} true {true:.3e} x err {xe:.2e}")
        rows.append((f, it, fl, k32, fl32, ko, flo, true, xe))
    for f, it, fl, k32, fl32, ko, flo, true, xe in rows:
        assert fl == flo == fl32 == hp.CONVERGED, (f, fl, flo, fl32)
        assert _iters_ok(it, k32, ko, 0.15), (f, it, k32, ko)
        assert true <= RTOL, (f, true)
        if s.frames[f].n <= 2048:
            assert xe <= 2 * _kappa(s.A[f]) * RTOL, (f, xe)


def test_paper2d_apply_matches_oracle():
    """y = M r on the one-layer frames (FP32 and BF16 factors) against the
    oracle's chain apply with the factors as the device holds them."""
    import torch
    from tests.gpu_helpers import rand_factors
    s = Side(DEF, _frames())
    for dtype in (hp.HP_F32, hp.HP_BF16):
        facs = [rand_factors(p, 10 + i, b_scale=1.0) for i, p in enumerate(s.parts)]
        fac, held = s.upload_factors(facs, dtype)
        r = np.random.default_rng(1).standard_normal(s.B.ntot).astype(np.float32)
        y = torch.zeros(s.B.ntot, dtype=torch.float32, device="cuda")
        s.B.apply(s.sys, fac, dtype, torch.tensor(r, device="cuda"), y)
        for f, yf in enumerate(s.split(y)):
            G, Bm, Ut, Vt, lam = held[f]
            exp = hmatrix.apply(s.parts[f], G, Bm, Ut, Vt, lam, s.A[f].diagonal(), r[s.rows(f)].astype(np.float64))
            assert relerr(yf, exp) <= 1e-5, (dtype, f, relerr(yf, exp))
