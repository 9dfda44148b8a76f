"""GPU parity of assembly, SpMV, the H-matrix apply and PCG against the oracle."""
import math

import numpy as np
import pytest

from oracle import grid, hmatrix, pcg as opcg
from paper_2605_13343_amd import hp, inputs
from tests.gpu_helpers import Side, f32, rand_factors, relerr

pytestmark = pytest.mark.gpu

PLAIN, DEF = inputs.MODEL_PLAIN, inputs.MODEL_DEFAULT


def _mixed_frames(n=5, seed=4000):
    return [inputs.make_frame("batch_mixed", seed + i) for i in range(n)]


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available()
    return torch


def test_assemble_matches_oracle(torch_cuda):
    s = Side(DEF, _mixed_frames(4) + [inputs.make_frame("largest16384", 5000)])
    nt = s.B.ntot
    sys = s.sys[:5 * nt].double().cpu().numpy().reshape(5, -1)
    sys8 = s.sys[5 * nt:].view(torch_cuda.float64).cpu().numpy().reshape(4, -1)
    for f, fr in enumerate(s.frames):
        A = s.A[f].tocsr()
        rows = s.rows(f)
        d = A.diagonal()
        assert relerr(sys[0, rows], d) <= 2e-7
        assert relerr(sys[4, rows], 1.0 / d) <= 2e-7
        assert relerr(sys8[0, rows], d) <= 1e-15
        pos = grid.positions(fr.nx, fr.ny, fr.nz).astype(int)
        inv = {tuple(p): i for i, p in enumerate(pos)}
        for ax, dims in ((1, (1, 0, 0)), (2, (0, 1, 0)), (3, (0, 0, 1))):
            exp = np.zeros(fr.n)
            for i, p in enumerate(pos):
                q = tuple(p + np.array(dims))
                if q in inv:
                    exp[i] = -A[i, inv[q]]
            assert relerr(sys[ax, rows], exp) <= 2e-7
            assert relerr(sys8[ax, rows], exp) <= 1e-15


def test_spmv_matches_oracle(torch_cuda):
    torch = torch_cuda
    s = Side(DEF, _mixed_frames(6))
    rng = np.random.default_rng(0)
    p = rng.standard_normal(s.B.ntot).astype(np.float32)
    q = torch.zeros_like(s.b)
    s.B.spmv(s.sys, torch.tensor(p, device="cuda"), q)
    for f, qf in enumerate(s.split(q)):
        assert relerr(qf, s.A[f] @ p[s.rows(f)].astype(np.float64)) <= 1e-6


@pytest.mark.parametrize("cfg", [PLAIN, DEF])
@pytest.mark.parametrize("dtype", [hp.HP_F32, hp.HP_BF16])
def test_apply_matches_oracle(torch_cuda, cfg, dtype):
    torch = torch_cuda
    frames = [inputs.make_frame("plain1024", 1000), inputs.make_frame("precision8192", 2000),
              inputs.make_frame_grid(4, 4, 4, 3)] if cfg is DEF else \
             [inputs.make_frame("plain1024", 1000), inputs.make_frame_grid(8, 8, 8, 7),
              inputs.make_frame_grid(4, 4, 2, 3)]
    frames = [f for f in frames if f.n % cfg.leaf == 0]
    s = Side(cfg, frames)
    facs = [rand_factors(p, 10 + i, b_scale=1.0) for i, p in enumerate(s.parts)]
    fac, held = s.upload_factors(facs, dtype)
    rng = np.random.default_rng(1)
    r = rng.standard_normal(s.B.ntot).astype(np.float32)
    y = torch.zeros(s.B.ntot, dtype=torch.float32, device="cuda")
    s.B.apply(s.sys, fac, dtype, torch.tensor(r, device="cuda"), y)
    for f, yf in enumerate(s.split(y)):
        G, Bm, Ut, Vt, lam = held[f]
        exp = hmatrix.apply(s.parts[f], G, Bm, Ut, Vt, lam, s.A[f].diagonal(), r[s.rows(f)].astype(np.float64))
        assert relerr(yf, exp) <= 1e-5, (f, relerr(yf, exp))


# Iteration counts: the device keeps vectors in FP32 (the paper's precision
# split) while the oracle is FP64 throughout, so Krylov orthogonality decays
# a little faster on the device; counts agree within 5 % (at least 3).
# Unpreconditioned CG on these kappa ~ 1e4 systems is the most sensitive and
# gets 10 %.
def iters_close(it, ko, frac=0.05):
    return abs(it - ko) <= max(3, int(frac * ko))


def _solve(s, precond, fac=None, fdtype=hp.HP_F32, **kw):
    import torch
    x = torch.zeros(s.B.ntot, dtype=torch.float64, device="cuda")
    res = s.B.pcg_solve(s.sys, fac, s.b, x, precond, fdtype=fdtype, **kw)
    return x, res


@pytest.mark.parametrize("precond", [hp.PRECOND_NONE, hp.PRECOND_JACOBI])
def test_pcg_classic_matches_oracle(torch_cuda, precond):
    s = Side(DEF, [inputs.make_frame("plain1024", 1000 + i) for i in range(3)] + _mixed_frames(3))
    x, res = _solve(s, precond, tol=1e-6)
    rows = []
    for f, xf in enumerate(s.split(x)):
        A, b = s.A[f], s.bo[f]
        M = opcg.jacobi(A) if precond == hp.PRECOND_JACOBI else None
        xo, ko, flo, _ = opcg.pcg(A, b, M, tol=1e-6)
        it, fl, rr = res[f]
        true = np.linalg.norm(b - A @ xf) / np.linalg.norm(b)
        xe = np.linalg.norm(xf - xo) / np.linalg.norm(xo)
        print(f"precond {precond} frame {f} N={s.frames[f].n} gpu {it} oracle {ko} true relres {true:.3e} "
              f"x err {xe:.2e}")
        rows.append((f, it, fl, ko, flo, true))
    for f, it, fl, ko, flo, true in rows:
        assert fl & hp.CONVERGED and flo == opcg.CONVERGED
        assert iters_close(it, ko, 0.10 if precond == hp.PRECOND_NONE else 0.05), (f, it, ko)
        assert true <= 1e-6, (f, true)


def test_cg_iterates_match_oracle_exactly_early(torch_cuda):
    """First iterations of unpreconditioned CG agree with the FP64 oracle to
    FP32 accuracy (no residual replacement, fixed iteration count)."""
    s = Side(DEF, [inputs.make_frame("plain1024", 1003)])
    for k in (1, 2, 7, 12):
        x, res = _solve_k(s, k)
        xo, ko, _, _ = opcg.pcg(s.A[0], s.bo[0], None, tol=0.0, max_iter=k, recompute_every=0, stagnation=False)
        assert res[0][0] == k
        assert relerr(s.split(x)[0], xo) <= 2e-5 * k


def _solve_k(s, k):
    import torch
    x = torch.zeros(s.B.ntot, dtype=torch.float64, device="cuda")
    res = s.B.pcg_solve(s.sys, None, s.b, x, hp.PRECOND_NONE, tol=0.0, max_iter=k, recompute_every=0,
                        fallback=False, stagnation=False, raise_on_fail=False)
    assert res[0][1] == hp.MAXITER
    return x, res


@pytest.mark.parametrize("dtype", [hp.HP_F32, hp.HP_BF16])
def test_pcg_hmat_matches_oracle(torch_cuda, dtype):
    frames = [inputs.make_frame("plain1024", 1000 + i) for i in range(2)] + _mixed_frames(3)
    s = Side(DEF, frames)
    facs = [rand_factors(p, 20 + i, b_scale=2e-4, shift=1.0) for i, p in enumerate(s.parts)]
    fac, held = s.upload_factors(facs, dtype)
    x, res = _solve(s, hp.PRECOND_HMAT, fac, dtype, tol=1e-6)
    for f, xf in enumerate(s.split(x)):
        A, b = s.A[f], s.bo[f]
        G, Bm, Ut, Vt, lam = held[f]
        dA = A.diagonal()
        Mf = lambda v: hmatrix.apply(s.parts[f], G, Bm, Ut, Vt, lam, dA, v)
        xo, ko, flo, _ = opcg.pcg(A, b, Mf, tol=1e-6)
        it, fl, rr = res[f]
        assert fl & hp.CONVERGED and flo == opcg.CONVERGED, (f, fl, flo)
        true = np.linalg.norm(b - A @ xf) / np.linalg.norm(b)
        print(f"hmat dtype {dtype} frame {f} N={s.frames[f].n} gpu {it} oracle {ko} true {true:.3e}")
        assert iters_close(it, ko), (f, it, ko)
        assert true <= 1e-6, (f, true)
        # the solution itself against the oracle's float64 PCG with the same
        # held factors: both follow the same Krylov path to the same stop
        xe = np.linalg.norm(xf - xo) / np.linalg.norm(xo)
        print(f"    x vs oracle PCG {xe:.2e}")
        assert xe <= 1e-5, (f, xe)


def test_batched_equals_single_and_deterministic(torch_cuda):
    frames = _mixed_frames(4)
    s = Side(DEF, frames)
    facs = [rand_factors(p, 30 + i, b_scale=2e-4, shift=1.0) for i, p in enumerate(s.parts)]
    fac, _ = s.upload_factors(facs, hp.HP_BF16)
    x1, r1 = _solve(s, hp.PRECOND_HMAT, fac, hp.HP_BF16)
    x2, r2 = _solve(s, hp.PRECOND_HMAT, fac, hp.HP_BF16)
    assert r1 == r2 and bool((x1 == x2).all())
    x3, r3 = _solve(s, hp.PRECOND_HMAT, fac, hp.HP_BF16, use_graph=False)
    assert r1 == r3 and bool((x1 == x3).all())
    # a tighter solve first: the next solve's first chunk (sized from the
    # previous solve's iterations) then runs past every frame's stop
    _, rt = _solve(s, hp.PRECOND_HMAT, fac, hp.HP_BF16, tol=1e-9)
    print("iterations", [r[0] for r in r1], [r[0] for r in rt])
    assert max(r[0] for r in rt) > max(r[0] for r in r1) + 2
    for use_graph in (True, False):
        x4, r4 = _solve(s, hp.PRECOND_HMAT, fac, hp.HP_BF16, use_graph=use_graph)
        assert r1 == r4 and bool((x1 == x4).all())
        _solve(s, hp.PRECOND_HMAT, fac, hp.HP_BF16, tol=1e-9)
    for f in range(len(frames)):
        s1 = Side(DEF, [frames[f]])
        fac1, _ = s1.upload_factors([facs[f]], hp.HP_BF16)
        xs, rs = _solve(s1, hp.PRECOND_HMAT, fac1, hp.HP_BF16)
        assert rs[0] == r1[f]
        assert np.array_equal(s1.split(xs)[0], s.split(x1)[f])


def test_fallback_on_indefinite_preconditioner(torch_cuda):
    s = Side(DEF, [inputs.make_frame("plain1024", 1000), inputs.make_frame("precision8192", 2001)])
    facs = []
    for i, p in enumerate(s.parts):
        G, Bm, Ut, Vt, lam = rand_factors(p, 40 + i, b_scale=2e-4, shift=1.0)
        facs.append((G, Bm, Ut, Vt, lam) if i == 0 else (-G, Bm, Ut, Vt, -lam))
    fac, _ = s.upload_factors(facs, hp.HP_F32)
    x, res = _solve(s, hp.PRECOND_HMAT, fac, hp.HP_F32, tol=1e-6)
    assert not (res[0][1] & hp.FELL_BACK)
    assert res[1][1] & hp.FELL_BACK and res[1][1] & hp.NOT_SPD and res[1][1] & hp.CONVERGED
    for f, xf in enumerate(s.split(x)):
        assert np.linalg.norm(s.bo[f] - s.A[f] @ xf) / np.linalg.norm(s.bo[f]) <= 1e-6
    with pytest.raises(hp.HPError) as e:
        _solve(s, hp.PRECOND_HMAT, fac, hp.HP_F32, fallback=False)
    assert e.value.status == 5


def _weak_factors(part, seed):
    """An SPD preconditioner too weak to cut iterations: M = diag(lam / A_ii)
    with lam spread log-uniformly over 8 decades (G, B, Ut, Vt zero), so
    cond(M A) is ~1e8 times cond(D^-1 A).  On these frames the oracle's
    ||r_100|| / ||r_0|| is ~0.73, far from the 0.5 stagnation threshold."""
    rng = np.random.default_rng(seed)
    K, L, Ls, n, MH = part["K"], part["L"], part["Ls"], part["n"], part["MH"]
    lam = 10.0 ** (-8.0 * rng.random(n))
    return (np.zeros((K, L, L)), np.zeros((MH, Ls, Ls)), np.zeros((n, Ls)), np.zeros((n, Ls)), lam)


@pytest.mark.parametrize("case", ["stagnated", "maxiter"])
def test_fallback_when_m_fails_to_cut_iterations(torch_cuda, case):
    """A positive definite M that does not cut iterations: PCG stops on the
    stagnation window (less than a 2x drop of ||r|| over 100 iterations) or,
    with that check off, on the iteration cap (200: the Jacobi restarts need
    70 and 141 more); the frame restarts as Jacobi-PCG from its current x and
    reaches the tolerance.  Flags and iteration counts
    follow the oracle's solve_with_fallback; a frame with a good M in the same
    batch is untouched."""
    frames = [inputs.make_frame("plain1024", 1000), inputs.make_frame("plain1024", 1001),
              inputs.make_frame("precision8192", 2000)]
    s = Side(DEF, frames)
    facs = [_weak_factors(s.parts[0], 1000), rand_factors(s.parts[1], 51, b_scale=2e-4, shift=1.0),
            _weak_factors(s.parts[2], 2000)]
    fac, held = s.upload_factors(facs, hp.HP_F32)
    kw = dict(tol=1e-6, stagnation=True, max_iter=10000) if case == "stagnated" else \
        dict(tol=1e-6, stagnation=False, max_iter=200)
    x, res = _solve(s, hp.PRECOND_HMAT, fac, hp.HP_F32, **kw)
    for f, xf in enumerate(s.split(x)):
        A, b = s.A[f], s.bo[f]
        G, Bm, Ut, Vt, lam = held[f]
        Mf = lambda v: hmatrix.apply(s.parts[f], G, Bm, Ut, Vt, lam, A.diagonal(), v)
        xo, ko, flo, _ = opcg.solve_with_fallback(A, b, Mf, tol=1e-6, max_iter=kw["max_iter"],
                                                  stagnation=kw["stagnation"])
        it, fl, _ = res[f]
        true = np.linalg.norm(b - A @ xf) / np.linalg.norm(b)
        print(f"{case} frame {f} N={s.frames[f].n}: gpu {it} flags {fl}, oracle {ko} flags {flo}, "
              f"true relres {true:.2e}")
        assert fl == flo, (f, fl, flo)
        assert true <= 1e-6, (f, true)
        if f == 1:
            # a usable M converges (~180 iterations, below the 200 cap)
            assert fl == hp.CONVERGED
            assert iters_close(it, ko), (f, it, ko)
        else:
            stop = hp.STAGNATED if case == "stagnated" else hp.MAXITER
            assert fl == hp.CONVERGED | stop | hp.FELL_BACK
            # the first pass stops at the same window or cap on both sides
            first = 100 if case == "stagnated" else kw["max_iter"]
            assert iters_close(it - first, ko - first), (f, it, ko)


def test_warm_first_chunk_that_stops_some_frames(torch_cuda):
    """A solve whose first chunk (sized from the batch's previous solve)
    stops some frames but not others: the stopped frames' x is copied out
    mid-solve and later chunks carry on with the rest.  Results equal a cold
    solve on a fresh batch bit for bit, with and without graphs."""
    frames = [inputs.make_frame("plain1024", 1000), inputs.make_frame("precision8192", 2003),
              inputs.make_frame("batch_mixed", 4007)]
    facs = None
    outs = {}
    for use_graph in (True, False):
        cold = Side(DEF, frames)
        if facs is None:
            facs = [rand_factors(p, 60 + i, b_scale=2e-4, shift=1.0) for i, p in enumerate(cold.parts)]
        fac_c, _ = cold.upload_factors(facs, hp.HP_BF16)
        xc, rc = _solve(cold, hp.PRECOND_HMAT, fac_c, hp.HP_BF16, tol=1e-9, use_graph=use_graph)
        warm = Side(DEF, frames)
        fac_w, _ = warm.upload_factors(facs, hp.HP_BF16)
        _, r7 = _solve(warm, hp.PRECOND_HMAT, fac_w, hp.HP_BF16, tol=1e-7, use_graph=use_graph)
        xw, rw = _solve(warm, hp.PRECOND_HMAT, fac_w, hp.HP_BF16, tol=1e-9, use_graph=use_graph)
        first = min((max(r[0] for r in r7) + 3) // 4 * 4, 256)  # the library's first-chunk rule
        its = [r[0] for r in rc]
        print(f"graph {use_graph}: first chunk {first}, cold 1e-9 iterations {its}")
        # the case this test is for: the first chunk stops some frames, not all
        assert min(its) <= first < max(its), (first, its)
        assert rw == rc
        assert bool((xw == xc).all())
        outs[use_graph] = (rc, xc.cpu())
    assert outs[True][0] == outs[False][0] and bool((outs[True][1] == outs[False][1]).all())


def test_frame_stop_times_follow_iterations(torch_cuda):
    """Device-clock stop stamps: in a batched solve every frame advances one
    iteration per kernel sequence, so a frame that needs more iterations stops
    later; all stops come after the solve's start."""
    s = Side(DEF, _mixed_frames(8))
    _, res = _solve(s, hp.PRECOND_JACOBI, tol=1e-6)
    stop, t0 = s.B.frame_times()
    its = [r[0] for r in res]
    print("iterations", its, "stop ms", np.round(stop, 3).tolist(), "solve start", t0)
    assert t0 == 0.0  # no inference ran before this solve: the solve's start is the reference
    assert (stop > 0).all()
    for f in range(len(its)):
        for g in range(len(its)):
            if its[f] < its[g]:
                assert stop[f] <= stop[g], (f, g, its[f], its[g], stop[f], stop[g])


def test_solve_step_graph_equals_separate_calls(torch_cuda):
    """hp_solve_step captures the inference, the PCG setup and the first chunk
    of iterations as one graph.  Its results equal hp_infer_factors followed by
    hp_pcg_solve bit for bit: on the capture, on a replay, and on a replay after
    the right-hand side and densities changed in place (the graph reads the
    buffers at each replay)."""
    import os
    torch = torch_cuda
    path = os.path.join(os.path.dirname(hp.__file__), "weights", "trained_L64.npz")
    z = np.load(path, allow_pickle=False)
    wt = torch.tensor(hp.pack_weights(DEF, {k: z[k] for k in z.files}), device="cuda")
    frames = _mixed_frames(6)
    s = Side(DEF, frames)
    fac = s.B.new_factors(hp.HP_BF16)

    def separate():
        s.B.infer_factors(wt, s.rho, s.sys, fac, hp.HP_BF16)
        x = torch.zeros(s.B.ntot, dtype=torch.float64, device="cuda")
        res = s.B.pcg_solve(s.sys, fac, s.b, x, hp.PRECOND_HMAT, fdtype=hp.HP_BF16, tol=1e-6)
        return x, res, fac.clone()

    def step():
        x = torch.zeros(s.B.ntot, dtype=torch.float64, device="cuda")
        res = s.B.solve_step(wt, s.rho, s.sys, fac, s.b, x, hp.HP_BF16, tol=1e-6)
        return x, res, fac.clone()

    x0, r0, f0 = separate()  # eager: tunes the GEMM tiles, sets the first-chunk length
    for k in range(2):       # capture, then replay
        x1, r1, f1 = step()
        assert r1 == r0 and torch.equal(x1, x0) and torch.equal(f1, f0), k
    # new inputs in the same buffers
    g = torch.Generator(device="cpu").manual_seed(9)
    s.b.copy_((torch.rand(s.B.ntot, generator=g) * 2 - 1).to("cuda"))
    s.rho.mul_(torch.where(torch.rand(s.B.ntot, generator=g) < 0.1, 10.0, 1.0).to("cuda"))
    s.B.assemble(s.rho, s.sys)
    x2, r2, f2 = step()
    x3, r3, f3 = separate()
    print("iterations", [r[0] for r in r0], "after the change", [r[0] for r in r3])
    assert r2 == r3 and torch.equal(x2, x3) and torch.equal(f2, f3)
    assert all(r[1] & hp.CONVERGED for r in r3)


def test_factor_buffers_must_be_16_byte_aligned(torch_cuda):
    """The factor-reading calls reject a buffer that is not 16-byte aligned
    (their kernels read it in 16-byte pieces) before launching anything."""
    import torch
    s = Side(DEF, [inputs.make_frame("plain1024", 1000)])
    fac, _ = s.upload_factors([rand_factors(s.parts[0], 60, b_scale=2e-4, shift=1.0)], hp.HP_BF16)
    big = torch.zeros(fac.numel() + 16, dtype=torch.uint8, device="cuda")
    off = big[8:8 + fac.numel()]
    off.copy_(fac)
    r = torch.ones_like(s.b)
    y = torch.zeros_like(s.b)
    with pytest.raises(RuntimeError, match="16-byte aligned"):
        s.B.apply(s.sys, off, hp.HP_BF16, r, y)
    x = torch.zeros(s.B.ntot, dtype=torch.float64, device="cuda")
    with pytest.raises(RuntimeError, match="16-byte aligned"):
        s.B.pcg_solve(s.sys, off, s.b, x, hp.PRECOND_HMAT, fdtype=hp.HP_BF16)
    s.B.apply(s.sys, fac, hp.HP_BF16, r, y)   # the aligned buffer still works
    torch.cuda.synchronize()
    assert torch.isfinite(y).all()
