"""GPU parity on padded frames (paper Sec. 8: the partition sized to a
maximum N, smaller frames padded to it; Supplementary "Grid and ordering":
the benchmark's W x H grid cut to its first N cells in Morton order): a
frame keeps its power-of-two box, hp_batch_set_regions names its own cells,
hp_assemble gives the padding identity rows.  Assembly, SpMV, Jacobi-PCG,
the FP32 network forward and PCG with the inferred factors against the
float64 oracle on the same padded systems."""
import numpy as np
import pytest

from oracle import grid, hmatrix, network, pcg as opcg
from paper_2605_13343_amd import hp, inputs
from tests.gpu_helpers import Side, relerr

pytestmark = pytest.mark.gpu

DEF = inputs.MODEL_DEFAULT


def _frames3d():
    # padded, truncated, unpadded and a larger padded frame in one batch
    return [inputs.make_padded_frame((16, 16, 8), (12, 10, 6, 720), 9300),
            inputs.make_padded_frame((16, 16, 8), (16, 13, 8, 1500), 9301),
            inputs.make_frame_grid(16, 16, 8, 9302),
            inputs.make_padded_frame((32, 16, 16), (27, 16, 11, 4000), 9303)]


def _frames2d():
    return [inputs.make_frame("paper2d_trunc_2048", 9310), inputs.make_frame("paper2d_trunc_2048", 9311),
            inputs.make_frame("paper2d_1024", 9312)]


def _expected_faces(A, fr):
    """w of each node's +x, +y, +z face from the oracle's operator (0 where
    there is no face)."""
    pos = grid.positions(fr.nx, fr.ny, fr.nz).astype(int)
    inv = {tuple(p): i for i, p in enumerate(pos)}
    A = A.tocsr()
    out = []
    for step in ((1, 0, 0), (0, 1, 0), (0, 0, 1)):
        e = np.zeros(fr.n)
        for i, p in enumerate(pos):
            j = inv.get(tuple(p + np.array(step)))
            if j is not None:
                e[i] = -A[i, j]
        out.append(e)
    return out


@pytest.mark.parametrize("which", ["3d", "2d"])
def test_padded_assemble_matches_oracle(which):
    import torch
    frames = _frames3d() if which == "3d" else _frames2d()
    s = Side(DEF, frames)
    nt = s.B.ntot
    sys = s.sys[:5 * nt].double().cpu().numpy().reshape(5, -1)
    sys8 = s.sys[5 * nt:].view(torch.float64).cpu().numpy().reshape(4, -1)
    for f, fr in enumerate(s.frames):
        A, rows = s.A[f], s.rows(f)
        d = A.diagonal()
        assert relerr(sys8[0, rows], d) <= 1e-15, f
        assert relerr(sys[0, rows], d) <= 2e-7 and relerr(sys[4, rows], 1.0 / d) <= 2e-7, f
        for ax, e in enumerate(_expected_faces(A, fr)):
            assert relerr(sys8[1 + ax, rows], e) <= 1e-15, (f, ax)
            assert relerr(sys[1 + ax, rows], e) <= 2e-7, (f, ax)
        if fr.region is not None:
            real = hp.region_mask(fr.nx, fr.ny, fr.nz, fr.region)
            assert (sys8[0, rows][~real] == 1.0).all()
            assert not sys8[1:, rows][:, ~real].any()
    # an unpadded frame is assembled bit for bit as in a batch without regions
    f = next(i for i, fr in enumerate(frames) if fr.region is None)
    sp = Side(DEF, [frames[f]])
    a = s.sys[5 * nt:].view(torch.float64).cpu().numpy().reshape(4, -1)[:, s.rows(f)]
    b = sp.sys[5 * sp.B.ntot:].view(torch.float64).cpu().numpy().reshape(4, -1)[:, sp.rows(0)]
    assert np.array_equal(a, b)


def test_padded_spmv_matches_oracle():
    import torch
    s = Side(DEF, _frames3d())
    p = np.random.default_rng(0).standard_normal(s.B.ntot).astype(np.float32)
    q = torch.zeros_like(s.b)
    s.B.spmv(s.sys, torch.tensor(p, device="cuda"), q)
    for f, qf in enumerate(s.split(q)):
        assert relerr(qf, s.A[f] @ p[s.rows(f)].astype(np.float64)) <= 1e-6, f


def test_set_regions_rejects_what_does_not_fit_and_changes_nothing():
    import torch
    frames = _frames3d()
    s = Side(DEF, frames)
    before = s.sys.clone()
    bad = [fr.region for fr in frames]
    bad[3] = (33, 16, 11, 10)                       # wider than the 32 x 16 x 16 box
    with pytest.raises(RuntimeError):
        s.B.set_regions(bad)
    bad[3] = (27, 16, 11, 27 * 16 * 11 + 1)         # more cells than the grid has
    with pytest.raises(RuntimeError):
        s.B.set_regions(bad)
    s.B.assemble(s.rho, s.sys, s.ops)
    torch.cuda.synchronize()
    assert torch.equal(before, s.sys)
    # back to whole boxes: the plain operator of every box
    s.B.set_regions([None] * len(frames))
    s.B.assemble(s.rho, s.sys, s.ops)
    nt = s.B.ntot
    d8 = s.sys[5 * nt:].view(torch.float64)[:nt].cpu().numpy()
    for f, fr in enumerate(frames):
        Ab = grid.assemble(fr.nx, fr.ny, fr.nz, np.asarray(fr.rho, np.float32).astype(np.float64))
        assert relerr(d8[s.rows(f)], Ab.diagonal()) <= 1e-15


@pytest.mark.parametrize("which,tol", [("3d", 1e-6), ("2d", 1e-8)])
def test_padded_jacobi_pcg_matches_oracle(which, tol):
    """Jacobi never mixes cells, so x stays exactly 0 on the padding; the
    iterations follow the oracle's FP32-iteration PCG on the padded system."""
    import torch
    s = Side(DEF, _frames3d() if which == "3d" else _frames2d())
    x = torch.zeros(s.B.ntot, dtype=torch.float64, device="cuda")
    res = s.B.pcg_solve(s.sys, None, s.b, x, hp.PRECOND_JACOBI, tol=tol, stagnation=False, max_iter=20000)
    for f, xf in enumerate(s.split(x)):
        fr, A, b = s.frames[f], s.A[f], s.bo[f]
        M = opcg.jacobi(A)
        xo, ko, flo, _ = opcg.pcg(A, b, M, tol=tol, max_iter=20000, stagnation=False)
        _, k32, fl32, _ = opcg.pcg(A, b, M, tol=tol, max_iter=20000, stagnation=False, fp32_iteration=True)
        it, fl, _ = res[f]
        true = np.linalg.norm(b - A @ xf) / np.linalg.norm(b)
        print(f"{which} frame {f} region {fr.region}: gpu {it} oracle fp32-iteration {k32} fp64 {ko} true {true:.2e}")
        assert fl & hp.CONVERGED and flo == fl32 == opcg.CONVERGED
        assert abs(it - k32) <= max(3, int(0.02 * k32)), (f, it, k32)
        assert true <= tol
        if fr.region is not None:
            real = hp.region_mask(fr.nx, fr.ny, fr.nz, fr.region)
            assert not xf[~real].any()
        if not fr.neumann:
            assert relerr(xf, xo) <= 1e-5


def _test_weights(cfg, seed=7):
    w = inputs.init_weights(cfg, seed)
    rng = np.random.default_rng(seed + 100)
    w["hv.w"] = (rng.standard_normal(w["hv.w"].shape) * 0.02).astype(np.float32)
    for k in list(w):
        if k.endswith(".b"):
            w[k] = (rng.standard_normal(w[k].shape) * 0.02).astype(np.float32)
    return w


@pytest.mark.parametrize("which", ["3d", "2d"])
def test_padded_forward_fp32_matches_oracle(which):
    """The network runs on the whole box, padding included: every factor
    tensor against the oracle forward on the same padded FrameSys."""
    import torch
    frames = _frames3d()[:2] if which == "3d" else _frames2d()[:1]
    s = Side(DEF, frames, with_net=True)
    w = _test_weights(DEF)
    wt = torch.tensor(hp.pack_weights(DEF, w), device="cuda")
    fac = s.B.new_factors(hp.HP_F32)
    s.B.infer_factors(wt, s.rho, s.sys, fac, hp.HP_F32)
    torch.cuda.synchronize()
    got = s.download_factors(fac, hp.HP_F32)
    wo = {k: np.asarray(v, np.float64) for k, v in w.items()}
    for f in range(len(frames)):
        o = {k: v.detach().numpy() for k, v in network.forward(DEF, wo, s.fs[f]).items()}
        G, B, Ut, Vt, lam = got[f]
        errs = {"G": relerr(G, hmatrix.gram(o["F"])), "B": relerr(B, hmatrix.coupling(o["U"], o["V"])),
                "Ut": relerr(Ut, o["Ut"]), "Vt": relerr(Vt, o["Vt"]), "lam": relerr(lam, o["lam"])}
        print(which, f, frames[f].region, {k: f"{v:.2e}" for k, v in errs.items()})
        for k, v in errs.items():
            assert v <= 1e-4, (f, k, v)


@pytest.mark.parametrize("which,weights,tol", [("3d", "seeded", 1e-6), ("2d", "trained_paper2d_L64.npz", 1e-8)])
def test_padded_hmat_pcg_with_inferred_factors_matches_oracle(which, weights, tol):
    """Inference (FP32) then PCG with the learned M on padded frames: flags
    and iterations against the oracle's PCG with the factors as the device
    holds them, and the frame's own residual within the tolerance (A has no
    coupling between frame cells and padding, so the frame's residual is
    part of the whole one).  3D frames with the seeded test weights (their M
    falls back to Jacobi) at 1e-6; the paper's truncated 2D grids with the
    2D-trained weights (no fallback) at the benchmark's 1e-8."""
    import os
    import torch
    # (the 2D case takes the two truncated frames: at N = 1,024 these weights
    # meet the rounding breakdown of the singular systems near 1e-8)
    frames = _frames3d() if which == "3d" else _frames2d()[:2]
    s = Side(DEF, frames)
    if weights == "seeded":
        w = _test_weights(DEF)
    else:
        z = np.load(os.path.join(os.path.dirname(hp.__file__), "weights", weights), allow_pickle=False)
        w = {k: z[k] for k in z.files}
    wt = torch.tensor(hp.pack_weights(DEF, w), device="cuda")
    fac = s.B.new_factors(hp.HP_F32)
    s.B.infer_factors(wt, s.rho, s.sys, fac, hp.HP_F32)
    x = torch.zeros(s.B.ntot, dtype=torch.float64, device="cuda")
    res = s.B.pcg_solve(s.sys, fac, s.b, x, hp.PRECOND_HMAT, fdtype=hp.HP_F32, tol=tol, max_iter=20000)
    held = s.download_factors(fac, hp.HP_F32)
    for f, xf in enumerate(s.split(x)):
        fr, A, b = s.frames[f], s.A[f], s.bo[f]
        G, Bm, Ut, Vt, lam = held[f]
        Mf = lambda v, f=f, G=G, Bm=Bm, Ut=Ut, Vt=Vt, lam=lam: hmatrix.apply(s.parts[f], G, Bm, Ut, Vt, lam,
                                                                              A.diagonal(), v)
        xo, ko, flo, _ = opcg.solve_with_fallback(A, b, Mf, tol=tol, max_iter=20000)
        _, k32, fl32, _ = opcg.solve_with_fallback(A, b, Mf, tol=tol, max_iter=20000, fp32_iteration=True)
        it, fl, _ = res[f]
        r = b - A @ xf
        real = np.ones(fr.n, bool) if fr.region is None else hp.region_mask(fr.nx, fr.ny, fr.nz, fr.region)
        own = np.linalg.norm(r[real]) / np.linalg.norm(b[real])
        print(f"{which} frame {f} region {fr.region}: gpu {it} flags {fl} oracle fp32-iteration {k32} fp64 {ko} "
              f"flags {flo} own relres {own:.2e}")
        assert fl == flo == fl32, (f, fl, flo, fl32)
        assert abs(it - k32) <= max(3, int(0.05 * k32)), (f, it, k32)
        assert own <= tol and np.linalg.norm(r) <= tol * np.linalg.norm(b)
        if not fr.neumann:
            assert relerr(xf[real], xo[real]) <= 1e-5
        if weights != "seeded":
            assert not fl & hp.FELL_BACK, (f, fl)
