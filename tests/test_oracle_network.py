"""Pins of the oracle's network, loss, gradient and optimiser (CPU only)."""
import dataclasses
import math

import numpy as np
import pytest
import scipy.sparse as sp
import torch

from oracle import grid, hmatrix, loss, network, partition, pcg
from paper_2605_13343_amd import inputs

TINY = inputs.ModelConfig(d=32, heads=2, layers=1, leaf=32, rank=8, edge_hidden=8)


@pytest.fixture(scope="module")
def tiny_sys():
    fr = inputs.make_frame_grid(8, 8, 4, seed=11, spheres=2, contrast=20.0)
    return network.FrameSys(fr.nx, fr.ny, fr.nz, fr.rho, TINY.leaf, TINY.rank)


@pytest.fixture(scope="module")
def c1_sys():
    fr = inputs.make_frame("plain1024", 1000)
    return fr, network.FrameSys(fr.nx, fr.ny, fr.nz, fr.rho, 32, 8)


def _rand_weights(cfg, seed, std=0.2):
    w = inputs.init_weights(cfg, seed, std=std)
    rng = np.random.default_rng(seed + 1)
    # non-trivial biases, LayerNorm affine and V head so every path carries signal
    for k in w:
        if k.endswith(".b") or k.endswith(".g") or k.startswith("hv."):
            w[k] = (w[k] + 0.1 * rng.standard_normal(w[k].shape)).astype(np.float32)
    return w


def test_param_count_soft_pin():
    # the paper quotes ~2.6 M parameters for d=128, n_l=3, h=8, L=128, L_s=32
    n = inputs.param_count(inputs.ModelConfig(leaf=128, rank=32, layers=3, heads=8))
    assert abs(n - 2.6e6) / 2.6e6 < 0.05


def test_offdiag_descriptors_bruteforce(tiny_sys):
    fs = tiny_sys
    part = fs.part
    Ad = fs.Ahat.toarray()
    for m in range(part["MH"]):
        for t in range(part["Ls"]):
            I = partition.strip_nodes(part, m, t, 0)
            for t2 in range(part["Ls"]):
                J = partition.strip_nodes(part, m, t2, 1)
                acc = np.zeros(4)
                for i in I:
                    for j in J:
                        acc[:3] += (fs.pos[j] - fs.pos[i]) / 4.0
                        acc[3] += Ad[i, j]
                acc /= len(I) * len(J)
                assert np.allclose(fs.desc_off[m, t, t2], acc, atol=1e-14)


def test_leaf_locality_without_highways(tiny_sys):
    fs = tiny_sys
    cfg = dataclasses.replace(TINY, highways=False, offdiag=False, gcn=0)
    w = _rand_weights(cfg, 3)
    f0 = network.forward(cfg, w, fs)
    feats = fs.feats.copy()
    fs.feats = feats.copy()
    fs.feats[40, :8] += 1.0                  # node 40 is in leaf 1 (L = 32)
    f1 = network.forward(cfg, w, fs)
    fs.feats = feats
    dF = (f1["F"] - f0["F"]).abs().sum(dim=(1, 2))
    assert dF[1] > 0 and torch.all(dF[[0, 2, 3, 4, 5, 6, 7]] == 0)
    dl = (f1["lam"] - f0["lam"]).abs().reshape(8, 32).sum(1)
    assert dl[1] > 0 and torch.all(dl[[0, 2, 3, 4, 5, 6, 7]] == 0)


def test_highways_spread_information(tiny_sys):
    fs = tiny_sys
    w = _rand_weights(TINY, 3)
    f0 = network.forward(TINY, w, fs)
    feats = fs.feats.copy()
    fs.feats = feats.copy()
    fs.feats[40, :8] += 1.0
    f1 = network.forward(TINY, w, fs)
    fs.feats = feats
    dF = (f1["F"] - f0["F"]).abs().sum(dim=(1, 2))
    assert torch.all(dF > 0)                 # every leaf sees the change


def test_highway_buffers_by_definition(tiny_sys):
    fs = tiny_sys
    w = _rand_weights(TINY, 5)
    tr = {}
    network.forward(TINY, w, fs, trace=tr)
    Xd, Xo = tr["attn0"]
    r, c, g = tr["hw0"]
    part = fs.part
    n, Ls, L = fs.n, part["Ls"], part["L"]
    p = L // Ls
    for i in (0, 37, 100, 255):
        k, l = divmod(i, L)
        rs, rc, cs, cc = Xd[i].clone(), 1, Xd[i].clone(), 1
        for m, (j, r0, c0, S) in enumerate(part["tiles"]):
            if r0 <= k < r0 + S:
                rs += Xo[m * Ls + l // p]
                rc += 1
            if c0 <= k < c0 + S:
                cs += Xo[m * Ls + l // p]
                cc += 1
        assert torch.allclose(r[i], rs / rc, atol=1e-13)
        assert torch.allclose(c[i], cs / cc, atol=1e-13)
    assert torch.allclose(g, torch.cat([Xd, Xo]).mean(0), atol=1e-13)


def test_seeded_init_M_is_spd(c1_sys):
    fr, fs = c1_sys
    w = inputs.init_weights(inputs.MODEL_PLAIN, 7)
    f = network.forward(inputs.MODEL_PLAIN, w, fs)
    G = hmatrix.gram(f["F"]).detach().numpy()
    B = hmatrix.coupling(f["U"], f["V"]).detach().numpy()
    assert np.all(B == 0)                     # zero V head at init
    M = hmatrix.explicit_M(fs.part, G, B, f["Ut"].detach().numpy(), f["Vt"].detach().numpy(),
                           f["lam"].detach().numpy(), fs.diagA)
    assert np.linalg.eigvalsh(M).min() > 0
    b = fr.b[grid.morton_perm(fr.nx, fr.ny, fr.nz)]
    x, it, fl, _ = pcg.pcg(fs.A, b, lambda v: M @ v, tol=1e-6)
    assert fl == pcg.CONVERGED
    xs = np.linalg.solve(fs.A.toarray(), b)
    assert np.linalg.norm(b - fs.A @ x) / np.linalg.norm(b) <= 1e-6
    assert np.linalg.norm(x - xs) / np.linalg.norm(xs) < 1e-3


# ------------------------------------------------------------------ loss

def _small_M(seed=0, n=256):
    rng = np.random.default_rng(seed)
    Q = rng.standard_normal((n, n))
    return Q @ Q.T / n + 0.1 * np.eye(n)


def test_loss_proposition_1():
    rng = np.random.default_rng(0)
    fr = inputs.make_frame_grid(8, 8, 4, 1)
    A = grid.assemble(fr.nx, fr.ny, fr.nz, fr.rho).toarray()
    M = _small_M()
    Z = rng.standard_normal((256, 8))
    Y = M @ A @ Z
    L0 = loss.cos_loss(Z, Y)
    assert 0.0 <= L0 <= 2.0
    for a in (1e-3, 0.5, 7.0, 1e4):                       # (1) positive-scale invariance
        assert math.isclose(loss.cos_loss(Z, a * Y), L0, rel_tol=1e-12)
    assert math.isclose(loss.cos_loss(Z, -Y), 2.0 - L0, rel_tol=1e-12)
    zh, yh = Z.ravel(), Y.ravel()                        # (2) projector identity
    cos = zh @ yh / (np.linalg.norm(zh) * np.linalg.norm(yh))
    assert math.isclose(L0, 1 - cos, rel_tol=1e-12)
    zs, ys = zh[:400], yh[:400]
    Pz = np.outer(zs, zs) / (zs @ zs)
    Py = np.outer(ys, ys) / (ys @ ys)
    c2 = (zs @ ys) ** 2 / ((zs @ zs) * (ys @ ys))
    assert math.isclose(0.5 * np.linalg.norm(Pz - Py) ** 2, 1 - c2, rel_tol=1e-10)
    assert abs(loss.cos_loss(Z, np.linalg.inv(A) @ A @ Z)) < 1e-13   # M = A^-1
    As = sp.csr_matrix(A)                                 # (3) SAI is not invariant
    s1 = loss.sai_loss(As, Z, M @ Z)
    s2 = loss.sai_loss(As, Z, 2.0 * M @ Z)
    assert abs(s1 - s2) > 1e-6 * abs(s1)


def test_probe_smoothing():
    fr = inputs.make_frame_grid(8, 8, 4, 2)
    A = grid.assemble(fr.nx, fr.ny, fr.nz, fr.rho)
    Z = inputs.rademacher(256, 4, 9)
    assert set(np.unique(Z)) == {-1.0, 1.0}
    one = np.ones((256, 1))
    Zs = loss.smooth_probes(A, one, sweeps=1)
    top = grid.positions(8, 8, 4)[:, 2] == 3
    assert np.allclose(Zs[~top], 1.0, atol=1e-14)        # constants survive off the Dirichlet rows
    assert np.allclose(Zs[top, 0], 1 - 0.6 * (1 / fr.rho[grid.morton_perm(8, 8, 4)][top]) / A.diagonal()[top])
    # one sweep equals (I - 0.6 D^-1 A) z written out densely
    Ad = A.toarray()
    Zd = (np.eye(256) - 0.6 * Ad / np.diag(Ad)[:, None]) @ Z
    assert np.allclose(loss.smooth_probes(A, Z, sweeps=1), Zd, atol=1e-13)


# ------------------------------------------------------------------ gradients

def test_gradient_central_differences(tiny_sys):
    fs = tiny_sys
    w = _rand_weights(TINY, 21, std=0.3)
    Z = loss.smooth_probes(fs.A, inputs.rademacher(fs.n, 4, 2))
    L0, g = loss.loss_and_grad(TINY, w, [fs], [Z])
    rng = np.random.default_rng(0)
    names = sorted(w)
    h = 1e-3
    checked = 0
    errs = []
    for name in names:
        flat = w[name].reshape(-1)
        for idx in rng.choice(flat.size, size=min(2, flat.size), replace=False):
            wp = {k: v.astype(np.float64).copy() for k, v in w.items()}
            wm = {k: v.astype(np.float64).copy() for k, v in w.items()}
            wp[name].reshape(-1)[idx] += h
            wm[name].reshape(-1)[idx] -= h
            with torch.no_grad():
                fd = (float(loss.batch_loss(TINY, wp, [fs], [Z])) -
                      float(loss.batch_loss(TINY, wm, [fs], [Z]))) / (2 * h)
            an = g[name].reshape(-1)[idx]
            errs.append((abs(fd - an), abs(an), name))
            checked += 1
    assert checked >= 64
    worst = max(errs)
    print('worst', worst)
    for e, a, name in errs:
        assert e <= 1e-5 * max(a, 1e-2), (name, e, a)


def test_gradient_random_direction(tiny_sys):
    fs = tiny_sys
    w = _rand_weights(TINY, 22, std=0.3)
    Z = loss.smooth_probes(fs.A, inputs.rademacher(fs.n, 4, 3))
    L0, g = loss.loss_and_grad(TINY, w, [fs], [Z])
    rng = np.random.default_rng(1)
    dirn = {k: rng.standard_normal(v.shape) for k, v in w.items()}
    nrm = math.sqrt(sum(float((v ** 2).sum()) for v in dirn.values()))
    dirn = {k: v / nrm for k, v in dirn.items()}
    h = 1e-3
    with torch.no_grad():
        lp = float(loss.batch_loss(TINY, {k: w[k] + h * dirn[k] for k in w}, [fs], [Z]))
        lm = float(loss.batch_loss(TINY, {k: w[k] - h * dirn[k] for k in w}, [fs], [Z]))
    fd = (lp - lm) / (2 * h)
    an = sum(float((g[k] * dirn[k]).sum()) for k in w)
    assert abs(fd - an) <= 1e-5 * abs(an)


def test_euler_identity_on_factors(c1_sys):
    """Prop. 1(1): M scales by a when F -> a^1/2 F, lam -> a lam and each of
    U, V, Ut, Vt -> a^1/4 X.  L is invariant, so the Euler sum vanishes."""
    fr, fs = c1_sys
    rng = np.random.default_rng(3)
    part = fs.part
    K, L, Ls, n, MH = part["K"], part["L"], part["Ls"], part["n"], part["MH"]
    T = lambda a: torch.tensor(a, dtype=torch.float64, requires_grad=True)
    F = T(rng.standard_normal((K, L, L)) * 0.1)
    U = T(rng.standard_normal((MH, Ls, Ls)) * 0.1)
    V = T(rng.standard_normal((MH, Ls, Ls)) * 0.1)
    Ut = T(rng.standard_normal((n, Ls)) * 0.1)
    Vt = T(rng.standard_normal((n, Ls)) * 0.1)
    lam = T(rng.uniform(0.1, 1, n))
    Z = inputs.rademacher(n, 16, 4).astype(np.float64)
    X = torch.as_tensor(fs.A @ Z)
    Y = hmatrix.apply(part, hmatrix.gram(F), hmatrix.coupling(U, V), Ut, Vt, lam,
                      torch.as_tensor(fs.diagA), X)
    Lc = loss.cos_loss(Z, Y)
    Lc.backward()
    e = 0.5 * (F.grad * F).sum() + (lam.grad * lam).sum() + 0.25 * sum(
        (t.grad * t).sum() for t in (U, V, Ut, Vt))
    scale = sum(float(t.grad.abs().mul(t.abs()).sum()) for t in (F, U, V, Ut, Vt, lam))
    assert abs(float(e)) <= 1e-12 * scale


def test_adamw_matches_torch():
    rng = np.random.default_rng(0)
    shapes = {"a": (5, 3), "b": (7,)}
    params = {k: rng.standard_normal(s) for k, s in shapes.items()}
    tp = {k: torch.tensor(v, requires_grad=True) for k, v in params.items()}
    opt = torch.optim.AdamW(list(tp.values()), lr=1e-3, weight_decay=1e-4)
    m = {k: np.zeros(s) for k, s in shapes.items()}
    v = {k: np.zeros(s) for k, s in shapes.items()}
    for step in range(1, 6):
        grads = {k: rng.standard_normal(s) * (3.0 if step % 2 else 0.01) for k, s in shapes.items()}
        for k in tp:
            tp[k].grad = torch.tensor(grads[k])
        torch.nn.utils.clip_grad_norm_(list(tp.values()), 1.0)
        opt.step()
        loss.adamw_step(params, grads, m, v, step)
        for k in tp:
            assert np.allclose(params[k], tp[k].detach().numpy(), rtol=1e-12, atol=1e-14)
