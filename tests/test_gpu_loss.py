"""GPU parity of the training objective: probes, cosine-Hutchinson loss and its
gradient with respect to the factor set, against the oracle (float64 autograd,
itself pinned by finite differences and Prop. 1)."""
import math

import numpy as np
import pytest

from oracle import grid, hmatrix, loss as oloss, partition
from paper_2605_13343_amd import hp, inputs
from tests.gpu_helpers import Side, relerr

pytestmark = pytest.mark.gpu

PLAIN, DEF = inputs.MODEL_PLAIN, inputs.MODEL_DEFAULT


def _factor_set(part, seed, scale=0.2):
    rng = np.random.default_rng(seed)
    K, L, Ls, n, MH = part["K"], part["L"], part["Ls"], part["n"], part["MH"]
    return dict(F=rng.standard_normal((K, L, L)) * scale / math.sqrt(L),
                U=rng.standard_normal((MH, Ls, Ls)) * scale, V=rng.standard_normal((MH, Ls, Ls)) * scale,
                Ut=rng.standard_normal((n, Ls)) * scale, Vt=rng.standard_normal((n, Ls)) * scale,
                lam=rng.uniform(0.2, 1.0, n))


def _setup(cfg, frames, seed=0):
    import torch
    s = Side(cfg, frames)
    s.B.train_init(16)
    facs = [_factor_set(p, seed + i) for i, p in enumerate(s.parts)]
    fset = s.B.new_factor_set()
    for f, fa in enumerate(facs):
        k0, m0, n0 = int(s.B.k0[f]), int(s.B.m0[f]), int(s.B.n0[f])
        p = s.parts[f]
        fset["F"][k0:k0 + p["K"]] = torch.tensor(fa["F"], dtype=torch.float32)
        if p["MH"]:
            fset["U"][m0:m0 + p["MH"]] = torch.tensor(fa["U"], dtype=torch.float32)
            fset["V"][m0:m0 + p["MH"]] = torch.tensor(fa["V"], dtype=torch.float32)
        for k in ("Ut", "Vt", "lam"):
            fset[k][n0:n0 + p["n"]] = torch.tensor(fa[k], dtype=torch.float32)
    # factors as the device holds them (FP32-rounded) for the oracle
    held = []
    for f in range(len(frames)):
        k0, m0, n0 = int(s.B.k0[f]), int(s.B.m0[f]), int(s.B.n0[f])
        p = s.parts[f]
        held.append(dict(F=fset["F"][k0:k0 + p["K"]].double().cpu().numpy(),
                         U=fset["U"][m0:m0 + p["MH"]].double().cpu().numpy(),
                         V=fset["V"][m0:m0 + p["MH"]].double().cpu().numpy(),
                         **{k: fset[k][n0:n0 + p["n"]].double().cpu().numpy() for k in ("Ut", "Vt", "lam")}))
    zraw = np.concatenate([inputs.rademacher(fr.n, 16, 77 + f) for f, fr in enumerate(frames)])
    zr = torch.tensor(zraw, device="cuda")
    z = torch.zeros_like(zr)
    x = torch.zeros_like(zr)
    s.B.probes(s.sys, zr, z, x, 2, 0.6)
    torch.cuda.synchronize()
    return s, fset, held, zraw, z, x


def _oracle_loss_grad(s, f, held, zraw_f):
    import torch
    A = s.A[f]
    Zs = oloss.smooth_probes(A, zraw_f)
    X = torch.as_tensor(A @ Zs)
    T = {k: torch.tensor(v, requires_grad=True) for k, v in held[f].items()}
    Y = hmatrix.apply(s.parts[f], hmatrix.gram(T["F"]), hmatrix.coupling(T["U"], T["V"]), T["Ut"], T["Vt"],
                      T["lam"], torch.as_tensor(A.diagonal()), X)
    L = oloss.cos_loss(Zs, Y)
    L.backward()
    return float(L.detach()), {k: v.grad.numpy() for k, v in T.items()}, Zs, X.numpy()


@pytest.mark.parametrize("cfg,recipes", [(PLAIN, [("plain1024", 1000), ("plain1024", 1001)]),
                                         (DEF, [("train4096", 3000000), ("batch_mixed", 4001)])])
def test_loss_and_factor_gradients_match_oracle(cfg, recipes):
    import torch
    frames = [inputs.make_frame(r, sd) for r, sd in recipes]
    s, fset, held, zraw, z, x = _setup(cfg, frames)
    nf = len(frames)
    losses = s.B.loss_fwd(s.sys, fset, x, z, 1.0 / nf)
    gset = {k: torch.zeros_like(v) for k, v in fset.items()}
    s.B.loss_bwd(s.sys, fset, x, z, gset)
    torch.cuda.synchronize()
    off = 0
    for f, fr in enumerate(frames):
        zf = zraw[off:off + fr.n]
        off += fr.n
        Lo, go, Zs, Xo = _oracle_loss_grad(s, f, held, zf)
        rows = s.rows(f)
        assert relerr(z.double().cpu().numpy()[rows], Zs) <= 1e-6
        assert relerr(x.double().cpu().numpy()[rows], Xo) <= 1e-6
        assert abs(losses[f] - Lo) <= 1e-5 * max(1.0, abs(Lo)), (losses[f], Lo)
        k0, m0, n0 = int(s.B.k0[f]), int(s.B.m0[f]), int(s.B.n0[f])
        p = s.parts[f]
        sl = {"F": slice(k0, k0 + p["K"]), "U": slice(m0, m0 + p["MH"]), "V": slice(m0, m0 + p["MH"]),
              "Ut": slice(n0, n0 + p["n"]), "Vt": slice(n0, n0 + p["n"]), "lam": slice(n0, n0 + p["n"])}
        errs = {}
        for k in hp.FACTOR_NAMES:
            g = gset[k][sl[k]].double().cpu().numpy() * nf   # gradient of the mean -> of loss_f
            errs[k] = relerr(g, go[k])
        print(f"frame {f} N={fr.n} loss gpu {losses[f]:.8f} oracle {Lo:.8f}", {k: f"{v:.1e}" for k, v in errs.items()})
        for k, v in errs.items():
            assert v <= 1e-3, (k, v)
        # Prop. 1(1) Euler identity on the device gradients
        G = {k: gset[k][sl[k]].double().cpu().numpy() for k in hp.FACTOR_NAMES}
        H = held[f]
        e = 0.5 * (G["F"] * H["F"]).sum() + (G["lam"] * H["lam"]).sum() + 0.25 * sum(
            (G[k] * H[k]).sum() for k in ("U", "V", "Ut", "Vt"))
        scale = sum(np.abs(G[k] * H[k]).sum() for k in hp.FACTOR_NAMES)
        assert abs(e) <= 1e-4 * scale, (e, scale)


def test_autograd_function_matches_direct_calls():
    import torch
    frames = [inputs.make_frame("plain1024", 1002)]
    s, fset, held, zraw, z, x = _setup(PLAIN, frames, seed=5)
    leaves = {k: v.clone().requires_grad_(True) for k, v in fset.items()}
    L = hp.cosine_hutchinson_loss(s.B, s.sys, x, z, *(leaves[k] for k in hp.FACTOR_NAMES))
    (3.0 * L).backward()
    Lo, go, _, _ = _oracle_loss_grad(s, 0, held, zraw)
    assert abs(float(L) - Lo) <= 1e-5
    for k in hp.FACTOR_NAMES:
        assert relerr(leaves[k].grad.double().cpu().numpy()[:go[k].shape[0]], 3.0 * go[k]) <= 1e-3, k
