"""What training gains: PCG with the learned preconditioner from the trained
weights (shipped in the package) against the same network at its seeded
initialisation and against Jacobi-PCG, on held-out frames of the training
size (N = 4,096) and of the precision workload (N = 8,192), to a 1e-6
relative residual."""
import os

import numpy as np
import pytest

from paper_2605_13343_amd import hp, inputs

pytestmark = pytest.mark.gpu

WEIGHTS = os.path.join(os.path.dirname(hp.__file__), "weights", "trained_L64.npz")


def _iters(cfg, frames, flat, precond):
    import torch
    dims = [(f.nx, f.ny, f.nz) for f in frames]
    perms = [hp.morton_order(*d) for d in dims]
    B = hp.Batch(cfg, dims)
    rho = torch.tensor(np.concatenate([f.rho[p] for f, p in zip(frames, perms)]).astype(np.float32), device="cuda")
    b = torch.tensor(np.concatenate([f.b[p] for f, p in zip(frames, perms)]).astype(np.float32), device="cuda")
    sys_ = B.new_sys()
    B.assemble(rho, sys_)
    fac = B.new_factors(hp.HP_BF16)
    if precond == hp.PRECOND_HMAT:
        B.infer_factors(flat, rho, sys_, fac, hp.HP_BF16)
    x = torch.zeros(B.ntot, dtype=torch.float64, device="cuda")
    res = B.pcg_solve(sys_, fac, b, x, precond, fdtype=hp.HP_BF16, tol=1e-6)
    assert all(r[1] & hp.CONVERGED for r in res)
    return [r[0] for r in res], [r[1] for r in res]


@pytest.mark.parametrize("recipe,seed0", [("train4096", 3900), ("precision8192", 2000)])
def test_trained_network_cuts_iterations(recipe, seed0):
    import torch
    assert os.path.exists(WEIGHTS), "trained weights are missing from the package"
    cfg = inputs.MODEL_DEFAULT
    z = np.load(WEIGHTS, allow_pickle=False)
    trained = torch.tensor(hp.pack_weights(cfg, {k: z[k] for k in z.files}), device="cuda")
    seeded = torch.tensor(hp.pack_weights(cfg, inputs.init_weights(cfg, 7)), device="cuda")
    frames = [inputs.make_frame(recipe, seed0 + f) for f in range(8)]
    it_t, fl_t = _iters(cfg, frames, trained, hp.PRECOND_HMAT)
    it_s, _ = _iters(cfg, frames, seeded, hp.PRECOND_HMAT)
    it_j, _ = _iters(cfg, frames, None, hp.PRECOND_JACOBI)
    print(recipe, "iterations trained", np.mean(it_t), "seeded init", np.mean(it_s), "jacobi", np.mean(it_j))
    # the learned M stays usable (no positivity loss, no fallback) ...
    assert not any(f & (hp.NOT_SPD | hp.FELL_BACK) for f in fl_t)
    # ... and training pays: fewer iterations than untrained and than Jacobi
    assert np.mean(it_t) < 0.8 * np.mean(it_s)
    assert np.mean(it_t) < 0.8 * np.mean(it_j)
