"""Full-size runs in the configurations bench.py times, checked through
properties the oracle can evaluate at any size: every frame's true relative
residual ||b - A x|| / ||b|| recomputed in float64 from the oracle's own A,
and, on sampled frames, the solution against a sparse direct solve of the
oracle's A (within 1e-5 at a 1e-6 relative residual)."""
import os

import numpy as np
import pytest
import scipy.sparse.linalg as spla

from paper_2605_13343_amd import hp, inputs
from tests.gpu_helpers import Side

pytestmark = pytest.mark.gpu

DEF = inputs.MODEL_DEFAULT
WEIGHTS = os.path.join(os.path.dirname(hp.__file__), "weights", "trained_L64.npz")


def _weights():
    if os.path.exists(WEIGHTS):
        z = np.load(WEIGHTS, allow_pickle=False)
        return {k: z[k] for k in z.files}
    return inputs.init_weights(DEF, 7)


def _solve_and_check(frames, precond, sample):
    import torch
    s = Side(DEF, frames)
    wt = torch.tensor(hp.pack_weights(DEF, _weights()), device="cuda")
    fac = s.B.new_factors(hp.HP_BF16)
    if precond == hp.PRECOND_HMAT:
        s.B.infer_factors(wt, s.rho, s.sys, fac, hp.HP_BF16)
    x = torch.zeros(s.B.ntot, dtype=torch.float64, device="cuda")
    res = s.B.pcg_solve(s.sys, fac, s.b, x, precond, fdtype=hp.HP_BF16, tol=1e-6, use_graph=True)
    xs = s.split(x)
    for f in range(len(frames)):
        assert res[f][1] & hp.CONVERGED, (f, res[f])
        rel = np.linalg.norm(s.bo[f] - s.A[f] @ xs[f]) / np.linalg.norm(s.bo[f])
        assert rel <= 1e-6, (f, rel)
    errs = []
    for f in sample:
        xd = spla.spsolve(s.A[f].tocsc(), s.bo[f])
        errs.append(np.linalg.norm(xs[f] - xd) / np.linalg.norm(xd))
    print("iterations", [r[0] for r in res], "sampled solution errors", [f"{e:.1e}" for e in errs])
    # ||x - x*|| / ||x*|| <= cond(A) * relres; the workload bound is 1e-5
    assert max(errs) <= 1e-5
    return res


def test_precision_workload_batched_bf16():
    """The bench step: 20 frames of N = 8,192, BF16 inference and apply,
    one batched hipGraph solve."""
    frames = [inputs.make_frame("precision8192", 2000 + f) for f in range(20)]
    res = _solve_and_check(frames, hp.PRECOND_HMAT, sample=[0, 7, 19])
    assert sum(1 for r in res if r[1] & hp.FELL_BACK) == 0


def test_precision_workload_jacobi():
    frames = [inputs.make_frame("precision8192", 2000 + f) for f in range(20)]
    _solve_and_check(frames, hp.PRECOND_JACOBI, sample=[3])


def test_batching_64_mixed_sizes():
    """64 frames with N drawn from {1,024, 2,048, 4,096, 8,192} in one launch."""
    frames = [inputs.make_frame("batch_mixed", 4000 + f) for f in range(64)]
    _solve_and_check(frames, hp.PRECOND_HMAT, sample=[0, 31, 63])


def test_largest_16384_with_fallback_enabled():
    frames = [inputs.make_frame("largest16384", 5000 + f) for f in range(4)]
    _solve_and_check(frames, hp.PRECOND_HMAT, sample=[1])
