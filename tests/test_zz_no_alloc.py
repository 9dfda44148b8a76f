"""The no-allocation apply (hp_apply_static) against hp_apply on a one-frame
batch: the same kernels on the library's fixed workspace instead of the
batch's, so the results must agree bit for bit.  Two calls in a row share
the workspace; the second is smaller, so stale contents of the first would
show."""
import ctypes as C

import numpy as np
import pytest

from paper_2605_13343_amd import hp, inputs

pytestmark = pytest.mark.gpu


def _frame_inputs(torch, cfg, recipe, seed, dtype, ncols):
    fr = inputs.make_frame(recipe, seed)
    perm = hp.morton_order(fr.nx, fr.ny, fr.nz)
    B = hp.Batch(cfg, [(fr.nx, fr.ny, fr.nz)])
    rho = torch.tensor(fr.rho[perm].astype(np.float32), device="cuda")
    sys_ = B.new_sys()
    B.assemble(rho, sys_)
    g = torch.Generator(device="cpu").manual_seed(seed)
    fac = B.new_factors(dtype)
    v = B.factor_views(fac, dtype)
    for name in ("G", "B", "Ut", "Vt"):
        t = v[name]
        t.copy_((torch.randn(t.shape, generator=g) * 0.1).to(t.dtype).to("cuda"))
    v["lam"].copy_(torch.rand(v["lam"].shape, generator=g).to("cuda"))
    r = torch.randn(ncols * B.ntot, generator=g).to("cuda")
    return fr, B, sys_, fac, r


@pytest.mark.parametrize("dtype", [hp.HP_BF16, hp.HP_F32])
def test_static_apply_equals_batch_apply(dtype):
    import torch
    assert torch.cuda.is_available()
    cases = [  # the second call of each pair is smaller than the first
        (inputs.MODEL_DEFAULT, "precision8192", 2000, 2),   # 32x16x16, L = 64
        (inputs.MODEL_DEFAULT, "batch_mixed", 4007, 1),     # 16x16x16, L = 64
        (inputs.MODEL_PLAIN, "largest16384", 5000, 1),      # 32x32x16 at L = 32
        (inputs.MODEL_PLAIN, "plain1024", 1000, 3),         # 16x8x8 at L = 32
    ]
    sizes = []
    for cfg, recipe, seed, ncols in cases:
        print(f"static apply: {recipe} seed {seed} L={cfg.leaf} ncols={ncols} dtype={dtype}", flush=True)
        fr, B, sys_, fac, r = _frame_inputs(torch, cfg, recipe, seed, dtype, ncols)
        sizes.append(fr.n)
        y_ref = torch.full_like(r, float("nan"))
        B.apply(sys_, fac, dtype, r, y_ref, ncols)
        y = torch.full_like(r, float("nan"))
        hp.apply_static((fr.nx, fr.ny, fr.nz), cfg.leaf, cfg.rank, sys_, fac, dtype, r, y, ncols)
        torch.cuda.synchronize()
        assert torch.isfinite(y_ref).all()
        assert torch.equal(y, y_ref), (recipe, seed, float((y - y_ref).abs().max()))
    assert sizes[1] < sizes[0] and sizes[3] < sizes[2]


def test_static_apply_rejects_what_does_not_fit():
    import torch
    lib = hp.lib()
    buf = torch.zeros(16, device="cuda")
    p = C.c_void_p(buf.data_ptr())
    # N = 2^21 exceeds the fixed workspace; a bad grid, (leaf, rank) and ncols are refused
    assert lib.hp_apply_static(128, 128, 128, 64, 16, p, p, 1, p, C.c_void_p(buf.data_ptr() + 32), 1, None) \
        == 2
    assert b"maximum" in lib.hp_last_error()
    assert lib.hp_apply_static(12, 8, 8, 64, 16, p, p, 1, p, C.c_void_p(buf.data_ptr() + 32), 1, None) == 2
    assert lib.hp_apply_static(16, 8, 8, 48, 12, p, p, 1, p, C.c_void_p(buf.data_ptr() + 32), 1, None) == 2
    assert lib.hp_apply_static(16, 8, 8, 32, 8, p, p, 1, p, C.c_void_p(buf.data_ptr() + 32), 0, None) == 1
    assert lib.hp_apply_static(16, 8, 8, 32, 8, p, None, 1, p, C.c_void_p(buf.data_ptr() + 32), 1, None) == 1
