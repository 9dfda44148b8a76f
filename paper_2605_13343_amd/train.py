"""Training of the preconditioner network on the GPU (Sec. 6).

Each step draws a batch of fresh synthetic systems, assembles them on the
device, draws Rademacher probes, and calls hp_train_step: the library's
hand-written forward and reverse kernels (smoothed probes, network forward
with saves, cosine-Hutchinson loss, reverse pass with per-layer
recomputation) and its AdamW kernel (global-norm clip, AdamW on FP32 master
weights).  The learning rate follows a reduce-on-plateau rule
(Supplementary "Optimizer and schedule": factor 0.5, patience 5 log steps,
relative threshold 5e-3, floor max(1e-3 lr, 1e-6)).

Validation solves held-out frames with PCG and the learned preconditioner and
reports mean iterations beside Jacobi-PCG, which is what training is for.

    python -m paper_2605_13343_amd.train --steps 2000 --out weights/trained_L64.npz
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time
from typing import Dict, List, Optional

import numpy as np

from . import hp, inputs


class Plateau:
    """Reduce-on-plateau on the logged loss (relative threshold mode)."""

    def __init__(self, lr: float, factor: float = 0.5, patience: int = 5, threshold: float = 5e-3):
        self.lr, self.factor, self.patience, self.threshold = lr, factor, patience, threshold
        self.min_lr = max(lr * 1e-3, 1e-6)
        self.best, self.bad = float("inf"), 0

    def update(self, value: float) -> float:
        if value < self.best * (1.0 - self.threshold):
            self.best, self.bad = value, 0
        else:
            self.bad += 1
            if self.bad > self.patience:
                self.lr = max(self.lr * self.factor, self.min_lr)
                self.bad = 0
        return self.lr


def unpack(cfg, flat: np.ndarray) -> Dict[str, np.ndarray]:
    return {name: flat[off:off + int(np.prod(shape))].reshape(shape).copy()
            for name, shape, off in hp.weight_layout(cfg)}


class Validator:
    """PCG iterations to a relative residual of 1e-6 on fixed held-out frames,
    learned preconditioner (BF16 inference and apply) against Jacobi."""

    def __init__(self, cfg, recipe: str, seeds: List[int], stream=None):
        import torch
        self.cfg = cfg
        frames = [inputs.make_frame(recipe, s) for s in seeds]
        dims = [(f.nx, f.ny, f.nz) for f in frames]
        perms = [hp.morton_order(*d) for d in dims]
        self.B = hp.Batch(cfg, dims, stream)
        self.rho = torch.tensor(np.concatenate([f.rho[p] for f, p in zip(frames, perms)]).astype(np.float32),
                                device="cuda")
        self.b = torch.tensor(np.concatenate([f.b[p] for f, p in zip(frames, perms)]).astype(np.float32),
                              device="cuda")
        self.sys = self.B.new_sys()
        self.B.assemble(self.rho, self.sys)
        self.fac = self.B.new_factors(hp.HP_BF16)
        self.x = torch.zeros(self.b.numel(), dtype=torch.float64, device="cuda")
        self.jacobi = self._solve(hp.PRECOND_JACOBI)

    def _solve(self, precond: int):
        self.x.zero_()
        res = self.B.pcg_solve(self.sys, self.fac, self.b, self.x, precond, hp.HP_BF16, 1e-6, fallback=True,
                               raise_on_fail=False)
        it = [r[0] for r in res]
        fell = sum(1 for r in res if r[1] & hp.FELL_BACK)
        spd = sum(1 for r in res if r[1] & hp.NOT_SPD)
        return float(np.mean(it)), fell, spd

    def __call__(self, flat) -> Dict[str, float]:
        self.B.infer_factors(flat, self.rho, self.sys, self.fac, hp.HP_BF16)
        it, fell, spd = self._solve(hp.PRECOND_HMAT)
        return {"hmat_iters": it, "fell_back": fell, "not_spd": spd, "jacobi_iters": self.jacobi[0]}


def train(cfg=inputs.MODEL_DEFAULT, steps: int = 2000, batch: int = 32, recipe: str = "train4096",
          lr: float = 1e-3, compute: int = hp.HP_BF16, seed_base: int = 3_000_000, init_seed: int = 7,
          log_every: int = 20, val_every: int = 200, val_recipe: str = "train4096",
          val_seeds: Optional[List[int]] = None, init: Optional[Dict[str, np.ndarray]] = None,
          plateau: bool = True, warmup: int = 0, extra_val: Optional[Dict[str, List[int]]] = None,
          log=print) -> Dict:
    import torch
    rc = inputs.RECIPES[recipe]
    if len(rc.grids) != 1:
        raise ValueError("training batches use one grid shape per recipe")
    dims = [rc.grids[0]] * batch
    perm = hp.morton_order(*rc.grids[0])
    n = int(np.prod(rc.grids[0]))
    B = hp.Batch(cfg, dims)
    sys_ = B.new_sys()
    w0 = init if init is not None else inputs.init_weights(cfg, init_seed)
    flat = torch.tensor(hp.pack_weights(cfg, w0), device="cuda")
    grad, m, v = torch.zeros_like(flat), torch.zeros_like(flat), torch.zeros_like(flat)
    vals = {val_recipe: Validator(cfg, val_recipe, val_seeds if val_seeds is not None
                                  else [3900 + f for f in range(20)])}
    for rname, seeds in (extra_val or {}).items():
        vals[rname] = Validator(cfg, rname, seeds)
    validate = lambda: {k: vv(flat) for k, vv in vals.items()}
    sched = Plateau(lr)
    cur_lr = lr * (1.0 / warmup if warmup > 0 else 1.0)
    hist = {"step": [], "loss": [], "lr": [], "val": [], "gnorm": []}
    v0 = validate()
    hist["val"].append((0, v0))
    log(json.dumps({"step": 0, "val": v0}))
    window, t0 = [], time.time()
    for step in range(1, steps + 1):
        seeds = [seed_base + batch * (step - 1) + i for i in range(batch)]
        frames = [inputs.make_frame(rc, s) for s in seeds]
        rho = torch.tensor(np.concatenate([f.rho[perm] for f in frames]).astype(np.float32), device="cuda")
        zr = torch.tensor(np.concatenate([inputs.rademacher(n, 16, s + 7_000_000) for s in seeds]), device="cuda")
        B.assemble(rho, sys_)
        loss, gn = B.train_step(flat, grad, m, v, rho, sys_, zr, step, compute, lr=cur_lr)
        if not np.isfinite(loss):
            raise FloatingPointError(f"loss is {loss} at step {step}")
        window.append(loss)
        if step < warmup:  # linear warm-up to the initial rate (an addition; the paper starts at lr)
            cur_lr = lr * (step + 1) / warmup
        if step % log_every == 0:
            ml = float(np.mean(window))
            window = []
            hist["step"].append(step)
            hist["loss"].append(ml)
            hist["lr"].append(cur_lr)
            hist["gnorm"].append(gn)
            if plateau and step > warmup:
                cur_lr = sched.update(ml)
            rec = {"step": step, "loss": round(ml, 6), "lr": cur_lr, "gnorm": round(gn, 4),
                   "ms_per_step": round((time.time() - t0) * 1e3 / step, 2)}
            if step % val_every == 0 or step == steps:
                vv = validate()
                hist["val"].append((step, vv))
                rec["val"] = vv
            log(json.dumps(rec))
    torch.cuda.synchronize()
    hist["seconds"] = time.time() - t0
    return {"weights": unpack(cfg, flat.cpu().numpy()), "history": hist}


def main(argv=None) -> int:
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--batch", type=int, default=32)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--warmup", type=int, default=0, help="linear warm-up steps (0: none)")
    ap.add_argument("--val-bench", action="store_true",
                    help="also validate on the precision workload frames (N = 8,192, seeds 2000..2019)")
    ap.add_argument("--recipe", default="train4096")
    ap.add_argument("--leaf", type=int, default=64)
    ap.add_argument("--fp32", action="store_true", help="FP32 compute instead of BF16")
    ap.add_argument("--no-plateau", action="store_true")
    ap.add_argument("--val-every", type=int, default=200)
    ap.add_argument("--val-recipe", default="train4096")
    ap.add_argument("--init", default=None, help="start from these weights (npz)")
    ap.add_argument("--out", default=None, help="write the trained weights here (npz)")
    ap.add_argument("--history", default=None, help="write the loss/validation history here (json)")
    a = ap.parse_args(argv)
    cfg = inputs.MODEL_DEFAULT if a.leaf == 64 else inputs.MODEL_PLAIN
    init = None
    if a.init:
        z = np.load(a.init, allow_pickle=False)
        init = {k: z[k] for k in z.files}
    r = train(cfg, steps=a.steps, batch=a.batch, recipe=a.recipe, lr=a.lr,
              compute=hp.HP_F32 if a.fp32 else hp.HP_BF16, plateau=not a.no_plateau, val_every=a.val_every,
              val_recipe=a.val_recipe, init=init, warmup=a.warmup,
              extra_val={"precision8192": list(range(2000, 2020))} if a.val_bench else None,
              log=lambda s: print(s, flush=True))
    if a.out:
        os.makedirs(os.path.dirname(os.path.abspath(a.out)), exist_ok=True)
        np.savez(a.out, **r["weights"])
    if a.history:
        with open(a.history, "w") as f:
            json.dump(r["history"], f)
    return 0


if __name__ == "__main__":
    sys.exit(main())
