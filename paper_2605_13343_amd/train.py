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

    python -m paper_2605_13343_amd.train --steps 3000 \
        --mix train4096:32,precision8192:16,largest16384:8 \
        --val train4096:3900,precision8192:2000,largest16384:7000 --out weights/trained_L64.npz
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


def recipe_grid(rc):
    """(nx, ny, nz) of a one-grid recipe: the box for padded frames."""
    if isinstance(rc, inputs.BarrierRecipe):
        g = rc.box if rc.box is not None else rc.grid
        return (g[0], g[1], 1)
    if len(rc.grids) != 1:
        raise ValueError("training batches use one grid shape per recipe")
    return rc.grids[0]


def recipe_region(rc):
    """(W, H, D, cells) of a padded recipe's frames (see inputs.Frame), else None."""
    if isinstance(rc, inputs.BarrierRecipe) and rc.box is not None:
        return (rc.grid[0], rc.grid[1], 1, rc.cells if rc.cells is not None else rc.grid[0] * rc.grid[1])
    return None


def frame_rhs(fr, perm) -> np.ndarray:
    """The frame's right-hand side in Morton order: for a padded frame b on
    its own cells (the library's mask), minus its mean there for the
    zero-flux operator, and 0 on the padding."""
    bm = np.asarray(fr.b, dtype=np.float64)[perm]
    if fr.region is None:
        return bm
    real = hp.region_mask(fr.nx, fr.ny, fr.nz, fr.region)
    bm = np.where(real, bm, 0.0)
    if fr.neumann:
        bm[real] -= bm[real].mean()
    return bm


def recipe_ops(rc) -> int:
    """Assembly bits: the paper's zero-flux operator for its 2D benchmark frames."""
    return hp.ASM_PAPER if isinstance(rc, inputs.BarrierRecipe) else 0


def recipe_tol(rc) -> float:
    """Relative residual of the solves: the paper's 1e-8 on its 2D benchmark,
    1e-6 on the 3D workloads."""
    return 1e-8 if isinstance(rc, inputs.BarrierRecipe) else 1e-6


class Validator:
    """PCG iterations to the recipe's relative residual (1e-6 on the 3D
    workloads, 1e-8 on the paper's 2D frames) on fixed held-out frames,
    learned preconditioner (BF16 inference and apply) against Jacobi."""

    def __init__(self, cfg, recipe: str, seeds: List[int], stream=None):
        import torch
        self.cfg = cfg
        rc = inputs.RECIPES[recipe]
        self.ops, self.tol = recipe_ops(rc), recipe_tol(rc)
        frames = [inputs.make_frame(recipe, s) for s in seeds]
        dims = [(f.nx, f.ny, f.nz) for f in frames]
        perms = [hp.morton_order(*d) for d in dims]
        self.B = hp.Batch(cfg, dims, stream)
        if any(f.region is not None for f in frames):
            self.B.set_regions([f.region for f in frames])
        self.rho = torch.tensor(np.concatenate([f.rho[p] for f, p in zip(frames, perms)]).astype(np.float32),
                                device="cuda")
        self.b = torch.tensor(np.concatenate([frame_rhs(f, p) for f, p in zip(frames, perms)]).astype(np.float32),
                              device="cuda")
        self.sys = self.B.new_sys()
        self.B.assemble(self.rho, self.sys, self.ops)
        self.fac = self.B.new_factors(hp.HP_BF16)
        self.x = torch.zeros(self.b.numel(), dtype=torch.float64, device="cuda")
        self.jacobi = self._solve(hp.PRECOND_JACOBI)

    def _solve(self, precond: int):
        self.x.zero_()
        res = self.B.pcg_solve(self.sys, self.fac, self.b, self.x, precond, hp.HP_BF16, self.tol, fallback=True,
                               raise_on_fail=False, max_iter=20000)
        it = [r[0] for r in res]
        fell = sum(1 for r in res if r[1] & hp.FELL_BACK)
        spd = sum(1 for r in res if r[1] & hp.NOT_SPD)
        return float(np.mean(it)), fell, spd

    def __call__(self, flat) -> Dict[str, float]:
        self.B.infer_factors(flat, self.rho, self.sys, self.fac, hp.HP_BF16)
        it, fell, spd = self._solve(hp.PRECOND_HMAT)
        return {"hmat_iters": it, "fell_back": fell, "not_spd": spd, "jacobi_iters": self.jacobi[0]}


# Seed bases of the training draws per recipe (disjoint from every
# validation and benchmark seed).
SEED_BASE = {"train4096": 3_000_000, "precision8192": 5_000_000, "largest16384": 6_000_000,
             "train1024": 16_000_000, "train2048": 17_000_000,
             "paper2d_trunc_2048": 18_000_000, "paper2d_trunc_8192": 19_000_000,
             "plain1024": 8_000_000, "paper2d_1024": 11_000_000, "paper2d_2048": 12_000_000,
             "paper2d_4096": 13_000_000, "paper2d_8192": 14_000_000, "paper2d_16384": 15_000_000}


def train(cfg=inputs.MODEL_DEFAULT, steps: int = 2000, mix=(("train4096", 32),), lr: float = 2e-4,
          compute: int = hp.HP_BF16, init_seed: int = 7, log_every: int = 20, val_every: int = 200,
          val: Optional[Dict[str, List[int]]] = None, init: Optional[Dict[str, np.ndarray]] = None,
          plateau: bool = True, warmup: int = 0, first_batch: int = 0, loss: str = "cos", log=print) -> Dict:
    """Train for `steps` steps; step s draws a fresh batch of mix[s % len(mix)]
    = (recipe, systems per batch) with seeds SEED_BASE[recipe] + batch * k + i
    (k counts that recipe's batches, from first_batch: a run that continues an
    earlier one starts past the batches it drew).  loss: "cos" (the
    cosine-Hutchinson loss) or "sai" (the SAI-style loss of the ablation)."""
    import torch
    trainers = []
    for recipe, batch in mix:
        rc = inputs.RECIPES[recipe]
        g = recipe_grid(rc)
        B = hp.Batch(cfg, [g] * batch)
        if recipe_region(rc) is not None:       # padded frames: the partition of the box
            B.set_regions([recipe_region(rc)] * batch)
        if loss == "sai":
            B.debug_set("sai_loss", 1)
        trainers.append({"recipe": recipe, "rc": rc, "batch": batch, "B": B, "sys": B.new_sys(),
                         "perm": hp.morton_order(*g), "n": int(np.prod(g)), "ops": recipe_ops(rc),
                         "count": first_batch})
    w0 = init if init is not None else inputs.init_weights(cfg, init_seed)
    flat = torch.tensor(hp.pack_weights(cfg, w0), device="cuda")
    grad, m, v = torch.zeros_like(flat), torch.zeros_like(flat), torch.zeros_like(flat)
    val = val if val is not None else {"train4096": [3900 + f for f in range(20)]}
    vals = {rname: Validator(cfg, rname, seeds) for rname, seeds in val.items()}
    validate = lambda: {k: vv(flat) for k, vv in vals.items()}
    sched = Plateau(lr)
    cur_lr = lr * (1.0 / warmup if warmup > 0 else 1.0)
    hist = {"step": [], "loss": [], "lr": [], "val": [], "gnorm": [], "mix": [list(x) for x in mix]}
    v0 = validate()
    hist["val"].append((0, v0))
    log(json.dumps({"step": 0, "val": v0}))
    window, t0 = [], time.time()
    for step in range(1, steps + 1):
        T = trainers[(step - 1) % len(trainers)]
        base = SEED_BASE.get(T["recipe"], 9_000_000) + T["batch"] * T["count"]
        T["count"] += 1
        seeds = [base + i for i in range(T["batch"])]
        frames = [inputs.make_frame(T["rc"], sd) for sd in seeds]
        rho = torch.tensor(np.concatenate([f.rho[T["perm"]] for f in frames]).astype(np.float32), device="cuda")
        zr = torch.tensor(np.concatenate([inputs.rademacher(T["n"], 16, sd + 7_000_000) for sd in seeds]),
                          device="cuda")
        T["B"].assemble(rho, T["sys"], T["ops"])
        loss, gn = T["B"].train_step(flat, grad, m, v, rho, T["sys"], zr, step, compute, lr=cur_lr)
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
    ap.add_argument("--lr", type=float, default=2e-4)
    ap.add_argument("--warmup", type=int, default=0, help="linear warm-up steps (0: none)")
    ap.add_argument("--mix", default="train4096:32",
                    help="comma-separated recipe:systems batches, used in turn (e.g. "
                         "train4096:32,precision8192:16,largest16384:8)")
    ap.add_argument("--leaf", type=int, default=64)
    ap.add_argument("--fp32", action="store_true", help="FP32 compute instead of BF16")
    ap.add_argument("--no-plateau", action="store_true")
    ap.add_argument("--val-every", type=int, default=200)
    ap.add_argument("--log-every", type=int, default=0,
                    help="optimizer steps per logged loss (the plateau rule's unit); default 20 per recipe "
                         "of the mix, so every window holds whole cycles")
    ap.add_argument("--val", default="train4096:3900",
                    help="comma-separated recipe:first_seed validation sets of 20 frames each")
    ap.add_argument("--init", default=None, help="start from these weights (npz)")
    ap.add_argument("--loss", default="cos", choices=("cos", "sai"),
                    help="cos: the cosine-Hutchinson loss; sai: the SAI-style loss of the loss ablation")
    ap.add_argument("--first-batch", type=int, default=0,
                    help="index of each recipe's first training batch (past those an earlier run drew)")
    ap.add_argument("--out", default=None, help="write the trained weights here (npz)")
    ap.add_argument("--history", default=None, help="write the loss/validation history here (json)")
    a = ap.parse_args(argv)
    cfg = inputs.MODEL_DEFAULT if a.leaf == 64 else inputs.MODEL_PLAIN
    init = None
    if a.init:
        z = np.load(a.init, allow_pickle=False)
        init = {k: z[k] for k in z.files}
    mix = [(t.split(":")[0], int(t.split(":")[1])) for t in a.mix.split(",")]
    val = {t.split(":")[0]: list(range(int(t.split(":")[1]), int(t.split(":")[1]) + 20)) for t in a.val.split(",")}
    log_every = a.log_every if a.log_every > 0 else 20 * len(mix)
    r = train(cfg, steps=a.steps, mix=mix, lr=a.lr, compute=hp.HP_F32 if a.fp32 else hp.HP_BF16,
              plateau=not a.no_plateau, val_every=a.val_every, val=val, init=init, warmup=a.warmup,
              first_batch=a.first_batch, loss=a.loss,
              log_every=log_every,
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
