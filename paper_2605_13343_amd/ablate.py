"""Architecture ablations (paper Sec. 7.3 "Architecture ablations", Table 5):
the same training recipe for the default model and for variants with fewer
transformer layers, without the highway buffers, and without the off-diagonal
stack; then PCG iterations and ms/frame of each on held-out frames.

Every variant trains from the same seeded initialisation with the same
batches (the three workload sizes in turn), the same rate and the same number
of steps, so the variants differ only in the architecture.  The measurement
is the benchmark's step (inference and PCG to a 1e-6 relative residual,
captured as one graph) on 20 frames of N = 8,192 (seeds 2000..2019) and 20 of
N = 4,096 (seeds 3900..3919), BF16.  The width d = 128 is fixed by the
library, so the paper's width ablation is not run.

  python -m paper_2605_13343_amd.ablate --steps 1500 --out results.json
"""
from __future__ import annotations

import argparse
import dataclasses
import json
import os
import sys
import time

import numpy as np

from paper_2605_13343_amd import hp, inputs
from paper_2605_13343_amd.train import train

VARIANTS = [
    ("default (4 layers, highways, off-diagonal stack)", {}),
    ("2 layers", {"layers": 2}),
    ("1 layer", {"layers": 1}),
    ("no highways", {"highways": False}),
    ("no off-diagonal stack", {"offdiag": False}),
]
MIX = (("train4096", 32), ("precision8192", 16), ("largest16384", 8))


def measure(cfg, weights, recipe: str, seed0: int, steps: int = 5):
    """Mean PCG iterations, fallbacks and ms/frame of the captured step on 20 frames."""
    import torch
    frames = [inputs.make_frame(recipe, seed0 + f) for f in range(20)]
    dims = [(f.nx, f.ny, f.nz) for f in frames]
    perm = hp.morton_order(*dims[0])
    B = hp.Batch(cfg, dims)
    rho = torch.tensor(np.concatenate([f.rho[perm] for f in frames]).astype(np.float32), device="cuda")
    b = torch.tensor(np.concatenate([f.b[perm] for f in frames]).astype(np.float32), device="cuda")
    sys_ = B.new_sys()
    B.assemble(rho, sys_)
    wt = torch.tensor(hp.pack_weights(cfg, weights), device="cuda")
    fac = B.new_factors(hp.HP_BF16)
    x = torch.zeros(B.ntot, dtype=torch.float64, device="cuda")
    B.infer_factors(wt, rho, sys_, fac, hp.HP_BF16)  # tunes the GEMM tiles
    res = None
    for _ in range(2):
        x.zero_()
        res = B.solve_step(wt, rho, sys_, fac, b, x, hp.HP_BF16, tol=1e-6)
    st = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(st)
    for _ in range(steps):
        x.zero_()
        res = B.solve_step(wt, rho, sys_, fac, b, x, hp.HP_BF16, tol=1e-6)
    e1.record(st)
    torch.cuda.synchronize()
    it = np.array([r[0] for r in res], dtype=np.float64)
    return {"iterations_mean": round(float(it.mean()), 2), "iterations_std": round(float(it.std()), 2),
            "fell_back": int(sum(1 for r in res if r[1] & hp.FELL_BACK)),
            "ms_per_frame": round(e0.elapsed_time(e1) / steps / len(frames), 4)}


def main(argv=None) -> int:
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--steps", type=int, default=1500)
    ap.add_argument("--lr", type=float, default=2e-4)
    ap.add_argument("--only", default=None, help="comma-separated variant indices")
    ap.add_argument("--out", default=None, help="write the results here (json)")
    a = ap.parse_args(argv)
    picks = range(len(VARIANTS)) if a.only is None else [int(v) for v in a.only.split(",")]
    out = {"steps": a.steps, "lr": a.lr, "mix": [list(m) for m in MIX], "variants": []}
    for i in picks:
        name, change = VARIANTS[i]
        cfg = dataclasses.replace(inputs.MODEL_DEFAULT, **change)
        t0 = time.time()
        r = train(cfg, steps=a.steps, mix=MIX, lr=a.lr, val={"precision8192": list(range(2000, 2020))},
                  val_every=a.steps, log_every=60, log=lambda s: print(f"[{name}] {s}", flush=True))
        secs = time.time() - t0
        m8 = measure(cfg, r["weights"], "precision8192", 2000)
        m4 = measure(cfg, r["weights"], "train4096", 3900)
        n_w = sum(int(np.prod(v.shape)) for v in r["weights"].values())
        rec = {"variant": name, "change": change, "parameters": n_w, "train_seconds": round(secs, 1),
               "final_loss": r["history"]["loss"][-1], "n8192": m8, "n4096": m4}
        print(json.dumps(rec), flush=True)
        out["variants"].append(rec)
        if a.out:  # after every variant, so a long run keeps what it finished
            os.makedirs(os.path.dirname(os.path.abspath(a.out)), exist_ok=True)
            with open(a.out, "w") as f:
                json.dump(out, f, indent=1)
    return 0


if __name__ == "__main__":
    sys.exit(main())
