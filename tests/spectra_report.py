"""Spectra of the preconditioned operator M A at N = 1,024 (the loss
ablation's spectral comparison, paper Sec. 7.3 "Training dynamics and loss").

For each weights file: the float64 oracle's forward on the 16 x 8 x 8 frames
of the plain workload (seeds 1000..1004), the explicit dense M, and the
eigenvalues of M A (real: M A is similar to A^1/2 M A^1/2).  Reported per
weights file: the condition number lambda_max / lambda_min of M A (mean over
the frames), its reduction against diag(A)^-1 A (Jacobi), whether M A is
positive definite, and where the eigenvalues sit relative to ||A|| (the
largest absolute row sum), the scale the SAI-style loss pins.

  python tests/spectra_report.py paper_2605_13343_amd/weights/trained_L64.npz [other.npz ...]

Test infrastructure: it runs the oracle only.
"""
from __future__ import annotations

import os
import sys

import numpy as np
import torch

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from oracle import hmatrix, loss, network  # noqa: E402
from paper_2605_13343_amd import inputs  # noqa: E402


def spectrum(cfg, weights, fr):
    fs = network.FrameSys(fr.nx, fr.ny, fr.nz, fr.rho.astype(np.float32).astype(np.float64), cfg.leaf, cfg.rank)
    with torch.no_grad():
        f = network.forward(cfg, {k: np.asarray(v, np.float64) for k, v in weights.items()}, fs)
    G = hmatrix.gram(f["F"]).numpy()
    B = hmatrix.coupling(f["U"], f["V"]).numpy()
    M = hmatrix.explicit_M(fs.part, G, B, f["Ut"].numpy(), f["Vt"].numpy(), f["lam"].numpy(), fs.diagA)
    A = fs.A.toarray()
    ev = np.sort(np.linalg.eigvals(M @ A).real)
    evj = np.sort(np.linalg.eigvals(A / fs.diagA[:, None]).real)
    return ev, evj, loss.sai_scale(fs.A)


def main(paths) -> int:
    cfg = inputs.MODEL_DEFAULT
    frames = [inputs.make_frame("plain1024", 1000 + f) for f in range(5)]
    for path in paths:
        z = np.load(path, allow_pickle=False)
        w = {k: z[k] for k in z.files}
        rows = [spectrum(cfg, w, fr) for fr in frames]
        kap = [ev[-1] / ev[0] if ev[0] > 0 else float("inf") for ev, _, _ in rows]
        kj = [evj[-1] / evj[0] for _, evj, _ in rows]
        spd = all(ev[0] > 0 for ev, _, _ in rows)
        mid = [float(np.median(ev)) for ev, _, _ in rows]
        print(f"{os.path.basename(path)}: kappa(MA) {np.mean(kap):.1f}  kappa(D^-1 A) {np.mean(kj):.1f}  "
              f"reduction {np.mean(kj) / np.mean(kap):.1f}x  MA positive definite {spd}  "
              f"median eigenvalue of MA {np.mean(mid):.3g}  ||A|| {np.mean([r[2] for r in rows]):.3g}  "
              f"eigenvalue range [{np.mean([r[0][0] for r in rows]):.3g}, {np.mean([r[0][-1] for r in rows]):.3g}]")
    return 0


if __name__ == "__main__":
    sys.exit(main(sys.argv[1:]))
