"""Training objective and optimiser (oracle, float64).

TEST INFRASTRUCTURE ONLY -- see oracle/__init__.py.
"""
from __future__ import annotations

import math
from typing import Dict, List, Sequence

import numpy as np
import torch

from . import hmatrix, network

F64 = torch.float64


def smooth_probes(A, Z: np.ndarray, omega: float = 0.6, sweeps: int = 2) -> np.ndarray:
    """Spectrally biased probes, Sec. 6.2 Eq. 8:
    z <- z - omega D^-1 A z, D = diag(A), applied `sweeps` times (the paper
    uses omega = 0.6 and two sweeps).  No gradient flows through this."""
    d = A.diagonal()
    Z = np.array(Z, dtype=np.float64)
    for _ in range(sweeps):
        Z = Z - omega * (A @ Z) / d[:, None]
    return Z


def cos_loss(Z, Y):
    """Cosine-Hutchinson loss, Sec. 6.1 Eq. (loss):
    1 - <Z, Y>_F / (||Z||_F ||Y||_F), one global angle over all N*K_z
    entries, with Y = M A Z."""
    if isinstance(Y, torch.Tensor):
        Z = torch.as_tensor(Z, dtype=F64)
        return 1.0 - (Z * Y).sum() / (torch.sqrt((Z * Z).sum()) * torch.sqrt((Y * Y).sum()))
    Z, Y = np.asarray(Z, np.float64), np.asarray(Y, np.float64)
    return 1.0 - float((Z * Y).sum() / (np.linalg.norm(Z) * np.linalg.norm(Y)))


def sai_loss(A, Z, Y):
    """SAI-style loss of Prop. 1(3): || (1/||A||) A M Z - Z ||_F^2 with
    ||A|| the spectral norm; here Y = M A Z is not what it needs, so the
    caller passes Y = M Z."""
    nA = float(np.linalg.norm(A.toarray(), 2))
    return float(np.linalg.norm((A @ Y) / nA - Z) ** 2)


def sai_scale(A) -> float:
    """||A|| of the trainable SAI loss: the largest absolute row sum
    max_i sum_j |A_ij| (the infinity norm, an upper bound of the spectral
    norm that is exact to compute in one pass; the loss pins M A to a fixed
    absolute scale either way)."""
    return float(np.max(np.asarray(abs(A).sum(axis=1)).ravel()))


def sai_train_loss(A, Z, Y):
    """The SAI-style loss of Prop. 1(3) as trained in the loss ablation:
    || A Y / ||A||_inf - Z ||_F^2 with Y = M Z (torch tensor or numpy)."""
    s = sai_scale(A)
    if isinstance(Y, torch.Tensor):
        A = A.tocsr()
        Asp = torch.sparse_csr_tensor(torch.as_tensor(A.indptr, dtype=torch.int64),
                                      torch.as_tensor(A.indices, dtype=torch.int64),
                                      torch.as_tensor(A.data, dtype=F64), size=A.shape)
        R = (Asp @ Y) / s - torch.as_tensor(np.asarray(Z, np.float64), dtype=F64)
        return (R * R).sum()
    R = (A @ np.asarray(Y, np.float64)) / s - np.asarray(Z, np.float64)
    return float((R * R).sum())


def system_loss(cfg, weights: Dict, fs: network.FrameSys, Z: np.ndarray, kind: str = "cos"):
    """Loss of one system.  Cosine (Sec. 6.1): X = A Z is a fixed input (no
    gradient through A), Y = M X with M built from the network's factors,
    1 - cos(Z, Y).  SAI (the loss ablation, Prop. 1(3)): Y = M Z and
    || A Y / ||A|| - Z ||_F^2."""
    f = network.forward(cfg, weights, fs)
    G = hmatrix.gram(f["F"])
    B = hmatrix.coupling(f["U"], f["V"])
    Zt = np.asarray(Z, np.float64)
    X = torch.as_tensor(Zt if kind == "sai" else fs.A @ Zt, dtype=F64)
    Y = hmatrix.apply(fs.part, G, B, f["Ut"], f["Vt"], f["lam"], torch.as_tensor(fs.diagA, dtype=F64), X)
    return sai_train_loss(fs.A, Zt, Y) if kind == "sai" else cos_loss(Z, Y)


def batch_loss(cfg, weights: Dict, systems: Sequence[network.FrameSys], probes: Sequence[np.ndarray],
               kind: str = "cos"):
    """Batch objective: mean over systems of each system's loss."""
    tot = 0.0
    for fs, Z in zip(systems, probes):
        tot = tot + system_loss(cfg, weights, fs, Z, kind)
    return tot / len(systems)


def loss_and_grad(cfg, weights_np: Dict[str, np.ndarray], systems, probes, kind: str = "cos"):
    """Loss and gradient w.r.t. every weight (float64, reverse mode)."""
    w = {k: torch.tensor(np.asarray(v, np.float64), dtype=F64, requires_grad=True)
         for k, v in weights_np.items()}
    L = batch_loss(cfg, w, systems, probes, kind)
    L.backward()
    return float(L.detach()), {k: v.grad.detach().numpy().copy() if v.grad is not None else np.zeros(v.shape)
                      for k, v in w.items()}


def adamw_step(params: Dict[str, np.ndarray], grads: Dict[str, np.ndarray],
               m: Dict[str, np.ndarray], v: Dict[str, np.ndarray], step: int,
               lr: float = 1e-3, betas=(0.9, 0.999), eps: float = 1e-8, wd: float = 1e-4,
               clip: float = 1.0):
    """Global-norm clip followed by AdamW with decoupled weight decay
    (Supplementary "Optimizer and schedule": PyTorch-default betas and eps,
    weight decay 1e-4, gradients clipped to l2 norm 1).  `step` counts from
    1.  Updates params, m, v in place; returns the pre-clip global norm."""
    gn = math.sqrt(sum(float(np.sum(np.asarray(g, np.float64) ** 2)) for g in grads.values()))
    scale = min(1.0, clip / (gn + 1e-6)) if clip else 1.0
    b1, b2 = betas
    for k in params:
        g = np.asarray(grads[k], np.float64) * scale
        p = np.asarray(params[k], np.float64)
        p = p * (1.0 - lr * wd)
        m[k] = b1 * m[k] + (1 - b1) * g
        v[k] = b2 * v[k] + (1 - b2) * g * g
        mh = m[k] / (1 - b1 ** step)
        vh = v[k] / (1 - b2 ** step)
        params[k] = p - lr * mh / (np.sqrt(vh) + eps)
    return gn
