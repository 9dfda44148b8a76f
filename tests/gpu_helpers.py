"""Helpers shared by the GPU parity tests: build the same seeded frames on
both sides (HIP library and CPU oracle) and move factors between them."""
from __future__ import annotations

import math
from typing import List, Sequence

import numpy as np

from oracle import grid, hmatrix, network, partition
from paper_2605_13343_amd import hp, inputs


def f32(a):
    """Inputs are FP32 on the device; the oracle gets the same rounded values."""
    return np.asarray(a, dtype=np.float32).astype(np.float64)


class Side:
    """One batch of frames on the GPU plus the oracle's view of each frame."""

    def __init__(self, cfg, frames: Sequence[inputs.Frame], with_net: bool = False):
        import torch
        self.cfg = cfg
        self.frames = list(frames)
        self.B = hp.Batch(cfg, [(f.nx, f.ny, f.nz) for f in self.frames])
        self.perms = [hp.morton_order(f.nx, f.ny, f.nz) for f in self.frames]
        self.padded = any(f.region is not None for f in self.frames)
        if self.padded:
            self.B.set_regions([f.region for f in self.frames])
        rho = np.concatenate([f.rho[p] for f, p in zip(self.frames, self.perms)]).astype(np.float32)
        b = np.concatenate([device_rhs(f)[p] for f, p in zip(self.frames, self.perms)]).astype(np.float32)
        self.rho = torch.tensor(rho, device="cuda")
        self.b = torch.tensor(b, device="cuda")
        self.sys = self.B.new_sys()
        kinds = {f.neumann for f in self.frames}
        assert len(kinds) == 1, "one operator per batch"
        self.neumann = kinds.pop()
        self.ops = hp.ASM_PAPER if self.neumann else 0
        self.B.assemble(self.rho, self.sys, self.ops)
        # oracle side (FP32-rounded inputs, FP64 arithmetic)
        self.A, self.bo, self.fs = [], [], []
        for f in self.frames:
            rr = f32(f.rho)
            self.A.append(grid.assemble(f.nx, f.ny, f.nz, rr, f.neumann, f.region))
            bl = grid.region_rhs(f.nx, f.ny, f.nz, f.b, f.region, f.neumann)
            self.bo.append(f32(bl)[grid.morton_perm(f.nx, f.ny, f.nz)])
            if with_net:
                self.fs.append(network.FrameSys(f.nx, f.ny, f.nz, rr, cfg.leaf, cfg.rank, f.neumann, f.region))
        self.parts = [partition.build(f.n, cfg.leaf, cfg.rank) for f in self.frames]

    def rows(self, f):
        n0 = int(self.B.n0[f])
        return slice(n0, n0 + self.frames[f].n)

    def split(self, v):
        v = v.detach().double().cpu().numpy() if hasattr(v, "detach") else np.asarray(v)
        return [v[self.rows(f)] for f in range(len(self.frames))]

    def upload_factors(self, facs, dtype):
        """facs[f] = (G, B, Ut, Vt, lam) float arrays.  Returns the device buffer
        and the factors as the device holds them (after rounding), float64."""
        import torch
        fac = self.B.new_factors(dtype)
        v = self.B.factor_views(fac, dtype)
        held = []
        for f, (G, Bm, Ut, Vt, lam) in enumerate(facs):
            k0, m0, n0 = int(self.B.k0[f]), int(self.B.m0[f]), int(self.B.n0[f])
            K, MH, n = G.shape[0], Bm.shape[0], Ut.shape[0]
            et = v["G"].dtype
            v["G"][k0:k0 + K] = torch.tensor(np.asarray(G), dtype=torch.float64).to(et)
            if MH:
                v["B"][m0:m0 + MH] = torch.tensor(np.asarray(Bm), dtype=torch.float64).to(et)
            v["Ut"][n0:n0 + n] = torch.tensor(np.asarray(Ut), dtype=torch.float64).to(et)
            v["Vt"][n0:n0 + n] = torch.tensor(np.asarray(Vt), dtype=torch.float64).to(et)
            v["lam"][n0:n0 + n] = torch.tensor(np.asarray(lam), dtype=torch.float32)
            torch.cuda.synchronize()
            held.append(tuple(t.double().cpu().numpy() for t in (
                v["G"][k0:k0 + K], v["B"][m0:m0 + MH], v["Ut"][n0:n0 + n], v["Vt"][n0:n0 + n], v["lam"][n0:n0 + n])))
        return fac, held

    def download_factors(self, fac, dtype):
        v = self.B.factor_views(fac, dtype)
        out = []
        for f in range(len(self.frames)):
            k0, m0, n0 = int(self.B.k0[f]), int(self.B.m0[f]), int(self.B.n0[f])
            p = self.parts[f]
            out.append(tuple(t.double().cpu().numpy() for t in (
                v["G"][k0:k0 + p["K"]], v["B"][m0:m0 + p["MH"]], v["Ut"][n0:n0 + p["n"]],
                v["Vt"][n0:n0 + p["n"]], v["lam"][n0:n0 + p["n"]])))
        return out


def device_rhs(fr) -> np.ndarray:
    """The right-hand side the device gets, lexicographic: for a padded
    frame b on the frame's cells (minus its mean there for the zero-flux
    operator) and 0 on the padding, the cells taken from the library's own
    mask (hp_region_mask), the arithmetic in the oracle's order."""
    if fr.region is None:
        return np.asarray(fr.b, dtype=np.float64)
    perm = hp.morton_order(fr.nx, fr.ny, fr.nz)
    real = np.zeros(fr.n, dtype=bool)
    real[perm] = hp.region_mask(fr.nx, fr.ny, fr.nz, fr.region)
    out = np.where(real, np.asarray(fr.b, dtype=np.float64), 0.0)
    if fr.neumann:
        out[real] -= out[real].mean()
    return out


def rand_factors(part, seed, b_scale=0.05, shift=0.0):
    """Random factors; with shift > 0 the leaf blocks are G = F F^T + shift I,
    and a small b_scale keeps M SPD (the diagonal part dominates)."""
    rng = np.random.default_rng(seed)
    K, L, Ls, n, MH = part["K"], part["L"], part["Ls"], part["n"], part["MH"]
    F = rng.standard_normal((K, L, L)) / math.sqrt(L)
    G = hmatrix.gram(F) + shift * np.eye(L)[None]
    Bm = rng.standard_normal((MH, Ls, Ls)) * b_scale
    Ut = rng.standard_normal((n, Ls)) / math.sqrt(L)
    Vt = rng.standard_normal((n, Ls)) / math.sqrt(L)
    lam = rng.uniform(0.2, 1.0, n)
    return G, Bm, Ut, Vt, lam


def relerr(a, b):
    a, b = np.asarray(a, np.float64), np.asarray(b, np.float64)
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))
