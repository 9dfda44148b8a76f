"""The learned H-matrix preconditioner M ~ A^-1: leaf Gram, explicit dense M
and the FMM-style apply chain (oracle, float64).

TEST INFRASTRUCTURE ONLY -- see oracle/__init__.py.

Factors of one frame (Sec. 4.4, Supplementary "Decoder heads"):
  F     [K, L, L]     leaf factors; diagonal block of M is F_k F_k^T
  U, V  [M_H, Ls, Ls] tile factors; coarse coupling B_m = U_m V_m^T
  Ut,Vt [N, Ls]       node bridges; leaf k owns rows [kL, kL+L)
  lam   [N]           Jacobi gate; adds diag(lam) diag(A)^-1

Reading of the diagonal stage (Sec. 4.2/4.4 vs Sec. 5): the block is
F_k F_k^T, applied here through its Gram G_k = F_k F_k^T.
"""
from __future__ import annotations

from typing import Dict

import numpy as np
import torch

from . import partition as _part


def gram(F):
    """G_k = F_k F_k^T for every leaf (batched matmul)."""
    if isinstance(F, torch.Tensor):
        return F @ F.transpose(-1, -2)
    return np.einsum("kij,klj->kil", F, F)


def coupling(U, V):
    """B_m = U_m V_m^T (Sec. 4.2, off-diagonal stack)."""
    if isinstance(U, torch.Tensor):
        return U @ V.transpose(-1, -2)
    return np.einsum("mij,mlj->mil", U, V)


def explicit_M(part: Dict, G, B, Ut, Vt, lam, diagA) -> np.ndarray:
    """Dense N x N matrix of the preconditioner:
        M = blockdiag(G_k) + diag(lam / A_ii)
            + sum_m [ E_Rm Ut_Rm B_m Vt_Cm^T E_Cm^T  +  its transpose ].
    Tile m couples leaf k in R_m with leaf k' in C_m through
    Ut_k B_m Vt_k'^T; the transposed block comes from t^c = B^T s^r
    (Sec. 5, restriction / aggregation / coupling / prolongation)."""
    G, B, Ut, Vt, lam, diagA = (np.asarray(a, dtype=np.float64) for a in (G, B, Ut, Vt, lam, diagA))
    n, L = part["n"], part["L"]
    M = np.zeros((n, n))
    for k in range(part["K"]):
        M[k * L:(k + 1) * L, k * L:(k + 1) * L] += G[k]
    M[np.arange(n), np.arange(n)] += lam / diagA
    for m, (j, r0, c0, S) in enumerate(part["tiles"]):
        rows = np.arange(r0 * L, (r0 + S) * L)
        cols = np.arange(c0 * L, (c0 + S) * L)
        blk = Ut[rows] @ B[m] @ Vt[cols].T
        M[np.ix_(rows, cols)] += blk
        M[np.ix_(cols, rows)] += blk.T
    return M


def apply(part: Dict, G, B, Ut, Vt, lam, diagA, r):
    """y = M r through the chain of Sec. 5 (one or many right-hand sides).

      diagonal:     y_k = G_k r_k + (lam / A_ii) r
      restriction:  u_k = Ut_k^T r_k,  v_k = Vt_k^T r_k
      aggregation:  s^r_m = sum_{k in R_m} u_k,  s^c_m = sum_{k in C_m} v_k
      coupling:     t^c_m = B_m^T s^r_m,  t^r_m = B_m s^c_m
      prolongation: y_k += Ut_k sum_{m: k in R_m} t^r_m + Vt_k sum_{m: k in C_m} t^c_m

    Works on torch float64 tensors (autograd flows) or numpy arrays.
    r is [N] or [N, ncols]."""
    is_np = not isinstance(r, torch.Tensor)
    T = lambda a: torch.as_tensor(np.asarray(a), dtype=torch.float64) if not isinstance(a, torch.Tensor) else a
    G, B, Ut, Vt, lam, diagA, r = (T(a) for a in (G, B, Ut, Vt, lam, diagA, r))
    vec = r.dim() == 1
    if vec:
        r = r[:, None]
    K, L, Ls = part["K"], part["L"], part["Ls"]
    nc = r.shape[1]
    rk = r.reshape(K, L, nc)
    y = (G @ rk).reshape(K * L, nc) + (lam / diagA)[:, None] * r
    Utk = Ut.reshape(K, L, Ls)
    Vtk = Vt.reshape(K, L, Ls)
    u = Utk.transpose(1, 2) @ rk          # [K, Ls, nc]
    v = Vtk.transpose(1, 2) @ rk
    Tr = [torch.zeros(Ls, nc, dtype=torch.float64) for _ in range(K)]
    Tc = [torch.zeros(Ls, nc, dtype=torch.float64) for _ in range(K)]
    for m, (j, r0, c0, S) in enumerate(part["tiles"]):
        sr = u[r0:r0 + S].sum(0)
        sc = v[c0:c0 + S].sum(0)
        tc = B[m].T @ sr
        tr = B[m] @ sc
        for k in range(r0, r0 + S):
            Tr[k] = Tr[k] + tr
        for k in range(c0, c0 + S):
            Tc[k] = Tc[k] + tc
    if K > 0 and part["MH"] > 0:
        Trs = torch.stack(Tr)                 # [K, Ls, nc]
        Tcs = torch.stack(Tc)
        y = y + (Utk @ Trs + Vtk @ Tcs).reshape(K * L, nc)
    if vec:
        y = y[:, 0]
    return y.detach().numpy() if is_np else y


def factors_from_packed(part: Dict, packed):
    """Split one frame's packed factor vector
    [G: K L^2][B: M_H Ls^2][Ut: N Ls][Vt: N Ls][lam: N] into its parts."""
    o, s = part["offsets"], part["sizes"]
    K, L, Ls, n, MH = part["K"], part["L"], part["Ls"], part["n"], part["MH"]
    g = lambda key: packed[o[key]:o[key] + s[key]]
    return (g("diag").reshape(K, L, L), g("B").reshape(MH, Ls, Ls), g("Ut").reshape(n, Ls),
            g("Vt").reshape(n, Ls), g("lam"))
