"""Network forward of the hierarchical transformer preconditioner (oracle,
PyTorch CPU float64; autograd provides the reference gradients).

TEST INFRASTRUCTURE ONLY -- see oracle/__init__.py.

The paper prints no weights and no activations, so no end-to-end forward
value of the paper can be compared.  The pieces are pinned instead: hand-
worked cases of the attention sublayer (head split of the QKV columns, the
1/sqrt(d_h) scale, pair-bias and output-map orientation), of the edge MLP
and exact-erf GELU, of all 20 encoder input columns on a 4 x 2 x 2 grid and
of the edge-descriptor sign; invariants (softmax rows, LayerNorm moments,
leaf locality with highways and the off-diagonal stack switched off,
highway buffers by definition, descriptors by brute force); the parameter
count against the paper's "~2.6 M"; finite differences for the gradient.

Structure (Sec. 4 and Supplementary "Network Architecture Details"):
  encoder   h = W2 GELU(W1 f + b1) + b2, then n_gcn times
            h <- h + GELU((D^-1 A h) Wg + bg)
  diagonal  tokens (K, L, d); n_l pre-LN blocks with within-leaf multi-head
  stack     attention, logits += per-head MLP_e(e_ij), e_ij = (dx/4, dy/4,
            dz/4, A_ij / sqrt(A_ii A_jj)), dx = pos(j) - pos(i)
  off-diag  tokens (M_H, L_s, d): token (m,t) = W_r mean(h over I_m^t)
  stack     + W_c mean(h over J_m^t) + b; same blocks; pair bias from the
            mean descriptor over I_m^t x J_m^t'
  highways  after each attention sublayer: r_i, c_i = count-normalised sums
            of the diagonal token i and of every off-diagonal token whose row
            (column) sub-strip holds i; g = mean of all tokens of the frame.
            Diagonal token reads (r_i, c_i, g); off-diagonal token (m,t)
            reads (mean r over I_m^t, mean c over J_m^t, g).  FFN input is
            LN([x; r; c; g]) (4d), FFN 4d -> 4d -> d, GELU, residual.
  heads     after a final LayerNorm per stack: F rows = MLP_leaf (d->d->L),
            U, V rows = linear d->L_s (off tokens), Ut, Vt rows = linear
            d->L_s (diag tokens), lam = softplus(linear d->1).
"""
from __future__ import annotations

import math
from typing import Dict, Optional

import numpy as np
import scipy.sparse as sp
import torch

from . import grid, partition

F64 = torch.float64


def gelu(x):
    """Exact (erf) GELU."""
    return 0.5 * x * (1.0 + torch.erf(x / math.sqrt(2.0)))


def layernorm(x, g, b, eps: float = 1e-5):
    mu = x.mean(-1, keepdim=True)
    var = ((x - mu) ** 2).mean(-1, keepdim=True)
    return (x - mu) / torch.sqrt(var + eps) * g + b


def softplus(x):
    return torch.clamp(x, min=0) + torch.log1p(torch.exp(-torch.abs(x)))


def softmax(s):
    e = torch.exp(s - s.max(-1, keepdim=True).values)
    return e / e.sum(-1, keepdim=True)


class FrameSys:
    """Fixed per-frame inputs of the network: operator, features, geometry,
    partition, and the two edge-descriptor tables."""

    def __init__(self, nx: int, ny: int, nz: int, rho_lex: np.ndarray, leaf: int, rank: int,
                 neumann: bool = False, region=None):
        self.nx, self.ny, self.nz = nx, ny, nz
        self.n = nx * ny * nz
        self.A = grid.assemble(nx, ny, nz, rho_lex, neumann, region)
        self.diagA = self.A.diagonal().copy()
        self.feats = grid.features(nx, ny, nz, rho_lex, neumann, region)
        self.pos = grid.positions(nx, ny, nz)
        self.part = partition.build(self.n, leaf, rank)
        self._descriptors()

    def _descriptors(self):
        part, n = self.part, self.n
        K, L, Ls = part["K"], part["L"], part["Ls"]
        p = L // Ls
        dinv = 1.0 / np.sqrt(self.diagA)
        Ahat = sp.diags(dinv) @ self.A @ sp.diags(dinv)
        self.Ahat = Ahat.tocsr()
        # D^-1 A for the GCN
        self.DinvA = (sp.diags(1.0 / self.diagA) @ self.A).tocoo()
        # diagonal stack: within-leaf descriptors [K, L, L, 4]
        posk = self.pos.reshape(K, L, 3)
        dpos = (posk[:, None, :, :] - posk[:, :, None, :]) / 4.0
        ah = np.zeros((K, L, L))
        coo = self.Ahat.tocoo()
        for i, j, a in zip(coo.row, coo.col, coo.data):
            if i // L == j // L:
                ah[i // L, i % L, j % L] = a
        self.desc_diag = np.concatenate([dpos, ah[..., None]], axis=-1)
        # off-diagonal stack: sub-strip index lists per level and pair descriptors
        MH = part["MH"]
        self.levels = []   # (first tile index, idxI [n_j, Ls, S p], idxJ)
        desc = np.zeros((MH, Ls, Ls, 4))
        m = 0
        for j in range(part["J"]):
            S = 1 << j
            nj = K // (2 * S)
            idxI = np.zeros((nj, Ls, S * p), dtype=np.int64)
            idxJ = np.zeros((nj, Ls, S * p), dtype=np.int64)
            for i in range(nj):
                for t in range(Ls):
                    idxI[i, t] = partition.strip_nodes(part, m + i, t, 0)
                    idxJ[i, t] = partition.strip_nodes(part, m + i, t, 1)
            self.levels.append((m, idxI, idxJ))
            for i in range(nj):
                mm = m + i
                cI = self.pos[idxI[i]].mean(1)        # [Ls, 3]
                cJ = self.pos[idxJ[i]].mean(1)
                desc[mm, :, :, :3] = (cJ[None, :, :] - cI[:, None, :]) / 4.0
                rows = idxI[i].reshape(-1)
                cols = idxJ[i].reshape(-1)
                sub = self.Ahat[rows][:, cols].tocoo()
                acc = np.zeros((Ls, Ls))
                for a, bb, val in zip(sub.row, sub.col, sub.data):
                    acc[a // (S * p), bb // (S * p)] += val
                desc[mm, :, :, 3] = acc / float((S * p) * (S * p))
            m += nj
        self.desc_off = desc


def _lin(x, w, name):
    return x @ w[name + ".w"] + w[name + ".b"]


def _edge_mlp(e, w, pre):
    return _lin(gelu(_lin(e, w, pre + "e1")), w, pre + "e2")


def _attention(X, bias, w, pre, H):
    """X [B, T, d] -> X + MHA(LN1(X)) with additive logit bias [B, H, T, T]."""
    B_, T_, d = X.shape
    dh = d // H
    a = layernorm(X, w[pre + "ln1.g"], w[pre + "ln1.b"])
    qkv = _lin(a, w, pre + "qkv")
    q = qkv[..., :d].reshape(B_, T_, H, dh).transpose(1, 2)
    k = qkv[..., d:2 * d].reshape(B_, T_, H, dh).transpose(1, 2)
    v = qkv[..., 2 * d:].reshape(B_, T_, H, dh).transpose(1, 2)
    S = q @ k.transpose(-1, -2) / math.sqrt(dh) + bias
    P = softmax(S)
    O = (P @ v).transpose(1, 2).reshape(B_, T_, d)
    return X + _lin(O, w, pre + "o")


def _ffn(X, ctx, w, pre):
    u = layernorm(torch.cat([X, ctx], dim=-1), w[pre + "ln2.g"], w[pre + "ln2.b"])
    return X + _lin(gelu(_lin(u, w, pre + "f1")), w, pre + "f2")


def forward(cfg, weights: Dict, fs: FrameSys, trace: Optional[Dict] = None) -> Dict:
    """One frame through the network; returns the factor tensors
    F [K,L,L], U, V [M_H,Ls,Ls], Ut, Vt [N,Ls], lam [N] (torch float64).
    weights: name -> tensor (float64, may require grad) or numpy array."""
    w = {k: (v if isinstance(v, torch.Tensor) else torch.as_tensor(np.asarray(v), dtype=F64))
         for k, v in weights.items()}
    part = fs.part
    n, K, L, Ls, MH = fs.n, part["K"], part["L"], part["Ls"], part["MH"]
    d, H = cfg.d, cfg.heads
    use_off = cfg.offdiag and MH > 0
    T = lambda a: torch.as_tensor(a, dtype=F64)

    # encoder
    h = _lin(gelu(_lin(T(fs.feats), w, "enc1")), w, "enc2")
    c = fs.DinvA
    DA = torch.sparse_coo_tensor(np.vstack([c.row, c.col]), T(c.data), (n, n)).coalesce()
    for gi in range(cfg.gcn):
        h = h + gelu(_lin(torch.sparse.mm(DA, h), w, f"gcn{gi}"))
    if trace is not None:
        trace["enc"] = h

    levels = [(m0, torch.as_tensor(I), torch.as_tensor(J)) for (m0, I, J) in fs.levels]

    def strip_mean(x, which):
        outs = [x[(I if which == 0 else J)].mean(2) for (_, I, J) in levels]
        return torch.cat(outs, 0).reshape(MH * Ls, x.shape[-1])

    Xd = h
    Xo = None
    if use_off:
        Xo = strip_mean(h, 0) @ w["pool.wr"] + strip_mean(h, 1) @ w["pool.wc"] + w["pool.b"]
    if trace is not None:
        trace["pool"] = Xo
    desc_d = T(fs.desc_diag)
    desc_o = T(fs.desc_off)
    for l in range(cfg.layers):
        pd, po = f"diag{l}.", f"off{l}."
        bias_d = _edge_mlp(desc_d, w, pd).permute(0, 3, 1, 2)       # [K, H, L, L]
        Xd = _attention(Xd.reshape(K, L, d), bias_d, w, pd, H).reshape(n, d)
        if use_off:
            bias_o = _edge_mlp(desc_o, w, po).permute(0, 3, 1, 2)   # [M_H, H, Ls, Ls]
            Xo = _attention(Xo.reshape(MH, Ls, d), bias_o, w, po, H).reshape(MH * Ls, d)
        if trace is not None:
            trace[f"attn{l}"] = (Xd, Xo)
        if cfg.highways:
            rs, cs = Xd, Xd
            rc = torch.ones(n, dtype=F64)
            cc = torch.ones(n, dtype=F64)
            tot = Xd.sum(0)
            cnt = n
            if use_off:
                for (m0, I, J) in levels:
                    nj, _, sp_ = I.shape
                    src = Xo[m0 * Ls:(m0 + nj) * Ls].reshape(nj, Ls, 1, d).expand(nj, Ls, sp_, d)
                    src = src.reshape(-1, d)
                    rs = rs.index_add(0, I.reshape(-1), src)
                    cs = cs.index_add(0, J.reshape(-1), src)
                    rc = rc.index_add(0, I.reshape(-1), torch.ones(I.numel(), dtype=F64))
                    cc = cc.index_add(0, J.reshape(-1), torch.ones(J.numel(), dtype=F64))
                tot = tot + Xo.sum(0)
                cnt += MH * Ls
            r = rs / rc[:, None]
            cb = cs / cc[:, None]
            g = tot / cnt
            ctx_d = torch.cat([r, cb, g.expand(n, d)], dim=-1)
            if use_off:
                ctx_o = torch.cat([strip_mean(r, 0), strip_mean(cb, 1), g.expand(MH * Ls, d)], dim=-1)
        else:
            ctx_d = torch.zeros(n, 3 * d, dtype=F64)
            ctx_o = torch.zeros(MH * Ls, 3 * d, dtype=F64) if use_off else None
        if trace is not None and cfg.highways:
            trace[f"hw{l}"] = (r, cb, g)
        Xd = _ffn(Xd, ctx_d, w, pd)
        if use_off:
            Xo = _ffn(Xo, ctx_o, w, po)
        if trace is not None:
            trace[f"ffn{l}"] = (Xd, Xo)

    Xdf = layernorm(Xd, w["diaglnf.g"], w["diaglnf.b"])
    F = _lin(gelu(_lin(Xdf, w, "hleaf1")), w, "hleaf2").reshape(K, L, L)
    Ut = _lin(Xdf, w, "hut")
    Vt = _lin(Xdf, w, "hvt")
    lam = softplus(_lin(Xdf, w, "hlam"))[:, 0]
    if use_off:
        Xof = layernorm(Xo, w["offlnf.g"], w["offlnf.b"])
        U = _lin(Xof, w, "hu").reshape(MH, Ls, Ls)
        V = _lin(Xof, w, "hv").reshape(MH, Ls, Ls)
    else:
        U = torch.zeros(MH, Ls, Ls, dtype=F64)
        V = torch.zeros(MH, Ls, Ls, dtype=F64)
    if trace is not None:
        trace["final"] = (Xdf, Xof if use_off else None)
    return dict(F=F, U=U, V=V, Ut=Ut, Vt=Vt, lam=lam)
