"""Thin Python binding of the C ABI in include/hp.h (ctypes; argument
marshalling only).  Every step of the method runs in the HIP library; torch is
used for device memory and streams.  There is no CPU fallback: the binding
raises if libhp.so is missing or a call fails."""
from __future__ import annotations

import ctypes as C
import os
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np

_LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libhp.so")
_lib = None

HP_F32, HP_BF16 = 0, 1
PRECOND_NONE, PRECOND_JACOBI, PRECOND_HMAT = 0, 1, 2
CONVERGED, NOT_SPD, STAGNATED, MAXITER, FELL_BACK = 1, 2, 4, 8, 16
ASM_NEUMANN, ASM_RHO_CONDUCTANCE = 1, 2
ASM_PAPER = ASM_NEUMANN | ASM_RHO_CONDUCTANCE   # the paper's benchmark operator


class HPError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"hp status {status}: {msg}")
        self.status = status


class ModelConfigC(C.Structure):
    _fields_ = [(n, C.c_int32) for n in ("d", "heads", "layers", "leaf", "rank", "edge_hidden", "gcn",
                                         "node_feats", "glob_feats", "highways", "offdiag")]


class PartitionInfo(C.Structure):
    _fields_ = [("n", C.c_int32), ("leaf", C.c_int32), ("rank", C.c_int32), ("K", C.c_int32), ("J", C.c_int32),
                ("MH", C.c_int32), ("P", C.c_int64), ("off_diag", C.c_int64), ("off_B", C.c_int64),
                ("off_Ut", C.c_int64), ("off_Vt", C.c_int64), ("off_lam", C.c_int64)]


class BatchInfo(C.Structure):
    _fields_ = [("nframes", C.c_int32), ("ntot", C.c_int64), ("ktot", C.c_int64), ("mtot", C.c_int64),
                ("sys_floats", C.c_int64), ("factor_bytes", C.c_int64 * 2), ("off_G", C.c_int64),
                ("off_B", C.c_int64), ("off_Ut", C.c_int64), ("off_Vt", C.c_int64), ("off_lam", C.c_int64),
                ("weight_floats", C.c_int64)]


class SolveOpts(C.Structure):
    _fields_ = [("precond", C.c_int32), ("fdtype", C.c_int32), ("tol", C.c_double), ("max_iter", C.c_int32),
                ("recompute_every", C.c_int32), ("fallback", C.c_int32), ("use_graph", C.c_int32),
                ("chunk", C.c_int32), ("stagnation", C.c_int32)]


class FactorSet(C.Structure):
    _fields_ = [(n, C.c_void_p) for n in ("F", "U", "V", "Ut", "Vt", "lam")]


class AdamWOpts(C.Structure):
    _fields_ = [("lr", C.c_double), ("beta1", C.c_double), ("beta2", C.c_double), ("eps", C.c_double),
                ("weight_decay", C.c_double), ("clip", C.c_double), ("step", C.c_int32)]


class SolveResult(C.Structure):
    _fields_ = [("iters", C.c_int32), ("flags", C.c_int32), ("relres", C.c_double)]


EXPORTS = {
    "hp_last_error": ([], C.c_char_p),
    "hp_morton_order": ([C.c_int32, C.c_int32, C.c_int32, C.c_void_p], C.c_int32),
    "hp_region_mask": ([C.c_int32, C.c_int32, C.c_int32, C.c_void_p, C.c_void_p], C.c_int32),
    "hp_batch_set_regions": ([C.c_void_p, C.c_void_p], C.c_int32),
    "hp_build_partition": ([C.c_int32, C.c_int32, C.c_int32, C.POINTER(PartitionInfo)] + [C.c_void_p] * 6,
                           C.c_int32),
    "hp_batch_create": ([C.POINTER(ModelConfigC), C.c_int32, C.c_void_p, C.c_void_p, C.POINTER(C.c_void_p)],
                        C.c_int32),
    "hp_batch_destroy": ([C.c_void_p], C.c_int32),
    "hp_batch_info": ([C.c_void_p, C.c_int32, C.POINTER(BatchInfo)], C.c_int32),
    "hp_batch_offsets": ([C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p], C.c_int32),
    "hp_assemble": ([C.c_void_p, C.c_void_p, C.c_void_p], C.c_int32),
    "hp_assemble_ops": ([C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32], C.c_int32),
    "hp_spmv": ([C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p], C.c_int32),
    "hp_apply": ([C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, C.c_int32], C.c_int32),
    "hp_apply_static": ([C.c_int32] * 5 + [C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, C.c_int32,
                                            C.c_void_p], C.c_int32),
    "hp_solve_step": ([C.c_void_p] * 5 + [C.c_int32, C.POINTER(SolveOpts), C.c_void_p, C.c_void_p,
                                            C.POINTER(SolveResult)], C.c_int32),
    "hp_frame_times": ([C.c_void_p, C.c_void_p, C.POINTER(C.c_double)], C.c_int32),
    "hp_pcg_solve": ([C.c_void_p, C.c_void_p, C.c_void_p, C.POINTER(SolveOpts), C.c_void_p, C.c_void_p,
                      C.POINTER(SolveResult)], C.c_int32),
    "hp_weight_count": ([C.POINTER(ModelConfigC), C.POINTER(C.c_int32), C.POINTER(C.c_int64)], C.c_int32),
    "hp_weight_info": ([C.POINTER(ModelConfigC), C.c_int32, C.c_char_p, C.POINTER(C.c_int32),
                        C.POINTER(C.c_int32), C.POINTER(C.c_int64)], C.c_int32),
    "hp_infer_factors": ([C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32], C.c_int32),
    "hp_debug_copy": ([C.c_void_p, C.c_char_p, C.c_void_p, C.c_int64], C.c_int32),
    "hp_profile_enable": ([C.c_void_p, C.c_char_p], C.c_int32),
    "hp_debug_set": ([C.c_void_p, C.c_char_p, C.c_int32], C.c_int32),
    "hp_autotune_report": ([C.c_void_p, C.c_char_p, C.c_int64, C.POINTER(C.c_int32)], C.c_int32),
    "hp_train_init": ([C.c_void_p, C.c_int32], C.c_int32),
    "hp_probes": ([C.c_void_p] * 5 + [C.c_int32, C.c_float], C.c_int32),
    "hp_loss_fwd": ([C.c_void_p, C.c_void_p, C.POINTER(FactorSet), C.c_void_p, C.c_void_p, C.c_double,
                     C.c_void_p], C.c_int32),
    "hp_loss_bwd": ([C.c_void_p, C.c_void_p, C.POINTER(FactorSet), C.c_void_p, C.c_void_p, C.POINTER(FactorSet)],
                    C.c_int32),
    "hp_train_grad": ([C.c_void_p] * 5 + [C.c_int32, C.c_float, C.c_int32, C.c_void_p, C.c_void_p], C.c_int32),
    "hp_train_step": ([C.c_void_p] * 8 + [C.c_int32, C.c_float, C.c_int32, C.POINTER(AdamWOpts), C.c_void_p,
                                            C.c_void_p], C.c_int32),
    "hp_adamw_step": ([C.c_void_p] * 5 + [C.c_int64, C.POINTER(AdamWOpts), C.c_void_p], C.c_int32),
    "hp_profile_read": ([C.c_void_p, C.POINTER(C.c_int32), C.POINTER(C.c_double), C.POINTER(C.c_double)],
                        C.c_int32),
}


def lib():
    """Load libhp.so (built in-tree by paper_2605_13343_amd.build)."""
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            raise RuntimeError(f"{_LIB_PATH} is missing: build it with paper_2605_13343_amd.build.build()")
        L = C.CDLL(_LIB_PATH)
        for name, (args, res) in EXPORTS.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = res
        _lib = L
    return _lib


def _check(status: int):
    if status != 0:
        raise HPError(status, lib().hp_last_error().decode())


def cfg_c(cfg) -> ModelConfigC:
    return ModelConfigC(cfg.d, cfg.heads, cfg.layers, cfg.leaf, cfg.rank, cfg.edge_hidden, cfg.gcn,
                        cfg.node_feats, cfg.glob_feats, int(cfg.highways), int(cfg.offdiag))


# ------------------------------------------------------------------ host-only calls

def morton_order(nx: int, ny: int, nz: int) -> np.ndarray:
    perm = np.zeros(nx * ny * nz, dtype=np.int32)
    _check(lib().hp_morton_order(nx, ny, nz, perm.ctypes.data))
    return perm


def region_mask(nx: int, ny: int, nz: int, region) -> np.ndarray:
    """Boolean [nx ny nz], Morton order of the box: the frame's own cells of
    region (W, H, D, n) (hp_region_mask)."""
    reg = np.array(region, dtype=np.int32)
    mask = np.zeros(nx * ny * nz, dtype=np.uint8)
    _check(lib().hp_region_mask(nx, ny, nz, reg.ctypes.data, mask.ctypes.data))
    return mask.astype(bool)


def build_partition(n: int, leaf: int, rank: int, tables: bool = True):
    info = PartitionInfo()
    if not tables:
        _check(lib().hp_build_partition(n, leaf, rank, C.byref(info), *([None] * 6)))
        return info, None
    _check(lib().hp_build_partition(n, leaf, rank, C.byref(info), *([None] * 6)))
    K, J, MH = info.K, info.J, info.MH
    t = {k: np.zeros(max(MH, 1), dtype=np.int32) for k in ("level", "row0", "col0", "span")}
    lt = np.zeros(max(K * J, 1), dtype=np.int32)
    ls = np.zeros(max(K * J, 1), dtype=np.int8)
    _check(lib().hp_build_partition(n, leaf, rank, C.byref(info), t["level"].ctypes.data, t["row0"].ctypes.data,
                                    t["col0"].ctypes.data, t["span"].ctypes.data, lt.ctypes.data, ls.ctypes.data))
    t = {k: v[:MH] for k, v in t.items()}
    t["leaf_tile"] = lt[:K * J].reshape(K, J)
    t["leaf_side"] = ls[:K * J].reshape(K, J)
    return info, t


def weight_layout(cfg) -> List[Tuple[str, Tuple[int, ...], int]]:
    c = cfg_c(cfg)
    cnt, fl = C.c_int32(), C.c_int64()
    _check(lib().hp_weight_count(C.byref(c), C.byref(cnt), C.byref(fl)))
    out = []
    name = C.create_string_buffer(64)
    for i in range(cnt.value):
        r, cc, off = C.c_int32(), C.c_int32(), C.c_int64()
        _check(lib().hp_weight_info(C.byref(c), i, name, C.byref(r), C.byref(cc), C.byref(off)))
        shape = (r.value, cc.value) if cc.value else (r.value,)
        out.append((name.value.decode(), shape, off.value))
    return out


def pack_weights(cfg, weights: Dict[str, np.ndarray]) -> np.ndarray:
    """Flatten a name -> array dict into the library's FP32 weight vector."""
    lay = weight_layout(cfg)
    tot = lay[-1][2] + int(np.prod(lay[-1][1]))
    out = np.zeros(tot, dtype=np.float32)
    for name, shape, off in lay:
        a = np.asarray(weights[name], dtype=np.float32)
        if a.shape != shape:
            raise ValueError(f"weight {name}: shape {a.shape} != {shape}")
        out[off:off + a.size] = a.ravel()
    return out


# ------------------------------------------------------------------ batches (GPU)

def apply_static(dims, leaf: int, rank: int, sys, fac, dtype: int, r, y, ncols: int = 1, stream=None):
    """y = M r for one frame with the library's fixed workspace (no batch, no
    allocation); r, y hold ncols columns of N values each."""
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    nx, ny, nz = (int(v) for v in dims)
    _check(lib().hp_apply_static(nx, ny, nz, int(leaf), int(rank), _ptr(sys), _ptr(fac), int(dtype), _ptr(r),
                                 _ptr(y), int(ncols), C.c_void_p(stream.cuda_stream)))


def _ptr(t) -> Optional[int]:
    return None if t is None else t.data_ptr()


class Batch:
    """A batch of frames (one leaf size) with device workspaces."""

    def __init__(self, cfg, dims: Sequence[Tuple[int, int, int]], stream=None):
        import torch
        self.cfg = cfg
        self.dims = [tuple(int(v) for v in d) for d in dims]
        self._c = cfg_c(cfg)
        arr = np.array(self.dims, dtype=np.int32).reshape(-1)
        if stream is None:
            stream = torch.cuda.current_stream()
        self.stream = stream
        h = C.c_void_p()
        _check(lib().hp_batch_create(C.byref(self._c), len(self.dims), arr.ctypes.data, C.c_void_p(stream.cuda_stream),
                                     C.byref(h)))
        self.h = h
        self.info = {}
        for dt in (HP_F32, HP_BF16):
            bi = BatchInfo()
            _check(lib().hp_batch_info(h, dt, C.byref(bi)))
            self.info[dt] = bi
        nf = len(self.dims)
        n0, k0, m0 = (np.zeros(nf, dtype=np.int64) for _ in range(3))
        _check(lib().hp_batch_offsets(h, n0.ctypes.data, k0.ctypes.data, m0.ctypes.data))
        self.n0, self.k0, self.m0 = n0, k0, m0
        self.ntot = self.info[0].ntot
        self.ktot = self.info[0].ktot
        self.mtot = self.info[0].mtot

    def __del__(self):
        try:
            if getattr(self, "h", None):
                lib().hp_batch_destroy(self.h)
                self.h = None
        except Exception:
            pass

    def set_regions(self, regions):
        """regions: one (W, H, D, n) or None (the whole box) per frame
        (hp_batch_set_regions)."""
        rows = [r if r is not None else (d[0], d[1], d[2], d[0] * d[1] * d[2]) for r, d in zip(regions, self.dims)]
        arr = np.array(rows, dtype=np.int32).reshape(-1)
        _check(lib().hp_batch_set_regions(self.h, arr.ctypes.data))

    # -- buffers
    def new_sys(self):
        import torch
        return torch.zeros(self.info[0].sys_floats, dtype=torch.float32, device="cuda")

    def new_factors(self, dtype: int):
        import torch
        return torch.zeros(self.info[dtype].factor_bytes[dtype], dtype=torch.uint8, device="cuda")

    def factor_views(self, fac, dtype: int) -> Dict[str, "torch.Tensor"]:
        """Typed views of the packed factor sections."""
        import torch
        bi = self.info[dtype]
        L, LS = self.cfg.leaf, self.cfg.rank
        et = torch.bfloat16 if dtype == HP_BF16 else torch.float32
        es = 2 if dtype == HP_BF16 else 4
        sec = lambda off, n, t, e: fac[off:off + n * e].view(t)
        return {
            "G": sec(bi.off_G, self.ktot * L * L, et, es).view(self.ktot, L, L),
            "B": sec(bi.off_B, self.mtot * LS * LS, et, es).view(self.mtot, LS, LS),
            "Ut": sec(bi.off_Ut, self.ntot * LS, et, es).view(self.ntot, LS),
            "Vt": sec(bi.off_Vt, self.ntot * LS, et, es).view(self.ntot, LS),
            "lam": sec(bi.off_lam, self.ntot, torch.float32, 4),
        }

    # -- calls
    def assemble(self, rho, sys, ops: int = 0):
        """ops: ASM_* bits (ASM_PAPER for the paper's 2D benchmark frames)."""
        if ops:
            _check(lib().hp_assemble_ops(self.h, _ptr(rho), _ptr(sys), ops))
        else:
            _check(lib().hp_assemble(self.h, _ptr(rho), _ptr(sys)))

    def spmv(self, sys, p, q):
        _check(lib().hp_spmv(self.h, _ptr(sys), _ptr(p), _ptr(q)))

    def apply(self, sys, fac, dtype: int, r, y, ncols: int = 1):
        """y = M r; r, y hold ncols columns of ntot values each (column-major)."""
        _check(lib().hp_apply(self.h, _ptr(sys), _ptr(fac), dtype, _ptr(r), _ptr(y), int(ncols)))

    def pcg_solve(self, sys, fac, b, x, precond: int, fdtype: int = HP_F32, tol: float = 1e-6,
                  max_iter: int = 10000, recompute_every: int = 25, fallback: bool = True,
                  use_graph: bool = True, chunk: int = 16, stagnation: bool = True, raise_on_fail: bool = True):
        """Returns [(iterations, flags, recurrence relres)] per frame.  With
        raise_on_fail False, HP_E_NOT_SPD / HP_E_NOCONV still return results."""
        o = SolveOpts(precond, fdtype, tol, max_iter, recompute_every, int(fallback), int(use_graph), chunk,
                      int(stagnation))
        res = (SolveResult * len(self.dims))()
        st = lib().hp_pcg_solve(self.h, _ptr(sys), _ptr(fac), C.byref(o), _ptr(b), _ptr(x), res)
        if not (st in (5, 6) and not raise_on_fail):
            _check(st)
        return [(r.iters, r.flags, r.relres) for r in res]

    def solve_step(self, weights, rho, sys, fac, b, x, compute: int, tol: float = 1e-6, max_iter: int = 10000,
                   recompute_every: int = 25, fallback: bool = True, use_graph: bool = True, chunk: int = 16,
                   stagnation: bool = True):
        """Inference then PCG with the learned preconditioner (one captured
        graph when use_graph and the inference was run eagerly before)."""
        o = SolveOpts(PRECOND_HMAT, compute, tol, max_iter, recompute_every, int(fallback), int(use_graph), chunk,
                      int(stagnation))
        res = (SolveResult * len(self.dims))()
        _check(lib().hp_solve_step(self.h, _ptr(weights), _ptr(rho), _ptr(sys), _ptr(fac), int(compute), C.byref(o),
                                   _ptr(b), _ptr(x), res))
        return [(r.iters, r.flags, r.relres) for r in res]

    def frame_times(self):
        """(per-frame stop times in ms after the step's start, solve start in ms)
        of the last solve, from device-clock stamps."""
        out = np.zeros(len(self.dims), dtype=np.float64)
        t0 = C.c_double()
        _check(lib().hp_frame_times(self.h, out.ctypes.data, C.byref(t0)))
        return out, t0.value

    def debug_set(self, name: str, value: int):
        _check(lib().hp_debug_set(self.h, name.encode(), int(value)))

    def autotune_report(self) -> List[str]:
        buf = C.create_string_buffer(1 << 16)
        n = C.c_int32(0)
        _check(lib().hp_autotune_report(self.h, buf, len(buf), C.byref(n)))
        return [ln for ln in buf.value.decode().splitlines() if ln]

    def profile_enable(self, kernel: str):
        _check(lib().hp_profile_enable(self.h, kernel.encode()))

    def profile_read(self):
        n, ms, work = C.c_int32(), C.c_double(), C.c_double()
        _check(lib().hp_profile_read(self.h, C.byref(n), C.byref(ms), C.byref(work)))
        return n.value, ms.value, work.value

    # -- training objective
    def train_init(self, kz: int = 16):
        _check(lib().hp_train_init(self.h, kz))

    def new_factor_set(self):
        import torch
        L, LS = self.cfg.leaf, self.cfg.rank
        z = lambda *s: torch.zeros(*s, dtype=torch.float32, device="cuda")
        m = max(self.mtot, 1)
        return dict(F=z(self.ktot, L, L), U=z(m, LS, LS), V=z(m, LS, LS), Ut=z(self.ntot, LS), Vt=z(self.ntot, LS),
                    lam=z(self.ntot))

    @staticmethod
    def _fs(d):
        return FactorSet(*(d[k].data_ptr() for k in ("F", "U", "V", "Ut", "Vt", "lam")))

    def probes(self, sys, zraw, z, x, sweeps: int = 2, omega: float = 0.6):
        _check(lib().hp_probes(self.h, _ptr(sys), _ptr(zraw), _ptr(z), _ptr(x), sweeps, omega))

    def loss_fwd(self, sys, fset, x, z, scale: float):
        out = np.zeros(len(self.dims), dtype=np.float64)
        fs = self._fs(fset)
        _check(lib().hp_loss_fwd(self.h, _ptr(sys), C.byref(fs), _ptr(x), _ptr(z), scale, out.ctypes.data))
        return out

    def loss_bwd(self, sys, fset, x, z, gset):
        fs, gs = self._fs(fset), self._fs(gset)
        _check(lib().hp_loss_bwd(self.h, _ptr(sys), C.byref(fs), _ptr(x), _ptr(z), C.byref(gs)))

    def infer_factors(self, weights, rho, sys, fac, compute: int):
        _check(lib().hp_infer_factors(self.h, _ptr(weights), _ptr(rho), _ptr(sys), _ptr(fac), compute))

    def train_grad(self, weights, rho, sys, zraw, grad, compute: int, sweeps: int = 2, omega: float = 0.6,
                   want_loss: bool = True):
        """Gradient of the batch-mean loss w.r.t. the flat weights into grad;
        returns the loss (synchronising) when want_loss."""
        out = C.c_double(0.0)
        _check(lib().hp_train_grad(self.h, _ptr(weights), _ptr(rho), _ptr(sys), _ptr(zraw), sweeps, omega, compute,
                                   _ptr(grad), C.byref(out) if want_loss else None))
        return out.value if want_loss else None

    def train_step(self, weights, grad, m, v, rho, sys, zraw, step: int, compute: int, lr: float = 1e-3,
                   betas=(0.9, 0.999), eps: float = 1e-8, weight_decay: float = 1e-4, clip: float = 1.0,
                   sweeps: int = 2, omega: float = 0.6, want_loss: bool = True):
        """One step: gradient at the current weights, then AdamW.  Returns
        (loss, pre-clip gradient norm) when want_loss (synchronising)."""
        o = AdamWOpts(lr, betas[0], betas[1], eps, weight_decay, clip, step)
        lo, gn = C.c_double(0.0), C.c_double(0.0)
        _check(lib().hp_train_step(self.h, _ptr(weights), _ptr(grad), _ptr(m), _ptr(v), _ptr(rho), _ptr(sys),
                                   _ptr(zraw), sweeps, omega, compute, C.byref(o),
                                   C.byref(lo) if want_loss else None, C.byref(gn) if want_loss else None))
        return (lo.value, gn.value) if want_loss else None

    def adamw_step(self, weights, grad, m, v, step: int, lr: float = 1e-3, betas=(0.9, 0.999), eps: float = 1e-8,
                   weight_decay: float = 1e-4, clip: float = 1.0, want_norm: bool = False):
        o = AdamWOpts(lr, betas[0], betas[1], eps, weight_decay, clip, step)
        out = C.c_double(0.0)
        _check(lib().hp_adamw_step(self.h, _ptr(weights), _ptr(grad), _ptr(m), _ptr(v), int(weights.numel()),
                                   C.byref(o), C.byref(out) if want_norm else None))
        return out.value if want_norm else None


FACTOR_NAMES = ("F", "U", "V", "Ut", "Vt", "lam")


def cosine_hutchinson_loss(batch: Batch, sys, x, z, F, U, V, Ut, Vt, lam):
    """Batch-mean cosine-Hutchinson loss as a differentiable torch function of
    the factor set; forward and backward run the library's kernels."""
    return _CosLoss.apply(batch, sys, x, z, F, U, V, Ut, Vt, lam)


def _make_cosloss():
    import torch

    class CosLoss(torch.autograd.Function):
        @staticmethod
        def forward(ctx, batch, sys, x, z, F, U, V, Ut, Vt, lam):
            fset = dict(F=F.contiguous(), U=U.contiguous(), V=V.contiguous(), Ut=Ut.contiguous(),
                        Vt=Vt.contiguous(), lam=lam.contiguous())
            nf = len(batch.dims)
            losses = batch.loss_fwd(sys, fset, x, z, 1.0 / nf)
            ctx.batch, ctx.sys = batch, sys
            ctx.save_for_backward(x, z, *(fset[k] for k in FACTOR_NAMES))
            return torch.tensor(float(losses.mean()), dtype=torch.float64, device=F.device)

        @staticmethod
        def backward(ctx, gout):
            x, z, *fs = ctx.saved_tensors
            fset = dict(zip(FACTOR_NAMES, fs))
            batch = ctx.batch
            g = float(gout)
            nf = len(batch.dims)
            batch.loss_fwd(ctx.sys, fset, x, z, g / nf)   # recompute the forward state
            gset = {k: torch.empty_like(v) for k, v in fset.items()}
            batch.loss_bwd(ctx.sys, fset, x, z, gset)
            return (None, None, None, None) + tuple(gset[k] for k in FACTOR_NAMES)

    return CosLoss


class _Lazy:
    def __init__(self):
        self.cls = None

    def apply(self, *a):
        if self.cls is None:
            self.cls = _make_cosloss()
        return self.cls.apply(*a)


_CosLoss = _Lazy()
