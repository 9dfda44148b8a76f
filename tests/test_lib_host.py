"""The C-ABI library on the CPU: it loads, exports every symbol the header
declares, and its integer host routines match the oracle bit for bit."""
import os
import re

import numpy as np
import pytest

from oracle import grid, partition
from paper_2605_13343_amd import hp, inputs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_symbols():
    txt = open(os.path.join(ROOT, "include", "hp.h")).read()
    return sorted(set(re.findall(r"^\s*(?:hp_status|const char\*)\s+(hp_\w+)\s*\(", txt, re.M)))


def test_library_exports_every_declared_symbol():
    L = hp.lib()
    syms = _declared_symbols()
    assert len(syms) >= 14
    for s in syms:
        assert hasattr(L, s), s


def _prototype_arity():
    """Parameter count of every function the header declares."""
    txt = open(os.path.join(ROOT, "include", "hp.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    out = {}
    for m in re.finditer(r"^\s*(?:hp_status|const char\*)\s+(hp_\w+)\s*\(([^)]*)\)\s*;", txt, re.M):
        args = m.group(2).strip()
        out[m.group(1)] = 0 if args in ("", "void") else len(args.split(","))
    return out


def test_binding_argument_counts_match_header():
    ar = _prototype_arity()
    assert set(hp.EXPORTS) <= set(ar), sorted(set(hp.EXPORTS) - set(ar))
    for name, (args, _) in hp.EXPORTS.items():
        assert len(args) == ar[name], (name, len(args), ar[name])


@pytest.mark.parametrize("dims", [(16, 8, 8), (16, 16, 8), (32, 16, 16), (5, 3, 2), (1, 1, 1), (32, 32, 1), (128, 64, 1)])
def test_morton_order_bit_exact(dims):
    assert np.array_equal(hp.morton_order(*dims), grid.morton_perm(*dims))


@pytest.mark.parametrize("n,L,Ls", [(1024, 32, 8), (8192, 64, 16), (16384, 64, 16), (64, 64, 16), (128, 64, 16)])
def test_partition_bit_exact(n, L, Ls):
    info, t = hp.build_partition(n, L, Ls)
    p = partition.build(n, L, Ls)
    assert (info.K, info.J, info.MH, info.P) == (p["K"], p["J"], p["MH"], p["P"])
    assert info.off_B == p["offsets"]["B"] and info.off_Ut == p["offsets"]["Ut"]
    assert info.off_Vt == p["offsets"]["Vt"] and info.off_lam == p["offsets"]["lam"]
    tiles = np.array(p["tiles"], dtype=np.int64).reshape(-1, 4)
    assert np.array_equal(t["level"], tiles[:, 0]) and np.array_equal(t["row0"], tiles[:, 1])
    assert np.array_equal(t["col0"], tiles[:, 2]) and np.array_equal(t["span"], tiles[:, 3])
    assert np.array_equal(t["leaf_tile"], p["leaf_tile"]) and np.array_equal(t["leaf_side"], p["leaf_side"])


def test_partition_shape_errors():
    with pytest.raises(hp.HPError) as e:
        hp.build_partition(1000, 64, 16)
    assert e.value.status == 2
    with pytest.raises(hp.HPError) as e:
        hp.build_partition(64 * 3, 64, 16)
    assert e.value.status == 2


@pytest.mark.parametrize("cfg", [inputs.MODEL_PLAIN, inputs.MODEL_DEFAULT])
def test_weight_layout_matches_spec(cfg):
    lay = hp.weight_layout(cfg)
    spec = inputs.weight_spec(cfg)
    assert [(n, s) for n, s, _ in lay] == [(n, tuple(s)) for n, s, _ in spec]
    off = 0
    for n, s, o in lay:
        assert o == off
        off += int(np.prod(s))
    w = inputs.init_weights(cfg, 1)
    flat = hp.pack_weights(cfg, w)
    assert flat.size == inputs.param_count(cfg)
