"""Hand-computed pins of the oracle's network pieces (CPU only).

Each case is small enough to work out by hand; the expected values below are
written from that working, not from the oracle's code.  They target the
mistakes a reading of Sec. 4.1-4.2 and the Supplementary "Network
Architecture Details" could plausibly make: the split of the QKV columns into
heads, the 1/sqrt(d_h) logit scale, the orientation of the pair bias and of
the [in, out] weight layout, the exact-erf GELU, the edge-descriptor sign and
every one of the 20 encoder input columns.
"""
import math

import numpy as np
import torch

from oracle import grid, network, partition

EPS = 1e-5
PHI1 = 0.8413447460685429       # standard normal CDF at 1
PHI_M1 = 0.15865525393145707    # ... at -1


def _t(a):
    return torch.tensor(a, dtype=torch.float64)


def test_gelu_exact_erf_values():
    g = network.gelu(_t([1.0, -1.0, 0.0, 2.0]))
    # GELU(x) = x Phi(x); Phi(2) = 0.9772498680518208
    assert abs(float(g[0]) - PHI1) < 1e-15
    assert abs(float(g[1]) + PHI_M1) < 1e-15
    assert float(g[2]) == 0.0
    assert abs(float(g[3]) - 2 * 0.9772498680518208) < 1e-15


def test_softplus_values():
    sp = network.softplus(_t([0.0, 40.0, -40.0, 1.0]))
    assert abs(float(sp[0]) - math.log(2.0)) < 1e-15
    assert abs(float(sp[1]) - 40.0) < 1e-15
    assert abs(float(sp[2]) - 4.248354255291589e-18) < 1e-30   # e^-40
    assert abs(float(sp[3]) - 1.3132616875182228) < 1e-15       # ln(1 + e)


def test_softmax_rows_sum_to_one_and_shift_invariance():
    rng = np.random.default_rng(0)
    s = _t(rng.standard_normal((5, 7)) * 30)
    p = network.softmax(s)
    assert torch.all(p >= 0)
    assert torch.allclose(p.sum(-1), torch.ones(5, dtype=torch.float64), atol=1e-15, rtol=0)
    assert torch.allclose(network.softmax(s + 123.0), p, atol=1e-15, rtol=0)
    # two logits: the first weight is the logistic function of their difference
    q = network.softmax(_t([[0.7, -0.3]]))
    assert abs(float(q[0, 0]) - 1.0 / (1.0 + math.exp(-1.0))) < 1e-15


def test_layernorm_moments_and_affine():
    rng = np.random.default_rng(1)
    x = _t(rng.standard_normal((6, 16)) * 3 + 2)
    y = network.layernorm(x, torch.ones(16, dtype=torch.float64), torch.zeros(16, dtype=torch.float64))
    var = x.var(-1, unbiased=False)
    assert torch.allclose(y.mean(-1), torch.zeros(6, dtype=torch.float64), atol=1e-14, rtol=0)
    # population variance of the output is var / (var + eps)
    assert torch.allclose(y.var(-1, unbiased=False), var / (var + EPS), atol=1e-14, rtol=0)
    # gain and shift act per feature: the row [1, -1, 1, -1] has mean 0, variance 1
    g, b = _t([1.0, 2.0, 3.0, 4.0]), _t([0.5, 0.0, -0.5, 1.0])
    z = network.layernorm(_t([[1.0, -1.0, 1.0, -1.0]]), g, b)
    s = 1.0 / math.sqrt(1.0 + EPS)
    assert torch.allclose(z, _t([[0.5 + s, -2 * s, -0.5 + 3 * s, 1.0 - 4 * s]]), atol=1e-15, rtol=0)


def test_edge_mlp_hand_case():
    # e1: 4 -> 2 with rows [in] x columns [out]; e2: 2 -> 1
    w = {"p.e1.w": _t([[1.0, -1.0], [5.0, 5.0], [0.0, 0.0], [0.0, 0.0]]), "p.e1.b": _t([0.0, 0.0]),
         "p.e2.w": _t([[2.0], [3.0]]), "p.e2.b": _t([0.5])}
    out = network._edge_mlp(_t([[1.0, 0.0, 0.0, 0.0]]), w, "p.")
    assert abs(float(out[0, 0]) - (2 * PHI1 - 3 * PHI_M1 + 0.5)) < 1e-15
    # the second input feeds both hidden units through row 1 of e1.w
    out = network._edge_mlp(_t([[0.0, 0.2, 0.0, 0.0]]), w, "p.")
    assert abs(float(out[0, 0]) - (5 * PHI1 + 0.5)) < 1e-15


def test_attention_hand_case_two_heads_three_tokens():
    """d = 4, two heads (d_h = 2, head h takes QKV columns [2h, 2h+2) of each
    of the Q, K, V blocks), three tokens, Q = K = V = LN(X) (identity QKV
    weights), a masked asymmetric pair bias that leaves each query two keys,
    and an output map that rotates the columns."""
    X = _t([[1.0, -1.0, 1.0, -1.0],
            [1.0, 1.0, -1.0, -1.0],
            [1.0, -1.0, -1.0, 1.0]])          # every row: mean 0, variance 1
    s = 1.0 / math.sqrt(1.0 + EPS)            # LN1 with unit gain: a = s X
    MASK = -1e30
    # allowed (query -> key: bias) per head; every other pair is masked
    allowed = {0: {0: {0: 0.3, 1: -0.2}, 1: {1: 0.1, 2: 0.5}, 2: {1: -0.4, 2: 0.0}},
               1: {0: {0: 0.2, 2: 0.1}, 1: {0: -0.3, 1: 0.0}, 2: {1: 0.25, 2: -0.1}}}
    bias = torch.full((1, 2, 3, 3), MASK, dtype=torch.float64)
    for h, rows in allowed.items():
        for i, keys in rows.items():
            for j, v in keys.items():
                bias[0, h, i, j] = v
    bv = [0.05, -0.05, 0.0, 0.1]
    Wo = torch.zeros(4, 4, dtype=torch.float64)
    for k in range(4):
        Wo[k, (k + 1) % 4] = 1.0                 # Y[:, k+1] = O[:, k]
    bo = [0.1, 0.2, 0.3, 0.4]
    eye = torch.eye(4, dtype=torch.float64)
    w = {"a.ln1.g": torch.ones(4, dtype=torch.float64), "a.ln1.b": torch.zeros(4, dtype=torch.float64),
         "a.qkv.w": torch.cat([eye, eye, eye], dim=1), "a.qkv.b": _t([0.0] * 8 + bv),
         "a.o.w": Wo, "a.o.b": _t(bo)}
    Y = network._attention(X.reshape(1, 3, 4), bias, w, "a.", 2)[0]

    # worked by hand: head 0 sees columns 0-1 of every token, head 1 columns 2-3
    # head 0 dots x_i[0:2].x_j[0:2]: (0,0)=2 (0,1)=0 (1,1)=2 (1,2)=0 (2,1)=0 (2,2)=2
    # head 1 dots x_i[2:4].x_j[2:4]: (0,0)=2 (0,2)=-2 (1,0)=0 (1,1)=2 (2,1)=0 (2,2)=2
    dots = {0: {(0, 0): 2, (0, 1): 0, (1, 1): 2, (1, 2): 0, (2, 1): 0, (2, 2): 2},
            1: {(0, 0): 2, (0, 2): -2, (1, 0): 0, (1, 1): 2, (2, 1): 0, (2, 2): 2}}
    O = np.zeros((3, 4))
    for h in (0, 1):
        for i in range(3):
            (j1, b1), (j2, b2) = allowed[h][i].items()
            # logit = s^2 dot / sqrt(2) + bias; weight of j1 = logistic(logit1 - logit2)
            delta = s * s * (dots[h][(i, j1)] - dots[h][(i, j2)]) / math.sqrt(2.0) + (b1 - b2)
            p = 1.0 / (1.0 + math.exp(-delta))
            for c in (2 * h, 2 * h + 1):
                v1 = s * float(X[j1, c]) + bv[c]
                v2 = s * float(X[j2, c]) + bv[c]
                O[i, c] = p * v1 + (1.0 - p) * v2
    expect = X.numpy() + np.roll(O, 1, axis=1) + np.array(bo)
    assert np.abs(Y.detach().numpy() - expect).max() < 1e-14


def _rho_4x2x2():
    rho = np.ones(16)
    rho[1] = 4.0          # cell (x=1, y=0, z=0), lexicographic id 1
    return rho


# Morton order of the 4 x 2 x 2 grid: x bit 0 -> code bit 0, y -> 1, z -> 2,
# x bit 1 -> code bit 3
MORTON_XYZ = [(0, 0, 0), (1, 0, 0), (0, 1, 0), (1, 1, 0), (0, 0, 1), (1, 0, 1), (0, 1, 1), (1, 1, 1),
              (2, 0, 0), (3, 0, 0), (2, 1, 0), (3, 1, 0), (2, 0, 1), (3, 0, 1), (2, 1, 1), (3, 1, 1)]
# A_ii by hand: one face weight 1 between two light cells, 2/(1+4) = 0.4 at
# the heavy cell's faces, plus 1/rho on the top layer (z = 1)
DIAG_BY_XYZ = {(0, 0, 0): 2.4, (1, 0, 0): 1.6, (2, 0, 0): 3.4, (3, 0, 0): 3.0,
               (0, 1, 0): 3.0, (1, 1, 0): 3.4, (2, 1, 0): 4.0, (3, 1, 0): 3.0,
               (0, 0, 1): 4.0, (1, 0, 1): 4.4, (2, 0, 1): 5.0, (3, 0, 1): 4.0,
               (0, 1, 1): 4.0, (1, 1, 1): 5.0, (2, 1, 1): 5.0, (3, 1, 1): 4.0}


def test_features_4x2x2_every_column():
    f = grid.features(4, 2, 2, _rho_4x2x2())
    assert f.shape == (16, 20)
    L4 = math.log(4.0)
    la = np.log([DIAG_BY_XYZ[p] for p in MORTON_XYZ])
    glob = [0.25,                          # log2(16) / 16
            L4,                            # log(rho_max / rho_min)
            L4 / 16, L4 * math.sqrt(15) / 16,   # mean, population std of log rho
            1.0 / 16,                      # heavy fraction
            la.mean(), la.std(), la.min(), la.max(),
            4 / 32, 2 / 32, 2 / 32]
    for m, (x, y, z) in enumerate(MORTON_XYZ):
        heavy = (x, y, z) == (1, 0, 0)
        node = [L4 if heavy else 0.0, (x + 0.5) / 4, (y + 0.5) / 2, (z + 0.5) / 2,
                1.0 if z == 1 else 0.0,    # top
                1.0,                       # side: every cell touches y = 0 or y = 1
                1.0 if z == 0 else 0.0,    # bottom
                math.log(DIAG_BY_XYZ[(x, y, z)])]
        assert np.abs(f[m] - np.array(node + glob)).max() < 1e-14, m
    # the diagonal itself, and the row of the heavy cell
    A = grid.assemble(4, 2, 2, _rho_4x2x2())
    assert np.allclose(A.diagonal(), [DIAG_BY_XYZ[p] for p in MORTON_XYZ], atol=1e-15, rtol=0)
    # heavy cell is Morton index 1; its neighbours (0,0,0), (1,1,0), (1,0,1), (2,0,0) are 0, 3, 5, 8
    row = A.getrow(1).toarray()[0]
    assert np.allclose(row[[0, 3, 5, 8]], -0.4, atol=1e-15, rtol=0) and abs(row[1] - 1.6) < 1e-15


def test_edge_descriptor_sign_hand_pair():
    fs = network.FrameSys(4, 2, 2, _rho_4x2x2(), 8, 2)
    # within leaf 0: query 0 at (0,0,0), key 1 at (1,0,0): dx = pos(key) - pos(query) = +1
    ahat = -0.4 / math.sqrt(2.4 * 1.6)
    assert np.allclose(fs.desc_diag[0, 0, 1], [0.25, 0.0, 0.0, ahat], atol=1e-15, rtol=0)
    assert np.allclose(fs.desc_diag[0, 1, 0], [-0.25, 0.0, 0.0, ahat], atol=1e-15, rtol=0)
    # (0,0,0) -> (0,1,0) is Morton 0 -> 2: +y; (0,0,0) -> (0,0,1) is 0 -> 4: +z
    assert np.allclose(fs.desc_diag[0, 0, 2, :3], [0.0, 0.25, 0.0], atol=1e-15, rtol=0)
    assert np.allclose(fs.desc_diag[0, 0, 4, :3], [0.0, 0.0, 0.25], atol=1e-15, rtol=0)
    # no stencil link: zero coupling entry
    assert fs.desc_diag[0, 0, 7, 3] == 0.0
    # off-diagonal (one tile at N = 16, L = 8): rows = leaf 0, columns = leaf 1, p = 4;
    # sub-strip 0 of leaf 0 is Morton 0..3 (x in {0,1}, y in {0,1}, z = 0): centroid (0.5, 0.5, 0)
    # sub-strip 0 of leaf 1 is Morton 8..11: centroid (2.5, 0.5, 0); dx = (2, 0, 0) / 4
    part = partition.build(16, 8, 2)
    assert part["MH"] == 1
    assert np.allclose(fs.desc_off[0, 0, 0, :3], [0.5, 0.0, 0.0], atol=1e-15, rtol=0)
    # couplings between Morton 0..3 and 8..11: (1,0,0)-(2,0,0) [heavy, 0.4] and (1,1,0)-(2,1,0) [1]
    a1 = -0.4 / math.sqrt(1.6 * 3.4)
    a2 = -1.0 / math.sqrt(3.4 * 4.0)
    assert abs(fs.desc_off[0, 0, 0, 3] - (a1 + a2) / 16) < 1e-15


def test_sai_ablation_loss_pins():
    """The SAI-style loss of the loss ablation (Prop. 1(3)), || A M Z / ||A|| - Z ||_F^2
    with ||A|| read as the largest absolute row sum: that scale equals the
    brute-force row sums and bounds the spectral norm; M = ||A|| A^-1 gives
    exactly zero; the loss is not invariant under M -> alpha M, and its minimum
    over scalings sits at the closed form beta* = <Z, W> / ||W||^2 (W = A M Z / ||A||)."""
    import warnings
    from oracle import grid, loss
    from paper_2605_13343_amd import inputs
    fr = inputs.make_frame_grid(4, 4, 4, 3)
    A = grid.assemble(fr.nx, fr.ny, fr.nz, fr.rho)
    Ad = A.toarray()
    s = loss.sai_scale(A)
    assert s == max(sum(abs(Ad[i, j]) for j in range(fr.n)) for i in range(fr.n))
    assert s >= np.linalg.norm(Ad, 2) - 1e-12
    rng = np.random.default_rng(4)
    Z = np.where(rng.random((fr.n, 3)) < 0.5, -1.0, 1.0)
    Minv = s * np.linalg.inv(Ad)
    assert loss.sai_train_loss(A, Z, Minv @ Z) <= 1e-20 * (Z * Z).sum()
    M = np.diag(1.0 / np.diag(Ad))  # Jacobi as a stand-in M
    L1 = loss.sai_train_loss(A, Z, M @ Z)
    assert abs(loss.sai_train_loss(A, Z, 2.0 * M @ Z) - L1) > 1e-3 * L1
    W = (A @ (M @ Z)) / s
    beta = float((Z * W).sum() / (W * W).sum())
    Lb = loss.sai_train_loss(A, Z, beta * M @ Z)
    for db in (-1e-3, 1e-3, -0.1, 0.1):
        assert Lb <= loss.sai_train_loss(A, Z, (beta + db) * M @ Z)
    assert abs(Lb - (Z * Z).sum() * (1.0 - (Z * W).sum() ** 2 / ((Z * Z).sum() * (W * W).sum()))) <= 1e-9 * L1
    # the torch form (autograd in the oracle's gradient) equals the numpy form
    import torch
    with warnings.catch_warnings():
        warnings.simplefilter("ignore")
        Lt = float(loss.sai_train_loss(A, Z, torch.as_tensor(M @ Z)))
    assert abs(Lt - L1) <= 1e-12 * L1
