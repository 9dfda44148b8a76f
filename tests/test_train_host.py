"""Host logic of the GPU trainer (no GPU): the reduce-on-plateau rule of
Supplementary "Optimizer and schedule" and the seed schedule."""
import numpy as np

from paper_2605_13343_amd import train


def test_plateau_halves_after_patience_and_stops_at_floor():
    p = train.Plateau(2e-4)
    assert p.min_lr == max(2e-4 * 1e-3, 1e-6)
    assert p.update(1.0) == 2e-4            # first value is an improvement
    for _ in range(5):                       # patience 5: five bad log steps keep the rate
        assert p.update(1.0) == 2e-4
    assert p.update(1.0) == 1e-4            # the sixth halves it
    # an improvement by more than the relative threshold resets the count
    assert p.update(0.99) == 1e-4 and p.bad == 0
    # less than the 5e-3 relative threshold counts as no improvement
    p.update(0.99 * (1 - 4e-3))
    assert p.bad == 1
    for _ in range(200):
        p.update(10.0)
    assert p.lr == p.min_lr


def test_training_seeds_avoid_validation_and_benchmark_seeds():
    held_out = set(range(2000, 2020)) | set(range(3900, 3920)) | set(range(7000, 7020))
    for recipe, base in train.SEED_BASE.items():
        # 10^5 steps of 32 systems stay inside a band that no held-out seed touches
        lo, hi = base, base + 32 * 100_000
        assert not any(lo <= s < hi for s in held_out), recipe
    bases = sorted(train.SEED_BASE.values())
    assert all(b - a >= 1_000_000 for a, b in zip(bases, bases[1:]))


def test_unpack_inverts_pack():
    from paper_2605_13343_amd import hp, inputs
    cfg = inputs.MODEL_PLAIN
    w = inputs.init_weights(cfg, 3)
    flat = hp.pack_weights(cfg, w)
    back = train.unpack(cfg, flat)
    assert set(back) == set(w)
    for k in w:
        assert np.array_equal(back[k], w[k])
