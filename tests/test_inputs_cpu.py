"""Seeded input generators (shared by the oracle tests and the GPU path as
data only): determinism, ranges, distributions, and the learned smoother's
draws (initial weights, crop offsets, epoch orders)."""
import numpy as np

import oracle.learned as LN
from paper_1210_7774_amd import inputs as I


def test_generators_are_deterministic():
    assert np.array_equal(I.normal_rhs(31, 2, 5), I.normal_rhs(31, 2, 5))
    assert not np.array_equal(I.normal_rhs(31, 2, 5), I.normal_rhs(31, 2, 6))
    assert np.array_equal(I.lognormal_coef_2d(31, 7), I.lognormal_coef_2d(31, 7))


def test_lognormal_field_statistics():
    """a = exp(g), g a zero-mean Gaussian field with sigma 1: over many
    seeds the sample mean of g is near 0 and its variance near 1."""
    gs = np.stack([I.gaussian_field_2d(63, s) for s in range(40)])
    assert gs.shape == (40, 65, 65)
    assert abs(gs.mean()) < 0.15
    assert abs(gs.var() - 1.0) < 0.2
    a = I.lognormal_coef_2d(63, 3)
    assert np.all(a > 0) and np.all(np.isfinite(a))


def test_he_normal_weights_layout_and_scale():
    w = I.he_normal_weights(7000)
    assert w.dtype == np.float32 and w.size == LN.NWEIGHTS
    # per layer: zero mean, std sqrt(2 / (9 c_in)) within sampling error
    k = 0
    for co, ci in LN.SHAPES:
        m = co * ci * 9
        part = w[k:k + m].astype(np.float64)
        want = np.sqrt(2.0 / (9 * ci))
        assert abs(part.std() / want - 1.0) < 4.0 / np.sqrt(m) + 0.02, (co, ci)
        k += m
    # the same draw as the oracle's He-normal helper with the same generator
    ref = LN.he_normal(I.rng(7000)).astype(np.float32)
    assert np.array_equal(w, ref)


def test_crop_offsets_in_range():
    off = I.crop_offsets(127, 32, 500, 9)
    assert off.dtype == np.int32 and off.shape == (500, 2)
    assert off.min() >= 0 and off.max() <= 127 - 32
    # both ends of the range occur for a large draw
    big = I.crop_offsets(40, 8, 20000, 10)
    assert big.min() == 0 and big.max() == 32


def test_epoch_orders_are_permutations():
    o = I.epoch_orders(100, 3, 11)
    assert o.dtype == np.int32 and o.size == 300
    for e in range(3):
        assert np.array_equal(np.sort(o[e * 100:(e + 1) * 100]), np.arange(100))
    assert not np.array_equal(o[:100], o[100:200])
