"""Host check of the ordering the Dormand-Prince error maximum relies on: the
stage-7 field pass folds the workgroups' largest per-cell error norms into
one word with an unsigned integer atomic maximum of their IEEE-754 single
bit patterns.  That equals the floating-point maximum because every value
folded is a non-negative float (a norm, +0 included) or +inf (a NaN norm is
mapped to +inf before the fold): for those, the bit patterns order as the
values do.  Checked here over random, subnormal and boundary values."""
import numpy as np


def _fold_bits(x):
    return np.max(np.asarray(x, dtype=np.float32).view(np.uint32))


def test_bits_max_equals_float_max_on_nonnegative_floats():
    rng = np.random.default_rng(20410)
    specials = np.array([0.0, np.float32(1e-45), np.float32(1.1754942e-38),
                         np.float32(1.1754944e-38), 1.0, 3.4028235e38,
                         np.inf], dtype=np.float32)
    for trial in range(200):
        n = int(rng.integers(1, 300))
        e = rng.uniform(-45, 38, size=n)
        x = (rng.uniform(0, 1, size=n) * 10.0 ** e).astype(np.float32)
        if trial % 3 == 0:
            x = np.concatenate([x, rng.choice(specials, size=3)])
        bits = _fold_bits(x)
        assert np.uint32(bits).view(np.float32) == np.max(x)
    # pairwise order of the special values matches their bit order
    for a in specials:
        for b in specials:
            ba, bb = np.float32(a).view(np.uint32), np.float32(b).view(np.uint32)
            assert (a < b) == (ba < bb) and (a == b) == (ba == bb)


def test_nan_is_mapped_before_the_fold():
    # every NaN pattern sorts above +inf as an unsigned word, so a NaN would
    # win the fold, but read back as a NaN the controller's fmax with the
    # cavity error would drop it and accept; the field pass therefore folds
    # +inf (reject) in its place
    inf_bits = np.float32(np.inf).view(np.uint32)
    for nan_bits in (0x7FC00000, 0x7F800001, 0xFFC00000, 0xFFFFFFFF):
        assert np.uint32(nan_bits) > inf_bits
        assert np.isnan(np.uint32(nan_bits).view(np.float32))
    assert np.fmax(np.float64(np.nan), 1e-9) == 1e-9
    x = np.array([0.5, np.nan, 2.0], dtype=np.float32)
    mapped = np.where(np.isnan(x), np.float32(np.inf), x)
    assert np.uint32(_fold_bits(mapped)).view(np.float32) == np.inf
    # a norm is never -0: squares and their sums are +0 at least
    z = np.float32(-0.0)
    assert np.signbit(np.sqrt(z * z + z * z + z * z)) == False
