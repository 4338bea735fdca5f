"""Pins of the binning oracle (Sec. III-A binning, the approximate order of
the footnote to Table II), checked against properties its formula does not
restate: the footnote's ordering, stability, and the exact sort it reduces to."""
import numpy as np
import pytest

from oracle import binning


def _cloud(rng, n, kind):
    if kind == "uniform":
        return rng.random((n, 3), dtype=np.float32)
    if kind == "ties":          # few distinct coordinates: bins hold equal values
        return rng.integers(-3, 4, (n, 3)).astype(np.float32)
    return (rng.standard_normal((n, 3)) * 40).astype(np.float32)


@pytest.mark.parametrize("kind", ["uniform", "ties", "wide"])
def test_footnote_order_and_stability(kind):
    rng = np.random.default_rng(3)
    for _ in range(30):
        n = int(rng.integers(1, 3000))
        pts = _cloud(rng, n, kind)
        axis = int(rng.integers(0, 3))
        bins = int(rng.integers(1, 300))
        perm, b = binning.bin_points(pts, axis, bins)
        assert sorted(perm.tolist()) == list(range(n))                 # a permutation
        bp = b[perm]
        assert np.all(np.diff(bp) >= 0)                                  # bins ascending
        assert bp.min() >= 0 and bp.max() < bins
        x = pts[perm, axis]
        for lo_bin, hi_bin in zip(np.unique(bp)[:-1], np.unique(bp)[1:]):
            # every point of a later bin has a larger coordinate (footnote)
            assert x[bp == hi_bin].min() > x[bp == lo_bin].max()
        for v in np.unique(bp):                                          # storage order kept inside a bin
            assert np.all(np.diff(perm[bp == v]) > 0)
        # equal coordinates never straddle bins
        for val in np.unique(pts[:, axis])[:20]:
            assert np.unique(b[pts[:, axis] == val]).size == 1


def test_one_bin_is_the_identity():
    rng = np.random.default_rng(4)
    pts = rng.random((500, 3), dtype=np.float32)
    assert binning.bin_points(pts, 1, 1)[0].tolist() == list(range(500))


def test_one_bin_per_integer_is_the_exact_sort():
    """Coordinates 0..N-1 in random order with N bins: t = x * N/(N-1) has
    floor x for x < N-1 and is clamped to N-1 at the top, so the binning is
    the exact sort."""
    rng = np.random.default_rng(5)
    for n in (2, 3, 17, 1000, 4099):
        x = rng.permutation(n).astype(np.float32)
        pts = np.stack([rng.random(n), x, rng.random(n)], 1).astype(np.float32)
        perm, _ = binning.bin_points(pts, 1, n)
        assert perm.tolist() == np.argsort(x, kind="stable").tolist()


def test_constant_coordinate_is_one_bin():
    pts = np.zeros((64, 3), np.float32)
    pts[:, 0] = 2.5
    perm, b = binning.bin_points(pts, 0, 16)
    assert perm.tolist() == list(range(64)) and np.all(b == 0)


def test_arguments_checked():
    with pytest.raises(ValueError):
        binning.bin_points(np.zeros((0, 3), np.float32), 0, 4)
    with pytest.raises(ValueError):
        binning.bin_points(np.zeros((4, 3), np.float32), 3, 4)
    with pytest.raises(ValueError):
        binning.bin_points(np.zeros((4, 3), np.float32), 0, 0)
