"""Pins of O1 (slab regeneration): Philox4x64-10 and Box-Muller."""
import numpy as np
import pytest

import oracle
import synth


@pytest.mark.parametrize("key,ctr", [
    ((5, 7), (0, 0, 0, 0)),
    ((2603165750, 0), (17, 3, 9, 0)),
    ((2 ** 64 - 1, 123), (2 ** 64 - 1, 5, 9, 2 ** 63)),  # carry into word 1
])
def test_philox_matches_numpy(key, ctr):
    """numpy.random.Philox emits f(c+1), f(c+2), ... for counter c."""
    bg = np.random.Philox(key=np.array(key, dtype=np.uint64),
                          counter=np.array(ctr, dtype=np.uint64))
    ref = bg.random_raw(12)
    c = [int(x) for x in ctr]
    blocks = []
    for n in range(1, 4):
        v = c[0] + n
        w1 = c[1] + (v >> 64)
        blocks.append([v & (2 ** 64 - 1), w1 & (2 ** 64 - 1), c[2], c[3]])
    mine = oracle.philox4x64_10(np.array(blocks, dtype=np.uint64), key).ravel()
    assert np.array_equal(ref, mine)


def test_box_muller_moments():
    n = 1 << 20
    ctr = np.zeros((n, 4), dtype=np.uint64)
    ctr[:, 0] = np.arange(n, dtype=np.uint64)
    w = oracle.philox4x64_10(ctr, (11, 0))
    z = oracle.box_muller(w[:, 0], w[:, 1])
    assert abs(z.mean()) < 5.0 / np.sqrt(n)
    assert abs(z.var() - 1.0) < 8.0 / np.sqrt(n)
    assert abs(np.mean(z ** 4) - 3.0) < 0.05
    assert np.isfinite(z).all()


def test_box_muller_extremes():
    """u1 never reaches 0 or 1: all-zero and all-one words stay finite."""
    x = np.array([0, 2 ** 64 - 1], dtype=np.uint64)
    z = oracle.box_muller(x, x)
    assert np.isfinite(z).all()
    # u1 = 0.5 * 2^-53 -> sqrt(-2 ln u1) = sqrt(2 * 53.69 * ln 2)
    assert np.isclose(z[0], np.sqrt(-2.0 * np.log(0.5 * 2.0 ** -53)))


def test_slab_counter_layout():
    """Slab element (i, a, P) depends only on its own counter (tile-order
    independent) and carries the two distance weights."""
    p = synth.config(0)
    B = oracle.slab(p, 3, impl="numpy")
    a, P = 17, 101
    ctr = np.array([[P, a, 3, 0]], dtype=np.uint64)
    w = oracle.philox4x64_10(ctr, (p.seed, 0))
    z = oracle.box_muller(w[:, 0], w[:, 1])[0]
    assert B[a, P] == (z * p.w_ia[3, a]) * p.w_iP[3, P]
    assert B.shape == (p.n_vir, p.n_aux)


def test_c_slab_matches_numpy():
    """The oracle's C slab routine against the numpy one: Philox words bit for
    bit (random counters and keys, carries included), slab elements within
    4 ulp (libm's log / cos against numpy's), a column subset equal to the
    same columns of the full slab."""
    from oracle import _clib
    rng = np.random.default_rng(3)
    ctr = rng.integers(0, 2 ** 63, size=(4096, 4), dtype=np.uint64)
    ctr[:5, 0] = np.uint64(2 ** 64 - 1)
    for key in ((5, 7), (2603165750, 0), (2 ** 64 - 1, 10)):
        assert np.array_equal(oracle.philox4x64_10(ctr, key), _clib.philox_raw(ctr, key))
    p = synth.config(0)
    for i in (0, 3, 7):
        Bn = oracle.slab(p, i, impl="numpy")
        Bc = oracle.slab(p, i)
        ulp = np.abs(Bc - Bn) / np.spacing(np.abs(Bn))
        assert ulp.max() <= 4
        cols = np.array([0, 5, 191, 17])
        assert np.array_equal(oracle.slab(p, i, cols=cols), Bc[:, cols])
