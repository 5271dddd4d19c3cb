"""Host-side logic of the library (no GPU needed): the pair classes and
trimer screening of mbe3_screen_lists against the oracle's brute-force
screening, with the paper's thresholds."""
import numpy as np
import pytest

import oracle
import synth
from oracle import weak


@pytest.fixture(scope="module")
def pkg():
    import paper_2603_16575_amd as m
    m._lib.load()
    return m


def test_screen_lists_thresholds(pkg):
    """Class boundaries as printed (distant below 1e-7, weak below 1e-2,
    close from 1e-2), the trimer boundary at s3b = 0.2, and the order of the
    returned lists."""
    vals = [0.0, 5e-8, 1e-7, 2e-4, 9.99e-3, 1e-2, 0.5]
    names = {0: "distant", 1: "weak", 2: "close"}
    pairs = np.array([[0, k + 1] for k in range(len(vals))])
    out = pkg.screen_lists(len(vals) + 1, pairs, vals)
    assert [names[int(c)] for c in out["classes"]] == [weak.pair_class(v) for v in vals]
    # trimers: (0,1,2) with metrics 0.3, 0.2, 0.1 +- a little
    for s_jk, keep in ((0.1 + 1e-12, True), (0.1 - 1e-9, False)):
        p3 = np.array([[1, 2], [0, 2], [0, 1]])
        got = pkg.screen_lists(3, p3, [s_jk, 0.2, 0.3])
        assert got["close"].tolist() == [[0, 1], [0, 2], [1, 2]]
        assert (len(got["trimers"]) == 1) == keep == weak.keep_trimer(0.3, 0.2, s_jk)
    # a weak side removes the trimer whatever the mean
    got = pkg.screen_lists(3, np.array([[0, 1], [0, 2], [1, 2]]), [0.9, 0.9, 5e-3])
    assert len(got["trimers"]) == 0 and got["weak"].tolist() == [[1, 2]]


def test_screen_lists_water40u_against_oracle(pkg):
    """Every pair of the 160-LMO lattice with its s2b from the oracle: the
    library's classes, close and weak lists and kept trimers equal the
    oracle's brute-force screening exactly."""
    prob = synth.config(1)
    ora = oracle.Oracle(prob)
    n = prob.n_occ
    iu = np.triu_indices(n, 1)
    pairs = np.stack(iu, 1).astype(np.int32)
    s = np.array([weak.s2b(ora, int(i), int(j)) for i, j in pairs])
    out = pkg.screen_lists(n, pairs[:, ::-1], s)  # either orientation accepted
    close, wk, tris = weak.screened_lists(n, {(int(i), int(j)): v for (i, j), v in zip(pairs, s)})
    assert [tuple(x) for x in out["close"].tolist()] == close
    assert [tuple(x) for x in out["weak"].tolist()] == wk
    assert [tuple(x) for x in out["trimers"].tolist()] == tris
    assert len(close) > 0 and len(wk) > 0 and 0 < len(tris) < 10000


def test_screen_lists_errors(pkg):
    lib = pkg._lib.load()
    with pytest.raises(pkg.Mbe3Error):
        pkg.screen_lists(3, np.array([[0, 1], [1, 0]]), [0.5, 0.5])  # repeated
    with pytest.raises(pkg.Mbe3Error):
        pkg.screen_lists(3, np.array([[0, 3]]), [0.5])  # out of range
    with pytest.raises(pkg.Mbe3Error):
        pkg.screen_lists(3, np.array([[1, 1]]), [0.5])  # same orbital
    with pytest.raises(pkg.Mbe3Error):
        pkg.screen_lists(3, np.array([[0, 1]]), [np.nan])
    assert "not finite" in lib.mbe3_last_error(None).decode()
    out = pkg.screen_lists(4, np.zeros((0, 2)), [])
    assert len(out["close"]) == len(out["weak"]) == len(out["trimers"]) == 0
