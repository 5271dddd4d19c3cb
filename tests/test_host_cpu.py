"""Host-side helpers of the package against the oracle (no GPU needed)."""
import dataclasses

import numpy as np
import pytest

import oracle
import synth


@pytest.fixture(scope="module")
def pkg():
    import paper_2603_16575_amd as m
    return m


def slot_list(prob):
    """Slots in the K layout: the diagonal (p, p) of every LMO, then the
    pairs in their sorted order."""
    return [(p, p) for p in range(prob.n_occ)] + [tuple(int(v) for v in pq) for pq in prob.pairs]


def test_first_order_dE_matches_finite_difference(pkg):
    """first_order_dE with the oracle's multipliers W reproduces the central
    difference of the oracle's MBE(3) energy along a random change of every
    K-bar block (diagonal slots, kept symmetric, and pairs): this fixes the
    slot weights 2 and 4 and the packing of the K layout."""
    prob = dataclasses.replace(synth.micro(4), tol=1e-13, max_iter=400)
    g = oracle.gradient(prob)
    ora0 = g["run"]["oracle"]
    slots = slot_list(prob)
    d = [oracle.orbs(p, q) for p, q in slots]
    d = [int(sum(prob.r[x] for x in o)) for o in d]
    k_off = np.concatenate([[0], np.cumsum(np.square(d))]).astype(np.int64)
    rng = np.random.default_rng(3)
    K0 = np.concatenate([ora0.Kbar(p, q).ravel() for p, q in slots])
    dK = rng.standard_normal(K0.shape) * np.abs(K0).max()
    for s in range(prob.n_occ):  # K-bar_pp = G G^T stays symmetric
        blk = dK[k_off[s]:k_off[s + 1]].reshape(d[s], d[s])
        dK[k_off[s]:k_off[s + 1]] = (0.5 * (blk + blk.T)).ravel()
    W = np.concatenate([g["W"][s].ravel() for s in slots])

    def energy_at(eps):
        ora = oracle.Oracle(prob)
        for s, (p, q) in enumerate(slots):
            blk = (K0 + eps * dK)[k_off[s]:k_off[s + 1]]
            ora._K[(p, q)] = blk.reshape(d[s], d[s])
        return oracle.energy(prob, ora=ora)

    h = 1e-5
    fd = (energy_at(h) - energy_at(-h)) / (2 * h)
    est, per = pkg.first_order_dE(k_off, prob.n_occ, K0 + dK, K0, W)
    assert per.shape == (len(slots),)
    assert np.isclose(per.sum(), est)
    assert abs(est - fd) <= 1e-7 * abs(fd)
    # a change of the diagonal slots alone carries weight 2, pairs alone 4
    mask = np.zeros_like(dK)
    mask[:k_off[prob.n_occ]] = 1.0
    e_diag, _ = pkg.first_order_dE(k_off, prob.n_occ, K0 + mask * dK, K0, W)
    assert np.isclose(e_diag, 2.0 * float(np.sum((mask * dK) * W)))


def test_pair_classes_match_oracle(pkg):
    """The package's class and trimer helpers use the oracle's thresholds."""
    from oracle import weak
    vals = [0.0, 5e-8, 1e-7, 2e-4, 9.99e-3, 1e-2, 0.5]
    names = {0: "distant", 1: "weak", 2: "close"}
    got = pkg.pair_classes(vals)
    assert [names[int(c)] for c in got] == [weak.pair_class(v) for v in vals]
    trip = [(0.3, 0.2, 0.1 + 1e-12), (0.3, 0.2, 0.1 - 1e-9), (0.05, 0.01, 0.02)]
    assert [bool(pkg.keep_trimers(*t)) for t in trip] == [weak.keep_trimer(*t) for t in trip]
