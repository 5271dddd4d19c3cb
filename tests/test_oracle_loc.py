"""Pins of the localization oracle (oracle/loc.py) against what the
mathematics fixes: the charges sum to the identity over the atoms, the pair
angle of eq. loc_theta (read with the two-argument arctangent) is the
maximizer of the functional over the rotation angle found by a dense scan,
each rotation raises the functional by exactly the printed increment, the
functional never decreases over a sweep, U stays orthogonal and relates the
final charges to the initial ones (P = U^T P0 U for every atom), and the
localization of orbitals mixed from localized ones recovers orbitals as
localized as those."""
import math

import numpy as np
import pytest

import synth
from oracle import loc


@pytest.fixture(scope="module")
def lp():
    return synth.loc_config(0)


def test_charges_sum_to_identity(lp):
    P = loc.charges(lp.C, lp.ao_off)
    assert P.shape == (lp.n_atom, lp.n_occ, lp.n_occ)
    assert np.abs(P.sum(0) - np.eye(lp.n_occ)).max() <= 1e-13
    assert np.array_equal(P, np.transpose(P, (0, 2, 1)))


def test_angle_maximizes_pair_functional(lp):
    """For several pairs: the printed angle (two-argument arctangent) beats
    every angle of a 20001-point scan of [-pi/4, pi/4] (the functional has
    period pi/2 in theta), and the one-argument reading loses whenever
    a > 0; the gain equals sqrt(a^2 + b^2)(1 - cos 4 theta)."""
    P0 = loc.charges(lp.C, lp.ao_off)
    n = lp.n_occ
    seen_pos_a = False
    for (i, j) in ((0, 1), (2, 9), (5, 30), (17, 18)):
        a, b = loc.pair_ab(P0, i, j)
        th = 0.25 * math.atan2(b, -a)

        def L_at(t):
            P, U = P0.copy(), np.eye(n)
            loc.rotate(P, U, i, j, math.cos(t), math.sin(t))
            return loc.functional(P)

        L0 = loc.functional(P0)
        scan = np.linspace(-math.pi / 4, math.pi / 4, 20001)
        best = max(L_at(t) for t in scan[::50])  # coarse, then refine around it
        assert L_at(th) >= best - 1e-12
        gain = math.sqrt(a * a + b * b) * (1 - math.cos(4 * th))
        assert abs((L_at(th) - L0) - gain) <= 1e-12 * max(1.0, gain)
        if a > 0:
            seen_pos_a = True
            th1 = 0.25 * math.atan(b / -a)
            assert L_at(th1) < L_at(th) - 1e-12 * max(1.0, gain)
    # the scan covers the period: L(theta + pi/2) = L(theta)
    assert abs(L_at(0.3) - L_at(0.3 + math.pi / 2)) <= 1e-12
    assert seen_pos_a


def test_sweeps_monotone_orthogonal_and_consistent(lp):
    P0 = loc.charges(lp.C, lp.ao_off)
    out = loc.jacobi_pm(P0)
    U, P = out["U"], out["P"]
    assert out["sweeps"] >= 2 and out["dL"][-1] <= loc.L_LOC
    assert np.abs(U.T @ U - np.eye(lp.n_occ)).max() <= 1e-12
    for A in range(lp.n_atom):
        assert np.abs(P[A] - U.T @ P0[A] @ U).max() <= 1e-12
    Ls = [loc.functional(P0)] + out["L"]
    assert all(b >= a - 1e-12 for a, b in zip(Ls, Ls[1:]))
    # the summed increments of a sweep are its gain
    for k in range(out["sweeps"]):
        assert abs((Ls[k + 1] - Ls[k]) - out["dL"][k]) <= 1e-10 * max(1.0, Ls[k + 1])
    # the charges of the localized orbitals equal those of C~ U
    Pc = loc.charges(lp.C @ U, lp.ao_off)
    assert np.abs(Pc - P).max() <= 1e-12


def test_recovers_localized_orbitals(lp):
    """Starting from orbitals mixed over the lattice, the functional ends at
    least as high as that of the localized orbitals the input was mixed from
    (within the convergence threshold)."""
    P0 = loc.charges(lp.C, lp.ao_off)
    out = loc.jacobi_pm(P0)
    L_loc_in = loc.functional(loc.charges(lp.C_loc, lp.ao_off))
    assert loc.functional(P0) < 0.5 * L_loc_in
    assert out["L"][-1] >= L_loc_in - 10 * loc.L_LOC
