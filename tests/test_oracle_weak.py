"""Pins of the oracle's screening metrics and weak-pair path (oracle/weak.py)
against what the mathematics fixes: exact values of s2b for equal and
orthogonal OSV spaces and its invariance under OSV rotations, the class and
trimer thresholds, the direct part of the canonical MP2 pair energy for
identity OSVs and a diagonal occupied Fock, the vanishing one-block residual,
and the diagonal amplitudes against the gradient's multipliers."""
import dataclasses
import types

import numpy as np
import pytest

import _pins
import oracle
import synth
from oracle import weak

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")


def osv_pair(n_vir, ri, rj, seed, overlap="random"):
    rng = np.random.default_rng(seed)
    if overlap == "orthogonal":
        q, _ = np.linalg.qr(rng.standard_normal((n_vir, ri + rj)))
        return q[:, :ri], q[:, ri:]
    qi, _ = np.linalg.qr(rng.standard_normal((n_vir, ri)))
    if overlap == "equal":
        u, _ = np.linalg.qr(rng.standard_normal((ri, ri)))
        return qi, qi @ u
    qj, _ = np.linalg.qr(rng.standard_normal((n_vir, rj)))
    return qi, qj


def ns(qi, qj):
    return types.SimpleNamespace(Q=[qi, qj], r=[qi.shape[1], qj.shape[1]])


def test_s2b_equal_orthogonal_rotation():
    qi, qj = osv_pair(40, 7, 7, 1, "equal")
    assert abs(weak.s2b(ns(qi, qj), 0, 1) - 1.0) <= 1e-13
    qi, qj = osv_pair(40, 6, 9, 2, "orthogonal")
    assert weak.s2b(ns(qi, qj), 0, 1) <= 1e-28
    qi, qj = osv_pair(40, 6, 9, 3)
    v = weak.s2b(ns(qi, qj), 0, 1)
    rng = np.random.default_rng(4)
    u, _ = np.linalg.qr(rng.standard_normal((6, 6)))
    w, _ = np.linalg.qr(rng.standard_normal((9, 9)))
    assert abs(weak.s2b(ns(qi @ u, qj @ w), 0, 1) - v) <= 1e-14
    # at most min(r_i, r_j) / sqrt(r_i r_j): the cosines of principal angles are <= 1
    assert 0.0 < v <= 6 / np.sqrt(54) + 1e-15


def test_classes_and_trimer_screen():
    assert weak.pair_class(0.0) == "distant"
    assert weak.pair_class(9.99e-8) == "distant"
    assert weak.pair_class(1e-7) == "weak"
    assert weak.pair_class(9.99e-3) == "weak"
    assert weak.pair_class(1e-2) == "close"
    assert weak.s3b(0.3, 0.2, 0.1) == pytest.approx(0.2)
    assert weak.keep_trimer(0.3, 0.2, 0.1 + 1e-12)
    assert not weak.keep_trimer(0.3, 0.2, 0.1 - 1e-9)


def test_weak_energy_canonical_direct_mp2():
    """Q_i = I and a diagonal occupied Fock: the weak amplitude is
    K_ab / (f_ii + f_jj - e_a - e_b) and the pair energy the direct part of
    the canonical MP2 energy of the ordered pairs ij and ji,
    2 sum_ab K_ab (2 K_ab) / D_ab."""
    prob = synth.micro(3, identity_q=True, diagonal_f=True)
    ora = oracle.Oracle(prob)
    B = [ora.B(i) for i in range(prob.n_occ)]
    fd = np.diag(prob.f_occ)
    zero = np.zeros((prob.n_vir, prob.n_vir))
    for i, j in ((0, 1), (0, 2), (1, 2)):
        K = _pins.full_K(B, i, j)
        D = fd[i] + fd[j] - prob.eps_vir[:, None] - prob.eps_vir[None, :]
        closed = 2.0 * np.sum(K * (2.0 * K) / D)
        T, e, _ = weak.weak_pair(ora, i, j, zero, zero)
        assert abs(e - closed) <= 1e-12 * abs(closed)
        assert np.allclose(T, K / D, rtol=0, atol=1e-12 * np.abs(K / D).max())


def test_weak_residual_vanishes():
    """General OSVs and occupied Fock: the amplitudes solve the one-block
    equation (reading W1), for any diagonal-pair amplitudes given."""
    prob = synth.micro(4)
    ora = oracle.Oracle(prob)
    rng = np.random.default_rng(5)
    Td = {}
    for i in range(prob.n_occ):
        a = rng.standard_normal((prob.r[i], prob.r[i])) * 1e-2
        Td[i] = a + a.T
    for i in range(prob.n_occ):
        for j in range(i + 1, prob.n_occ):
            T, e, K = weak.weak_pair(ora, i, j, Td[i], Td[j])
            R = weak.weak_residual(ora, i, j, T, Td[i], Td[j])
            assert np.abs(R).max() <= 1e-12 * np.abs(K).max()
            assert e == pytest.approx(4.0 * np.sum(K * T), rel=1e-14)


def test_diagonal_amplitudes_match_multipliers():
    """T^MBE_ii (eq. tmbediag) against the diagonal blocks of the gradient's
    multipliers W_pp = sum_F c_F (2 T^F_pp - T^F_pp^T), which equal it for
    the symmetric diagonal amplitudes."""
    prob = dataclasses.replace(synth.micro(4), tol=1e-12, max_iter=300)
    g = oracle.gradient(prob)
    Td = weak.mbe3_diagonal_amplitudes(prob)
    for i in range(prob.n_occ):
        W = g["W"][(i, i)]
        assert np.abs(Td[i] - W).max() <= 1e-10 * np.abs(W).max()


def test_weak_residual_is_close_pair_block():
    """Reading W1 pinned by another route: the close-pair residual of eq.
    res_close (Oracle.residual, the dimer ij as the fragment) with every
    block of T_ij zeroed except the direct (mu_i, nu_j) one, tau, and the
    diagonal-pair amplitudes T_ii, T_jj set, has as its (mu_i, nu_j) block
    the one-block residual at tau: K_(i,j) + F_ii tau + tau F_jj
    - (f_ii + f_jj) tau - f_ij (T_ii S_ij + S_ij T_jj).  Checked at random
    tau (so every term counts) and at the weak-pair solution (block zero);
    f is made strongly non-diagonal so that the coupling term matters."""
    prob = synth.micro(4)
    f = prob.f_occ.copy()
    off = ~np.eye(prob.n_occ, dtype=bool)
    f[off] *= 8.0
    prob = dataclasses.replace(prob, f_occ=f)
    ora = oracle.Oracle(prob)
    rng = np.random.default_rng(11)
    Td = {}
    for i in range(prob.n_occ):
        a = rng.standard_normal((prob.r[i], prob.r[i])) * 1e-2
        Td[i] = a + a.T
    for i, j in ((0, 1), (0, 3), (1, 2)):
        ri, rj = prob.r[i], prob.r[j]
        T_sol, _, K = weak.weak_pair(ora, i, j, Td[i], Td[j])
        coupling = np.abs(f[i, j] * (Td[i] @ ora.S(i, j) + ora.S(i, j) @ Td[j])).max()
        assert coupling > 1e-3 * np.abs(K).max()  # the term is not negligible
        for tau in (rng.standard_normal((ri, rj)) * 1e-2, T_sol):
            Tij = np.zeros((ri + rj, ri + rj))
            Tij[:ri, ri:] = tau
            T = {(i, i): Td[i], (j, j): Td[j], (i, j): Tij}
            R = ora.residual(i, j, (i, j), T)
            block = R[:ri, ri:]
            ref = weak.weak_residual(ora, i, j, tau, Td[i], Td[j])
            assert np.abs(block - ref).max() <= 1e-13 * np.abs(K).max()
        # at the solution the block vanishes
        assert np.abs(block).max() <= 1e-12 * np.abs(K).max()
