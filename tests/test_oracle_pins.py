"""Pins of the oracle's O2-O7 against closed forms, a dense full-space solve,
special cases and invariances (no GPU)."""
import dataclasses

import numpy as np
import pytest

import oracle
import synth
import _pins


def _strong_coupling(p, scale=8.0):
    """Same problem with the off-diagonal occupied Fock scaled up, so that a
    missing or mis-signed coupling term changes energies visibly."""
    f = p.f_occ.copy()
    off = ~np.eye(p.n_occ, dtype=bool)
    f[off] *= scale
    return dataclasses.replace(p, f_occ=f)


def test_kbar_two_routes():
    """O3: 4-block K from projected slabs equals V^T (B_p B_q^T) V."""
    p = synth.config(0)
    ora = oracle.Oracle(p)
    for (a, b) in [(0, 1), (2, 5), (3, 3), (0, 7)]:
        V = p.Q[a] if a == b else np.concatenate([p.Q[a], p.Q[b]], 1)
        ref = V.T @ _pins.full_K([ora.B(i) for i in range(p.n_occ)], a, b) @ V
        got = ora.Kbar(a, b)
        assert np.allclose(got, ref, rtol=0, atol=1e-13 * np.abs(ref).max())


def test_pair_basis_properties():
    """O4: X^T S X = 1 and X^T F X = diag(eps~) for the 4-block S, F."""
    p = synth.config(0)
    ora = oracle.Oracle(p)
    for (a, b) in [(0, 1), (1, 4), (2, 2)]:
        o = oracle.orbs(a, b)
        S, F = ora.Sblk(o, o), ora.Fblk(o, o)
        X, et = ora.basis(a, b)
        assert np.allclose(X.T @ S @ X, np.eye(X.shape[1]), atol=1e-12)
        assert np.allclose(X.T @ F @ X, np.diag(et), atol=1e-12)
        V = p.Q[a] if a == b else np.concatenate([p.Q[a], p.Q[b]], 1)
        assert np.allclose(S, V.T @ V, atol=1e-14)
        assert np.allclose(F, V.T @ np.diag(p.eps_vir) @ V, atol=1e-13)


@pytest.mark.parametrize("n_occ,scale", [(3, 1.0), (3, 8.0), (4, 8.0)])
def test_fragments_match_kronecker_solve(n_occ, scale):
    """O5/O6: every fragment's converged energy equals the dense solution of
    the projected full-space residual equations (Kronecker form)."""
    p = _strong_coupling(synth.micro(n_occ), scale)
    ora = oracle.Oracle(p)
    B = [ora.B(i) for i in range(p.n_occ)]
    for f in p.frags:
        fr = [int(x) for x in f if x >= 0]
        s = ora.solve_fragment(fr, 1e-13, 400)
        assert s["converged"]
        Ek, t = _pins.kron_fragment_solve(B, p.Q, p.eps_vir, p.f_occ, fr)
        assert abs(s["E"] - Ek) <= 1e-12 * abs(Ek)
        assert abs(s["E_lin"] - Ek) <= 1e-10 * abs(Ek)
        # amplitudes, mapped to the full space, agree as well
        for (a, b), Tab in s["T"].items():
            V = p.Q[a] if a == b else np.concatenate([p.Q[a], p.Q[b]], 1)
            assert np.allclose(V @ Tab @ V.T, t[(a, b)], atol=1e-12 * np.abs(t[(a, b)]).max())


@pytest.mark.parametrize("n_occ", [3, 4])
def test_warm_started_fragments_match_kronecker_solve(n_occ):
    """Trimers started from their monomer/dimer solutions converge to the
    same dense solution, in fewer updates than from T = 0."""
    p = dataclasses.replace(_strong_coupling(synth.micro(n_occ), 8.0), tol=1e-13,
                            max_iter=400)
    ora = oracle.Oracle(p)
    cold = oracle.run(p, ora=ora)
    warm = oracle.run(p, ora=ora, warm_start=True)
    B = [ora.B(i) for i in range(p.n_occ)]
    tri = p.frags[:, 2] >= 0
    for k in np.nonzero(tri)[0]:
        fr = [int(x) for x in p.frags[k] if x >= 0]
        Ek, _ = _pins.kron_fragment_solve(B, p.Q, p.eps_vir, p.f_occ, fr)
        assert abs(warm["e_frag"][k] - Ek) <= 1e-12 * abs(Ek)
    assert np.array_equal(warm["e_frag"][~tri], cold["e_frag"][~tri])
    assert warm["iters"][tri].sum() < cold["iters"][tri].sum()


def test_three_orbital_fragment_equals_full_system():
    """A 3-orbital system: MBE(3) telescopes to the trimer, which is the whole
    (unexpanded) OSV-MP2 problem."""
    p = _strong_coupling(synth.micro(3), 8.0)
    out = oracle.run(p)
    E, _ = oracle.mbe3_energy(p.frags, out["e_frag"])
    ora = out["oracle"]
    Ek, _ = _pins.kron_fragment_solve([ora.B(i) for i in range(3)], p.Q,
                                      p.eps_vir, p.f_occ, [0, 1, 2])
    assert abs(E - out["e_frag"][-1]) <= 1e-15
    assert abs(E - Ek) <= 1e-12 * abs(Ek)


def test_canonical_closed_form():
    """Q_i = 1 and diagonal f: MBE(3)-OSV-MP2 is canonical MP2 (eq. mp2_tmat).
    The 4-block pair overlaps are rank deficient here, which exercises the
    canonical orthogonalisation."""
    p = synth.micro(3, identity_q=True, diagonal_f=True)
    ora = oracle.Oracle(p)
    E = oracle.energy(p, ora=ora)
    ref = _pins.canonical_mp2([ora.B(i) for i in range(3)], p.eps_vir,
                              np.diag(p.f_occ))
    assert abs(E - ref) <= 1e-12 * abs(ref)
    X, _ = ora.basis(0, 1)
    assert X.shape == (2 * p.n_vir, p.n_vir)


def test_diagonal_fock_zero_trimer_increment():
    """Diagonal f decouples the pairs: every trimer increment vanishes."""
    p = synth.config(0, diagonal_f=True)
    out = oracle.run(p)
    E, incr = oracle.mbe3_energy(p.frags, out["e_frag"])
    ntri = len(p.trimers)
    assert np.abs(incr[-ntri:]).max() <= 1e-13
    assert np.abs(incr[:-ntri]).max() > 1e-4


def test_mbe_coefficients_identities():
    """sum c_F = n_occ - n_pair + n_tri and sum c_F |F| = n_occ; the c_F form
    equals the increment form."""
    for p in (synth.config(0), synth.config(1)):
        frags = p.frags
        c = oracle.mbe3_coefficients(p.n_occ, frags)
        size = (frags >= 0).sum(1)
        assert c.sum() == p.n_occ - len(p.pairs) + len(p.trimers)
        assert (c * size).sum() == p.n_occ
    p = synth.config(0)
    e = np.random.default_rng(1).standard_normal(p.n_frag)
    E, _ = oracle.mbe3_energy(p.frags, e)
    c = oracle.mbe3_coefficients(p.n_occ, p.frags)
    assert abs(E - np.dot(c, e)) < 1e-12


def test_fragment_energy_sum_matches_amplitude_expansion():
    """The MBE of fragment energies equals the energy of the MBE(3) amplitudes
    built term by term from eqs. tmbediag / tmbeoff / deltaoff."""
    p = _strong_coupling(synth.micro(4), 8.0)
    p = dataclasses.replace(p, tol=1e-13, max_iter=400)
    out = oracle.run(p, keep_T=True)
    E_lin, _ = oracle.mbe3_energy(p.frags, out["e_lin"])
    E_amp = _pins.amplitude_expansion_energy(out["oracle"], p.frags, out["T"])
    assert abs(E_lin - E_amp) <= 1e-13 * abs(E_amp)


def test_osv_rotation_invariance():
    """E depends on span(Q_i) only."""
    p = synth.config(0)
    ora = oracle.Oracle(p)
    out = oracle.run(p, ora=ora)
    E, _ = oracle.mbe3_energy(p.frags, out["e_frag"])
    g = np.random.default_rng(3)
    Q2 = []
    for q in p.Q:
        U, _ = np.linalg.qr(g.standard_normal((q.shape[1], q.shape[1])))
        Q2.append(q @ U)
    p2 = dataclasses.replace(p, Q=Q2, tol=1e-11)
    p1 = dataclasses.replace(p, tol=1e-11)
    E1 = oracle.energy(p1, ora=oracle.Oracle(p1, slabs=ora._slabs))
    E2 = oracle.energy(p2, ora=oracle.Oracle(p2, slabs=ora._slabs))
    assert abs(E1 - E2) <= 1e-12 * abs(E1)
    assert abs(E - E1) <= 1e-9 * abs(E1)


def test_homogeneity():
    """E(lambda B) = lambda^4 E(B);  E(lambda eps, lambda f) = E / lambda."""
    p = dataclasses.replace(synth.config(0), tol=1e-12)
    ora = oracle.Oracle(p)
    E = oracle.energy(p, ora=ora)
    lam = 1.7
    slabs = {i: lam * ora.B(i) for i in range(p.n_occ)}
    E2 = oracle.energy(p, ora=oracle.Oracle(p, slabs=slabs))
    assert abs(E2 - lam ** 4 * E) <= 1e-12 * abs(E2)
    p3 = dataclasses.replace(p, eps_vir=lam * p.eps_vir, f_occ=lam * p.f_occ,
                             tol=1e-12 * lam ** -1)
    E3 = oracle.energy(p3, ora=oracle.Oracle(p3, slabs=ora._slabs))
    assert abs(E3 - E / lam) <= 1e-12 * abs(E)


def test_hylleraas_second_order():
    """The Hylleraas energy of an unconverged iterate errs quadratically in the
    residual while the linear energy errs linearly."""
    p = _strong_coupling(synth.micro(4), 8.0)
    ora = oracle.Oracle(p)
    frag = [0, 1, 2, 3]
    ref = ora.solve_fragment(frag, 1e-14, 400)["E"]
    errs = []
    for n in range(1, 6):
        s = ora.solve_fragment(frag, 0.0, n)
        errs.append((s["res"], abs(s["E"] - ref), abs(s["E_lin"] - ref)))
    for res, eh, el in errs[1:]:
        assert eh < 0.05 * el
        assert eh < 10.0 * res ** 2
