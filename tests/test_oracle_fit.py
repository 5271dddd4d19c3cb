"""Pins of the oracle's sparse fitting domains (oracle/fit.py) against what
the mathematics fixes: the metric of a rank-one slab in closed form, its
invariance under rotations of the orbital index (and not of the auxiliary
one), its expectation for the seeded Gaussian slabs, the restricted pair
integrals against an explicit sum over the union of two domains (the
printed D_i u D_j, which neither domain alone nor their intersection
gives), the stored Gamma~ blocks' column sets, the limits l_fit below every
metric (the unrestricted method, bit for bit) and above every metric (no
integrals, zero energy), and a restricted trimer against the Kronecker
dense solve fed the union-restricted full-space integrals."""
import numpy as np
import pytest

import _pins
import oracle
import synth
from oracle import fit


def test_metric_rank_one_closed_form():
    """B_i = u v^T: s_fit[A] = v_A^2 |u|^2."""
    p = synth.micro(3)
    rng = np.random.default_rng(11)
    slabs, expect = {}, {}
    for i in range(p.n_occ):
        u = rng.standard_normal(p.n_vir)
        v = rng.standard_normal(p.n_aux)
        slabs[i] = np.outer(u, v)
        expect[i] = v * v * float(u @ u)
    ora = oracle.Oracle(p, slabs=slabs)
    for i in range(p.n_occ):
        assert np.allclose(fit.fit_metric(ora, i), expect[i], rtol=1e-14, atol=0)


def test_metric_rotation_of_orbital_index_only():
    """Rotating the orbital index of a slab keeps every column norm; rotating
    the auxiliary index does not (the sum runs over the right index)."""
    p = synth.micro(3)
    base = oracle.Oracle(p)
    rng = np.random.default_rng(12)
    U, _ = np.linalg.qr(rng.standard_normal((p.n_vir, p.n_vir)))
    V, _ = np.linalg.qr(rng.standard_normal((p.n_aux, p.n_aux)))
    rot_a = oracle.Oracle(p, slabs={i: U @ base.B(i) for i in range(p.n_occ)})
    rot_P = oracle.Oracle(p, slabs={i: base.B(i) @ V for i in range(p.n_occ)})
    for i in range(p.n_occ):
        s = fit.fit_metric(base, i)
        assert np.allclose(fit.fit_metric(rot_a, i), s, rtol=1e-12, atol=0)
        assert not np.allclose(fit.fit_metric(rot_P, i), s, rtol=1e-3, atol=0)


def test_metric_expectation_of_seeded_slabs():
    """B_i[a,P] = z w_ia w_iP with z standard normal: E s_fit[i,P] =
    w_iP^2 sum_a w_ia^2.  The ratio averaged over the 1536 (i, P) of the
    8-LMO chain is 1 within four standard errors (each ratio has variance
    at most 2)."""
    p = synth.config(0)
    ora = oracle.Oracle(p)
    s = fit.fit_metrics(ora)
    expect = (p.w_iP ** 2) * np.sum(p.w_ia ** 2, axis=1)[:, None]
    ratio = s / expect
    assert abs(ratio.mean() - 1.0) <= 4.0 * np.sqrt(2.0 / ratio.size)


def partial_threshold(s):
    """A threshold that splits every LMO's auxiliary set."""
    return float(np.median(s))


def domains(s, l_fit, n):
    return [set(np.nonzero(fit.domain(s[i], l_fit))[0].tolist()) for i in range(n)]


def test_restricted_K_is_the_union_sum():
    """K_(pq) of the restricted oracle against an explicit loop over the
    auxiliary functions in D_p or D_q, with the unrestricted projections
    (eqs. osv_imua, osv_close_k: A' in D_p u D_q); the diagonal slot over
    D_p.  The threshold splits every domain, so the union differs from
    each domain and from the intersection."""
    p = synth.micro(3)
    base = oracle.Oracle(p)
    s = fit.fit_metrics(base)
    l_fit = partial_threshold(s)
    D = domains(s, l_fit, p.n_occ)
    assert all(0 < len(d) < p.n_aux for d in D)
    ora = fit.restricted_oracle(p, l_fit, base=base)
    for a in range(p.n_occ):
        for b in range(a, p.n_occ):
            union = sorted(D[a] | D[b])
            if a != b:
                assert len(union) > max(len(D[a]), len(D[b]))
                assert len(D[a] & D[b]) < len(union)
            o = oracle.orbs(a, b)
            L = np.concatenate([base.gamma(a, x) for x in o], 0)
            R = np.concatenate([base.gamma(b, x) for x in o], 0)
            K = np.zeros((L.shape[0], R.shape[0]))
            for A in union:
                K += np.outer(L[:, A], R[:, A])
            got = ora.Kbar(a, b)
            assert np.allclose(got, K, rtol=0, atol=1e-14 * np.abs(K).max())
            if a != b:
                # the one-block weak integral over the same union
                Kw = np.zeros((p.r[a], p.r[b]))
                for A in union:
                    Kw += np.outer(base.gamma(a, a)[:, A], base.gamma(b, b)[:, A])
                assert np.allclose(ora.weak_K(a, b), Kw, rtol=0,
                                   atol=1e-14 * np.abs(Kw).max())


def test_stored_gamma_blocks_column_sets():
    """eq. osv_imua stored over the domains: block (i, x), x != i, on
    D_i u D_x; the diagonal block on the union of D_q over q in N+(i)
    (every pair (i, q) reads it over D_i u D_q); values equal to the
    unrestricted projection there."""
    p = synth.micro(4)
    base = oracle.Oracle(p)
    s = fit.fit_metrics(base)
    l_fit = partial_threshold(s)
    D = domains(s, l_fit, p.n_occ)
    ora = fit.restricted_oracle(p, l_fit, base=base)
    for i in range(p.n_occ):
        for x in p.neighbours(i):
            x = int(x)
            want = D[i] | D[x] if x != i else set().union(*[D[int(q)] for q in p.neighbours(i)])
            g = ora.gamma_fit(i, x)
            cols = set(np.nonzero(np.any(g != 0.0, axis=0))[0].tolist())
            assert cols == want, (i, x)
            idx = sorted(want)
            assert np.array_equal(g[:, idx], base.gamma(i, x)[:, idx])


def test_thresholds_at_the_limits():
    p = synth.micro(3)
    base = oracle.Oracle(p)
    s = fit.fit_metrics(base)
    assert s.min() > 0.0
    every = fit.restricted_oracle(p, 0.0, base=base)
    none = fit.restricted_oracle(p, float(s.max()), base=base)
    for a in range(p.n_occ):
        for b in range(a, p.n_occ):
            assert np.array_equal(every.Kbar(a, b), base.Kbar(a, b))
            assert not np.any(none.Kbar(a, b))
    assert oracle.energy(p, ora=none) == 0.0


def test_restricted_fragment_matches_kronecker_solve():
    """The restricted trimer of a 3-orbital chain against the dense
    full-space solve fed K_pq = B_p[:, U] B_q[:, U]^T with U = D_p u D_q
    (D_p for p = q), written from the slabs (no oracle pair blocks)."""
    p = synth.micro(3)
    base = oracle.Oracle(p)
    s = fit.fit_metrics(base)
    l_fit = partial_threshold(s)
    ora = fit.restricted_oracle(p, l_fit, base=base)
    st = ora.solve_fragment([0, 1, 2], 1e-13, 400)
    assert st["converged"]
    mask = fit.domain(s, l_fit)
    B = [base.B(i) for i in range(p.n_occ)]

    def K_union(a, b):
        U = mask[a] | mask[b]
        return B[a][:, U] @ B[b][:, U].T

    Ek, _ = _pins.kron_fragment_solve(B, p.Q, p.eps_vir, p.f_occ, [0, 1, 2], Kfun=K_union)
    assert abs(st["E"] - Ek) <= 1e-12 * abs(Ek)
    # and the restriction changes the energy
    full = base.solve_fragment([0, 1, 2], 1e-13, 400)
    assert abs(full["E"] - st["E"]) > 1e-6 * abs(full["E"])


def test_lazy_restricted_oracle_matches_eager():
    """A RestrictedOracle computing each metric on first use gives bit for
    bit the metrics and pair integrals of one given every metric up front."""
    p = synth.micro(4)
    base = oracle.Oracle(p)
    s = fit.fit_metrics(base)
    l_fit = partial_threshold(s)
    eager = fit.restricted_oracle(p, l_fit, base=base, s_fit=s)
    lazy = fit.RestrictedOracle(p, l_fit)
    for a in range(p.n_occ):
        for b in range(a, p.n_occ):
            assert np.array_equal(lazy.Kbar(a, b), eager.Kbar(a, b))
    for i in range(p.n_occ):
        assert np.array_equal(lazy.s[i], s[i])
