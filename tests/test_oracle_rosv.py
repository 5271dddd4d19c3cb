"""Pins of the randomized OSV oracle (oracle/rosv.py) against what the
mathematics fixes: the semicanonical amplitudes in closed form for a
rank-one slab and their symmetry and positive semidefiniteness (a Schur
product of Gram and Cauchy matrices), the counter layout of the Gaussian
rows, an exactly low-rank matrix (the range finder stops after its rank
and the SVD returns its spectrum and range), and, on a helix of LMOs, the
randomized OSVs against the exact eigendecomposition of T_ii (eq. osv_gen)
within the range finder's guarantee: ||(1 - Z^T Z) T|| <= l_osv, each
singular value within l_osv below its eigenvalue, each exact OSV with
eigenvalue lambda >= 10 l_osv inside the range up to l_osv / lambda."""
import math

import numpy as np
import pytest

import oracle
import synth
from oracle import rosv as R

HELIX64 = dict(name="helix64", geometry="helix", n_occ=64, n_vir=256, n_aux=768,
               r=(24, 80), cutoff=6.0, tol=1e-7)


@pytest.fixture(scope="module")
def helix():
    return synth.build(HELIX64, 12345)


def test_semicanonical_T_rank_one_closed_form():
    rng = np.random.default_rng(1)
    n, m = 30, 50
    u, v = rng.standard_normal(n), rng.standard_normal(m)
    eps = np.sort(rng.uniform(0.2, 4.0, n))
    f = -0.7
    keep = rng.random(m) < 0.5
    T = R.semicanonical_T(np.outer(u, v), eps, f, keep)
    closed = np.outer(u, u) * float(v[keep] @ v[keep]) / (eps[:, None] + eps[None, :] - 2 * f)
    assert np.allclose(T, closed, rtol=1e-13, atol=0)


def test_semicanonical_T_symmetric_psd(helix):
    B = oracle.slab(helix, 5)
    T = R.semicanonical_T(B, helix.eps_vir, helix.f_occ[5, 5])
    assert np.array_equal(T, T.T)
    lam = np.linalg.eigvalsh(T)
    assert lam.min() >= -1e-14 * lam.max()


def test_gaussian_rows_counter_layout():
    """Row s, column a of LMO i is the Box-Muller normal of the Philox block
    at counter (a, s, i, 0) under key (seed, 11); the C and numpy routines
    agree within 4 ulp."""
    seed, i = 2603165754, 17
    G = R.gaussian_rows(seed, i, 12, 40)
    Gn = R.gaussian_rows(seed, i, 12, 40, impl="numpy")
    assert np.max(np.abs(G - Gn) / np.spacing(np.abs(Gn))) <= 4
    s, a = 7, 33
    w = oracle.philox4x64_10(np.array([[a, s, i, 0]], dtype=np.uint64), (seed, 11))
    assert Gn[s, a] == oracle.box_muller(w[:, 0], w[:, 1])[0]


def test_exact_low_rank():
    """T = U diag(sigma) U^T of rank 12: the range finder accepts exactly 12
    rows, the singular values are sigma and the OSVs span U."""
    rng = np.random.default_rng(7)
    n, k = 200, 12
    U, _ = np.linalg.qr(rng.standard_normal((n, k)))
    sig = np.geomspace(1.0, 2e-4, k)
    T = (U * sig) @ U.T
    G = rng.standard_normal((R.R_BLOCK + 60, n))
    out = R.rosv(T, G, l_osv=1e-4)
    assert out["rows"] == k and not out["capped"]
    assert np.allclose(out["w"], sig, rtol=1e-12, atol=0)
    P = out["Q"] @ out["Q"].T
    assert np.abs(P - U @ U.T).max() <= 1e-12
    assert np.abs(out["Q"].T @ out["Q"] - np.eye(k)).max() <= 1e-13
    # a smaller threshold drops nothing more; a larger one cuts the spectrum
    out2 = R.rosv(T, G, l_osv=1e-2)
    assert len(out2["w"]) == int((sig >= 1e-2).sum())


@pytest.mark.parametrize("i", [0, 31, 63])
def test_helix_against_exact_osvs(helix, i):
    out = R.lmo_rosv(helix, i, l_fit=1e-6, n_max=128)
    T = out["T"]
    Z, w = out["Z"], out["w"]
    l_osv = R.L_OSV
    assert not out["capped"]
    assert np.abs(Z @ Z.T - np.eye(out["rows"])).max() <= 1e-13
    lam_all = np.sort(np.linalg.eigvalsh(T))[::-1]
    # the range finder's guarantee, and the a posteriori residual
    resid = np.linalg.norm(T - Z.T @ (Z @ T), 2)
    assert resid <= l_osv
    k = len(w)
    # singular values of Z T = those of the projected T: within resid below
    assert np.all(w <= lam_all[:k] * (1 + 1e-12)) and np.all(lam_all[:k] - w <= resid * (1 + 1e-9))
    # hence the counts agree unless an eigenvalue lies in [l_osv, l_osv + resid)
    if not np.any((lam_all >= l_osv) & (lam_all < l_osv + resid)):
        assert k == int((lam_all >= l_osv).sum())
    U, lam = R.exact_osv(T)
    for j in range(len(lam)):
        if lam[j] >= 10 * l_osv:
            u = U[:, j]
            assert np.linalg.norm(u - Z.T @ (Z @ u)) <= resid / lam[j] * (1 + 1e-9)
    # the stopping rule: every pending row at the stop is below the test
    assert out["pending_max"] <= out["threshold"]
    assert out["threshold"] == l_osv / (10 * math.sqrt(2 / math.pi))
