"""Pins of O8 (gradient through Hylleraas stationarity)."""
import dataclasses

import numpy as np
import pytest

import oracle
import synth
import _pins


@pytest.fixture(scope="module")
def grad0():
    p = dataclasses.replace(synth.config(0), tol=1e-13, max_iter=400)
    ora = oracle.Oracle(p)
    g = oracle.gradient(p, ora=ora)
    return p, ora, g


def test_euler_identity(grad0):
    """E is homogeneous of degree 4 in the slabs: sum B . dE/dB = 4 E."""
    p, ora, g = grad0
    s = sum(np.sum(ora.B(i) * g["dB"][i]) for i in range(p.n_occ))
    assert abs(s - 4.0 * g["E"]) <= 1e-12 * abs(g["E"])


def test_fd_fock(grad0):
    """Central differences (h = 1e-5) moving f_xy and f_yx together."""
    p, ora, g = grad0
    h = 1e-5
    for (x, y) in [(0, 1), (2, 5), (3, 3), (0, 7), (6, 7)]:
        E = []
        for s in (+1, -1):
            f = p.f_occ.copy()
            f[x, y] += s * h
            if x != y:
                f[y, x] += s * h
            q = dataclasses.replace(p, f_occ=f)
            E.append(oracle.energy(q, ora=oracle.Oracle(q, slabs=ora._slabs)))
        fd = (E[0] - E[1]) / (2 * h)
        an = g["df"][x, y] * (2.0 if x != y else 1.0)
        assert abs(fd - an) <= 1e-7 * max(abs(an), 1e-3), (x, y, fd, an)


def test_fd_slab_probe(grad0):
    """Central difference of E along the probe direction Delta (Philox key
    word 1 = 10), the direction the library's probe mode regenerates."""
    p, ora, g = grad0
    D = {i: oracle.probe_direction(p, i) for i in range(p.n_occ)}
    h = 1e-5
    E = []
    for s in (+1, -1):
        sl = {i: ora.B(i) + s * h * D[i] for i in range(p.n_occ)}
        E.append(oracle.energy(p, ora=oracle.Oracle(p, slabs=sl)))
    fd = (E[0] - E[1]) / (2 * h)
    an = sum(np.sum(g["dB"][i] * D[i]) for i in range(p.n_occ))
    assert abs(fd - an) <= 1e-7 * abs(an)


def test_probe_direction_stream():
    """Delta is the slab's generator under key word 1 = 10: the C and numpy
    routes agree to 4 ulp; its normals have mean 0 and variance 1 and are
    uncorrelated with the slab's (independent Philox streams), within four
    standard errors over the 8-LMO chain's 1.2e6 elements."""
    p = synth.config(0)
    zs, zd = [], []
    for i in range(p.n_occ):
        w = p.w_ia[i][:, None] * p.w_iP[i][None, :]
        d = oracle.probe_direction(p, i)
        dn = oracle.probe_direction(p, i, cols=np.arange(0, p.n_aux, 7), impl="numpy")
        ref = d[:, ::7]
        assert np.all(np.abs(dn - ref) <= 4 * np.spacing(np.abs(ref)))
        zd.append((d / w).ravel())
        zs.append((oracle.slab(p, i) / w).ravel())
    zd, zs = np.concatenate(zd), np.concatenate(zs)
    se = 1.0 / np.sqrt(zd.size)
    assert abs(zd.mean()) <= 4 * se
    assert abs(zd.var() - 1.0) <= 4 * np.sqrt(2.0) * se
    assert abs(np.mean(zd * zs)) <= 4 * se
    assert not np.array_equal(zd, zs)


def test_canonical_gradient_closed_form():
    """Q_i = 1, diagonal f: dE/dB_i = 4 sum_j (2 t_ij - t_ij^T) B_j with the
    canonical amplitudes t_ij = K_ij / (f_ii + f_jj - e_a - e_b)."""
    p = synth.micro(3, identity_q=True, diagonal_f=True)
    ora = oracle.Oracle(p)
    g = oracle.gradient(p, ora=ora)
    B = [ora.B(i) for i in range(3)]
    fd = np.diag(p.f_occ)
    for i in range(3):
        ref = np.zeros_like(B[i])
        for j in range(3):
            D = fd[i] + fd[j] - p.eps_vir[:, None] - p.eps_vir[None, :]
            t = _pins.full_K(B, i, j) / D
            ref += 4.0 * (2.0 * t - t.T) @ B[j]
        assert np.allclose(g["dB"][i], ref, rtol=0, atol=1e-12 * np.abs(ref).max())
