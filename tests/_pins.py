"""Independent routes used to pin the oracle (test helpers).

Nothing here reuses the oracle's pair-block assembly: the Kronecker solve
works with full virtual-space amplitudes t_pq = V T V^T and the full-space
residual, and the closed forms are written from eq. mp2_tmat.
"""
import numpy as np


def full_K(B, p, q):
    """K_pq[a,b] = sum_P (pa|P)(qb|P) in the full virtual space."""
    return B[p] @ B[q].T


def _V(Q, p, q):
    return Q[p] if p == q else np.concatenate([Q[p], Q[q]], 1)


def _commutation(n):
    """P with vec(X^T) = P vec(X) for n x n X (row-major vec)."""
    P = np.zeros((n * n, n * n))
    for i in range(n):
        for j in range(n):
            P[j * n + i, i * n + j] = 1.0
    return P


def kron_fragment_solve(B, Q, eps, f, frag, Kfun=None):
    """Solve the projected full-space residual equations of one fragment.

    Unknowns: T_s for every p <= q in the fragment, t_pq = V T V^T.
    Equations: V_pq^T r_pq V_pq = 0 with
      r_pq = K_pq + eps t_pq + t_pq eps - sum_k (f_pk t_kq + f_kq t_pk),
    k over the fragment, written with Kronecker products and solved densely.
    Returns (E, t) with E = sum_{ordered p,q} <K_pq, 2 t_pq - t_pq^T> and the
    full-space amplitudes t[(p, q)] for all ordered pairs.  Kfun(p, q)
    (optional) supplies the full-space K_pq in place of B_p B_q^T.
    """
    if Kfun is None:
        Kfun = lambda p, q: full_K(B, p, q)
    frag = sorted(frag)
    n = len(eps)
    I = np.eye(n)
    E_op = np.diag(eps)
    Pn = _commutation(n)
    plist = [(p, q) for a, p in enumerate(frag) for q in frag[a:]]
    V = {t: _V(Q, *t) for t in plist}
    dims = {t: V[t].shape[1] for t in plist}
    offs, o = {}, 0
    for t in plist:
        offs[t] = o
        o += dims[t] ** 2
    nunk = o

    def lift(x, y):
        """Matrix mapping the unknown vector to vec(t_xy) (full space)."""
        s = (min(x, y), max(x, y))
        M = np.zeros((n * n, nunk))
        block = np.kron(V[s], V[s])
        if x > y:
            block = Pn @ block
        M[:, offs[s]:offs[s] + dims[s] ** 2] = block
        return M

    A = np.zeros((nunk, nunk))
    rhs = np.zeros(nunk)
    for t in plist:
        p, q = t
        Lin = (np.kron(E_op, I) + np.kron(I, E_op)) @ lift(p, q)
        for k in frag:
            Lin -= f[p, k] * lift(k, q) + f[k, q] * lift(p, k)
        proj = np.kron(V[t].T, V[t].T)
        sl = slice(offs[t], offs[t] + dims[t] ** 2)
        A[sl] = proj @ Lin
        rhs[sl] = -(proj @ Kfun(p, q).ravel())
    x = np.linalg.solve(A, rhs)
    t_full = {}
    for x_ in frag:
        for y_ in frag:
            t_full[(x_, y_)] = (lift(x_, y_) @ x).reshape(n, n)
    E = 0.0
    for (x_, y_), t in t_full.items():
        E += np.sum(Kfun(x_, y_) * (2.0 * t - t.T))
    return E, t_full


def canonical_mp2(B, eps, f_diag, pairs_all=True):
    """Closed-form canonical MP2 (eq. mp2_tmat) with a diagonal occupied Fock.

    E = sum_{i,j} sum_{ab} K_ij^ab (2 K_ij^ab - K_ij^ba) / (f_ii + f_jj - e_a - e_b)
    """
    n_occ = len(f_diag)
    E = 0.0
    for i in range(n_occ):
        for j in range(n_occ):
            K = full_K(B, i, j)
            D = f_diag[i] + f_diag[j] - eps[:, None] - eps[None, :]
            E += np.sum(K * (2.0 * K - K.T) / D)
    return E


def amplitude_expansion_energy(ora, frags, T_list):
    """Energy of the MBE(3) amplitudes built literally from eqs. tmbediag,
    tmbeoff and deltaoff, with E = sum <K, 2T - T^T> (diag once, pairs twice).
    """
    Tf = {}
    for f, T in zip(frags, T_list):
        Tf[tuple(int(x) for x in f if x >= 0)] = T
    singles = sorted(o[0] for o in Tf if len(o) == 1)
    pairs = sorted(o for o in Tf if len(o) == 2)
    tris = sorted(o for o in Tf if len(o) == 3)
    E = 0.0
    for i in singles:
        Ti = Tf[(i,)][(i, i)]
        acc = Ti.copy()
        dT2 = {}
        for (a, b) in pairs:
            if i in (a, b):
                k = b if a == i else a
                dT2[k] = Tf[(a, b)][(i, i)] - Ti
                acc += dT2[k]
        for o in tris:
            if i in o:
                k, l = [x for x in o if x != i]
                acc += Tf[o][(i, i)] - dT2[k] - dT2[l] - Ti
        E += np.sum(ora.Kbar(i, i) * (2.0 * acc - acc.T))
    for (a, b) in pairs:
        Tab = Tf[(a, b)][(a, b)]
        acc = Tab.copy()
        for o in tris:
            if a in o and b in o:
                acc += Tf[o][(a, b)] - Tab
        E += 2.0 * np.sum(ora.Kbar(a, b) * (2.0 * acc - acc.T))
    return E
