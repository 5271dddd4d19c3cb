"""Plain FP64 CPU oracle of the MBE(3)-OSV-MP2 hot path.

TEST INFRASTRUCTURE ONLY: nothing in the product path may import this module.
It is deliberately slow and direct: each function restates one equation or
one step of an algorithm of the paper (Liang & Yang, "Multi-GPU
MBE(3)-OSV-MP2 for Performant Large-Scale ab initio Calculations",
arXiv:2603.16575), with library matmul / eigh as its only primitives.

Notation (paper section "MBE(3)-OSV-MP2 Method"):
  B_i[a,P] = (ia|P)           fitted RI slab of LMO i (stands in for the
                              fitted Gamma_i of eq. fitting; MO index a in
                              place of the AO index)
  Q_i                         OSVs of LMO i, Q_i^T Q_i = 1
  V_pq = [Q_p Q_q], V_pp = Q_p  pair domain (eq. 4block_osv; diagonal pairs
                              use the single block)
  S_(A,B) = V_A^T V_B, F_(A,B) = V_A^T diag(eps) V_B
  T_pq                        amplitudes in the V_pq basis, T_qp obtained by
                              the block swap of T_pq^T
Readings of points the paper leaves open are listed in the repository's
design notes and restated at each function below.
"""
from __future__ import annotations

import math
import os
from collections import OrderedDict
from typing import Dict, Iterable, Optional, Sequence, Tuple

import numpy as np

from .philox import box_muller, philox4x64_10

STREAM_SLAB = 0
STREAM_PROBE = 10


# --------------------------------------------------------------------------
# O1: regenerated slab (stand-in for the direct Gamma_i generator, Alg. 1)
# --------------------------------------------------------------------------
def slab(prob, i: int, cols=None, impl: str = "c") -> np.ndarray:
    """B_i[a,P] = z(seed,i,a,P) * w_ia[i,a] * w_iP[i,P] (in that order).

    z is the Box-Muller normal of words 0 and 1 of the Philox4x64-10 block at
    counter (P, a, i, 0) under key (seed, 0).  The product is evaluated left to
    right.  Plays the role of the fitted Gamma_i of eq. fitting.  ``cols``
    (optional) restricts P to a list of auxiliary indices.

    impl "c": the same definition in the oracle's own C routine
    (oracle/csrc/slab.c, libm log and cos), fast enough for slabs of tens of
    millions of elements; "numpy": vectorised numpy (its own log and cos).
    The two agree bit for bit on the Philox words and to 4 ulp on the slab
    (pinned in the test-suite).
    """
    return _weighted_normals(prob, i, STREAM_SLAB, cols, impl)


def probe_direction(prob, i: int, cols=None, impl: str = "c") -> np.ndarray:
    """Delta_i[a,P] = z'(seed,i,a,P) * w_ia[i,a] * w_iP[i,P]: the direction
    along which the gradient is probed, the slab's own definition with key
    (seed, 10) in place of (seed, 0), so that it has the slab's scale and
    its normals are independent of the slab's."""
    return _weighted_normals(prob, i, STREAM_PROBE, cols, impl)


def _weighted_normals(prob, i, stream, cols, impl):
    nv = prob.n_vir
    P = np.arange(prob.n_aux) if cols is None else np.asarray(cols)
    if impl == "c":
        from . import _clib
        return _clib.normal_slab((prob.seed, stream), i, nv, P,
                                 prob.w_ia[i], prob.w_iP[i])
    ctr = np.zeros((nv, len(P), 4), dtype=np.uint64)
    ctr[..., 0] = P.astype(np.uint64)[None, :]
    ctr[..., 1] = np.arange(nv, dtype=np.uint64)[:, None]
    ctr[..., 2] = np.uint64(i)
    w = philox4x64_10(ctr, (prob.seed, stream))
    z = box_muller(w[..., 0], w[..., 1])
    return (z * prob.w_ia[i][:, None]) * prob.w_iP[i][P][None, :]


def orbs(p: int, q: int) -> Tuple[int, ...]:
    """Orbitals spanning the pair domain of the ordered pair (p, q)."""
    return (p,) if p == q else (p, q)


def swap_blocks(M: np.ndarray, ra: int, rb: int) -> np.ndarray:
    """Given M in the [Q_a Q_b] basis, return M^T expressed in [Q_b Q_a].

    This is how an amplitude (or multiplier) of the ordered pair (b, a) is
    obtained from that of (a, b): t_ba = t_ab^T in the full virtual space.
    """
    pos = np.concatenate([np.arange(ra) + rb, np.arange(rb)])
    out = np.empty_like(M)
    out[np.ix_(pos, pos)] = M.T
    return out


class _Bounded(OrderedDict):
    """A dict that forgets its least recently used entries beyond ``cap``
    (None: unbounded).  Only memory changes: a forgotten value is computed
    again, by the same arithmetic, when asked for."""

    def __init__(self, cap=None, init=None):
        super().__init__(init or {})
        self.cap = cap

    def __getitem__(self, k):
        v = super().__getitem__(k)
        self.move_to_end(k)
        return v

    def __setitem__(self, k, v):
        super().__setitem__(k, v)
        self.move_to_end(k)
        if self.cap is not None:
            while len(self) > self.cap:
                super().__delitem__(next(iter(self)))


class Oracle:
    """All intermediates of the hot path for one Problem.

    ``slabs``: optional explicit {i: B_i} replacing the regenerated slabs
    (used for derivative checks along a perturbed slab).  ``max_slabs`` /
    ``max_gammas`` (optional) bound how many regenerated slabs and projected
    blocks stay cached (for workloads whose slabs do not fit in host
    memory); explicit slabs are always kept.
    """

    def __init__(self, prob, slabs: Optional[Dict[int, np.ndarray]] = None,
                 max_slabs: Optional[int] = None, max_gammas: Optional[int] = None):
        self.prob = prob
        self.f = np.asarray(prob.f_occ, dtype=np.float64)
        self.eps = np.asarray(prob.eps_vir, dtype=np.float64)
        self.Q = prob.Q
        self.r = [int(x) for x in prob.r]
        if slabs is not None:
            self._slabs = dict(slabs)
        else:
            self._slabs = _Bounded(max_slabs)
        self._gamma = _Bounded(max_gammas)
        self._S: Dict[Tuple[int, int], np.ndarray] = {}
        self._F: Dict[Tuple[int, int], np.ndarray] = {}
        self._K: Dict[Tuple[int, int], np.ndarray] = {}
        self._basis: Dict[Tuple[int, int], tuple] = {}

    # ---- O1 / O2 ---------------------------------------------------------
    def B(self, i: int) -> np.ndarray:
        if i not in self._slabs:
            self._slabs[i] = slab(self.prob, i)
        return self._slabs[i]

    def gamma(self, i: int, x: int) -> np.ndarray:
        """O2, eq. osv_imua: Gamma~_{i,x} = Q_x^T B_i  ([r_x, n_aux])."""
        key = (i, x)
        if key not in self._gamma:
            self._gamma[key] = self.Q[x].T @ self.B(i)
        return self._gamma[key]

    def project_all(self, i: int, nbrs: Sequence[int]) -> np.ndarray:
        """Gamma~ rows of LMO i for every x in N+(i), stacked in order."""
        return np.concatenate([self.gamma(i, int(x)) for x in nbrs], 0)

    # ---- Alg. 5: OSV overlap and Fock blocks ------------------------------
    def S(self, x: int, y: int) -> np.ndarray:
        """S_(x,y) = Q_x^T Q_y."""
        if (x, y) not in self._S:
            self._S[(x, y)] = self.Q[x].T @ self.Q[y]
        return self._S[(x, y)]

    def F(self, x: int, y: int) -> np.ndarray:
        """F_(x,y) = Q_x^T diag(f_aa) Q_y."""
        if (x, y) not in self._F:
            self._F[(x, y)] = self.Q[x].T @ (self.eps[:, None] * self.Q[y])
        return self._F[(x, y)]

    def Sblk(self, A: Sequence[int], B: Sequence[int]) -> np.ndarray:
        """4-block overlap S_(A,B) = V_A^T V_B (eq. 4block_osv)."""
        return np.block([[self.S(a, b) for b in B] for a in A])

    def Fblk(self, A: Sequence[int], B: Sequence[int]) -> np.ndarray:
        return np.block([[self.F(a, b) for b in B] for a in A])

    # ---- O3: pair exchange integrals (eq. osv_close_k) --------------------
    def Kbar(self, p: int, q: int) -> np.ndarray:
        """K_(pq,pq) = [G~_{p,p}; G~_{p,q}] [G~_{q,p}; G~_{q,q}]^T, p <= q.

        Reading of eq. osv_close_k: the right factor holds the slab of q
        projected on both OSV blocks of the pair, as K^{ab}_pq = (pa|qb).
        """
        assert p <= q
        key = (p, q)
        if key not in self._K:
            o = orbs(p, q)
            L = np.concatenate([self.gamma(p, x) for x in o], 0)
            R = np.concatenate([self.gamma(q, x) for x in o], 0)
            self._K[key] = L @ R.T
        return self._K[key]

    # ---- O4: pair preconditioner basis (eq. prec_eig) ----------------------
    def basis(self, p: int, q: int):
        """X, eps~ with F X = S X diag(eps~), X^T S X = 1 (p <= q).

        Canonical orthogonalisation: eigenvectors of S_(pq,pq) with
        eigenvalue above tau_S, scaled by s^-1/2, then the eigenvectors of
        F in that basis.
        """
        assert p <= q
        key = (p, q)
        if key not in self._basis:
            o = orbs(p, q)
            Sm, Fm = self.Sblk(o, o), self.Fblk(o, o)
            s, U = np.linalg.eigh(Sm)
            keep = s > self.prob.tau_S
            X0 = U[:, keep] / np.sqrt(s[keep])[None, :]
            et, Z = np.linalg.eigh(X0.T @ Fm @ X0)
            self._basis[key] = (X0 @ Z, et)
        return self._basis[key]

    def denom(self, p: int, q: int) -> np.ndarray:
        """E~_(pq)[mu,nu] = f_pp + f_qq - eps~_mu - eps~_nu."""
        _, et = self.basis(p, q)
        return self.f[p, p] + self.f[q, q] - et[:, None] - et[None, :]

    # ---- O5: residual of one pair inside a fragment (eq. res_close) -------
    def get_T(self, T: dict, p: int, q: int) -> np.ndarray:
        """Amplitude of the ordered pair (p, q) from the stored p<=q ones."""
        if p <= q:
            return T[(p, q)]
        return swap_blocks(T[(q, p)], self.r[q], self.r[p])

    def residual(self, p: int, q: int, frag: Sequence[int], T: dict):
        """R_(pq,pq) with the k-sum restricted to the fragment, p <= q.

        R = K + F T S + S T F - sum_k [ f_pk S_(pq,kq) T_kq S_(kq,pq)
                                       + f_kq S_(pq,pk) T_pk S_(pk,pq) ]
        i.e. eq. res_close with its Kronecker deltas written out.
        """
        o = orbs(p, q)
        Sm, Fm = self.Sblk(o, o), self.Fblk(o, o)
        Tpq = T[(p, q)]
        R = self.Kbar(p, q) + Fm @ Tpq @ Sm + Sm @ Tpq @ Fm
        for k in frag:
            Sa = self.Sblk(o, orbs(k, q))
            R = R - self.f[p, k] * (Sa @ self.get_T(T, k, q) @ Sa.T)
            Sb = self.Sblk(o, orbs(p, k))
            R = R - self.f[k, q] * (Sb @ self.get_T(T, p, k) @ Sb.T)
        return R

    # ---- O5 + O6: one fragment, Alg. 7 (close clusters) -------------------
    def solve_fragment(self, frag: Sequence[int], tol: float, max_iter: int,
                       T0: Optional[dict] = None):
        """Iterate a cluster's residual equations to convergence.

        T starts at zero, or at T0[(p, q)] for the pairs T0 lists (the
        initial amplitudes are left open by Alg. 7; the fixed point does not
        depend on them).  Each sweep evaluates every pair residual from the
        same amplitudes (Jacobi order), transforms it to the pseudo-canonical
        basis, R~ = X^T R X, stops when max|R~| < tol, and otherwise applies
        T += X (R~ / E~) X^T (Alg. 7).  The energy is the Hylleraas
        functional sum_{p,q in F} <2T_pq - T_pq^T, K_pq + R_pq> (Frobenius
        product; off-diagonal pairs twice), which equals the paper's
        <K (2T - T^dagger)> at R = 0.
        """
        frag = sorted(int(x) for x in frag if x >= 0)
        plist = [(p, q) for a, p in enumerate(frag) for q in frag[a:]]
        T = {}
        for (p, q) in plist:
            d = sum(self.r[x] for x in orbs(p, q))
            T[(p, q)] = np.zeros((d, d)) if not T0 or (p, q) not in T0 else T0[(p, q)].copy()
        it = 0
        while True:
            R = {t: self.residual(t[0], t[1], frag, T) for t in plist}
            Rt = {}
            res = 0.0
            for t in plist:
                X, _ = self.basis(*t)
                Rt[t] = X.T @ R[t] @ X
                res = max(res, float(np.abs(Rt[t]).max()))
            if res < tol or it >= max_iter:
                break
            for t in plist:
                X, _ = self.basis(*t)
                T[t] = T[t] + X @ (Rt[t] / self.denom(*t)) @ X.T
            it += 1
        e_h, e_lin = [], []
        for (p, q) in plist:
            w = 1.0 if p == q else 2.0
            Tt = 2.0 * T[(p, q)] - T[(p, q)].T
            e_h.append(w * float(np.sum(Tt * (self.Kbar(p, q) + R[(p, q)]))))
            e_lin.append(w * float(np.sum(Tt * self.Kbar(p, q))))
        return dict(E=math.fsum(e_h), E_lin=math.fsum(e_lin), iters=it,
                    res=res, converged=res < tol, T=T)


# --------------------------------------------------------------------------
# O7: MBE(3) energy (eqs. tmbediag, tmbeoff, deltaoff)
# --------------------------------------------------------------------------
def mbe3_energy(frags: np.ndarray, e_frag: np.ndarray):
    """E = sum_i E_i + sum_ij dE_ij + sum_ijk dE_ijk over the given fragments.

    dE_ij = E_ij - E_i - E_j and dE_ijk = E_ijk - dE_ij - dE_ik - dE_jk
    - E_i - E_j - E_k: the energy of the amplitude expansion of eqs.
    tmbediag/tmbeoff, which is linear in the amplitudes.  Summed exactly
    rounded (math.fsum).  Returns (E, increments per fragment).
    """
    e1, e2 = {}, {}
    for f, e in zip(frags, e_frag):
        o = tuple(int(x) for x in f if x >= 0)
        if len(o) == 1:
            e1[o[0]] = e
    incr = np.zeros(len(frags))
    for n, (f, e) in enumerate(zip(frags, e_frag)):
        o = tuple(int(x) for x in f if x >= 0)
        if len(o) == 1:
            incr[n] = e
        elif len(o) == 2:
            incr[n] = e - e1[o[0]] - e1[o[1]]
            e2[o] = incr[n]
    for n, (f, e) in enumerate(zip(frags, e_frag)):
        o = tuple(int(x) for x in f if x >= 0)
        if len(o) == 3:
            i, j, k = o
            incr[n] = (e - e2[(i, j)] - e2[(i, k)] - e2[(j, k)]
                       - e1[i] - e1[j] - e1[k])
    return math.fsum(incr.tolist()), incr


def mbe3_coefficients(n_occ: int, frags: np.ndarray) -> np.ndarray:
    """c_F with E = sum_F c_F E_F, from expanding the increments above.

    c_ijk = 1, c_ij = 1 - #kept trimers containing ij,
    c_i = 1 - #kept pairs containing i + #kept trimers containing i.
    """
    deg = np.zeros(n_occ, dtype=np.int64)
    tri_i = np.zeros(n_occ, dtype=np.int64)
    tri_ij: Dict[Tuple[int, int], int] = {}
    for f in frags:
        o = [int(x) for x in f if x >= 0]
        if len(o) == 2:
            deg[o] += 1
        elif len(o) == 3:
            tri_i[o] += 1
            for a, b in ((o[0], o[1]), (o[0], o[2]), (o[1], o[2])):
                tri_ij[(a, b)] = tri_ij.get((a, b), 0) + 1
    c = np.zeros(len(frags))
    for n, f in enumerate(frags):
        o = [int(x) for x in f if x >= 0]
        if len(o) == 1:
            c[n] = 1 - deg[o[0]] + tri_i[o[0]]
        elif len(o) == 2:
            c[n] = 1 - tri_ij.get((o[0], o[1]), 0)
        else:
            c[n] = 1.0
    return c


# --------------------------------------------------------------------------
# Driver: the whole forward path
# --------------------------------------------------------------------------
_POOL_ORACLE = None
_POOL_WARM = None


def _own_pair(f) -> Optional[Tuple[int, int]]:
    """The pair slot a monomer or dimer fragment is the fragment of."""
    o = [int(x) for x in f if x >= 0]
    if len(o) == 1:
        return (o[0], o[0])
    if len(o) == 2:
        return (min(o), max(o))
    return None


def _warm_T0(f, warm):
    """Initial amplitudes of a trimer: each of its pairs from the solution of
    that pair's own fragment (monomer or dimer)."""
    if warm is None or (np.asarray(f) >= 0).sum() < 3:
        return None
    o = sorted(int(x) for x in f if x >= 0)
    return {(p, q): warm[(p, q)] for a, p in enumerate(o) for q in o[a:]}


def _one_blas_thread():
    """Pool workers each run one BLAS thread (the pool is the parallelism;
    a BLAS pool per worker would oversubscribe the cores)."""
    try:
        from threadpoolctl import threadpool_limits
        threadpool_limits(1)
    except ImportError:
        pass


def _solve_chunk(args):
    frags, tol, max_iter, keep_T = args
    ora = _POOL_ORACLE
    out = []
    for f in frags:
        s = ora.solve_fragment(f, tol, max_iter, _warm_T0(f, _POOL_WARM))
        if not keep_T:
            s.pop("T")
        out.append(s)
    return out


def prepare(ora: Oracle, frags: np.ndarray) -> None:
    """Fill the Gamma~, K, S/F and basis caches needed by ``frags``."""
    prob = ora.prob
    pairs = set()
    for f in frags:
        o = sorted(int(x) for x in f if x >= 0)
        for a, p in enumerate(o):
            for q in o[a:]:
                pairs.add((p, q))
    for (p, q) in sorted(pairs):
        ora.Kbar(p, q)
        ora.basis(p, q)
    for (p, q) in sorted(pairs):
        ora.S(q, p)


def _solve_list(ora, frags, tol, max_iter, keep_T, workers, warm):
    global _POOL_ORACLE, _POOL_WARM
    if workers <= 1 or len(frags) < 64:
        return [ora.solve_fragment(f, tol, max_iter, _warm_T0(f, warm)) for f in frags]
    import multiprocessing as mp
    _POOL_ORACLE, _POOL_WARM = ora, warm
    chunks = np.array_split(np.arange(len(frags)), workers * 8)
    ctx = mp.get_context("fork")
    with ctx.Pool(workers, initializer=_one_blas_thread) as pool:
        parts = pool.map(_solve_chunk,
                         [(frags[c], tol, max_iter, keep_T) for c in chunks])
    _POOL_ORACLE, _POOL_WARM = None, None
    return [s for part in parts for s in part]


def run(prob, frags: Optional[np.ndarray] = None, workers: int = 1,
        keep_T: bool = False, ora: Optional[Oracle] = None,
        warm_start: bool = False):
    """Solve ``frags`` (default: all fragments) and return per-fragment data.

    warm_start: every monomer and dimer is solved first from T = 0 (those of
    the trimers in ``frags`` too, if absent), and each trimer starts from
    the solutions of its pairs' own fragments; otherwise all start at T = 0.
    Returns dict with e_frag, e_lin, iters, converged (arrays in fragment
    order) and, if keep_T, the list of amplitude dicts.
    """
    if frags is None:
        frags = prob.frags
    ora = ora or Oracle(prob)
    prepare(ora, frags)
    tol, max_iter = prob.tol, prob.max_iter
    warm = None
    if warm_start:
        need = set()
        for f in frags:
            o = sorted(int(x) for x in f if x >= 0)
            for a, p in enumerate(o):
                for q in o[a:]:
                    need.add((p, q))
        own = np.array([[p, -1, -1] if p == q else [p, q, -1] for (p, q) in sorted(need)],
                       dtype=np.int32).reshape(-1, 3)
        sub = _solve_list(ora, own, tol, max_iter, True, workers, None)
        warm = {}
        for f, s in zip(own, sub):
            t = _own_pair(f)
            warm[t] = s["T"][t]
    res = _solve_list(ora, frags, tol, max_iter, keep_T, workers, warm)
    out = dict(e_frag=np.array([s["E"] for s in res]),
               e_lin=np.array([s["E_lin"] for s in res]),
               iters=np.array([s["iters"] for s in res], dtype=np.int64),
               converged=np.array([s["converged"] for s in res]),
               res=np.array([s["res"] for s in res]))
    if keep_T:
        out["T"] = [s["T"] for s in res]
    out["oracle"] = ora
    return out


def energy(prob, workers: int = 1, ora: Optional[Oracle] = None) -> float:
    """MBE(3)-OSV-MP2 correlation energy of the Problem."""
    frags = prob.frags
    out = run(prob, frags, workers=workers, ora=ora)
    return mbe3_energy(frags, out["e_frag"])[0]


# --------------------------------------------------------------------------
# O8: gradient through Hylleraas stationarity
# --------------------------------------------------------------------------
def fragment_gradient(ora: Oracle, frag: Sequence[int], T: dict):
    """Explicit derivatives of one fragment's Hylleraas energy at its
    converged amplitudes T (stored p <= q), the unit the MBE sums:
      Tt[(p, q)] = 2 T_pq - T_pq^T                      (multiplier share)
      g[x, y]    = dE_F/df_xy
                 = -[ sum_q <T~_xq, S_(xq,yq) T_yq S_(yq,xq)>
                    + sum_p <T~_py, S_(py,px) T_px S_(px,py)> ]
    with p, q, x, y over the fragment's orbitals (ordered pairs), i.e. the
    f-dependent terms of eq. res_close inside the functional.
    """
    o = sorted(int(x) for x in frag if x >= 0)
    Tt = {t: 2.0 * v - v.T for t, v in T.items()}
    g = np.zeros((ora.prob.n_occ, ora.prob.n_occ))
    for x in o:
        for y in o:
            acc = 0.0
            for q in o:
                Sa = ora.Sblk(orbs(x, q), orbs(y, q))
                Txq = ora.get_T(T, x, q)
                acc += np.sum((2.0 * Txq - Txq.T)
                              * (Sa @ ora.get_T(T, y, q) @ Sa.T))
            for p in o:
                Sb = ora.Sblk(orbs(p, y), orbs(p, x))
                Tpy = ora.get_T(T, p, y)
                acc += np.sum((2.0 * Tpy - Tpy.T)
                              * (Sb @ ora.get_T(T, p, x) @ Sb.T))
            g[x, y] = -acc
    return Tt, g


def gradient(prob, workers: int = 1, ora: Optional[Oracle] = None):
    """dE/dB_i (dict of [n_vir, n_aux]) and dE/df (symmetric [n_occ, n_occ]).

    Each fragment energy is stationary in its amplitudes, so its derivative
    with respect to K or f is the explicit derivative of the Hylleraas
    functional at the converged amplitudes (fragment_gradient), summed with
    the MBE(3) coefficients:
      W_pq = sum_{F containing p,q} c_F (2 T^F_pq - T^F_pq^T)
      dE/dB_i = 4 sum_{q in N+(i)} V_iq W_iq V_iq^T B_q
      dE/df = sum_F c_F g_F
    The symmetric gradient (g + g^T)/2 is returned.
    """
    frags = prob.frags
    out = run(prob, frags, workers=workers, keep_T=True, ora=ora)
    ora = out["oracle"]
    c = mbe3_coefficients(prob.n_occ, frags)
    W: Dict[Tuple[int, int], np.ndarray] = {}
    g = np.zeros((prob.n_occ, prob.n_occ))
    for f, cF, T in zip(frags, c, out["T"]):
        Tt, gF = fragment_gradient(ora, f, T)
        for t, v in Tt.items():
            W[t] = W.get(t, 0.0) + cF * v
        g += cF * gF
    dB = {}
    for i in range(prob.n_occ):
        acc = np.zeros((prob.n_vir, prob.n_aux))
        for q in prob.neighbours(i):
            q = int(q)
            if q == i:
                Wii = W[(i, i)]
                Wii = 0.5 * (Wii + Wii.T)
                acc += 4.0 * ora.Q[i] @ (Wii @ (ora.Q[i].T @ ora.B(i)))
            else:
                Wiq = W[(i, q)] if i < q else swap_blocks(W[(q, i)], ora.r[q], ora.r[i])
                V = np.concatenate([ora.Q[i], ora.Q[q]], 1)
                acc += 4.0 * V @ (Wiq @ (V.T @ ora.B(q)))
        dB[i] = acc
    E = mbe3_energy(frags, out["e_frag"])[0]
    return dict(E=E, dB=dB, df=0.5 * (g + g.T), W=W, c=c, run=out)
