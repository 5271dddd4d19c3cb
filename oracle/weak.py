"""Pair screening and the weak-pair path of MBE(3)-OSV-MP2.

TEST INFRASTRUCTURE ONLY: nothing in the product path may import this module.

  O9  s2b / s3b metrics, pair classes, trimer screening
      (eqs. s2b, s3b; thresholds from the section on OSV overlap and Fock
      computation)
  O10 weak pairs: one-block exchange integrals (eq. osv_weak_k), the
      one-block residual (eq. res_weak) solved directly in the diagonal
      pairs' pseudo-canonical bases, and the pair energy (the weak-pair part
      of Alg. 7)

Readings (the printed eq. res_weak does not type-check; the design notes
list them with the others):
  W1  T_(i,j) F_(j,i) -> T_(i,j) F_(j,j), (f_ij + f_ii) -> (f_ii + f_jj),
      S_(i,i) T_(j,j) -> S_(i,j) T_(j,j).  With orthonormal OSVs of one LMO
      (S_(i,i) = 1) these are the (mu_i, nu_j) block of eq. res_close for the
      pair ij with the exchange blocks dropped:
        R_(i,j) = K_(i,j) + T_(i,j) F_(j,j) + F_(i,i) T_(i,j)
                  - (f_ii + f_jj) T_(i,j) - f_ij [T_(i,i) S_(i,j) + S_(i,j) T_(j,j)].
  W2  T_(i,i) are the MBE(3) diagonal amplitudes T^MBE_ii = sum_F c_F T^F_ii
      (eq. tmbediag); the function below takes them as inputs.
  W3  Pair energy of an unordered weak pair i < j: 4 <K_(i,j), T_(i,j)>, the
      close-pair energy w <2T - T^T, K> (w = 2) restricted to the one block
      (the exchange block of K is dropped with the exchange amplitudes); the
      paper's 2 <K T> is read per ordered pair.  The canonical-MP2 pin fixes
      this factor independently.
"""
from __future__ import annotations

import math
from typing import Dict, Iterable, Sequence, Tuple

import numpy as np

from .mbe3 import mbe3_coefficients, run

# pair classes (section on OSV overlap and Fock computation)
S2B_DISTANT = 1e-7   # s2b below: discarded
S2B_CLOSE = 1e-2     # s2b at or above: close pair; in between: weak pair
S3B_KEEP = 0.2       # trimers with s3b below are discarded


def s2b(ora, i: int, j: int) -> float:
    """eq. s2b: sum_{mu nu} <mu_i|nu_j>^2 / sqrt(r_i r_j)."""
    S = ora.Q[i].T @ ora.Q[j]
    return float(np.sum(S * S) / math.sqrt(ora.r[i] * ora.r[j]))


def pair_class(value: float) -> str:
    """'distant', 'weak' or 'close' by the s2b thresholds."""
    if value < S2B_DISTANT:
        return "distant"
    return "weak" if value < S2B_CLOSE else "close"


def s3b(s_ij: float, s_ik: float, s_jk: float) -> float:
    """eq. s3b: the mean of the trimer's three pair metrics."""
    return (s_ij + s_ik + s_jk) / 3.0


def keep_trimer(s_ij: float, s_ik: float, s_jk: float) -> bool:
    return s3b(s_ij, s_ik, s_jk) >= S3B_KEEP


def mbe3_diagonal_amplitudes(prob, out=None) -> Dict[int, np.ndarray]:
    """T^MBE_ii = sum over fragments F containing i of c_F T^F_(i,i)
    (eq. tmbediag), from an oracle run with keep_T (done here if not given)."""
    if out is None:
        out = run(prob, prob.frags, keep_T=True)
    c = mbe3_coefficients(prob.n_occ, prob.frags)
    T = {}
    for f, cF, Tf in zip(prob.frags, c, out["T"]):
        for x in (int(v) for v in f if v >= 0):
            T[x] = T.get(x, 0.0) + cF * Tf[(x, x)]
    return T


def weak_K(ora, i: int, j: int) -> np.ndarray:
    """eq. osv_weak_k: K_(i,j) = Gamma~_(i,i) Gamma~_(j,j)^T  (r_i x r_j)."""
    return ora.gamma(i, i) @ ora.gamma(j, j).T


def weak_pair(ora, i: int, j: int, T_ii: np.ndarray, T_jj: np.ndarray):
    """One weak pair (i != j): the amplitudes T_(i,j) that make the
    one-block residual (reading W1) vanish, found the way the paper's
    weak-pair loop does: the residual at T_(i,j) = 0, transformed into the
    diagonal pairs' pseudo-canonical bases (eq. prec_eig for (i,i) and
    (j,j)), divided by f_ii + f_jj - eps~_mu - eps~_nu and transformed back.
    Returns (T_(i,j), energy 4 <K_(i,j), T_(i,j)> (reading W3), K_(i,j))."""
    f = ora.f
    K = weak_K(ora, i, j)
    S = ora.Q[i].T @ ora.Q[j]
    R0 = K - f[i, j] * (T_ii @ S + S @ T_jj)
    Xi, ei = ora.basis(i, i)
    Xj, ej = ora.basis(j, j)
    Rt = Xi.T @ R0 @ Xj
    Tt = Rt / (f[i, i] + f[j, j] - ei[:, None] - ej[None, :])
    T = Xi @ Tt @ Xj.T
    return T, 4.0 * float(np.sum(K * T)), K


def weak_residual(ora, i: int, j: int, T: np.ndarray, T_ii: np.ndarray,
                  T_jj: np.ndarray) -> np.ndarray:
    """The one-block residual of reading W1 at T_(i,j) = T."""
    f = ora.f
    S = ora.Q[i].T @ ora.Q[j]
    Fi = ora.F(i, i)
    Fj = ora.F(j, j)
    return (weak_K(ora, i, j) + T @ Fj + Fi @ T - (f[i, i] + f[j, j]) * T
            - f[i, j] * (T_ii @ S + S @ T_jj))


def weak_energies(ora, pairs: Iterable[Sequence[int]],
                  T_diag: Dict[int, np.ndarray]) -> np.ndarray:
    """Pair energies of the listed weak pairs (i < j) from the diagonal
    amplitudes T_diag[i] (reading W2)."""
    return np.array([weak_pair(ora, int(i), int(j), T_diag[int(i)], T_diag[int(j)])[1]
                     for i, j in pairs])


def screened_lists(n_occ: int, s2b_of: Dict[Tuple[int, int], float]):
    """The pair and trimer lists the paper's screening gives (section on OSV
    overlap and Fock computation), by brute force: every candidate pair
    (i < j, metric s2b_of[(i, j)]) classed by pair_class; every triple
    i < j < k whose three pairs are all close candidates kept when
    keep_trimer holds.  Returns (close pairs, weak pairs, trimers) as sorted
    lists of tuples."""
    cls = {t: pair_class(v) for t, v in s2b_of.items()}
    close = sorted(t for t, c in cls.items() if c == "close")
    weak = sorted(t for t, c in cls.items() if c == "weak")
    is_close = set(close)
    tris = []
    for i in range(n_occ):
        for j in range(i + 1, n_occ):
            if (i, j) not in is_close:
                continue
            for k in range(j + 1, n_occ):
                if (i, k) in is_close and (j, k) in is_close and \
                        keep_trimer(s2b_of[(i, j)], s2b_of[(i, k)], s2b_of[(j, k)]):
                    tris.append((i, j, k))
    return close, weak, tris
