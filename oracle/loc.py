"""Occupied-orbital localization: Pipek-Mezey with Jacobi sweeps and Loewdin
charges (the paper's section on occupied orbital localization, Alg. 2 and
eq. loc_theta).

TEST INFRASTRUCTURE ONLY: nothing in the product path may import this module.

  O13 charges      P^A_ij = sum_{alpha in A} C~_{alpha i} C~_{alpha j} for
                   symmetrically orthonormalized MO coefficients C~
      functional   L = sum_{i, A} (P^A_ii)^2
      jacobi_pm    sweeps over the pairs i < j in order: a_ij, b_ij and the
                   angle of eq. loc_theta, the increment
                   sqrt(a^2 + b^2)(1 - cos 4 theta), rotation of the columns
                   of U and of both orbital indices of P, until a sweep's
                   summed increment is at most l_loc

Readings (listed with the others in the design notes):
  L1  theta = (1/4) arctan(b / -a) is the two-argument arctangent,
      4 theta = atan2(b, -a): it maximizes L over the pair rotation, where
      the one-argument form picks the minimizer whenever a > 0.  With it the
      printed increment is exactly the gain of the rotation.
  L2  The loop runs while the previous sweep's summed increment exceeds
      l_loc (the first sweep always runs); l_loc = 1e-3 as in the paper.
  L3  A pair is rotated when |sin theta| >= 1e-10, as printed; the
      rotation is i' = cos(theta) i + sin(theta) j, j' = cos(theta) j -
      sin(theta) i, on the columns of U, then on the first and the second
      orbital index of every P^A.
"""
from __future__ import annotations

import math

import numpy as np

L_LOC = 1e-3
SIN_MIN = 1e-10


def charges(C: np.ndarray, ao_off: np.ndarray) -> np.ndarray:
    """[n_atom, n, n] Loewdin charges P^A = C_A^T C_A over the AOs of A."""
    return np.stack([C[a0:a1].T @ C[a0:a1] for a0, a1 in zip(ao_off[:-1], ao_off[1:])])


def functional(P: np.ndarray) -> float:
    """L = sum_{i,A} (P^A_ii)^2."""
    d = np.diagonal(P, axis1=1, axis2=2)
    return float(np.sum(d * d))


def pair_ab(P: np.ndarray, i: int, j: int):
    """eq. loc_theta: a_ij and b_ij."""
    Pij, Pii, Pjj = P[:, i, j], P[:, i, i], P[:, j, j]
    a = float(np.sum(Pij * Pij - 0.25 * (Pii - Pjj) ** 2))
    b = float(np.sum(Pij * (Pii - Pjj)))
    return a, b


def rotate(P: np.ndarray, U: np.ndarray, i: int, j: int, c: float, s: float) -> None:
    """Reading L3, in place: columns of U, first then second index of P."""
    ui, uj = U[:, i].copy(), U[:, j].copy()
    U[:, i], U[:, j] = c * ui + s * uj, c * uj - s * ui
    pi, pj = P[:, i, :].copy(), P[:, j, :].copy()
    P[:, i, :], P[:, j, :] = c * pi + s * pj, c * pj - s * pi
    pi, pj = P[:, :, i].copy(), P[:, :, j].copy()
    P[:, :, i], P[:, :, j] = c * pi + s * pj, c * pj - s * pi


def jacobi_pm(P0: np.ndarray, l_loc: float = L_LOC, max_sweeps: int = 100):
    """Alg. 2 on the charges P0 ([n_atom, n, n], not modified).  Returns
    dict(U [n, n], P, dL per sweep, L per sweep end, sweeps, rotations per
    sweep)."""
    P = P0.copy()
    n = P.shape[1]
    U = np.eye(n)
    dLs, Ls, rots = [], [], []
    dL = math.inf
    while dL > l_loc and len(dLs) < max_sweeps:
        dL, nrot = 0.0, 0
        for i in range(n):
            for j in range(i + 1, n):
                a, b = pair_ab(P, i, j)
                theta = 0.25 * math.atan2(b, -a)
                s, c = math.sin(theta), math.cos(theta)
                if abs(s) >= SIN_MIN:
                    dL += math.sqrt(a * a + b * b) * (1.0 - math.cos(4.0 * theta))
                    rotate(P, U, i, j, c, s)
                    nrot += 1
        dLs.append(dL)
        Ls.append(functional(P))
        rots.append(nrot)
    return dict(U=U, P=P, dL=dLs, L=Ls, sweeps=len(dLs), rotations=rots)
