"""Sparse fitting domains of MBE(3)-OSV-MP2 (eq. sparse_fit_metric).

TEST INFRASTRUCTURE ONLY: nothing in the product path may import this module.

  O11 fit_metric  s_fit[i, A] = sum over the slab's orbital index of
                  B_i[., A]^2, for every auxiliary function A
      domain      D_i = {A : s_fit[i, A] > l_fit}
      restricted  the method with the exchange integrals of every pair
                  (p, q) summed over A in D_p u D_q only (the diagonal pair
                  over D_p), from the unrestricted slabs

Readings (listed with the others in the design notes):
  F1  The metric sums over the slab's first index, the virtual MO a here,
      where the paper's fitted Gamma_i carries the AO index alpha; the slab
      stands in for Gamma_i throughout (O1).
  F2  Eqs. osv_imua, osv_close_k and osv_weak_k (and the contraction loop of
      Alg. 6) run A' over D_i u D_j, the union of the two LMOs' domains.
      K_(pq,pq) therefore sums over D_p u D_q, and every Gamma~ block it
      reads is taken on that set, including Gamma~_{p,p} on D_q \\ D_p (Alg.
      6 fetches the diagonal-pair blocks for each pair's union, so they are
      known beyond their own LMO's domain); the diagonal slot (p, p) sums
      over D_p.  Pair bases, residuals, energies and the MBE(3) sum run
      unchanged on these integrals.  Stored per block, eq. osv_imua gives
      Gamma~_{i,x} on D_i u D_x (x != i) and, for the diagonal block read by
      every pair (i, q), on the union of D_q over q in N+(i).
  F3  Selection is strict, as printed: A is kept when s_fit > l_fit.  The
      sparsity table's threshold is 1e-6.
"""
from __future__ import annotations

from typing import Dict, Optional

import numpy as np

from .mbe3 import Oracle, orbs

L_FIT = 1e-6  # the paper's fitting threshold (sparsity table)


def column_metric(B: np.ndarray) -> np.ndarray:
    """eq. sparse_fit_metric for one slab: sum over its first index of the
    squared elements, one value per auxiliary function."""
    return np.sum(B * B, axis=0)


def fit_metric(ora: Oracle, i: int) -> np.ndarray:
    """s_fit[i, A] = sum_a B_i[a, A]^2, shape [n_aux]."""
    return column_metric(ora.B(i))


def fit_metrics(ora: Oracle) -> np.ndarray:
    """s_fit of every LMO, [n_occ, n_aux]."""
    return np.stack([fit_metric(ora, i) for i in range(ora.prob.n_occ)])


def domain(s_fit: np.ndarray, l_fit: float) -> np.ndarray:
    """Membership of D_i (reading F3): s_fit > l_fit, elementwise."""
    return s_fit > l_fit


class RestrictedOracle(Oracle):
    """The method restricted to the fitting domains (reading F2).

    The slabs stay unrestricted; the metric of LMO i is computed from its
    slab on first use (or taken from ``s_fit``), and K_(pq,pq) sums over
    D_p u D_q only.  ``base`` (optional) lends its already regenerated
    slabs."""

    def __init__(self, prob, l_fit: float, base: Optional[Oracle] = None,
                 s_fit: Optional[np.ndarray] = None):
        super().__init__(prob, slabs=base._slabs if base is not None else None)
        self.l_fit = l_fit
        self.s: Dict[int, np.ndarray] = {}
        if s_fit is not None:
            self.s = {i: np.asarray(s_fit[i]) for i in range(prob.n_occ)}

    def metric(self, i: int) -> np.ndarray:
        if i not in self.s:
            self.s[i] = column_metric(self.B(i))
        return self.s[i]

    def dom(self, i: int) -> np.ndarray:
        """D_i as a boolean mask over the auxiliary functions."""
        return domain(self.metric(i), self.l_fit)

    def pair_union(self, p: int, q: int) -> np.ndarray:
        """The auxiliary functions a pair's integrals sum over: D_p u D_q."""
        return self.dom(p) | self.dom(q)

    def Kbar(self, p: int, q: int) -> np.ndarray:
        """eq. osv_close_k over A' in D_p u D_q (reading F2):
        K_(pq,pq) = sum_{A' in D_p u D_q} L[:, A'] R[:, A']^T with
        L = [G~_{p,p}; G~_{p,q}], R = [G~_{q,p}; G~_{q,q}] (p <= q)."""
        assert p <= q
        key = (p, q)
        if key not in self._K:
            U = self.pair_union(p, q)
            o = orbs(p, q)
            L = np.concatenate([self.gamma(p, x)[:, U] for x in o], 0)
            R = np.concatenate([self.gamma(q, x)[:, U] for x in o], 0)
            self._K[key] = L @ R.T
        return self._K[key]

    def gamma_fit(self, i: int, x: int) -> np.ndarray:
        """Gamma~_{i,x} as eq. osv_imua stores it over the domains (reading
        F2): columns outside D_i u D_x (x != i), or outside the union of
        D_q over q in N+(i) for the diagonal block, set to zero."""
        if x != i:
            keep = self.dom(i) | self.dom(x)
        else:
            keep = np.zeros(self.prob.n_aux, dtype=bool)
            for q in self.prob.neighbours(i):
                keep |= self.dom(int(q))
        return np.where(keep[None, :], self.gamma(i, x), 0.0)

    def weak_K(self, i: int, j: int) -> np.ndarray:
        """eq. osv_weak_k over A' in D_i u D_j:
        K_(i,j) = sum_{A'} G~_{i,i}[:, A'] G~_{j,j}[:, A']^T."""
        U = self.pair_union(i, j)
        return self.gamma(i, i)[:, U] @ self.gamma(j, j)[:, U].T


def restricted_oracle(prob, l_fit: float, base: Optional[Oracle] = None,
                      s_fit: Optional[np.ndarray] = None) -> RestrictedOracle:
    """The restricted method (reading F2) with the metric ``s_fit`` if given,
    else computed from the slabs (those of ``base`` when given)."""
    return RestrictedOracle(prob, l_fit, base=base, s_fit=s_fit)
