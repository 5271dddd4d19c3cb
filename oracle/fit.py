"""Sparse fitting domains of MBE(3)-OSV-MP2 (eq. sparse_fit_metric).

TEST INFRASTRUCTURE ONLY: nothing in the product path may import this module.

  O11 fit_metric  s_fit[i, A] = sum over the slab's orbital index of
                  B_i[., A]^2, for every auxiliary function A
      domain      D_i = {A : s_fit[i, A] > l_fit}
      restricted  the method with every product over the auxiliary index of
                  slab i limited to D_i: an Oracle whose slabs are B_i with
                  the columns outside D_i set to zero

Readings (listed with the others in the design notes):
  F1  The metric sums over the slab's first index, the virtual MO a here,
      where the paper's fitted Gamma_i carries the AO index alpha; the slab
      stands in for Gamma_i throughout (O1).
  F2  Gamma~_i exists on D_i only, so a pair's exchange integrals
      K_(pq) = sum_A Gamma~_p[., A] Gamma~_q[., A] run over D_p and D_q
      together, the intersection of the two domains: zeroing the columns
      of each slab outside its own domain gives exactly that sum, and the
      same restricted slabs feed every later step unchanged.
  F3  Selection is strict, as printed: A is kept when s_fit > l_fit.  The
      sparsity table's threshold is 1e-6.
"""
from __future__ import annotations

from typing import Dict, Optional

import numpy as np

from .mbe3 import Oracle, slab

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


def restricted_oracle(prob, l_fit: float, base: Optional[Oracle] = None,
                      s_fit: Optional[np.ndarray] = None) -> Oracle:
    """An Oracle for the method restricted to the fitting domains (reading
    F2): slab i keeps its columns in D_i and is zero elsewhere.  ``s_fit``
    (optional) supplies the metric, else it is computed from ``base``."""
    base = base or Oracle(prob)
    if s_fit is None:
        s_fit = fit_metrics(base)
    mask = domain(s_fit, l_fit)
    slabs: Dict[int, np.ndarray] = {
        i: base.B(i) * mask[i][None, :] for i in range(prob.n_occ)}
    return Oracle(prob, slabs=slabs)


class RestrictedOracle(Oracle):
    """The restricted method with slabs restricted when first used (for
    samples of large workloads): slab i is regenerated, its metric kept in
    ``s[i]``, and its columns outside D_i set to zero, as in
    restricted_oracle."""

    def __init__(self, prob, l_fit: float):
        super().__init__(prob)
        self.l_fit = l_fit
        self.s: Dict[int, np.ndarray] = {}

    def B(self, i: int) -> np.ndarray:
        if i not in self._slabs:
            b = slab(self.prob, i)
            self.s[i] = column_metric(b)
            self._slabs[i] = b * domain(self.s[i], self.l_fit)[None, :]
        return self._slabs[i]
