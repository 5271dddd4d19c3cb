"""Randomized OSV generation (the paper's section on randomized OSV
generation: Alg. 3 with eqs. mp2_tkk, rsvd_z, tsub, tii_rsvd, back_q,
rsvd_za).

TEST INFRASTRUCTURE ONLY: nothing in the product path may import this module.

  O12 semicanonical_T  T_ii[a,b] = sum_{A' in D_i} B_i[a,A'] B_i[b,A']
                                   / (f_aa + f_bb - 2 f_ii)      (eq. mp2_tkk)
      gaussian_rows    the Gaussian test rows G (first r) and G-bar (the
                       next n_max) of LMO i, counter-based
      rosv             adaptive randomized range finder over the rows of
                       Y = G T, row Gram-Schmidt (eq. rsvd_za), T~ = Z T
                       (eq. tsub), SVD T~ = Q~ w V~^T (eq. tii_rsvd),
                       Q_i = Z^T Q~ (eq. back_q), columns with w >= l_osv
      exact_osv        the definition the randomized scheme approximates
                       (eq. osv_gen): eigenvectors of T_ii with eigenvalue
                       >= l_osv

Readings (listed with the others in the design notes):
  R1  The slab B_i (the fitted (ia|P) stand-in) plays the MO-indexed
      Gamma~_i^{aA'} of eq. mp2_tkk; D_i is the fitting domain of eq.
      sparse_fit_metric (every A' when no threshold is given).
  R2  The Gaussian rows are counter-based so that both sides draw the same
      matrix: row s, column a of LMO i is the Box-Muller normal of words 0
      and 1 of the Philox4x64-10 block at counter (a, s, i, 0) under key
      (seed, 11).  Rows 0 .. r-1 form G, rows r .. r + n_max - 1 form
      G-bar (row r + s - 1 draws the sample y^(s+r)).
  R3  The loop runs while the largest norm among the r pending rows exceeds
      l_osv / (10 sqrt(2/pi)), as printed, and stops at n_max rows at the
      latest (the paper pre-allocates N_rosv^max rows).  Each step takes
      the first pending row, orthogonalises it against the accepted rows
      (eq. rsvd_za), normalises and accepts it, appends the next sample
      orthogonalised against the rows accepted before this step, and
      removes the new row's component from every pending row.
  R4  The singular values w of T~ are compared with l_osv (columns with
      w >= l_osv are kept), largest first.
"""
from __future__ import annotations

import math

import numpy as np

from .mbe3 import slab
from .philox import box_muller, philox4x64_10

STREAM_ROSV = 11
R_BLOCK = 10        # rows per block of the stopping test (the paper's r)
L_OSV = 1e-4        # the paper's OSV threshold


def semicanonical_T(B: np.ndarray, eps: np.ndarray, f_ii: float,
                    keep: np.ndarray = None) -> np.ndarray:
    """eq. mp2_tkk: T[a,b] = sum_{A' in D} B[a,A'] B[b,A'] / (eps_a + eps_b
    - 2 f_ii), D given by the boolean mask ``keep`` over the columns (all
    columns when None)."""
    Bd = B if keep is None else B[:, keep]
    return (Bd @ Bd.T) / (eps[:, None] + eps[None, :] - 2.0 * f_ii)


def gaussian_rows(seed: int, i: int, n_rows: int, n_vir: int,
                  impl: str = "c") -> np.ndarray:
    """Reading R2: [n_rows, n_vir] standard normals at counters
    (a, s, i, 0), key (seed, 11); impl "c" through the oracle's C routine
    (the slab routine with row s in place of the virtual index and column a
    in place of the auxiliary one), "numpy" vectorised here."""
    if impl == "c":
        from . import _clib
        return _clib.normal_slab((seed, STREAM_ROSV), i, n_rows, np.arange(n_vir))
    ctr = np.zeros((n_rows, n_vir, 4), dtype=np.uint64)
    ctr[..., 0] = np.arange(n_vir, dtype=np.uint64)[None, :]
    ctr[..., 1] = np.arange(n_rows, dtype=np.uint64)[:, None]
    ctr[..., 2] = np.uint64(i)
    w = philox4x64_10(ctr, (seed, STREAM_ROSV))
    return box_muller(w[..., 0], w[..., 1])


def rosv(T: np.ndarray, G_all: np.ndarray, l_osv: float = L_OSV,
         r: int = R_BLOCK, n_max: int = None):
    """Alg. 3 on one symmetric T (n x n) with the Gaussian rows G_all
    ([r + n_max, n], reading R2).  Returns dict(Q [n, k], w [k], Z [s, n],
    rows s, capped: whether the loop stopped at n_max, pending_max: the
    largest pending row norm at the stop, threshold: the stopping test's
    bound)."""
    n = T.shape[0]
    if n_max is None:
        n_max = G_all.shape[0] - r
    thr = l_osv / (10.0 * math.sqrt(2.0 / math.pi))
    Y = G_all[:r] @ T                    # pending rows y^(1..r)
    Ybar = G_all[r:r + n_max] @ T        # the later samples
    Z = np.zeros((0, n))
    s = 0
    while s < n_max and max(float(np.linalg.norm(y)) for y in Y) > thr:
        s += 1
        y = Y[0]
        zt = y - (y @ Z.T) @ Z           # eq. rsvd_za
        z = zt / np.linalg.norm(zt)
        Z_prev = Z
        Z = np.vstack([Z, z])
        y_new = Ybar[s - 1] - (Ybar[s - 1] @ Z_prev.T) @ Z_prev
        Y = np.vstack([Y[1:], y_new])
        Y = Y - np.outer(Y @ z, z)       # remove the accepted direction
    pending = max(float(np.linalg.norm(y)) for y in Y)
    Tt = Z @ T                            # eq. tsub
    Qt, w, _ = np.linalg.svd(Tt, full_matrices=False)   # eq. tii_rsvd
    Q = Z.T @ Qt                          # eq. back_q
    keep = w >= l_osv
    return dict(Q=Q[:, keep], w=w[keep], Z=Z, rows=s, capped=s == n_max and s > 0,
                pending_max=pending, threshold=thr)


def exact_osv(T: np.ndarray, l_osv: float = L_OSV):
    """eq. osv_gen: eigenvectors of T with eigenvalue >= l_osv, largest
    first (the definition the randomized scheme approximates)."""
    lam, U = np.linalg.eigh(T)
    order = np.argsort(-lam)
    lam, U = lam[order], U[:, order]
    keep = lam >= l_osv
    return U[:, keep], lam[keep]


def lmo_rosv(prob, i: int, l_fit: float = None, n_max: int = 128,
             l_osv: float = L_OSV):
    """The randomized OSVs of LMO i of a workload: T_ii from its slab on the
    fitting domain (all columns when l_fit is None), the counter-based
    Gaussian rows, Alg. 3.  Returns rosv's dict plus T."""
    B = slab(prob, i)
    keep = None if l_fit is None else np.sum(B * B, axis=0) > l_fit
    T = semicanonical_T(B, np.asarray(prob.eps_vir), float(prob.f_occ[i, i]), keep)
    G = gaussian_rows(prob.seed, i, R_BLOCK + n_max, prob.n_vir)
    out = rosv(T, G, l_osv=l_osv, n_max=n_max)
    out["T"] = T
    return out
