"""CPU oracle for the MBE(3)-OSV-MP2 hot path (arXiv:2603.16575).

TEST INFRASTRUCTURE.  Only the test-suite, the smoke check and the CPU
baseline leg of the benchmark may import or run anything in this package; the
product path (the HIP library and its Python binding) never does.  The oracle
shares no code with the HIP path: the only common module is the seeded input
generator ``synth``.

Plain FP64 numpy, one fragment at a time, in the order of the paper's
equations and algorithms:
  O1 slab            counter-based (ia|P) regeneration     (Alg. 1 stand-in)
  O2 Oracle.gamma    OSV projection                        (eq. osv_imua)
  O3 Oracle.Kbar     4-block pair exchange integrals       (eq. osv_close_k)
  O4 Oracle.basis    pair preconditioner basis             (eq. prec_eig)
  O5 Oracle.residual fragment residual                     (eq. res_close)
  O6 solve_fragment  Jacobi iterations + Hylleraas energy  (Alg. 7)
  O7 mbe3_energy     MBE(3) inclusion-exclusion            (eqs. tmbediag, tmbeoff)
  O8 gradient        dE/d(ia|P), dE/df via stationarity    (derived; no paper formula)
  O9 weak.s2b, ...   pair metrics, classes, trimer screen  (eqs. s2b, s3b)
  O10 weak.weak_pair one-block weak-pair amplitudes/energy (eqs. osv_weak_k, res_weak)
  O11 fit.fit_metric sparse fitting metric and domains     (eq. sparse_fit_metric)

Pins (tests/test_oracle_*.py) tie each step to something other than itself:
numpy's own Philox, a full-space Kronecker dense solve, the canonical MP2
closed form (eq. mp2_tmat), vanishing trimer increments for a diagonal
occupied Fock matrix, the amplitude form of the expansion, invariance under
OSV rotations, homogeneity and the Euler identity, and central finite
differences.
"""
from .mbe3 import (Oracle, gradient, energy, fragment_gradient,
                   mbe3_coefficients, mbe3_energy, orbs, probe_direction, run, slab,
                   swap_blocks)
from .philox import box_muller, philox4x64_10
from . import fit, weak

__all__ = ["Oracle", "gradient", "energy", "fragment_gradient",
           "mbe3_coefficients", "mbe3_energy",
           "orbs", "probe_direction", "run", "slab", "swap_blocks", "box_muller",
           "philox4x64_10", "fit", "weak"]
