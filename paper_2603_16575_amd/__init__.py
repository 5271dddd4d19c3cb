"""MBE(3)-OSV-MP2 hot path on AMD Instinct MI355X (gfx950).

Python face of the C-ABI library ``libmbe3osv`` (include/mbe3osv.h).  The
entry points keep the C names: ``osv_project``, ``pair_K``,
``fragment_solve``, ``mbe3_energy``, ``mbe3_backward`` and
``mbe3_pair_basis``; ``Mbe3`` owns a library handle for one problem.  Device
arrays are torch CUDA (HIP) tensors, which supply memory and the stream; the
arithmetic runs in the library.  ``energy_fn`` exposes the energy as a
differentiable torch function of the slab and the occupied Fock matrix.
"""
import ctypes

import numpy as np

from . import _lib
from ._lib import (MBE3_EHIP, MBE3_EINVAL, MBE3_ENOCONV, MBE3_ENOMEM,
                   MBE3_ENONFINITE, MBE3_FP64, MBE3_GRAD_GAMMA, MBE3_GRAD_PROBE,
                   MBE3_GRAD_SLAB, MBE3_MIXED_BF16, MBE3_MIXED_BF16_PROJ, MBE3_OK, Mbe3Error)

__all__ = ["Mbe3", "Mbe3Error", "osv_project", "pair_K", "fragment_solve",
           "mbe3_energy", "mbe3_backward", "mbe3_pair_basis", "energy_fn",
           "MBE3_OK", "MBE3_EINVAL", "MBE3_ENOMEM", "MBE3_EHIP",
           "MBE3_ENOCONV", "MBE3_ENONFINITE", "MBE3_GRAD_SLAB",
           "MBE3_GRAD_GAMMA", "MBE3_GRAD_PROBE", "MBE3_FP64", "MBE3_MIXED_BF16",
           "MBE3_MIXED_BF16_PROJ", "L_FIT", "screen_lists",
           "S2B_DISTANT", "S2B_CLOSE", "S3B_KEEP", "pm_localize", "L_LOC"]


def _f64(t):
    import torch
    assert t.dtype == torch.float64 and t.is_cuda and t.is_contiguous()
    return t


class Mbe3:
    """One problem on one device.

    Q, eps_vir, f_occ, w_ia, w_iP (or slab): contiguous float64 CUDA tensors,
    kept referenced by the handle.  r, pairs, frags: host int arrays.
    precision: MBE3_FP64, MBE3_MIXED_BF16 (split projection and pair_K) or
        MBE3_MIXED_BF16_PROJ (split projection, FP64 pair_K).
    warm_start: trimers start from the converged monomer/dimer amplitudes
    (same solution to the threshold, fewer updates); False: T = 0 throughout.
    """

    def __init__(self, *, r, Q, eps_vir, f_occ, pairs, frags, seed=0,
                 w_ia=None, w_iP=None, slab=None, tol=1e-8, max_iter=100,
                 tau_S=1e-8, stream=None, precision=MBE3_FP64, warm_start=True):
        import torch
        lib = _lib.load()
        self._keep = [Q, eps_vir, f_occ, w_ia, w_iP, slab]
        self.f_occ, self.slab = f_occ, slab
        for t in (Q, eps_vir, f_occ, w_ia, w_iP, slab):
            if t is not None:
                _f64(t)
        self.device = Q.device
        self.r = np.ascontiguousarray(r, dtype=np.int32)
        self.pairs = np.ascontiguousarray(pairs, dtype=np.int32).reshape(-1, 2)
        self.frags = np.ascontiguousarray(frags, dtype=np.int32).reshape(-1, 3)
        n_occ = len(self.r)
        p = _lib.Mbe3Problem()
        p.n_occ = n_occ
        p.n_vir = int(eps_vir.numel())
        p.n_aux = int(w_iP.shape[1]) if w_iP is not None else int(slab.shape[2])
        p.r = _lib.ptr(self.r)
        p.Q = _lib.ptr(Q)
        p.eps_vir = _lib.ptr(eps_vir)
        p.f_occ = _lib.ptr(f_occ)
        p.seed = int(seed)
        p.w_ia = _lib.ptr(w_ia)
        p.w_iP = _lib.ptr(w_iP)
        p.slab = _lib.ptr(slab)
        p.n_pair = len(self.pairs)
        p.pairs = _lib.ptr(self.pairs) if len(self.pairs) else None
        p.n_frag = len(self.frags)
        p.frags = _lib.ptr(self.frags)
        p.tol = float(tol)
        p.max_iter = int(max_iter)
        p.tau_S = float(tau_S)
        p.precision = int(precision)
        p.warm_start = int(bool(warm_start))
        self.precision = int(precision)
        if stream is None:
            stream = torch.cuda.current_stream(self.device)
        self.stream = stream
        self._h = ctypes.c_void_p()
        rc = lib.mbe3_create(ctypes.byref(self._h), ctypes.byref(p),
                             ctypes.c_void_p(stream.cuda_stream))
        _lib.check(rc, None)
        lay = _lib.Mbe3Layout()
        _lib.check(lib.mbe3_get_layout(self._h, ctypes.byref(lay)), self._h)
        self.layout = lay
        self.n_occ = n_occ
        self.n_vir = p.n_vir
        self.n_aux = p.n_aux
        self.n_frag = lay.n_frag
        self.g_off = np.zeros(n_occ + 1, dtype=np.int64)
        _lib.check(lib.mbe3_gamma_offsets(self._h, _lib.ptr(self.g_off)), self._h)
        self.k_off = np.zeros(lay.n_slot + 1, dtype=np.int64)
        _lib.check(lib.mbe3_k_offsets(self._h, _lib.ptr(self.k_off)), self._h)
        self.x_off = np.zeros(lay.n_slot + 1, dtype=np.int64)
        self.e_off = np.zeros(lay.n_slot + 1, dtype=np.int64)
        _lib.check(lib.mbe3_basis_offsets(self._h, _lib.ptr(self.x_off),
                                          _lib.ptr(self.e_off)), self._h)

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            _lib.load().mbe3_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---- allocation helpers (torch owns memory) ----
    def empty_gamma(self):
        import torch
        return torch.empty(self.layout.gamma_elems, dtype=torch.float64,
                           device=self.device)

    def empty_K(self):
        import torch
        return torch.empty(self.layout.k_elems, dtype=torch.float64,
                           device=self.device)

    # ---- C-ABI calls ----
    def osv_project(self, gamma):
        _lib.check(_lib.load().osv_project(self._h, _lib.ptr(_f64(gamma)),
                                           gamma.numel()), self._h)
        return gamma

    def pair_K(self, gamma, K):
        _lib.check(_lib.load().pair_K(self._h, _lib.ptr(_f64(gamma)),
                                      _lib.ptr(_f64(K)), K.numel()), self._h)
        return K

    def fragment_solve(self, K, e_frag, iters, W=None, check=True):
        rc = _lib.load().fragment_solve(self._h, _lib.ptr(_f64(K)),
                                        _lib.ptr(e_frag), _lib.ptr(iters),
                                        _lib.ptr(W))
        if check:
            _lib.check(rc, self._h)
        return rc

    def mbe3_energy(self, e_frag, incr=None):
        out = np.zeros(1, dtype=np.float64)
        _lib.check(_lib.load().mbe3_energy(self._h, _lib.ptr(e_frag),
                                           _lib.ptr(out), _lib.ptr(incr)),
                   self._h)
        return float(out[0])

    def mbe3_backward(self, gamma, W, dE=1.0, mode=MBE3_GRAD_SLAB, out=None,
                      dEdF=None, probe=False):
        """dE * dE/d(slab) (mode MBE3_GRAD_SLAB, [n_occ, n_vir, n_aux]) or
        dE * dE/dGamma (MBE3_GRAD_GAMMA, gamma layout) into ``out``, and
        dE * dE/df_occ into ``dEdF`` when given.  Returns (out, probe) with
        probe = <dE dE/dGamma, Gamma> (host float) if requested.  Mode
        MBE3_GRAD_PROBE: ``out`` (gamma layout) receives the projected probe
        direction and probe = (dE <dE/dB, Delta>, dE <dE/dB, B>)."""
        import torch
        if out is None:
            shape = ((self.n_occ, self.n_vir, self.n_aux) if mode == MBE3_GRAD_SLAB
                     else (int(self.layout.gamma_elems),))
            out = torch.empty(shape, dtype=torch.float64, device=self.device)
        if mode == MBE3_GRAD_PROBE:
            probe = True
        pr = np.zeros(2, dtype=np.float64)
        _lib.check(_lib.load().mbe3_backward(
            self._h, float(dE), _lib.ptr(_f64(gamma)), _lib.ptr(_f64(W)),
            int(mode), _lib.ptr(_f64(out)), out.numel(),
            _lib.ptr(None if dEdF is None else _f64(dEdF)),
            _lib.ptr(pr) if probe else None), self._h)
        if mode == MBE3_GRAD_PROBE:
            return out, (float(pr[0]), float(pr[1]))
        return out, (float(pr[0]) if probe else None)

    def set_slab_shift(self, t):
        """osv_project regenerates B + t Delta from the next call on."""
        _lib.check(_lib.load().mbe3_set_slab_shift(self._h, float(t)), self._h)

    def mbe3_pair_basis(self):
        import torch
        X = torch.empty(int(self.x_off[-1]), dtype=torch.float64, device=self.device)
        et = torch.empty(int(self.e_off[-1]), dtype=torch.float64, device=self.device)
        rank = torch.empty(int(self.layout.n_slot), dtype=torch.int32, device=self.device)
        _lib.check(_lib.load().mbe3_pair_basis(self._h, _lib.ptr(X), _lib.ptr(et),
                                               _lib.ptr(rank)), self._h)
        return X, et, rank

    def screen(self, pairs):
        """s2b (eq. s2b) of each listed pair (host int array [n, 2]) as a
        float64 tensor on the device; screen_lists applies the paper's
        thresholds."""
        import torch
        pr = np.ascontiguousarray(np.asarray(pairs, dtype=np.int32).reshape(-1, 2))
        out = torch.empty(len(pr), dtype=torch.float64, device=self.device)
        _lib.check(_lib.load().mbe3_screen(self._h, _lib.ptr(pr), len(pr),
                                           _lib.ptr(out)), self._h)
        return out

    def screen_noalloc(self, pairs, out=None):
        """screen() through mbe3_screen_noalloc (no device allocation in the
        library; the caller passes the output tensor or one is made here)."""
        import torch
        pr = np.ascontiguousarray(np.asarray(pairs, dtype=np.int32).reshape(-1, 2))
        if out is None:
            out = torch.empty(len(pr), dtype=torch.float64, device=self.device)
        _lib.check(_lib.load().mbe3_screen_noalloc(self._h, _lib.ptr(pr), len(pr),
                                                   _lib.ptr(out)), self._h)
        return out

    def weak_pairs(self, pairs, gamma, W):
        """Energies of weak pairs (host int array [n, 2], i < j) from
        osv_project's gamma and fragment_solve's multipliers W (their
        diagonal slots are the MBE(3) diagonal amplitudes), as a float64
        tensor on the device."""
        import torch
        pr = np.ascontiguousarray(np.asarray(pairs, dtype=np.int32).reshape(-1, 2))
        e = torch.empty(len(pr), dtype=torch.float64, device=self.device)
        _lib.check(_lib.load().mbe3_weak_pairs(self._h, _lib.ptr(pr), len(pr),
                                               _lib.ptr(_f64(gamma)), _lib.ptr(_f64(W)),
                                               _lib.ptr(e)), self._h)
        return e

    def set_timing(self, enable=True):
        _lib.check(_lib.load().mbe3_set_timing(self._h, int(bool(enable))), self._h)

    def get_timing(self):
        """{phase: (ms, regions)} accumulated since set_timing."""
        ms = np.zeros(len(_lib.PHASES), dtype=np.float64)
        n = np.zeros(len(_lib.PHASES), dtype=np.int64)
        _lib.check(_lib.load().mbe3_get_timing(self._h, _lib.ptr(ms), _lib.ptr(n)), self._h)
        return {ph: (float(ms[k]), int(n[k])) for k, ph in enumerate(_lib.PHASES)}

    # ---- tile shapes of the grouped GEMMs ----
    def autotune(self, reps=3, dB=True, gamma=None, K=None):
        """Time every GEMM tile shape on every task list of this handle and
        keep the fastest; returns the report (one line per list).  gamma and
        K (layout-sized, contents overwritten) serve as the products'
        operands; new ones are made when not given, and a dB buffer when dB
        is True."""
        import torch
        if gamma is None:
            gamma = self.empty_gamma()
            gamma.zero_()
        if K is None:
            K = self.empty_K()
            K.zero_()
        d = None
        if dB:
            d = torch.zeros((self.n_occ, self.n_vir, self.n_aux), dtype=torch.float64,
                            device=self.device)
        torch.cuda.synchronize(self.device)
        lib = _lib.load()
        _lib.check(lib.mbe3_autotune(self._h, _lib.ptr(_f64(gamma)), gamma.numel(),
                                     _lib.ptr(_f64(K)), K.numel(), _lib.ptr(d),
                                     0 if d is None else d.numel(), int(reps)), self._h)
        return lib.mbe3_tune_report(self._h).decode()

    def set_gemm_shape(self, shape, list_index=-1):
        """Force one tile shape (index into _lib.GEMM_SHAPES, or its name)
        on one task list or (-1) on all."""
        if isinstance(shape, str):
            shape = _lib.GEMM_SHAPES.index(shape)
        _lib.check(_lib.load().mbe3_set_gemm_shape(self._h, int(list_index), int(shape)),
                   self._h)

    # ---- recorded launches (one HIP graph per handle) ----
    def fit_metric(self, out=None):
        """Sparse fitting metric (eq. sparse_fit_metric) of every LMO and
        auxiliary function, s_fit[i, P] = sum_a B_i[a, P]^2, as a float64
        [n_occ, n_aux] tensor on the device."""
        import torch
        if out is None:
            out = torch.empty((self.n_occ, self.n_aux), dtype=torch.float64,
                              device=self.device)
        _lib.check(_lib.load().mbe3_fit_metric(self._h, _lib.ptr(_f64(out))), self._h)
        return out

    def fit_mask(self, s_fit, l_fit, g):
        """Zero, in place, the elements of gamma-layout ``g`` outside the
        columns the fitting domains D = {s_fit > l_fit} select for its rows
        (block (i, x): D_i u D_x; block (i, i): the union of D_q over
        N+(i)); returns g."""
        _lib.check(_lib.load().mbe3_fit_mask(self._h, _lib.ptr(_f64(s_fit)),
                                             float(l_fit), _lib.ptr(_f64(g)),
                                             g.numel()), self._h)
        return g

    def project_fit(self, s_fit, l_fit, gamma):
        """osv_project over the fitting domains s_fit > l_fit only: the
        columns each row needs regenerated and projected (as fit_mask
        selects them), the others zero; returns gamma."""
        _lib.check(_lib.load().mbe3_project_fit(self._h, _lib.ptr(_f64(s_fit)),
                                                float(l_fit), _lib.ptr(_f64(gamma)),
                                                gamma.numel()), self._h)
        return gamma

    def pair_K_fit(self, s_fit, l_fit, K):
        """pair_K with every slot (p, q) summed over the union of the two
        fitting domains D_p u D_q (s_fit > l_fit; D_p for a diagonal slot),
        from the needed columns only (Gamma~ is not formed); returns K."""
        _lib.check(_lib.load().mbe3_pair_K_fit(self._h, _lib.ptr(_f64(s_fit)),
                                               float(l_fit), _lib.ptr(_f64(K)),
                                               K.numel()), self._h)
        return K

    def rosv(self, n_max=128, l_osv=1e-4, s_fit=None, l_fit=0.0):
        """Randomized OSVs of every LMO (mbe3_rosv): T_ii from the slab on
        the fitting domain s_fit > l_fit (all columns without s_fit), the
        adaptive range finder, the SVD and the cut at l_osv.  Returns dict
        Q [n_occ, n_max, n_vir] (rows = OSVs), w [n_occ, n_max], n_osv
        [n_occ], rows [n_occ] (device tensors)."""
        import torch
        dev = self.device
        Q = torch.empty((self.n_occ, n_max, self.n_vir), dtype=torch.float64, device=dev)
        w = torch.empty((self.n_occ, n_max), dtype=torch.float64, device=dev)
        k = torch.empty(self.n_occ, dtype=torch.int32, device=dev)
        rows = torch.empty(self.n_occ, dtype=torch.int32, device=dev)
        _lib.check(_lib.load().mbe3_rosv(
            self._h, _lib.ptr(None if s_fit is None else _f64(s_fit)), float(l_fit),
            float(l_osv), int(n_max), _lib.ptr(Q), _lib.ptr(w), _lib.ptr(k),
            _lib.ptr(rows)), self._h)
        return dict(Q=Q, w=w, n_osv=k, rows=rows)

    def first_order_dE(self, K_a, K_b, W, per_slot=None):
        """First-order energy change sum_s c_s <K_a,s - K_b,s, W_s> (c_s = 2
        diagonal, 4 pair slots) of moving K from K_b to K_a, W the
        multipliers of fragment_solve at K_b.  Returns (total, per-slot
        float64 tensor on the device)."""
        import torch
        if per_slot is None:
            per_slot = torch.empty(int(self.layout.n_slot), dtype=torch.float64,
                                   device=self.device)
        out = np.zeros(1, dtype=np.float64)
        _lib.check(_lib.load().mbe3_first_order_dE(
            self._h, _lib.ptr(_f64(K_a)), _lib.ptr(_f64(K_b)), _lib.ptr(_f64(W)),
            _lib.ptr(_f64(per_slot)), _lib.ptr(out)), self._h)
        return float(out[0]), per_slot

    def graph_begin(self, with_grad=False):
        _lib.check(_lib.load().mbe3_graph_begin(self._h, int(bool(with_grad))), self._h)

    def graph_end(self):
        _lib.check(_lib.load().mbe3_graph_end(self._h), self._h)

    def graph_launch(self):
        """Replay the recorded graph; returns the MBE(3) energy if the
        recording contained mbe3_energy, else None."""
        out = np.full(1, np.nan, dtype=np.float64)
        _lib.check(_lib.load().mbe3_graph_launch(self._h, _lib.ptr(out)), self._h)
        return None if np.isnan(out[0]) else float(out[0])

    def capture_step(self, grad=False, dB=None, dEdF=None):
        """Record one forward (osv_project -> pair_K -> fragment_solve ->
        mbe3_energy) and, with grad=True, the backward into dB
        (dE/d(ia|P), [n_occ, n_vir, n_aux], allocated if None) and dEdF.
        Returns the buffers the graph writes on every graph_launch()."""
        import torch
        gamma, K = self.empty_gamma(), self.empty_K()
        e = torch.empty(self.n_frag, dtype=torch.float64, device=self.device)
        it = torch.empty(self.n_frag, dtype=torch.int32, device=self.device)
        W = self.empty_K() if grad else None
        if grad and dB is None:
            dB = torch.empty((self.n_occ, self.n_vir, self.n_aux), dtype=torch.float64,
                             device=self.device)
        if grad and dEdF is None:
            dEdF = torch.empty((self.n_occ, self.n_occ), dtype=torch.float64,
                               device=self.device)
        torch.cuda.synchronize(self.device)  # the buffers exist before replays
        self.graph_begin(with_grad=grad)
        try:
            self.osv_project(gamma)
            self.pair_K(gamma, K)
            self.fragment_solve(K, e, it, W)
            self.mbe3_energy(e)
            if grad:
                self.mbe3_backward(gamma, W, dE=1.0, mode=MBE3_GRAD_SLAB, out=dB,
                                   dEdF=dEdF)
        finally:
            self.graph_end()
        return dict(gamma=gamma, K=K, e_frag=e, iters=it, W=W,
                    dB=dB if grad else None, dEdF=dEdF if grad else None)

    def forward(self, grad=False, l_fit=None):
        """osv_project -> pair_K -> fragment_solve -> mbe3_energy; with
        grad=True fragment_solve also returns the multipliers W.  With
        l_fit, the method over the sparse fitting domains s_fit > l_fit:
        mbe3_fit_metric -> mbe3_pair_K_fit (each pair over D_p u D_q) ->
        fragment_solve -> mbe3_energy (s_fit returned, no dense gamma)."""
        import torch
        s_fit = gamma = None
        if l_fit is None:
            gamma = self.osv_project(self.empty_gamma())
            K = self.pair_K(gamma, self.empty_K())
        else:
            s_fit = self.fit_metric()
            K = self.pair_K_fit(s_fit, l_fit, self.empty_K())
        e = torch.empty(self.n_frag, dtype=torch.float64, device=self.device)
        it = torch.empty(self.n_frag, dtype=torch.int32, device=self.device)
        W = self.empty_K() if grad else None
        self.fragment_solve(K, e, it, W)
        E = self.mbe3_energy(e)
        return dict(E=E, gamma=gamma, K=K, e_frag=e, iters=it, W=W, s_fit=s_fit)


def _energy_function():
    import torch

    class _Mbe3Energy(torch.autograd.Function):
        """E(slab, f_occ) with the library's forward and backward."""

        @staticmethod
        def forward(ctx, h, slab, f_occ):
            if h.slab is None or slab.data_ptr() != h.slab.data_ptr() or \
                    f_occ.data_ptr() != h.f_occ.data_ptr():
                raise ValueError("energy_fn: slab and f_occ must be the tensors "
                                 "the handle was created with")
            out = h.forward(grad=True)
            ctx.h = h
            ctx.saved = (out["gamma"], out["W"])
            return torch.tensor(out["E"], dtype=torch.float64, device=slab.device)

        @staticmethod
        def backward(ctx, gE):
            h = ctx.h
            gamma, W = ctx.saved
            dE = float(gE)
            dF = torch.empty((h.n_occ, h.n_occ), dtype=torch.float64, device=h.device)
            dB, _ = h.mbe3_backward(gamma, W, dE=dE, mode=MBE3_GRAD_SLAB, dEdF=dF)
            return None, dB, dF

    return _Mbe3Energy


_ENERGY_FN = None


def energy_fn(h, slab, f_occ):
    """Differentiable MBE(3)-OSV-MP2 energy (0-d float64 tensor) of the
    handle's problem.  ``slab`` ([n_occ, n_vir, n_aux]) and ``f_occ`` must be
    the tensors the handle was created with (the library reads them in
    place); their gradients come from mbe3_backward."""
    global _ENERGY_FN
    if _ENERGY_FN is None:
        _ENERGY_FN = _energy_function()
    return _ENERGY_FN.apply(h, slab, f_occ)


# sparse fitting threshold of the paper's sparsity table (eq. sparse_fit_metric)
L_FIT = 1e-6


L_LOC = 1e-3  # the paper's localization threshold


def pm_localize(C, ao_off, l_loc=L_LOC, max_sweeps=100, stream=None, check=True):
    """Pipek-Mezey localization with Jacobi sweeps (mbe3_pm_localize) of the
    orthonormalized MO coefficients C (float64 CUDA tensor [n_ao, n_occ])
    with the AOs of atom A at ao_off[A] .. ao_off[A+1]-1 (host ints).
    Returns dict(U [n_occ, n_occ], P [n_occ, n_occ, n_atom] (device), dL
    and rotations per sweep, sweeps, status)."""
    import torch
    lib = _lib.load()
    C = _f64(C)
    off = np.ascontiguousarray(ao_off, dtype=np.int32)
    n_ao, n_occ = int(C.shape[0]), int(C.shape[1])
    n_atom = len(off) - 1
    P = torch.empty((n_occ, n_occ, n_atom), dtype=torch.float64, device=C.device)
    U = torch.empty((n_occ, n_occ), dtype=torch.float64, device=C.device)
    dL = np.zeros(max(int(max_sweeps), 1), dtype=np.float64)
    rot = np.zeros(max(int(max_sweeps), 1), dtype=np.int32)
    ns = np.zeros(1, dtype=np.int32)
    if stream is None:
        stream = torch.cuda.current_stream(C.device)
    rc = lib.mbe3_pm_localize(_lib.ptr(C), _lib.ptr(off), n_ao, n_occ, n_atom, float(l_loc),
                              int(max_sweeps), _lib.ptr(P), _lib.ptr(U), _lib.ptr(dL),
                              _lib.ptr(rot), _lib.ptr(ns), ctypes.c_void_p(stream.cuda_stream))
    if check:
        _lib.check(rc, None)
    k = int(ns[0])
    return dict(U=U, P=P, dL=dL[:k].copy(), rotations=rot[:k].copy(), sweeps=k, status=rc)


S2B_DISTANT, S2B_CLOSE, S3B_KEEP = 1e-7, 1e-2, 0.2  # the paper's thresholds


def screen_lists(n_occ, pairs, s2b, t_distant=S2B_DISTANT, t_close=S2B_CLOSE,
                 t_trimer=S3B_KEEP):
    """Pair classes and kept trimers (mbe3_screen_lists) of candidate pairs
    (host [n, 2]) with metrics s2b (host [n]): dict with classes (int8 per
    pair: 0 distant, 1 weak, 2 close), close, weak ([m, 2], i < j) and
    trimers ([t, 3])."""
    lib = _lib.load()
    pr = np.ascontiguousarray(np.asarray(pairs, dtype=np.int32).reshape(-1, 2))
    sv = np.ascontiguousarray(np.asarray(s2b, dtype=np.float64).reshape(-1))
    n = len(pr)
    cls = np.zeros(n, dtype=np.int8)
    close = np.zeros((n, 2), dtype=np.int32)
    weak = np.zeros((n, 2), dtype=np.int32)
    nc, nw, nt = (np.zeros(1, dtype=np.int64) for _ in range(3))
    args = (int(n_occ), _lib.ptr(pr) if n else None, n, _lib.ptr(sv) if n else None,
            float(t_distant), float(t_close), float(t_trimer), _lib.ptr(cls),
            _lib.ptr(close), _lib.ptr(nc), _lib.ptr(weak), _lib.ptr(nw))
    _lib.check(lib.mbe3_screen_lists(*args, None, 0, _lib.ptr(nt)), None)
    tri = np.zeros((max(int(nt[0]), 1), 3), dtype=np.int32)
    _lib.check(lib.mbe3_screen_lists(*args, _lib.ptr(tri), len(tri), _lib.ptr(nt)), None)
    return dict(classes=cls, close=close[:int(nc[0])].copy(), weak=weak[:int(nw[0])].copy(),
                trimers=tri[:int(nt[0])].copy())


def osv_project(h, gamma):
    return h.osv_project(gamma)


def pair_K(h, gamma, K):
    return h.pair_K(gamma, K)


def fragment_solve(h, K, e_frag, iters, W=None):
    return h.fragment_solve(K, e_frag, iters, W)


def mbe3_energy(h, e_frag, incr=None):
    return h.mbe3_energy(e_frag, incr)


def mbe3_backward(h, gamma, W, dE=1.0, mode=MBE3_GRAD_SLAB, out=None,
                  dEdF=None, probe=False):
    return h.mbe3_backward(gamma, W, dE, mode, out, dEdF, probe)


def mbe3_pair_basis(h):
    return h.mbe3_pair_basis()


def from_problem(prob, device="cuda:0", **kw):
    """Build an Mbe3 handle from a seeded synthetic Problem (input marshalling)."""
    import torch
    dev = torch.device(device)
    t = lambda a: torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64), device=dev)
    args = dict(r=prob.r, Q=t(prob.QT_packed), eps_vir=t(prob.eps_vir),
                f_occ=t(prob.f_occ), pairs=prob.pairs, frags=prob.frags,
                seed=prob.seed, w_ia=t(prob.w_ia), w_iP=t(prob.w_iP),
                tol=prob.tol, max_iter=prob.max_iter, tau_S=prob.tau_S)
    args.update(kw)
    return Mbe3(**args)


def plan_check(*, r, pairs, frags, n_vir, n_aux, tol=1e-8, max_iter=100,
               tau_S=1e-8, explicit_slab=False, precision=MBE3_FP64,
               warm_start=True):
    """Build and bounds-check every execution plan without a device.

    Returns the layout; raises Mbe3Error with the library's message on
    invalid lists or a planner bug."""
    lib = _lib.load()
    r = np.ascontiguousarray(r, dtype=np.int32)
    pairs = np.ascontiguousarray(pairs, dtype=np.int32).reshape(-1, 2)
    frags = np.ascontiguousarray(frags, dtype=np.int32).reshape(-1, 3)
    fake = 0x1000  # never dereferenced by the planner
    p = _lib.Mbe3Problem()
    p.n_occ, p.n_vir, p.n_aux = len(r), int(n_vir), int(n_aux)
    p.r = _lib.ptr(r)
    p.Q = p.eps_vir = p.f_occ = fake
    p.w_ia = p.w_iP = None if explicit_slab else fake
    p.slab = fake if explicit_slab else None
    p.n_pair = len(pairs)
    p.pairs = _lib.ptr(pairs) if len(pairs) else None
    p.n_frag = len(frags)
    p.frags = _lib.ptr(frags)
    p.tol, p.max_iter, p.tau_S, p.precision = tol, max_iter, tau_S, int(precision)
    p.warm_start = int(bool(warm_start))
    lay = _lib.Mbe3Layout()
    rc = lib.mbe3_plan_check(ctypes.byref(p), ctypes.byref(lay))
    _lib.check(rc, None)
    return lay
