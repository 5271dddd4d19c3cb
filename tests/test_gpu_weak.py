"""Pair screening (mbe3_screen) and weak pairs (mbe3_weak_pairs) through the
C-ABI against the oracle (needs an MI355X): s2b of every pair, weak-pair
energies with the MBE(3) diagonal amplitudes of each side's own solve, the
canonical-MP2 closed form for identity OSVs, sampled pairs beyond the
cutoff of the 160-LMO water lattice with seeded diagonal amplitudes shared
by both sides, and argument errors."""
import dataclasses
import sys

import numpy as np
import pytest

import _pins
import oracle
import synth
from oracle import weak

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def m():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    import paper_2603_16575_amd as pkg
    pkg._lib.load()
    return pkg


def all_pairs(n):
    return np.array([(i, j) for i in range(n) for j in range(i + 1, n)], dtype=np.int32)


def w_from_blocks(h, prob, blocks):
    """A K-layout W whose diagonal slots hold the given r_i x r_i blocks."""
    import torch
    W = np.zeros(int(h.k_off[-1]))
    for i, b in enumerate(blocks):
        W[h.k_off[i]:h.k_off[i + 1]] = np.asarray(b).ravel()
    return torch.as_tensor(W, device="cuda:0")


def test_screen_chain8(m):
    import torch
    say("case: chain8, s2b of all 28 pairs (both orders) vs oracle")
    prob = synth.config(0)
    h = m.from_problem(prob)
    ora = oracle.Oracle(prob)
    pr = all_pairs(prob.n_occ)
    both = np.concatenate([pr, pr[:, ::-1]], 0)
    s = h.screen(both).cpu().numpy()
    ref = np.array([weak.s2b(ora, int(i), int(j)) for i, j in both])
    rel = float(np.abs(s - ref).max() / np.abs(ref).max())
    say(f"  s2b range {ref.min():.3e}..{ref.max():.3e}, max rel diff {rel:.2e}")
    assert rel <= 1e-13
    h.close()


def test_weak_pairs_chain8_own_solves(m):
    """Every pair of chain8 as a weak pair: the GPU from its own solve's
    multipliers, the oracle from its own T^MBE_ii (both warm-started)."""
    import torch
    say("case: chain8, weak-pair energies of all pairs, each side's own T^MBE_ii")
    prob = dataclasses.replace(synth.config(0), tol=1e-11, max_iter=300)
    h = m.from_problem(prob)
    out = h.forward(grad=True)
    pr = all_pairs(prob.n_occ)
    e = h.weak_pairs(pr, out["gamma"], out["W"]).cpu().numpy()
    ref_run = oracle.run(prob, keep_T=True, warm_start=True)
    Td = weak.mbe3_diagonal_amplitudes(prob, ref_run)
    ref = weak.weak_energies(ref_run["oracle"], pr, Td)
    rel = float(np.abs(e - ref).max() / np.abs(ref).max())
    say(f"  E_weak(all pairs) GPU {e.sum():.12e} oracle {ref.sum():.12e}, max rel {rel:.2e}")
    assert rel <= 1e-9
    h.close()


def test_weak_pairs_identity_canonical(m):
    """Identity OSVs and a diagonal occupied Fock: e_ij = 4 sum K^2 / D, the
    direct part of canonical MP2 for the ordered pairs ij and ji."""
    import torch
    say("case: micro n_occ=3, identity OSVs, diagonal Fock: weak energies vs closed form")
    prob = synth.micro(3, identity_q=True, diagonal_f=True)
    h = m.from_problem(prob)
    gamma = h.osv_project(h.empty_gamma())
    W = torch.zeros(int(h.k_off[-1]), dtype=torch.float64, device="cuda:0")
    pr = all_pairs(prob.n_occ)
    e = h.weak_pairs(pr, gamma, W).cpu().numpy()
    ora = oracle.Oracle(prob)
    B = [ora.B(i) for i in range(prob.n_occ)]
    fd = np.diag(prob.f_occ)
    for k, (i, j) in enumerate(pr):
        K = _pins.full_K(B, i, j)
        D = fd[i] + fd[j] - prob.eps_vir[:, None] - prob.eps_vir[None, :]
        closed = 4.0 * np.sum(K * K / D)
        say(f"  pair ({i},{j}): {e[k]!r} closed form {closed!r}")
        assert abs(e[k] - closed) <= 1e-12 * abs(closed)
    h.close()


def lattice_sample(prob, n_lmo=8):
    """LMOs around LMO 0 and every pair among them that the cutoff dropped."""
    d = np.sqrt(((prob.x_occ - prob.x_occ[0]) ** 2).sum(1))
    near = [0] + [int(x) for x in np.argsort(d)[1:] if 6.0 < d[x] < 11.0][:n_lmo - 1]
    kept = {(int(a), int(b)) for a, b in prob.pairs}
    pr = [(min(a, b), max(a, b)) for k, a in enumerate(near) for b in near[k + 1:]]
    return np.array([p for p in pr if p not in kept], dtype=np.int32)


def test_weak_pairs_water40u_sampled(m):
    """Pairs beyond the cutoff among 8 LMOs of the 160-LMO lattice, in the
    full-size handle: s2b and weak energies with seeded diagonal amplitudes
    given to both sides."""
    import torch
    say("case: water40u, pairs beyond the cutoff among 8 LMOs, seeded T_ii")
    prob = synth.config(1)
    pr = lattice_sample(prob)
    assert len(pr) >= 10
    h = m.from_problem(prob)
    s = h.screen(pr).cpu().numpy()
    Td = synth.diagonal_amplitudes(prob)
    gamma = h.osv_project(h.empty_gamma())
    e = h.weak_pairs(pr, gamma, w_from_blocks(h, prob, Td)).cpu().numpy()
    torch.cuda.synchronize()
    ora = oracle.Oracle(prob)
    s_ref = np.array([weak.s2b(ora, int(i), int(j)) for i, j in pr])
    e_ref = np.array([weak.weak_pair(ora, int(i), int(j), Td[i], Td[j])[1] for i, j in pr])
    rs = float(np.abs(s - s_ref).max() / np.abs(s_ref).max())
    re = float(np.abs(e - e_ref).max() / np.abs(e_ref).max())
    cls = m.screen_lists(prob.n_occ, pr, s)["classes"]
    say(f"  {len(pr)} pairs, classes {np.bincount(cls, minlength=3).tolist()}, "
        f"s2b rel {rs:.2e}, e rel {re:.2e}, sum e {e.sum():.6e}")
    assert rs <= 1e-13 and re <= 1e-11
    h.close()
    del gamma
    torch.cuda.empty_cache()


def test_weak_and_screen_errors(m):
    import torch
    say("case: micro n_occ=3, bad pairs and empty lists")
    prob = synth.micro(3)
    h = m.from_problem(prob)
    gamma = h.osv_project(h.empty_gamma())
    W = torch.zeros(int(h.k_off[-1]), dtype=torch.float64, device="cuda:0")
    for bad in ([[1, 1]], [[2, 1]], [[0, 3]], [[-1, 2]]):
        with pytest.raises(m.Mbe3Error) as ei:
            h.weak_pairs(np.array(bad), gamma, W)
        assert ei.value.code == m.MBE3_EINVAL
    for bad in ([[1, 1]], [[0, 3]]):
        with pytest.raises(m.Mbe3Error) as ei:
            h.screen(np.array(bad))
        assert ei.value.code == m.MBE3_EINVAL
    assert h.screen(np.zeros((0, 2))).numel() == 0
    assert h.weak_pairs(np.zeros((0, 2)), gamma, W).numel() == 0
    # still usable
    assert h.screen(np.array([[2, 0]])).cpu().numpy()[0] > 0
    h.close()


def test_weak_and_screen_refused_while_recording(m):
    """Both calls allocate, so a recording refuses them (MBE3_EINVAL) and
    the handle stays usable eagerly afterwards."""
    import torch
    say("case: micro n_occ=3, screening and weak pairs while recording")
    prob = dataclasses.replace(synth.micro(3), tol=1e-10, max_iter=300)
    h = m.from_problem(prob)
    out = h.forward(grad=True)
    pr = all_pairs(prob.n_occ)
    e_ref = h.weak_pairs(pr, out["gamma"], out["W"]).cpu().numpy()
    torch.cuda.synchronize()
    h.graph_begin(with_grad=False)
    with pytest.raises(m.Mbe3Error) as ei:
        h.screen(pr)
    assert ei.value.code == m.MBE3_EINVAL
    with pytest.raises(m.Mbe3Error) as ei:
        h.weak_pairs(pr, out["gamma"], out["W"])
    assert ei.value.code == m.MBE3_EINVAL
    with pytest.raises(m.Mbe3Error):
        h.graph_end()  # the recording saw an error
    e = h.weak_pairs(pr, out["gamma"], out["W"]).cpu().numpy()
    assert np.array_equal(e, e_ref)
    h.close()


def test_water40u_paper_classes(m):
    """The 160-LMO lattice screened the paper's way instead of by distance:
    s2b of all 12720 pairs on the GPU (mbe3_screen), classes and trimers
    (mbe3_screen_lists) equal to the oracle's brute-force screening of its
    own s2b; close pairs and the kept trimers solved as fragments, weak
    pairs through mbe3_weak_pairs with the MBE(3) diagonal amplitudes of
    that solve.  Against the oracle: every fragment containing LMO 0 and
    every 97th fragment one by one, and the weak-pair energies of pairs
    among a few LMOs, each side from its own T^MBE_ii (both from T = 0)."""
    import torch
    say("case: water40u with the paper's s2b / s3b screening, sampled vs oracle")
    prob = synth.config(1)
    n = prob.n_occ
    cand = all_pairs(n)
    mono = np.full((n, 3), -1, dtype=np.int32)
    mono[:, 0] = np.arange(n)
    h0 = m.from_problem(prob, pairs=np.zeros((0, 2), dtype=np.int32), frags=mono)
    s = h0.screen(cand).cpu().numpy()
    h0.close()
    lists = m.screen_lists(n, cand, s)
    ora = oracle.Oracle(prob)
    s_ref = np.array([weak.s2b(ora, int(i), int(j)) for i, j in cand])
    rs = float(np.abs(s - s_ref).max() / np.abs(s_ref).max())
    # no metric within rounding of a class threshold or of the trimer mean
    gap = min(float(np.min(np.abs(s_ref - t) / t)) for t in (m.S2B_DISTANT, m.S2B_CLOSE))
    close, wk, tris = weak.screened_lists(n, {(int(i), int(j)): v for (i, j), v in zip(cand, s_ref)})
    say(f"  s2b rel {rs:.2e}, nearest class threshold {gap:.1e} away; close {len(close)}, "
        f"weak {len(wk)}, trimers {len(tris)} (oracle {len(lists['close'])}, "
        f"{len(lists['weak'])}, {len(lists['trimers'])} on the GPU)")
    assert rs <= 1e-13 and gap > 1e-10
    assert [tuple(x) for x in lists["close"].tolist()] == close
    assert [tuple(x) for x in lists["weak"].tolist()] == wk
    assert [tuple(x) for x in lists["trimers"].tolist()] == tris
    prob2 = dataclasses.replace(prob, pairs=lists["close"], trimers=lists["trimers"])
    h = m.from_problem(prob2, warm_start=False)
    out = h.forward(grad=True)
    e = out["e_frag"].cpu().numpy()
    it = out["iters"].cpu().numpy()
    assert (it >= 0).all() and np.isfinite(e).all()
    fr = prob2.frags
    pick = np.unique(np.concatenate([np.nonzero((fr == 0).any(1))[0],
                                     np.arange(0, len(fr), 97)]))
    ora2 = oracle.Oracle(prob2)
    res = oracle.run(prob2, frags=fr[pick], ora=ora2)
    dE = float(np.abs(e[pick] - res["e_frag"]).max())
    say(f"  {len(fr)} fragments, E_MBE(3) = {out['E']:.10f}; {len(pick)} sampled: "
        f"max |dE_F| {dE:.3e}")
    assert dE <= 1e-12
    assert np.array_equal(it[pick], res["iters"])
    # weak pairs among a few LMOs: T^MBE_ii from every fragment containing i
    wl = lists["weak"]
    sel = wl[(wl[:, 0] == 0) | (wl[:, 0] == 1)][:4]
    S = sorted(set(int(v) for v in sel.ravel()))
    ew = h.weak_pairs(sel, out["gamma"], out["W"]).cpu().numpy()
    coef = oracle.mbe3_coefficients(n, fr)
    fidx = np.nonzero(np.isin(fr, S).any(1))[0]
    rT = oracle.run(prob2, frags=fr[fidx], ora=ora2, keep_T=True)
    Td = {i: 0.0 for i in S}
    for f, cF, T in zip(fr[fidx], coef[fidx], rT["T"]):
        for x in (int(v) for v in f if v >= 0):
            if x in Td:
                Td[x] = Td[x] + cF * T[(x, x)]
    ew_ref = weak.weak_energies(ora2, sel, Td)
    rw = float(np.abs(ew - ew_ref).max() / np.abs(ew_ref).max())
    E_weak_all = float(h.weak_pairs(wl, out["gamma"], out["W"]).sum())
    say(f"  weak pairs {sel.tolist()}: rel diff {rw:.2e}; all {len(wl)} weak pairs "
        f"E_weak = {E_weak_all:.10f}, E_MBE(3) + E_weak = {out['E'] + E_weak_all:.10f}")
    assert rw <= 1e-9
    h.close()
    del out
    torch.cuda.empty_cache()
