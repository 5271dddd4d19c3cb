"""Sparse fitting domains (mbe3_fit_metric, mbe3_fit_mask, mbe3_project_fit,
mbe3_pair_K_fit) through the C-ABI against the oracle (needs an MI355X): the
metric of every (i, P) of the 8-LMO chain and of sampled (i, P) of the
1024-LMO helix; Gamma~ as stored over the domains (block (i, x) on
D_i u D_x, the diagonal block on the union over N+(i)); pair integrals
summed over D_p u D_q; fragment and MBE(3) energies at a threshold that
splits the domains; the exact masking pattern; a recorded restriction
replayed; argument errors; the metric of a given slab array; the same
restricted integrals in the split-precision forms; sampled fragments of the
restricted 160-LMO lattice at full size; the projection over the domains
only (bit for bit the masked dense path) and pair_K over the unions, with
sampled slots and fragments of the helix against the oracle."""
import dataclasses
import sys

import numpy as np
import pytest

import _workloads
import oracle
import synth
from oracle import fit

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


def rel(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def split_threshold(s):
    """The midpoint between the two middle metrics: about half of the
    (i, P) leave their domains and no metric lies near the threshold."""
    v = np.sort(np.asarray(s).ravel())
    k = len(v) // 2
    return 0.5 * (v[k - 1] + v[k])


def gamma_block(h, prob, gamma, i, x):
    nb = prob.neighbours(i)
    row = int(h.g_off[i]) + int(sum(prob.r[y] for y in nb if y < x))
    return gamma.view(-1, prob.n_aux)[row:row + int(prob.r[x])].cpu().numpy()


def k_block(h, prob, K, s):
    off = int(h.k_off[s])
    p, q = (s, s) if s < prob.n_occ else tuple(prob.pairs[s - prob.n_occ])
    d = int(prob.r[p] + (prob.r[q] if p != q else 0))
    return K[off:off + d * d].view(d, d).cpu().numpy(), (int(p), int(q))


def row_blocks(h, prob):
    """(LMO i, block orbital x) of every gamma row."""
    rl = np.empty(int(h.g_off[-1]), dtype=np.int64)
    rx = np.empty_like(rl)
    for i in range(prob.n_occ):
        row = int(h.g_off[i])
        for x in prob.neighbours(i):
            rl[row:row + int(prob.r[x])] = i
            rx[row:row + int(prob.r[x])] = int(x)
            row += int(prob.r[x])
    return rl, rx


def keep_mask(h, prob, s, l_fit):
    """Columns kept in every gamma row by the union rule, from the metric
    (written out here: D_i u D_x, or the union over N+(i) for x = i)."""
    D = s > l_fit
    rl, rx = row_blocks(h, prob)
    C = np.stack([np.any(D[prob.neighbours(i)], axis=0) for i in range(prob.n_occ)])
    return np.where((rl == rx)[:, None], C[rl], D[rl] | D[rx])


def test_fit_metric_chain8(m):
    say("case: chain8, s_fit of all 8 x 192 (i, P) vs oracle")
    prob = synth.config(0)
    h = m.from_problem(prob)
    s = h.fit_metric().cpu().numpy()
    ref = fit.fit_metrics(oracle.Oracle(prob))
    r = float(np.max(np.abs(s - ref) / ref))
    say(f"  s_fit range {ref.min():.3e}..{ref.max():.3e}, max rel diff {r:.2e}")
    assert r <= 1e-13
    h.close()


def test_fit_restricted_chain8(m):
    """Gamma~ as stored over the domains, K over D_p u D_q and the energies at
    a threshold splitting the domains, both sides from T = 0 (the oracle's
    iterates)."""
    import torch
    say("case: chain8, restricted forward (split threshold) vs oracle")
    prob = synth.config(0)
    h = m.from_problem(prob, warm_start=False)
    base = oracle.Oracle(prob)
    s_ref = fit.fit_metrics(base)
    l_fit = split_threshold(s_ref)
    out = h.forward(l_fit=l_fit)
    torch.cuda.synchronize()
    s = out["s_fit"].cpu().numpy()
    gap = float(np.min(np.abs(s_ref - l_fit)) / l_fit)
    assert gap > 1e-10
    assert np.array_equal(s > l_fit, s_ref > l_fit)
    kept = float(np.mean(s_ref > l_fit))
    say(f"  l_fit {l_fit:.3e}, kept {kept:.3f}, nearest metric {gap:.1e} (relative) away")
    ora = fit.restricted_oracle(prob, l_fit, base=base, s_fit=s_ref)
    g = h.project_fit(out["s_fit"], l_fit, h.empty_gamma())
    for i in range(prob.n_occ):
        for x in prob.neighbours(i):
            gb = gamma_block(h, prob, g, i, int(x))
            r = ora.gamma_fit(i, int(x))
            assert np.array_equal(gb == 0.0, r == 0.0), (i, x)
            assert np.abs(gb - r).max() <= 1e-13 * np.abs(r).max(), (i, x)
    for sl in range(h.layout.n_slot):
        k, (p, q) = k_block(h, prob, out["K"], sl)
        r = ora.Kbar(p, q)
        assert np.abs(k - r).max() <= 1e-13 * np.abs(r).max(), sl
    ref = oracle.run(prob, ora=ora)
    E_ref, _ = oracle.mbe3_energy(prob.frags, ref["e_frag"])
    e = out["e_frag"].cpu().numpy()
    full = h.forward()
    say(f"  E restricted GPU {out['E']:.14f} oracle {E_ref:.14f}; "
        f"unrestricted {full['E']:.14f}")
    assert np.abs(e - ref["e_frag"]).max() <= 1e-12
    assert np.array_equal(out["iters"].cpu().numpy(), ref["iters"])
    assert abs(out["E"] - E_ref) <= 1e-10
    assert abs(out["E"] - full["E"]) > 1e-6 * abs(full["E"])
    h.close()


def test_fit_mask_pattern_and_errors(m):
    """The mask writes zeros exactly outside the domains and leaves every
    other element bit for bit; bad arguments are refused."""
    import torch
    say("case: chain8, mask pattern on random rows, argument errors")
    prob = synth.config(0)
    h = m.from_problem(prob)
    s = h.fit_metric()
    sn = s.cpu().numpy()
    l_fit = split_threshold(sn)
    g = torch.randn(int(h.layout.gamma_elems), dtype=torch.float64, device="cuda:0")
    g0 = g.cpu().numpy().reshape(-1, prob.n_aux)
    h.fit_mask(s, l_fit, g)
    keep = keep_mask(h, prob, sn, l_fit)
    assert 0.3 < keep.mean() < 1.0
    got = g.cpu().numpy().reshape(-1, prob.n_aux)
    assert np.array_equal(got, np.where(keep, g0, 0.0))
    # below every metric: nothing changes; above every metric: all zero
    g1 = torch.randn_like(g)
    ref1 = g1.clone()
    h.fit_mask(s, -1.0, g1)
    assert torch.equal(g1, ref1)
    h.fit_mask(s, float(sn.max()), g1)
    assert not torch.any(g1)
    for bad in (float("nan"),):
        with pytest.raises(m.Mbe3Error) as ei:
            h.fit_mask(s, bad, g)
        assert ei.value.code == m.MBE3_EINVAL
    with pytest.raises(m.Mbe3Error) as ei:
        h.fit_mask(s, l_fit, g[:-1])
    assert ei.value.code == m.MBE3_EINVAL
    lib = m._lib.load()
    assert lib.mbe3_fit_metric(h._h, None) == m.MBE3_EINVAL
    assert lib.mbe3_fit_mask(h._h, None, 0.0, m._lib.ptr(g), g.numel()) == m.MBE3_EINVAL
    # still usable
    assert torch.equal(h.fit_metric(), s)
    h.close()


def test_fit_recorded_replays(m):
    """osv_project, fit_metric and fit_mask recorded once and replayed three
    times, each replay equal bit for bit to the eager calls."""
    import torch
    say("case: chain8, recorded restriction replayed 3 times vs eager")
    prob = synth.config(0)
    h = m.from_problem(prob)
    s_e = h.fit_metric()
    l_fit = split_threshold(s_e.cpu().numpy())
    g_e = h.fit_mask(s_e, l_fit, h.osv_project(h.empty_gamma()))
    torch.cuda.synchronize()
    gamma = h.empty_gamma()
    s = torch.empty((prob.n_occ, prob.n_aux), dtype=torch.float64, device="cuda:0")
    torch.cuda.synchronize()
    h.graph_begin()
    try:
        h.osv_project(gamma)
        h.fit_metric(out=s)
        h.fit_mask(s, l_fit, gamma)
    finally:
        h.graph_end()
    for rep in range(3):
        gamma.fill_(1.0)
        s.zero_()
        torch.cuda.synchronize()
        h.graph_launch()
        torch.cuda.synchronize()
        assert torch.equal(s, s_e), rep
        assert torch.equal(gamma, g_e), rep
    h.close()


def test_fit_metric_helix1024_sampled(m):
    """Sampled (i, P) of the 1024-LMO helix against the oracle's slab
    columns, and the share of each domain kept at the paper's threshold."""
    import torch
    say("case: helix1024, s_fit at 24 sampled (i, P) vs oracle slab columns")
    prob = _workloads.config(4)
    h = m.from_problem(prob)
    s = h.fit_metric().cpu().numpy()
    torch.cuda.synchronize()
    rng = np.random.default_rng(5)
    worst = 0.0
    for _ in range(4):
        i = int(rng.integers(prob.n_occ))
        cols = np.sort(rng.choice(prob.n_aux, 6, replace=False))
        B = oracle.slab(prob, i, cols=cols)
        ref = np.sum(B * B, axis=0)
        worst = max(worst, float(np.max(np.abs(s[i, cols] - ref) / ref)))
    kept = float(np.mean(s > m.L_FIT))
    say(f"  max rel diff {worst:.2e}; kept at l_fit = 1e-6: {kept:.4f}")
    assert worst <= 1e-13
    assert 0.0 < kept < 0.1
    h.close()


def test_fit_metric_given_slab(m):
    """The metric read from a given slab array (no regeneration) against the
    oracle's metric of the same slabs, and the regenerated one."""
    import torch
    say("case: micro n_occ=4, s_fit from an explicit slab vs oracle and regenerated")
    prob = synth.micro(4)
    slab = np.stack([oracle.slab(prob, i) for i in range(prob.n_occ)])
    h = m.from_problem(prob, slab=torch.as_tensor(slab, device="cuda:0"),
                       w_ia=None, w_iP=None)
    s = h.fit_metric().cpu().numpy()
    ref = fit.fit_metrics(oracle.Oracle(prob, slabs={i: slab[i] for i in range(prob.n_occ)}))
    hr = m.from_problem(prob)
    sr = hr.fit_metric().cpu().numpy()
    r1 = float(np.max(np.abs(s - ref) / ref))
    r2 = float(np.max(np.abs(s - sr) / sr))
    say(f"  given vs oracle {r1:.2e}, given vs regenerated {r2:.2e}")
    assert r1 <= 1e-13 and r2 <= 1e-13
    h.close()
    hr.close()


@pytest.mark.parametrize("form", ["MBE3_MIXED_BF16", "MBE3_MIXED_BF16_PROJ"])
def test_fit_restricted_split_precision(m, form):
    """pair_K over the domains runs in FP64 in every precision mode: a
    split-precision handle returns bit for bit the FP64 handle's restricted
    integrals."""
    import torch
    say(f"case: chain8, pair_K over the domains on a {form} handle vs FP64")
    prob = synth.config(0)
    h64 = m.from_problem(prob)
    s = h64.fit_metric()
    l_fit = split_threshold(s.cpu().numpy())
    K64 = h64.pair_K_fit(s, l_fit, h64.empty_K())
    h = m.from_problem(prob, precision=getattr(m, form))
    K = h.pair_K_fit(s, l_fit, h.empty_K())
    torch.cuda.synchronize()
    assert torch.equal(K, K64)
    h.close()
    h64.close()


def test_fit_restricted_water40u_sampled(m):
    """The 160-LMO lattice in the benchmark's launch shape with the domains
    cut at l_fit = 5e-3 (about half of each kept): the metric and domain
    decisions of every LMO a sampled fragment touches, and the sampled
    fragments' restricted energies and update counts, one by one, against
    the oracle (both from T = 0)."""
    import torch
    say("case: water40u restricted forward (l_fit 5e-3), sampled oracle fragments")
    prob = synth.config(1)
    l_fit = 5e-3
    h = m.from_problem(prob, warm_start=False)
    out = h.forward(l_fit=l_fit)
    torch.cuda.synchronize()
    s = out["s_fit"].cpu().numpy()
    e = out["e_frag"].cpu().numpy()
    it = out["iters"].cpu().numpy()
    assert (it >= 0).all() and np.isfinite(e).all()
    kept = float(np.mean(s > l_fit))
    fr = prob.frags
    i0 = np.nonzero((fr == 0).any(1))[0]
    pick = np.unique(np.concatenate([i0[:6], i0[-6:], np.arange(0, len(fr), 19999),
                                     [len(fr) - 1]]))
    ora = fit.RestrictedOracle(prob, l_fit)
    res = oracle.run(prob, frags=fr[pick], ora=ora)
    worst_s, gap = 0.0, np.inf
    for i, si in ora.s.items():
        worst_s = max(worst_s, float(np.max(np.abs(s[i] - si) / si)))
        gap = min(gap, float(np.min(np.abs(si - l_fit)) / l_fit))
        assert np.array_equal(s[i] > l_fit, si > l_fit), i
    dE = float(np.abs(e[pick] - res["e_frag"]).max())
    say(f"  kept {kept:.3f}; {len(ora.s)} LMOs: s_fit rel {worst_s:.2e}, nearest metric "
        f"{gap:.1e} from l_fit; {len(pick)} fragments: max |dE_F| {dE:.3e}; E = {out['E']:.10f}")
    assert worst_s <= 1e-13 and gap > 1e-10
    assert 0.3 < kept < 0.7
    assert dE <= 1e-12
    assert np.array_equal(it[pick], res["iters"])
    h.close()


def test_project_fit_equals_project_then_mask(m):
    """mbe3_project_fit (only the kept columns regenerated and projected)
    against osv_project followed by mbe3_fit_mask, bit for bit, at a
    splitting threshold and at both limits; a given slab array too."""
    import torch
    say("case: chain8 / micro4 given slab, restricted projection vs project + mask")
    prob = synth.config(0)
    h = m.from_problem(prob)
    s = h.fit_metric()
    sn = s.cpu().numpy()
    for l_fit in (split_threshold(sn), -1.0, float(sn.max())):
        ref = h.fit_mask(s, l_fit, h.osv_project(h.empty_gamma()))
        got = h.project_fit(s, l_fit, h.empty_gamma())
        torch.cuda.synchronize()
        assert torch.equal(got, ref), l_fit
    h.close()
    p4 = synth.micro(4)
    slab = np.stack([oracle.slab(p4, i) for i in range(p4.n_occ)])
    h = m.from_problem(p4, slab=torch.as_tensor(slab, device="cuda:0"), w_ia=None, w_iP=None)
    s = h.fit_metric()
    l_fit = split_threshold(s.cpu().numpy())
    ref = h.fit_mask(s, l_fit, h.osv_project(h.empty_gamma()))
    got = h.project_fit(s, l_fit, h.empty_gamma())
    torch.cuda.synchronize()
    assert torch.equal(got, ref)
    with pytest.raises(m.Mbe3Error) as ei:
        h.project_fit(s, float("nan"), got)
    assert ei.value.code == m.MBE3_EINVAL
    h.close()


def test_project_fit_helix1024(m):
    """The 1024-LMO helix at the paper's l_fit = 1e-6 (about 2% of each
    domain kept): the restricted projection equals osv_project + mask bit
    for bit over all of Gamma~, and both are timed."""
    import time
    import torch
    say("case: helix1024, restricted projection at l_fit 1e-6 vs project + mask")
    prob = _workloads.config(4)
    h = m.from_problem(prob)
    s = h.fit_metric()
    g = h.empty_gamma()
    times = {}
    for name in ("dense", "restricted"):
        for _ in range(2):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            if name == "dense":
                h.osv_project(g)
            else:
                h.project_fit(s, m.L_FIT, g2)
            torch.cuda.synchronize()
            times[name] = time.perf_counter() - t0
        if name == "dense":
            h.fit_mask(s, m.L_FIT, g)
            g2 = h.empty_gamma()
    torch.cuda.synchronize()
    kept = float((s > m.L_FIT).double().mean())
    say(f"  kept {kept:.4f}; osv_project {times['dense'] * 1e3:.1f} ms, "
        f"restricted projection {times['restricted'] * 1e3:.1f} ms")
    assert torch.equal(g2, g)
    h.close()
    del g, g2
    torch.cuda.empty_cache()


def test_pair_K_fit_chain8(m):
    """pair_K over the unions D_p u D_q against the oracle's restricted K at a
    splitting threshold; below every metric it is the unrestricted pair_K,
    above every metric zero."""
    import torch
    say("case: chain8, pair_K over D_p u D_q vs oracle and the limits")
    prob = synth.config(0)
    h = m.from_problem(prob)
    s = h.fit_metric()
    sn = s.cpu().numpy()
    base = oracle.Oracle(prob)
    full = h.pair_K(h.osv_project(h.empty_gamma()), h.empty_K())
    got = h.pair_K_fit(s, -1.0, h.empty_K())
    torch.cuda.synchronize()
    d = float((got - full).abs().max()) / float(full.abs().max())
    say(f"  every column kept: max |K_fit - K| / max|K| = {d:.2e}")
    assert d <= 1e-13
    assert not torch.any(h.pair_K_fit(s, float(sn.max()), h.empty_K()))
    l_fit = split_threshold(sn)
    ora = fit.restricted_oracle(prob, l_fit, base=base, s_fit=fit.fit_metrics(base))
    K = h.pair_K_fit(s, l_fit, h.empty_K())
    worst = 0.0
    for sl in range(h.layout.n_slot):
        k, (p, q) = k_block(h, prob, K, sl)
        r = ora.Kbar(p, q)
        worst = max(worst, float(np.abs(k - r).max() / np.abs(r).max()))
    say(f"  split threshold: max rel diff to the oracle {worst:.2e}")
    assert worst <= 1e-13
    h.close()


def helix_sample_slots(prob):
    """Diagonal slots and pairs around LMOs 1, 2 and 500 of the helix."""
    n = prob.n_occ
    pr = [tuple(int(v) for v in pq) for pq in prob.pairs]
    want = [(1, 2), (1, 4), (500, 501), (499, 502)]
    slots = [1, 2, 500]
    for w in want:
        if w in pr:
            slots.append(n + pr.index(w))
    return slots


def test_pair_K_fit_helix1024(m):
    """The 1024-LMO helix at l_fit = 1e-6: pair_K over the unions
    (projection of the needed columns included) against the oracle on
    sampled slots, timed against the dense pair_K."""
    import time
    import torch
    say("case: helix1024, pair_K over the domain unions vs oracle slots")
    prob = _workloads.config(4)
    h = m.from_problem(prob)
    s = h.fit_metric()
    g = h.osv_project(h.empty_gamma())
    K_ref, K = h.empty_K(), h.empty_K()
    for _ in range(2):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        h.pair_K(g, K_ref)
        torch.cuda.synchronize()
        t_dense = time.perf_counter() - t0
    del g
    torch.cuda.empty_cache()
    for _ in range(2):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        h.pair_K_fit(s, m.L_FIT, K)
        torch.cuda.synchronize()
        t_fit = time.perf_counter() - t0
    ora = fit.RestrictedOracle(prob, m.L_FIT)
    worst = 0.0
    for sl in helix_sample_slots(prob):
        k, (p, q) = k_block(h, prob, K, sl)
        r = ora.Kbar(p, q)
        worst = max(worst, float(np.abs(k - r).max() / np.abs(r).max()))
    kept = [int(ora.dom(i).sum()) for i in ora.s]
    say(f"  dense pair_K {t_dense * 1e3:.1f} ms; projection + pair_K over the unions "
        f"{t_fit * 1e3:.1f} ms; domain sizes {kept}; sampled slots max rel diff {worst:.2e}")
    assert worst <= 1e-12
    h.close()


def test_fit_helix1024_restricted_energy(m):
    """End to end on the 1024-LMO helix at the paper's l_fit = 1e-6: the
    MBE(3) energy from pair_K over the unions D_p u D_q (Gamma~ never formed
    densely) next to the unrestricted energy, and every fragment containing
    the pair (1, 2) against the restricted oracle, one by one (both from
    T = 0)."""
    import time
    import torch
    say("case: helix1024, restricted MBE(3) energy (l_fit 1e-6), sampled oracle fragments")
    prob = _workloads.config(4)
    h = m.from_problem(prob, warm_start=False)
    e = torch.empty(prob.n_frag, dtype=torch.float64, device="cuda:0")
    it = torch.empty(prob.n_frag, dtype=torch.int32, device="cuda:0")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s = h.fit_metric()
    K = h.pair_K_fit(s, m.L_FIT, h.empty_K())
    h.fragment_solve(K, e, it)
    E_fit = h.mbe3_energy(e)
    t_fit = time.perf_counter() - t0
    t0 = time.perf_counter()
    out = h.forward()
    t_full = time.perf_counter() - t0
    rel = (E_fit - out["E"]) / abs(out["E"])
    say(f"  E restricted {E_fit:.10f} ({t_fit * 1e3:.0f} ms with the metric), "
        f"unrestricted {out['E']:.10f} ({t_full * 1e3:.0f} ms), relative change {rel:.2e}")
    assert np.isfinite(E_fit) and (it >= 0).all()
    fr = prob.frags
    idx = np.nonzero((fr == 1).any(1) & (fr == 2).any(1))[0]
    ora = fit.RestrictedOracle(prob, m.L_FIT)
    res = oracle.run(prob, frags=fr[idx], ora=ora)
    dE = np.abs(e.cpu().numpy()[idx] - res["e_frag"])
    say(f"  fragments {fr[idx].tolist()}: max |dE_F| vs restricted oracle {dE.max():.3e}")
    assert dE.max() <= 1e-12
    h.close()
    del out, K, s
    torch.cuda.empty_cache()
