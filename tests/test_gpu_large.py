"""Wide pair domains (the eight-wave LDS solver up to 128, the streamed
solver and the global-workspace eigensolver above): a small oracle-checked
problem with D up to 160, and the large configurations 2 (D <= 128, 470k
fragments) and 4 (D <= 160) on the GPU with sampled checks (needs an
MI355X)."""
import dataclasses
import json
import os
import sys

import numpy as np
import pytest

import _workloads
import oracle
import synth

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


def strong(p, scale=8.0):
    f = p.f_occ.copy()
    off = ~np.eye(p.n_occ, dtype=bool)
    f[off] *= scale
    return dataclasses.replace(p, f_occ=f)


def big_micro():
    """4 LMOs with 56-80 OSVs each: pair dimensions 112-160, diagonal 64-80."""
    p = synth.micro(4, n_vir=192, n_aux=48, r=(56, 80))
    return dataclasses.replace(strong(p), tol=1e-11, max_iter=300)


def test_large_pairs_energy_vs_oracle(m):
    say("case: micro n_occ=4, r 56-80 (D up to 160), strong coupling, vs oracle")
    prob = big_micro()
    d = np.concatenate([prob.r, prob.r[prob.pairs[:, 0]] + prob.r[prob.pairs[:, 1]]])
    say(f"pair dims {sorted(set(int(x) for x in d))}")
    assert d.max() > 96
    h = m.from_problem(prob, warm_start=False)
    out = h.forward()
    ref = oracle.run(prob)
    e = out["e_frag"].cpu().numpy()
    E_ref, _ = oracle.mbe3_energy(prob.frags, ref["e_frag"])
    say(f"max |dE_F| = {np.abs(e - ref['e_frag']).max():.3e}, dE = {out['E'] - E_ref:.3e}")
    assert np.abs(e - ref["e_frag"]).max() <= 1e-12
    assert np.array_equal(out["iters"].cpu().numpy(), ref["iters"])
    assert abs(out["E"] - E_ref) <= 1e-11
    # pair bases of the large slots (global-workspace eigensolver)
    X, et, rank = h.mbe3_pair_basis()
    X, et, rank = X.cpu().numpy(), et.cpu().numpy(), rank.cpu().numpy()
    ora = ref["oracle"]
    for s in range(h.layout.n_slot):
        p, q = (s, s) if s < prob.n_occ else tuple(int(v) for v in prob.pairs[s - prob.n_occ])
        o = oracle.orbs(p, q)
        S, F = ora.Sblk(o, o), ora.Fblk(o, o)
        dd = S.shape[0]
        D = (dd + 15) // 16 * 16
        Xs = X[h.x_off[s]:h.x_off[s + 1]].reshape(dd, D)[:, :rank[s]]
        es = et[h.e_off[s]:h.e_off[s] + rank[s]]
        assert np.allclose(Xs.T @ S @ Xs, np.eye(rank[s]), atol=1e-11)
        assert np.allclose(Xs.T @ F @ Xs, np.diag(es), atol=1e-11)
    h.close()


def mid_micro():
    """4 LMOs with 50-64 OSVs each: pair dimensions 100-128 (the eight-wave
    LDS solver), diagonal 50-64."""
    p = synth.micro(4, n_vir=192, n_aux=48, r=(50, 64))
    return dataclasses.replace(strong(p), tol=1e-11, max_iter=300)


def test_mid_pairs_energy_and_gradient_vs_oracle(m):
    """Pair dimensions 100-128 (padded 112 / 128): energies, update counts
    and the gradient (solve, store and gradient-pass instances) against the
    oracle."""
    import torch
    say("case: micro n_occ=4, r 50-64 (D 112-128), strong coupling, vs oracle")
    prob = mid_micro()
    d = prob.r[prob.pairs[:, 0]] + prob.r[prob.pairs[:, 1]]
    say(f"pair dims {sorted(set(int(x) for x in d))}")
    assert 96 < d.max() <= 128
    h = m.from_problem(prob, warm_start=False)
    out = h.forward()
    ref = oracle.run(prob)
    e = out["e_frag"].cpu().numpy()
    say(f"max |dE_F| = {np.abs(e - ref['e_frag']).max():.3e}")
    assert np.abs(e - ref["e_frag"]).max() <= 1e-12
    assert np.array_equal(out["iters"].cpu().numpy(), ref["iters"])
    out = h.forward(grad=True)
    dF = torch.empty((prob.n_occ, prob.n_occ), dtype=torch.float64, device="cuda:0")
    dB, _ = h.mbe3_backward(out["gamma"], out["W"], dEdF=dF)
    g = oracle.gradient(prob)
    dBn = dB.cpu().numpy()
    rb = max(float(np.abs(dBn[i] - g["dB"][i]).max() / np.abs(g["dB"][i]).max())
             for i in range(prob.n_occ))
    rf = float(np.abs(dF.cpu().numpy() - g["df"]).max() / np.abs(g["df"]).max())
    say(f"dB rel {rb:.2e}, df rel {rf:.2e}")
    assert rb <= 1e-10 and rf <= 1e-10
    h.close()


def test_large_pairs_backward_vs_oracle(m):
    import torch
    say("case: micro n_occ=4, r 56-80, backward vs oracle.gradient")
    prob = big_micro()
    h = m.from_problem(prob, warm_start=False)  # the oracle's iterates
    out = h.forward(grad=True)
    dF = torch.empty((prob.n_occ, prob.n_occ), dtype=torch.float64, device="cuda:0")
    dB, _ = h.mbe3_backward(out["gamma"], out["W"], dEdF=dF)
    g = oracle.gradient(prob)
    dBn = dB.cpu().numpy()
    rb = max(float(np.abs(dBn[i] - g["dB"][i]).max() / np.abs(g["dB"][i]).max())
             for i in range(prob.n_occ))
    rf = float(np.abs(dF.cpu().numpy() - g["df"]).max() / np.abs(g["df"]).max())
    say(f"dB rel {rb:.2e}, df rel {rf:.2e}")
    assert rb <= 1e-10 and rf <= 1e-10
    h.close()


def test_large_pairs_mixed(m):
    say("case: micro n_occ=4, r 56-80, split precision vs oracle energy")
    prob = big_micro()
    h = m.from_problem(prob, precision=m.MBE3_MIXED_BF16)
    out = h.forward()
    ref = oracle.run(prob)
    E_ref, _ = oracle.mbe3_energy(prob.frags, ref["e_frag"])
    say(f"mixed dE = {out['E'] - E_ref:.3e} (E = {E_ref:.6f})")
    assert abs(out["E"] - E_ref) <= 1e-7 * abs(E_ref)
    h.close()


def gamma_block(h, prob, gamma, i, x):
    nb = [int(y) for y in prob.neighbours(i)]
    row = int(h.g_off[i]) + sum(int(prob.r[y]) for y in nb if y < x)
    g = gamma.view(-1, prob.n_aux)
    return g[row:row + int(prob.r[x])]


def test_water128u_sampled(m):
    """water128u (512 LMOs, n_vir 2432, n_aux 7040, D up to 128, 470k
    fragments) in full on the GPU: every fragment converged and finite, and
    the fragments of one trimer with a 128-wide pair (with its dimers and
    monomers) against the oracle, one by one; its projected blocks too; and
    the stored oracle sample of 5915 fragments (every 97th and every one
    containing LMO 0) with their update counts, and sampled K-bar elements
    of eight slots."""
    import torch
    say("case: water128u full forward, sampled oracle trimer")
    prob = synth.config(2)
    h = m.from_problem(prob, warm_start=False)  # the oracle's iterates
    out = h.forward()
    e = out["e_frag"].cpu().numpy()
    it = out["iters"].cpu().numpy()
    say(f"water128u: E = {out['E']:.10f}, iterations {np.bincount(it).tolist()}")
    assert (it >= 0).all() and np.isfinite(e).all()
    r = prob.r
    fr = prob.frags
    tri = fr[fr[:, 2] >= 0]
    dmaxs = np.maximum.reduce([r[tri[:, 0]] + r[tri[:, 1]], r[tri[:, 0]] + r[tri[:, 2]],
                               r[tri[:, 1]] + r[tri[:, 2]]])
    t = tri[int(np.argmax(dmaxs))]
    say(f"sample trimer {t.tolist()}, largest pair dimension {int(dmaxs.max())}")
    i, j, k = (int(v) for v in t)
    sub = [(i, -1, -1), (j, -1, -1), (k, -1, -1), (i, j, -1), (i, k, -1), (j, k, -1), (i, j, k)]
    idx = [int(np.nonzero((fr == np.array(f)).all(1))[0][0]) for f in sub]
    ora = oracle.Oracle(prob)
    for a in (i, j):
        for x in (i, j, k):
            got = gamma_block(h, prob, out["gamma"], a, x).cpu().numpy()
            ref = ora.gamma(a, x)
            assert np.abs(got - ref).max() <= 1e-13 * np.abs(ref).max()
    res = oracle.run(prob, frags=fr[idx], ora=ora)
    dE = np.abs(e[idx] - res["e_frag"])
    say(f"sampled fragments: max |dE_F| = {dE.max():.3e}")
    assert dE.max() <= 1e-12
    # the stored oracle sample (tests/golden/make_golden_water128u.py, oracle
    # only): every 97th fragment and every fragment containing LMO 0, from
    # T = 0, with their update counts, and 16 seeded elements and the norm
    # of eight K-bar slots
    g = json.load(open(os.path.join(os.path.dirname(__file__), "golden",
                                    "water128u_sample_oracle.json")))
    assert g["n_frag"] == prob.n_frag and g["converged"]
    sidx = np.asarray(g["sample_index"])
    ref_e = np.array([float(v) for v in g["e_frag"]])
    d_e = np.abs(e[sidx] - ref_e)
    same_it = it[sidx] == np.asarray(g["iters"])
    say(f"golden sample: {len(sidx)} fragments, max |dE_F| = {d_e.max():.3e}, "
        f"update counts equal {int(same_it.sum())}/{len(sidx)}, "
        f"sum dE = {float(np.sum(e[sidx]) - np.sum(ref_e)):.3e}")
    assert d_e.max() <= 1e-12
    assert same_it.all()
    slot = {(int(a), int(b)): prob.n_occ + k for k, (a, b) in enumerate(prob.pairs)}
    for ks in g["k_slots"]:
        p_, q_ = ks["p"], ks["q"]
        sidx_k = p_ if p_ == q_ else slot[(p_, q_)]
        blk = out["K"][int(h.k_off[sidx_k]):int(h.k_off[sidx_k + 1])].cpu().numpy()
        assert blk.size == ks["d"] ** 2
        fro = float(ks["frobenius"])
        got = blk[np.asarray(ks["flat_index"])]
        want = np.array([float(v) for v in ks["values"]])
        assert np.abs(got - want).max() <= 1e-13 * fro, (p_, q_)
        assert abs(float(np.linalg.norm(blk)) - fro) <= 1e-13 * fro, (p_, q_)
    h.close()
    del out
    torch.cuda.empty_cache()


def helix_problem():
    """configuration 4 (1024-LMO helix), built once per test process."""
    return _workloads.config(4)


def overlap_eigs(prob, s):
    """Eigenvalues of the pair overlap S_(pq,pq) of slot s (host, ascending),
    written from the OSVs directly (eq. 4block_osv)."""
    n = prob.n_occ
    p, q = (s, s) if s < n else (int(prob.pairs[s - n][0]), int(prob.pairs[s - n][1]))
    V = prob.Q[p] if p == q else np.concatenate([prob.Q[p], prob.Q[q]], 1)
    return np.linalg.eigvalsh(V.T @ V)


def test_helix1024_rank_and_sampled_fragments(m):
    """helix1024 OSV spaces of neighbouring LMOs nearly coincide (pair-overlap
    eigenvalues down to 1e-13), so the rank rule of the overlap step decides
    which pair space each side solves in.  Every slot's kept rank on the GPU
    must equal the number of overlap eigenvalues above tau_S (the oracle's
    canonical orthogonalisation); then the fragments around the slots with
    the smallest overlap eigenvalues and the one nearest tau_S, and every
    fragment containing the pair (1, 2), one by one against the oracle."""
    import torch
    say("case: helix1024 overlap ranks of every slot, sampled fragments vs oracle")
    prob = helix_problem()
    n = prob.n_occ
    h = m.from_problem(prob, warm_start=False)  # the oracle's iterates
    out = h.forward()
    _, _, rank = h.mbe3_pair_basis()
    rank = rank.cpu().numpy()
    e = out["e_frag"].cpu().numpy()
    it = out["iters"].cpu().numpy()
    assert (it >= 0).all() and np.isfinite(e).all()
    n_slot = int(h.layout.n_slot)
    lam_min = np.empty(n_slot)
    gap = np.empty(n_slot)
    want = np.empty(n_slot, dtype=np.int64)
    for s in range(n_slot):
        ev = overlap_eigs(prob, s)
        lam_min[s] = ev[0]
        gap[s] = np.min(np.abs(ev - prob.tau_S)) / prob.tau_S
        want[s] = int((ev > prob.tau_S).sum())
    full = np.array([prob.r[s] if s < n else prob.r[prob.pairs[s - n][0]] + prob.r[prob.pairs[s - n][1]]
                     for s in range(n_slot)])
    bad = np.nonzero(rank != want)[0]
    say(f"helix1024: {n_slot} slots, {int((want < full).sum())} rank deficient, "
        f"min lambda {lam_min.min():.2e}, nearest |lambda - tau|/tau {gap.min():.2e}, "
        f"rank mismatches {len(bad)} {bad[:8].tolist()}")
    assert len(bad) == 0
    # sampled fragments
    fr = prob.frags
    pick = set()
    tight = [int(s) for s in np.argsort(lam_min)[:2]] + [int(np.argmin(gap))]
    slot_pairs = [(s, s) if s < n else tuple(int(v) for v in prob.pairs[s - n]) for s in tight]
    slot_pairs.append((1, 2))
    for (p, q) in slot_pairs:
        has = (fr == p).any(1) & (fr == q).any(1)
        if p == q:
            has &= fr[:, 1] < 0  # the monomer only
        rows = np.nonzero(has)[0]
        pick.update(int(x) for x in rows[:3] if (p, q) != (1, 2))
        if (p, q) == (1, 2):
            pick.update(int(x) for x in rows)
    idx = np.array(sorted(pick))
    say(f"sampled slots {slot_pairs}, {len(idx)} fragments: {fr[idx].tolist()}")
    res = oracle.run(prob, frags=fr[idx])
    dE = np.abs(e[idx] - res["e_frag"])
    say(f"helix1024 sampled fragments: max |dE_F| = {dE.max():.3e}, "
        f"iterations GPU {it[idx].tolist()} oracle {res['iters'].tolist()}")
    assert dE.max() <= 1e-12
    h.close()
    del out
    torch.cuda.empty_cache()


def test_helix1024_forward_and_gradient(m):
    """helix1024 (1024 LMOs, n_vir 4096, n_aux 12288, D up to 160), FP64:
    every fragment converged and finite; projected blocks of the two LMOs
    with the most OSVs against the oracle on a subset of auxiliary columns;
    the gradient in the compressed (Gamma) layout, since a dense dE/d(ia|P)
    would take 412 GB: Euler probe <dE/dGamma, Gamma> = 4 E, the probe
    mode's <dE/dB, Delta> against a central difference of the GPU energy
    along the regenerated direction Delta, and dE/df_xy
    against a central difference of the GPU energy (h = 1e-4: the difference
    E(+h) - E(-h) is ~6e-9 Eh against ~1e-14 Eh of rounding in E)."""
    import torch
    say("case: helix1024 forward and backward, FP64, tol 1e-10")
    # converged tighter than the workload's 1e-7: the stationarity argument
    # leaves a first-order error of the size of the residual, which is 1e-5
    # of these small f derivatives at tol 1e-7
    prob = dataclasses.replace(helix_problem(), tol=1e-10)
    f = torch.as_tensor(prob.f_occ.copy(), device="cuda:0")
    h = m.from_problem(prob, f_occ=f)
    out = h.forward(grad=True)
    it = out["iters"].cpu().numpy()
    E = out["E"]
    say(f"helix1024: E = {E:.10f}, iterations {np.bincount(it).tolist()}")
    assert (it >= 0).all() and np.isfinite(out["e_frag"].cpu().numpy()).all()
    cols = np.arange(0, prob.n_aux, 97)
    ora = oracle.Oracle(prob)
    for i in np.argsort(prob.r)[-2:]:
        i = int(i)
        B = oracle.slab(prob, i, cols=cols)
        for x in prob.neighbours(i):
            x = int(x)
            got = gamma_block(h, prob, out["gamma"], i, x)[:, cols].cpu().numpy()
            ref = ora.Q[x].T @ B
            assert np.abs(got - ref).max() <= 1e-13 * np.abs(ref).max()
    dF = torch.empty_like(f)
    dG, probe = h.mbe3_backward(out["gamma"], out["W"], mode=m.MBE3_GRAD_GAMMA,
                                dEdF=dF, probe=True)
    say(f"helix1024: probe / 4E - 1 = {probe / (4 * E) - 1:.3e}")
    assert abs(probe / (4.0 * E) - 1.0) <= 1e-4
    # directional derivative along the probe direction Delta (dG as the
    # workspace for Q^T Delta), against a fourth-order central difference of
    # the GPU energy with the slabs regenerated as B + s Delta
    _, (pr_d, pr_e) = h.mbe3_backward(out["gamma"], out["W"], mode=m.MBE3_GRAD_PROBE,
                                      out=dG)
    assert pr_e == probe
    x, y = (int(v) for v in prob.pairs[len(prob.pairs) // 2])
    an = 2.0 * float(dF[x, y])
    del out, dG
    torch.cuda.empty_cache()
    t = 1e-4
    Ed = {}
    for k in (1, -1, 2, -2):
        h.set_slab_shift(k * t)
        Ed[k] = h.forward()["E"]
    h.set_slab_shift(0.0)
    fd_d = (8.0 * (Ed[1] - Ed[-1]) - (Ed[2] - Ed[-2])) / (12.0 * t)
    say(f"helix1024: <dE/dB, Delta> probe {pr_d:.10e} fd {fd_d:.10e} "
        f"rel {abs(fd_d - pr_d) / abs(pr_d):.2e}")
    assert abs(fd_d - pr_d) <= 1e-6 * abs(pr_d)
    step = 1e-4
    Es = []
    for sgn in (+1, -1):
        ff = prob.f_occ.copy()
        ff[x, y] += sgn * step
        ff[y, x] += sgn * step
        f.copy_(torch.as_tensor(ff, device="cuda:0"))
        Es.append(h.forward()["E"])
    fd = (Es[0] - Es[1]) / (2 * step)
    say(f"helix1024: dE/df_{x}{y} fd {fd:.10e} analytic {an:.10e}")
    assert abs(fd - an) <= 1e-5 * max(abs(an), 1e-8)
    h.close()


def test_water128u_mixed_vs_fp64(m):
    """Both split-precision forms on water128u (512 LMOs, 470k fragments): total
    and per-fragment deviation from the FP64 GPU path, which the test above
    ties to the oracle on sampled fragments.  Budget 1e-6 Eh on the total."""
    import torch
    say("case: water128u in split precision vs FP64 path")
    prob = synth.config(2)
    h = m.from_problem(prob)
    out = h.forward()
    E64, e64 = out["E"], out["e_frag"].cpu().numpy()
    h.close()
    del out, h
    torch.cuda.empty_cache()
    for form in ("MBE3_MIXED_BF16", "MBE3_MIXED_BF16_PROJ"):
        h = m.from_problem(prob, precision=getattr(m, form))
        out = h.forward()
        Em, em = out["E"], out["e_frag"].cpu().numpy()
        h.close()
        del out, h
        torch.cuda.empty_cache()
        d = np.abs(em - e64)
        say(f"water128u {form}: E = {Em:.10f} (FP64 {E64:.10f}), "
            f"|dE| = {abs(Em - E64):.3e}, max |dE_F| = {d.max():.3e}, mean {d.mean():.3e}")
        assert np.isfinite(em).all()
        assert abs(Em - E64) <= 1e-6
