"""HIP path vs the CPU oracle, through the C-ABI (needs an MI355X)."""
import dataclasses
import sys

import numpy as np
import pytest

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


def gamma_block(h, prob, gamma, i, x):
    nb = prob.neighbours(i)
    row = int(h.g_off[i]) + int(sum(prob.r[y] for y in nb if y < x))
    g = gamma.view(-1, prob.n_aux)
    return g[row:row + int(prob.r[x])].cpu().numpy()


def k_block(h, prob, K, s):
    off = int(h.k_off[s])
    p, q = (s, s) if s < prob.n_occ else tuple(prob.pairs[s - prob.n_occ])
    d = int(prob.r[p] + (prob.r[q] if p != q else 0))
    return K[off:off + d * d].view(d, d).cpu().numpy(), (int(p), int(q))


def run_all(m, prob, **kw):
    import torch
    h = m.from_problem(prob, **kw)
    out = h.forward()
    torch.cuda.synchronize()
    return h, out


def test_chain8_end_to_end(m):
    say("case: chain8 full forward vs oracle (T = 0 starts)")
    prob = synth.config(0)
    h, out = run_all(m, prob, warm_start=False)
    ref = oracle.run(prob)
    ora = ref["oracle"]
    E_ref, _ = oracle.mbe3_energy(prob.frags, ref["e_frag"])
    # O2: every projected block
    for i in range(prob.n_occ):
        for x in prob.neighbours(i):
            g = gamma_block(h, prob, out["gamma"], i, int(x))
            r = ora.gamma(i, int(x))
            assert np.abs(g - r).max() <= 1e-13 * np.abs(r).max(), (i, x)
    # O3: every pair K
    for s in range(h.layout.n_slot):
        k, (p, q) = k_block(h, prob, out["K"], s)
        r = ora.Kbar(p, q)
        assert np.abs(k - r).max() <= 1e-13 * np.abs(r).max(), s
    e = out["e_frag"].cpu().numpy()
    it = out["iters"].cpu().numpy()
    say(f"chain8: E_gpu={out['E']:.16f} E_ref={E_ref:.16f} dE={out['E'] - E_ref:.3e}")
    assert np.abs(e - ref["e_frag"]).max() <= 1e-12
    assert np.array_equal(it, ref["iters"])
    assert abs(out["E"] - E_ref) <= 1e-10
    h.close()


def test_pair_basis_gauge_invariants(m):
    say("case: chain8 pair bases (eq. prec_eig) vs oracle S, F")
    prob = synth.config(0)
    h = m.from_problem(prob)
    X, et, rank = h.mbe3_pair_basis()
    X, et, rank = X.cpu().numpy(), et.cpu().numpy(), rank.cpu().numpy()
    ora = oracle.Oracle(prob)
    for s in range(h.layout.n_slot):
        p, q = (s, s) if s < prob.n_occ else tuple(int(v) for v in prob.pairs[s - prob.n_occ])
        o = oracle.orbs(p, q)
        S, F = ora.Sblk(o, o), ora.Fblk(o, o)
        d = S.shape[0]
        D = (d + 15) // 16 * 16
        Xs = X[h.x_off[s]:h.x_off[s + 1]].reshape(d, D)[:, :rank[s]]
        es = et[h.e_off[s]:h.e_off[s] + rank[s]]
        Xr, er = ora.basis(p, q)
        assert rank[s] == Xr.shape[1]
        assert np.allclose(Xs.T @ S @ Xs, np.eye(rank[s]), atol=1e-12)
        assert np.allclose(Xs.T @ F @ Xs, np.diag(es), atol=1e-12)
        assert np.allclose(es, er, rtol=0, atol=1e-12)
        # projector onto the pair space, gauge free
        assert np.allclose(Xs @ Xs.T, Xr @ Xr.T, atol=1e-10)
    h.close()


def test_slab_regeneration_ulps(m):
    """Identity OSVs make the projection return the slab itself (each output
    is one product with an exact 1), so the regenerated slab is compared to
    the oracle's element by element."""
    say("case: slab regeneration, identity OSVs, n_vir=64 n_aux=192")
    cfg = dict(synth.CONFIGS[0])
    prob = synth.build(cfg, synth.SEED_BASE, identity_q=True, diagonal_f=True)
    prob = dataclasses.replace(prob, pairs=prob.pairs[:0], trimers=prob.trimers[:0])
    import torch
    h = m.from_problem(prob)
    g = h.osv_project(h.empty_gamma())
    torch.cuda.synchronize()
    g = g.view(prob.n_occ, prob.n_vir, prob.n_aux).cpu().numpy()
    worst = 0
    for i in range(prob.n_occ):
        ref = oracle.slab(prob, i)
        ulp = np.abs(g[i] - ref) / np.spacing(np.abs(ref))
        worst = max(worst, float(ulp.max()))
    say(f"slab: max ulp difference {worst}")
    assert worst <= 4
    h.close()


@pytest.mark.parametrize("n_occ", [3, 4])
def test_micro_strong_coupling(m, n_occ):
    say(f"case: micro n_occ={n_occ} strong coupling, all fragments")
    prob = dataclasses.replace(strong(synth.micro(n_occ)), tol=1e-12, max_iter=300)
    h, out = run_all(m, prob, warm_start=False)
    ref = oracle.run(prob)
    e = out["e_frag"].cpu().numpy()
    assert np.abs(e - ref["e_frag"]).max() <= 1e-13
    E_ref, _ = oracle.mbe3_energy(prob.frags, ref["e_frag"])
    assert abs(out["E"] - E_ref) <= 1e-12
    h.close()


def test_explicit_slab_matches_regenerated(m):
    say("case: explicit slab input == regenerated slab, micro n_occ=4")
    import torch
    prob = strong(synth.micro(4))
    slab = np.stack([oracle.slab(prob, i) for i in range(prob.n_occ)])
    h1, out1 = run_all(m, prob)
    h2, out2 = run_all(m, prob, slab=torch.as_tensor(slab, device="cuda:0"),
                       w_ia=None, w_iP=None)
    e1, e2 = out1["e_frag"].cpu().numpy(), out2["e_frag"].cpu().numpy()
    assert np.abs(e1 - e2).max() <= 1e-14
    h1.close()
    h2.close()


def test_water40u_sampled(m):
    """water40u (160 LMOs, 89969 fragments) in the benchmark's launch shape:
    fragment energies of a deterministic sample against the oracle, one by
    one; projected blocks and K of sampled orbitals/pairs."""
    say("case: water40u full forward, sampled oracle fragments")
    prob = synth.config(1)
    h, out = run_all(m, prob, warm_start=False)  # the oracle's iterates
    e = out["e_frag"].cpu().numpy()
    it = out["iters"].cpu().numpy()
    assert (it >= 0).all() and np.isfinite(e).all()
    fr = prob.frags
    pick = np.unique(np.concatenate([
        np.nonzero((fr == 0).any(1))[0][:40],
        np.arange(0, len(fr), 4999),
        [len(fr) - 1]]))
    ora = oracle.Oracle(prob)
    for i, x in [(0, 0), (0, int(prob.neighbours(0)[-1])), (77, 77)]:
        g = gamma_block(h, prob, out["gamma"], i, x)
        r = ora.gamma(i, x)
        assert np.abs(g - r).max() <= 1e-13 * np.abs(r).max()
    for s in [0, prob.n_occ, prob.n_occ + 2000, h.layout.n_slot - 1]:
        k, (p, q) = k_block(h, prob, out["K"], s)
        r = ora.Kbar(p, q)
        assert np.abs(k - r).max() <= 1e-13 * np.abs(r).max()
    res = oracle.run(prob, frags=fr[pick], ora=ora)
    say(f"water40u: {len(pick)} sampled fragments, max |dE_F| = "
        f"{np.abs(e[pick] - res['e_frag']).max():.3e}, E = {out['E']:.12f}")
    assert np.abs(e[pick] - res["e_frag"]).max() <= 1e-12
    assert np.array_equal(it[pick], res["iters"])
    h.close()


def test_failure_modes(m):
    import torch
    say("case: failure modes (no convergence, non-finite Fock, bad lists)")
    prob = dataclasses.replace(synth.config(0), max_iter=1)
    h = m.from_problem(prob)
    gamma = h.osv_project(h.empty_gamma())
    K = h.pair_K(gamma, h.empty_K())
    e = torch.empty(h.n_frag, dtype=torch.float64, device="cuda:0")
    it = torch.empty(h.n_frag, dtype=torch.int32, device="cuda:0")
    rc = h.fragment_solve(K, e, it, check=False)
    assert rc == m.MBE3_ENOCONV
    itn = it.cpu().numpy()
    assert (itn[:prob.n_occ] == 1).all() and (itn < 0).any()
    h.close()
    f = synth.config(0).f_occ.copy()
    f[2, 3] = f[3, 2] = np.nan
    prob = dataclasses.replace(synth.config(0), f_occ=f)
    h = m.from_problem(prob)
    gamma = h.osv_project(h.empty_gamma())
    K = h.pair_K(gamma, h.empty_K())
    rc = h.fragment_solve(K, e, it, check=False)
    assert rc == m.MBE3_ENONFINITE
    assert np.isnan(e.cpu().numpy()).any()
    h.close()
    p = synth.config(0)
    with pytest.raises(m.Mbe3Error) as ex:
        m.from_problem(dataclasses.replace(p, pairs=p.pairs[1:]))
    assert ex.value.code == m.MBE3_EINVAL


def test_deterministic(m):
    say("case: chain8 twice, bitwise equal")
    prob = synth.config(0)
    _, o1 = run_all(m, prob)
    _, o2 = run_all(m, prob)
    assert o1["E"] == o2["E"]
    assert np.array_equal(o1["e_frag"].cpu().numpy(), o2["e_frag"].cpu().numpy())


def test_water40u_total_vs_golden(m):
    """Full water40u (160 LMOs): E against the oracle's full run (written by
    tests/golden/make_golden.py, oracle only), |dE| <= 1e-10 Eh; the update
    count histogram and every 1000th fragment energy as well."""
    import json
    import os
    say("case: water40u total energy vs golden oracle run")
    g = json.load(open(os.path.join(os.path.dirname(__file__), "golden",
                                    "water40u_oracle.json")))
    prob = synth.config(1)
    h, out = run_all(m, prob, warm_start=False)
    E_ref = float(g["E_total"])
    say(f"water40u: E_gpu={out['E']:.13f} E_oracle={E_ref:.13f} "
        f"dE={out['E'] - E_ref:.3e}")
    assert abs(out["E"] - E_ref) <= 1e-10
    it = out["iters"].cpu().numpy()
    assert np.bincount(it).tolist() == g["iters_hist"]
    e = out["e_frag"].cpu().numpy()
    idx = np.array(g["sample_index"])
    ref = np.array([float(x) for x in g["sample_e_frag"]])
    assert np.abs(e[idx] - ref).max() <= 1e-12
    h.close()


def test_warm_start_water40u(m):
    """Trimers started from their monomer/dimer solutions converge to the same
    energies in fewer updates than from T = 0.  Both stop at max|R~| < 1e-7;
    the Hylleraas error of a stopping point is second order in the residual
    and of one sign, so over 84k trimers the two totals may differ by a few
    1e-9 Eh (each fragment by ~1e-12)."""
    say("case: water40u warm vs T = 0 starts")
    prob = synth.config(1)
    hc, oc = run_all(m, prob, warm_start=False)
    ec, ic = oc["e_frag"].cpu().numpy(), oc["iters"].cpu().numpy()
    Ec = oc["E"]
    hc.close()
    hw, ow = run_all(m, prob)
    ew, iw = ow["e_frag"].cpu().numpy(), ow["iters"].cpu().numpy()
    hw.close()
    tri = prob.frags[:, 2] >= 0
    say(f"warm: dE = {ow['E'] - Ec:.3e}, max |dE_F| = {np.abs(ew - ec).max():.3e}, "
        f"trimer updates {ic[tri].mean():.3f} -> {iw[tri].mean():.3f}")
    # monomers and dimers start from T = 0 either way (their chunks may use a
    # different kernel instance, so only rounding may differ)
    assert np.abs(ew[~tri] - ec[~tri]).max() <= 1e-14 and np.array_equal(iw[~tri], ic[~tri])
    assert np.abs(ew - ec).max() <= 1e-11
    assert abs(ow["E"] - Ec) <= 2e-8
    assert iw[tri].mean() < ic[tri].mean()


def test_water40u_warm_vs_golden(m):
    """Full water40u (160 LMOs) as the benchmark runs it (trimers warm started)
    against the oracle's full run with the same starts (written by
    tests/golden/make_golden.py --warm): |dE| <= 1e-10 Eh, the update-count
    histogram, and every 1000th fragment energy."""
    import json
    import os
    say("case: water40u warm-started total vs golden oracle run")
    g = json.load(open(os.path.join(os.path.dirname(__file__), "golden",
                                    "water40u_oracle_warm.json")))
    prob = synth.config(1)
    h, out = run_all(m, prob)
    E_ref = float(g["E_total"])
    say(f"water40u warm: E_gpu={out['E']:.13f} E_oracle={E_ref:.13f} "
        f"dE={out['E'] - E_ref:.3e}")
    assert abs(out["E"] - E_ref) <= 1e-10
    it = out["iters"].cpu().numpy()
    assert np.bincount(it).tolist() == g["iters_hist"]
    e = out["e_frag"].cpu().numpy()
    idx = np.array(g["sample_index"])
    ref = np.array([float(x) for x in g["sample_e_frag"]])
    assert np.abs(e[idx] - ref).max() <= 1e-12
    h.close()
