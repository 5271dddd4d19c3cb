"""Split-precision projection and pair_K (MBE3_MIXED_BF16, and
MBE3_MIXED_BF16_PROJ with its FP64 pair_K) against the FP64 oracle, through
the C-ABI (needs an MI355X).

Error model of one projection product c = sum_k a_k b_k: each operand
carries 24 significant bits (three relative bf16 pieces), the dropped cross
products are below 3 * 2^-24 of |a_k b_k|, and the FP32 accumulation of K
terms adds at most K * 2^-24 of sum |a_k b_k| (worst case, one rounding per
step).  The tests bound |c_mixed - c| by (K + 8) * 2^-24 * sum_k |a_k| |b_k|
element by element and require the typical error (RMS over elements,
relative to the same scale) to be far below it.

The split pair_K carries each row of gamma on a fixed-point grid of the
row, so an element is off by at most 2^-23 of its row's largest magnitude,
and every block sum of one product class is exact; with all nine products
kept, |K_mixed - K| <= 2^-23 (max|L_p| sum_P |R_qP| + max|R_q| sum_P |L_pP|)
plus the FP32 rounding of the correction sums, below 2^-24 of
sum_P |L_pP| |R_qP|."""
import dataclasses
import json
import os
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


def gamma_rows_of(h, prob, gamma, i):
    g = gamma.view(-1, prob.n_aux)
    return g[int(h.g_off[i]):int(h.g_off[i + 1])].cpu().numpy()


def check_products(m, prob, prec):
    import torch
    h = m.from_problem(prob, precision=prec)
    gamma = h.osv_project(h.empty_gamma())
    torch.cuda.synchronize()
    ora = oracle.Oracle(prob)
    eps = 2.0 ** -24
    worst = 0.0
    rms = []
    for i in range(prob.n_occ):
        nb = [int(x) for x in prob.neighbours(i)]
        Qn = np.concatenate([ora.Q[x] for x in nb], 1)        # n_vir x rows
        B = ora.B(i)
        ref = Qn.T @ B
        scale = np.abs(Qn).T @ np.abs(B)
        err = np.abs(gamma_rows_of(h, prob, gamma, i) - ref)
        worst = max(worst, float((err / scale).max()))
        rms.append(float(np.sqrt(np.mean((err / scale) ** 2))))
    bound = (prob.n_vir + 8) * eps
    say(f"projection: worst err/scale {worst:.3e}, rms {max(rms):.3e}, bound {bound:.3e}")
    assert worst <= bound
    assert max(rms) <= 8 * eps
    # pair_K from the oracle's own FP64 projection (isolates the K product)
    g64 = np.zeros(int(h.layout.gamma_elems))
    gv = g64.reshape(-1, prob.n_aux)
    for i in range(prob.n_occ):
        nb = [int(x) for x in prob.neighbours(i)]
        gv[int(h.g_off[i]):int(h.g_off[i + 1])] = np.concatenate([ora.gamma(i, x) for x in nb], 0)
    K = h.pair_K(torch.as_tensor(g64, device="cuda:0"), h.empty_K())
    torch.cuda.synchronize()
    Kn = K.cpu().numpy()
    worst_k = 0.0
    for s in range(h.layout.n_slot):
        p, q = (s, s) if s < prob.n_occ else tuple(int(v) for v in prob.pairs[s - prob.n_occ])
        o = oracle.orbs(p, q)
        L = np.concatenate([ora.gamma(p, x) for x in o], 0)
        R = np.concatenate([ora.gamma(q, x) for x in o], 0)
        d = L.shape[0]
        got = Kn[h.k_off[s]:h.k_off[s] + d * d].reshape(d, d)
        scale = np.abs(L) @ np.abs(R).T
        if prec == m.MBE3_MIXED_BF16:
            grid = (np.abs(L).max(1)[:, None] * np.abs(R).sum(1)[None, :]
                    + np.abs(L).sum(1)[:, None] * np.abs(R).max(1)[None, :])
            bound = 2.0 ** -23 * grid + eps * scale
        else:  # FP64 pair_K
            bound = (prob.n_aux + 8) * 2.0 ** -53 * scale
        worst_k = max(worst_k, float((np.abs(got - L @ R.T) / bound).max()))
    say(f"pair_K: worst err / bound {worst_k:.3e}")
    assert worst_k <= 1.0
    h.close()


FORMS = ["MBE3_MIXED_BF16", "MBE3_MIXED_BF16_PROJ"]


@pytest.mark.parametrize("form", FORMS)
def test_mixed_products_chain8(m, form):
    say(f"case: chain8 {form} projection and pair_K vs oracle")
    check_products(m, synth.config(0), getattr(m, form))


@pytest.mark.parametrize("form", FORMS)
def test_mixed_products_padded_sizes(m, form):
    """n_vir, n_aux not multiples of 8: zero-padded plane rows."""
    say(f"case: micro n_occ=4, n_vir=21, n_aux=35, {form} products vs oracle")
    check_products(m, synth.micro(4, n_vir=21, n_aux=35), getattr(m, form))


def test_mixed_explicit_slab_equals_regenerated(m):
    import torch
    say("case: micro n_occ=4 mixed, explicit slab == regenerated")
    prob = synth.micro(4)
    slab = np.stack([oracle.slab(prob, i) for i in range(prob.n_occ)])
    h1 = m.from_problem(prob, precision=m.MBE3_MIXED_BF16)
    h2 = m.from_problem(prob, precision=m.MBE3_MIXED_BF16,
                        slab=torch.as_tensor(slab, device="cuda:0"), w_ia=None, w_iP=None)
    g1 = h1.osv_project(h1.empty_gamma())
    g2 = h2.osv_project(h2.empty_gamma())
    torch.cuda.synchronize()
    assert torch.equal(g1, g2)
    h1.close()
    h2.close()


@pytest.mark.parametrize("form", FORMS)
def test_mixed_energy_micro(m, form):
    say(f"case: micro n_occ=4 {form} energy vs oracle")
    prob = dataclasses.replace(synth.micro(4), tol=1e-12, max_iter=300)
    h = m.from_problem(prob, precision=getattr(m, form))
    out = h.forward()
    ref = oracle.run(prob)
    E_ref, _ = oracle.mbe3_energy(prob.frags, ref["e_frag"])
    say(f"micro mixed: dE = {out['E'] - E_ref:.3e} (E = {E_ref:.6f})")
    assert abs(out["E"] - E_ref) <= 1e-7 * abs(E_ref)
    h.close()


@pytest.mark.parametrize("form", FORMS)
def test_mixed_energy_water40u(m, form):
    """water40u (160 LMOs) in the benchmark's launch shape: the mixed total energy
    against the oracle's full run (|dE| <= 1e-6 Eh, the budget of the mixed
    form), and per-fragment deviations from the FP64 GPU path."""
    import torch
    say(f"case: water40u {form} vs golden oracle and FP64 path")
    g = json.load(open(os.path.join(os.path.dirname(__file__), "golden",
                                    "water40u_oracle.json")))
    E_ref = float(g["E_total"])
    prob = synth.config(1)
    hm = m.from_problem(prob, precision=getattr(m, form))
    om = hm.forward()
    E_m = om["E"]
    em = om["e_frag"].cpu().numpy()
    Km = om["K"].cpu().numpy()
    hm.close()
    del om, hm
    torch.cuda.empty_cache()
    hf = m.from_problem(prob)
    of = hf.forward(grad=True)
    ef = of["e_frag"].cpu().numpy()
    est, per = hf.first_order_dE(torch.as_tensor(Km, device="cuda:0"), of["K"], of["W"])
    per = per.cpu().numpy()
    E_f = of["E"]
    hf.close()
    d = np.abs(em - ef)
    top = np.argsort(-np.abs(per))[:3]
    say(f"water40u {form}: E = {E_m:.12f}, |E - E_oracle| = {abs(E_m - E_ref):.3e}, "
        f"max |dE_F| vs FP64 = {d.max():.3e}, mean {d.mean():.3e}")
    say(f"  E - E_fp64 = {E_m - E_f:.4e}, first-order estimate {est:.4e}; "
        f"largest slots {top.tolist()}: {per[top].tolist()}")
    assert abs(E_m - E_ref) <= 1e-6
    # E depends on the split products only through K-bar: the estimate
    # holds to second order (and the solver's stopping threshold)
    assert abs(est - (E_m - E_f)) <= 0.05 * abs(E_m - E_f) + 1e-9
    assert d.max() <= 1e-7


def test_first_order_dE_matches_finite_difference(m):
    """mbe3_first_order_dE with the oracle's multipliers W reproduces the
    central difference of the oracle's MBE(3) energy along a random change
    of every K-bar block (diagonal slots, kept symmetric, and pairs): this
    fixes the slot weights 2 and 4 and the packing of the K layout."""
    import torch
    say("case: micro n_occ=4, first-order dE vs oracle central difference")
    prob = dataclasses.replace(synth.micro(4), tol=1e-13, max_iter=400)
    g = oracle.gradient(prob)
    ora0 = g["run"]["oracle"]
    h = m.from_problem(prob)
    n = prob.n_occ
    slots = [(p, p) for p in range(n)] + [tuple(int(v) for v in pq) for pq in prob.pairs]
    k_off = h.k_off
    d = [int(round(np.sqrt(k_off[s + 1] - k_off[s]))) for s in range(len(slots))]
    rng = np.random.default_rng(3)
    K0 = np.concatenate([ora0.Kbar(p, q).ravel() for p, q in slots])
    dK = rng.standard_normal(K0.shape) * np.abs(K0).max()
    for s in range(n):  # K-bar_pp = G G^T stays symmetric
        blk = dK[k_off[s]:k_off[s + 1]].reshape(d[s], d[s])
        dK[k_off[s]:k_off[s + 1]] = (0.5 * (blk + blk.T)).ravel()
    W = np.concatenate([g["W"][s].ravel() for s in slots])

    def energy_at(eps):
        ora = oracle.Oracle(prob)
        for s, (p, q) in enumerate(slots):
            ora._K[(p, q)] = (K0 + eps * dK)[k_off[s]:k_off[s + 1]].reshape(d[s], d[s])
        return oracle.energy(prob, ora=ora)

    step = 1e-5
    fd = (energy_at(step) - energy_at(-step)) / (2 * step)
    t = lambda a: torch.as_tensor(np.ascontiguousarray(a), device="cuda:0")
    est, per = h.first_order_dE(t(K0 + dK), t(K0), t(W))
    per = per.cpu().numpy()
    say(f"  first-order {est:.12e}, central difference {fd:.12e}")
    assert per.shape == (len(slots),)
    assert abs(per.sum() - est) <= 1e-13 * abs(est)
    assert abs(est - fd) <= 1e-7 * abs(fd)
    mask = np.zeros_like(dK)
    mask[:k_off[n]] = 1.0
    e_diag, _ = h.first_order_dE(t(K0 + mask * dK), t(K0), t(W))
    assert abs(e_diag - 2.0 * float(np.sum((mask * dK) * W))) <= 1e-12 * abs(e_diag)
    with pytest.raises(m.Mbe3Error) as ei:
        m._lib.check(m._lib.load().mbe3_first_order_dE(h._h, None, None, None, None, None),
                     h._h)
    assert ei.value.code == m.MBE3_EINVAL
    h.close()
