"""mbe3_backward and fragment_solve's multipliers against the CPU oracle's
gradient (Hylleraas stationarity), through the C-ABI (needs an MI355X)."""
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


def slot_pq(prob, s):
    return (s, s) if s < prob.n_occ else tuple(int(v) for v in prob.pairs[s - prob.n_occ])


def w_block(h, prob, W, s):
    p, q = slot_pq(prob, s)
    d = int(prob.r[p] + (prob.r[q] if p != q else 0))
    off = int(h.k_off[s])
    return W[off:off + d * d].view(d, d).cpu().numpy()


def rel(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def check_vs_oracle(m, prob, tol_rel):
    import torch
    h = m.from_problem(prob, warm_start=False)  # the oracle's iterates
    out = h.forward(grad=True)
    dF = torch.empty((prob.n_occ, prob.n_occ), dtype=torch.float64, device="cuda:0")
    dB, probe = h.mbe3_backward(out["gamma"], out["W"], dEdF=dF, probe=True)
    dG, probe_g = h.mbe3_backward(out["gamma"], out["W"], mode=m.MBE3_GRAD_GAMMA,
                                  probe=True)
    torch.cuda.synchronize()
    g = oracle.gradient(prob)
    ora = g["run"]["oracle"]
    worst_w = max(rel(w_block(h, prob, out["W"], s), g["W"][slot_pq(prob, s)])
                  for s in range(h.layout.n_slot))
    dBn = dB.cpu().numpy()
    worst_b = max(rel(dBn[i], g["dB"][i]) for i in range(prob.n_occ))
    worst_f = rel(dF.cpu().numpy(), g["df"])
    euler = sum(float(np.sum(ora.B(i) * g["dB"][i])) for i in range(prob.n_occ))
    say(f"W rel {worst_w:.2e}  dB rel {worst_b:.2e}  df rel {worst_f:.2e}  "
        f"probe {probe:.15e} oracle <B, dB> {euler:.15e} 4E {4 * g['E']:.15e}")
    assert worst_w <= tol_rel
    assert worst_b <= tol_rel
    assert worst_f <= tol_rel
    assert probe == probe_g
    assert abs(probe - euler) <= tol_rel * abs(euler)
    # probe mode: <dE/dB, Delta> against the oracle's dense gradient, the
    # Euler sum bit for bit that of the other modes, and out = Q^T Delta
    dD, (pr_d, pr_e) = h.mbe3_backward(out["gamma"], out["W"], mode=m.MBE3_GRAD_PROBE)
    D = [oracle.probe_direction(prob, i) for i in range(prob.n_occ)]
    dirn = sum(float(np.sum(D[i] * g["dB"][i])) for i in range(prob.n_occ))
    scale = sum(float(np.sum(np.abs(D[i] * g["dB"][i]))) for i in range(prob.n_occ))
    say(f"probe mode: <dE/dB, Delta> {pr_d:.15e} oracle {dirn:.15e} (sum |.| {scale:.3e})")
    assert pr_e == probe
    assert abs(pr_d - dirn) <= tol_rel * scale
    oD = oracle.Oracle(prob, slabs={i: D[i] for i in range(prob.n_occ)})
    dDn = dD.cpu().numpy().reshape(-1, prob.n_aux)
    for i in range(prob.n_occ):
        row = int(h.g_off[i])
        for x in prob.neighbours(i):
            rx = int(prob.r[x])
            assert rel(dDn[row:row + rx], oD.gamma(i, int(x))) <= 1e-13
            row += rx
    # un-projection of the GAMMA output reproduces the SLAB output
    dGn = dG.cpu().numpy().reshape(-1, prob.n_aux)
    for i in range(prob.n_occ):
        acc = np.zeros((prob.n_vir, prob.n_aux))
        row = int(h.g_off[i])
        for x in prob.neighbours(i):
            rx = int(prob.r[x])
            acc += ora.Q[int(x)] @ dGn[row:row + rx]
            row += rx
        assert rel(dBn[i], acc) <= 1e-12
    h.close()
    return g


def test_backward_chain8_vs_oracle(m):
    say("case: chain8 backward vs oracle.gradient, tol 1e-11")
    prob = dataclasses.replace(synth.config(0), tol=1e-11, max_iter=300)
    check_vs_oracle(m, prob, 1e-10)


@pytest.mark.parametrize("n_occ", [3, 4])
def test_backward_micro_strong(m, n_occ):
    say(f"case: micro n_occ={n_occ} strong coupling backward vs oracle.gradient")
    prob = dataclasses.replace(strong(synth.micro(n_occ)), tol=1e-12, max_iter=300)
    check_vs_oracle(m, prob, 1e-10)


def richardson_fd(h, t):
    """(8 (E(t) - E(-t)) - (E(2t) - E(-2t))) / 12 t of the GPU forward along
    the probe direction (slabs regenerated as B + s Delta)."""
    E = {}
    for k in (1, -1, 2, -2):
        h.set_slab_shift(k * t)
        E[k] = h.forward()["E"]
    h.set_slab_shift(0.0)
    return (8.0 * (E[1] - E[-1]) - (E[2] - E[-2])) / (12.0 * t)


def test_probe_mode_fd_chain8(m):
    """The probe mode's <dE/dB, Delta> against a fourth-order central
    difference of the GPU energy along Delta (t = 1e-4 on slabs of the same
    scale: truncation ~t^4, rounding ~1e-15 E / t); shift 0 gives the
    unshifted energy back bit for bit."""
    say("case: chain8 probe mode vs GPU central difference along Delta, tol 1e-12")
    prob = dataclasses.replace(synth.config(0), tol=1e-12, max_iter=400)
    h = m.from_problem(prob)
    E_ref = h.forward()["E"]
    out = h.forward(grad=True)
    _, (pr_d, pr_e) = h.mbe3_backward(out["gamma"], out["W"], mode=m.MBE3_GRAD_PROBE)
    fd = richardson_fd(h, 1e-4)
    E0 = h.forward()["E"]
    say(f"probe {pr_d:.12e} fd {fd:.12e} rel {abs(fd - pr_d) / abs(pr_d):.2e}")
    assert E0 == E_ref
    assert abs(fd - pr_d) <= 1e-8 * abs(pr_d)
    assert abs(pr_e - 4.0 * out["E"]) <= 1e-9 * abs(out["E"])
    h.close()


def test_probe_mode_errors(m):
    import torch
    say("case: micro n_occ=3 probe mode and slab shift argument errors")
    prob = synth.micro(3)
    h = m.from_problem(prob)
    out = h.forward(grad=True)
    with pytest.raises(m.Mbe3Error):  # out aliasing gamma
        h.mbe3_backward(out["gamma"], out["W"], mode=m.MBE3_GRAD_PROBE, out=out["gamma"])
    with pytest.raises(m.Mbe3Error):
        h.set_slab_shift(float("nan"))
    h.set_slab_shift(1e-3)
    s_fit = torch.empty((prob.n_occ, prob.n_aux), dtype=torch.float64, device="cuda:0")
    with pytest.raises(m.Mbe3Error):  # only osv_project takes the shift
        h.fit_metric(s_fit)
    h.set_slab_shift(0.0)
    h.fit_metric(s_fit)
    h.close()
    hs = m.from_problem(prob, precision=m.MBE3_MIXED_BF16)
    with pytest.raises(m.Mbe3Error):
        hs.set_slab_shift(1e-3)
    hs.set_slab_shift(0.0)
    hs.close()


def test_euler_identity_tight(m):
    """At tight convergence <dE/dGamma, Gamma> = 4 E (degree-4 homogeneity)."""
    say("case: chain8 Euler identity on the GPU, tol 1e-13")
    prob = dataclasses.replace(synth.config(0), tol=1e-13, max_iter=400)
    h = m.from_problem(prob)
    out = h.forward(grad=True)
    _, probe = h.mbe3_backward(out["gamma"], out["W"], mode=m.MBE3_GRAD_GAMMA,
                               probe=True)
    say(f"probe {probe:.15e} 4E {4 * out['E']:.15e}")
    assert abs(probe - 4.0 * out["E"]) <= 1e-12 * abs(out["E"])
    h.close()


def test_energy_fn_autograd(m):
    """torch autograd through energy_fn: slab.grad and f_occ.grad equal the
    oracle's gradient times the upstream factor."""
    import torch
    say("case: energy_fn autograd, micro n_occ=4 strong, explicit slab")
    prob = dataclasses.replace(strong(synth.micro(4)), tol=1e-12, max_iter=300)
    slab = torch.as_tensor(np.stack([oracle.slab(prob, i) for i in range(prob.n_occ)]),
                           device="cuda:0").requires_grad_(True)
    f = torch.as_tensor(prob.f_occ.copy(), device="cuda:0").requires_grad_(True)
    h = m.from_problem(prob, slab=slab.detach(), f_occ=f.detach(), w_ia=None, w_iP=None,
                       warm_start=False)
    E = m.energy_fn(h, slab, f)
    (3.0 * E).backward()
    g = oracle.gradient(prob)
    assert abs(float(E.detach()) - g["E"]) <= 1e-12
    dB = slab.grad.cpu().numpy()
    for i in range(prob.n_occ):
        assert rel(dB[i], 3.0 * g["dB"][i]) <= 1e-10
    assert rel(f.grad.cpu().numpy(), 3.0 * g["df"]) <= 1e-10
    h.close()


def test_backward_fd_on_gpu(m):
    """Central difference of the GPU energy along a random slab direction
    (stream 10 of the input generator) and along f_01 + f_10, against the
    GPU gradient: the backward agrees with the forward it differentiates."""
    import torch
    say("case: chain8 GPU finite differences, explicit slab, tol 1e-13")
    prob = dataclasses.replace(synth.config(0), tol=1e-13, max_iter=400)
    B = np.stack([oracle.slab(prob, i) for i in range(prob.n_occ)])
    rg = synth.rng(prob.seed, synth.STREAM_PROBE)
    D = rg.standard_normal(B.shape) * prob.w_ia[:, :, None] * prob.w_iP[:, None, :]
    slab = torch.as_tensor(B.copy(), device="cuda:0")
    f = torch.as_tensor(prob.f_occ.copy(), device="cuda:0")
    h = m.from_problem(prob, slab=slab, f_occ=f, w_ia=None, w_iP=None)
    out = h.forward(grad=True)
    dF = torch.empty_like(f)
    dB, _ = h.mbe3_backward(out["gamma"], out["W"], dEdF=dF)
    an = float(torch.sum(dB * torch.as_tensor(D, device="cuda:0")))
    step = 1e-5
    E = []
    for sgn in (+1, -1):
        slab.copy_(torch.as_tensor(B + sgn * step * D, device="cuda:0"))
        E.append(h.forward()["E"])
    slab.copy_(torch.as_tensor(B, device="cuda:0"))
    fd = (E[0] - E[1]) / (2 * step)
    say(f"slab direction: fd {fd:.12e} analytic {an:.12e}")
    assert abs(fd - an) <= 1e-7 * abs(an)
    Ef = []
    for sgn in (+1, -1):
        ff = prob.f_occ.copy()
        ff[0, 1] += sgn * step
        ff[1, 0] += sgn * step
        f.copy_(torch.as_tensor(ff, device="cuda:0"))
        Ef.append(h.forward()["E"])
    fdf = (Ef[0] - Ef[1]) / (2 * step)
    anf = 2.0 * float(dF[0, 1])
    say(f"f_01 direction: fd {fdf:.12e} analytic {anf:.12e}")
    assert abs(fdf - anf) <= 1e-7 * max(abs(anf), 1e-3)
    h.close()


def test_backward_errors(m):
    import torch
    say("case: backward argument errors")
    prob = synth.config(0)
    h = m.from_problem(prob)
    out = h.forward(grad=False)
    W = h.empty_K()
    dF = torch.empty((prob.n_occ, prob.n_occ), dtype=torch.float64, device="cuda:0")
    with pytest.raises(m.Mbe3Error) as ex:  # no fragment_solve with W yet
        h.mbe3_backward(out["gamma"], W, dEdF=dF)
    assert ex.value.code == m.MBE3_EINVAL
    small = torch.empty(10, dtype=torch.float64, device="cuda:0")
    with pytest.raises(m.Mbe3Error) as ex:
        h.mbe3_backward(out["gamma"], W, out=small)
    assert ex.value.code == m.MBE3_EINVAL
    with pytest.raises(m.Mbe3Error) as ex:
        h.mbe3_backward(out["gamma"], W, mode=7)
    assert ex.value.code == m.MBE3_EINVAL
    h.close()


def test_backward_water40u_sampled(m):
    """water40u (160 LMOs, 89969 fragments) in the benchmark's launch shape:
    multipliers of sampled pair slots and dE/df of the same pairs against
    the oracle (every fragment containing the pair, solved one by one), and
    sampled dGamma blocks recomputed on the host from the multipliers."""
    import torch
    say("case: water40u backward, sampled oracle slots")
    prob = synth.config(1)
    h = m.from_problem(prob, warm_start=False)  # the oracle's iterates
    out = h.forward(grad=True)
    dF = torch.empty((prob.n_occ, prob.n_occ), dtype=torch.float64, device="cuda:0")
    dG, probe = h.mbe3_backward(out["gamma"], out["W"], mode=m.MBE3_GRAD_GAMMA,
                                dEdF=dF, probe=True)
    dB, _ = h.mbe3_backward(out["gamma"], out["W"], mode=m.MBE3_GRAD_SLAB)
    torch.cuda.synchronize()
    say(f"water40u: E {out['E']:.12f}  probe/4E - 1 = {probe / (4 * out['E']) - 1:.3e}")
    assert np.isfinite(probe) and abs(probe / (4.0 * out["E"]) - 1.0) < 1e-3
    fr = prob.frags
    c = oracle.mbe3_coefficients(prob.n_occ, fr)
    ora = oracle.Oracle(prob)
    dFn = dF.cpu().numpy()
    for s in [prob.n_occ, prob.n_occ + 2000, h.layout.n_slot - 1]:
        p, q = slot_pq(prob, s)
        sel = np.nonzero((fr == p).any(1) & (fr == q).any(1))[0]
        res = oracle.run(prob, frags=fr[sel], keep_T=True, ora=ora)
        Wref = 0.0
        gref = 0.0
        for k, F in enumerate(sel):
            Tt, gF = oracle.fragment_gradient(ora, fr[F], res["T"][k])
            Wref = Wref + c[F] * Tt[(p, q)]
            gref = gref + c[F] * 0.5 * (gF[p, q] + gF[q, p])
        rw = rel(w_block(h, prob, out["W"], s), Wref)
        say(f"slot {s} ({p},{q}): {len(sel)} fragments, W rel {rw:.2e}, "
            f"df {dFn[p, q]:.12e} vs {gref:.12e}")
        assert rw <= 1e-9
        assert abs(dFn[p, q] - gref) <= 1e-9 * max(abs(gref), 1e-8)
    # dGamma~_{i,x} for sampled destinations from the GPU multipliers
    Wd = out["W"].cpu().numpy()
    gam = out["gamma"].view(-1, prob.n_aux).cpu().numpy()
    dGn = dG.view(-1, prob.n_aux).cpu().numpy()

    def gblk(M, i, x):
        nb = [int(y) for y in prob.neighbours(i)]
        row = int(h.g_off[i]) + sum(int(prob.r[y]) for y in nb if y < x)
        return M[row:row + int(prob.r[x])]

    slot = {(int(a), int(b)): prob.n_occ + k for k, (a, b) in enumerate(prob.pairs)}

    def wfull(p, q):
        s = p if p == q else slot[(min(p, q), max(p, q))]
        d = int(prob.r[p] + (prob.r[q] if p != q else 0))
        return Wd[h.k_off[s]:h.k_off[s] + d * d].reshape(d, d)

    for i, x in [(5, 5), (5, int(prob.neighbours(5)[-1])), (100, int(prob.neighbours(100)[0]))]:
        ri, rx = int(prob.r[i]), int(prob.r[x])
        ref = np.zeros((rx, prob.n_aux))
        if x == i:
            Wii = wfull(i, i)
            ref += 2.0 * (Wii + Wii.T) @ gblk(gam, i, i)
            for q in prob.neighbours(i):
                q = int(q)
                if q == i:
                    continue
                rq = int(prob.r[q])
                Wm = wfull(i, q)
                if i < q:
                    R = np.vstack([gblk(gam, q, i), gblk(gam, q, q)])
                    ref += 4.0 * Wm[:ri] @ R
                else:
                    L = np.vstack([gblk(gam, q, q), gblk(gam, q, i)])
                    ref += 4.0 * Wm[:, rq:].T @ L
        else:
            Wm = wfull(i, x)
            if i < x:
                R = np.vstack([gblk(gam, x, i), gblk(gam, x, x)])
                ref += 4.0 * Wm[ri:] @ R
            else:
                L = np.vstack([gblk(gam, x, x), gblk(gam, x, i)])
                ref += 4.0 * Wm[:, :rx].T @ L
        assert rel(gblk(dGn, i, x), ref) <= 1e-12, (i, x)
    # un-projection of a sampled orbital
    dBn = dB[7].cpu().numpy()
    acc = np.zeros((prob.n_vir, prob.n_aux))
    for x in prob.neighbours(7):
        acc += ora.Q[int(x)] @ gblk(dGn, 7, int(x))
    assert rel(dBn, acc) <= 1e-12
    h.close()
