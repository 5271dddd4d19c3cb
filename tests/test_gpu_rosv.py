"""Randomized OSV generation (mbe3_rosv) through the C-ABI against the
oracle's Alg. 3 (needs an MI355X): every LMO of a 64-LMO helix (on the
fitting domains and on all columns), a chain whose flat spectrum runs the
range finder into its row cap, and sampled LMOs of the 1024-LMO helix
(timed over all 1024): the accepted row count and kept OSV count exactly,
the singular values, and the OSV span (projector), plus argument errors."""
import sys
import time

import numpy as np
import pytest

import _workloads
import synth
from oracle import fit
from oracle import rosv as R

pytestmark = pytest.mark.gpu

HELIX64 = dict(name="helix64", geometry="helix", n_occ=64, n_vir=256, n_aux=768,
               r=(24, 80), cutoff=6.0, tol=1e-7)


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


def compare(prob, out, lmos, l_fit, n_max, tag):
    """GPU rosv output against the oracle for the given LMOs; returns the
    worst singular-value and projector differences."""
    Q = out["Q"].cpu().numpy()
    w = out["w"].cpu().numpy()
    k = out["n_osv"].cpu().numpy()
    rows = out["rows"].cpu().numpy()
    worst_w = worst_p = 0.0
    for i in lmos:
        ref = R.lmo_rosv(prob, int(i), l_fit=l_fit, n_max=n_max)
        assert rows[i] == ref["rows"], (tag, i, rows[i], ref["rows"])
        assert k[i] == len(ref["w"]), (tag, i, k[i], len(ref["w"]))
        wi = w[i, :k[i]]
        worst_w = max(worst_w, float(np.max(np.abs(wi - ref["w"]) / ref["w"])))
        Qi = Q[i, :k[i]].T  # n_vir x k
        assert np.abs(Qi.T @ Qi - np.eye(k[i])).max() <= 1e-12
        P = Qi @ Qi.T
        Pr = ref["Q"] @ ref["Q"].T
        worst_p = max(worst_p, float(np.abs(P - Pr).max()))
        assert not np.any(Q[i, k[i]:]) and not np.any(w[i, k[i]:])
    return worst_w, worst_p


@pytest.mark.parametrize("use_fit", [True, False])
def test_rosv_helix64_every_lmo(m, use_fit):
    say(f"case: helix64 (64 LMOs, n_vir 256), rOSV of every LMO, fitting domains {use_fit}")
    prob = synth.build(HELIX64, 12345)
    h = m.from_problem(prob)
    s = h.fit_metric() if use_fit else None
    l_fit = 1e-6 if use_fit else None
    out = h.rosv(n_max=128, s_fit=s, l_fit=l_fit if use_fit else 0.0)
    ww, wp = compare(prob, out, range(prob.n_occ), l_fit, 128, "helix64")
    k = out["n_osv"].cpu().numpy()
    say(f"  OSVs per LMO {k.min()}-{k.max()}, rows {out['rows'].cpu().numpy().min()}-"
        f"{out['rows'].cpu().numpy().max()}; max rel |dw| {ww:.2e}, max |dP| {wp:.2e}")
    assert ww <= 1e-10 and wp <= 1e-9
    h.close()


def test_rosv_row_cap_chain8(m):
    """chain8's slabs have a flat T_ii spectrum (nearly every direction above
    l_osv): the loop stops at the n_max cap on both sides."""
    say("case: chain8, rOSV capped at n_max = 24 rows")
    prob = synth.config(0)
    h = m.from_problem(prob)
    out = h.rosv(n_max=24)
    rows = out["rows"].cpu().numpy()
    assert (rows == 24).all()
    ww, wp = compare(prob, out, range(prob.n_occ), None, 24, "chain8")
    say(f"  max rel |dw| {ww:.2e}, max |dP| {wp:.2e}")
    assert ww <= 1e-10 and wp <= 1e-9
    for bad in (dict(n_max=0), dict(n_max=100000), dict(l_osv=0.0)):
        with pytest.raises(m.Mbe3Error) as ei:
            h.rosv(**bad)
        assert ei.value.code == m.MBE3_EINVAL
    h.close()


def test_rosv_helix1024(m):
    """All 1024 LMOs of the helix at l_fit = 1e-6 (timed), three of them
    against the oracle."""
    import torch
    say("case: helix1024, rOSV of all 1024 LMOs on the fitting domains, 3 vs oracle")
    prob = _workloads.config(4)
    h = m.from_problem(prob)
    s = h.fit_metric()
    out = h.rosv(n_max=128, s_fit=s, l_fit=fit.L_FIT)  # first call: warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    out = h.rosv(n_max=128, s_fit=s, l_fit=fit.L_FIT)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    k = out["n_osv"].cpu().numpy()
    rows = out["rows"].cpu().numpy()
    say(f"  {dt * 1e3:.1f} ms for 1024 LMOs; OSVs per LMO {k.min()}-{k.max()} "
        f"(mean {k.mean():.1f}), rows {rows.min()}-{rows.max()}")
    assert (rows < 128).all()
    ww, wp = compare(prob, out, [1, 500, 1023], fit.L_FIT, 128, "helix1024")
    say(f"  sampled LMOs: max rel |dw| {ww:.2e}, max |dP| {wp:.2e}")
    assert ww <= 1e-10 and wp <= 1e-9
    h.close()
