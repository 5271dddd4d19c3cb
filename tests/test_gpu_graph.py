"""Recorded launches (one HIP graph per handle) against the same calls run
eagerly, through the C-ABI (needs an MI355X).

Every kernel of the path reduces in a fixed order, so each replay must give
the eager results bit for bit.  Replays alternate with eager forward passes
into other buffers and with synchronisations, and every replay is checked."""
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


def eager_step(h, grad):
    import torch
    out = h.forward(grad=grad)
    if grad:
        dF = torch.empty((h.n_occ, h.n_occ), dtype=torch.float64, device=h.device)
        dB, _ = h.mbe3_backward(out["gamma"], out["W"], dEdF=dF)
        out["dB"], out["dEdF"] = dB, dF
    torch.cuda.synchronize()
    return out


def same(a, b):
    import torch
    return a.shape == b.shape and bool(torch.equal(a, b))


def check_replays(h, ref, grad, n_rep=3, between=True):
    import torch
    bufs = h.capture_step(grad=grad)
    keys = ["gamma", "K", "e_frag", "iters"] + (["W", "dB", "dEdF"] if grad else [])
    for rep in range(n_rep):
        E = h.graph_launch()
        torch.cuda.synchronize()
        bad = [k for k in keys if not same(bufs[k], ref[k])]
        say(f"  replay {rep}: E = {E!r} (eager {ref['E']!r}), differing buffers: {bad}")
        assert E == ref["E"]
        assert not bad
        if between:  # the program's own eager work between replays
            other = eager_step(h, grad)
            assert other["E"] == ref["E"]
            del other
    return bufs


def test_graph_replays_micro_forward_backward(m):
    """Forward + backward of a 4-LMO problem recorded once, replayed 3 times;
    the energy also against the oracle."""
    import torch
    say("case: micro n_occ=4, recorded forward + backward, 3 replays vs eager")
    prob = dataclasses.replace(synth.micro(4), tol=1e-10, max_iter=300)
    h = m.from_problem(prob)
    ref = eager_step(h, grad=True)
    ora = oracle.run(prob)
    E_ref, _ = oracle.mbe3_energy(prob.frags, ora["e_frag"])
    assert abs(ref["E"] - E_ref) <= 1e-10
    bufs = check_replays(h, ref, grad=True)
    # the replay left dE/df for a following eager backward
    dF = torch.empty_like(ref["dEdF"])
    h.mbe3_backward(bufs["gamma"], bufs["W"], dEdF=dF)
    torch.cuda.synchronize()
    assert same(dF, ref["dEdF"])
    h.close()


def test_graph_timing_chain8(m):
    """Timing on while recording: the phase events live in the graph and
    every replay adds one region per recorded phase scope."""
    say("case: chain8, recorded forward with timing, 2 replays")
    prob = synth.config(0)
    h = m.from_problem(prob)
    h.set_timing(True)
    ref = eager_step(h, grad=False)
    eager_t = h.get_timing()
    h.set_timing(True)
    check_replays(h, ref, grad=False, n_rep=2, between=False)
    t = h.get_timing()
    say(f"  eager regions {dict((k, v[1]) for k, v in eager_t.items())}")
    say(f"  graph regions {dict((k, v[1]) for k, v in t.items())}")
    for ph, (ms, n) in eager_t.items():
        assert t[ph][1] == 2 * n
        if n:
            assert t[ph][0] > 0.0
    h.close()


def test_graph_replays_water40u_forward_backward(m):
    """water40u (89969 fragments) forward + backward as one graph:
    replays equal the eager step and the energy matches the oracle's full
    run (trimers warm-started)."""
    import torch
    say("case: water40u, recorded forward + backward, 2 replays vs eager")
    g = json.load(open(os.path.join(os.path.dirname(__file__), "golden",
                                    "water40u_oracle_warm.json")))
    prob = synth.config(1)
    h = m.from_problem(prob)
    ref = eager_step(h, grad=True)
    say(f"  eager E = {ref['E']!r}, oracle {g['E_total']}")
    assert abs(ref["E"] - float(g["E_total"])) <= 2e-8
    check_replays(h, ref, grad=True, n_rep=2, between=True)
    h.close()
    del ref
    torch.cuda.empty_cache()


def test_graph_errors(m):
    """Misuse is refused with MBE3_EINVAL and leaves the handle usable."""
    import torch
    say("case: micro n_occ=3, graph misuse")
    prob = synth.micro(3)
    h = m.from_problem(prob)
    with pytest.raises(m.Mbe3Error) as ei:
        h.graph_launch()
    assert ei.value.code == m.MBE3_EINVAL
    # gradient plans are not made while recording
    gamma, K = h.empty_gamma(), h.empty_K()
    e = torch.empty(h.n_frag, dtype=torch.float64, device=h.device)
    it = torch.empty(h.n_frag, dtype=torch.int32, device=h.device)
    W = h.empty_K()
    torch.cuda.synchronize()
    h.graph_begin(with_grad=False)
    with pytest.raises(m.Mbe3Error) as ei:
        h.graph_begin()
    assert ei.value.code == m.MBE3_EINVAL
    h.osv_project(gamma)
    h.pair_K(gamma, K)
    with pytest.raises(m.Mbe3Error) as ei:
        h.fragment_solve(K, e, it, W)
    assert ei.value.code == m.MBE3_EINVAL
    with pytest.raises(m.Mbe3Error) as ei:
        h.graph_end()
    assert ei.value.code == m.MBE3_EINVAL
    # timing cannot change while recording; the probe is refused
    h.graph_begin(with_grad=True)
    with pytest.raises(m.Mbe3Error):
        h.set_timing(True)
    h.osv_project(gamma)
    h.pair_K(gamma, K)
    h.fragment_solve(K, e, it, W)
    with pytest.raises(m.Mbe3Error):
        h.mbe3_backward(gamma, W, probe=True)
    with pytest.raises(m.Mbe3Error):
        h.graph_end()
    with pytest.raises(m.Mbe3Error):
        h.graph_launch()
    # still usable eagerly, and a clean recording works afterwards
    ref = eager_step(h, grad=True)
    check_replays(h, ref, grad=True, n_rep=2, between=False)
    h.close()


@pytest.mark.parametrize("form", ["MBE3_MIXED_BF16", "MBE3_MIXED_BF16_PROJ"])
def test_graph_replays_split_precision(m, form):
    """The split-precision forms recorded (their regeneration, splits and
    bf16 products included): replays equal the eager step bit for bit."""
    say(f"case: micro n_occ=4, {form}, recorded forward + backward, 2 replays vs eager")
    prob = dataclasses.replace(synth.micro(4, n_vir=21, n_aux=35), tol=1e-10, max_iter=300)
    h = m.from_problem(prob, precision=getattr(m, form))
    ref = eager_step(h, grad=True)
    check_replays(h, ref, grad=True, n_rep=2, between=True)
    h.close()
