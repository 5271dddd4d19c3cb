"""Tile shapes of the grouped FP64 GEMMs and the autotuner, through the
C-ABI (needs an MI355X).

Every shape accumulates each output over k in the same order, so forcing
any shape on every task list must reproduce the planned shapes' forward and
backward bit for bit; the planned path is itself checked against the
oracle."""
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


def step(h):
    import torch
    out = h.forward(grad=True)
    dF = torch.empty((h.n_occ, h.n_occ), dtype=torch.float64, device=h.device)
    dB, _ = h.mbe3_backward(out["gamma"], out["W"], dEdF=dF)
    torch.cuda.synchronize()
    out["dB"], out["dEdF"] = dB, dF
    return out


KEYS = ["gamma", "K", "e_frag", "iters", "W", "dB", "dEdF"]


def differing(a, b):
    import torch
    return [k for k in KEYS if not torch.equal(a[k], b[k])]


@pytest.mark.parametrize("prob_name", ["micro5_ragged", "chain8"])
def test_every_shape_bitwise(m, prob_name):
    if prob_name == "chain8":
        prob = synth.config(0)
    else:  # sizes off every tile multiple
        prob = dataclasses.replace(synth.micro(5, n_vir=37, n_aux=53), tol=1e-10,
                                   max_iter=300)
    say(f"case: {prob_name}, every GEMM shape on every list vs the planned shapes")
    h = m.from_problem(prob)
    ref = step(h)
    ora = oracle.run(prob)
    E_ref, _ = oracle.mbe3_energy(prob.frags, ora["e_frag"])
    assert abs(ref["E"] - E_ref) <= 1e-10
    for k, name in enumerate(m._lib.GEMM_SHAPES):
        h.set_gemm_shape(k)
        out = step(h)
        bad = differing(out, ref)
        say(f"  shape {name}: E = {out['E']!r}, differing: {bad}")
        assert out["E"] == ref["E"]
        assert not bad
    h.close()


def test_autotune_water40u(m):
    """water40u (160 LMOs): the tuned step equals the planned one bit for bit,
    and every list's report lists all shapes."""
    import torch
    say("case: water40u, autotune, tuned forward + backward vs planned")
    prob = synth.config(1)
    h = m.from_problem(prob)
    ref = step(h)
    rep = h.autotune(reps=2)
    say(rep)
    lines = [ln for ln in rep.splitlines() if ln.strip()]
    assert len(lines) >= 10
    for ln in lines:
        for name in m._lib.GEMM_SHAPES:
            assert f" {name} " in ln
    out = step(h)
    bad = differing(out, ref)
    say(f"  tuned E = {out['E']!r} (planned {ref['E']!r}), differing: {bad}")
    assert out["E"] == ref["E"]
    assert not bad
    h.close()
    del ref, out
    torch.cuda.empty_cache()


@pytest.mark.parametrize("form", ["MBE3_MIXED_BF16", "MBE3_MIXED_BF16_PROJ"])
def test_autotune_mixed_micro(m, form):
    """A split-precision handle tunes only the lists it launches (the split
    products have their own task lists instead of the FP64 ones: the
    projection in both forms, pair_K in MBE3_MIXED_BF16); the tuned step
    equals the planned one."""
    say(f"case: micro n_occ=4 {form}, autotune, tuned vs planned")
    prob = dataclasses.replace(synth.micro(4), tol=1e-10, max_iter=300)
    h = m.from_problem(prob, precision=getattr(m, form))
    ref = step(h)
    rep = h.autotune(reps=1)
    say(rep)
    heads = [ln.split(":", 1)[0] for ln in rep.splitlines() if ln.strip()]
    names = [hd.split(" ", 1)[1].rsplit(" (", 1)[0] for hd in heads]
    assert names and not any(n.startswith("project") for n in names)
    has_pk = any(n.startswith("pair_K") for n in names)
    assert has_pk == (form == "MBE3_MIXED_BF16_PROJ")
    out = step(h)
    bad = differing(out, ref)
    say(f"  tuned E = {out['E']!r} (planned {ref['E']!r}), differing: {bad}")
    assert out["E"] == ref["E"]
    assert not bad
    h.close()
