"""The library's host code (planner, bounds checks, list validation, the
host-only screening call) under AddressSanitizer and UndefinedBehaviorSanitizer
(no GPU needed): the library is rebuilt with the sanitizers on its host code
only and driven in a child process that preloads the ASan runtime, over every
workload configuration, the split-precision plans, rejected inputs and a
problem whose slab buffer is larger than any device (planned, never
allocated).  Any sanitizer report aborts the child and fails the test."""
import os
import subprocess
import sys
import textwrap

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

CHILD = textwrap.dedent("""
    import sys
    sys.path.insert(0, {root!r})
    import numpy as np
    import paper_2603_16575_amd._lib as L
    L.LIB_PATH = {lib!r}
    import paper_2603_16575_amd as m
    import synth

    def plan(p, **kw):
        return m.plan_check(r=p.r, pairs=p.pairs, frags=p.frags, n_vir=p.n_vir,
                            n_aux=p.n_aux, **kw)

    def rejected(fn):
        try:
            fn()
        except m.Mbe3Error as e:
            return e.code
        raise SystemExit("accepted an invalid input")

    precs = (m.MBE3_FP64, m.MBE3_MIXED_BF16, m.MBE3_MIXED_BF16_PROJ)
    for k in (0, 1, 2, 4):
        p = synth.config(k)
        for prec in (precs if k < 2 else (m.MBE3_FP64,)):
            for warm in (True, False):
                assert plan(p, precision=prec, warm_start=warm).n_frag == p.n_frag
        print("planned configuration", k, flush=True)
    mp = synth.micro(4)
    plan(mp, explicit_slab=True)
    for prec in precs[1:]:
        m.plan_check(r=mp.r, pairs=mp.pairs, frags=mp.frags, n_vir=mp.n_vir + 3,
                     n_aux=mp.n_aux + 5, explicit_slab=True, precision=prec)
    # rejected lists and sizes
    p = synth.config(0)
    fr = p.frags
    keep = ~((fr[:, 0] == 0) & (fr[:, 1] == 1) & (fr[:, 2] == -1))
    kw = dict(r=p.r, n_vir=p.n_vir, n_aux=p.n_aux)
    codes = [
        rejected(lambda: m.plan_check(pairs=p.pairs, frags=fr[keep], **kw)),
        rejected(lambda: m.plan_check(pairs=p.pairs[1:], frags=p.frags, **kw)),
        rejected(lambda: m.plan_check(pairs=p.pairs[:, ::-1], frags=p.frags, **kw)),
        rejected(lambda: m.plan_check(r=np.full(p.n_occ, p.n_vir + 1), pairs=p.pairs,
                                      frags=p.frags, n_vir=p.n_vir, n_aux=p.n_aux)),
        rejected(lambda: m.plan_check(pairs=p.pairs, frags=np.array([[0, 0, -1]]), **kw)),
        rejected(lambda: m.plan_check(pairs=p.pairs, frags=np.array([[0, 99, -1]]), **kw)),
        rejected(lambda: plan(p, precision=7)),
    ]
    assert all(c == m.MBE3_EINVAL for c in codes), codes
    # one LMO whose slab alone (20000 x 2e6 doubles, 320 GB) exceeds a
    # device: the plan holds, only the allocation could fail
    lay = m.plan_check(r=[1], pairs=np.zeros((0, 2)), frags=[[0, -1, -1]],
                       n_vir=20000, n_aux=2000000)
    assert lay.gamma_elems == 2000000
    # host-only screening into the paper's classes and kept trimers
    rng = np.random.default_rng(5)
    n = 40
    iu = np.stack(np.triu_indices(n, 1), 1)
    s = rng.uniform(0.0, 0.6, len(iu)) ** 3
    out = m.screen_lists(n, iu, s)
    assert len(out["close"]) + len(out["weak"]) <= len(iu)
    for bad in ([[0, 1], [1, 0]], [[0, n]], [[2, 2]]):
        rejected(lambda: m.screen_lists(n, np.array(bad), [0.5] * len(bad)))
    print("sanitized host run clean", flush=True)
""")


@pytest.mark.slow
def test_host_code_under_asan_ubsan(tmp_path):
    from paper_2603_16575_amd import build as b
    rt = b.asan_runtime()
    if rt is None:
        pytest.skip("no ASan runtime next to hipcc's clang")
    lib = b.build(out=str(tmp_path / "libmbe3osv_asan.so"), host_sanitize=True)
    env = dict(os.environ)
    env["LD_PRELOAD"] = rt
    env["ASAN_OPTIONS"] = "detect_leaks=0:halt_on_error=1:abort_on_error=1"
    env["UBSAN_OPTIONS"] = "halt_on_error=1:print_stacktrace=1"
    env["OMP_NUM_THREADS"] = "1"
    res = subprocess.run([sys.executable, "-c", CHILD.format(root=ROOT, lib=lib)],
                         env=env, capture_output=True, text=True, timeout=1500)
    tail = (res.stdout + res.stderr)[-4000:]
    assert res.returncode == 0, tail
    assert "sanitized host run clean" in res.stdout, tail
    assert "runtime error" not in res.stderr and "AddressSanitizer" not in res.stderr, tail
