"""mbe3_screen_noalloc (the allocation-free variant of mbe3_screen) through
the C-ABI against mbe3_screen (needs an MI355X): two calls in a row on the
160-LMO lattice, the second with fewer pairs, each bit for bit the
allocating call's s2b; a request beyond the scratch array is refused with
a clear error and leaves the handle usable."""
import sys

import numpy as np
import pytest

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


def test_screen_noalloc_matches_screen(m):
    import torch
    say("case: water40u, mbe3_screen_noalloc vs mbe3_screen, two calls")
    prob = synth.config(1)
    n = prob.n_occ
    cand = np.array([(i, j) for i in range(n) for j in range(i + 1, n)], dtype=np.int32)
    lib = m._lib.load()
    cap = int(lib.mbe3_screen_noalloc_max_bytes())
    h = m.from_problem(prob)
    first, second = cand[:6000], cand[7000:7400][:, ::-1]  # the second smaller, reversed
    for k, pr in enumerate((first, second)):
        pr = np.ascontiguousarray(pr)
        ref = h.screen(pr)
        out = torch.full((len(pr),), float("nan"), dtype=torch.float64, device="cuda:0")
        rc = lib.mbe3_screen_noalloc(h._h, m._lib.ptr(pr), len(pr), m._lib.ptr(out))
        assert rc == m.MBE3_OK, lib.mbe3_last_error(h._h).decode()
        torch.cuda.synchronize()
        say(f"  call {k + 1}: {len(pr)} pairs, equal {torch.equal(out, ref)}")
        assert torch.equal(out, ref)
    # beyond the scratch array: refused, with the sizes in the message
    rc = lib.mbe3_screen_noalloc(h._h, m._lib.ptr(cand), len(cand), m._lib.ptr(out))
    msg = lib.mbe3_last_error(h._h).decode()
    say(f"  all {len(cand)} pairs ({cap} bytes of scratch): rc {rc}, {msg}")
    assert rc == m.MBE3_EINVAL and "scratch" in msg
    # still usable afterwards
    pr = np.ascontiguousarray(cand[:50])
    assert torch.equal(h.screen_noalloc(pr), h.screen(pr))
    h.close()
