"""The C-ABI library loads, exports what include/mbe3osv.h declares, and
plans real workloads within bounds (no GPU needed)."""
import ctypes
import os
import re

import numpy as np
import pytest

import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def pkg():
    import paper_2603_16575_amd as m
    m._lib.load()
    return m


def declared_functions():
    src = open(os.path.join(ROOT, "include", "mbe3osv.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:int|const char \*)\s*\**\s*(\w+)\s*\(", src, re.M)))


def test_header_symbols_exported(pkg):
    names = declared_functions()
    assert "osv_project" in names and "fragment_solve" in names
    lib = ctypes.CDLL(pkg._lib.LIB_PATH)
    for n in names:
        assert hasattr(lib, n), n
    assert sorted(pkg._lib.EXPORTS) == names


@pytest.mark.parametrize("k", [0, 1])
@pytest.mark.parametrize("precision", ["MBE3_FP64", "MBE3_MIXED_BF16",
                                       "MBE3_MIXED_BF16_PROJ"])
def test_plan_check_small_workloads(pkg, k, precision):
    p = synth.config(k)
    prec = getattr(pkg, precision)
    lay = pkg.plan_check(r=p.r, pairs=p.pairs, frags=p.frags, n_vir=p.n_vir,
                         n_aux=p.n_aux, precision=prec)
    rows = sum(int(p.r[p.neighbours(i)].sum()) for i in range(p.n_occ))
    assert lay.gamma_rows == rows
    assert lay.n_frag == p.n_frag
    d = np.concatenate([p.r, p.r[p.pairs[:, 0]] + p.r[p.pairs[:, 1]]])
    assert lay.k_elems == int((d.astype(np.int64) ** 2).sum())


@pytest.mark.parametrize("k", [2, 4])
def test_plan_check_large_workloads(pkg, k):
    """Configurations 2 (470k fragments, D <= 128) and 4 (D <= 160) plan and
    pass every bounds check, both precisions."""
    p = synth.config(k)
    for prec in (pkg.MBE3_FP64, pkg.MBE3_MIXED_BF16, pkg.MBE3_MIXED_BF16_PROJ):
        lay = pkg.plan_check(r=p.r, pairs=p.pairs, frags=p.frags, n_vir=p.n_vir,
                             n_aux=p.n_aux, precision=prec)
        assert lay.n_frag == p.n_frag


def test_plan_check_micro_explicit_slab(pkg):
    p = synth.micro(4)
    pkg.plan_check(r=p.r, pairs=p.pairs, frags=p.frags, n_vir=p.n_vir,
                   n_aux=p.n_aux, explicit_slab=True)
    # split planes pad rows to a multiple of 8: odd sizes plan as well
    for prec in (pkg.MBE3_MIXED_BF16, pkg.MBE3_MIXED_BF16_PROJ):
        pkg.plan_check(r=p.r, pairs=p.pairs, frags=p.frags, n_vir=p.n_vir + 3,
                       n_aux=p.n_aux + 5, explicit_slab=True, precision=prec)


def test_plan_check_rejects_unknown_precision(pkg):
    p = synth.micro(3)
    with pytest.raises(pkg.Mbe3Error) as ex:
        pkg.plan_check(r=p.r, pairs=p.pairs, frags=p.frags, n_vir=p.n_vir,
                       n_aux=p.n_aux, precision=7)
    assert ex.value.code == pkg.MBE3_EINVAL


def test_plan_check_rejects_bad_lists(pkg):
    p = synth.config(0)
    kw = dict(r=p.r, n_vir=p.n_vir, n_aux=p.n_aux)
    with pytest.raises(pkg.Mbe3Error) as e:  # trimer whose dimer is missing
        fr = p.frags
        keep = ~((fr[:, 0] == 0) & (fr[:, 1] == 1) & (fr[:, 2] == -1))
        pkg.plan_check(pairs=p.pairs, frags=fr[keep], **kw)
    assert e.value.code == pkg.MBE3_EINVAL and "lacks dimer" in str(e.value)
    with pytest.raises(pkg.Mbe3Error) as e:  # pair not kept
        pkg.plan_check(pairs=p.pairs[1:], frags=p.frags, **kw)
    assert e.value.code == pkg.MBE3_EINVAL
    with pytest.raises(pkg.Mbe3Error) as e:  # unsorted pair
        bad = p.pairs.copy()
        bad[0] = bad[0][::-1]
        pkg.plan_check(pairs=bad, frags=p.frags, **kw)
    assert e.value.code == pkg.MBE3_EINVAL
    with pytest.raises(pkg.Mbe3Error) as e:  # r out of range
        pkg.plan_check(r=np.full(p.n_occ, p.n_vir + 1), pairs=p.pairs,
                       frags=p.frags, n_vir=p.n_vir, n_aux=p.n_aux)
    assert e.value.code == pkg.MBE3_EINVAL
