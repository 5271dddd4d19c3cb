"""Degenerate problem shapes through the C-ABI against the oracle (needs an
MI355X): one orbital, orbitals too far apart to pair, dimers without any
trimer, and identity OSVs (every pair overlap singular: the canonical
orthogonalisation drops half of each pair space, and with a diagonal
occupied Fock the MBE(3) energy is the canonical MP2 closed form)."""
import sys

import numpy as np
import pytest

import _pins
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


def chain(n, spacing, cutoff, **kw):
    cfg = dict(name=f"chain{n}", geometry="chain", n_occ=n, spacing=spacing,
               n_vir=16, n_aux=24, r=(3, 4), cutoff=cutoff, tol=1e-12)
    return synth.build(cfg, 11, **kw)


def forward_backward_vs_oracle(m, prob):
    import torch
    h = m.from_problem(prob, warm_start=False)
    out = h.forward(grad=True)
    dF = torch.empty((prob.n_occ, prob.n_occ), dtype=torch.float64, device="cuda:0")
    dB, _ = h.mbe3_backward(out["gamma"], out["W"], dEdF=dF)
    torch.cuda.synchronize()
    ref = oracle.run(prob)
    E_ref, _ = oracle.mbe3_energy(prob.frags, ref["e_frag"])
    e = out["e_frag"].cpu().numpy()
    g = oracle.gradient(prob)
    dBn = dB.cpu().numpy()
    gB = np.stack([g["dB"][i] for i in range(prob.n_occ)])
    rb = float(np.abs(dBn - gB).max() / np.abs(gB).max())
    rf = float(np.abs(dF.cpu().numpy() - g["df"]).max() / np.abs(g["df"]).max())
    say(f"  {prob.name}: {prob.n_frag} fragments, dE = {out['E'] - E_ref:.2e}, "
        f"max |dE_F| = {np.abs(e - ref['e_frag']).max():.2e}, dB rel {rb:.1e}, df rel {rf:.1e}")
    assert np.abs(e - ref["e_frag"]).max() <= 1e-12
    assert abs(out["E"] - E_ref) <= 1e-12
    assert rb <= 1e-10 and rf <= 1e-10
    h.close()
    return out


def test_single_orbital(m):
    say("case: one orbital (one monomer, no pairs)")
    forward_backward_vs_oracle(m, synth.micro(1))


def test_no_pairs(m):
    say("case: three orbitals 10 apart, cutoff 6 (monomers only)")
    prob = chain(3, 10.0, 6.0)
    assert len(prob.pairs) == 0
    forward_backward_vs_oracle(m, prob)


def test_dimers_without_trimers(m):
    say("case: four orbitals 4 apart, cutoff 6 (neighbour pairs, no trimer)")
    prob = chain(4, 4.0, 6.0)
    assert len(prob.pairs) == 3 and len(prob.trimers) == 0
    forward_backward_vs_oracle(m, prob)


def test_identity_osv_canonical_mp2(m):
    """Q_i = I (r_i = n_vir): each pair overlap [[I, I], [I, I]] has the
    eigenvalues 0 and 2 (n_vir each), the Cholesky step flags every pair and
    the eigen route keeps n_vir columns; with a diagonal Fock the result is
    the closed-form canonical MP2 energy of all pairs."""
    say("case: micro n_occ=3, identity OSVs, diagonal Fock, vs canonical MP2")
    prob = synth.micro(3, identity_q=True, diagonal_f=True)
    h = m.from_problem(prob, warm_start=False)
    out = h.forward()
    X, et, rank = h.mbe3_pair_basis()
    rank = rank.cpu().numpy()
    ora = oracle.Oracle(prob)
    ref = _pins.canonical_mp2([ora.B(i) for i in range(prob.n_occ)], prob.eps_vir,
                              np.diag(prob.f_occ))
    say(f"  E = {out['E']!r}, closed form {ref!r}, dE = {out['E'] - ref:.2e}, "
        f"ranks {rank.tolist()}")
    assert np.all(rank[:prob.n_occ] == prob.n_vir)
    assert np.all(rank[prob.n_occ:] == prob.n_vir)
    assert abs(out["E"] - ref) <= 1e-12 * abs(ref)
    # the kept pair bases are S-orthonormal and diagonalise F
    X, et = X.cpu().numpy(), et.cpu().numpy()
    for s in range(prob.n_occ, h.layout.n_slot):
        p, q = (int(v) for v in prob.pairs[s - prob.n_occ])
        o = oracle.orbs(p, q)
        S, F = ora.Sblk(o, o), ora.Fblk(o, o)
        d = S.shape[0]
        D = (d + 15) // 16 * 16
        Xs = X[h.x_off[s]:h.x_off[s + 1]].reshape(d, D)[:, :rank[s]]
        es = et[h.e_off[s]:h.e_off[s] + rank[s]]
        assert np.allclose(Xs.T @ S @ Xs, np.eye(rank[s]), atol=1e-12)
        assert np.allclose(Xs.T @ F @ Xs, np.diag(es), atol=1e-12)
    h.close()


def test_create_enomem_then_usable(m):
    """A problem whose single-LMO slab buffer (20000 x 2e6 doubles, 320 GB)
    exceeds the device: mbe3_create returns MBE3_ENOMEM with the size in the
    message, frees what it had allocated, and the device takes the next
    handle normally."""
    import torch
    say("case: mbe3_create beyond device memory (320 GB slab buffer) -> MBE3_ENOMEM")
    nv, na = 20000, 2000000
    dev = "cuda:0"
    Q = torch.ones((nv, 1), dtype=torch.float64, device=dev) / np.sqrt(nv)
    eps = torch.linspace(0.5, 3.0, nv, dtype=torch.float64, device=dev)
    f = torch.full((1, 1), -0.5, dtype=torch.float64, device=dev)
    w_ia = torch.ones((1, nv), dtype=torch.float64, device=dev)
    w_iP = torch.ones((1, na), dtype=torch.float64, device=dev)
    free0, _ = torch.cuda.mem_get_info()
    with pytest.raises(m.Mbe3Error) as ex:
        m.Mbe3(r=[1], Q=Q, eps_vir=eps, f_occ=f, pairs=np.zeros((0, 2)),
               frags=[[0, -1, -1]], w_ia=w_ia, w_iP=w_iP)
    say(f"  {ex.value}")
    assert ex.value.code == m.MBE3_ENOMEM and "bytes" in str(ex.value)
    torch.cuda.synchronize()
    free1, _ = torch.cuda.mem_get_info()
    assert free1 >= free0 - (64 << 20)  # the partial workspace was released
    forward_backward_vs_oracle(m, synth.micro(3))
