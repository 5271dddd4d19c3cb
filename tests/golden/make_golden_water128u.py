"""Write tests/golden/water128u_sample_oracle.json from the CPU oracle only.

water128u (512 LMOs, n_vir 2432, n_aux 7040, 470430 fragments) is too large
for a full oracle run, so the fixture holds a fixed deterministic sample:
every 97th fragment plus every fragment containing LMO 0, solved from T = 0
(oracle.run), with their update counts, and 16 seeded elements of the pair
integrals K of eight slots (two diagonal, three pairs of LMO 0, three
others of the sample).  The oracle keeps at most 96 regenerated slabs and
3000 projected blocks in memory at a time.  Usage:
    python tests/golden/make_golden_water128u.py [workers]
"""
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import oracle  # noqa: E402
import synth  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "water128u_sample_oracle.json")


def sample_index(prob):
    fr = prob.frags
    return np.unique(np.concatenate([np.arange(0, len(fr), 97),
                                     np.nonzero((fr == 0).any(1))[0]]))


def sample_slots(prob, frags):
    """Eight (p, q) slots: (0, 0), (1, 1), three pairs of LMO 0, three
    other pairs of the sampled fragments (seeded choice)."""
    pairs = sorted({(int(a), int(b)) for f in frags for a in f for b in f
                    if 0 <= a < b})
    zero = [t for t in pairs if t[0] == 0][:3]
    rest = [t for t in pairs if t[0] != 0]
    rng = np.random.default_rng(97)
    other = [rest[k] for k in sorted(rng.choice(len(rest), 3, replace=False))]
    return [(0, 0), (1, 1)] + zero + other


def main():
    workers = int(sys.argv[1]) if len(sys.argv) > 1 else os.cpu_count()
    t0 = time.time()
    prob = synth.config(2)
    idx = sample_index(prob)
    frags = prob.frags[idx]
    ora = oracle.Oracle(prob, max_slabs=96, max_gammas=3000)
    oracle.mbe3.prepare(ora, frags)
    ora._slabs.clear()   # the solves need K, bases and overlaps only
    ora._gamma.clear()
    print(f"prepared {len(idx)} fragments in {time.time() - t0:.0f} s", flush=True)
    out = oracle.run(prob, frags=frags, workers=workers, ora=ora)
    rng = np.random.default_rng(2)
    kslots = []
    for (p, q) in sample_slots(prob, frags):
        K = ora.Kbar(p, q)
        pos = rng.integers(0, K.size, 16)
        kslots.append({"p": p, "q": q, "d": int(K.shape[0]), "flat_index": pos.tolist(),
                       "values": [repr(float(K.flat[k])) for k in pos],
                       "frobenius": repr(float(np.linalg.norm(K)))})
    rec = {
        "workload": "water128u (512 LMOs, 470430 fragments); every 97th fragment and "
                    "every fragment containing LMO 0, each from T = 0",
        "n_frag": int(prob.n_frag),
        "sample_index": idx.tolist(),
        "e_frag": [repr(float(x)) for x in out["e_frag"]],
        "iters": out["iters"].tolist(),
        "converged": bool(out["converged"].all()),
        "k_slots": kslots,
        "oracle_seconds": round(time.time() - t0, 1),
        "workers": workers,
    }
    with open(OUT, "w") as f:
        json.dump(rec, f, indent=0)
    print(OUT, len(idx), "fragments", rec["oracle_seconds"], "s")


if __name__ == "__main__":
    main()
