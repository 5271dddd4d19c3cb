"""Write tests/golden/water40u_oracle.json (every fragment from T = 0) or,
with --warm, water40u_oracle_warm.json (trimers started from their
monomer/dimer solutions) from the CPU oracle only.

Full MBE(3) energy of water40u (160 LMOs, 89969 fragments), its
update-count histogram and every 1000th fragment energy, computed by
oracle.run with a process pool.  Usage:
    python tests/golden/make_golden.py [workers] [--warm]
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


def main():
    args = [a for a in sys.argv[1:] if not a.startswith("--")]
    warm = "--warm" in sys.argv[1:]
    workers = int(args[0]) if args else os.cpu_count()
    t0 = time.time()
    prob = synth.config(1)
    out = oracle.run(prob, workers=workers, warm_start=warm)
    E, _ = oracle.mbe3_energy(prob.frags, out["e_frag"])
    idx = np.arange(0, prob.n_frag, 1000)
    rec = {
        "workload": "water40u (160 LMOs, 89969 fragments)",
        "start": "trimers from monomer/dimer solutions" if warm else "T = 0",
        "n_frag": int(prob.n_frag),
        "E_total": repr(float(E)),
        "converged": bool(out["converged"].all()),
        "iters_hist": np.bincount(out["iters"]).tolist(),
        "sample_index": idx.tolist(),
        "sample_e_frag": [repr(float(x)) for x in out["e_frag"][idx]],
        "oracle_seconds": round(time.time() - t0, 1),
        "workers": workers,
    }
    name = "water40u_oracle_warm.json" if warm else "water40u_oracle.json"
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), name)
    with open(path, "w") as f:
        json.dump(rec, f, indent=1)
    print(path, rec["E_total"], rec["oracle_seconds"], "s")


if __name__ == "__main__":
    main()
