"""Write tests/golden/water40u_oracle.json from the CPU oracle only.

Full MBE(3) energy of configuration 1 (water40u, 89969 fragments), its
update-count histogram and every 1000th fragment energy, computed by
oracle.run with a process pool.  Usage:
    python tests/golden/make_golden.py [workers]
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
    workers = int(sys.argv[1]) if len(sys.argv) > 1 else os.cpu_count()
    t0 = time.time()
    prob = synth.config(1)
    out = oracle.run(prob, workers=workers)
    E, _ = oracle.mbe3_energy(prob.frags, out["e_frag"])
    idx = np.arange(0, prob.n_frag, 1000)
    rec = {
        "workload": "configuration 1 (water40u)",
        "n_frag": int(prob.n_frag),
        "E_total": repr(float(E)),
        "converged": bool(out["converged"].all()),
        "iters_hist": np.bincount(out["iters"]).tolist(),
        "sample_index": idx.tolist(),
        "sample_e_frag": [repr(float(x)) for x in out["e_frag"][idx]],
        "oracle_seconds": round(time.time() - t0, 1),
        "workers": workers,
    }
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "water40u_oracle.json")
    with open(path, "w") as f:
        json.dump(rec, f, indent=1)
    print(path, rec["E_total"], rec["oracle_seconds"], "s")


if __name__ == "__main__":
    main()
