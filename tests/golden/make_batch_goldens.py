"""Write the FP64 oracle's forces for selected instances of the seeded uneven batch.

Calls only the oracle and the seeded workload generator.  The batch is the
seed-2404 draw of cubic boxes (edge in {64, 96, 128, 192} = lambda,
R ~ U[4, 16], c_p/c0 ~ U[0.8, 1.5], kh ~ U[0, pi/2], c0 = 1/3), objects
placed from the oracle's cavity calibration; each selected instance runs 30
periods with the last 10 averaged.

usage: python tests/golden/make_batch_goldens.py I [I ...]   (instance indices)
"""
import json
import math
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
import workloads  # noqa: E402

OUT = os.path.join(HERE, "batch2404_oracle_forces.json")
SEED, N = 2404, 256


def main(idx):
    c0 = workloads.BATCH_C0
    cal = {e: oracle.cavity_calibration(e, c0, 2 * math.pi * c0 / e) for e in workloads.BATCH_EDGES}
    probs = workloads.batch(SEED, N, {e: c["x_mid"] for e, c in cal.items()},
                            {e: c["k"] for e, c in cal.items()})
    try:
        with open(OUT) as fh:
            data = json.load(fh)
    except OSError:
        data = {"seed": SEED, "n": N, "instances": {}}
    for i in idx:
        p = probs[i]
        t0 = time.time()
        r = oracle.run(p, p["n_steps"])
        data["instances"][str(i)] = {
            "edge": p["nx"], "radius": p["radius"], "cp_ratio": p["cp_ratio"], "kh": p["kh"],
            "center": list(p["center"]), "n_steps": p["n_steps"], "avg_start": p["avg_start"],
            "F_avg": list(r["F_avg"]), "n_acc": r["n_acc"], "seconds": time.time() - t0}
        with open(OUT, "w") as fh:
            json.dump(data, fh, indent=1)
        print(f"instance {i} (edge {p['nx']}): F = {r['F_avg']} ({time.time() - t0:.0f} s)",
              flush=True)


if __name__ == "__main__":
    main([int(a) for a in sys.argv[1:]])
