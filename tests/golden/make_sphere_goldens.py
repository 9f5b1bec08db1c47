"""Write the FP64 oracle's time-averaged forces for the full-size 3D sphere workload.

Calls only the oracle (and the seeded workload generator): 256 x 128 x 128
D3Q7, lambda = 256, c0 = 0.5, c_p/c0 = 1.1, R = 12, 2048 Fibonacci points,
30 periods with the last 10 averaged, at the requested positions
kh_j = j (pi/2)/15.  Each position costs about 6.4e10 cell updates on the
host (tens of minutes).

usage: python tests/golden/make_sphere_goldens.py J [J ...]
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

OUT = os.path.join(HERE, "sphere3d_oracle_forces.json")


def main(js):
    lam, c0 = 256.0, 0.5
    cal = oracle.cavity_calibration(256, c0, 2 * math.pi * c0 / lam)
    try:
        with open(OUT) as fh:
            data = json.load(fh)
    except OSError:
        data = {"workload": "3D sphere 256x128x128, lambda=256, c0=0.5, c_p/c0=1.1, R=12, "
                            "N=2048, 30 periods, last 10 averaged",
                "x_mid": cal["x_mid"], "k": cal["k"], "A": cal["A"], "Pa": cal["Pa"],
                "positions": {}}
    khs = workloads.sphere_3d_positions(16)
    for j in js:
        p = workloads.sphere_3d(cal["x_mid"], cal["k"], khs[j])
        t0 = time.time()
        r = oracle.run(p, p["n_steps"])
        data["positions"][str(j)] = {"kh": khs[j], "center": list(p["center"]),
                                     "F_avg": list(r["F_avg"]), "n_acc": r["n_acc"],
                                     "seconds": time.time() - t0}
        with open(OUT, "w") as fh:
            json.dump(data, fh, indent=1)
        print(f"position {j}: F = {r['F_avg']} ({time.time() - t0:.0f} s)", flush=True)


if __name__ == "__main__":
    main([int(a) for a in sys.argv[1:]])
