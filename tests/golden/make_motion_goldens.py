"""Write the FP64 oracle's time-averaged force on a small sphere at nine positions, the reference
for the particle-motion test.

Calls only the oracle (and the seeded workload layout): a cubic box of edge 60 = lambda, D3Q7,
c0 = 1/3, sphere R = 4 cells (k R = 2 pi 4/60 = 0.419) with c_p/c0 = 1.2, 2048 Fibonacci
points on R_s = R + 2, at kh_j = j (pi/2)/8, j = 0..8, measured from the central antinode of
the oracle's own cavity calibration; 30 periods with the last 10 averaged.  The amplitude Pa =
c0^2 A of the calibration is stored with the forces.

usage: python tests/golden/make_motion_goldens.py
"""
import json
import math
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
import workloads  # noqa: E402

OUT = os.path.join(HERE, "motion_sphere60_oracle_forces.json")
EDGE, C0, R, RATIO, N_POS = 60, 1.0 / 3.0, 4.0, 1.2, 9


def main():
    lam = float(EDGE)
    cal = oracle.cavity_calibration(EDGE, C0, 2 * math.pi * C0 / lam)
    data = {"workload": f"cubic box {EDGE}^3, lambda = {EDGE}, c0 = 1/3, R = {R}, c_p/c0 = {RATIO}, "
                        "N = 2048, 30 periods, last 10 averaged",
            "edge": EDGE, "c0": C0, "R": R, "cp_ratio": RATIO, "lam": lam,
            "x_mid": cal["x_mid"], "k": cal["k"], "A": cal["A"], "Pa": cal["Pa"], "positions": []}
    for j in range(N_POS):
        kh = j * (math.pi / 2) / (N_POS - 1)
        p = workloads.sphere_3d(cal["x_mid"], cal["k"], kh, shape=(EDGE, EDGE, EDGE), lam=lam, R=R,
                                cp_ratio=RATIO, n_surf=2048, c0=C0)
        assert workloads.geometry_ok(p)
        t0 = time.time()
        r = oracle.run(p, p["n_steps"])
        data["positions"].append({"kh": kh, "center": list(p["center"]), "F_avg": list(r["F_avg"]),
                                  "n_acc": r["n_acc"], "seconds": time.time() - t0})
        with open(OUT, "w") as fh:
            json.dump(data, fh, indent=1)
        print(f"kh_{j} = {kh:.4f}: F = {r['F_avg']} ({time.time() - t0:.0f} s)", flush=True)


if __name__ == "__main__":
    main()
