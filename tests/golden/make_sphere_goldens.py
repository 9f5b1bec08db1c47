"""Write the FP64 oracle's time-averaged forces for the full-size 3D sphere workload.

Calls only the oracle (and the seeded workload generator): 256 x 128 x 128
D3Q7, lambda = 256, c0 = 0.5, c_p/c0 = 1.1, R = 12, 2048 Fibonacci points,
30 periods with the last 10 averaged, at the requested positions
kh_j = j (pi/2)/15.  Each position costs about 6.4e10 cell updates on the
host (tens of minutes).

usage: python tests/golden/make_sphere_goldens.py [--segments K] [--out FILE] J [J ...]
       python tests/golden/make_sphere_goldens.py --merge FILE [FILE ...]
(--segments runs each position as K consecutive pieces of the same run, printing after each,
with the same result bit for bit; --merge adds the positions of other output files.)
"""
import argparse
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


def main(js, out=OUT, segments=0):
    lam, c0 = 256.0, 0.5
    cal = oracle.cavity_calibration(256, c0, 2 * math.pi * c0 / lam)
    try:
        with open(out) as fh:
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
        if segments > 0:
            r = oracle.run_segments(p, p["n_steps"], segments, progress=lambda t: print(
                f"  position {j}: {t} of {p['n_steps']} steps ({time.time() - t0:.0f} s)",
                flush=True))
        else:
            r = oracle.run(p, p["n_steps"])
        data["positions"][str(j)] = {"kh": khs[j], "center": list(p["center"]),
                                     "F_avg": list(r["F_avg"]), "n_acc": r["n_acc"],
                                     "seconds": time.time() - t0}
        with open(out, "w") as fh:
            json.dump(data, fh, indent=1)
        print(f"position {j}: F = {r['F_avg']} ({time.time() - t0:.0f} s)", flush=True)


def merge(files):
    """Add the positions of other output files (same workload and calibration) to OUT."""
    with open(OUT) as fh:
        data = json.load(fh)
    for f in files:
        with open(f) as fh:
            other = json.load(fh)
        for key in ("x_mid", "k", "A", "Pa"):
            assert other[key] == data[key], key
        data["positions"].update(other["positions"])
    data["positions"] = dict(sorted(data["positions"].items(), key=lambda kv: int(kv[0])))
    with open(OUT, "w") as fh:
        json.dump(data, fh, indent=1)


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("--segments", type=int, default=0)
    ap.add_argument("--out", default=OUT)
    ap.add_argument("--merge", nargs="+")
    ap.add_argument("positions", nargs="*", type=int)
    a = ap.parse_args()
    if a.merge:
        merge(a.merge)
    else:
        main(a.positions, a.out, a.segments)
