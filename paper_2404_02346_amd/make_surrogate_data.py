"""Generate lattice Boltzmann force data for the surrogate on the GPU.

Seeded draws of the uneven batch generator (cubic boxes with edge in
{64, 96, 128, 192} = lambda, R ~ U[4, 16], c_p/c0 ~ U[0.8, 1.5],
kh ~ U[0, pi/2], c0 = 1/3) are kept when k R <= kr_max, run to 30 drive
periods in batched handles (last 10 averaged) and written as JSON rows
(edge, R, kR, kh, ratio, F, F/F0).

usage: python -m paper_2404_02346_amd.make_surrogate_data --seed 2405 --n 4096 --out FILE
       (samples 0 .. n-1; --start S writes samples S .. n-1 only)
       python -m paper_2404_02346_amd.make_surrogate_data --merge PART... --out FILE
       (joins consecutive ranges of one seed, e.g. runs split to bound their length)
       python -m paper_2404_02346_amd.make_surrogate_data --channel --seed S --n N --out FILE
       (small k R in [0.05, 2 pi 4/192): boxes lambda x 64 x 64, workloads.channel_draws)
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--seed", type=int)
    ap.add_argument("--n", type=int)
    ap.add_argument("--start", type=int, default=0)
    ap.add_argument("--merge", nargs="+")
    ap.add_argument("--kr-max", type=float, default=0.6)
    ap.add_argument("--chunk", type=int, default=256)
    ap.add_argument("--storage", default="f32")
    ap.add_argument("--channel", action="store_true",
                    help="small-kR draws in boxes lambda x 64 x 64 instead of the cubic batch")
    ap.add_argument("--out", required=True)
    a = ap.parse_args()
    from paper_2404_02346_amd import surrogate as S
    if a.merge:
        parts = []
        for f in a.merge:
            with open(f) as fh:
                parts.append(json.load(fh))
        data = S.merge(parts)
        data["wall_seconds"] = sum(d.get("wall_seconds", 0.0) for d in parts)
    else:
        if a.seed is None or a.n is None:
            ap.error("--seed and --n are required unless --merge is given")
        import torch
        torch.cuda.set_device(0)
        t0 = time.time()
        if a.channel:
            data = S.generate_channel(a.seed, a.n, storage=a.storage, chunk=min(a.chunk, 32),
                                      start=a.start)
        else:
            data = S.generate(a.seed, a.n, kr_max=a.kr_max, storage=a.storage, chunk=a.chunk,
                              start=a.start)
        data["wall_seconds"] = time.time() - t0
    os.makedirs(os.path.dirname(os.path.abspath(a.out)), exist_ok=True)
    with open(a.out, "w") as fh:
        json.dump(data, fh, indent=0)
    print(json.dumps({k: v for k, v in data.items() if k != "rows"}), flush=True)


if __name__ == "__main__":
    main()
