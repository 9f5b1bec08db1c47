"""MLP surrogate of the time-averaged radiation force, trained on batched LB runs.

The network (include/lb_mlp.h; BF16 MFMA forward, backward and Adam kernels in
csrc/lb_mlp.hip) maps (k R, k h, c_p/c0, 1/R), each mapped linearly from the
training box to [-1, 1], to F / F0 with F0 = pi R^3 Pa^2 k / (3 rho0 c0^2),
the scale of the small-sphere force (eq. ARF_Gorkov_3D): F/F0 -> f1 sin 2kh
as kR -> 0, f1 = 1 - c0^2/c_p^2 for a density-matched sphere.  R is the
radius in lattice cells: at fixed (k R, k h, c_p/c0) the lattice's force
still moves by a few percent between R = 4 and R = 16 cells, so the
resolution is an input (left out, it is scatter the network cannot fit).

Training data come from the batched lattice Boltzmann runs (lbwave.LBWave
with many uneven instances); the same LB stays the reference for the error
and the fallback for queries outside the training box.
"""
from __future__ import annotations

import ctypes as C
import math
import os

import numpy as np

from . import lbwave

# input box mapped to [-1, 1] (the network's nominal domain); the fourth
# input is 1/R with R the radius in cells, R in 4 .. 16
BOX = {"kR": (0.05, 0.6), "kh": (0.0, math.pi / 2), "ratio": (0.8, 1.5),
       "inv_R": (1.0 / 16.0, 1.0 / 4.0)}
# where the network is trusted: the whole input box.  The cubic batch generator cannot make k R
# below 2 pi R_min / edge_max = 2 pi 4 / 192 = 0.131; the training data add draws of k R in
# [0.05, 0.131) in boxes lambda x 64 x 64 (workloads.channel_draws), so the trained network
# covers k R from 0.05.  Queries outside the box go to the LB.
TRUST = {"kR": BOX["kR"], "kh": BOX["kh"], "ratio": BOX["ratio"], "inv_R": BOX["inv_R"]}
N_IN = 4
C0 = 1.0 / 3.0  # fluid sound speed of the batched boxes (keeps c_p <= 0.5 < 1/sqrt(3))
# the LB force data (paper_2404_02346_amd/data): training and held-out sets of both generators
DATA_DIR = os.path.join(os.path.dirname(os.path.abspath(__file__)), "data")
TRAIN_FILES = ("lb_forces_seed2405_n4096.json", "lb_forces_channel_seed2408_n704.json")
TEST_FILES = ("lb_forces_seed2406_n512.json", "lb_forces_channel_seed2409_n88.json")


def data_paths(files):
    """Full paths of data files named in DATA_DIR."""
    return [os.path.join(DATA_DIR, f) for f in files]


def load_sets(files):
    """The data sets of the given files (names in DATA_DIR)."""
    import json
    out = []
    for f in data_paths(files):
        with open(f) as fh:
            out.append(json.load(fh))
    return out


_fp = C.POINTER(C.c_float)


def _mlp_lib():
    L = lbwave.lib()
    if not getattr(L, "_mlp_ready", False):
        vp = C.c_void_p
        L.lb_mlp_num_params.restype = C.c_int32
        L.lb_mlp_workspace_bytes.argtypes = [C.c_int32]
        L.lb_mlp_workspace_bytes.restype = C.c_size_t
        L.lb_mlp_create.argtypes = [C.c_int32, vp, C.c_size_t, vp, C.POINTER(vp)]
        L.lb_mlp_destroy.argtypes = [vp]
        L.lb_mlp_set_params.argtypes = [vp, _fp]
        L.lb_mlp_get_params.argtypes = [vp, _fp]
        L.lb_mlp_forward.argtypes = [vp, vp, C.c_int32, vp]
        L.lb_mlp_forward_layered.argtypes = [vp, vp, C.c_int32, vp]
        L.lb_mlp_grad.argtypes = [vp, vp, vp, C.c_int32, _fp, C.POINTER(C.c_double)]
        L.lb_mlp_train_step.argtypes = [vp, vp, vp, C.c_int32, C.c_float, C.c_float, C.c_float,
                                        C.c_float]
        L.lb_mlp_train_steps.argtypes = [vp, vp, vp, C.c_int32, C.c_int32, _fp, C.c_float,
                                         C.c_float, C.c_float]
        L.lb_mlp_last_loss.argtypes = [vp, C.POINTER(C.c_double)]
        L.lb_mlp_mfma_probe.argtypes = [vp, vp, vp, vp]
        L.lb_mlp_activation.argtypes = [vp, C.c_int64, C.c_int32, vp, vp]
        L._mlp_ready = True
    return L


def num_params() -> int:
    return int(_mlp_lib().lb_mlp_num_params())


DIMS = (N_IN, 256, 256, 256, 256, 1)


def init_params(seed: int) -> np.ndarray:
    """Seeded initial parameters: every weight and bias of a layer ~ U(-1/sqrt(fan_in), 1/sqrt(fan_in)).

    (On the LB force data this small uniform start generalises far better
    than a variance-preserving N(0, 2/fan_in) start: held-out maximum error
    about 0.3% against 2.5% for the same FP32 training.)
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for i in range(len(DIMS) - 1):
        n, k = DIMS[i + 1], DIMS[i]
        bound = 1.0 / math.sqrt(k)
        out.append(rng.uniform(-bound, bound, size=n * k))
        out.append(rng.uniform(-bound, bound, size=n))
    return np.concatenate(out).astype(np.float32)


def _inputs(kR, kh, ratio, R):
    kR, kh, ratio, R = np.broadcast_arrays(*(np.asarray(v, dtype=np.float64)
                                             for v in (kR, kh, ratio, R)))
    return ((kR, "kR"), (kh, "kh"), (ratio, "ratio"), (1.0 / R, "inv_R"))


def normalize(kR, kh, ratio, R) -> np.ndarray:
    """Map (kR, kh, c_p/c0, 1/R) from the training box to [-1, 1]^4 (B x 4 float32)."""
    cols = []
    for v, key in _inputs(kR, kh, ratio, R):
        lo, hi = BOX[key]
        cols.append(2.0 * (v - lo) / (hi - lo) - 1.0)
    return np.stack(cols, axis=-1).astype(np.float32).reshape(-1, N_IN)


def in_box(kR, kh, ratio, R) -> np.ndarray:
    """True where the network is trusted (inside the training box)."""
    cols = _inputs(kR, kh, ratio, R)
    ok = np.ones(cols[0][0].shape, bool)
    for v, key in cols:
        lo, hi = TRUST[key]
        ok &= (v >= lo * (1 - 1e-12)) & (v <= hi * (1 + 1e-12))
    return ok


class MLP:
    """Handle on the GPU network (lb_mlp_create) with a torch workspace and stream."""

    def __init__(self, max_batch: int = 4096, params=None, seed: int = 0, stream=None):
        import torch
        L = _mlp_lib()
        self.max_batch = int(max_batch)
        nb = L.lb_mlp_workspace_bytes(self.max_batch)
        self.ws = torch.empty(nb, dtype=torch.uint8, device="cuda")
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        self._h = C.c_void_p()
        lbwave._check(L.lb_mlp_create(self.max_batch, C.c_void_p(self.ws.data_ptr()), nb,
                                      C.c_void_p(self.stream.cuda_stream), C.byref(self._h)))
        self.set_params(init_params(seed) if params is None else params)

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            _mlp_lib().lb_mlp_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_params(self, p):
        a = np.ascontiguousarray(np.asarray(p, dtype=np.float32))
        assert a.size == num_params()
        lbwave._check(_mlp_lib().lb_mlp_set_params(self._h, a.ctypes.data_as(_fp)))

    def params(self) -> np.ndarray:
        out = np.empty(num_params(), dtype=np.float32)
        lbwave._check(_mlp_lib().lb_mlp_get_params(self._h, out.ctypes.data_as(_fp)))
        return out

    def _dev(self, a, cols=None):
        import torch
        t = torch.as_tensor(np.ascontiguousarray(np.asarray(a, dtype=np.float32)), device="cuda")
        return t if cols is None else t.reshape(-1, cols)

    def forward_dev(self, x_dev, y_dev, B: int, layered: bool = False):
        """y = net(x) on device tensors: the fused inference launch, or the training forward."""
        fn = _mlp_lib().lb_mlp_forward_layered if layered else _mlp_lib().lb_mlp_forward
        lbwave._check(fn(self._h, C.c_void_p(x_dev.data_ptr()), int(B),
                         C.c_void_p(y_dev.data_ptr())))

    def predict(self, x, layered: bool = False, chunk: int = 1 << 22) -> np.ndarray:
        import torch
        x = np.asarray(x, dtype=np.float32).reshape(-1, N_IN)
        out = np.empty(len(x), dtype=np.float32)
        step = self.max_batch if layered else chunk
        for s in range(0, len(x), step):
            xb = self._dev(x[s: s + step], N_IN)
            yb = torch.empty(len(xb), dtype=torch.float32, device="cuda")
            self.forward_dev(xb, yb, len(xb), layered)
            out[s: s + len(xb)] = yb.cpu().numpy()
        return out

    def grad(self, x, t):
        x_d, t_d = self._dev(x, N_IN), self._dev(t)
        g = np.empty(num_params(), dtype=np.float32)
        loss = C.c_double()
        lbwave._check(_mlp_lib().lb_mlp_grad(self._h, C.c_void_p(x_d.data_ptr()),
                                             C.c_void_p(t_d.data_ptr()), len(t_d),
                                             g.ctypes.data_as(_fp), C.byref(loss)))
        return loss.value, g

    def train(self, x, t, steps: int, lr: float = 1e-3, batch: int | None = None, seed: int = 0,
              beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8, lr_final: float = None,
              log_every: int = 0):
        """Adam on the mean squared error; mini-batches drawn with a seeded permutation."""
        import torch
        x = np.asarray(x, dtype=np.float32).reshape(-1, N_IN)
        t = np.asarray(t, dtype=np.float32).reshape(-1)
        n = len(t)
        batch = min(batch or n, self.max_batch, n)
        x_d, t_d = self._dev(x, N_IN), self._dev(t)
        rng = np.random.Generator(np.random.PCG64(seed))
        L = _mlp_lib()
        losses = []
        sched = np.array([lr if lr_final is None else lr * (lr_final / lr) ** (s / max(steps - 1, 1))
                          for s in range(steps)], dtype=np.float32)

        def log(s):
            if log_every and (s % log_every == 0 or s == steps - 1):
                v = C.c_double()
                lbwave._check(L.lb_mlp_last_loss(self._h, C.byref(v)))
                losses.append((s, v.value))

        if batch == n:
            # full batch: the steps between two logged losses go down in one call
            marks = sorted({0, steps} | ({s + 1 for s in range(0, steps, log_every)} | {steps}
                                         if log_every else set()))
            for a, b in zip(marks[:-1], marks[1:]):
                lbwave._check(L.lb_mlp_train_steps(self._h, C.c_void_p(x_d.data_ptr()),
                                                   C.c_void_p(t_d.data_ptr()), n, b - a,
                                                   sched[a:b].ctypes.data_as(_fp), beta1, beta2,
                                                   eps))
                log(b - 1)
            return losses
        order = rng.permutation(n)
        pos = 0
        for s in range(steps):
            if pos + batch > n:
                order, pos = rng.permutation(n), 0
            idx = torch.as_tensor(order[pos: pos + batch], device="cuda")
            pos += batch
            xb, tb = x_d[idx].contiguous(), t_d[idx].contiguous()
            lbwave._check(L.lb_mlp_train_step(self._h, C.c_void_p(xb.data_ptr()),
                                              C.c_void_p(tb.data_ptr()), len(tb), float(sched[s]),
                                              beta1, beta2, eps))
            log(s)
        return losses


def mfma_probe(A_bits: np.ndarray, B_bits: np.ndarray) -> np.ndarray:
    """One 16x16x32 BF16 MFMA tile through the library (lane-layout check)."""
    import torch
    a = torch.as_tensor(np.ascontiguousarray(A_bits.astype(np.int16)), device="cuda")
    b = torch.as_tensor(np.ascontiguousarray(B_bits.astype(np.int16)), device="cuda")
    d = torch.zeros(256, dtype=torch.float32, device="cuda")
    s = torch.cuda.current_stream()
    lbwave._check(_mlp_lib().lb_mlp_mfma_probe(C.c_void_p(a.data_ptr()), C.c_void_p(b.data_ptr()),
                                               C.c_void_p(d.data_ptr()),
                                               C.c_void_p(s.cuda_stream)))
    return d.cpu().numpy().reshape(16, 16)


def activation(z: np.ndarray, derivative: bool = False) -> np.ndarray:
    """The network's GELU (or its derivative) as the library computes it, in FP32."""
    import torch
    zt = torch.as_tensor(np.ascontiguousarray(z, dtype=np.float32).ravel(), device="cuda")
    out = torch.empty_like(zt)
    s = torch.cuda.current_stream()
    lbwave._check(_mlp_lib().lb_mlp_activation(C.c_void_p(zt.data_ptr()), zt.numel(),
                                               int(bool(derivative)), C.c_void_p(out.data_ptr()),
                                               C.c_void_p(s.cuda_stream)))
    return out.cpu().numpy().reshape(np.shape(z))


# ---------------------------------------------------------------------------
# Training data from batched LB runs
# ---------------------------------------------------------------------------

def calibrate_edges(edges, c0: float = C0):
    """GPU cavity calibration per box edge (lambda = edge): antinode, wavenumber, Pa."""
    out = {}
    for e in edges:
        cal = lbwave.cavity_calibrate(int(e), c0, 2 * math.pi * c0 / e)
        out[int(e)] = cal
    return out


def force_scale(R, Pa, lam, c0: float = C0, rho0: float = 1.0):
    """F0 = pi R^3 Pa^2 k / (3 rho0 c0^2) with k = 2 pi / lambda."""
    k = 2 * math.pi / lam
    return math.pi * R ** 3 * Pa ** 2 * k / (3 * rho0 * c0 ** 2)


def run_batch(problems, storage: str = "f32", autotune: bool = True, stream=None,
              graph: int = 64):
    """Run uneven instances in one handle to their own lengths; returns forces and timing."""
    import time

    import torch
    h = lbwave.LBWave(problems, storage=storage, stream=stream, freeze_at_n_steps=True)
    tune = None
    if autotune:
        tune = h.autotune(2)
    h.set_graph(graph)
    n = max(int(p["n_steps"]) for p in problems)
    if graph > 0 and n > 2 * graph:
        # capture and instantiate the replayed step sequence before the clock starts
        h.step(2 * graph + 8)
        h.reset()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    h.step(n)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    F, nacc = h.force()
    variant = tuple(h.variant()) + (h.steps_per_launch(),)
    h.close()
    updates = sum(int(p["nx"]) * int(p["ny"]) * int(p["nz"]) * int(p["n_steps"]) for p in problems)
    return {"F": F, "n_acc": nacc, "seconds": dt, "updates": updates, "variant": variant,
            "autotune_ms": tune}


def generate(seed: int, n: int, cal=None, kr_max: float = 0.6, storage: str = "f32",
             chunk: int = 256, n_periods: int = 30, avg_periods: int = 10, start: int = 0,
             verbose: bool = True):
    """Seeded samples start .. n-1 of the batch generator (k R <= kr_max) with their LB forces.

    The draws are sequential, so samples [a, b) and [b, c) together are
    samples [a, c); every instance runs independently of the others in its
    handle, so the forces do not depend on how the samples are split.
    """
    import workloads
    cal = cal or calibrate_edges(workloads.BATCH_EDGES)
    x_mid = {e: c["x_mid"] for e, c in cal.items()}
    kk = {e: c["k"] for e, c in cal.items()}
    probs, info = workloads.batch(seed, n, x_mid, kk, kr_max=kr_max, n_periods=n_periods,
                                  avg_periods=avg_periods, return_draws=True)
    rows, secs, upd = [], 0.0, 0
    for s in range(start, n, chunk):
        part = probs[s: min(s + chunk, n)]
        r = run_batch(part, storage=storage)
        secs += r["seconds"]
        upd += r["updates"]
        if verbose:
            print(f"batch {s // chunk}: {len(part)} instances, {r['updates']:.3e} updates in "
                  f"{r['seconds']:.1f} s, variant {r['variant']}", flush=True)
        for p, F in zip(part, r["F"]):
            lam = p["lam"]
            R = p["radius"]
            F0 = force_scale(R, cal[int(p["nx"])]["Pa"], lam)
            rows.append({"edge": int(p["nx"]), "R": R, "ratio": p["cp_ratio"], "kh": p["kh"],
                         "kR": 2 * math.pi * R / lam, "F": [float(v) for v in F],
                         "F_over_F0": float(F[0] / F0)})
    return {"seed": seed, "n": n - start, "start": start, "kr_max": kr_max, "storage": storage,
            "rows": rows, "rejected_draws": info["rejected"], "lb_seconds": secs,
            "lb_updates": upd}


def generate_channel(seed: int, n: int, cal=None, storage: str = "f32", chunk: int = 32,
                     start: int = 0, verbose: bool = True):
    """Seeded samples start .. n-1 at small k R (workloads.channel_draws: boxes lambda x 64 x 64,
    k R in [0.05, 2 pi 4/192)) with their LB forces, as generate() does for the cubic boxes."""
    import workloads
    draws, rejected = workloads.channel_draws(seed, n)
    draws = draws[start:]
    cal = dict(cal or {})
    missing = sorted({d[0] for d in draws} - set(cal))
    if missing:
        cal.update(calibrate_edges(missing))
    rows, secs, upd = [], 0.0, 0
    for s in range(0, len(draws), chunk):
        part = draws[s: s + chunk]
        probs = [workloads.channel_problem(d, cal[d[0]]["x_mid"], cal[d[0]]["k"]) for d in part]
        for p in probs:
            if not workloads.geometry_ok(p):
                raise ValueError("channel box cannot hold its object")
        r = run_batch(probs, storage=storage)
        secs += r["seconds"]
        upd += r["updates"]
        if verbose:
            print(f"channel batch {(start + s) // chunk}: {len(part)} instances, "
                  f"{r['updates']:.3e} updates in {r['seconds']:.1f} s", flush=True)
        for p, d, F in zip(probs, part, r["F"]):
            lam, R = d[0], d[1]
            F0 = force_scale(R, cal[lam]["Pa"], lam)
            rows.append({"edge": int(lam), "box": [int(lam), int(p["ny"]), int(p["nz"])],
                         "R": R, "ratio": d[2], "kh": d[3], "kR": 2 * math.pi * R / lam,
                         "F": [float(v) for v in F], "F_over_F0": float(F[0] / F0)})
    return {"seed": seed, "n": n - start, "start": start, "kr_max": 2 * math.pi * 4.0 / 192.0,
            "storage": storage, "generator": "channel", "rows": rows, "rejected_draws": rejected,
            "lb_seconds": secs, "lb_updates": upd}


def merge(parts):
    """Join consecutive sample ranges of one seed (as written by generate) into one data set."""
    parts = sorted(parts, key=lambda d: d.get("start", 0))
    pos = parts[0].get("start", 0)
    for d in parts:
        if d["seed"] != parts[0]["seed"] or d["kr_max"] != parts[0]["kr_max"] \
                or d["storage"] != parts[0]["storage"] or d.get("start", 0) != pos:
            raise ValueError("parts are not consecutive ranges of one seeded data set")
        pos += d["n"]
    rows = [r for d in parts for r in d["rows"]]
    if any(d.get("generator") != parts[0].get("generator") for d in parts):
        raise ValueError("parts come from different generators")
    out = {"generator": parts[0]["generator"]} if "generator" in parts[0] else {}
    return {**out, "seed": parts[0]["seed"], "n": len(rows), "start": parts[0].get("start", 0),
            "kr_max": parts[0]["kr_max"], "storage": parts[0]["storage"], "rows": rows,
            "rejected_draws": parts[-1]["rejected_draws"],
            "lb_seconds": sum(d["lb_seconds"] for d in parts),
            "lb_updates": sum(d["lb_updates"] for d in parts)}


def table(*datasets):
    """Columns (kR, kh, c_p/c0, R in cells, F/F0) over the rows of one or more data sets."""
    rows = [r for d in datasets for r in d["rows"]]
    return tuple(np.array([r[key] for r in rows]) for key in ("kR", "kh", "ratio", "R",
                                                                "F_over_F0"))


def fit(train_sets, steps: int = 16000, lr: float = 2e-3, lr_final: float = 3e-5, seed: int = 0,
        batch: int | None = None, log_every: int = 2000):
    """Train a network on LB data sets with the standard recipe.

    Adam on the mean squared error of F/F0, learning rate decayed
    geometrically from lr to lr_final, full batch unless ``batch`` is given.
    Returns (network, loss log, seconds).
    """
    import time

    import torch
    tr = table(*train_sets)
    net = MLP(max_batch=len(tr[0]), seed=seed)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    log = net.train(normalize(*tr[:4]), tr[4], steps=steps, lr=lr, lr_final=lr_final,
                    batch=batch, log_every=log_every)
    torch.cuda.synchronize()
    return net, log, time.perf_counter() - t0


def closed_form_ratio(kh, ratio):
    """Small-sphere limit of F/F0 for a density-matched sphere: f1 sin 2kh, f1 = 1 - 1/ratio^2."""
    return (1.0 - 1.0 / np.asarray(ratio) ** 2) * np.sin(2 * np.asarray(kh))


def error_metric(pred, ref):
    """max |pred - ref| / max |ref| over the set and its RMS counterpart, plus the
    plain relative error max |pred - ref| / |ref| over the samples with
    |ref| >= 0.2 max |ref| (away from the zeros of the force)."""
    pred, ref = np.asarray(pred, dtype=np.float64), np.asarray(ref, dtype=np.float64)
    scale = np.abs(ref).max()
    e = np.abs(pred - ref) / scale
    big = np.abs(ref) >= 0.2 * scale
    rel = np.abs(pred - ref)[big] / np.abs(ref[big])
    return {"max": float(e.max()), "rms": float(np.sqrt(np.mean(e ** 2))),
            "rel_max_large": float(rel.max()), "n_large": int(big.sum())}


class Surrogate:
    """Trained network with the plain LB as fallback outside the training box.

    A fallback query runs a box of length lambda = 2 pi R / kR cells
    (rounded, at least min_edge), so that it keeps the requested resolution R
    as closely as the integer length allows, and of cross-section
    width x width cells: the paper's L_y = L_z = 64 (Sec. Results and
    discussion), or the length if that is smaller.  The sphere and its
    integration surface (radius R + 2, kernel reach 1.5) fit across 64 cells
    for every R <= 16.
    """

    def __init__(self, mlp: MLP, min_edge: int = 32, width: int = 64, cal=None):
        self.mlp = mlp
        self.min_edge = min_edge
        self.width = width
        self.cal = dict(cal or {})

    def predict(self, kR, kh, ratio, R):
        """F/F0 for each query (R in cells); LB runs for the queries outside the box."""
        import workloads
        kR, kh, ratio, R = (np.atleast_1d(v) for v in
                            np.broadcast_arrays(*(np.asarray(v, dtype=np.float64)
                                                  for v in (kR, kh, ratio, R))))
        ok = in_box(kR, kh, ratio, R)
        out = np.empty(kR.shape)
        if ok.any():
            out[ok] = self.mlp.predict(normalize(kR[ok], kh[ok], ratio[ok], R[ok]))
        bad = np.where(~ok)[0]
        if len(bad):
            edges = [max(self.min_edge, int(round(2 * math.pi * R[i] / kR[i]))) for i in bad]
            missing = sorted(set(edges) - set(self.cal))
            if missing:
                self.cal.update(calibrate_edges(missing))
            probs = []
            for i, e in zip(bad, edges):
                c = self.cal[e]
                w = min(e, self.width)
                p = workloads.sphere_3d(c["x_mid"], c["k"], float(kh[i]), shape=(e, w, w),
                                        lam=float(e), R=float(kR[i] * e / (2 * math.pi)),
                                        cp_ratio=float(ratio[i]), n_surf=2048, c0=C0)
                if not workloads.geometry_ok(p):
                    raise ValueError(f"fallback box {e} x {w} x {w} cannot hold R = "
                                     f"{p['radius']:.2f} with its integration surface")
                probs.append(p)
            r = run_batch(probs, autotune=False)
            for j, (i, e) in enumerate(zip(bad, edges)):
                out[i] = r["F"][j, 0] / force_scale(probs[j]["radius"], self.cal[e]["Pa"],
                                                     float(e))
        return out, ~ok
