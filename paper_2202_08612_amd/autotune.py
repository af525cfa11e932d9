"""Autotuner of the launch shapes of the triples path.

The library exposes five launch-shape knobs per workspace (``mlcc3_tuning``): the persistent
grid of the d-contraction GEMM, the K split of the N_V-wide back-contraction GEMMs, the block
tile of the N_O-wide back-contraction GEMMs, the form of the contravariant pass and the number
of vectors that share one launch.  None of them changes what is computed.  ``autotune`` times
the caller's own right and left transforms (same problem, vectors and precision) under
candidate settings, one knob at a time starting from the library defaults (coordinate
descent; a candidate must win by more than ``margin``), leaves the workspace set to the
winner and caches it in a JSON file keyed by the sizes, the vector count, the precision and
the GPU architecture, so that later runs on the same shapes skip the timing.
"""
from __future__ import annotations

import json
import os
import time

import torch

from . import mlcc3

# candidate values per knob, in tuning order; 0 is the library default
CANDIDATES = {
    "dc_wg_per_cu": [0, 1, 3, 4, -1],
    "back_ksplit": [0, 1, 2, 4, 8],
    "narrow_tile": [0, 41, 21, 42, 22, 44, 12],
    "contra_form": [0, 1, 2],
    "vec_group": [0, 1, 2, 4, 8, 16],
}


def default_cache_path():
    return os.environ.get("MLCC3_AUTOTUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "mlcc3", "autotune.json"))


def gpu_arch(device=None):
    p = torch.cuda.get_device_properties(device if device is not None else torch.cuda.current_device())
    return str(getattr(p, "gcnArchName", p.name)).split(":")[0]


def cache_key(dims, nvec, precision, arch):
    return (f"{arch}|n_o={dims.n_o},n_v={dims.n_v},N_O={dims.N_O},N_V={dims.N_V},rank={dims.n_chol}"
            f"|nvec={nvec}|{precision}")


def candidates(dims, nvec):
    """Candidate values that can make a difference at these sizes."""
    c = {k: list(v) for k, v in CANDIDATES.items()}
    # the default is the orbit pass when 16 | n_v or n_v > 64, else the per-sub-cube pass
    c["contra_form"] = [0, 1] if (dims.n_v % 16 == 0 or dims.n_v > 64) else [0, 2]
    c["vec_group"] = [v for v in c["vec_group"] if v == 0 or v < nvec]
    return c


def load_cache(path):
    try:
        with open(path) as f:
            db = json.load(f)
        return db if isinstance(db, dict) else {}
    except (OSError, ValueError):
        return {}


def _save_cache(path, db):
    d = os.path.dirname(path)
    if d:
        os.makedirs(d, exist_ok=True)
    tmp = f"{path}.{os.getpid()}.tmp"
    with open(tmp, "w") as f:
        json.dump(db, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def autotune(ws, ground, omega, R, L=None, precision="fp64", cache=None, reps=2, margin=0.01, force=False):
    """Pick the launch shapes for right (and left, if L is given) transforms of the vectors R
    (and L) at frequencies omega.  Returns (tuning, report); ws keeps the chosen tuning."""
    d = ground.dims
    nvec = len(R)
    key = cache_key(d, nvec, precision, gpu_arch(ws.device))
    path = default_cache_path() if cache is None else cache
    db = load_cache(path)
    if key in db and not force:
        tuning = db[key]["tuning"]
        ws.set_tuning(tuning)
        return tuning, dict(db[key], cached=True, key=key)

    # first call prepares the ground-state blocks on this workspace; later calls reuse them
    mlcc3.right_transform(ws, ground, omega, R, precision=precision)

    def run():
        mlcc3.right_transform(ws, ground, omega, R, reuse_ground=True, precision=precision)
        if L:
            mlcc3.left_transform(ws, ground, omega, L, reuse_ground=True, precision=precision)

    def timed(tuning):
        ws.set_tuning(tuning)
        run()                                # warm-up: allocates what this shape needs
        torch.cuda.synchronize(ws.device)
        t0 = time.perf_counter()
        for _ in range(reps):
            run()
        torch.cuda.synchronize(ws.device)
        return (time.perf_counter() - t0) / reps * 1e3

    best = {k: 0 for k in mlcc3.TUNING_FIELDS}
    t_default = t_best = timed(best)
    trials = [{"tuning": dict(best), "ms": t_default}]
    for knob, values in candidates(d, nvec).items():
        for v in values:
            if v == best[knob]:
                continue
            trial = dict(best, **{knob: v})
            t = timed(trial)
            trials.append({"tuning": trial, "ms": t})
            if t < t_best * (1.0 - margin):
                best, t_best = trial, t
    ws.set_tuning(best)
    entry = {"tuning": best, "ms": t_best, "default_ms": t_default, "reps": reps,
             "workload": "right" + (" + left" if L else "") + " transform", "trials": trials,
             "time": time.strftime("%Y-%m-%dT%H:%M:%S")}
    db = load_cache(path)                    # merge with entries written meanwhile
    db[key] = entry
    _save_cache(path, db)
    return best, dict(entry, cached=False, key=key)
