"""Persisted launch tuning of the 3D level.

dgh_autotune times every launch candidate of a bound context on its own
workload; this keeps the result in a JSON file keyed by what the choice
depends on -- the GPU architecture, the arithmetic (FP64, FP32 or BF16
contractions), the degree N, the HABC order P, the number of shots, the
number of tetrahedra and the candidate count of the library -- so that a
later run of the same workload applies the stored choice without timing.
"""
from __future__ import annotations

import json
import os
import tempfile

PRECISION = {0: "fp64", 2: "fp32", 3: "bf16"}


def default_path():
    return os.environ.get("DGHABC_TUNING_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "dghabc",
                                       "tuning.json"))


def cache_key(solver, arch):
    k = solver.counts
    return (f"{arch}|{PRECISION.get(solver.precision, solver.precision)}|N{k['N']}|P{k['P']}"
            f"|shots{k['n_shots']}|K{k['K']}|cands{solver.tuning_count()}")


def _arch(device):
    import torch
    return torch.cuda.get_device_properties(device).gcnArchName.split(":")[0]


def load(path):
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def tune(solver, path=None, launches=10):
    """Applies the stored candidate for this workload, or times them all
    (dgh_autotune), applies the fastest and stores it.  Returns (candidate,
    ms per launch of every candidate or None when taken from the file,
    cached flag)."""
    path = path or default_path()
    key = cache_key(solver, _arch(solver.device))
    cache = load(path)
    rec = cache.get(key)
    if rec is not None and 0 <= int(rec["candidate"]) < solver.tuning_count():
        solver.set_tuning(int(rec["candidate"]))
        return int(rec["candidate"]), None, True
    best, ms = solver.autotune(launches)
    cache = load(path)                     # merge with writes made meanwhile
    cache[key] = {"candidate": int(best), "ms_per_launch": [float(v) for v in ms],
                  "launches": int(launches)}
    os.makedirs(os.path.dirname(os.path.abspath(path)), exist_ok=True)
    fd, tmp = tempfile.mkstemp(dir=os.path.dirname(os.path.abspath(path)), suffix=".tmp")
    with os.fdopen(fd, "w") as f:
        json.dump(cache, f, indent=1, sort_keys=True)
    os.replace(tmp, path)
    return int(best), ms, False
