"""The persisted launch tuning (host logic, no GPU): the first run of a
workload times the candidates and stores the fastest under a key of the
architecture, arithmetic, N, P, shots, mesh size and candidate count; a
second run applies the stored choice without timing; another workload
times again; a stored index out of range is ignored."""
import json

import numpy as np

from paper_1610_05023_amd import tuning


class FakeSolver:
    def __init__(self, N=4, P=6, precision=0, shots=1, K=384000, count=12, best=7):
        self.counts = {"N": N, "P": P, "n_shots": shots, "K": K}
        self.precision, self.device = precision, 0
        self._count, self._best = count, best
        self.timed, self.applied = 0, None

    def tuning_count(self):
        return self._count

    def autotune(self, launches):
        self.timed += 1
        ms = np.linspace(1.0, 2.0, self._count)
        ms[self._best] = 0.5
        self.applied = self._best
        return self._best, ms

    def set_tuning(self, c):
        self.applied = c


def test_tuning_is_stored_and_reused(tmp_path, monkeypatch):
    monkeypatch.setattr(tuning, "_arch", lambda dev: "gfx950")
    path = str(tmp_path / "tune.json")
    a = FakeSolver()
    best, ms, cached = tuning.tune(a, path)
    assert (best, cached, a.timed) == (7, False, 1) and ms[7] == 0.5
    b = FakeSolver(best=3)                      # same workload: the stored choice
    best, ms, cached = tuning.tune(b, path)
    assert (best, cached, b.timed, b.applied) == (7, True, 0, 7) and ms is None
    c = FakeSolver(N=5, best=2)                 # another workload: timed
    best, _, cached = tuning.tune(c, path)
    assert (best, cached, c.timed) == (2, False, 1)
    data = json.load(open(path))
    assert len(data) == 2 and all(k.startswith("gfx950|fp64|") for k in data)
    # a library with fewer candidates than the stored index times again
    d = FakeSolver(count=6, best=1)
    data[tuning.cache_key(d, "gfx950")] = {"candidate": 9}
    json.dump(data, open(path, "w"))
    best, _, cached = tuning.tune(d, path)
    assert (best, cached, d.timed) == (1, False, 1)
