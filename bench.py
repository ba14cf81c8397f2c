#!/usr/bin/env python3
"""Throughput of the FP64 DG + HABC time step on one MI355X.

Workload: a 40^3 x 6 = 384,000-tet Kuhn mesh of the unit cube, degree N = 4
(Np = 35), HABC order P = 6 on all six faces with edge and corner
compatibility, five random horizontal layers (seed 2), a Ricker point source
near the centre.  A step is five Runge-Kutta stages, each running the volume,
face, edge and corner levels (all of the step); inputs are resident in HBM
before the timed region.

Prints one JSON line: DOF-updates/s per RK stage (the paper's unknown count
over all levels), the roofline of the dominant (3D) kernel from HIP events
recorded by the library around each of its launches in the timed region,
and the FP64 CPU oracle timed on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, nominal
METRIC = "DOF-updates/s per RK stage (FP64 vs mixed/batched) + fraction of HBM roofline"


def bytes_per_tet_stage(Np, word=8):
    """Algorithmic HBM bytes of the 3D level per tet per stage: q and res read
    and written (16 Np words of `word` bytes), 27 per-tet FP64 constants, 20
    bytes of connectivity."""
    return 16 * Np * word + 27 * 8 + 20


def bytes_per_stage(K, Ktri, Klin, N, P, word3=8, shots=1):
    """Algorithmic HBM bytes of one RK stage over all levels: the 3D level as
    above; per triangle q2 and res2 read and written (4 P 3 Np2 FP64 words)
    and 4 coupling words per node (the new 3D trace read, qb3 and q0_3
    written); per line q1 and res1 read and written (4 P^2 2 Np1 words).
    Per-tet constants are counted once per shot (the kernels re-read them
    per shot)."""
    Np = (N + 1) * (N + 2) * (N + 3) // 6
    Np2 = (N + 1) * (N + 2) // 2
    Np1 = N + 1
    b3 = K * bytes_per_tet_stage(Np, word3)
    b2 = Ktri * (4 * P * 3 * Np2 + 4 * Np2) * 8
    b1 = Klin * 4 * P * P * 2 * Np1 * 8
    return (b3 + b2 + b1) * shots


TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "k_level3_layered40_traffic.txt")
KERNEL3_SOURCES = ["levels_fp64.hip", "kernels.hpp", "levels.hpp"]


def profiled_traffic():
    """HBM bytes per launch of the 3D kernel on the 40^3 workload, from the
    committed rocprofv3 FETCH_SIZE / WRITE_SIZE summary (scaled by the
    calibration recorded there); None once the kernel sources differ from
    the ones the counters were taken with."""
    import hashlib
    try:
        fields = {}
        for line in open(TRAFFIC_PROFILE).read().splitlines():
            key, sep, val = line.partition(": ")
            if sep and key in ("traffic_bytes_per_launch_k_level3", "source_sha256"):
                fields[key] = val.strip()
    except OSError:
        return None
    h = hashlib.sha256()
    for f in KERNEL3_SOURCES:
        with open(os.path.join(ROOT, "paper_1610_05023_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    if fields.get("source_sha256") != h.hexdigest() or "traffic_bytes_per_launch_k_level3" not in fields:
        return None
    return float(fields["traffic_bytes_per_launch_k_level3"])


def kernel_name(prec, N, tuned):
    """The 3D kernel a launch runs: the tile-on-chip kernel where the tile
    fits (FP64 N <= 4, FP32 and BF16 N <= 5) unless tuning chose register
    streaming (launch candidates 6 and above there)."""
    base = {0: "k_level3", 2: "k_level3_f32", 3: "k_level3_bf16"}[prec]
    on_chip = N <= (4 if prec == 0 else 5)
    cand = tuned.get("candidate", 0) if isinstance(tuned, dict) else 0
    return base + "_dma" if on_chip and cand < 6 else base


def achieved_gbs(alg_bytes, avg_ms):
    return alg_bytes / (avg_ms * 1e-3) / 1e9


def build_workload(n=40, N=4, P=6):
    import numpy as np
    import workloads as w
    cfg = w.config("2")
    VX, E = w.kuhn_mesh(n)
    rho, c, *_ = w.layered_medium(n, seed=2)
    h = 1.0 / n
    xs = (0.5 + 0.3 * h, 0.5 + 0.2 * h, 0.5 + 0.1 * h)
    f0 = float(w.source_material(n, xs, c)) / (10.0 * h)
    dt = w.kuhn_dt(n, N, float(c.max()))
    return dict(VX=VX, E=E, rho=rho, c=c, xs=xs, f0=f0, t0=1.25 / f0, dt=dt, n=n, N=N, P=P,
                cfg=cfg)


def build_batch_workload(n=20, N=4, P=3, shots=64):
    """Many independent shots on one mesh: 20^3 x 6 = 48,000 tets, N = 4,
    HABC P = 3 on all faces, rho = c = 1, one Ricker source per shot at a
    random interior position (seed 4), f0 = 2, t0 = 0.625."""
    import numpy as np
    import workloads as w
    VX, E = w.kuhn_mesh(n)
    K = E.shape[0]
    return dict(VX=VX, E=E, rho=np.ones(K), c=np.ones(K), xs=w.shot_positions(shots, seed=4),
                f0=2.0, t0=0.625, dt=w.kuhn_dt(n, N, 1.0), n=n, N=N, P=P, shots=shots)


def run_uneven(args):
    """Uneven batch: meshes of 10^3, 16^3 and 24^3 cells (x 6 tets), N = 4,
    HABC P = 3, rho = c = 1, one Ricker source each at a seeded interior
    position, FP64 or the FP32 or BF16 variant (--precision); stepped as one group
    (one 3D launch per stage over all their tiles) and, for comparison, one
    after the other."""
    import numpy as np
    import torch
    import workloads as w
    from paper_1610_05023_amd import Solver
    from paper_1610_05023_amd.binding import step_group
    N, P, sizes = 4, 3, (10, 16, 24)
    prec = {"fp64": 0, "fp32": 2, "bf16": 3}[args.precision]
    name = {0: "FP64", 2: "FP32", 3: "BF16-contraction"}[prec]
    solvers, U = [], 0
    xs = w.shot_positions(len(sizes), seed=6)
    for j, n in enumerate(sizes):
        VX, E = w.kuhn_mesh(n)
        K = E.shape[0]
        s = Solver(VX, E, N, P, np.ones(K), np.ones(K), precision=prec).bind()
        s.set_source(xs[j], 2.0, 0.625)
        k = s.counts
        U += w.n_unknowns(k["K"], k["Ktri"], k["Klin"], N, P)
        solvers.append(s)
    dt = w.kuhn_dt(max(sizes), N, 1.0)
    step_group(solvers, args.warmup, dt, 0.0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    step_group(solvers, args.steps, dt, args.warmup * dt)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    t0 = time.perf_counter()
    for s in solvers:
        s.step(args.steps, dt, (args.warmup + args.steps) * dt)
    torch.cuda.synchronize()
    el_sep = time.perf_counter() - t0
    finite = all(s.check()[0] == "DGH_OK" for s in solvers)
    print(f"[bench] uneven group: {args.steps} steps in {el:.3f} s; one after the other "
          f"{el_sep:.3f} s; check={finite}", file=sys.stderr, flush=True)
    out = {
        "metric": METRIC, "value": U * 5 * args.steps / el, "unit": "DOF-updates/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": el / args.steps * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": {0: "f64", 2: "f32", 3: "bf16"}[prec], "data": "synthetic",
        "config": {"workload": f"uneven group: {name} DG+HABC steps of "
                               "three Kuhn meshes of "
                               "10^3, 16^3 and 24^3 cells x 6 tets stepped together, N=4, HABC "
                               "P=3, rho=c=1, one Ricker source each (seed 6)",
                   "unknowns": U, "dt": dt, "parallelism": "single GPU",
                   "separate_ms_per_step": el_sep / args.steps * 1e3,
                   "group_speedup": el_sep / el},
        "roofline": None, "cpu_baseline": None,
    }
    print(json.dumps(out))


def run_reflection(args):
    """Accuracy of the absorbing boundary at full size.  The 40^3 x 6-tet
    layered case with its Ricker source is run with HABC P = 6 and P = 3 and
    with the basic ABC (P = 0).  The reference is the doubled domain [-0.5, 1.5]^3
    (80^3 x 6 tets, the same cell size, layers extended sideways and the
    bottom and top layers downwards and upwards, HABC P = 6).  All three are
    stepped to t = 0.45.  The waves reach the unit cube's faces from
    t = 0.17; what the reference's own boundary reflects cannot come back
    into the unit cube before t = 0.5.  Reports the relative l2 error of q3
    over the unit cube.  With --closure the learned closure is trained first
    and evaluated on the same case with P = 0.  The teacher runs are P = 6
    runs of Gaussian pulses, always at this case's N and time step, so that
    the network's history of step ends spans the same time as in use.
    --teacher small uses the test's small recipe (six pulses on 8^3 x 6
    tets, c = 1); --teacher case uses four pulses on this case's own mesh
    and medium, centred away from the source; --teacher parity uses 200
    runs of the 8^3 x 6-tet parity case (N = 3, HABC P = 3, rho = c = 1,
    Gaussian pulse of width 0.05) at seeded random centres, each at that
    case's own time step to t = 1, and trains with the BF16 gradient
    (FP32 master weights)."""
    import numpy as np
    import torch
    import workloads as w
    from paper_1610_05023_amd import Solver
    cfg = w.config("2")
    n, N, dt = cfg.n, cfg.N, cfg.dt
    steps = int(round(0.45 / dt))
    _, _, cuts, cvals, rvals = w.layered_medium(n, seed=2)

    def medium(m, shift):
        k = (np.arange(6 * m ** 3) // 6) // (m * m)          # cell layer of each element
        layer = np.searchsorted(cuts, np.clip(k - shift, 0, n - 1), side="right")
        return rvals[layer].copy(), cvals[layer].copy()

    # the closure's time scales: the library's default for this case's mesh
    # (1.25, 2.5, 5, 10 cell crossings at the fastest speed), shared by the
    # teacher runs and the evaluation
    tau = [1.25 * 2 ** k * (1.0 / n) / float(cvals.max()) for k in range(4)]

    def run(VX, E, rho, c, P, label, closure=None):
        t0 = time.perf_counter()
        s = Solver(VX, E, N, P, rho, c).bind()
        if closure is not None:
            s.set_closure_memory(tau)
            s.set_closure(closure)
        s.set_source(cfg.source, cfg.f0, cfg.t0)
        done = 0
        while done < steps:
            k = min(1000, steps - done)
            s.step(k, dt, done * dt)
            done += k
            torch.cuda.synchronize()
            print(f"[bench] reflection {label}: {done}/{steps} steps, "
                  f"{time.perf_counter() - t0:.1f} s", file=sys.stderr, flush=True)
        q3 = s.read_fields(["q3"])["q3"]
        s.close()
        return q3

    VX, E = w.kuhn_mesh(n)
    rho, c = medium(n, 0)
    inner = {f"P={P}": run(VX, E, rho, c, P, f"P={P}") for P in (6, 3, 0)}
    if args.closure:
        from paper_1610_05023_amd.closure import teacher_samples, train
        t0 = time.perf_counter()
        print(f"[bench] reflection: training the closure ({args.teacher} teacher runs)",
              file=sys.stderr, flush=True)
        train_kw = dict(iters=2500, batch=4096, lr=1e-3, seed=5)
        if args.teacher == "parity":
            c1 = w.config("1")
            VXt, Et = w.kuhn_mesh(c1.n)
            Kt = Et.shape[0]
            steps1 = int(round(1.0 / c1.dt))
            every = int(round(0.04 / c1.dt))
            X, Y = teacher_samples(VXt, Et, c1.N, c1.P, np.ones(Kt), np.ones(Kt), c1.dt,
                                   np.random.default_rng(11).uniform(0.25, 0.75, size=(200, 3)),
                                   c1.extra["width"], steps=steps1, every=every,
                                   start=int(round(0.2 / c1.dt)), tau=tau)
            train_kw = dict(iters=6000, batch=16384, lr=1e-3, seed=5, bf16=True)
        elif args.teacher == "small":
            nt = 8
            VXt, Et = w.kuhn_mesh(nt)
            Kt = Et.shape[0]
            dt_small = w.kuhn_dt(nt, 3, 1.0)          # the time step of the small recipe
            every = int(round(10 * dt_small / dt))
            X, Y = teacher_samples(VXt, Et, N, 6, np.ones(Kt), np.ones(Kt), dt,
                                   np.random.default_rng(5).uniform(0.3, 0.7, size=(6, 3)),
                                   0.15, steps=int(round(700 * dt_small / dt)), every=every,
                                   start=6 * every, tau=tau)
        else:
            # the case's own mesh and medium with P = 6: Gaussian pulses (width
            # 0.08, about the source's wavelength) at seeded interior centres
            # other than the source's, to the same time
            X, Y = teacher_samples(VX, E, N, 6, rho, c, dt,
                                   np.random.default_rng(7).uniform(0.25, 0.75, size=(4, 3)),
                                   0.08, steps=steps, every=400, start=400, tau=tau)
        wts, losses = train(X, Y, log_every=train_kw["iters"] // 4, **train_kw)
        print(f"[bench] reflection: losses {[(t, f'{l:.3e}') for t, l in losses]}, target "
              f"mean square {float(np.mean(Y.astype(np.float64) ** 2)):.3e}",
              file=sys.stderr, flush=True)
        print(f"[bench] reflection: closure trained on {len(Y)} samples in "
              f"{time.perf_counter() - t0:.1f} s", file=sys.stderr, flush=True)
        inner["closure"] = run(VX, E, rho, c, 0, "closure", closure=wts)
    m = 2 * n
    VXo, Eo = w.kuhn_mesh(m, lo=(-0.5,) * 3, hi=(1.5,) * 3)
    rho_o, c_o = medium(m, n // 2)
    ref = run(VXo, Eo, rho_o, c_o, 6, "reference")
    e = np.arange(6 * n ** 3)
    cell, t = e // 6, e % 6
    i, j, k = cell % n, (cell // n) % n, cell // (n * n)
    eo = (((k + n // 2) * m + (j + n // 2)) * m + (i + n // 2)) * 6 + t
    r = ref[eo]
    err = {k: float(np.linalg.norm(q - r) / np.linalg.norm(r)) for k, q in inner.items()}
    print(json.dumps({"workload": "reflection: 40^3 x 6 layered case with its Ricker source "
                                  "against the doubled domain [-0.5, 1.5]^3 (80^3 x 6 tets, "
                                  "HABC P=6), t = 0.45",
                      "steps": steps, "dt": dt,
                      "teacher": args.teacher if args.closure else None,
                      "relative_l2_error_q3_unit_cube": err,
                      "reference_q3_norm": float(np.linalg.norm(r))}))


def run_validation(args):
    """Section 4.1's validation benchmark on a Kuhn stand-in for the paper's
    70,895-tet mesh: 23^3 x 6 = 73,002 tets of [-0.5, 0.5]^3, N = 3,
    rho = c = 1, the Ricker source (f0 = 2.5, t0 = 0.5) at the centre and at
    (0.2, 0.1, 0), HABC orders 0 (the basic ABC), 2, 4, ..., 12 on all six
    faces (or, with --free-surface, p = 0 on z = 0.5 and HABC on the other
    five faces, against the image solution), stepped on the GPU in FP64 to
    t = --t-final.  Error(t) is the paper's relative energy norm against the
    free-space (or image) solution, with the Dirichlet run's energy as
    denominator, both integrated by a degree-7 quadrature on every tet.
    Prints one JSON line with the curves (every --sample time units)."""
    import numpy as np
    import workloads as w
    from paper_1610_05023_amd.validation import run_benchmark
    n, N = args.valid_n, 3
    VX, E = w.kuhn_mesh(n, lo=(-0.5,) * 3, hi=(0.5,) * 3)
    dt = w.kuhn_dt(n, N, 1.0)
    orders = tuple(int(v) for v in args.orders.split(","))
    extra = {}
    if args.matched and 3 not in orders:
        orders = tuple(sorted(orders + (3,)))     # the Pade condition of the same order
    if args.matched:
        # coefficients making the P = 3 condition exact at 20, 38 and 52
        # degrees, the incidences a centred source produces on the faces
        from paper_1610_05023_amd.habc_params import angle_matched_gamma
        extra["P=3 matched 20,38,52 deg"] = (3, angle_matched_gamma(np.radians([20, 38, 52])))
    t_start = time.perf_counter()
    res = run_benchmark(VX, E, dt, N=N, orders=orders, free_surface=args.free_surface,
                        t_final=args.t_final, sample=args.sample, extra=extra,
                        log=lambda m: print(f"[bench] validation {m}", file=sys.stderr,
                                            flush=True))
    labels = [(P, f"P={P}") for P in orders] + [(k, k) for k in extra]
    out = {"workload": ("validation benchmark, Section 4.1: " + (
        "free surface p = 0 on z = 0.5, HABC on the other faces, image solution"
        if args.free_surface else "HABC on all faces, free-space solution") +
        f"; Kuhn mesh {n}^3 x 6 = {E.shape[0]} tets of [-0.5, 0.5]^3, N = {N}, rho = c = 1, "
        "Ricker f0 = 2.5, t0 = 0.5, FP64"), "dt": dt, "orders": list(orders),
        "wall_s": time.perf_counter() - t_start, "sources": {}}
    for xs, rec in res.items():
        curves = {lab: [round(float(v), 6) for v in rec[key]] for key, lab in labels}
        summary = {}
        for key, lab in labels:
            e = np.array(rec[key])
            tt = np.array(rec["times"])
            after = tt >= 1.0
            summary[lab] = {"error_at_t1": float(np.interp(1.0, tt, e)),
                                 "min_after_t1": float(e[after].min()),
                                 "t_of_min": float(tt[after][np.argmin(e[after])]),
                                 "max_after_t1": float(e[after].max()),
                                 "final": float(e[-1])}
        out["sources"][str(list(xs))] = {"E_src": rec["E_src"],
                                         "E_src_library": rec["E_src_library"],
                                         "times": [round(float(t), 6) for t in rec["times"]],
                                         "error": curves, "summary": summary}
    print(json.dumps(out))


def _host_cpu():
    """Host CPU count and model (as the kernel reports them)."""
    model = None
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return os.cpu_count(), model


def cpu_baseline(wl):
    """The FP64 oracle (numpy, as is) on a bounded sample of the bench's own
    workload `wl` (the same 40^3 x 6 mesh, medium, degree, HABC order and
    source): its set-up is not timed; then 2 steps (10 Runge-Kutta stages)
    with numpy's BLAS limited to one thread (the reported value: the oracle is
    mostly single-threaded elementwise numpy, so this is what one core does)
    and 1 step with the BLAS pool as numpy starts it.  DOF-updates/s per
    stage, as the GPU value."""
    import workloads as w
    from oracle.solver import Oracle
    from threadpoolctl import threadpool_info, threadpool_limits
    blas = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    N, P, dt = wl["N"], wl["P"], wl["dt"]
    t_set = time.perf_counter()
    o = Oracle(wl["VX"], wl["E"], N, P, wl["rho"], wl["c"])
    o.set_source(wl["xs"], wl["f0"], wl["t0"])
    t_set = time.perf_counter() - t_set
    U = w.n_unknowns(o.m.K, o.m.Ktri, o.m.Klin, N, P)
    rates = {}
    for label, limit, steps in (("one", 1, 2), ("all", None, 1)):
        o.reset()
        o.s["q3"] = w.random_array(o.s["q3"].shape, 1) * 1e-3
        with threadpool_limits(limits=limit):
            t = time.perf_counter()
            o.step(steps, dt)
            el = time.perf_counter() - t
        rates[label] = (U * 5 * steps / el, el, 5 * steps)
    cpus, model = _host_cpu()
    n = wl["n"]
    return {"value": rates["one"][0], "unit": "DOF-updates/s", "cores": 1, "kind": "oracle",
            "sample": f"numpy FP64 oracle on the bench workload itself ({o.m.K}-tet "
                      f"{n}^3 x 6 mesh, N={N}, P={P}, layered medium, source), "
                      f"{rates['one'][2]} RK stages in {rates['one'][1]:.1f} s with BLAS on one "
                      f"thread (oracle set-up, {t_set:.0f} s, not timed)",
            "all_threads_value": rates["all"][0], "all_threads_blas": int(blas),
            "all_threads_seconds": rates["all"][1], "all_threads_stages": rates["all"][2],
            "host_cpus": cpus, "host_cpu_model": model}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--n", type=int, default=40)
    ap.add_argument("--workload", choices=["layered", "batch", "uneven", "reflection",
                                           "validation"],
                    default="layered",
                    help="layered: the 40^3 layered-medium step (default); batch: 64 shots "
                         "on a 20^3 mesh stepped together")
    ap.add_argument("--shots", type=int, default=64)
    ap.add_argument("--precision", choices=["fp64", "fp32", "bf16"], default="fp64",
                    help="fp32: FP32 3D state and contractions on the FP32 MFMA; bf16: FP32 "
                         "3D state with the contractions on the BF16 MFMA; FP64 boundary "
                         "levels in both")
    ap.add_argument("--order", type=int, default=None, help="override the degree N")
    ap.add_argument("--habc", type=int, default=None, help="override the HABC order P")
    ap.add_argument("--autotune", action="store_true",
                    help="time the 3D launch candidates on this workload and keep the fastest")
    ap.add_argument("--closure", action="store_true",
                    help="P = 0 with the learned boundary closure (layered workload: seeded "
                         "random weights, the cost does not depend on them; reflection "
                         "workload: trained first, then evaluated)")
    ap.add_argument("--teacher", choices=["small", "case", "parity"], default="small",
                    help="reflection --closure: teacher runs of the small recipe (8^3, c = 1), "
                         "on the case's own mesh and medium, or 200 runs of the 8^3 parity "
                         "case (BF16 training)")
    ap.add_argument("--candidate", type=int, default=None,
                    help="force a launch tuning candidate of the 3D level")
    ap.add_argument("--tuning-cache", default=None,
                    help="--autotune: JSON file of stored choices (default: "
                         "$DGHABC_TUNING_CACHE or ~/.cache/dghabc/tuning.json)")
    ap.add_argument("--graph", action="store_true",
                    help="replayed stepping: every step runs as one captured HIP graph")
    ap.add_argument("--valid-n", type=int, default=23,
                    help="validation: cells per axis of the Kuhn mesh of [-0.5, 0.5]^3")
    ap.add_argument("--orders", default="0,2,4,6,8,10,12",
                    help="validation: HABC orders (0 = basic ABC)")
    ap.add_argument("--free-surface", action="store_true",
                    help="validation: p = 0 on z = 0.5, HABC on the other faces")
    ap.add_argument("--matched", action="store_true",
                    help="validation: add HABC P = 3 with coefficients matched to 20, 38 and "
                         "52 degrees")
    ap.add_argument("--t-final", type=float, default=5.0)
    ap.add_argument("--sample", type=float, default=0.25)
    ap.add_argument("--calib-copy", action="store_true",
                    help="run 1 GiB reference kernels first (for PMC byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: the step runs on one GPU only (asked for --gpus {args.gpus}); "
              "sharding across GPUs is not implemented.", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch
    import workloads as w
    from paper_1610_05023_amd import Solver

    if args.calib_copy:
        # reference kernels of known traffic for the PMC byte counters: a
        # 1 GiB fill (writes 1 GiB) and an elementwise y = x + 1 (reads
        # 1 GiB, writes 1 GiB), twice
        x = torch.ones(1 << 27, dtype=torch.float64, device="cuda")
        for _ in range(2):
            y = x + 1.0
        torch.cuda.synchronize()
        print("[bench] calibration: 1 GiB fill, 2 x (1 GiB read + 1 GiB write)", file=sys.stderr)
        del x, y
    if args.workload == "reflection":
        return run_reflection(args)
    if args.workload == "validation":
        return run_validation(args)
    if args.workload == "uneven":
        run_uneven(args)
        return
    batch = args.workload == "batch"
    if batch:
        wl = build_batch_workload(shots=args.shots)
        nsh = wl["shots"]
    else:
        wl = build_workload(n=args.n)
        nsh = 1
    if args.order is not None:
        wl["N"] = args.order
        wl["dt"] = __import__("workloads").kuhn_dt(wl["n"], wl["N"], float(wl["c"].max()))
    if args.habc is not None:
        wl["P"] = args.habc
    if args.closure:
        wl["P"] = 0
    K = wl["E"].shape[0]
    t_setup = time.perf_counter()
    prec = {"fp64": 0, "fp32": 2, "bf16": 3}[args.precision]
    s = Solver(wl["VX"], wl["E"], wl["N"], wl["P"], wl["rho"], wl["c"], device=0,
               n_shots=nsh, precision=prec).bind()
    if batch:
        for j in range(nsh):
            s.set_source(wl["xs"][j], wl["f0"], wl["t0"], shot=j)
    else:
        s.set_source(wl["xs"], wl["f0"], wl["t0"])
    k = s.counts
    U = w.n_unknowns(k["K"], k["Ktri"], k["Klin"], wl["N"], wl["P"]) * nsh
    print(f"[bench] setup {time.perf_counter() - t_setup:.1f} s; K={K} Ktri={k['Ktri']} "
          f"Klin={k['Klin']} unknowns={U}", file=sys.stderr, flush=True)
    dt = wl["dt"]
    if args.closure:
        from paper_1610_05023_amd.binding import CLOSURE_PARAMS
        wts = (0.1 * np.random.default_rng(5).standard_normal(CLOSURE_PARAMS)).astype(np.float32)
        wts[0], wts[1] = 1.0, 0.95
        s.set_closure(wts)
    tuned = None
    if args.candidate is not None:
        s.set_tuning(args.candidate)
        tuned = {"candidate": args.candidate, "forced": True}
    if args.autotune:
        from paper_1610_05023_amd.tuning import tune
        best, ms, cached = tune(s, args.tuning_cache, 10)
        tuned = {"candidate": best, "from_cache": cached,
                 "ms_per_launch": None if ms is None else [round(float(v), 4) for v in ms]}
        print(f"[bench] autotune: candidate {best}"
              + (" (stored)" if cached else f" of {list(np.round(ms, 4))} ms"),
              file=sys.stderr, flush=True)
    if args.graph:
        s.set_graph(True)               # each step replays one captured HIP graph
    s.step(args.warmup, dt, 0.0)
    torch.cuda.synchronize()
    if not args.graph:
        s.kernel_timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.step(args.steps, dt, args.warmup * dt)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    if args.graph:
        # kernel durations come from HIP events around eager launches
        s.set_graph(False)
        s.kernel_timing(True)
        s.step(20, dt, (args.warmup + args.steps) * dt)
        torch.cuda.synchronize()
    ms3, n3 = s.kernel_time(3)
    s.kernel_timing(False)
    # measured device copy (torch, 2 x 1 GiB moved per copy) as a second
    # bandwidth reference beside the nominal peak
    xa = torch.empty(1 << 27, dtype=torch.float64, device="cuda")
    xb = torch.empty_like(xa)
    for _ in range(3):
        xb.copy_(xa)
    torch.cuda.synchronize()
    tc = time.perf_counter()
    for _ in range(10):
        xb.copy_(xa)
    torch.cuda.synchronize()
    copy_gbs = 2 * xa.numel() * 8 / ((time.perf_counter() - tc) / 10) / 1e9
    del xa, xb
    finite = all(s.check(shot=j)[0] == "DGH_OK" for j in range(nsh))
    value = U * 5 * args.steps / el
    avg3_ms = ms3 / max(n3, 1)
    # per-tet constants are read once per shot in this kernel
    alg = bytes_per_tet_stage(k["Np"], 4 if prec else 8) * K * nsh
    achieved = achieved_gbs(alg, avg3_ms)
    # the whole step against the same peak: all levels' algorithmic bytes
    step_alg = 5 * bytes_per_stage(K, k["Ktri"], k["Klin"], wl["N"], wl["P"],
                                   4 if prec else 8, nsh)
    step_gbs = step_alg / (el / args.steps) / 1e9
    print(f"[bench] {args.steps} steps in {el:.3f} s; 3D kernel avg {avg3_ms * 1e3:.1f} us over "
          f"{n3} launches; {achieved_gbs(alg, avg3_ms):.0f} GB/s; check={finite}",
          file=sys.stderr, flush=True)
    default_cfg = (not batch and args.n == 40 and prec == 0 and args.order is None
                   and args.habc is None)
    traffic = profiled_traffic() if default_cfg else None
    cpu = None
    if not args.no_cpu_baseline and not batch:
        try:
            cpu = cpu_baseline(wl)
        except Exception as ex:  # reported, never fatal for the GPU figure
            cpu = {"value": None, "error": repr(ex)}
    ptag = {0: "FP64", 2: "FP32-3D", 3: "BF16-contraction FP32-3D"}[prec]
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "DOF-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": el * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {0: "f64", 2: "f32 (3D level) + f64 (boundary levels)",
                  3: "bf16 contractions, f32 3D state + f64 (boundary levels)"}[prec],
        "data": "synthetic",
        "config": ({"workload": f"{ptag} DG+HABC step, {args.n}^3 x 6 "
                                f"= {K}-tet Kuhn mesh of the unit cube, N={wl['N']}, HABC "
                                f"P={wl['P']} with edges and corners, 5 random layers (seed 2), "
                                f"Ricker point source"}
                   if not batch else
                   {"workload": f"{ptag} DG+HABC step, {nsh} shots "
                                f"stepped together on a {wl['n']}^3 x 6 = {K}-tet Kuhn mesh, "
                                f"N={wl['N']}, HABC P={wl['P']}, rho=c=1, one Ricker source per "
                                f"shot (seed 4)",
                    "shots": nsh}) | {
                   "K_tet": K, "K_tri": k["Ktri"], "K_lin": k["Klin"], "K_pnt": k["Kpnt"],
                   "N": wl["N"], "P": wl["P"], "unknowns": U, "dt": dt,
                   "parallelism": "single GPU",
                   "step_mode": "hip graph per step" if args.graph else "eager launches",
                   "boundary": "learned closure (P = 0)" if args.closure else f"HABC P={wl['P']}",
                   "tuning": tuned if tuned is not None else "default (tile on chip, XCD ranges)"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": traffic,
                     "traffic_unit": "bytes per launch (rocprofv3 FETCH_SIZE x2.0 + WRITE_SIZE x1.0)",
                     "kernel": kernel_name(prec, wl["N"], tuned) +
                               " (3D volume + surface + LSRK update)",
                     "avg_us": avg3_ms * 1e3, "alg_bytes_per_launch": alg,
                     "step_achieved": step_gbs, "step_frac": step_gbs / HBM_PEAK_GBS,
                     "measured_copy_gbs": copy_gbs,
                     "frac_of_measured_copy": achieved / copy_gbs,
                     "step_frac_of_measured_copy": step_gbs / copy_gbs,
                     "step_alg_bytes": step_alg,
                     "step_note": "all levels' algorithmic bytes per step / ms_per_step"},
        "cpu_baseline": cpu,
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
