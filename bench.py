"""Benchmark of the G1-G2 hot path on one MI355X.

Workload (the configuration the headline metric is quoted on): general-basis
second-Born G1-G2 propagation, Nb = 32 spin orbitals, random GUE h (sigma=1),
w = sum_Q B^Q x B^Q from a rank-64 Hermitian factor, 8 particles in the
Aufbau state of h, G2(0) = 0, RK4 with dt = 0.01.  Inputs are seeded and
synthetic (workloads.general_system).

One "step" = one full RK4 step (4 right-hand sides) of G1 and G2.  The binary64
path is the headline value; the mixed path (binary32 matrix-core contractions,
binary64 state) is reported beside it with its error against the binary64 run.

Prints ONE JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "RK4 steps/s & achieved TFLOP/s of G2 RHS, FP64 vs mixed at stated error"
PEAK_FP64_MFMA = 78.6      # TFLOP/s, MI355X dense FP64 matrix
PEAK_FP32_MFMA = 157.3     # TFLOP/s, MI355X dense FP32 matrix
PEAK_HBM = 8000.0          # GB/s


def flops_per_rhs(nb: int) -> dict:
    """Algorithmic real flops of one general-basis SOA right-hand side: 8 per
    complex multiply-add, Hermiticity halving assumed:
    gen_vt 2 nb^5, gen_main 5 nb^5 (T sandwich 2, commutator 2, collision 1)."""
    n5 = float(nb) ** 5
    return {"gen_vt": 8 * 2 * n5, "gen_main": 8 * 5 * n5, "total": 8 * 7 * n5}


def time_propagator(p, dt, steps, warmup, stream, torch):
    p.step(dt, warmup)
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    w0 = time.perf_counter()
    p.step(dt, steps)
    ev1.record(stream)
    torch.cuda.synchronize()
    w1 = time.perf_counter()
    return ev0.elapsed_time(ev1), (w1 - w0) * 1e3


def cpu_baseline(system, seconds: float = 15.0):
    """The FP64 oracle on the host cores, timed on a bounded number of RK4
    steps of the same workload (starting from the same initial state)."""
    import torch
    from oracle import integrate as OI
    nthreads = torch.get_num_threads()
    f = OI.general_rhs_fn(system.h0, system.w, "soa")
    g1 = torch.as_tensor(system.g1, dtype=torch.complex128)
    g2 = torch.zeros((system.nb,) * 4, dtype=torch.complex128)
    OI.rk4_step(f, 0.0, (g1, g2), system.dt)          # warm-up
    n, t0 = 0, time.perf_counter()
    while True:
        g1, g2 = OI.rk4_step(f, n * system.dt, (g1, g2), system.dt)
        n += 1
        el = time.perf_counter() - t0
        if el > seconds or n >= 200:
            break
    return {"value": n / el, "unit": "RK4 steps/s", "cores": nthreads, "kind": "oracle",
            "sample": f"{n} RK4 steps of the Nb=32 SOA workload (torch CPU complex128, "
                      f"{nthreads} threads), {el:.1f} s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the G1-G2 workload here runs on a single "
              "MI355X (see DESIGN.md for how it would shard); use --gpus 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_2002_12717_amd import binding as B
    from workloads import general_system

    torch.cuda.set_device(0)
    system = general_system()
    nb = system.nb
    stream = torch.cuda.Stream()
    fl = flops_per_rhs(nb)

    res = {}
    for prec in ("fp64", "mixed"):
        p = B.Propagator(B.GENERAL, B.SOA, nb, system.h0, system.g1, w=system.w,
                         precision=B.FP64 if prec == "fp64" else B.MIXED, stream=stream.cuda_stream)
        ms, wall_ms = time_propagator(p, system.dt, args.steps, args.warmup, stream, torch)
        g1, _, t = p.get_state()
        prof = p.profile_rhs(reps=20)
        obs = p.observables()
        res[prec] = dict(ms=ms, wall_ms=wall_ms, g1=g1, prof=prof, obs=obs, t=t)
        p.close()

    f64, mx = res["fp64"], res["mixed"]
    ms_step = f64["ms"] / args.steps
    steps_per_s = 1e3 / ms_step
    mx_ms_step = mx["ms"] / args.steps
    err_mixed = float(np.abs(mx["g1"] - f64["g1"]).max() / np.abs(f64["g1"]).max())
    e_err_mixed = abs(mx["obs"]["E_tot"] - f64["obs"]["E_tot"]) / max(abs(f64["obs"]["E_tot"]), 1.0)

    main_ms = f64["prof"].get("gen_main")
    achieved = fl["gen_main"] / (main_ms * 1e-3) / 1e12
    roofline = {"kernel": "gen_main", "bound": "mfma", "achieved": round(achieved, 3),
                "peak": PEAK_FP64_MFMA, "unit": "TFLOP/s", "frac": round(achieved / PEAK_FP64_MFMA, 4),
                "traffic": None, "kernel_ms": round(main_ms, 5),
                "flop_per_launch": fl["gen_main"]}
    rhs_ms = sum(f64["prof"].values())
    out = {
        "metric": METRIC,
        "value": round(steps_per_s, 2),
        "unit": "RK4 steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "general-basis SOA G1-G2, Nb=32 spin orbitals, rank-64 w, "
                               "8 particles, dt=0.01, RK4",
                   "nb": nb, "rank": 64, "nocc": 8, "dt": system.dt, "selfenergy": "SOA",
                   "parallelism": "single GPU"},
        "g2_rhs_tflops": round(4 * fl["total"] / (ms_step * 1e-3) / 1e12, 3),
        "roofline": roofline,
        "kernels_ms_per_rhs": {k: round(v, 5) for k, v in f64["prof"].items()},
        "rhs_ms_sum": round(rhs_ms, 5),
        "mixed": {"dtype": "f32 contractions / f64 state",
                  "value": round(1e3 / mx_ms_step, 2), "ms_per_step": round(mx_ms_step, 5),
                  "speedup_vs_fp64": round(ms_step / mx_ms_step, 3),
                  "g2_rhs_tflops": round(4 * fl["total"] / (mx_ms_step * 1e-3) / 1e12, 3),
                  "err_G1_vs_fp64": err_mixed, "err_E_vs_fp64": e_err_mixed,
                  "kernels_ms_per_rhs": {k: round(v, 5) for k, v in mx["prof"].items()},
                  "peak": PEAK_FP32_MFMA},
        "sim_time": f64["t"],
        "wall_ms_fp64": round(f64["wall_ms"], 3),
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(system)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
