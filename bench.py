"""Benchmark of the G1-G2 hot path on one MI355X.

Default workload (the headline: the largest single-GPU configuration of the
metric): general-basis GW G1-G2 propagation, Nb = 64 spin orbitals (G2 is
64^4 complex, 268 MB in binary64), random GUE h (sigma = 1), w = sum_Q B^Q x
B^Q from a rank-128 Hermitian factor, 16 particles in the Aufbau state of h,
G2(0) = 0, a one-step kick dh = 0.1 GUE, RK4 with dt = 0.01 (500 steps).
Inputs are seeded and synthetic (workloads.gw_system).

One "step" = one full RK4 step (four right-hand sides) of G1 and G2.  The
binary64 path is the headline value; the mixed path (binary32 matrix-core
contractions, binary64 state) is reported beside it, with the errors of both
against the binary64 run over the whole 500-step propagation (and against the
stored oracle trajectory of tests/golden/ when present).  The Nb = 32 SOA
workload is reported as an extra key.  Other workloads of the paper's shape
are available with --workload (general_soa, general_ladder, hubbard_chain with
--ns, hubbard_2d, hubbard_batch, hubbard_adjoint, scaling).

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

# HBM bytes per launch measured with rocprofv3 FETCH_SIZE / WRITE_SIZE (scaled by
# the copy calibration; profiles/hbm_traffic_counters.md).  A figure is only
# reported while the kernel's source file still has the hash it had when the
# counters were taken (source_hash below: the whole file, so that a change of
# the kernel or of how it is launched voids it).
TRAFFIC = {
    "gen_main/f64": {"bytes": 75.9e6, "src": "general.hip", "sha1": "10279bdbe35c"},
    "gen_main/f32": {"bytes": 50.7e6, "src": "general.hip", "sha1": "10279bdbe35c"},
    "gen_gemm/f64": {"bytes": 5.177e9, "src": "general.hip", "sha1": "10279bdbe35c"},
    "gen_gemm/f32": {"bytes": 3.017e9, "src": "general.hip", "sha1": "10279bdbe35c"},
    "hub_stage/2d": {"bytes": 2.385e9, "src": "hubbard.hip", "sha1": "94601047d47b"},
    "hub_stage/2d/mixed": {"bytes": 1.634e9, "src": "hubbard.hip", "sha1": "94601047d47b"},
    "hub_stage/2d/tpp": {"bytes": 2.443e9, "src": "hubbard.hip", "sha1": "94601047d47b"},
    "jel_stage/gw": {"bytes": 2.03e9, "src": "jellium.hip", "sha1": "370a4e568f25"},
    "jel_stage/gw/mixed": {"bytes": 1.70e9, "src": "jellium.hip", "sha1": "370a4e568f25"},
    "jel_stage/tpp": {"bytes": 4.651e9, "src": "jellium.hip", "sha1": "370a4e568f25"},
    "jel_lad/tpp": {"bytes": 0.968e9, "src": "jellium.hip", "sha1": "370a4e568f25"},
}


def source_hash(src: str) -> str:
    """sha1 (first 12 hex digits) of a kernel source file of the library, its
    comments and whitespace removed (so that only a change of code voids it)."""
    import hashlib
    import re
    with open(os.path.join(ROOT, "paper_2002_12717_amd", "csrc", src)) as f:
        text = f.read()
    text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
    text = re.sub(r"//[^\n]*", " ", text)
    return hashlib.sha1(" ".join(text.split()).encode()).hexdigest()[:12]


def traffic(key):
    t = TRAFFIC.get(key)
    if t is None:
        return None
    return t["bytes"] if source_hash(t["src"]) == t["sha1"] else None


SE_CODES = {"soa": lambda B: B.SOA, "gw": lambda B: B.GW, "tpp": lambda B: B.TPP, "tph": lambda B: B.TPH,
            "dsl": lambda B: B.DSL}
# Hubbard G2 channels per selfenergy: GW and DSL propagate three
HUB_CHANNELS = {"soa": 1, "tpp": 1, "tph": 1, "gw": 3, "dsl": 3}


def soa_flops(nb: int) -> dict:
    """Algorithmic real flops of one general-basis right-hand side (8 per complex
    multiply-add; Hermiticity halving assumed): gen_vt 2 nb^5, gen_main 5 nb^5
    (T sandwich 2, commutator 2, collision integral 1)."""
    n5 = float(nb) ** 5
    return {"gen_vt": 16 * n5, "gen_main": 40 * n5, "soa_total": 56 * n5}


def gw_flops(nb: int) -> dict:
    """GW adds h^eps (2 nb^5) and the polarization GEMM (nb^6) per RHS."""
    d = soa_flops(nb)
    d["gen_heps"] = 16 * float(nb) ** 5
    d["gen_gemm"] = 8 * float(nb) ** 6
    d["total"] = d["soa_total"] + d["gen_heps"] + d["gen_gemm"]
    return d


def ladder_flops(nb: int, se: str) -> dict:
    """Each T-matrix ladder adds its quasi-Hamiltonian (two one-sided products
    per side of the sandwich: 4 nb^5) and one GEMM (nb^6); DSL adds GW's
    polarization as well.  gen_gemm is the flops of one GEMM launch."""
    d = soa_flops(nb)
    n5, n6 = float(nb) ** 5, float(nb) ** 6
    nlad = {"tpp": 1, "tph": 1, "dsl": 2}[se]
    ngemm = nlad + (1 if se == "dsl" else 0)
    d["gen_hlad"] = 32 * n5
    d["gen_gemm"] = 8 * n6
    d["total"] = d["soa_total"] + nlad * d["gen_hlad"] + ngemm * d["gen_gemm"] + \
        (16 * n5 if se == "dsl" else 0.0)
    return d


def timed_steps(p, dt, steps, warmup, stream, torch):
    """Wall and event time of `steps` RK4 steps after `warmup` steps."""
    if warmup:
        p.step(dt, warmup)
    p.prepare_graph(dt)             # the replayed graph is captured before the timed region
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    w0 = time.perf_counter()
    try:
        p.step(dt, steps)
    except Exception as e:          # the divergence guard fires after the steps ran
        if getattr(e, "status", None) != -5:
            raise
    ev1.record(stream)
    torch.cuda.synchronize()
    w1 = time.perf_counter()
    return ev0.elapsed_time(ev1), (w1 - w0) * 1e3


def kernel_table(prof: dict) -> dict:
    return {k: {"ms_avg": round(v[0] / max(v[1], 1), 6), "launches": v[1]} for k, v in prof.items()}


def host_info() -> dict:
    """CPU model, logical CPUs and the BLAS that torch's CPU kernels call."""
    import torch
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    blas = "unknown"
    for line in torch.__config__.show().splitlines():
        if "Math Kernel Library" in line or "OpenBLAS" in line:
            blas = line.strip(" -")
            break
    return {"cpu_model": model, "logical_cpus": os.cpu_count(), "blas": blas,
            "torch_threads": torch.get_num_threads()}


def cpu_baseline_gw(system, seconds: float = 12.0):
    """The FP64 oracle's right-hand side of the Nb = 64 GW workload on the host
    cores (at the initial state; the cost of every term is independent of the
    values), timed over a bounded number of evaluations; an RK4 step is four."""
    import torch
    from oracle import general as OG
    nthreads = torch.get_num_threads()
    T = lambda x: torch.as_tensor(x, dtype=torch.complex128)  # noqa: E731
    h, w, g1 = T(system.h0), T(system.w), T(system.g1)
    g2 = torch.zeros((system.nb,) * 4, dtype=torch.complex128)
    OG.rhs(h, w, g1, g2, "gw")                      # warm-up
    n, t0 = 0, time.perf_counter()
    while True:
        OG.rhs(h, w, g1, g2, "gw")
        n += 1
        el = time.perf_counter() - t0
        if el > seconds or n >= 20:
            break
    per_rhs = el / n
    return {"value": round(1.0 / (4.0 * per_rhs), 5), "unit": "RK4 steps/s", "cores": nthreads,
            "kind": "oracle",
            "sample": f"{n} right-hand sides of the Nb=64 GW workload (torch CPU complex128, {nthreads} "
                      f"threads, {el:.1f} s, {per_rhs:.2f} s each), four per RK4 step",
            "host": host_info()}


def cpu_baseline_general(system, seconds: float = 15.0):
    """The FP64 oracle on the host cores, timed on a bounded number of RK4 steps
    of the same workload from the same initial state."""
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
    return {"value": round(n / el, 4), "unit": "RK4 steps/s", "cores": nthreads, "kind": "oracle",
            "sample": f"{n} RK4 steps of the Nb=32 SOA workload from t=0 (torch CPU complex128, "
                      f"{nthreads} threads, {el:.1f} s)", "host": host_info()}


def cpu_baseline_hubbard(system, seconds: float = 15.0, selfenergy: str = "soa"):
    import torch
    from oracle import integrate as OI
    nthreads = torch.get_num_threads()
    f = OI.hubbard_rhs_fn(system, selfenergy)
    y = OI.hubbard_initial(system, selfenergy)
    y = list(OI.rk4_step(f, 0.0, y, system.dt))
    n, t0 = 0, time.perf_counter()
    while True:
        y = list(OI.rk4_step(f, n * system.dt, y, system.dt))
        n += 1
        el = time.perf_counter() - t0
        if el > seconds or n >= 2000:
            break
    return {"value": round(n / el, 4), "unit": "RK4 steps/s", "cores": nthreads, "kind": "oracle",
            "sample": f"{n} RK4 steps of the {system.name} workload (torch CPU, {nthreads} threads, "
                      f"{el:.1f} s)"}


def base_line(args, steps_per_s, ms_step, dtype, config):
    return {"metric": METRIC, "value": round(steps_per_s, 3), "unit": "RK4 steps/s", "n_gpus": 1,
            "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_step, 6),
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": dtype,
            "data": "synthetic", "config": config}


# --------------------------------------------------------------------------- workloads
GOLDEN = os.path.join(ROOT, "tests", "golden")


def trajectory(B, system, code, prec, stream, nsteps, stops):
    """Propagate the workload from t = 0 (one-step kick included) for nsteps
    steps; G1 and E_tot at every step in `stops` (and at 0 and nsteps)."""
    p = B.Propagator(B.GENERAL, code, system.nb, system.h0, system.g1, w=system.w, precision=prec,
                     stream=stream.cuda_stream)
    stops = sorted(set(q for q in stops if 0 < q <= nsteps) | {nsteps})
    out = {}

    def record(n):
        g1, _, _ = p.get_state(with_g2=False)
        out[n] = (g1, p.observables()["E_tot"])

    record(0)
    n = 0
    if system.kick is not None:
        p.set_h0(system.h0 + system.kick)
        p.step(system.dt, 1)
        p.set_h0(system.h0)
        n = 1
        if 1 in stops:
            record(1)
    for q in stops:
        if q > n:
            p.step(system.dt, q - n)
            n = q
            record(n)
    p.close()
    return out


def trajectory_error(a, ref):
    """Max over common times of max|dG1| / max|G1_ref| and |dE| / max(|E_ref(0)|, 1)."""
    import numpy as np
    common = sorted(set(a) & set(ref))
    e_scale = max(abs(ref[0][1]), 1.0)
    eg = max(float(np.abs(a[n][0] - ref[n][0]).max() / np.abs(ref[n][0]).max()) for n in common)
    ee = max(abs(a[n][1] - ref[n][1]) / e_scale for n in common)
    return {"G1": eg, "E": ee, "steps_compared": len(common)}


def golden_error(traj, g):
    """Errors of a trajectory against the stored oracle trajectory: G1 in full
    where stored, at the stored entries elsewhere; E where stored."""
    import numpy as np
    eg, ee, n_g1 = 0.0, 0.0, 0
    e_scale = max(abs(float(g["E_tot"][0])), 1.0)
    for k, n in enumerate(g["full_steps"]):
        if int(n) in traj:
            ref = g["full_g1"][k]
            eg = max(eg, float(np.abs(traj[int(n)][0] - ref).max() / np.abs(ref).max()))
            n_g1 += 1
    if "g1_idx" in g.files:
        idx = g["g1_idx"]
        for k, n in enumerate(g["samp_steps"]):
            if int(n) in traj:
                got = traj[int(n)][0][idx[:, 0], idx[:, 1]]
                eg = max(eg, float(np.abs(got - g["samp_g1"][k]).max() / g["samp_scale"][k]))
                n_g1 += 1
    n_e = 0
    for k, n in enumerate(g["obs_steps"]):
        if int(n) in traj:
            ee = max(ee, abs(traj[int(n)][1] - float(g["E_tot"][k])) / e_scale)
            n_e += 1
    return {"G1": eg, "E": ee, "G1_times": n_g1, "E_times": n_e}


def run_general(args, torch, B, se="soa", accuracy=True, steps=None, warmup=None, profile_steps=None):
    import numpy as np
    from workloads import general_system, gw_system
    gw = se != "soa"               # every closure beyond SOA runs on the Nb = 64 system
    system = gw_system() if gw else general_system()
    nb = system.nb
    steps = args.steps if steps is None else steps
    warmup = args.warmup if warmup is None else warmup
    profile_steps = args.profile_steps if profile_steps is None else profile_steps
    stream = torch.cuda.Stream()
    fl = soa_flops(nb) if se == "soa" else (gw_flops(nb) if se == "gw" else ladder_flops(nb, se))
    code = {"soa": B.SOA, "gw": B.GW, "tpp": B.TPP, "tph": B.TPH, "dsl": B.DSL}[se]
    res = {}
    for prec in ("fp64", "mixed"):
        p = B.Propagator(B.GENERAL, code, nb, system.h0, system.g1, w=system.w,
                         precision=B.FP64 if prec == "fp64" else B.MIXED, stream=stream.cuda_stream)
        if system.kick is not None:          # one-step kick, then the static h0
            p.set_h0(system.h0 + system.kick)
            p.step(system.dt, 1)
            p.set_h0(system.h0)
        ms, wall = timed_steps(p, system.dt, steps, warmup, stream, torch)
        prof = p.profile(system.dt, profile_steps)
        res[prec] = dict(ms=ms, wall=wall, prof=prof)
        p.close()
    f64, mx = res["fp64"], res["mixed"]
    ms_step = f64["ms"] / steps
    mx_step = mx["ms"] / steps
    dom = "gen_gemm" if gw else "gen_main"
    tot_ms, cnt = f64["prof"][dom]
    achieved = fl[dom] * cnt / (tot_ms * 1e-3) / 1e12
    rhs_flops = fl["total"] if gw else fl["soa_total"]
    config = {"workload": (f"general-basis {se.upper()} G1-G2, Nb={nb} spin orbitals, "
                           f"rank-{system.meta['rank']} w, {system.meta['nocc']} particles, "
                           + ("one-step kick 0.1 GUE, " if system.kick is not None else "")
                           + f"dt={system.dt}, RK4, {system.nsteps} steps"),
              "nb": nb, "rank": system.meta["rank"], "nocc": system.meta["nocc"], "dt": system.dt,
              "nsteps": system.nsteps, "selfenergy": se.upper(), "parallelism": "single GPU"}
    out = base_line(args, 1e3 / ms_step, ms_step, "f64", config)
    out["steps"], out["warmup"] = steps, warmup
    mx_tot, mx_cnt = mx["prof"][dom]
    mx_ach = fl[dom] * mx_cnt / (mx_tot * 1e-3) / 1e12
    out.update({
        "g2_rhs_tflops": round(4 * rhs_flops / (ms_step * 1e-3) / 1e12, 3),
        "roofline": {"kernel": dom, "bound": "mfma", "achieved": round(achieved, 3),
                     "peak": PEAK_FP64_MFMA, "unit": "TFLOP/s", "frac": round(achieved / PEAK_FP64_MFMA, 4),
                     "traffic": traffic("gen_gemm/f64") if gw else traffic("gen_main/f64"),
                     "kernel_ms_avg": round(tot_ms / cnt, 6),
                     "flop_per_launch": fl[dom], "launches": cnt},
        "kernels": kernel_table(f64["prof"]),
        "mixed": {"dtype": "f32 contractions / f64 state", "value": round(1e3 / mx_step, 3),
                  "ms_per_step": round(mx_step, 6), "speedup_vs_fp64": round(ms_step / mx_step, 3),
                  "g2_rhs_tflops": round(4 * rhs_flops / (mx_step * 1e-3) / 1e12, 3),
                  "roofline": {"kernel": dom, "achieved": round(mx_ach, 3), "peak": PEAK_FP32_MFMA,
                               "unit": "TFLOP/s", "frac": round(mx_ach / PEAK_FP32_MFMA, 4),
                               "traffic": traffic("gen_gemm/f32") if gw else traffic("gen_main/f32")},
                  "kernels": kernel_table(mx["prof"])},
    })
    if gw:
        # gen_gemm forms each complex multiply-add with three real products
        # (Re = ArBr - AiBi, Im = (Ar+Ai)(Br+Bi) - ArBr - AiBi): 6 real flops
        # executed for the 8 of the algorithmic count, so the algorithmic rate
        # can exceed the matrix peak; the matrix cores' own use is 3/4 of it
        out["roofline"]["executed_flop_per_launch"] = 0.75 * fl[dom]
        out["roofline"]["matrix_core_frac"] = round(0.75 * achieved / PEAK_FP64_MFMA, 4)
        out["mixed"]["roofline"]["matrix_core_frac"] = round(0.75 * mx_ach / PEAK_FP32_MFMA, 4)
    if accuracy and se in ("soa", "gw"):
        every = 25 if gw else 50
        gname = "general_gw_nb64.npz" if gw else "general_soa_nb32.npz"
        gpath = os.path.join(GOLDEN, gname)
        g = np.load(gpath) if os.path.exists(gpath) else None
        stops = set(range(every, system.nsteps + 1, every))
        if g is not None:
            stops |= set(int(n) for n in g["full_steps"]) | set(int(n) for n in g["samp_steps"])
        tr = {prec: trajectory(B, system, code, B.FP64 if prec == "fp64" else B.MIXED, stream,
                               system.nsteps, stops) for prec in ("fp64", "mixed")}
        mvf = trajectory_error(tr["mixed"], tr["fp64"])
        acc = {"steps": system.nsteps, "mixed_vs_fp64": mvf}
        if g is not None:
            acc["fp64_vs_oracle"] = golden_error(tr["fp64"], g)
            acc["mixed_vs_oracle"] = golden_error(tr["mixed"], g)
            acc["oracle_trajectory"] = f"tests/golden/{gname} (written by tests/golden/make_golden.py)"
        out["accuracy"] = acc
        out["mixed"]["err_G1_vs_fp64"] = mvf["G1"]
        out["mixed"]["err_E_vs_fp64"] = mvf["E"]
    if not args.no_cpu_baseline:
        if se == "gw":
            out["cpu_baseline"] = cpu_baseline_gw(system)
        elif se == "soa":
            out["cpu_baseline"] = cpu_baseline_general(system)
    return out


def summary(line: dict) -> dict:
    """The compact form of a workload's line, for an extra key of the headline."""
    keep = ("value", "unit", "ms_per_step", "steps", "warmup", "dtype", "config", "g2_rhs_tflops",
            "roofline", "accuracy")
    out = {k: line[k] for k in keep if k in line}
    m = line.get("mixed", {})
    out["mixed"] = {k: m[k] for k in ("value", "ms_per_step", "speedup_vs_fp64", "err_G1_vs_fp64",
                                      "err_E_vs_fp64", "roofline") if k in m}
    return out


def run_hubbard(args, torch, B, kind):
    import numpy as np
    from workloads import adjoint_system, hubbard_chain_system
    system = hubbard_chain_system(ns=args.ns) if kind == "hubbard_chain" else adjoint_system()
    ns = system.ns
    stream = torch.cuda.Stream()
    se = args.selfenergy or "soa"

    def run(prec):
        p = B.Propagator(B.HUBBARD, SE_CODES[se](B), ns, system.h0, system.g1, U=system.U,
                         stream=stream.cuda_stream, precision=prec)
        if system.drive is not None:
            d = system.drive
            p.set_drive(d.x, d.c, d.t_center, d.tau)
        path = p.step_path()        # the library's own choice of kernels for these steps
        ms, _ = timed_steps(p, system.dt, args.steps, args.warmup, stream, torch)
        prof = p.profile(system.dt, args.profile_steps)
        obs = p.observables()
        g1, _, _ = p.get_state()
        p.close()
        return ms, prof, obs, g1, path

    ms, prof, obs, g1_64, path = run(B.FP64)
    # a small cluster runs whole steps in the persistent work-group: its time is
    # not that of the launched stages the per-launch profile times
    persistent = path == "hub_persistent"
    ms_step = ms / args.steps
    n4 = float(ns) ** 4
    tot_ms, cnt = prof["hub_stage"]
    # algorithmic bytes: 256 B per complex128 G2 element per RK4 step (4 launches);
    # Hubbard GW and DSL propagate three G2 channels
    bytes_per_launch = 64.0 * n4 * HUB_CHANNELS[se]
    achieved = bytes_per_launch * cnt / (tot_ms * 1e-3) / 1e9
    name = f"1D chain, {ns} sites" if kind == "hubbard_chain" else "2D 8x8 open cluster, driven"
    config = {"workload": f"Hubbard {se.upper()} G1-G2, {name}, U={system.U}, dt={system.dt}, RK4",
              "ns": ns, "U": system.U, "dt": system.dt, "selfenergy": se.upper(),
              "parallelism": "single GPU"}
    out = base_line(args, 1e3 / ms_step, ms_step, "f64", config)
    stage_roof = {"kernel": "hub_stage", "bound": "hbm", "achieved": round(achieved, 2),
                  "peak": PEAK_HBM, "unit": "GB/s", "frac": round(achieved / PEAK_HBM, 4),
                  # the counters were taken on the SOA and TPP instantiations
                  "traffic": (traffic("hub_stage/2d") if se == "soa" else traffic("hub_stage/2d/tpp")
                              if se == "tpp" else None) if kind == "hubbard_2d" else None,
                  "kernel_ms_avg": round(tot_ms / cnt, 6),
                  "bytes_per_launch": bytes_per_launch, "launches": cnt}
    out.update({
        "path": path,
        # the persistent kernel keeps the state on chip: no HBM roofline applies
        # to it (it is bound by its LDS reads and barriers), so none is reported
        "roofline": None if persistent else stage_roof,
        "kernels": kernel_table(prof),
        "observables": {k: obs[k] for k in ("t", "E_tot", "docc")},
    })
    if persistent:
        out["launched_stage_roofline"] = stage_roof
    # mixed precision: binary32 G2 stage copies, 52 B per element and launch
    # (binary64 y and acc, binary32 stage input and output)
    mx_ms, mx_prof, mx_obs, g1_mx, _ = run(B.MIXED)
    mx_step = mx_ms / args.steps
    mx_tot, mx_cnt = mx_prof["hub_stage"]
    mx_ach = 52.0 * n4 * HUB_CHANNELS[se] * mx_cnt / (mx_tot * 1e-3) / 1e9
    out["mixed"] = {"dtype": "f64 state, f32 G2 stage copies", "value": round(1e3 / mx_step, 3),
                    "ms_per_step": round(mx_step, 6), "speedup_vs_fp64": round(ms_step / mx_step, 3),
                    "err_G1_vs_fp64": float(np.abs(g1_mx - g1_64).max() / np.abs(g1_64).max()),
                    "err_E_vs_fp64": abs(mx_obs["E_tot"] - obs["E_tot"]) / max(abs(obs["E_tot"]), 1.0),
                    "roofline": {"kernel": "hub_stage", "achieved": round(mx_ach, 2), "peak": PEAK_HBM,
                                 "unit": "GB/s", "frac": round(mx_ach / PEAK_HBM, 4),
                                 "traffic": traffic("hub_stage/2d/mixed")
                                 if kind == "hubbard_2d" and se == "soa" else None}}
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline_hubbard(system, selfenergy=se)
    return out


def run_jellium(args, torch, B):
    """Jellium after an interaction quench (6 x 6 x 6 momenta, spin-polarized
    Fermi-Dirac start, Coulomb v): steps/s of both precisions, the HBM roofline
    of the streaming stage kernel, and the mixed-precision error against
    binary64 over the whole propagation."""
    import numpy as np
    from workloads import jellium_system
    se = args.selfenergy or "gw"
    if se not in ("soa", "gw", "tpp", "tph"):
        raise SystemExit("jellium takes --selfenergy soa, gw, tpp or tph")
    ladder = se in ("tpp", "tph")
    s = jellium_system()
    nb = s.nb
    code = {"soa": B.SOA, "gw": B.GW, "tpp": B.TPP, "tph": B.TPH}[se]
    stream = torch.cuda.Stream()
    res = {}
    for prec in ("fp64", "mixed"):
        p = B.Jellium(code, s.dims, s.eps, s.v, s.g1, stream=stream.cuda_stream,
                      precision=B.FP64 if prec == "fp64" else B.MIXED)
        ms, _ = timed_steps(p, s.dt, args.steps, args.warmup, stream, torch)
        prof = p.profile(s.dt, args.profile_steps)
        p.close()
        # the whole propagation from t = 0, G1 and E every 50 steps
        q = B.Jellium(code, s.dims, s.eps, s.v, s.g1, stream=stream.cuda_stream,
                      precision=B.FP64 if prec == "fp64" else B.MIXED)
        traj = {0: (q.get_state(with_g2=False)[0], q.observables()["E_tot"])}
        for n in range(50, 0 if args.no_accuracy else s.nsteps + 1, 50):
            q.step(s.dt, 50)
            traj[n] = (q.get_state(with_g2=False)[0], q.observables()["E_tot"])
        q.close()
        res[prec] = dict(ms=ms, prof=prof, traj=traj)
    f64, mx = res["fp64"], res["mixed"]
    ms_step = f64["ms"] / args.steps
    mx_step = mx["ms"] / args.steps
    n2 = 3.0 * nb ** 3
    tot, cnt = f64["prof"]["jel_stage"]
    # 48, 80, 80, 48 B per element over the four stages; the T matrices read
    # the ladder sums at the element and at its partner (32 B more)
    extra = 32.0 if ladder else 0.0
    bytes_launch = (64.0 + extra) * n2
    ach = bytes_launch * cnt / (tot * 1e-3) / 1e9
    mtot, mcnt = mx["prof"]["jel_stage"]
    mbytes = (52.0 + extra) * n2      # binary32 stage copies: 40, 64, 64, 40 B
    mach = mbytes * mcnt / (mtot * 1e-3) / 1e9
    stage_roof = {"kernel": "jel_stage", "bound": "hbm", "achieved": round(ach, 2), "peak": PEAK_HBM,
                  "unit": "GB/s", "frac": round(ach / PEAK_HBM, 4),
                  "traffic": traffic("jel_stage/gw") if se == "gw" else traffic("jel_stage/tpp") if se == "tpp" else None,
                  "kernel_ms_avg": round(tot / cnt, 6), "bytes_per_launch": bytes_launch, "launches": cnt}
    roof, lad_roof, mx_lad = stage_roof, None, None
    if ladder:
        # the ladder sums, a transform of each G2 row: the stage input read once
        # and the sums written once, 32 B per element (binary64; 24 B when the
        # stage input is binary32, three of the four stages of a mixed step)
        lbytes = 32.0 * n2
        ltot, lcnt = f64["prof"]["jel_lad"]
        lach = lbytes * lcnt / (ltot * 1e-3) / 1e9
        lad_roof = {"kernel": "jel_lad", "bound": "hbm", "achieved": round(lach, 2), "peak": PEAK_HBM,
                    "unit": "GB/s", "frac": round(lach / PEAK_HBM, 4),
                    "traffic": traffic("jel_lad/tpp") if se == "tpp" else None,
                    "kernel_ms_avg": round(ltot / lcnt, 6), "bytes_per_launch": lbytes, "launches": lcnt}
        mlt, mlc = mx["prof"]["jel_lad"]
        mlb = 26.0 * n2
        mx_lad = {"kernel": "jel_lad", "achieved": round(mlb * mlc / (mlt * 1e-3) / 1e9, 2), "peak": PEAK_HBM,
                  "unit": "GB/s", "frac": round(mlb * mlc / (mlt * 1e-3) / 1e9 / PEAK_HBM, 4),
                  "bytes_per_launch": mlb}
        if ltot > tot:
            roof = lad_roof
    err = trajectory_error(mx["traj"], f64["traj"])
    e0 = f64["traj"][0][1]
    drift = max(abs(v[1] - e0) for v in f64["traj"].values()) / max(abs(e0), 1.0)
    m = s.meta
    config = {"workload": f"jellium {se.upper()} G1-G2, {s.dims[0]}x{s.dims[1]}x{s.dims[2]} plane waves "
                          f"(periodic momentum grid), Coulomb v with coupling {m['coupling']}, box {m['lbox']:.4f}, "
                          f"Fermi-Dirac start T={m['temperature']}, mu={m['mu']}, dt={s.dt}, RK4, {s.nsteps} steps",
              "nb": nb, "g2_elements": int(n2), "selfenergy": se.upper(), "parallelism": "single GPU"}
    out = base_line(args, 1e3 / ms_step, ms_step, "f64", config)
    out.update({
        "roofline": roof,
        "kernels": kernel_table(f64["prof"]),
        "energy_drift_rel": drift,
        "mixed": {"dtype": "f32 G2 stage copies / f64 state and arithmetic", "value": round(1e3 / mx_step, 3),
                  "ms_per_step": round(mx_step, 6), "speedup_vs_fp64": round(ms_step / mx_step, 3),
                  "err_G1_vs_fp64": err["G1"], "err_E_vs_fp64": err["E"],
                  "roofline": {"kernel": "jel_stage", "achieved": round(mach, 2), "peak": PEAK_HBM,
                               "unit": "GB/s", "frac": round(mach / PEAK_HBM, 4), "bytes_per_launch": mbytes,
                               "traffic": traffic("jel_stage/gw/mixed") if se == "gw" else None},
                  "kernels": kernel_table(mx["prof"])},
    })
    if ladder:
        out["stage_roofline" if roof is lad_roof else "ladder_roofline"] = stage_roof if roof is lad_roof else lad_roof
        out["mixed"]["ladder_roofline"] = mx_lad
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline_jellium(s, se)
    return out


def cpu_baseline_jellium(system, se, seconds: float = 12.0):
    """The oracle's jellium right-hand side on the host cores at the workload's
    initial state, over a bounded number of evaluations; four per RK4 step."""
    import torch
    from oracle import jellium as OJ
    nthreads = torch.get_num_threads()
    g1 = torch.as_tensor(system.g1, dtype=torch.complex128)
    nb = system.nb
    g2 = torch.zeros((2, 2, nb, nb, nb), dtype=torch.complex128)
    if se in ("soa", "gw"):   # warm-up (one T-matrix right-hand side takes seconds to a minute)
        OJ.rhs(system.eps, system.v, g1, g2, system.dims, se)
    n, t0 = 0, time.perf_counter()
    while True:
        OJ.rhs(system.eps, system.v, g1, g2, system.dims, se)
        n += 1
        el = time.perf_counter() - t0
        if el > seconds or n >= 20:
            break
    per = el / n
    return {"value": round(1.0 / (4.0 * per), 5), "unit": "RK4 steps/s", "cores": nthreads, "kind": "oracle",
            "sample": f"{n} right-hand sides of the jellium workload (torch CPU complex128, {nthreads} threads, "
                      f"{el:.1f} s, {per:.2f} s each), four per RK4 step", "host": host_info()}


def cpu_baseline_batch(clusters, seconds: float = 15.0, selfenergy: str = "tpp"):
    """Oracle on the host: one RK4 step per cluster for the first clusters of the
    batch until the time budget is spent; the whole-batch rate is extrapolated
    with the G2 element count (the oracle's per-step cost is proportional to it)."""
    import torch
    from oracle import integrate as OI
    nthreads = torch.get_num_threads()
    t0 = time.perf_counter()
    el_done, q = 0, 0
    while q < len(clusters) and time.perf_counter() - t0 < seconds:
        c = clusters[q]
        f = OI.hubbard_rhs_fn(c, selfenergy)
        y = OI.hubbard_initial(c, selfenergy)
        OI.rk4_step(f, 0.0, y, c.dt)
        el_done += c.ns ** 4
        q += 1
    el = time.perf_counter() - t0
    total = sum(c.ns ** 4 for c in clusters)
    return {"value": round(el_done / total / el, 6), "unit": "RK4 steps/s", "cores": nthreads,
            "kind": "oracle",
            "sample": f"one RK4 step of the first {q} of {len(clusters)} clusters ({el:.1f} s), "
                      f"extrapolated to the whole batch by G2 element count"}


def run_copy_calibration(args, torch):
    """A plain device copy of 1 GiB (torch's copy kernel), four times: the
    achievable copy bandwidth of the part, and the program that calibrates the
    HBM traffic counters (its FETCH_SIZE / WRITE_SIZE per dispatch correspond to
    1 GiB read and 1 GiB written)."""
    n = (1 << 30) // 8
    a = torch.ones(n, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    reps = 4
    ev0.record()
    for _ in range(reps):
        b.copy_(a)
    ev1.record()
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1) / reps
    gbs = 2.0 * (1 << 30) / (ms * 1e-3) / 1e9
    return {"metric": "device copy bandwidth (read + write)", "value": round(gbs, 1), "unit": "GB/s",
            "n_gpus": 1, "higher_is_better": True, "vs_baseline": None, "dtype": "f64", "data": "synthetic",
            "config": {"workload": "copy of a 1 GiB device buffer, 4 repetitions"},
            "ms_per_copy": round(ms, 4), "frac_of_peak": round(gbs / PEAK_HBM, 4)}


def run_scaling(args, torch, B):
    """Cost of an RK4 step against the basis size, fitted as a power law, next
    to the paper's scalings (Sec. VII, Tab. I): general basis SOA ~ Nb^5, GW
    ~ Nb^6; Hubbard basis ~ Ns^4 after the reformulations; and cost linear in
    the number of steps.  Timing only (graph-replayed steps, binary64)."""
    import numpy as np
    from workloads import adjoint_system, general_system, gw_system
    stream = torch.cuda.Stream()

    def per_step(p, dt, steps, warm):
        ms, _ = timed_steps(p, dt, steps, warm, stream, torch)
        return ms / steps

    def fit(rows):
        x = np.log([r[0] for r in rows])
        y = np.log([r[1] for r in rows])
        return {"all_sizes": round(float(np.polyfit(x, y, 1)[0]), 3),
                "two_largest": round(float((y[-1] - y[-2]) / (x[-1] - x[-2])), 3)}

    res = {}
    rows = []
    for nb in (16, 32, 48, 64):
        sy = general_system(nb=nb, rank=2 * nb, nocc=nb // 4)
        p = B.Propagator(B.GENERAL, B.SOA, nb, sy.h0, sy.g1, w=sy.w, stream=stream.cuda_stream)
        rows.append((nb, per_step(p, sy.dt, 48 if nb <= 32 else 16, 8)))
        if nb == 32:   # linear in the number of steps
            t1 = per_step(p, sy.dt, 64, 0) * 64
            t2 = per_step(p, sy.dt, 128, 0) * 128
            res["steps_ratio_128_over_64"] = round(t2 / t1, 3)
        p.close()
    res["general_soa"] = {"ms_per_step": {str(n): round(t, 5) for n, t in rows}, "exponent": fit(rows), "paper": 5}
    rows = []
    for nb in (16, 32, 48, 64):
        sy = gw_system(nb=nb, rank=2 * nb, nocc=nb // 4)
        p = B.Propagator(B.GENERAL, B.GW, nb, sy.h0, sy.g1, w=sy.w, stream=stream.cuda_stream)
        rows.append((nb, per_step(p, sy.dt, 16 if nb <= 32 else 4, 4 if nb <= 32 else 1)))
        p.close()
    res["general_gw"] = {"ms_per_step": {str(n): round(t, 5) for n, t in rows}, "exponent": fit(rows), "paper": 6}
    rows = []
    for lx, ly in ((4, 4), (4, 6), (6, 6), (6, 8), (8, 8)):
        sy = adjoint_system(lx=lx, ly=ly)    # open lx x ly cluster; its drive is not set
        p = B.Propagator(B.HUBBARD, B.SOA, sy.ns, sy.h0, sy.g1, U=sy.U, stream=stream.cuda_stream)
        rows.append((sy.ns, per_step(p, sy.dt, 40, 8)))
        p.close()
    res["hubbard_soa"] = {"ms_per_step": {str(n): round(t, 5) for n, t in rows}, "exponent": fit(rows), "paper": 4}
    return {
        "metric": "cost of an RK4 step against the basis size: fitted exponents (Tab. I)",
        "value": res["general_soa"]["exponent"]["two_largest"], "unit": "exponent (general SOA, Nb 48 -> 64)",
        "n_gpus": 1, "higher_is_better": False, "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "general SOA Nb 16-64, general GW Nb 16-64, Hubbard SOA open clusters Ns 16-64"},
        "scaling_fit": res,
    }


def run_batch(args, torch, B):
    import numpy as np
    from paper_2002_12717_amd import autotune
    from workloads import batched_clusters
    clusters = batched_clusters()
    ns = [c.ns for c in clusters]
    n4 = float(sum(n ** 4 for n in ns))
    stream = torch.cuda.Stream()
    dt = clusters[0].dt
    se = args.selfenergy or "tpp"
    res = {}
    for prec in ("fp64", "mixed"):
        b = autotune.make_batch(B, clusters, SE_CODES[se](B), stream=stream.cuda_stream,
                                precision=B.FP64 if prec == "fp64" else B.MIXED)
        ms, wall = timed_steps(b, dt, args.steps, args.warmup, stream, torch)
        g1 = [b.get_cluster(q, with_g2=False)[0] for q in range(len(ns))]
        obs = b.observables()
        prof = b.profile(dt, args.profile_steps)
        b.close()
        res[prec] = dict(ms=ms, g1=g1, obs=obs, prof=prof)
    f64, mx = res["fp64"], res["mixed"]
    ms_step = f64["ms"] / args.steps
    mx_step = mx["ms"] / args.steps
    tot_ms, cnt = f64["prof"]["hub_stage"]
    # algorithmic bytes per G2 element and RK4 step: 256 (binary64 stage copies)
    # or 208 (binary32 stage copies); the four stage launches share them
    nch = HUB_CHANNELS[se]
    bytes_per_launch = 64.0 * n4 * nch
    achieved = bytes_per_launch * cnt / (tot_ms * 1e-3) / 1e9
    mx_tot, mx_cnt = mx["prof"]["hub_stage"]
    mx_bytes = 52.0 * n4 * nch
    mx_ach = mx_bytes * mx_cnt / (mx_tot * 1e-3) / 1e9
    err_g1 = max(float(np.abs(m - f).max() / np.abs(f).max()) for m, f in zip(mx["g1"], f64["g1"]))
    err_e = max(abs(m["E_tot"] - f["E_tot"]) / max(abs(f["E_tot"]), 1.0)
                for m, f in zip(mx["obs"], f64["obs"]))
    config = {"workload": f"ragged batch of {len(ns)} periodic 2D Hubbard clusters (Lx,Ly in 3..6), "
                          f"{se.upper()}, dt={dt}, RK4, one launch per stage, graph-captured steps",
              "clusters": len(ns), "g2_elements": int(n4), "ns_min": min(ns), "ns_max": max(ns),
              "selfenergy": se.upper(), "stage_kernel": autotune.load_table().get("kernel", "library default"),
              "chunk_per_class": autotune.load_table().get("chunk_per_class"),
              "parallelism": "single GPU"}
    out = base_line(args, 1e3 / ms_step, ms_step, "f64", config)
    out.update({
        "roofline": {"kernel": "hub_stage", "bound": "hbm", "achieved": round(achieved, 2),
                     "peak": PEAK_HBM, "unit": "GB/s", "frac": round(achieved / PEAK_HBM, 4),
                     "traffic": None, "kernel_ms_avg": round(tot_ms / cnt, 6),
                     "bytes_per_launch": bytes_per_launch, "launches": cnt},
        "kernels": kernel_table(f64["prof"]),
        "mixed": {"dtype": "f32 G2 stage copies / f64 state and arithmetic",
                  "value": round(1e3 / mx_step, 3), "ms_per_step": round(mx_step, 6),
                  "speedup_vs_fp64": round(ms_step / mx_step, 3),
                  "err_G1_vs_fp64": err_g1, "err_E_vs_fp64": err_e,
                  "roofline": {"kernel": "hub_stage", "achieved": round(mx_ach, 2), "peak": PEAK_HBM,
                               "unit": "GB/s", "frac": round(mx_ach / PEAK_HBM, 4),
                               "bytes_per_launch": mx_bytes},
                  "kernels": kernel_table(mx["prof"])},
        "diverged": any(bool(o["diverged"]) for o in f64["obs"]),
        "one_cluster_at_a_time": one_at_a_time(clusters, se, stream, torch, B, ms_step),
    })
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline_batch(clusters, selfenergy=se)
    return out


def one_at_a_time(clusters, se, stream, torch, B, batch_ms_step, steps: int = 16):
    """The same clusters propagated one after another, each in its own
    single-cluster context (binary64, graph-captured steps): one context per
    distinct cluster size is timed and the per-step times are summed over the
    batch's clusters."""
    per_ns = {}
    for c in clusters:
        if c.ns in per_ns:
            continue
        p = B.Propagator(B.HUBBARD, SE_CODES[se](B), c.ns, c.h0, c.g1, U=c.U, stream=stream.cuda_stream)
        ms, _ = timed_steps(p, c.dt, steps, 2, stream, torch)
        p.close()
        per_ns[c.ns] = ms / steps
    seq = sum(per_ns[c.ns] for c in clusters)
    return {"ms_per_step": round(seq, 4), "batch_speedup": round(seq / batch_ms_step, 3),
            "ms_per_step_by_ns": {str(k): round(v, 5) for k, v in sorted(per_ns.items())}}


def cpu_baseline_adjoint(seconds: float = 15.0):
    """The oracle's gradient (torch autograd through the RK4 map, CPU, binary64)
    on the reduced 4x4 driven cluster, as many steps as fit the time budget,
    extrapolated to the 8x8 cluster by the G2 element count (64^4 / 16^4)."""
    import numpy as np
    import torch
    from oracle import adjoint as OA
    from workloads import adjoint_system
    nthreads = torch.get_num_threads()
    s = adjoint_system(lx=4, ly=4, nmodes=16, T=0.4, dt=0.01)
    a = np.full(s.ns, 1.0 / s.ns)
    b = np.zeros(s.ns)
    n = 10
    t0 = time.perf_counter()
    OA.loss_and_gradient(s, a, b, nsteps=n)
    el = time.perf_counter() - t0
    if el < seconds / 4:
        n = max(n, int(n * seconds / max(el, 1e-3) / 2))
        t0 = time.perf_counter()
        OA.loss_and_gradient(s, a, b, nsteps=n)
        el = time.perf_counter() - t0
    scale = (16.0 / 64.0) ** 4
    return {"value": round(n / el * scale, 6), "unit": "gradient RK4 steps/s", "cores": nthreads,
            "kind": "oracle",
            "sample": f"autograd gradient of the mean double occupation over {n} RK4 steps of the "
                      f"4x4 driven cluster ({el:.1f} s), scaled by (16/64)^4 to the 8x8 cluster"}


def run_adjoint(args, torch, B):
    """Gradients of the final-time mean double occupation and of the density
    imbalance of the driven 8x8 cluster with respect to the 64 drive
    coefficients and U: one checkpointed forward pass and two reverse sweeps."""
    import numpy as np
    from workloads import adjoint_system
    s = adjoint_system()
    ns = s.ns
    stream = torch.cuda.Stream()
    p = B.Propagator(B.HUBBARD, B.SOA, ns, s.h0, s.g1, U=s.U, stream=stream.cuda_stream)
    d = s.drive
    p.set_drive(d.x, d.c, d.t_center, d.tau)
    nmodes = len(d.c)
    a_docc, b_docc = np.full(ns, 1.0 / ns), np.zeros(ns)
    npart = float(np.trace(-1j * s.g1[0]).real + np.trace(-1j * s.g1[1]).real)
    side = (d.x < 0).astype(np.float64) - (d.x > 0).astype(np.float64)
    a_imb, b_imb = np.zeros(ns), side / npart
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    p.forward_checkpointed(s.dt, args.steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    L1, g1c, g1U = p.adjoint(a_docc, b_docc, nmodes)
    t2 = time.perf_counter()
    L2, g2c, g2U = p.adjoint(a_imb, b_imb, nmodes)
    t3 = time.perf_counter()
    obs = p.observables()
    # per-kernel times of one more reverse sweep (events after every launch)
    aprof = p.profile_adjoint(a_docc, b_docc)
    prof = p.profile(s.dt, args.profile_steps)
    p.close()
    fwd_ms = (t1 - t0) * 1e3
    rev_ms = (t3 - t1) * 1e3 / 2
    total_ms = fwd_ms + 2 * rev_ms
    ms_step = total_ms / args.steps
    tot_ms, cnt = prof["hub_stage"]
    bytes_per_launch = 64.0 * float(ns) ** 4
    achieved = bytes_per_launch * cnt / (tot_ms * 1e-3) / 1e9
    # adj_slice_red, the reverse sweep's dominant kernel: per G2 element it reads
    # the cotangent, the stage state, lambda and the running sum and writes the
    # running sum and the next cotangent where the stage has them: 64, 96, 96
    # and 64 B over the four stages of a step, 80 B per launch on average
    a_tot, a_cnt = aprof["adj_slice_red"]
    a_bytes = 80.0 * float(ns) ** 4
    a_ach = a_bytes * a_cnt / (a_tot * 1e-3) / 1e9
    config = {"workload": f"gradient of the final-time mean double occupation and density imbalance "
                          f"of the driven 8x8 Hubbard cluster (SOA, U={s.U}, {nmodes} Gaussian pulses) "
                          f"with respect to the pulse coefficients and U, checkpointed discrete adjoint "
                          f"of RK4, dt={s.dt}",
              "ns": ns, "U": s.U, "dt": s.dt, "nsteps": args.steps, "selfenergy": "SOA",
              "parallelism": "single GPU"}
    out = base_line(args, 1e3 / ms_step, ms_step, "f64", config)
    out["unit"] = "gradient RK4 steps/s"
    out.update({
        "forward_ms": round(fwd_ms, 3), "reverse_ms_per_loss": round(rev_ms, 3),
        "roofline": {"kernel": "adj_slice_red", "bound": "hbm", "achieved": round(a_ach, 2),
                     "peak": PEAK_HBM, "unit": "GB/s", "frac": round(a_ach / PEAK_HBM, 4),
                     "traffic": None, "kernel_ms_avg": round(a_tot / a_cnt, 6),
                     "bytes_per_launch": a_bytes, "launches": a_cnt},
        "forward_roofline": {"kernel": "hub_stage", "bound": "hbm", "achieved": round(achieved, 2),
                             "peak": PEAK_HBM, "unit": "GB/s", "frac": round(achieved / PEAK_HBM, 4),
                             "kernel_ms_avg": round(tot_ms / cnt, 6), "bytes_per_launch": bytes_per_launch,
                             "launches": cnt},
        "adjoint_kernels": kernel_table(aprof),
        "losses": {"docc": L1, "imbalance": L2},
        "grad_norms": {"docc_c": float(np.linalg.norm(g1c)), "docc_U": g1U,
                       "imbalance_c": float(np.linalg.norm(g2c)), "imbalance_U": g2U},
        "observables": {k: obs[k] for k in ("t", "E_tot", "docc", "imbalance")},
    })
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline_adjoint()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None,
                    help="timed RK4 steps (default: 40 for general_gw and general_ladder, 500 otherwise)")
    ap.add_argument("--warmup", type=int, default=None, help="untimed steps before them (default 8 / 20)")
    ap.add_argument("--profile-steps", type=int, default=None,
                    help="steps of the per-launch profile (default 8 for the Nb = 64 workloads, 50 otherwise)")
    ap.add_argument("--no-accuracy", action="store_true",
                    help="skip the full-length accuracy runs of the general workloads")
    ap.add_argument("--no-extra", action="store_true",
                    help="general_gw: skip the Nb = 32 SOA line reported beside the headline")
    ap.add_argument("--workload", default="general_gw",
                    choices=["general_soa", "general_gw", "general_ladder", "hubbard_chain",
                             "hubbard_2d", "hubbard_batch", "hubbard_adjoint", "jellium", "scaling",
                             "copy_calibration"])
    ap.add_argument("--selfenergy", default=None, choices=["soa", "gw", "tpp", "tph", "dsl"],
                    help="Hubbard workloads: override the workload's selfenergy (hubbard_batch: "
                         "TPP, hubbard_chain/hubbard_2d: SOA; any of the five); general_ladder: "
                         "tpp, tph or dsl (default dsl)")
    ap.add_argument("--ns", type=int, default=8,
                    help="hubbard_chain: number of sites (default 8; 2-7 take the persistent kernel)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this G1-G2 workload runs on a single MI355X; "
              "use --gpus 1", file=sys.stderr)
        sys.exit(2)
    big = args.workload in ("general_gw", "general_ladder")
    if args.steps is None:
        args.steps = 40 if big else 500
    if args.warmup is None:
        args.warmup = 8 if big else 20
    if args.profile_steps is None:
        args.profile_steps = 8 if big else 50
    import torch
    from paper_2002_12717_amd import binding as B
    torch.cuda.set_device(0)
    if args.workload == "general_soa":
        out = run_general(args, torch, B, accuracy=not args.no_accuracy)
    elif args.workload == "general_gw":
        out = run_general(args, torch, B, se="gw", accuracy=not args.no_accuracy)
        if not args.no_extra:   # the Nb = 32 SOA workload beside it, its own step counts
            out["general_soa_nb32"] = summary(run_general(args, torch, B, se="soa", accuracy=not args.no_accuracy,
                                                          steps=500, warmup=20, profile_steps=50))
    elif args.workload == "general_ladder":
        se = args.selfenergy or "dsl"
        if se not in ("tpp", "tph", "dsl"):
            ap.error("general_ladder takes --selfenergy tpp, tph or dsl")
        out = run_general(args, torch, B, se=se, accuracy=False)
    elif args.workload == "hubbard_batch":
        out = run_batch(args, torch, B)
    elif args.workload == "scaling":
        out = run_scaling(args, torch, B)
    elif args.workload == "hubbard_adjoint":
        out = run_adjoint(args, torch, B)
    elif args.workload == "jellium":
        out = run_jellium(args, torch, B)
    elif args.workload == "copy_calibration":
        out = run_copy_calibration(args, torch)
    else:
        out = run_hubbard(args, torch, B, args.workload)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
