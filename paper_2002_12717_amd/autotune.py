"""Autotuner of the ragged Hubbard batch.  It first chooses the stage kernel
(row kernel: positive chunks; per-element kernel: negative chunks), then, per
cluster size class, the number of G2 elements handled by one work-group of
the flat work list of g1g2_batch_init (the row kernel rounds it to whole wave
units of rows).  Coordinate descent over the classes; each candidate is timed
with HIP events over whole RK4 steps on the real batch.  The table is written
as JSON and read back by ``chunks_for``.
"""
from __future__ import annotations

import json
import os
import sys
import time

PKG = os.path.dirname(os.path.abspath(__file__))
TABLE = os.path.join(PKG, "tuning", "hubbard_batch.json")
CLASSES = [(1, 16), (17, 25), (26, 49)]          # ns ranges (inclusive)
# > 0: row stage kernel (elements per work-group, rounded to whole wave units);
# < 0: per-element stage kernel with |value| elements per work-group
CANDIDATES_ROW = [256, 512, 1024, 2048, 4096]
CANDIDATES_FLAT = [-256, -512, -1024, -2048]
DEFAULT = 1024


def class_of(ns: int) -> int:
    for q, (lo, hi) in enumerate(CLASSES):
        if lo <= ns <= hi:
            return q
    return len(CLASSES) - 1


def load_table(path: str = TABLE) -> dict:
    if os.path.exists(path):
        with open(path) as f:
            return json.load(f)
    return {}


def chunks_for(ns_list, table=None):
    table = load_table() if table is None else table
    per = table.get("chunk_per_class", [DEFAULT] * len(CLASSES))
    return [int(per[class_of(n)]) for n in ns_list]


def _time(B, torch, clusters, selfenergy, chunks, steps, stream):
    b = B.Batch(selfenergy, [c.ns for c in clusters], [c.U for c in clusters],
                [c.h0 for c in clusters], [c.g1 for c in clusters], chunk=chunks,
                stream=stream.cuda_stream)
    dt = clusters[0].dt
    b.step(dt, 2)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    b.step(dt, steps)
    e1.record(stream)
    torch.cuda.synchronize()
    b.close()
    return e0.elapsed_time(e1) / steps


def tune(n_clusters: int = 512, steps: int = 8, selfenergy_name: str = "tpp", out: str = TABLE):
    import torch
    sys.path.insert(0, os.path.dirname(PKG))
    from paper_2002_12717_amd import binding as B
    from workloads import batched_clusters
    clusters = batched_clusters(n=n_clusters)
    se = B.TPP if selfenergy_name == "tpp" else B.SOA
    stream = torch.cuda.Stream()
    ns = [c.ns for c in clusters]
    log = []
    # the kernel variant is global: pick it first with uniform chunks
    best, base = None, float("inf")
    for start in (DEFAULT, -256):
        trial = [start] * len(CLASSES)
        ms = _time(B, torch, clusters, se, [trial[class_of(n)] for n in ns], steps, stream)
        log.append({"chunk_per_class": trial, "ms_per_step": ms})
        print(f"start {trial} {ms:.3f} ms/step", flush=True)
        if ms < base:
            base, best = ms, trial
    cands = CANDIDATES_ROW if best[0] > 0 else CANDIDATES_FLAT
    for q in range(len(CLASSES)):
        for cand in cands:
            if cand == best[q]:
                continue
            trial = list(best)
            trial[q] = cand
            ms = _time(B, torch, clusters, se, [trial[class_of(n)] for n in ns], steps, stream)
            log.append({"chunk_per_class": trial, "ms_per_step": ms})
            print(f"class {q} chunk {cand}: {ms:.3f} ms/step", flush=True)
            if ms < base:
                base, best = ms, trial
    table = {"chunk_per_class": best, "classes_ns": CLASSES, "ms_per_step": base,
             "workload": f"{n_clusters} periodic 2D Hubbard clusters, {selfenergy_name.upper()}",
             "device": torch.cuda.get_device_name(0), "date": time.strftime("%Y-%m-%d"),
             "trials": log}
    os.makedirs(os.path.dirname(out), exist_ok=True)
    with open(out, "w") as f:
        json.dump(table, f, indent=1)
    print("best", best, f"{base:.3f} ms/step ->", out, flush=True)
    return table


if __name__ == "__main__":
    tune(out=sys.argv[1] if len(sys.argv) > 1 else TABLE)
