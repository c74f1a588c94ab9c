"""Autotuner of the ragged Hubbard batch.  It first chooses the stage kernel
(the slice kernel, the row kernel, or the per-element kernel, which negative
chunks select), then, per cluster size class, the number of G2 elements one
work-group of the flat work list of g1g2_batch_init handles: for the slice
kernel the most elements a work item stages in LDS (whole (i,j) slices; the
launch sizes its LDS for the longest item, so shorter items leave room for
more work-groups per compute unit), for the row kernel its granularity
(rounded to whole wave units of rows), for the per-element kernel its
elements per work-group.  Coordinate descent over the classes; each candidate
is timed with HIP events over whole RK4 steps on the real batch.  The table is
written as JSON and read back by ``chunks_for`` and ``flags_for``.
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
# slice kernel: elements per work item (4096 is the library's default and limit)
CANDIDATES_SLICE = [1024, 2048, 3072, 4096]
DEFAULT = 1024
START = {"slice": 4096, "row": DEFAULT, "element": -256}


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


KERNELS = ("slice", "row", "element")


def chunks_for(ns_list, table=None):
    table = load_table() if table is None else table
    per = table.get("chunk_per_class", [DEFAULT] * len(CLASSES))
    return [int(per[class_of(n)]) for n in ns_list]


def flags_for(table=None) -> int:
    """g1g2_desc flags that select the tuned stage kernel (0: the library's choice)."""
    from . import binding as B
    table = load_table() if table is None else table
    return {"slice": B.HUB_SLICE_KERNEL, "row": B.HUB_ROW_KERNEL}.get(table.get("kernel"), 0)


def make_batch(B, clusters, selfenergy, stream=0, precision=None, table=None):
    """g1g2_batch_init of the clusters with the stage kernel and the per-class
    chunks of the tuning table (the stored one by default)."""
    table = load_table() if table is None else table
    ns = [c.ns for c in clusters]
    return B.Batch(selfenergy, ns, [c.U for c in clusters], [c.h0 for c in clusters],
                   [c.g1 for c in clusters], chunk=chunks_for(ns, table), stream=stream,
                   precision=B.FP64 if precision is None else precision, flags=flags_for(table))


def _time(B, torch, clusters, selfenergy, chunks, steps, stream, flags=0):
    b = B.Batch(selfenergy, [c.ns for c in clusters], [c.U for c in clusters],
                [c.h0 for c in clusters], [c.g1 for c in clusters], chunk=chunks,
                stream=stream.cuda_stream, flags=flags)
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
    kflags = {"slice": B.HUB_SLICE_KERNEL, "row": B.HUB_ROW_KERNEL, "element": 0}
    best, base, kernel = None, float("inf"), None
    for kern in KERNELS:
        trial = [START[kern]] * len(CLASSES)
        ms = _time(B, torch, clusters, se, [trial[class_of(n)] for n in ns], steps, stream, kflags[kern])
        log.append({"kernel": kern, "chunk_per_class": trial, "ms_per_step": ms})
        print(f"kernel {kern} {trial} {ms:.3f} ms/step", flush=True)
        if ms < base:
            base, best, kernel = ms, trial, kern
    cands = {"slice": CANDIDATES_SLICE, "row": CANDIDATES_ROW, "element": CANDIDATES_FLAT}[kernel]
    for q in range(len(CLASSES)):
        for cand in cands:
            if cand == best[q]:
                continue
            trial = list(best)
            trial[q] = cand
            ms = _time(B, torch, clusters, se, [trial[class_of(n)] for n in ns], steps, stream,
                       kflags[kernel])
            log.append({"kernel": kernel, "chunk_per_class": trial, "ms_per_step": ms})
            print(f"class {q} chunk {cand}: {ms:.3f} ms/step", flush=True)
            if ms < base:
                base, best = ms, trial
    table = {"kernel": kernel, "chunk_per_class": best, "classes_ns": CLASSES, "ms_per_step": base,
             "workload": f"{n_clusters} periodic 2D Hubbard clusters, {selfenergy_name.upper()}",
             "device": torch.cuda.get_device_name(0), "date": time.strftime("%Y-%m-%d"),
             "trials": log}
    os.makedirs(os.path.dirname(out), exist_ok=True)
    with open(out, "w") as f:
        json.dump(table, f, indent=1)
    print("best", kernel, best, f"{base:.3f} ms/step ->", out, flush=True)
    return table


if __name__ == "__main__":
    tune(out=sys.argv[1] if len(sys.argv) > 1 else TABLE)
