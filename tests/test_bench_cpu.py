"""Host-side checks of bench.py (no GPU): the one-GPU contract, the
algorithmic counts the roofline divides by, and the rule that ties stored
traffic counters to the code they were taken on."""
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=300)
    assert r.returncode != 0
    assert "--gpus 1" in r.stderr
    assert r.stdout.strip() == ""                 # no JSON line for a refused run


def test_algorithmic_counts():
    # 8 real flops per complex multiply-add: the T sandwich (2 Nb^5 in gen_vt and
    # 2 Nb^5 in gen_main), the commutator (2 Nb^5) and I (1 Nb^5); Pi is Nb^6
    nb = 32
    f = bench.soa_flops(nb)
    assert f["gen_vt"] == 16 * nb ** 5 and f["gen_main"] == 40 * nb ** 5 and f["soa_total"] == 56 * nb ** 5
    g = bench.gw_flops(64)
    assert g["gen_gemm"] == 8 * 64 ** 6 and g["gen_heps"] == 16 * 64 ** 5


def test_source_hash_ignores_comments_not_code(tmp_path, monkeypatch):
    csrc = tmp_path / "paper_2002_12717_amd" / "csrc"
    csrc.mkdir(parents=True)
    (csrc / "a.hip").write_text("// header\nint f(int x) { return x + 1; }  /* note */\n")
    (csrc / "b.hip").write_text("int f(int x)\n{\n    return x + 1;   // the same code\n}\n")
    (csrc / "c.hip").write_text("int f(int x) { return x + 2; }\n")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.source_hash("a.hip") == bench.source_hash("b.hip")
    assert bench.source_hash("a.hip") != bench.source_hash("c.hip")
