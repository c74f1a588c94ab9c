"""CPU checks of the C-ABI library: it builds for gfx950, loads, and exports
every function that include/g1g2.h declares (no compute call needs a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    txt = open(os.path.join(ROOT, "include", "g1g2.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(g1g2_[a-z0-9_]+)\s*\(", txt)))


@pytest.fixture(scope="module")
def so_path():
    from paper_2002_12717_amd import build
    if not os.path.exists(build.LIB):
        build.build()
    return build.LIB


def test_header_declares_the_boundary():
    names = _declared()
    for n in ("g1g2_init", "g1g2_rhs", "g1g2_step_rk4", "g1g2_observables", "g1g2_destroy"):
        assert n in names


def test_library_exports_every_declared_symbol(so_path):
    lib = ctypes.CDLL(so_path)
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_signatures_cover_header(so_path):
    from paper_2002_12717_amd import binding
    lib = binding.load(so_path)
    for n in _declared():
        assert n in binding._SIGS, n
        assert getattr(lib, n).argtypes is not None or n in ("g1g2_strerror",)


def test_strerror_needs_no_device(so_path):
    from paper_2002_12717_amd import binding
    lib = binding.load(so_path)
    assert lib.g1g2_strerror(-5) == b"propagation diverged"
    assert lib.g1g2_strerror(0) == b"ok"


def test_init_rejects_bad_arguments_without_device(so_path):
    """Argument validation happens before any device call."""
    from paper_2002_12717_amd import binding
    lib = binding.load(so_path)
    ctx = ctypes.c_void_p()
    d = binding.Desc(0, 0, 0, 0, 0, 0.0)       # nb = 0
    assert lib.g1g2_init(ctypes.byref(ctx), ctypes.byref(d), None, None, None, None, None) == binding.EINVAL
    buf = (ctypes.c_double * 64)()
    d = binding.Desc(0, binding.SOA, 0, 0, 65, 0.0)  # the general basis stops at nb = 64
    assert lib.g1g2_init(ctypes.byref(ctx), ctypes.byref(d), buf, buf, buf, None, None) == binding.EUNSUPPORTED
    d = binding.Desc(0, binding.SOA, 0, binding.DSL_EXCHANGE, 4, 0.0)   # a DSL-only flag
    assert lib.g1g2_init(ctypes.byref(ctx), ctypes.byref(d), buf, buf, buf, None, None) == binding.EUNSUPPORTED
    d = binding.Desc(0, 5, 0, 0, 4, 0.0)             # no such selfenergy
    assert lib.g1g2_init(ctypes.byref(ctx), ctypes.byref(d), buf, buf, buf, None, None) == binding.EINVAL


def test_batch_init_rejects_empty_batch(so_path):
    """A batch needs at least one cluster; checked before any device call."""
    from paper_2002_12717_amd import binding
    lib = binding.load(so_path)
    ctx = ctypes.c_void_p()
    d = binding.Desc(1, binding.TPP, 0, 0, 4, 0.0)
    assert lib.g1g2_batch_init(ctypes.byref(ctx), ctypes.byref(d), 0, None, None, None, None, None,
                               None) == binding.EINVAL


def test_autotune_table_lookup():
    """The autotuner's table maps cluster sizes to chunks by class and names
    the stage kernel by its g1g2_desc flag."""
    from paper_2002_12717_amd import autotune
    from paper_2002_12717_amd import binding as B
    table = {"kernel": "row", "chunk_per_class": [256, 512, 4096]}
    assert autotune.chunks_for([9, 16, 17, 25, 26, 36], table) == [256, 256, 512, 512, 4096, 4096]
    assert autotune.flags_for(table) == B.HUB_ROW_KERNEL
    assert autotune.flags_for({"kernel": "slice"}) == B.HUB_SLICE_KERNEL
    assert autotune.flags_for({"kernel": "element"}) == 0
    assert autotune.flags_for({}) == 0


def test_tuning_table_drives_batch_init(monkeypatch):
    """The batch the benchmark and the tests build takes the tuning table's
    stage kernel and per-class chunks as the g1g2_batch_init arguments."""
    import numpy as np
    from paper_2002_12717_amd import autotune
    from paper_2002_12717_amd import binding as B
    from workloads import batched_clusters
    seen = {}

    class FakeLib:
        def g1g2_batch_init(self, ctx, desc, n, ns, U, h0, g1, chunk, stream):
            seen["flags"] = desc._obj.flags
            seen["n"] = n
            seen["chunk"] = np.ctypeslib.as_array(ctypes.cast(chunk, ctypes.POINTER(ctypes.c_int32)),
                                                  (n,)).copy()
            return B.OK

        def g1g2_destroy(self, ctx):
            pass

    monkeypatch.setattr(B, "load", lambda *a: FakeLib())
    cl = batched_clusters(n=40)
    table = {"kernel": "slice", "chunk_per_class": [1024, 2048, 3072]}
    b = autotune.make_batch(B, cl, B.TPP, table=table)
    assert seen["flags"] == B.HUB_SLICE_KERNEL and seen["n"] == 40
    want = [1024 if c.ns <= 16 else (2048 if c.ns <= 25 else 3072) for c in cl]
    assert list(seen["chunk"]) == want and len(set(want)) > 1
    b.ctx = None
    table = {"kernel": "row", "chunk_per_class": [256, 512, 4096]}
    autotune.make_batch(B, cl, B.TPP, table=table)
    assert seen["flags"] == B.HUB_ROW_KERNEL
    assert list(seen["chunk"]) == [256 if c.ns <= 16 else (512 if c.ns <= 25 else 4096) for c in cl]


def test_jellium_init_rejects_bad_arguments_without_device(so_path):
    """Jellium argument checks precede any device call: the grid must match
    nb, v[0] must vanish, and DSL is not offered."""
    import numpy as np
    from paper_2002_12717_amd import binding
    lib = binding.load(so_path)
    ctx = ctypes.c_void_p()
    dims = np.array([2, 2, 1], np.int32)
    eps = np.zeros(8)
    v = np.full(4, 0.1)
    g1 = np.zeros(8, np.complex128)
    P = lambda a: a.ctypes.data  # noqa: E731
    d = binding.Desc(binding.JELLIUM, binding.SOA, 0, 0, 5, 0.0)          # nb != 2 * 2 * 1
    v0 = v.copy()
    v0[0] = 0.0
    assert lib.g1g2_jellium_init(ctypes.byref(ctx), ctypes.byref(d), P(dims), P(eps), P(v0), P(g1), None,
                                 None) == binding.EINVAL
    d = binding.Desc(binding.JELLIUM, binding.SOA, 0, 0, 4, 0.0)
    assert lib.g1g2_jellium_init(ctypes.byref(ctx), ctypes.byref(d), P(dims), P(eps), P(v), P(g1), None,
                                 None) == binding.EINVAL                # v[0] != 0
    d = binding.Desc(binding.JELLIUM, binding.DSL, 0, 0, 4, 0.0)
    assert lib.g1g2_jellium_init(ctypes.byref(ctx), ctypes.byref(d), P(dims), P(eps), P(v0), P(g1), None,
                                 None) == binding.EUNSUPPORTED
    d = binding.Desc(binding.JELLIUM, binding.SOA, 0, 0, 4, 0.0)         # g1g2_init is not the entry
    assert lib.g1g2_init(ctypes.byref(ctx), ctypes.byref(d), P(eps), P(v0), P(g1), None, None) == binding.EINVAL
