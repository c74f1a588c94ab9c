"""Thin ctypes binding of libg1g2.so (argument marshalling only).

Every numerical step runs inside the HIP library; this module only converts
Python arguments (numpy arrays on the host, torch tensors on the device) into
the plain pointers and sizes of the C ABI declared in include/g1g2.h.  It
raises if the library is missing: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, c_double, c_int32, c_int64, c_void_p

import numpy as np

PKG = os.path.dirname(os.path.abspath(__file__))
LIBPATH = os.path.join(PKG, "libg1g2.so")

GENERAL, HUBBARD, JELLIUM = 0, 1, 2
SOA, GW, TPP, TPH, DSL = 0, 1, 2, 3, 4
FP64, MIXED = 0, 1
PTR_DEVICE, GW_EXCHANGE, HUB_ROW_KERNEL, HUB_SLICE_KERNEL, DSL_EXCHANGE, JEL_LAD_ROWS2 = 1, 2, 4, 8, 16, 32
OK, EINVAL, ENOMEM, EDEVICE, EUNSUPPORTED, EDIVERGED, ESTATE = 0, -1, -2, -3, -4, -5, -6
PATHS = {0: "general", 1: "hub_persistent", 2: "hub_slice", 3: "hub_row", 4: "hub_element", 5: "jellium"}


class Desc(ctypes.Structure):
    _fields_ = [("basis", c_int32), ("selfenergy", c_int32), ("precision", c_int32),
                ("flags", c_int32), ("nb", c_int32), ("U", c_double)]


class Obs(ctypes.Structure):
    _fields_ = [("t", c_double), ("N", c_double * 2), ("E_kin", c_double), ("E_mf", c_double),
                ("E_corr", c_double), ("E_tot", c_double), ("docc", c_double),
                ("herm_resid", c_double), ("exch_resid", c_double), ("imbalance", c_double),
                ("diverged", c_int32), ("step", c_int64), ("diverged_step", c_int64)]


_SIGS = {
    "g1g2_init": (c_int32, [POINTER(c_void_p), POINTER(Desc), c_void_p, c_void_p, c_void_p, c_void_p,
                            c_void_p]),
    "g1g2_jellium_init": (c_int32, [POINTER(c_void_p), POINTER(Desc), c_void_p, c_void_p, c_void_p, c_void_p,
                                    c_void_p, c_void_p]),
    "g1g2_rhs": (c_int32, [c_void_p, c_double, c_void_p, c_void_p, c_void_p, c_void_p]),
    "g1g2_rhs_noalloc": (c_int32, [c_void_p, c_double, c_void_p, c_void_p, c_void_p, c_void_p]),
    "g1g2_step_rk4": (c_int32, [c_void_p, c_double, c_int64]),
    "g1g2_observables": (c_int32, [c_void_p, POINTER(Obs)]),
    "g1g2_site_observables": (c_int32, [c_void_p, c_void_p, c_void_p, c_void_p]),
    "g1g2_get_state": (c_int32, [c_void_p, c_void_p, c_void_p, POINTER(c_double)]),
    "g1g2_set_state": (c_int32, [c_void_p, c_void_p, c_void_p, c_double]),
    "g1g2_set_h0": (c_int32, [c_void_p, c_void_p]),
    "g1g2_set_U": (c_int32, [c_void_p, c_double]),
    "g1g2_set_drive": (c_int32, [c_void_p, c_void_p, c_int32, c_void_p, c_void_p, c_double]),
    "g1g2_set_switch": (c_int32, [c_void_p, c_double, c_double]),
    "g1g2_profile": (c_int32, [c_void_p, c_double, c_int64, c_int32, c_void_p, c_void_p,
                               POINTER(c_int32)]),
    "g1g2_profile_name": (ctypes.c_char_p, [c_void_p, c_int32]),
    "g1g2_profile_adjoint": (c_int32, [c_void_p, c_void_p, c_void_p, c_int32, c_void_p, c_void_p,
                                       POINTER(c_int32)]),
    "g1g2_prepare_graph": (c_int32, [c_void_p, c_double]),
    "g1g2_step_path": (c_int32, [c_void_p, POINTER(c_int32)]),
    "g1g2_batch_init": (c_int32, [POINTER(c_void_p), POINTER(Desc), c_int32, c_void_p, c_void_p,
                                  c_void_p, c_void_p, c_void_p, c_void_p]),
    "g1g2_batch_observables": (c_int32, [c_void_p, c_void_p]),
    "g1g2_batch_get_state": (c_int32, [c_void_p, c_int32, c_void_p, c_void_p]),
    "g1g2_forward_checkpointed": (c_int32, [c_void_p, c_double, c_int64, c_int32]),
    "g1g2_adjoint": (c_int32, [c_void_p, c_void_p, c_void_p, c_void_p, POINTER(c_double),
                               POINTER(c_double)]),
    "g1g2_destroy": (None, [c_void_p]),
    "g1g2_strerror": (ctypes.c_char_p, [c_int32]),
    "g1g2_last_error": (ctypes.c_char_p, [c_void_p]),
}

_lib = None


def load(path: str = LIBPATH):
    """dlopen libg1g2.so and declare the signatures of every exported call."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with paper_2002_12717_amd.build.build()")
    # torch ships its own HIP runtime under the same soname (libamdhip64.so.7);
    # loading it first makes the library bind to that copy, so the process holds
    # one HIP runtime (loaded the other way round, the system copy binds first and
    # torch's device calls fail)
    import torch  # noqa: F401
    lib = ctypes.CDLL(path)
    for name, (res, args) in _SIGS.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


class G1G2Error(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"status {status}: {msg}")
        self.status = status


def _ptr(x):
    """Raw pointer of a contiguous complex128/float64 numpy array or torch tensor."""
    if x is None:
        return None
    if isinstance(x, np.ndarray):
        if not x.flags.c_contiguous:
            raise ValueError("array must be C-contiguous")
        return x.ctypes.data
    if hasattr(x, "data_ptr"):
        if not x.is_contiguous():
            raise ValueError("tensor must be contiguous")
        return x.data_ptr()
    raise TypeError(type(x))


def _c128(a):
    if a is None:
        return None
    if hasattr(a, "data_ptr"):
        return a
    return np.ascontiguousarray(a, dtype=np.complex128)


class Propagator:
    """One g1g2_ctx.  Host numpy inputs by default; ``device=True`` passes the
    data pointers of device tensors instead (flag G1G2_PTR_DEVICE)."""

    def __init__(self, basis: int, selfenergy: int, nb: int, h0, G1_0, w=None, G2_0=None,
                 U: float = 0.0, precision: int = FP64, flags: int = 0, stream: int = 0,
                 device: bool = False):
        self.lib = load()
        self.basis, self.nb = basis, nb
        self.flags = flags | (PTR_DEVICE if device else 0)
        self.desc = Desc(basis, selfenergy, precision, self.flags, nb, float(U))
        self._keep = [_c128(h0), _c128(G1_0), _c128(w), _c128(G2_0)]
        ctx = c_void_p()
        st = self.lib.g1g2_init(ctypes.byref(ctx), ctypes.byref(self.desc), _ptr(self._keep[0]),
                                _ptr(self._keep[2]), _ptr(self._keep[1]), _ptr(self._keep[3]),
                                c_void_p(stream) if stream else None)
        self._keep = None
        if st != OK:
            raise G1G2Error(st, self.lib.g1g2_strerror(st).decode())
        self.ctx = ctx

    # ------------------------------------------------------------------ helpers
    def _check(self, st: int):
        if st != OK:
            raise G1G2Error(st, self.lib.g1g2_last_error(self.ctx).decode()
                            or self.lib.g1g2_strerror(st).decode())

    def shapes(self):
        """G1 and G2 shapes of the ABI layout; Hubbard GW stores three G2 channels
        (up-down-up-down, up-up-up-up, down-down-down-down), and so does Hubbard DSL;
        jellium keeps the diagonal G1 [2][nb] and the up-up, up-down and down-down
        blocks [3][nb]^3 of G2 in the momentum-transfer layout."""
        nb = self.nb
        if self.basis == JELLIUM:
            return (2, nb), (3, nb, nb, nb)
        g1 = (2, nb, nb) if self.basis == HUBBARD else (nb, nb)
        if self.basis == HUBBARD and self.desc.selfenergy in (GW, DSL):
            return g1, (3, nb, nb, nb, nb)
        return g1, (nb, nb, nb, nb)

    # ------------------------------------------------------------------ ABI calls
    def rhs(self, t: float, G1, G2, dG1, dG2):
        self._check(self.lib.g1g2_rhs(self.ctx, float(t), _ptr(G1), _ptr(G2), _ptr(dG1), _ptr(dG2)))

    def rhs_noalloc(self, t: float, G1, G2, dG1, dG2):
        """g1g2_rhs_noalloc: device tensors only; stream-ordered, no synchronization."""
        self._check(self.lib.g1g2_rhs_noalloc(self.ctx, float(t), _ptr(G1), _ptr(G2), _ptr(dG1), _ptr(dG2)))

    def step(self, dt: float, nsteps: int):
        self._check(self.lib.g1g2_step_rk4(self.ctx, float(dt), int(nsteps)))

    def observables(self) -> dict:
        o = Obs()
        self._check(self.lib.g1g2_observables(self.ctx, ctypes.byref(o)))
        return dict(t=o.t, N=(o.N[0], o.N[1]), E_kin=o.E_kin, E_mf=o.E_mf, E_corr=o.E_corr,
                    E_tot=o.E_tot, docc=o.docc, herm_resid=o.herm_resid, exch_resid=o.exch_resid,
                    imbalance=o.imbalance, diverged=o.diverged, step=o.step,
                    diverged_step=o.diverged_step)

    def site_observables(self):
        nu, nd, dc = (np.zeros(self.nb) for _ in range(3))
        self._check(self.lib.g1g2_site_observables(self.ctx, _ptr(nu), _ptr(nd), _ptr(dc)))
        return nu, nd, dc

    def get_state(self, G1=None, G2=None, with_g2: bool = True):
        """Copy the state out; host numpy arrays are allocated when not given
        (with_g2=False copies G1 and t only)."""
        s1, s2 = self.shapes()
        if G1 is None:
            G1 = np.zeros(s1, np.complex128)
        if G2 is None and with_g2 and not (self.flags & PTR_DEVICE):
            G2 = np.zeros(s2, np.complex128)
        t = c_double()
        self._check(self.lib.g1g2_get_state(self.ctx, _ptr(G1), _ptr(G2), ctypes.byref(t)))
        return G1, G2, t.value

    def set_state(self, G1, G2=None, t: float = 0.0):
        G1, G2 = _c128(G1), _c128(G2)
        self._check(self.lib.g1g2_set_state(self.ctx, _ptr(G1), _ptr(G2), float(t)))

    def set_h0(self, h0):
        h0 = _c128(h0)
        self._check(self.lib.g1g2_set_h0(self.ctx, _ptr(h0)))

    def set_U(self, U: float):
        self._check(self.lib.g1g2_set_U(self.ctx, float(U)))

    def set_drive(self, x, c, t_center, tau: float):
        x = np.ascontiguousarray(x, np.float64)
        c = np.ascontiguousarray(c, np.float64)
        tc = np.ascontiguousarray(t_center, np.float64)
        self._check(self.lib.g1g2_set_drive(self.ctx, _ptr(x), int(len(c)), _ptr(c), _ptr(tc),
                                             float(tau)))

    def set_switch(self, t_on: float, tau: float):
        """Adiabatic switching U(t) = U phi(t) or w(t) = w phi(t), a sin^2 ramp from t_on over tau (0: off)."""
        self._check(self.lib.g1g2_set_switch(self.ctx, float(t_on), float(tau)))

    def forward_checkpointed(self, dt: float, nsteps: int, interval: int = 0):
        self._check(self.lib.g1g2_forward_checkpointed(self.ctx, float(dt), int(nsteps), int(interval)))

    def adjoint(self, a, b, n_drive: int = 0):
        """(loss, dL/dc [n_drive], dL/dU) after forward_checkpointed."""
        a = np.ascontiguousarray(a, np.float64)
        b = np.ascontiguousarray(b, np.float64)
        gc = np.zeros(max(n_drive, 1))
        gU, L = c_double(), c_double()
        self._check(self.lib.g1g2_adjoint(self.ctx, _ptr(a), _ptr(b), _ptr(gc), ctypes.byref(gU),
                                          ctypes.byref(L)))
        return L.value, gc[:n_drive], gU.value

    def profile(self, dt: float = 0.0, nsteps: int = 0) -> dict:
        """Per-kernel time of nsteps RK4 steps (or of one RHS for nsteps = 0):
        {name: (total_ms, launches)}."""
        ms = np.zeros(64)
        cnt = np.zeros(64, np.int32)
        n = c_int32()
        self._check(self.lib.g1g2_profile(self.ctx, float(dt), int(nsteps), 64, _ptr(ms), _ptr(cnt),
                                          ctypes.byref(n)))
        return {self.lib.g1g2_profile_name(self.ctx, k).decode(): (float(ms[k]), int(cnt[k]))
                for k in range(n.value)}

    def profile_adjoint(self, a, b) -> dict:
        """Per-kernel time of one reverse sweep (after forward_checkpointed):
        {name: (total_ms, launches)}."""
        a = np.ascontiguousarray(a, np.float64)
        b = np.ascontiguousarray(b, np.float64)
        ms = np.zeros(64)
        cnt = np.zeros(64, np.int32)
        n = c_int32()
        self._check(self.lib.g1g2_profile_adjoint(self.ctx, _ptr(a), _ptr(b), 64, _ptr(ms), _ptr(cnt),
                                                  ctypes.byref(n)))
        return {self.lib.g1g2_profile_name(self.ctx, k).decode(): (float(ms[k]), int(cnt[k]))
                for k in range(n.value)}

    def step_path(self) -> str:
        """The kernels the library takes for g1g2_step_rk4 on this context."""
        v = c_int32()
        self._check(self.lib.g1g2_step_path(self.ctx, ctypes.byref(v)))
        return PATHS[v.value]

    def prepare_graph(self, dt: float):
        """Capture the replayed steps of size dt now (no-op without a stream)."""
        self._check(self.lib.g1g2_prepare_graph(self.ctx, float(dt)))

    def close(self):
        if getattr(self, "ctx", None):
            self.lib.g1g2_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch(Propagator):
    """A ragged batch of Hubbard clusters in one context (g1g2_batch_init)."""

    def __init__(self, selfenergy: int, ns, U, h0s, g1s, chunk=None, stream: int = 0,
                 precision: int = FP64, flags: int = 0):
        self.lib = load()
        self.basis, self.flags = HUBBARD, flags
        self.ns = [int(x) for x in ns]
        n = len(self.ns)
        self.nb = max(self.ns)
        self.desc = Desc(HUBBARD, selfenergy, precision, flags, self.nb, 0.0)
        h = [np.ascontiguousarray(a, np.complex128) for a in h0s]
        g = [np.ascontiguousarray(a, np.complex128) for a in g1s]
        ns_a = np.asarray(self.ns, np.int32)
        U_a = np.ascontiguousarray(U, np.float64)
        hp = (c_void_p * n)(*[a.ctypes.data for a in h])
        gp = (c_void_p * n)(*[a.ctypes.data for a in g])
        ch = None if chunk is None else np.ascontiguousarray(chunk, np.int32)
        ctx = c_void_p()
        st = self.lib.g1g2_batch_init(ctypes.byref(ctx), ctypes.byref(self.desc), n, _ptr(ns_a),
                                      _ptr(U_a), hp, gp, _ptr(ch), c_void_p(stream) if stream else None)
        if st != OK:
            raise G1G2Error(st, self.lib.g1g2_strerror(st).decode())
        self.ctx = ctx

    def observables(self):
        obs = (Obs * len(self.ns))()
        self._check(self.lib.g1g2_batch_observables(self.ctx, obs))
        return [dict(t=o.t, N=(o.N[0], o.N[1]), E_kin=o.E_kin, E_mf=o.E_mf, E_corr=o.E_corr,
                     E_tot=o.E_tot, docc=o.docc, imbalance=o.imbalance, diverged=o.diverged,
                     step=o.step, diverged_step=o.diverged_step) for o in obs]

    def get_cluster(self, c: int, with_g2: bool = True):
        ns = self.ns[c]
        g1 = np.zeros((2, ns, ns), np.complex128)
        shape = ((3,) if self.desc.selfenergy in (GW, DSL) else ()) + (ns,) * 4
        g2 = np.zeros(shape, np.complex128) if with_g2 else None
        self._check(self.lib.g1g2_batch_get_state(self.ctx, int(c), _ptr(g1), _ptr(g2)))
        return g1, g2


class Jellium(Propagator):
    """A jellium context (g1g2_jellium_init): momenta on the periodic grid
    ``dims``, energies eps [2][nb], interaction v [nb] (v[0] = 0), G1_0 the
    diagonal G^< [2][nb]; G2_0 [3][nb]^3 or None."""

    def __init__(self, selfenergy: int, dims, eps, v, G1_0, G2_0=None, precision: int = FP64,
                 flags: int = 0, stream: int = 0):
        self.lib = load()
        d3 = (list(dims) + [1, 1])[:3]
        self.dims = tuple(int(x) for x in d3)
        self.basis = JELLIUM
        self.nb = self.dims[0] * self.dims[1] * self.dims[2]
        self.flags = flags
        self.desc = Desc(JELLIUM, selfenergy, precision, flags, self.nb, 0.0)
        dm = np.asarray(self.dims, np.int32)
        ep = np.ascontiguousarray(eps, np.float64)
        vv = np.ascontiguousarray(v, np.float64)
        g1, g2 = _c128(G1_0), _c128(G2_0)
        ctx = c_void_p()
        st = self.lib.g1g2_jellium_init(ctypes.byref(ctx), ctypes.byref(self.desc), _ptr(dm), _ptr(ep), _ptr(vv),
                                        _ptr(g1), _ptr(g2), c_void_p(stream) if stream else None)
        if st != OK:
            raise G1G2Error(st, self.lib.g1g2_strerror(st).decode())
        self.ctx = ctx
