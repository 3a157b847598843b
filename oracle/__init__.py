"""Plain FP64 CPU oracle of the relativistic SHASTA time step.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  The product path
(``paper_1206_0919_amd``) never imports it and shares no code with it.

The arithmetic lives in ``shasta_oracle.c`` (plain C, built with gcc
``-O2 -fno-fast-math -ffp-contract=off -fopenmp``); this module only marshals
numpy arrays through ctypes.  Each wrapper names the passage of
"Relativistic Hydrodynamics on Graphic Cards" (arXiv:1206.0919) that the C
function follows.

Every function of the oracle is pinned by ``tests/test_oracle_*.py`` to
something other than itself (closed forms, exact identities, invariants, the
exact Riemann solution); none is "parity unpinned".
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "shasta_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

CFLAGS = ["-O2", "-fno-fast-math", "-ffp-contract=off", "-fopenmp", "-fPIC",
          "-shared", "-std=c99", "-Wall"]

EOS_IDEAL = 0
EOS_BAG = 1
EOS_TABLE = 2
EOS_BARYON = 3


def build(src: str = _SRC, out: str = _LIB, extra=()) -> str:
    """Compile the oracle with gcc (always recompiles)."""
    cmd = ["gcc", *CFLAGS, *extra, src, "-o", out, "-lm"]
    subprocess.run(cmd, check=True)
    return out


class _Eos(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int), ("B", ctypes.c_double),
                ("e_H", ctypes.c_double), ("n", ctypes.c_int),
                ("te", ctypes.POINTER(ctypes.c_double)),
                ("tp", ctypes.POINTER(ctypes.c_double)),
                ("cs2", ctypes.c_double), ("mass", ctypes.c_double)]


_dp = ctypes.POINTER(ctypes.c_double)
_lib_cache = {}


def load(path: str = _LIB):
    """Load (building first if absent) the oracle shared library."""
    if path in _lib_cache:
        return _lib_cache[path]
    if not os.path.exists(path):
        if path == _LIB:
            build()
        else:
            raise FileNotFoundError(path)
    lib = ctypes.CDLL(path)
    lib.orc_pressure.restype = ctypes.c_double
    lib.orc_pressure.argtypes = [ctypes.POINTER(_Eos), ctypes.c_double, ctypes.c_double]
    lib.orc_recover.restype = ctypes.c_int
    lib.orc_recover.argtypes = [ctypes.POINTER(_Eos)] + [ctypes.c_double] * 5 + \
        [_dp] * 6 + [ctypes.POINTER(ctypes.c_int)] * 3
    lib.orc_prim_to_cons.restype = None
    lib.orc_prim_to_cons.argtypes = [ctypes.POINTER(_Eos), ctypes.c_int64] + [_dp] * 10
    lib.orc_cons_to_prim.restype = None
    lib.orc_cons_to_prim.argtypes = [ctypes.POINTER(_Eos), ctypes.c_int64] + [_dp] * 11
    lib.orc_fct_1d.restype = None
    lib.orc_fct_1d.argtypes = [ctypes.c_int, _dp, _dp, _dp, ctypes.c_int,
                               ctypes.c_double, ctypes.c_double, _dp, _dp]
    lib.orc_sweep.restype = None
    lib.orc_sweep.argtypes = [ctypes.POINTER(_Eos), ctypes.c_int, ctypes.c_int,
                              ctypes.c_int, ctypes.c_int, ctypes.c_double,
                              ctypes.c_double, ctypes.POINTER(_dp), _dp, _dp,
                              ctypes.POINTER(ctypes.c_int64), ctypes.c_int]
    lib.orc_run.restype = None
    lib.orc_run.argtypes = [ctypes.POINTER(_Eos), ctypes.c_int, ctypes.c_int,
                            ctypes.c_int, ctypes.c_double, ctypes.c_double,
                            ctypes.c_int64, ctypes.c_int, ctypes.POINTER(_dp),
                            _dp, _dp, ctypes.POINTER(ctypes.c_int64), ctypes.c_int]
    lib.orc_axis_of.restype = ctypes.c_int
    lib.orc_axis_of.argtypes = [ctypes.c_int64, ctypes.c_int]
    lib.orc_sum.restype = ctypes.c_double
    lib.orc_sum.argtypes = [ctypes.c_int64, _dp]
    lib.orc_max_threads.restype = ctypes.c_int
    lib.orc_max_threads.argtypes = []
    _lib_cache[path] = lib
    return lib


def _ptr(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(_dp)


def make_eos(kind: int = EOS_IDEAL, B: float = 0.0, e_H: float = 0.0, table=None,
             cs2: float = 1.0 / 3.0, mass: float = 0.0):
    """EOS descriptor; for EOS_TABLE, table = (node energy densities, node
    pressures); for EOS_BARYON, p = cs2 (e - mass n).  Returns (descriptor,
    arrays it points into)."""
    if kind == EOS_TABLE:
        te = np.ascontiguousarray(table[0], dtype=np.float64)
        tp = np.ascontiguousarray(table[1], dtype=np.float64)
        assert te.size == tp.size >= 2
        return _Eos(int(kind), 0.0, 0.0, te.size, _ptr(te), _ptr(tp), 0.0, 0.0), (te, tp)
    return _Eos(int(kind), float(B), float(e_H), 0, None, None, float(cs2), float(mass)), ()


class Oracle:
    """Thin ctypes front end; state lives in numpy arrays owned by the caller."""

    def __init__(self, eos_kind=EOS_IDEAL, B=0.0, e_H=0.0, lib_path=_LIB, table=None,
                 cs2=1.0 / 3.0, mass=0.0):
        self.lib_path = lib_path
        self.lib = load(lib_path)
        self.eos, self._keep = make_eos(eos_kind, B, e_H, table, cs2, mass)

    # eq. (cf-*) and the EOS closure
    def pressure(self, e: float, n: float = 0.0) -> float:
        return self.lib.orc_pressure(ctypes.byref(self.eos), float(e), float(n))

    # Sec. 3 last paragraph: fixed-point eigenframe recovery of one cell
    def recover(self, E, Mx, My, Mz, R=0.0):
        out = [ctypes.c_double() for _ in range(6)]
        it, cl, fl = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
        ok = self.lib.orc_recover(ctypes.byref(self.eos), float(E), float(Mx),
                                  float(My), float(Mz), float(R),
                                  *[ctypes.byref(o) for o in out],
                                  ctypes.byref(it), ctypes.byref(cl), ctypes.byref(fl))
        e, p, v, vx, vy, vz = (o.value for o in out)
        return dict(e=e, p=p, v=v, vx=vx, vy=vy, vz=vz, iters=it.value,
                    clamped=cl.value, floored=fl.value, converged=bool(ok))

    def prim_to_cons(self, e, vx, vy, vz, n):
        e, vx, vy, vz, n = (np.ascontiguousarray(a, dtype=np.float64).ravel()
                            for a in (e, vx, vy, vz, n))
        out = [np.empty_like(e) for _ in range(5)]
        self.lib.orc_prim_to_cons(ctypes.byref(self.eos), e.size,
                                  *[_ptr(a) for a in (e, vx, vy, vz, n)],
                                  *[_ptr(a) for a in out])
        return out

    def cons_to_prim(self, E, Mx, My, Mz, R):
        E, Mx, My, Mz, R = (np.ascontiguousarray(a, dtype=np.float64).ravel()
                            for a in (E, Mx, My, Mz, R))
        out = [np.empty_like(E) for _ in range(6)]
        self.lib.orc_cons_to_prim(ctypes.byref(self.eos), E.size,
                                  *[_ptr(a) for a in (E, Mx, My, Mz, R)],
                                  *[_ptr(a) for a in out])
        return dict(zip(("e", "p", "vx", "vy", "vz", "n"), out))

    # Sec. 3 eqs. shasta-diff .. shasta-n on one pencil with its halo
    def fct_1d(self, U, eps, f=None, lam=0.0, diff=1.0):
        U = np.ascontiguousarray(U, dtype=np.float64)
        eps = np.ascontiguousarray(eps, dtype=np.float64)
        N = U.size - 6
        has_src = f is not None
        f = np.zeros_like(U) if f is None else np.ascontiguousarray(f, dtype=np.float64)
        out = np.empty(N)
        flux = np.zeros(2)
        self.lib.orc_fct_1d(N, _ptr(U), _ptr(eps), _ptr(f), int(has_src),
                            float(lam), float(diff), _ptr(out), _ptr(flux))
        return out, flux

    @staticmethod
    def _fields(U):
        assert len(U) == 5
        shape = U[0].shape
        for a in U:
            assert a.shape == shape and a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
        nz, ny, nx = shape
        arr = (_dp * 5)(*[_ptr(a) for a in U])
        return nx, ny, nz, arr

    # One directional sweep (Sec. 3 half-step predictor + corrector)
    def sweep(self, U, axis, lam, diff=1.0, nthreads=0):
        nx, ny, nz, arr = self._fields(U)
        ledger = np.zeros(5)
        maxeps = np.zeros(1)
        cnt = (ctypes.c_int64 * 4)()
        self.lib.orc_sweep(ctypes.byref(self.eos), nx, ny, nz, int(axis),
                           float(lam), float(diff), arr, _ptr(ledger),
                           _ptr(maxeps), cnt, int(nthreads))
        return ledger, float(maxeps[0]), list(cnt)

    # nsteps time steps with the Listing 2 axis cycle; U updated in place
    def run(self, U, lam, nsteps, k0=0, diff=1.0, nthreads=0, ledger=None):
        nx, ny, nz, arr = self._fields(U)
        ledger = np.zeros(5) if ledger is None else ledger
        maxeps = np.zeros(1)
        cnt = (ctypes.c_int64 * 4)()
        self.lib.orc_run(ctypes.byref(self.eos), nx, ny, nz, float(lam),
                         float(diff), int(k0), int(nsteps), arr, _ptr(ledger),
                         _ptr(maxeps), cnt, int(nthreads))
        return ledger, float(maxeps[0]), list(cnt)

    def axis_of(self, step, sweep):
        return self.lib.orc_axis_of(int(step), int(sweep))

    def total(self, a):
        a = np.ascontiguousarray(a, dtype=np.float64).ravel()
        return self.lib.orc_sum(a.size, _ptr(a))

    def max_threads(self):
        return self.lib.orc_max_threads()
