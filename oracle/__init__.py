"""Plain FP64 CPU oracle for the limited-1PN N-body equations (ctypes wrapper).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, ``__graft_entry__.smoke()``
and the CPU-baseline leg of ``bench.py``; never by the product package.  The C
source (``pnref.c``) shares no code with the HIP library.

All arrays are numpy float64, C-contiguous.  ``pos``/``vel`` are ``[N, 3]``,
``mass`` is ``[N]``; body 0 is the massive object (the paper's body #1).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libpnref.so")
_SRC = os.path.join(_HERE, "pnref.c")

_dp = ctypes.POINTER(ctypes.c_double)
_i64 = ctypes.c_int64
_i64p = ctypes.POINTER(ctypes.c_int64)


def build(force: bool = True) -> str:
    """Compile ``pnref.c`` into ``libpnref.so`` with gcc (-O2, no FMA contraction)."""
    if force or not os.path.exists(_LIB_PATH):
        cmd = ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC",
               "-shared", "-std=c11", "-Wall", "-o", _LIB_PATH + ".tmp", _SRC, "-lm"]
        subprocess.check_call(cmd)
        os.replace(_LIB_PATH + ".tmp", _LIB_PATH)
    return _LIB_PATH


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        lib = ctypes.CDLL(_LIB_PATH)
        sig = {
            "pnref_newton": [_dp, _dp, _i64, ctypes.c_double, ctypes.c_double, _dp, _dp],
            "pnref_correction": [_dp, _dp, _dp, _i64, ctypes.c_double, ctypes.c_double,
                                 ctypes.c_double, _dp, _dp, _dp],
            "pnref_accel": [_dp, _dp, _dp, _i64, ctypes.c_double, ctypes.c_double,
                            ctypes.c_double, _dp, _dp, _dp],
            "pnref_accel_rows": [_dp, _dp, _dp, _i64, ctypes.c_double, ctypes.c_double,
                                 ctypes.c_double, _i64p, _i64, _dp, _dp, _dp],
            "pnref_literal": [_dp, _dp, _dp, _i64, ctypes.c_double, ctypes.c_double,
                              ctypes.c_double, _dp],
            "pnref_eih": [_dp, _dp, _dp, _i64, ctypes.c_double, ctypes.c_double,
                          ctypes.c_double, _dp, _dp],
            "pnref_eih2": [_dp, _dp, _dp, _i64, ctypes.c_double, ctypes.c_double,
                           ctypes.c_double, _dp, _dp, _dp],
            "pnref_eih2_rows": [_dp, _dp, _dp, _i64, ctypes.c_double, ctypes.c_double,
                                ctypes.c_double, _i64p, _i64, _dp, _dp, _dp],
            "pnref_twobody": [_dp, _dp, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                              ctypes.c_double, _dp, _dp],
            "pnref_step": [_dp, _dp, _dp, _i64, ctypes.c_double, ctypes.c_double,
                           ctypes.c_double, ctypes.c_double, _i64],
            "pnref_diagnostics": [_dp, _dp, _dp, _i64, ctypes.c_double, ctypes.c_double,
                                  ctypes.c_double, _dp],
            "pnref_jerk": [_dp, _dp, _dp, _i64, ctypes.c_double, ctypes.c_double,
                           ctypes.c_double, ctypes.c_double, _dp, _dp],
            "pnref_hermite": [_dp, _dp, _dp, _i64, ctypes.c_double, ctypes.c_double,
                              ctypes.c_double, ctypes.c_double, _i64, ctypes.c_double],
            "pnref_jerk_rows": [_dp, _dp, _dp, _i64, ctypes.c_double, ctypes.c_double,
                                ctypes.c_double, _i64p, _i64, _dp, _dp],
            "pnref_jerk_exact": [_dp, _dp, _dp, _i64, ctypes.c_double, ctypes.c_double,
                                 ctypes.c_double, _dp, _dp],
        }
        for name, argtypes in sig.items():
            fn = getattr(lib, name)
            fn.argtypes = argtypes
            fn.restype = ctypes.c_int
        _lib = lib
    return _lib


def _arr(a, shape=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if shape is not None and a.shape != shape:
        raise ValueError(f"expected shape {shape}, got {a.shape}")
    return a


def _p(a):
    return a.ctypes.data_as(_dp)


def _check(rc, name):
    if rc != 0:
        raise ValueError(f"{name} returned {rc}")


def newton(pos, mass, G, eps):
    """Newtonian acceleration [N,3] and potential [N] (Eqs. (1), (4), (10))."""
    N = len(mass)
    pos, mass = _arr(pos, (N, 3)), _arr(mass, (N,))
    acc, phi = np.empty((N, 3)), np.empty(N)
    _check(_load().pnref_newton(_p(pos), _p(mass), N, G, eps, _p(acc), _p(phi)), "pnref_newton")
    return acc, phi


def correction(pos, vel, mass, G, c, eps, phi, acc_newton):
    """lambda * limited-1PN part for all bodies, from Newtonian phi and acceleration."""
    N = len(mass)
    pos, vel, mass = _arr(pos, (N, 3)), _arr(vel, (N, 3)), _arr(mass, (N,))
    phi, acc_newton = _arr(phi, (N,)), _arr(acc_newton, (N, 3))
    out = np.empty((N, 3))
    _check(_load().pnref_correction(_p(pos), _p(vel), _p(mass), N, G, c, eps, _p(phi),
                                    _p(acc_newton), _p(out)), "pnref_correction")
    return out


def accel(pos, vel, mass, G, c, eps):
    """(acc_newton [N,3], phi [N], acc_1pn [N,3]) for all bodies."""
    N = len(mass)
    pos, vel, mass = _arr(pos, (N, 3)), _arr(vel, (N, 3)), _arr(mass, (N,))
    aN, phi, a1 = np.empty((N, 3)), np.empty(N), np.empty((N, 3))
    _check(_load().pnref_accel(_p(pos), _p(vel), _p(mass), N, G, c, eps, _p(aN), _p(phi),
                               _p(a1)), "pnref_accel")
    return aN, phi, a1


def accel_rows(pos, vel, mass, G, c, eps, rows):
    """Same as :func:`accel` for the given body indices only."""
    N = len(mass)
    pos, vel, mass = _arr(pos, (N, 3)), _arr(vel, (N, 3)), _arr(mass, (N,))
    rows = np.ascontiguousarray(rows, dtype=np.int64)
    R = len(rows)
    aN, phi, a1 = np.empty((R, 3)), np.empty(R), np.empty((R, 3))
    _check(_load().pnref_accel_rows(_p(pos), _p(vel), _p(mass), N, G, c, eps,
                                    rows.ctypes.data_as(_i64p), R, _p(aN), _p(phi), _p(a1)),
           "pnref_accel_rows")
    return aN, phi, a1


def literal(pos, vel, mass, G, c, eps):
    """Total acceleration from Eqs. (1)-(6) transcribed term by term."""
    N = len(mass)
    pos, vel, mass = _arr(pos, (N, 3)), _arr(vel, (N, 3)), _arr(mass, (N,))
    acc = np.empty((N, 3))
    _check(_load().pnref_literal(_p(pos), _p(vel), _p(mass), N, G, c, eps, _p(acc)),
           "pnref_literal")
    return acc


def eih(pos, vel, mass, G, c, eps):
    """Unrestricted EIH: (acc_newton, lambda * 1PN part), brute force O(N^3)."""
    N = len(mass)
    pos, vel, mass = _arr(pos, (N, 3)), _arr(vel, (N, 3)), _arr(mass, (N,))
    aN, a1 = np.empty((N, 3)), np.empty((N, 3))
    _check(_load().pnref_eih(_p(pos), _p(vel), _p(mass), N, G, c, eps, _p(aN), _p(a1)),
           "pnref_eih")
    return aN, a1


def eih2(pos, vel, mass, G, c, eps):
    """Unrestricted EIH, potentials summed once: (acc_newton, phi, lambda * 1PN part)."""
    N = len(mass)
    pos, vel, mass = _arr(pos, (N, 3)), _arr(vel, (N, 3)), _arr(mass, (N,))
    aN, phi, a1 = np.empty((N, 3)), np.empty(N), np.empty((N, 3))
    _check(_load().pnref_eih2(_p(pos), _p(vel), _p(mass), N, G, c, eps, _p(aN), _p(phi), _p(a1)),
           "pnref_eih2")
    return aN, phi, a1


def eih2_rows(pos, vel, mass, G, c, eps, rows):
    """Same as :func:`eih2` for the given body indices only (one O(N^2)
    Newtonian pass, then O(N) per row)."""
    N = len(mass)
    pos, vel, mass = _arr(pos, (N, 3)), _arr(vel, (N, 3)), _arr(mass, (N,))
    rows = np.ascontiguousarray(rows, dtype=np.int64)
    R = len(rows)
    aN, phi, a1 = np.empty((R, 3)), np.empty(R), np.empty((R, 3))
    _check(_load().pnref_eih2_rows(_p(pos), _p(vel), _p(mass), N, G, c, eps,
                                   rows.ctypes.data_as(_i64p), R, _p(aN), _p(phi), _p(a1)),
           "pnref_eih2_rows")
    return aN, phi, a1


def twobody(x, v, m1, m2, G, c):
    """Two-body 1PN relative acceleration: (Newtonian, lambda * 1PN)."""
    x, v = _arr(x, (3,)), _arr(v, (3,))
    aN, a1 = np.empty(3), np.empty(3)
    _check(_load().pnref_twobody(_p(x), _p(v), m1, m2, G, c, _p(aN), _p(a1)), "pnref_twobody")
    return aN, a1


def step(pos, vel, mass, G, c, eps, dt, nsteps):
    """Advance copies of (pos, vel) by nsteps classical RK4 steps; returns them."""
    N = len(mass)
    pos, vel, mass = _arr(pos, (N, 3)).copy(), _arr(vel, (N, 3)).copy(), _arr(mass, (N,))
    _check(_load().pnref_step(_p(pos), _p(vel), _p(mass), N, G, c, eps, dt, nsteps),
           "pnref_step")
    return pos, vel


def jerk(pos, vel, mass, G, c, eps, h=1e-4):
    """(acceleration, jerk along the motion) by Richardson central differences."""
    N = len(mass)
    pos, vel, mass = _arr(pos, (N, 3)), _arr(vel, (N, 3)), _arr(mass, (N,))
    a, j = np.empty((N, 3)), np.empty((N, 3))
    _check(_load().pnref_jerk(_p(pos), _p(vel), _p(mass), N, G, c, eps, h, _p(a), _p(j)),
           "pnref_jerk")
    return a, j


def jerk_exact(pos, vel, mass, G, c, eps, rows=None):
    """(acceleration, jerk along the motion) by complex-step differentiation:
    exact to rounding.  ``rows``: body indices (default all); star rows cost
    O(N) each after one O(N^2) evaluation, the massive object's row O(N^2)."""
    N = len(mass)
    pos, vel, mass = _arr(pos, (N, 3)), _arr(vel, (N, 3)), _arr(mass, (N,))
    if rows is None:
        a, j = np.empty((N, 3)), np.empty((N, 3))
        _check(_load().pnref_jerk_exact(_p(pos), _p(vel), _p(mass), N, G, c, eps, _p(a), _p(j)),
               "pnref_jerk_exact")
        return a, j
    rows = np.ascontiguousarray(rows, dtype=np.int64)
    R = len(rows)
    a, j = np.empty((R, 3)), np.empty((R, 3))
    _check(_load().pnref_jerk_rows(_p(pos), _p(vel), _p(mass), N, G, c, eps,
                                   rows.ctypes.data_as(_i64p), R, _p(a), _p(j)),
           "pnref_jerk_rows")
    return a, j


def hermite(pos, vel, mass, G, c, eps, dt, nsteps, h=0.0):
    """Advance copies of (pos, vel) by nsteps fixed Hermite steps; returns them.
    Jerks are exact (complex step) for h = 0, else Richardson quotients of step h."""
    N = len(mass)
    pos, vel, mass = _arr(pos, (N, 3)).copy(), _arr(vel, (N, 3)).copy(), _arr(mass, (N,))
    _check(_load().pnref_hermite(_p(pos), _p(vel), _p(mass), N, G, c, eps, dt, nsteps, h),
           "pnref_hermite")
    return pos, vel


def diagnostics(pos, vel, mass, G, c, eps):
    """Eqs. (7)-(8): array [E_N, lambda*E_1PN, P_N(3), lambda*P_1PN(3)]."""
    N = len(mass)
    pos, vel, mass = _arr(pos, (N, 3)), _arr(vel, (N, 3)), _arr(mass, (N,))
    out = np.empty(8)
    _check(_load().pnref_diagnostics(_p(pos), _p(vel), _p(mass), N, G, c, eps, _p(out)),
           "pnref_diagnostics")
    return out


def set_threads(n: int | None) -> None:
    """Set the OpenMP thread count used by later oracle calls (None = runtime default)."""
    lib = ctypes.CDLL("libgomp.so.1")
    if n is not None:
        lib.omp_set_num_threads(int(n))


def max_threads() -> int:
    lib = ctypes.CDLL("libgomp.so.1")
    lib.omp_get_max_threads.restype = ctypes.c_int
    return int(lib.omp_get_max_threads())
