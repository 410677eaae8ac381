"""ctypes binding of libpn (include/pn.h): argument marshalling only.

Every function takes torch tensors on the GPU (float64, contiguous) and
passes their device pointers to the C ABI; all arithmetic runs in the HIP
kernels.  The library must have been built (``python -m
paper_1801_07986_amd.build``); there is no fallback.
"""
from __future__ import annotations

import ctypes
import math
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpn.so")

PN_OK, PN_EINVAL, PN_ENONFINITE, PN_EDEVICE, PN_ENOMEM = 0, -1, -2, -3, -4
PN_FP64, PN_MIXED = 0, 1
PN_ASYNC, PN_NOGRAPH, PN_TIMING = 1, 2, 4

EXPORTS = ("pn_potential_accel", "pn_correction", "pn_accel", "pn_step", "pn_diagnostics",
           "pn_step_batched", "pn_strerror", "pn_last_timing", "pn_release", "pn_set_shape",
           "pn_accel_eih", "pn_encounters", "pn_jerk", "pn_step_hermite", "pn_query_shape", "pn_accel_noalloc", "pn_set_batch_shape",
           "pn_query_batch_shape", "pn_set_stage_kernel", "pn_query_stage_kernel")
TUNED_PATH = os.path.join(HERE, "tuned_shapes.json")


class PNError(RuntimeError):
    def __init__(self, code: int, name: str, text: str):
        super().__init__(f"{name} failed with code {code}: {text}")
        self.code = code


_lib = None


def load():
    """Load libpn.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              f"`python -m paper_1801_07986_amd.build`")
        lib = ctypes.CDLL(LIB_PATH)
        vp, d, i64, i32 = ctypes.c_void_p, ctypes.c_double, ctypes.c_int64, ctypes.c_int
        lib.pn_potential_accel.argtypes = [vp, vp, vp, i64, d, d, d, vp, vp, vp, i32]
        lib.pn_correction.argtypes = [vp, vp, vp, i64, d, d, d, vp, vp, vp, vp, i32]
        lib.pn_accel.argtypes = [vp, vp, vp, i64, d, d, d, i32, vp, vp, vp, vp, i32]
        lib.pn_accel_noalloc.argtypes = [vp, vp, vp, i64, d, d, d, i32, vp, vp, vp, vp, i32]
        lib.pn_accel_eih.argtypes = [vp, vp, vp, i64, d, d, d, i32, vp, vp, vp, vp, i32]
        lib.pn_encounters.argtypes = [vp, vp, vp, i64, d, d, d, vp, vp, i32]
        lib.pn_step.argtypes = [vp, vp, vp, i64, d, d, d, d, i64, i32, vp, i32]
        lib.pn_jerk.argtypes = [vp, vp, vp, i64, d, d, d, vp, vp, vp, i32]
        lib.pn_step_hermite.argtypes = [vp, vp, vp, i64, d, d, d, d, i64, vp, i32]
        lib.pn_diagnostics.argtypes = [vp, vp, vp, i64, d, d, d, vp, vp, i32]
        lib.pn_step_batched.argtypes = [ctypes.c_int32, vp, vp, vp, vp, vp, vp, vp, d, i64, i32,
                                        vp, i32]
        lib.pn_strerror.argtypes = [i32]
        lib.pn_strerror.restype = ctypes.c_char_p
        lib.pn_last_timing.argtypes = [vp]
        lib.pn_release.argtypes = []
        lib.pn_set_shape.argtypes = [i32, i64, i64, i32, i32, i32]
        lib.pn_query_shape.argtypes = [i32, i64, vp]
        lib.pn_set_batch_shape.argtypes = [i32, i32, i32]
        lib.pn_query_batch_shape.argtypes = [i32, ctypes.c_int32, vp, vp]
        lib.pn_set_stage_kernel.argtypes = [i32, i64, i64, i32]
        lib.pn_query_stage_kernel.argtypes = [i32, i64]
        for name in EXPORTS:
            if name != "pn_strerror":
                getattr(lib, name).restype = i32
        _lib = lib
        install_tuned_shapes()
    return _lib


def install_tuned_shapes(path: str | None = None) -> int:
    """Install the autotuner's shape table (tuned_shapes.json) into the library."""
    import json

    path = path or TUNED_PATH
    if not os.path.exists(path):
        return 0
    with open(path) as f:
        table = json.load(f)
    _lib.pn_set_shape(-1, 0, 0, 0, 0, 0)
    _lib.pn_set_batch_shape(-1, 0, 0)
    _lib.pn_set_stage_kernel(-1, 0, 0, 0)
    n = 0
    for e in table.get("entries", []):
        prec = PN_MIXED if e["precision"] == "mixed" else PN_FP64
        _check(_lib.pn_set_shape(prec, int(e["n_min"]), int(e["n_max"]), int(e["ipt"]),
                                 int(e["ws"]), int(e["nsplit"])), "pn_set_shape")
        n += 1
    for e in table.get("batched", []):
        prec = PN_MIXED if e["precision"] == "mixed" else PN_FP64
        _check(_lib.pn_set_batch_shape(prec, int(e["ipt"]), int(e["nsplit"])),
               "pn_set_batch_shape")
        n += 1
    for e in table.get("stage", []):
        prec = PN_MIXED if e["precision"] == "mixed" else PN_FP64
        _check(_lib.pn_set_stage_kernel(prec, int(e["n_min"]), int(e["n_max"]), int(e["ns"])),
               "pn_set_stage_kernel")
        n += 1
    return n


def pn_set_shape(precision, n_min, n_max, ipt, ws, nsplit):
    return _check(load().pn_set_shape(precision, n_min, n_max, ipt, ws, nsplit), "pn_set_shape")


def pn_query_shape(precision, N):
    """(ipt, ws, nsplit, iblocks) of the sweep an N-body evaluation would launch."""
    out = (ctypes.c_int * 4)()
    _check(load().pn_query_shape(precision, int(N), ctypes.cast(out, ctypes.c_void_p)),
           "pn_query_shape")
    return tuple(out)


def pn_set_stage_kernel(precision, n_min, n_max, ns):
    return _check(load().pn_set_stage_kernel(precision, int(n_min), int(n_max), int(ns)),
                  "pn_set_stage_kernel")


def pn_query_stage_kernel(precision, N):
    """Stars per workgroup of pn_step's one-launch stages for an N-body system (0: two kernels)."""
    rc = load().pn_query_stage_kernel(precision, int(N))
    if rc < 0:
        _check(rc, "pn_query_stage_kernel")
    return rc


def pn_set_batch_shape(precision, ipt, nsplit):
    return _check(load().pn_set_batch_shape(precision, ipt, nsplit), "pn_set_batch_shape")


def pn_query_batch_shape(precision, offsets):
    """(ipt, [j-splits of each system]) that pn_step_batched would use."""
    n_sys = len(offsets) - 1
    off = (ctypes.c_int64 * (n_sys + 1))(*[int(o) for o in offsets])
    out = (ctypes.c_int * (n_sys + 1))()
    _check(load().pn_query_batch_shape(precision, n_sys, ctypes.cast(off, ctypes.c_void_p),
                                       ctypes.cast(out, ctypes.c_void_p)), "pn_query_batch_shape")
    return out[0], list(out[1:])


def _check(rc: int, name: str) -> int:
    if rc != PN_OK:
        raise PNError(rc, name, load().pn_strerror(rc).decode())
    return rc


def _ptr(t, numel=None):
    """Device pointer of a contiguous float64 CUDA/HIP tensor on the current
    device.  numel, when given, is the element count the library will access
    (3N for [N][3] arrays, N for [N]): the C ABI sees only pointers, so a
    shorter buffer is rejected here rather than read past its end."""
    if t is None:
        return None
    import torch

    if not isinstance(t, torch.Tensor) or t.dtype != torch.float64 or not t.is_contiguous() \
            or t.device.type != "cuda":
        raise TypeError("expected a contiguous float64 tensor on the GPU")
    if t.device.index is not None and t.device.index != torch.cuda.current_device():
        raise ValueError(f"tensor on {t.device}, but the current device is "
                         f"cuda:{torch.cuda.current_device()}")
    if numel is not None and t.numel() != numel:
        raise ValueError(f"expected {numel} elements, got a tensor of shape {tuple(t.shape)}")
    return ctypes.c_void_p(t.data_ptr())


def _stream(stream):
    if stream is None:
        return None
    return ctypes.c_void_p(int(stream.cuda_stream if hasattr(stream, "cuda_stream") else stream))


def _n(mass) -> int:
    """N from the mass vector (which must be one-dimensional)."""
    if getattr(mass, "dim", lambda: 1)() != 1:
        raise ValueError("mass must be a vector of N elements")
    return int(mass.shape[0])


def pn_potential_accel(pos, vel, mass, G, c, eps, acc_newton, phi, stream=None, flags=0):
    n = _n(mass)
    return _check(load().pn_potential_accel(_ptr(pos, 3 * n), _ptr(vel, 3 * n), _ptr(mass), n, G,
                                            c, eps, _ptr(acc_newton, 3 * n), _ptr(phi, n),
                                            _stream(stream), flags),
                  "pn_potential_accel")


def pn_correction(pos, vel, mass, G, c, eps, phi, acc_newton, acc_1pn, stream=None, flags=0):
    n = _n(mass)
    return _check(load().pn_correction(_ptr(pos, 3 * n), _ptr(vel, 3 * n), _ptr(mass), n, G, c,
                                       eps, _ptr(phi, n), _ptr(acc_newton, 3 * n),
                                       _ptr(acc_1pn, 3 * n), _stream(stream), flags),
                  "pn_correction")


def pn_accel(pos, vel, mass, G, c, eps, precision, acc_newton=None, phi=None, acc_1pn=None,
             stream=None, flags=0):
    n = _n(mass)
    return _check(load().pn_accel(_ptr(pos, 3 * n), _ptr(vel, 3 * n), _ptr(mass), n, G, c, eps,
                                  precision, _ptr(acc_newton, 3 * n), _ptr(phi, n),
                                  _ptr(acc_1pn, 3 * n), _stream(stream), flags), "pn_accel")


def pn_accel_noalloc(pos, vel, mass, G, c, eps, precision, acc_newton=None, phi=None,
                     acc_1pn=None, stream=None, flags=0):
    n = _n(mass)
    return _check(load().pn_accel_noalloc(_ptr(pos, 3 * n), _ptr(vel, 3 * n), _ptr(mass), n, G, c,
                                          eps, precision, _ptr(acc_newton, 3 * n), _ptr(phi, n),
                                          _ptr(acc_1pn, 3 * n), _stream(stream), flags),
                  "pn_accel_noalloc")


def pn_accel_eih(pos, vel, mass, G, c, eps, precision, acc_newton=None, phi=None, acc_1pn=None,
                 stream=None, flags=0):
    n = _n(mass)
    return _check(load().pn_accel_eih(_ptr(pos, 3 * n), _ptr(vel, 3 * n), _ptr(mass), n, G, c,
                                      eps, precision, _ptr(acc_newton, 3 * n), _ptr(phi, n),
                                      _ptr(acc_1pn, 3 * n), _stream(stream), flags),
                  "pn_accel_eih")


def pn_step(pos, vel, mass, G, c, eps, dt, nsteps, precision=PN_FP64, stream=None, flags=0):
    n = _n(mass)
    return _check(load().pn_step(_ptr(pos, 3 * n), _ptr(vel, 3 * n), _ptr(mass), n, G, c, eps, dt,
                                 int(nsteps), precision, _stream(stream), flags), "pn_step")


def pn_jerk(pos, vel, mass, G, c, eps, acc, jerk, stream=None, flags=0):
    n = _n(mass)
    return _check(load().pn_jerk(_ptr(pos, 3 * n), _ptr(vel, 3 * n), _ptr(mass), n, G, c, eps,
                                 _ptr(acc, 3 * n), _ptr(jerk, 3 * n), _stream(stream), flags),
                  "pn_jerk")


def pn_step_hermite(pos, vel, mass, G, c, eps, dt, nsteps, stream=None, flags=0):
    n = _n(mass)
    return _check(load().pn_step_hermite(_ptr(pos, 3 * n), _ptr(vel, 3 * n), _ptr(mass), n, G, c,
                                         eps, dt, int(nsteps), _stream(stream), flags),
                  "pn_step_hermite")


def pn_diagnostics(pos, vel, mass, G, c, eps, stream=None, flags=0):
    out = (ctypes.c_double * 8)()
    n = _n(mass)
    _check(load().pn_diagnostics(_ptr(pos, 3 * n), _ptr(vel, 3 * n), _ptr(mass), n, G, c, eps,
                                 ctypes.cast(out, ctypes.c_void_p), _stream(stream), flags),
           "pn_diagnostics")
    return list(out)


def pn_encounters(pos, vel, mass, G, c, r_close, stream=None, flags=0):
    out = (ctypes.c_double * 8)()
    n = _n(mass)
    _check(load().pn_encounters(_ptr(pos, 3 * n), _ptr(vel, 3 * n), _ptr(mass), n, G, c, r_close,
                                ctypes.cast(out, ctypes.c_void_p), _stream(stream), flags),
           "pn_encounters")
    return {"min_r_bh": out[0], "nearest_to_bh": int(out[1]), "n_close_bh": int(out[2]),
            "min_r_pair": out[3], "pair": (int(out[4]), int(out[5])),
            "max_bh_pair_1pn_ratio": out[6], "most_relativistic": int(out[7])}


def pn_step_batched(offsets, G, c, eps, pos, vel, mass, dt, nsteps, precision=PN_FP64,
                    stream=None, flags=0):
    n_sys = len(offsets) - 1
    off = (ctypes.c_int64 * (n_sys + 1))(*[int(o) for o in offsets])
    g = (ctypes.c_double * n_sys)(*[float(x) for x in G])
    cc = (ctypes.c_double * n_sys)(*[float(x) for x in c])
    ee = (ctypes.c_double * n_sys)(*[float(x) for x in eps])
    cast = lambda a: ctypes.cast(a, ctypes.c_void_p)  # noqa: E731
    n = int(offsets[-1])
    return _check(load().pn_step_batched(n_sys, cast(off), cast(g), cast(cc), cast(ee),
                                         _ptr(pos, 3 * n), _ptr(vel, 3 * n), _ptr(mass, n), dt,
                                         int(nsteps), precision, _stream(stream), flags),
                  "pn_step_batched")


def pn_last_timing():
    out = (ctypes.c_double * 3)()
    _check(load().pn_last_timing(ctypes.cast(out, ctypes.c_void_p)), "pn_last_timing")
    return {"launches": int(out[0]), "total_ms": out[1], "pairs_per_launch": out[2]}


def pn_release():
    return _check(load().pn_release(), "pn_release")


def pn_strerror(code: int) -> str:
    return load().pn_strerror(code).decode()


INF = math.inf
