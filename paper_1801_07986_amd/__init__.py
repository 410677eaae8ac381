"""MI355X-native limited-1PN direct N-body hot path (arXiv:1801.07986).

The compute path is ``libpn.so`` (HIP kernels for gfx950 behind the C ABI of
``include/pn.h``); this package exposes it to Python through ctypes with the
same names (``pn_potential_accel``, ``pn_correction``, ``pn_accel``,
``pn_step``, ``pn_diagnostics``, ``pn_step_batched``, ...).  Importing the
package does not load the library; the first use of a ``pn_*`` name does, and
raises ImportError if it has not been built.

``paper_1801_07986_amd.inputs`` holds the seeded synthetic input generators.
"""
from __future__ import annotations

_BINDING_NAMES = (
    "pn_potential_accel", "pn_correction", "pn_accel", "pn_accel_eih", "pn_step", "pn_diagnostics",
    "pn_step_batched", "pn_encounters", "pn_last_timing", "pn_release", "pn_strerror", "PNError",
    "PN_OK", "PN_EINVAL", "PN_ENONFINITE", "PN_EDEVICE", "PN_ENOMEM", "PN_FP64", "PN_MIXED",
    "PN_ASYNC", "PN_NOGRAPH", "PN_TIMING", "load", "LIB_PATH", "EXPORTS", "pn_set_shape",
    "install_tuned_shapes", "pn_jerk", "pn_step_hermite", "pn_query_shape", "pn_accel_noalloc",
    "pn_set_batch_shape", "pn_query_batch_shape", "pn_set_stage_kernel", "pn_query_stage_kernel",
)


def __getattr__(name):
    if name in _BINDING_NAMES:
        from . import _binding

        if name.startswith("pn_") and name not in ("pn_strerror",):
            _binding.load()
        return getattr(_binding, name)
    raise AttributeError(name)
