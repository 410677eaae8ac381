"""The C ABI library: loads on a machine without a GPU, exports every entry
point include/pn.h declares, and rejects invalid arguments before any device
work (so these run on the CPU)."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pn.h")


def _declared():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\*?\s+\*?(pn_\w+)\(", text, re.M)))


@pytest.fixture(scope="module")
def lib():
    from paper_1801_07986_amd import _binding

    if not os.path.exists(_binding.LIB_PATH):
        from paper_1801_07986_amd import build

        build.build()
    return _binding.load()


def test_header_declares_the_entry_points():
    names = _declared()
    for required in ("pn_potential_accel", "pn_correction", "pn_step", "pn_accel", "pn_accel_eih",
                     "pn_diagnostics", "pn_step_batched", "pn_strerror", "pn_release",
                     "pn_last_timing", "pn_jerk", "pn_step_hermite"):
        assert required in names


def test_library_exports_every_declared_symbol(lib):
    from paper_1801_07986_amd import _binding

    out = subprocess.run(["nm", "-D", "--defined-only", _binding.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = set(re.findall(r" T (pn_\w+)$", out, re.M))
    for name in _declared():
        assert name in exported, name
        assert hasattr(lib, name)


def test_library_holds_gfx950_code(lib):
    from paper_1801_07986_amd import _binding

    blob = open(_binding.LIB_PATH, "rb").read()
    assert b"gfx950" in blob


FAKE = ctypes.c_void_p(4096)  # aligned, never dereferenced: validation fails first
MIS = ctypes.c_void_p(4097)   # misaligned


def test_validation_without_device(lib):
    EINVAL = -1
    d = FAKE
    # N < 2
    assert lib.pn_potential_accel(d, d, d, 1, 1.0, 30.0, 0.0, d, d, None, 0) == EINVAL
    # G <= 0, c <= 0, c NaN, eps < 0, eps inf
    assert lib.pn_potential_accel(d, d, d, 16, 0.0, 30.0, 0.0, d, d, None, 0) == EINVAL
    assert lib.pn_potential_accel(d, d, d, 16, 1.0, -1.0, 0.0, d, d, None, 0) == EINVAL
    assert lib.pn_potential_accel(d, d, d, 16, 1.0, float("nan"), 0.0, d, d, None, 0) == EINVAL
    assert lib.pn_potential_accel(d, d, d, 16, 1.0, 30.0, -1e-3, d, d, None, 0) == EINVAL
    assert lib.pn_potential_accel(d, d, d, 16, 1.0, 30.0, float("inf"), d, d, None, 0) == EINVAL
    # null or misaligned pointers
    assert lib.pn_potential_accel(None, d, d, 16, 1.0, 30.0, 0.0, d, d, None, 0) == EINVAL
    assert lib.pn_potential_accel(MIS, d, d, 16, 1.0, 30.0, 0.0, d, d, None, 0) == EINVAL
    assert lib.pn_correction(d, None, d, 16, 1.0, 30.0, 0.0, d, d, d, None, 0) == EINVAL
    assert lib.pn_correction(d, d, d, 16, 1.0, 30.0, 0.0, None, d, d, None, 0) == EINVAL
    # pn_step: bad dt, negative nsteps, unknown precision
    assert lib.pn_step(d, d, d, 16, 1.0, 30.0, 0.0, float("nan"), 1, 0, None, 0) == EINVAL
    assert lib.pn_step(d, d, d, 16, 1.0, 30.0, 0.0, 1e-4, -1, 0, None, 0) == EINVAL
    assert lib.pn_step(d, d, d, 16, 1.0, 30.0, 0.0, 1e-4, 1, 7, None, 0) == EINVAL
    assert lib.pn_accel(d, d, d, 16, 1.0, 30.0, 0.0, 9, d, d, d, None, 0) == EINVAL
    assert lib.pn_accel_eih(d, None, d, 16, 1.0, 30.0, 0.0, 0, d, d, d, None, 0) == EINVAL
    assert lib.pn_accel_eih(d, d, d, 16, 1.0, 30.0, 0.0, 5, d, d, d, None, 0) == EINVAL
    assert lib.pn_set_shape(0, 10, 5, 1, 4, 0) == EINVAL
    assert lib.pn_set_shape(0, 2, 5, 3, 4, 0) == EINVAL
    assert lib.pn_set_shape(0, 2, 5, 1, 2, 0) == EINVAL  # wavefronts per i-range: 1, 4 or 8
    assert lib.pn_diagnostics(d, d, d, 16, 1.0, 30.0, 0.0, None, None, 0) == EINVAL
    assert lib.pn_encounters(d, d, d, 2, 1.0, 30.0, 0.1, d, None, 0) == EINVAL
    assert lib.pn_encounters(d, d, d, 16, 1.0, 30.0, -0.1, d, None, 0) == EINVAL
    assert lib.pn_encounters(d, None, d, 16, 1.0, 30.0, 0.1, d, None, 0) == EINVAL
    assert lib.pn_encounters(d, d, d, 16, 0.0, 30.0, 0.1, d, None, 0) == EINVAL
    assert lib.pn_last_timing(None) == EINVAL
    # pn_jerk: both outputs required; pn_step_hermite: dt > 0, nsteps >= 0
    assert lib.pn_jerk(d, d, d, 16, 1.0, 30.0, 0.0, None, d, None, 0) == EINVAL
    assert lib.pn_jerk(d, d, d, 16, 1.0, 30.0, 0.0, d, None, None, 0) == EINVAL
    assert lib.pn_jerk(d, None, d, 16, 1.0, 30.0, 0.0, d, d, None, 0) == EINVAL
    assert lib.pn_step_hermite(d, d, d, 16, 1.0, 30.0, 0.0, 0.0, 1, None, 0) == EINVAL
    assert lib.pn_step_hermite(d, d, d, 16, 1.0, 30.0, 0.0, -1e-3, 1, None, 0) == EINVAL
    assert lib.pn_step_hermite(d, d, d, 16, 1.0, 30.0, 0.0, 1e-3, -2, None, 0) == EINVAL
    assert lib.pn_step_hermite(d, d, d, 1, 1.0, 30.0, 0.0, 1e-3, 1, None, 0) == EINVAL


def test_noalloc_limits_without_device(lib):
    """pn_accel_noalloc rejects, before any device work, a size whose scratch
    exceeds its fixed array even with one j-split, and PN_TIMING; the error
    text names the sizes."""
    EINVAL = -1
    d = FAKE
    assert lib.pn_accel_noalloc(d, d, d, 400000, 1.0, 30.0, 0.0, 0, d, d, d, None, 0) == EINVAL
    msg = lib.pn_strerror(EINVAL).decode()
    assert "pn_accel_noalloc" in msg and "400000" in msg and str(64 << 20) in msg
    assert lib.pn_accel_noalloc(d, d, d, 400000, 1.0, 30.0, 0.0, 1, d, d, d, None, 0) == EINVAL
    assert lib.pn_accel_noalloc(d, d, d, 16, 1.0, 30.0, 0.0, 0, d, d, d, None, 4) == EINVAL
    assert "PN_TIMING" in lib.pn_strerror(EINVAL).decode()
    assert lib.pn_accel_noalloc(d, d, d, 16, 1.0, 30.0, 0.0, 3, d, d, d, None, 0) == EINVAL
    assert lib.pn_accel_noalloc(d, None, d, 16, 1.0, 30.0, 0.0, 0, d, d, d, None, 0) == EINVAL
    # a later argument error without detail does not repeat the old text
    assert lib.pn_accel_noalloc(d, d, d, 1, 1.0, 30.0, 0.0, 0, d, d, d, None, 0) == EINVAL
    assert lib.pn_strerror(EINVAL).decode() == "invalid argument"


def test_batched_validation_without_device(lib):
    EINVAL = -1
    d = FAKE
    off = (ctypes.c_int64 * 3)(0, 10, 11)  # second system has a single body
    p = (ctypes.c_double * 2)(1.0, 1.0)
    cast = lambda a: ctypes.cast(a, ctypes.c_void_p)  # noqa: E731
    assert lib.pn_step_batched(2, cast(off), cast(p), cast(p), cast(p), d, d, d, 1e-4, 1, 0,
                               None, 0) == EINVAL
    off = (ctypes.c_int64 * 3)(1, 10, 20)  # must start at 0
    assert lib.pn_step_batched(2, cast(off), cast(p), cast(p), cast(p), d, d, d, 1e-4, 1, 0,
                               None, 0) == EINVAL
    assert lib.pn_step_batched(0, cast(off), cast(p), cast(p), cast(p), d, d, d, 1e-4, 1, 0,
                               None, 0) == EINVAL


def test_stage_kernel_table_without_device(lib, monkeypatch):
    """pn_set_stage_kernel / pn_query_stage_kernel are host-only: entries by
    precision and size range (the first match wins), clearing, the PN_STAGE_NS
    override, and argument checks."""
    from paper_1801_07986_amd import _binding

    EINVAL = -1
    monkeypatch.delenv("PN_STAGE_NS", raising=False)
    try:
        assert lib.pn_set_stage_kernel(-1, 0, 0, 0) == 0
        assert lib.pn_query_stage_kernel(0, 100) == 0 and lib.pn_query_stage_kernel(1, 100) == 0
        assert lib.pn_set_stage_kernel(0, 2, 300, 4) == 0
        assert lib.pn_set_stage_kernel(0, 301, 1000, 8) == 0
        assert lib.pn_set_stage_kernel(0, 2, 5000, 16) == 0  # covered below 1001 by the first two
        assert lib.pn_set_stage_kernel(1, 50, 60, 2) == 0
        assert [lib.pn_query_stage_kernel(0, n) for n in (2, 300, 301, 1000, 1001, 5000, 5001)] == \
            [4, 4, 8, 8, 16, 16, 0]
        assert [lib.pn_query_stage_kernel(1, n) for n in (49, 50, 60, 61)] == [0, 2, 2, 0]
        monkeypatch.setenv("PN_STAGE_NS", "2")
        assert lib.pn_query_stage_kernel(0, 5001) == 2
        monkeypatch.setenv("PN_STAGE_NS", "0")
        assert lib.pn_query_stage_kernel(0, 100) == 0
        monkeypatch.delenv("PN_STAGE_NS")
        for args in ((2, 2, 10, 4), (0, 1, 10, 4), (0, 10, 9, 4), (0, 2, 10, 3), (0, 2, 10, 0),
                     (0, 2, 10, 32)):
            assert lib.pn_set_stage_kernel(*args) == EINVAL
        assert lib.pn_query_stage_kernel(0, 1) == EINVAL
        assert lib.pn_query_stage_kernel(2, 100) == EINVAL
        assert lib.pn_set_stage_kernel(-1, 0, 0, 0) == 0
        assert lib.pn_query_stage_kernel(0, 100) == 0
    finally:
        _binding.install_tuned_shapes()


def test_batch_shape_without_device(lib):
    """pn_set_batch_shape / pn_query_batch_shape are host-only: the default
    rule (1 i per lane; a common split count giving ~16k sweep workgroups, at
    most 16, capped per system at Ns / 128), a forced shape, and argument
    checks."""
    from paper_1801_07986_amd import _binding

    EINVAL = -1
    off = [0, 1000, 1003, 6003]  # Ns = 999, 2, 4999
    try:
        for prec in (0, 1):
            lib.pn_set_batch_shape(prec, 1, 0)
            ipt, splits = _binding.pn_query_batch_shape(prec, off)
            tot = -(-999 // 64) + 1 + -(-4999 // 64)
            common = max(1, min(16, -(-16384 // tot)))
            assert ipt == 1 and splits == [max(1, min(common, n // 128)) for n in (999, 2, 4999)]
            lib.pn_set_batch_shape(prec, 2, 5)
            ipt, splits = _binding.pn_query_batch_shape(prec, off)
            assert ipt == 2 and splits == [5, 1, 5]
        assert lib.pn_set_batch_shape(0, 3, 0) == EINVAL
        assert lib.pn_set_batch_shape(0, 1, 65) == EINVAL
        assert lib.pn_set_batch_shape(4, 1, 0) == EINVAL
        out = (ctypes.c_int * 4)()
        bad = (ctypes.c_int64 * 3)(0, 10, 11)
        assert lib.pn_query_batch_shape(0, 2, ctypes.cast(bad, ctypes.c_void_p),
                                        ctypes.cast(out, ctypes.c_void_p)) == EINVAL
        assert lib.pn_query_batch_shape(0, 0, ctypes.cast(bad, ctypes.c_void_p),
                                        ctypes.cast(out, ctypes.c_void_p)) == EINVAL
    finally:
        _binding.install_tuned_shapes()


def test_strerror(lib):
    for code in (0, -1, -2, -3, -4, 99):
        assert isinstance(lib.pn_strerror(code), bytes)


def test_binding_fails_loudly_without_library(monkeypatch, tmp_path):
    from paper_1801_07986_amd import _binding

    monkeypatch.setattr(_binding, "_lib", None)
    monkeypatch.setattr(_binding, "LIB_PATH", str(tmp_path / "missing.so"))
    with pytest.raises(ImportError):
        _binding.load()


def test_binding_rejects_host_tensors():
    torch = pytest.importorskip("torch")
    from paper_1801_07986_amd import _binding

    x = torch.zeros(4, 3, dtype=torch.float64)
    with pytest.raises(TypeError):
        _binding._ptr(x)


def test_query_shape_follows_the_tuned_table(lib):
    """pn_query_shape is host-only: the shape the library would launch, from
    the table the binding installs when it loads."""
    import json

    from paper_1801_07986_amd import _binding

    table = json.load(open(_binding.TUNED_PATH))
    for e in table["entries"]:
        prec = 0 if e["precision"] == "fp64" else 1
        N = e["measured_N"]
        ipt, ws, nsplit, iblocks = _binding.pn_query_shape(prec, N)
        assert (ipt, ws) == (e["ipt"], e["ws"])
        assert iblocks == -(-(N - 1) // ((256 if ws == 1 else 64) * ipt))
        if e["nsplit"] > 0:  # the split count rounds through the j-chunk size
            Ns = N - 1
            want = max(1, min(e["nsplit"], Ns))
            jchunk = -(-Ns // want)
            assert nsplit == -(-Ns // jchunk)
    # eight wavefronts per i-range: i-blocks of 64 lanes, as with four
    _binding.pn_set_shape(-1, 0, 0, 0, 0, 0)
    _binding.pn_set_shape(0, 2, 1 << 28, 2, 8, 12)
    try:
        assert tuple(_binding.pn_query_shape(0, 16384)) == (2, 8, 12, 128)
    finally:
        _binding.install_tuned_shapes()
    EINVAL = -1
    out = (ctypes.c_int * 4)()
    assert lib.pn_query_shape(0, 1, ctypes.cast(out, ctypes.c_void_p)) == EINVAL
    assert lib.pn_query_shape(7, 100, ctypes.cast(out, ctypes.c_void_p)) == EINVAL
    assert lib.pn_query_shape(0, 100, None) == EINVAL


def test_bench_refuses_more_than_one_gpu():
    """bench.py measures one GPU; asked for more it exits with a message
    (before touching torch or the GPU)."""
    import sys

    res = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                         capture_output=True, text=True, timeout=120)
    assert res.returncode == 2
    assert "one GPU" in res.stderr


def test_table32_oracle_leg_runs_the_protocol():
    """bench.py's Table 3.2 oracle leg (CPU only): within its time budget it
    runs energy, 32 RK4 steps, energy; without budget it extrapolates from
    one evaluation and says so."""
    import sys

    import numpy as np

    sys.path.insert(0, ROOT)
    import bench
    import oracle
    from paper_1801_07986_amd import inputs

    pos, vel, mass = inputs.cold_sphere_bh(63, seed=3)
    r = bench.oracle_table32(oracle, pos, vel, mass, samples=3, budget_s=60.0)
    assert r["runs"] == 3 and r["kind"].startswith("measured") and r["mean_s"] > 0
    assert np.isfinite(r["std_s"])
    r = bench.oracle_table32(oracle, pos, vel, mass, samples=3, budget_s=0.0)
    assert r["runs"] == 0 and r["kind"].startswith("extrapolated") and r["std_s"] is None


def test_autotune_partial_retune_keeps_other_entries(tmp_path, monkeypatch):
    """autotune --sizes: the re-tuned sizes replace their entries, the others
    are kept, and the ranges are those of a full run over the union of sizes
    (host logic; the timing is replaced by a stub)."""
    import json

    from paper_1801_07986_amd import autotune

    src = os.path.join(ROOT, "paper_1801_07986_amd", "tuned_shapes.json")
    with open(src) as f:
        old = json.load(f)
    out = tmp_path / "t.json"
    out.write_text(json.dumps(old))

    def fake_tune(sizes, log=print, precisions=("fp64", "mixed")):
        return [dict(N=N, precision=p, ipt=2, ws=1, nsplit=7, step_ms=1.0, default_step_ms=2.0)
                for N in sizes for p in precisions]

    monkeypatch.setattr(autotune, "tune", fake_tune)
    autotune.main(["--sizes", "1024,5000", "--out", str(out)])
    new = json.loads(out.read_text())
    assert new["stage"] == old["stage"] and new["batched"] == old["batched"]
    for prec in ("fp64", "mixed"):
        e_old = [e for e in old["entries"] if e["precision"] == prec]
        e_new = [e for e in new["entries"] if e["precision"] == prec]
        assert [e["measured_N"] for e in e_new] == sorted(
            {e["measured_N"] for e in e_old if e["measured_N"] != 1024} | {1024, 5000})
        for e in e_new:
            if e["measured_N"] in (1024, 5000):
                assert (e["ipt"], e["ws"], e["nsplit"]) == (2, 1, 7)
            else:
                o = next(x for x in e_old if x["measured_N"] == e["measured_N"])
                assert (e["ipt"], e["ws"], e["nsplit"]) == (o["ipt"], o["ws"], o["nsplit"])
        # ranges tile [2, 2^28] without gaps or overlaps
        assert e_new[0]["n_min"] == 2 and e_new[-1]["n_max"] == 1 << 28
        assert all(a["n_max"] + 1 == b["n_min"] for a, b in zip(e_new, e_new[1:]))


def test_autotune_one_precision_keeps_the_other(tmp_path, monkeypatch):
    """autotune --precision: only that precision's entries are re-measured
    (at --sizes, or over the whole ladder); the other precision's table is
    kept unchanged (host logic; the timing is replaced by a stub)."""
    import json

    from paper_1801_07986_amd import autotune

    src = os.path.join(ROOT, "paper_1801_07986_amd", "tuned_shapes.json")
    with open(src) as f:
        old = json.load(f)
    asked = []

    def fake_tune(sizes, log=print, precisions=("fp64", "mixed")):
        asked.append((list(sizes), tuple(precisions)))
        return [dict(N=N, precision=p, ipt=2, ws=1, nsplit=7, step_ms=1.0, default_step_ms=2.0)
                for N in sizes for p in precisions]

    monkeypatch.setattr(autotune, "tune", fake_tune)
    shape = lambda e: (e["measured_N"], e["ipt"], e["ws"], e["nsplit"])  # noqa: E731
    by_prec = lambda t, p: [shape(e) for e in t["entries"] if e["precision"] == p]  # noqa: E731

    out = tmp_path / "a.json"
    out.write_text(json.dumps(old))
    autotune.main(["--sizes", "65536,131072", "--precision", "fp64", "--out", str(out)])
    new = json.loads(out.read_text())
    assert asked[-1] == ([65536, 131072], ("fp64",))
    assert by_prec(new, "mixed") == by_prec(old, "mixed")
    assert new["stage"] == old["stage"] and new["batched"] == old["batched"]
    for n, ipt, ws, ns in by_prec(new, "fp64"):
        o = next(x for x in by_prec(old, "fp64") if x[0] == n)
        assert (ipt, ws, ns) == ((2, 1, 7) if n in (65536, 131072) else o[1:])
    assert len(by_prec(new, "fp64")) == len(by_prec(old, "fp64"))

    out = tmp_path / "b.json"
    out.write_text(json.dumps(old))
    autotune.main(["--precision", "mixed", "--quick", "--out", str(out)])
    new = json.loads(out.read_text())
    assert asked[-1] == (autotune.QUICK_SIZES, ("mixed",))
    assert by_prec(new, "fp64") == by_prec(old, "fp64")
    assert by_prec(new, "mixed") == [(n, 2, 1, 7) for n in autotune.QUICK_SIZES]
    for prec in ("fp64", "mixed"):
        e_new = [e for e in new["entries"] if e["precision"] == prec]
        assert e_new[0]["n_min"] == 2 and e_new[-1]["n_max"] == 1 << 28
        assert all(a["n_max"] + 1 == b["n_min"] for a, b in zip(e_new, e_new[1:]))
