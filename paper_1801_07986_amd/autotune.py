"""Launch-shape autotuner for the star-star sweep.

For each precision and a ladder of system sizes it times whole RK4 steps
(pn_step: the chained sequence of sweeps and epilogues, replayed as a graph;
wall clock around a run of steps on the caller's stream) over the candidate
shapes

    ipt in {1, 2}   i-bodies per lane
    ws in {1, 4, 8} wavefronts sharing one i-range (8: workgroups of 512 threads)
    nsplit          j-range splits (at least 4 j per wavefront, or 0 = the
                    library's default rule)

At small N the step is latency-bound and more splits (shorter j-loops on
more SIMDs) pay even at a few j per wavefront; at large N the sweep is
compute-bound and the split count matters little.

and writes the fastest shape per size as a table of N-ranges (boundaries at
the geometric midpoints between measured sizes) to ``tuned_shapes.json``,
which the binding installs into the library with ``pn_set_shape`` when it is
loaded.  Shapes change only the speed: every shape computes the same sums.

With --batched it instead tunes pn_step_batched on the benchmark's 256-system
ensemble (N ~ U{1024..16384}): whole ensemble steps over i-bodies per lane
(1 or 2, every system) x the common j-split count (the rule, 1, 2, 4, 8), per
precision, and stores the fastest under "batched" in the same table
(installed with pn_set_batch_shape).

With --stage it tunes pn_step's one-launch stages (k_stage) for small
systems: at each size up to 4096 bodies, whole RK4 steps with 2, 4, 8 or 16
stars per workgroup against the chained two-kernel stages in their tuned
shape; the sizes where a one-launch stage wins become "stage" entries of the
same table (installed with pn_set_stage_kernel).

With --sizes N,... and/or --precision fp64|mixed it re-tunes only those sizes
and/or that precision and keeps the table's other entries.

Usage (on the GPU):  python -m paper_1801_07986_amd.autotune [--out PATH]
                     [--quick | --batched | --stage | --sizes N,...] [--precision fp64|mixed]
"""
from __future__ import annotations

import argparse
import itertools
import json
import math
import os
import sys
import time

SIZES = [100, 300, 1024, 2048, 4096, 8192, 16384, 32768, 65536, 131072, 262144]
QUICK_SIZES = [100, 1024, 4096, 16384, 65536]
SPLITS = (0, 1, 2, 4, 8, 12, 16, 24, 32, 48, 64, 128)


def candidates(N: int):
    """(ipt, ws, nsplit); nsplit 0 is the library's default rule for that N."""
    Ns = N - 1
    for ipt, ws in itertools.product((1, 2), (1, 4, 8)):
        for ns in SPLITS:
            if ns <= 1 or ns <= max(1, Ns // (4 * ws)):
                yield ipt, ws, ns


def time_step(pn, torch, P, V, Mm, prec, budget_s=0.05, reps=3):
    """Best of `reps` runs of whole RK4 steps (each run at least budget_s of
    wall clock); ms per step.  The first call captures the step graph."""
    stream = torch.cuda.current_stream()
    pn.pn_step(P, V, Mm, 1.0, 30.0, 1e-4, 1e-7, 2, prec, stream=stream)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    pn.pn_step(P, V, Mm, 1.0, 30.0, 1e-4, 1e-7, 1, prec, stream=stream)
    torch.cuda.synchronize()
    one = max(time.perf_counter() - t0, 1e-6)
    steps = max(1, min(2000, int(budget_s / one)))
    best = None
    for _ in range(reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        pn.pn_step(P, V, Mm, 1.0, 30.0, 1e-4, 1e-7, steps, prec, stream=stream)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) / steps * 1e3
        best = ms if best is None else min(best, ms)
    return best


PRECISIONS = ("fp64", "mixed")


def tune(sizes, log=print, precisions=PRECISIONS):
    import torch

    import paper_1801_07986_amd as pn
    from paper_1801_07986_amd import inputs

    pn.load()
    pn.pn_set_shape(-1, 0, 0, 0, 0, 0)  # measure without any installed table,
    pn.pn_set_stage_kernel(-1, 0, 0, 0)  # with the chained stages
    results = []
    for N in sizes:
        pos, vel, mass = inputs.plummer_bh(N, 0.1, 9)
        P = torch.from_numpy(pos).cuda()
        V = torch.from_numpy(vel).cuda()
        Mm = torch.from_numpy(mass).cuda()
        for prec_name, prec in (("fp64", pn.PN_FP64), ("mixed", pn.PN_MIXED)):
            if prec_name not in precisions:
                continue
            best = None
            for ipt, ws, ns in candidates(N):
                os.environ["PN_SHAPE"] = f"{ipt},{ws},{ns}"
                ms = time_step(pn, torch, P, V, Mm, prec)
                log(f"[autotune]   N={N} {prec_name} ipt={ipt} ws={ws} nsplit={ns}: {ms:.4f} ms/step")
                if best is None or ms < best[0]:
                    best = (ms, ipt, ws, ns)
            os.environ.pop("PN_SHAPE", None)
            default_ms = time_step(pn, torch, P, V, Mm, prec)
            ms, ipt, ws, ns = best
            results.append(dict(N=N, precision=prec_name, ipt=ipt, ws=ws, nsplit=ns,
                                step_ms=ms, default_step_ms=default_ms))
            log(f"[autotune] N={N} {prec_name}: best ipt={ipt} ws={ws} nsplit={ns} "
                f"{ms:.4f} ms/step (default rule {default_ms:.4f} ms)")
    return results


BATCH_CANDIDATES = [(ipt, ns) for ipt in (1, 2) for ns in (0, 1, 2, 4, 8)]


def tune_batched(log=print, steps=2, reps=2):
    """Fastest (ipt, common split count) of pn_step_batched per precision on
    the 256-system ensemble, timing whole ensemble steps (graph replay)."""
    import numpy as np
    import torch

    import paper_1801_07986_amd as pn
    from paper_1801_07986_amd import inputs

    pn.load()
    systems = inputs.ensemble()
    ps, vs, ms, off = [], [], [], [0]
    for s in systems:
        p, v, m = inputs.plummer_bh(s["N"], s["M_bh"], s["seed"])
        ps.append(p)
        vs.append(v)
        ms.append(m)
        off.append(off[-1] + s["N"])
    P = torch.from_numpy(np.concatenate(ps)).cuda()
    V = torch.from_numpy(np.concatenate(vs)).cuda()
    Mm = torch.from_numpy(np.concatenate(ms)).cuda()
    Gs = [1.0] * len(systems)
    cs = [s["c"] for s in systems]
    es = [s["eps"] for s in systems]
    out = []
    for prec_name, prec in (("fp64", pn.PN_FP64), ("mixed", pn.PN_MIXED)):
        timings = {}
        for ipt, ns in BATCH_CANDIDATES:
            os.environ["PN_BATCH_SHAPE"] = f"{ipt},{ns}"
            pn.pn_step_batched(off, Gs, cs, es, P, V, Mm, 1e-7, 1, prec)  # captures the graph
            torch.cuda.synchronize()
            best = None
            for _ in range(reps):
                t0 = time.perf_counter()
                pn.pn_step_batched(off, Gs, cs, es, P, V, Mm, 1e-7, steps, prec)
                torch.cuda.synchronize()
                ms_step = (time.perf_counter() - t0) / steps * 1e3
                best = ms_step if best is None else min(best, ms_step)
            timings[(ipt, ns)] = best
            log(f"[autotune] ensemble {prec_name} ipt={ipt} splits={ns or 'rule'}: "
                f"{best:.3f} ms/step")
        os.environ.pop("PN_BATCH_SHAPE", None)
        (ipt, ns), ms_best = min(timings.items(), key=lambda kv: kv[1])
        out.append(dict(precision=prec_name, ipt=ipt, nsplit=ns, step_ms=round(ms_best, 4),
                        default_step_ms=round(timings[(1, 0)], 4), n_sys=len(systems),
                        bodies=int(off[-1])))
        log(f"[autotune] ensemble {prec_name}: best ipt={ipt} splits={ns or 'rule'} "
            f"{ms_best:.3f} ms/step (1 i per lane, rule: {timings[(1, 0)]:.3f})")
    return out


STAGE_SIZES = [100, 300, 1024, 2048, 4096]
STAGE_NS = (2, 4, 8, 16)


def tune_stage(log=print):
    """Sizes (and stars per workgroup) where pn_step's one-launch stages beat
    the chained stages in the installed shapes; whole RK4 steps."""
    import torch

    import paper_1801_07986_amd as pn
    from paper_1801_07986_amd import inputs

    pn.load()  # the chained stages keep the installed shape table
    pn.pn_set_stage_kernel(-1, 0, 0, 0)
    rows = []
    for N in STAGE_SIZES:
        pos, vel, mass = inputs.plummer_bh(N, 0.1, 9)
        P = torch.from_numpy(pos).cuda()
        V = torch.from_numpy(vel).cuda()
        Mm = torch.from_numpy(mass).cuda()
        for prec_name, prec in (("fp64", pn.PN_FP64), ("mixed", pn.PN_MIXED)):
            os.environ["PN_STAGE_NS"] = "0"
            chain = time_step(pn, torch, P, V, Mm, prec)
            best = (chain, 0)
            for ns in STAGE_NS:
                os.environ["PN_STAGE_NS"] = str(ns)
                ms = time_step(pn, torch, P, V, Mm, prec)
                log(f"[autotune]   N={N} {prec_name} one-launch stages, {ns} stars per workgroup: "
                    f"{ms:.4f} ms/step")
                if ms < best[0]:
                    best = (ms, ns)
            rows.append(dict(N=N, precision=prec_name, ns=best[1], step_ms=best[0],
                             chain_step_ms=chain))
            log(f"[autotune] N={N} {prec_name}: chained {chain:.4f} ms/step, best "
                f"{'chained' if best[1] == 0 else f'{best[1]} stars per workgroup'} {best[0]:.4f}")
    os.environ.pop("PN_STAGE_NS", None)
    entries = []
    for prec in ("fp64", "mixed"):
        rs = sorted((r for r in rows if r["precision"] == prec), key=lambda r: r["N"])
        for k, r in enumerate(rs):
            if r["ns"] == 0:
                continue
            lo = 2 if k == 0 else int(math.sqrt(rs[k - 1]["N"] * r["N"])) + 1
            hi = int(math.sqrt(r["N"] * (rs[k + 1]["N"] if k + 1 < len(rs) else 2 * r["N"])))
            entries.append(dict(precision=prec, n_min=lo, n_max=hi, ns=r["ns"], measured_N=r["N"],
                                step_ms=round(r["step_ms"], 5),
                                chain_step_ms=round(r["chain_step_ms"], 5)))
    return entries


def to_table(results):
    entries = []
    for prec in ("fp64", "mixed"):
        rows = sorted((r for r in results if r["precision"] == prec), key=lambda r: r["N"])
        for k, r in enumerate(rows):
            lo = 2 if k == 0 else int(math.sqrt(rows[k - 1]["N"] * r["N"])) + 1
            hi = (1 << 28) if k == len(rows) - 1 else int(math.sqrt(r["N"] * rows[k + 1]["N"]))
            entries.append(dict(precision=prec, n_min=lo, n_max=hi, ipt=r["ipt"], ws=r["ws"],
                                nsplit=r["nsplit"], measured_N=r["N"],
                                step_ms=round(r["step_ms"], 5),
                                default_step_ms=round(r["default_step_ms"], 5)))
    return {"device": "MI355X (gfx950)", "tool": "paper_1801_07986_amd.autotune",
            "created": time.strftime("%Y-%m-%d %H:%M:%S"), "entries": entries}


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=os.path.join(os.path.dirname(os.path.abspath(__file__)),
                                                  "tuned_shapes.json"))
    ap.add_argument("--quick", action="store_true")
    ap.add_argument("--sizes", default=None,
                    help="comma-separated N: re-tune these sizes only, keeping the table's "
                         "other entries (ranges are recomputed over all measured sizes)")
    ap.add_argument("--precision", choices=PRECISIONS, default=None,
                    help="re-tune this precision only, keeping the other's entries")
    ap.add_argument("--batched", action="store_true",
                    help="tune pn_step_batched's shape only (kept with the existing table)")
    ap.add_argument("--stage", action="store_true",
                    help="tune pn_step's one-launch stages only (kept with the existing table)")
    args = ap.parse_args(argv)
    log = lambda m: print(m, file=sys.stderr, flush=True)  # noqa: E731
    old = {}
    if os.path.exists(args.out):
        with open(args.out) as f:
            old = json.load(f)
    if args.batched:
        table = dict(old)
        table["batched"] = tune_batched(log=log)
        table["batched_created"] = time.strftime("%Y-%m-%d %H:%M:%S")
    elif args.stage:
        table = dict(old)
        table["stage"] = tune_stage(log=log)
        table["stage_created"] = time.strftime("%Y-%m-%d %H:%M:%S")
    else:
        precs = (args.precision,) if args.precision else PRECISIONS
        if args.sizes:
            sizes = sorted({int(s) for s in args.sizes.split(",")})
        else:
            sizes = QUICK_SIZES if args.quick else SIZES
        if args.sizes or args.precision:
            # an entry is re-measured only if both its size and its precision are
            kept = [dict(N=e["measured_N"], precision=e["precision"], ipt=e["ipt"], ws=e["ws"],
                         nsplit=e["nsplit"], step_ms=e["step_ms"],
                         default_step_ms=e["default_step_ms"])
                    for e in old.get("entries", [])
                    if not (e["measured_N"] in sizes and e["precision"] in precs)
                    and (args.sizes or e["precision"] not in precs)]
            table = to_table(kept + tune(sizes, log=log, precisions=precs))
        else:
            table = to_table(tune(sizes, log=log))
        for key in ("batched", "stage"):
            if key in old:
                table[key] = old[key]
                table[key + "_created"] = old.get(key + "_created")
    with open(args.out, "w") as f:
        json.dump(table, f, indent=1)
        f.write("\n")
    print(json.dumps(table))


if __name__ == "__main__":
    main()
