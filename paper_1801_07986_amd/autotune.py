"""Launch-shape autotuner for the star-star sweep.

For each precision and a ladder of system sizes it times complete force
evaluations (prologue, pair sweep, epilogue; pn_accel on the caller's stream,
HIP events around it) over the candidate shapes

    ipt in {1, 2}   i-bodies per lane
    ws in {1, 4}    wavefronts sharing one i-range
    nsplit          j-range splits (powers of two with at least 32 j per
                    wavefront, or 0 = the library's default rule)

and writes the fastest shape per size as a table of N-ranges (boundaries at
the geometric midpoints between measured sizes) to ``tuned_shapes.json``,
which the binding installs into the library with ``pn_set_shape`` when it is
loaded.  Shapes change only the speed: every shape computes the same sums.

Usage (on the GPU):  python -m paper_1801_07986_amd.autotune [--out PATH] [--quick]
"""
from __future__ import annotations

import argparse
import itertools
import json
import math
import os
import sys
import time

SIZES = [1024, 2048, 4096, 8192, 16384, 32768, 65536, 131072, 262144]
QUICK_SIZES = [1024, 4096, 16384, 65536]


def candidates(N: int):
    """(ipt, ws, nsplit); nsplit 0 is the library's default rule for that N."""
    Ns = N - 1
    for ipt, ws in itertools.product((1, 2), (1, 4)):
        for ns in (0, 1, 2, 4, 8, 16, 32, 64, 128):
            if ns <= 1 or ns <= max(1, Ns // (32 * ws)):
                yield ipt, ws, ns


def time_eval(pn, torch, P, V, Mm, out, prec, reps_min=3, budget_s=0.05):
    stream = torch.cuda.current_stream()
    pn.pn_accel(P, V, Mm, 1.0, 30.0, 1e-4, prec, out, None, None, stream=stream)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    reps, total = 0, 0.0
    while reps < reps_min or total < budget_s * 1e3:
        e0.record(stream)
        pn.pn_accel(P, V, Mm, 1.0, 30.0, 1e-4, prec, out, None, None, stream=stream,
                    flags=pn.PN_ASYNC)
        e1.record(stream)
        e1.synchronize()
        total += e0.elapsed_time(e1)
        reps += 1
        if reps >= 50:
            break
    return total / reps


def tune(sizes, log=print):
    import torch

    import paper_1801_07986_amd as pn
    from paper_1801_07986_amd import inputs

    pn.load()
    pn.pn_set_shape(-1, 0, 0, 0, 0, 0)  # measure without any installed table
    results = []
    for N in sizes:
        pos, vel, mass = inputs.plummer_bh(N, 0.1, 9)
        P = torch.from_numpy(pos).cuda()
        V = torch.from_numpy(vel).cuda()
        Mm = torch.from_numpy(mass).cuda()
        out = torch.empty((N, 3), dtype=torch.float64, device="cuda")
        for prec_name, prec in (("fp64", pn.PN_FP64), ("mixed", pn.PN_MIXED)):
            best = None
            for ipt, ws, ns in candidates(N):
                os.environ["PN_SHAPE"] = f"{ipt},{ws},{ns}"
                ms = time_eval(pn, torch, P, V, Mm, out, prec)
                if best is None or ms < best[0]:
                    best = (ms, ipt, ws, ns)
            os.environ.pop("PN_SHAPE", None)
            default_ms = time_eval(pn, torch, P, V, Mm, out, prec)
            ms, ipt, ws, ns = best
            results.append(dict(N=N, precision=prec_name, ipt=ipt, ws=ws, nsplit=ns,
                                eval_ms=ms, default_eval_ms=default_ms))
            log(f"[autotune] N={N} {prec_name}: best ipt={ipt} ws={ws} nsplit={ns} "
                f"{ms:.4f} ms/eval (default rule {default_ms:.4f} ms)")
    return results


def to_table(results):
    entries = []
    for prec in ("fp64", "mixed"):
        rows = sorted((r for r in results if r["precision"] == prec), key=lambda r: r["N"])
        for k, r in enumerate(rows):
            lo = 2 if k == 0 else int(math.sqrt(rows[k - 1]["N"] * r["N"])) + 1
            hi = (1 << 28) if k == len(rows) - 1 else int(math.sqrt(r["N"] * rows[k + 1]["N"]))
            entries.append(dict(precision=prec, n_min=lo, n_max=hi, ipt=r["ipt"], ws=r["ws"],
                                nsplit=r["nsplit"], measured_N=r["N"],
                                eval_ms=round(r["eval_ms"], 5),
                                default_eval_ms=round(r["default_eval_ms"], 5)))
    return {"device": "MI355X (gfx950)", "tool": "paper_1801_07986_amd.autotune",
            "created": time.strftime("%Y-%m-%d %H:%M:%S"), "entries": entries}


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=os.path.join(os.path.dirname(os.path.abspath(__file__)),
                                                  "tuned_shapes.json"))
    ap.add_argument("--quick", action="store_true")
    args = ap.parse_args(argv)
    res = tune(QUICK_SIZES if args.quick else SIZES,
               log=lambda m: print(m, file=sys.stderr, flush=True))
    table = to_table(res)
    with open(args.out, "w") as f:
        json.dump(table, f, indent=1)
        f.write("\n")
    print(json.dumps(table))


if __name__ == "__main__":
    main()
