#!/usr/bin/env python3
"""Throughput benchmark of the limited-1PN direct N-body hot path on one MI355X.

Default workload: Plummer sphere N = 16384 (16383 equal-mass stars, total
star mass 1, scale radius 1, G = 1) plus a black hole of mass 0.05 at rest at
the origin, c = 30, eps = 1e-4, FP64, fixed RK4 steps of dt = 1e-4.  One
"step" is one RK4 step = 4 force evaluations (each: prologue, fused star-star
sweep, epilogue with the Runge-Kutta stage update).  Inputs are resident on
the GPU before the timed region.

Metric: pair interactions per second = 4 * steps * N^2 / wall time.

Printed (one JSON line on stdout): value, roofline of the fused pair kernel
(its average duration measured live with HIP events on the stream it runs on),
the CPU oracle timed on a bounded sample on this host, and a secondary
N = 65536 mixed-precision vs FP64 comparison.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Algorithmic flops per star-star pair interaction of the fused Newtonian +
# 1PN sweep, counted on the expression tree the sweep evaluates (add/sub/mul
# = 1, FMA = 2, rsqrt = 1; the refinement of the FP64 reciprocal square root
# is overhead and not counted):
#   potential + Newtonian pull: x_ij 3 sub; R^2 3 FMA; rsqrt; R^-2, G m R^-1,
#     G m R^-3 3 mul; U += 1 add; G += 3 FMA                          -> 20
#   1PN pair sum: x.s_j 1 mul + 2 FMA; (x.s_j) R^-1 1 mul; S' 7 FMA (the
#     square, 4 v_i.v_j, x.b_j/2); x.k_i 1 mul + 2 FMA; D' 1 FMA; the two
#     coefficients 2 mul; Q += 6 FMA; sum of D' coefficients 1 add;
#     Q7 += 3 FMA                                                     -> 48
FLOP_PER_PAIR_FUSED = 68.0
PEAK_FP64_VALU = 78.6e12  # 256 CUs x 2.4 GHz x 64 FMA lanes x 2 flop
# The mixed sweep uses no packed FP32, yet measurably issues faster than the
# FP64 one (above 78.6 TFLOP/s-equivalent), so it is held to the FP32 vector
# figure of the chip (157.3 TFLOP/s), the stricter denominator.
PEAK_FP32_VALU = 157.3e12
# HBM bytes per fused-sweep launch from rocprofv3 PMC runs of this file
# (FETCH_SIZE x 2.0 + WRITE_SIZE x 1.0, KiB per dispatch; the factors are what
# the two counters read for a 512 MiB device copy, --copy-calibration 512).
# Measured for the kernels as they stand; drop an entry when its kernel changes.
# Keyed by (workload, kernel, j-splits): the launch shape comes from the tuned
# table, so a figure applies only to the kernel and split count it was taken on.
TRAFFIC_BYTES = {
    # FETCH 7288.77 KiB, WRITE 17291.1 KiB per launch
    ("plummer_n16384_fp64", "k_pair_bh<double,3,2,8>", 12): 32633487,
    # FETCH 49328.6 KiB, WRITE 94334.7 KiB per launch
    ("plummer_n65536_mixed", "k_pair_bh<float,3,1,8>", 16): 197623706,
}


def log(msg: str) -> None:
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default="plummer_n16384_fp64")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-secondary", action="store_true", help="skip the N=65536 comparison")
    ap.add_argument("--table32", action="store_true",
                    help="replicate the paper's Table 3.2 timing protocol instead")
    ap.add_argument("--samples", type=int, default=10, help="samples per N for --table32")
    ap.add_argument("--study", nargs="*", metavar="WORKLOAD", default=None,
                    help="only run the named workloads (default: the 16k, 64k and 256k ones) "
                         "for their full simulated time: energy/momentum drift, massive-object "
                         "encounter diagnostics, and for mixed ones an FP64 rerun")
    ap.add_argument("--dt-div", type=int, default=1,
                    help="--study: divide the workload's dt by this (same simulated time)")
    ap.add_argument("--hermite", type=int, default=0, metavar="STEPS",
                    help="only time STEPS fourth-order Hermite steps of the workload")
    ap.add_argument("--ensemble", type=int, default=0, metavar="STEPS",
                    help="only time STEPS steps of the 256-system ensemble, batched and "
                         "system by system")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only copy a MIB-MiB buffer 5 times (HBM counter calibration)")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py: this library runs on one GPU only (no multi-GPU path); "
              "run with --gpus 1", file=sys.stderr)
        return 2

    import torch

    import paper_1801_07986_amd as pn
    from paper_1801_07986_amd import inputs

    if args.copy_calibration:
        return copy_calibration(torch, args.copy_calibration)
    pn.load()
    if args.study is not None:
        names = args.study or ["plummer_n16384_fp64", "plummer_n65536_mixed",
                               "plummer_n262144_mixed"]
        for name in names:
            print(json.dumps(study(pn, torch, inputs, name, args.dt_div)), flush=True)
        return 0
    if args.hermite:
        print(json.dumps(hermite(pn, torch, inputs, None, args.workload, None, args.hermite)),
              flush=True)
        return 0
    if args.table32:
        print(json.dumps(table32(pn, torch, inputs, args.samples, not args.no_cpu)), flush=True)
        return 0
    if args.ensemble:
        print(json.dumps(ensemble(pn, torch, inputs, torch.cuda.current_stream(), args.ensemble)),
              flush=True)
        return 0
    w = inputs.WORKLOADS[args.workload]
    N, c, eps, dt = w["N"], w["c"], w["eps"], w["dt"]
    prec = pn.PN_MIXED if w["precision"] == "mixed" else pn.PN_FP64
    G = 1.0
    log(f"workload {args.workload}: N={N} M_bh={w['M_bh']} c={c} eps={eps} dt={dt} "
        f"precision={w['precision']} steps={args.steps} warmup={args.warmup}")
    pos0, vel0, mass0 = inputs.plummer_bh(N, w["M_bh"], w["seed"])
    dev = torch.device("cuda:0")
    pos = torch.from_numpy(pos0).to(dev)
    vel = torch.from_numpy(vel0).to(dev)
    mass = torch.from_numpy(mass0).to(dev)
    stream = torch.cuda.current_stream()

    # warmup (also captures the step graph)
    pn.pn_step(pos, vel, mass, G, c, eps, dt, args.warmup, prec, stream=stream)
    torch.cuda.synchronize()
    log("warmup done")

    # timed region: exactly K steps
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    pn.pn_step(pos, vel, mass, G, c, eps, dt, args.steps, prec, stream=stream)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    wall = t1 - t0
    pairs = 4.0 * args.steps * float(N) * float(N)
    value = pairs / wall
    log(f"timed {args.steps} steps in {wall:.4f} s -> {value:.4e} pair/s")

    # dominant kernel: the fused pair sweep, timed per launch with HIP events
    # on the stream it runs on (direct launches, same kernels and shapes).  In
    # RK4 steps every sweep but a call's first is k_pair_bh (the sweep plus
    # one workgroup doing the previous stage's massive-object update)
    tsteps = max(2, min(25, args.steps))
    pn.pn_step(pos, vel, mass, G, c, eps, dt, tsteps, prec, stream=stream, flags=pn.PN_TIMING)
    tm = pn.pn_last_timing()
    avg_s = tm["total_ms"] / tm["launches"] / 1e3
    flops = FLOP_PER_PAIR_FUSED * tm["pairs_per_launch"]
    achieved = flops / avg_s
    peak = PEAK_FP64_VALU if prec == pn.PN_FP64 else PEAK_FP32_VALU
    ipt, ws, nsplit, _ = pn.pn_query_shape(prec, N)
    kname = f"k_pair_bh<{'double' if prec == pn.PN_FP64 else 'float'},3,{ipt},{ws}>"
    traffic = TRAFFIC_BYTES.get((args.workload, kname, nsplit))
    roofline = {"bound": "alu", "achieved": achieved / 1e12, "peak": peak / 1e12,
                "unit": "TFLOP/s", "frac": achieved / peak, "traffic": traffic,
                "kernel": kname, "nsplit": nsplit, "avg_launch_ms": avg_s * 1e3,
                "launches": tm["launches"],
                "flop_per_pair": FLOP_PER_PAIR_FUSED}
    log(f"pair kernel avg {avg_s * 1e3:.4f} ms over {tm['launches']} launches -> "
        f"{achieved / 1e12:.2f} TFLOP/s ({achieved / peak:.1%} of peak)")

    result = {
        "metric": "pair interactions/s (Newton+1PN)",
        "value": value,
        "unit": "pair/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if prec == pn.PN_FP64 else "f32+f64",
        "data": "synthetic (seeded Plummer sphere + black hole)",
        "config": {"workload": args.workload, "N": N, "M_bh": w["M_bh"], "c": c, "eps": eps,
                   "dt": dt, "integrator": "RK4", "precision": w["precision"],
                   "evals_per_step": 4, "pairs_per_eval": "N^2"},
        "roofline": roofline,
    }

    if not args.no_secondary:
        result["secondary"] = secondary(pn, torch, inputs, stream)
        result["hermite"] = hermite(pn, torch, inputs, stream, args.workload,
                                    result["ms_per_step"])
        result["eih"] = eih(pn, torch, inputs, stream)
        result["ensemble"] = ensemble(pn, torch, inputs, stream)

    if not args.no_cpu:
        result["cpu_baseline"] = cpu_baseline(pos0, vel0, mass0, G, c, eps)

    print(json.dumps(result), flush=True)
    return 0


def secondary(pn, torch, inputs, stream):
    """N = 65536 (M = 0.1, c = 30): mixed precision vs FP64, 10 RK4 steps each."""
    w = inputs.WORKLOADS["plummer_n65536_mixed"]
    N = w["N"]
    pos0, vel0, mass0 = inputs.plummer_bh(N, w["M_bh"], w["seed"])
    out = {"workload": "plummer_n65536", "N": N, "steps": 10}
    for name, prec in (("mixed", pn.PN_MIXED), ("fp64", pn.PN_FP64)):
        pos = torch.from_numpy(pos0).cuda()
        vel = torch.from_numpy(vel0).cuda()
        mass = torch.from_numpy(mass0).cuda()
        pn.pn_step(pos, vel, mass, 1.0, w["c"], w["eps"], w["dt"], 1, prec, stream=stream)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        pn.pn_step(pos, vel, mass, 1.0, w["c"], w["eps"], w["dt"], 10, prec, stream=stream)
        torch.cuda.synchronize()
        dt_wall = time.perf_counter() - t0
        out[name + "_pair_per_s"] = 4.0 * 10 * N * N / dt_wall
        log(f"secondary N={N} {name}: {out[name + '_pair_per_s']:.4e} pair/s")
    out["mixed_over_fp64"] = out["mixed_pair_per_s"] / out["fp64_pair_per_s"]
    return out


def study(pn, torch, inputs, workload, dt_div=1, chunks=10):
    """A workload run for its full simulated time (RK4, its precision; with
    dt_div > 1 at dt / dt_div and dt_div times the steps), in `chunks`
    pieces, recording after each the Eq. (7) energy error, Eq. (8) momentum
    change and the massive object's encounter diagnostics (nearest star, stars
    within 10 Schwarzschild radii, largest 1PN/Newton ratio of a
    massive-object pair); a mixed-precision workload is rerun in FP64 from
    the same state."""
    w = inputs.WORKLOADS[workload]
    N, c, eps = w["N"], w["c"], w["eps"]
    dt, steps = w["dt"] / dt_div, w["steps"] * dt_div
    pos0, vel0, mass0 = inputs.plummer_bh(N, w["M_bh"], w["seed"])
    mass = torch.from_numpy(mass0).cuda()
    r_close = 10.0 * 2.0 * w["M_bh"] / (c * c)
    out = {"workload": workload, "N": N, "steps": steps, "dt": dt, "t_end": steps * dt,
           "r_close_10_schwarzschild": r_close}

    def diag(pos, vel):
        d = pn.pn_diagnostics(pos, vel, mass, 1.0, c, eps)
        e = pn.pn_encounters(pos, vel, mass, 1.0, c, r_close)
        return {"E": d[0] + d[1], "E_N": d[0], "E_1PN": d[1],
                "P": [d[2] + d[5], d[3] + d[6], d[4] + d[7]],
                "min_r_bh": e["min_r_bh"], "nearest_to_bh": e["nearest_to_bh"],
                "n_within_10_rs": e["n_close_bh"],
                "max_bh_pair_1pn_ratio": e["max_bh_pair_1pn_ratio"],
                "most_relativistic": e["most_relativistic"], "min_r_pair": e["min_r_pair"]}

    psc = float(np.abs(mass0[:, None] * vel0).sum())
    precs = [w["precision"]] + (["fp64"] if w["precision"] == "mixed" else [])
    finals = {}
    for name in precs:
        prec = pn.PN_MIXED if name == "mixed" else pn.PN_FP64
        pos = torch.from_numpy(pos0).cuda()
        vel = torch.from_numpy(vel0).cuda()
        d0 = diag(pos, vel)
        hist, wall, done = [], 0.0, 0
        for k in range(chunks):
            n = steps * (k + 1) // chunks - done
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            pn.pn_step(pos, vel, mass, 1.0, c, eps, dt, n, prec)
            torch.cuda.synchronize()
            wall += time.perf_counter() - t0
            done += n
            d = diag(pos, vel)
            h = {"t": done * dt, "dE_rel": (d["E"] - d0["E"]) / abs(d0["E"]),
                 "min_r_bh": d["min_r_bh"], "nearest_to_bh": d["nearest_to_bh"],
                 "max_bh_pair_1pn_ratio": d["max_bh_pair_1pn_ratio"],
                 "most_relativistic": d["most_relativistic"]}
            hist.append(h)
            log(f"study {workload} {name} dt={dt:g}: t={h['t']:.4f} dE/E={h['dE_rel']:+.3e} "
                f"min_r_bh={h['min_r_bh']:.3e} ratio={h['max_bh_pair_1pn_ratio']:.3e} "
                f"(#{h['most_relativistic']})")
        r = {"wall_s": wall, "pair_per_s": 4.0 * steps * float(N) * float(N) / wall,
             "start": d0, "end": d, "dE_rel": (d["E"] - d0["E"]) / abs(d0["E"]),
             "dE_1PN_rel": (d["E_1PN"] - d0["E_1PN"]) / abs(d0["E"]),
             "dP_max_over_sum_m_abs_v": max(abs(a - b) for a, b in zip(d["P"], d0["P"])) / psc,
             "history": hist}
        out[name] = r
        finals[name] = (pos.cpu().numpy(), vel.cpu().numpy())
    if len(finals) == 2:
        (pm, vm), (pf, vf) = finals["mixed"], finals["fp64"]
        out["mixed_vs_fp64_end"] = {
            "max_abs_dx": float(np.abs(pm - pf).max()),
            "max_abs_dv": float(np.abs(vm - vf).max()),
            "dE_rel_difference": out["mixed"]["dE_rel"] - out["fp64"]["dE_rel"]}
    return out


def eih(pn, torch, inputs, stream, reps=20):
    """Unrestricted EIH evaluations (every pair at full 1PN order, two sweeps
    over all N bodies) of the N = 16384 and N = 65536 inputs: pair
    interactions (N^2 per evaluation) per second, FP64 and mixed, against the
    limited evaluation of the same input."""
    out = {}
    for name in ("plummer_n16384_fp64", "plummer_n65536_mixed"):
        w = inputs.WORKLOADS[name]
        N = w["N"]
        pos0, vel0, mass0 = inputs.plummer_bh(N, w["M_bh"], w["seed"])
        P, V, M = (torch.from_numpy(a).cuda() for a in (pos0, vel0, mass0))
        acc = torch.empty((N, 3), dtype=torch.float64, device="cuda")
        r = {"N": N}
        for pname, prec in (("fp64", pn.PN_FP64), ("mixed", pn.PN_MIXED)):
            for kind, fn in (("eih", pn.pn_accel_eih), ("limited", pn.pn_accel)):
                fn(P, V, M, 1.0, w["c"], w["eps"], prec, acc, stream=stream)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                for _ in range(reps):
                    fn(P, V, M, 1.0, w["c"], w["eps"], prec, acc, stream=stream,
                       flags=pn.PN_ASYNC)
                torch.cuda.synchronize()
                ms = (time.perf_counter() - t0) / reps * 1e3
                r[f"{kind}_{pname}_ms"] = ms
                r[f"{kind}_{pname}_pair_per_s"] = float(N) * N / (ms * 1e-3)
            log(f"eih N={N} {pname}: {r[f'eih_{pname}_ms']:.3f} ms/eval "
                f"(limited {r[f'limited_{pname}_ms']:.3f} ms)")
        out[name.split("_")[1]] = r
    return out


def hermite(pn, torch, inputs, stream, workload, rk4_ms, steps=50):
    """The same workload advanced by the fourth-order Hermite scheme (FP64):
    per step one FP64 evaluation and one dual-number jerk sweep."""
    w = inputs.WORKLOADS[workload]
    N = w["N"]
    pos0, vel0, mass0 = inputs.plummer_bh(N, w["M_bh"], w["seed"])
    pos = torch.from_numpy(pos0).cuda()
    vel = torch.from_numpy(vel0).cuda()
    mass = torch.from_numpy(mass0).cuda()
    pn.pn_step_hermite(pos, vel, mass, 1.0, w["c"], w["eps"], w["dt"], 2, stream=stream)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    pn.pn_step_hermite(pos, vel, mass, 1.0, w["c"], w["eps"], w["dt"], steps, stream=stream)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) / steps * 1e3
    log(f"hermite N={N}: {ms:.4f} ms/step")
    out = {"workload": workload, "N": N, "steps": steps, "ms_per_step": ms}
    if rk4_ms:
        out.update(rk4_ms_per_step=rk4_ms, hermite_over_rk4_time=ms / rk4_ms)
    return out


def ensemble(pn, torch, inputs, stream, steps=2):
    """256 independent Plummer + black-hole systems, N ~ U{1024..16384},
    M_bh ~ U[0.01, 0.1], c ~ U[20, 100]: pn_step_batched (one launch per phase
    for all systems, graph-captured step) vs the same systems stepped one
    after another with pn_step, FP64 and mixed."""
    systems = inputs.ensemble()
    ps, vs, ms, off = [], [], [], [0]
    for s in systems:
        p, v, m = inputs.plummer_bh(s["N"], s["M_bh"], s["seed"])
        ps.append(p)
        vs.append(v)
        ms.append(m)
        off.append(off[-1] + s["N"])
    pos0, vel0, mass0 = np.concatenate(ps), np.concatenate(vs), np.concatenate(ms)
    Gs = [1.0] * len(systems)
    cs = [s["c"] for s in systems]
    es = [s["eps"] for s in systems]
    pairs = 4.0 * steps * sum(float(s["N"]) ** 2 for s in systems)
    out = {"workload": "ensemble256", "n_sys": len(systems), "bodies": int(off[-1]),
           "steps": steps, "pairs_per_step": pairs / steps}
    for name, prec in (("fp64", pn.PN_FP64), ("mixed", pn.PN_MIXED)):
        pos = torch.from_numpy(pos0).cuda()
        vel = torch.from_numpy(vel0).cuda()
        mass = torch.from_numpy(mass0).cuda()
        pn.pn_step_batched(off, Gs, cs, es, pos, vel, mass, 1e-4, 1, prec, stream=stream)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        pn.pn_step_batched(off, Gs, cs, es, pos, vel, mass, 1e-4, steps, prec, stream=stream)
        torch.cuda.synchronize()
        tb = time.perf_counter() - t0
        out[f"batched_{name}_pair_per_s"] = pairs / tb
        log(f"ensemble batched {name}: {pairs / tb:.4e} pair/s")
        views = [(pos[off[k]:off[k + 1]], vel[off[k]:off[k + 1]], mass[off[k]:off[k + 1]])
                 for k in range(len(systems))]
        for k, (p, v, m) in enumerate(views):  # warm every system's graph
            pn.pn_step(p, v, m, 1.0, cs[k], es[k], 1e-4, 1, prec, stream=stream,
                       flags=pn.PN_ASYNC | pn.PN_NOGRAPH)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k, (p, v, m) in enumerate(views):
            pn.pn_step(p, v, m, 1.0, cs[k], es[k], 1e-4, steps, prec, stream=stream,
                       flags=pn.PN_ASYNC | pn.PN_NOGRAPH)
        torch.cuda.synchronize()
        ts = time.perf_counter() - t0
        out[f"sequential_{name}_pair_per_s"] = pairs / ts
        out[f"batched_over_sequential_{name}"] = ts / tb
        log(f"ensemble sequential {name}: {pairs / ts:.4e} pair/s")
    return out


def copy_calibration(torch, mib):
    """A plain device-to-device copy of known size, 5 times: the reference
    for scaling the HBM counters (FETCH_SIZE, WRITE_SIZE) of a PMC run."""
    n = mib * (1 << 20) // 8
    src = torch.rand(n, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    for _ in range(5):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes": n * 8, "copies": 5}), flush=True)
    return 0


# The paper's Table 3.2 (Sec. 3.2): elapsed time of 32 RK4 steps plus the total
# energy at the start and the end, mean and standard deviation of 10 samples,
# on an NVIDIA Tesla K20c and on one core of an Intel Core i7-3770K.  Context
# only (other hardware); the initial conditions of those runs are not stated.
PAPER_TABLE32 = {100: (1.5392, 0.1299, 0.3479, 0.0043), 300: (1.9651, 0.1308, 3.0501, 0.0060),
                 1000: (1.941, 0.1222, 33.652, 0.0881), 3000: (5.0517, 0.1284, 302.31, 0.10062),
                 10000: (38.934, 0.0100, 3358.6, 2.1313), 30000: (339.956, 0.1391, 30188, 17.482)}


def oracle_table32(oracle, pos0, vel0, mass0, samples, budget_s):
    """The oracle under the Table 3.2 protocol (energy, 32 RK4 steps of 2^-17,
    energy; its own RK4, four force evaluations per step): as many of
    `samples` runs as fit in budget_s (mean, standard deviation); when not
    even one fits, 128 evaluations + 2 energies scaled from one of each,
    labelled extrapolated."""
    dt = 2.0 ** -17
    t0 = time.perf_counter()
    oracle.accel(pos0, vel0, mass0, 1.0, 1.0, 1e-3)
    t_eval = time.perf_counter() - t0
    t0 = time.perf_counter()
    oracle.diagnostics(pos0, vel0, mass0, 1.0, 1.0, 1e-3)
    t_en = time.perf_counter() - t0
    est = 128 * t_eval + 2 * t_en
    k = int(min(samples, budget_s // est))
    if k < 1:
        return {"mean_s": est, "std_s": None, "runs": 0,
                "kind": "extrapolated: 128 x one force evaluation + 2 x one energy"}
    times = []
    for _ in range(k):
        t0 = time.perf_counter()
        oracle.diagnostics(pos0, vel0, mass0, 1.0, 1.0, 1e-3)
        oracle.step(pos0, vel0, mass0, 1.0, 1.0, 1e-3, dt, 32)
        oracle.diagnostics(pos0, vel0, mass0, 1.0, 1.0, 1e-3)
        times.append(time.perf_counter() - t0)
    return {"mean_s": float(np.mean(times)), "std_s": float(np.std(times)), "runs": k,
            "kind": f"measured: the protocol run {k} time(s)"}


def table32(pn, torch, inputs, samples, with_cpu, oracle_budget_s=40.0):
    """Table 3.2 protocol on this GPU: for each N, `samples` runs of (energy,
    32 RK4 steps, energy) on the paper's test model (cold shell 1 < r < 10,
    M = 100 m, c = G = 1, eps = 1e-3, dt = 2^-17), wall time from inputs on the
    GPU to the final energy on the host.  CPU leg: the oracle (one thread, as
    the paper's single core, and all threads) under the same protocol, up to
    `samples` runs within oracle_budget_s per N and thread count, else
    extrapolated from one evaluation (see oracle_table32)."""
    import oracle

    rows = []
    dt = 2.0 ** -17
    default_threads = oracle.max_threads()
    for N, paper in PAPER_TABLE32.items():
        pos0, vel0, mass0 = inputs.cold_sphere_bh(N - 1, seed=N)
        times = []
        for k in range(samples + 1):
            pos = torch.from_numpy(pos0).cuda()
            vel = torch.from_numpy(vel0).cuda()
            mass = torch.from_numpy(mass0).cuda()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            e0 = pn.pn_diagnostics(pos, vel, mass, 1.0, 1.0, 1e-3)
            pn.pn_step(pos, vel, mass, 1.0, 1.0, 1e-3, dt, 32, pn.PN_FP64)
            e1 = pn.pn_diagnostics(pos, vel, mass, 1.0, 1.0, 1e-3)
            t = time.perf_counter() - t0
            if k > 0:  # the first run captures the step graph
                times.append(t)
        row = {"N": N, "gpu_mean_s": float(np.mean(times)), "gpu_std_s": float(np.std(times)),
               "energy_rel_change": abs((e1[0] + e1[1]) - (e0[0] + e0[1])) / abs(e0[0] + e0[1]),
               "paper_k20c_mean_s": paper[0], "paper_k20c_std_s": paper[1],
               "paper_cpu1_mean_s": paper[2], "paper_cpu1_std_s": paper[3]}
        if with_cpu:
            for label, threads in (("cpu1", 1), ("cpu_all", default_threads)):
                oracle.set_threads(threads)
                r = oracle_table32(oracle, pos0, vel0, mass0, samples, oracle_budget_s)
                r["threads"] = oracle.max_threads()
                row[f"oracle_{label}"] = r
                log(f"table32 N={N} oracle {label} ({r['threads']} threads): {r['mean_s']:.3f} s "
                    f"({r['kind']})")
            oracle.set_threads(default_threads)
        rows.append(row)
        log(f"table32 N={N}: GPU {row['gpu_mean_s'] * 1e3:.2f} +- {row['gpu_std_s'] * 1e3:.2f} ms "
            f"(paper K20c {paper[0]} s, paper 1 core {paper[2]} s)")
    return {"protocol": "Table 3.2: 32 RK4 steps + energy at start and end", "samples": samples,
            "initial_conditions": "cold shell 1<r<10, M=100m, c=G=1, eps=1e-3, dt=2^-17",
            "oracle_budget_s_per_N_and_thread_count": oracle_budget_s, "rows": rows}


def cpu_baseline(pos, vel, mass, G, c, eps, budget_s=12.0):
    """The oracle (plain FP64 C, OpenMP over bodies) on this host's cores: full
    force evaluations of the same workload, repeated until ~budget_s."""
    import oracle

    oracle.build(force=False)
    threads = oracle.max_threads()
    N = len(mass)
    n_eval, t_used = 0, 0.0
    while t_used < budget_s and n_eval < 50:
        t0 = time.perf_counter()
        oracle.accel(pos, vel, mass, G, c, eps)
        t_used += time.perf_counter() - t0
        n_eval += 1
        log(f"cpu oracle eval {n_eval}: {t_used:.2f} s")
    # one thread: star rows of the same evaluation (each sums over all N bodies;
    # the massive object's row, an O(N^2) sum of its own, is left out)
    oracle.set_threads(1)
    rows = np.arange(1, N, 8, dtype=np.int64)
    n1, t1 = 0, 0.0
    while t1 < 4.0 and n1 < 20:
        t0 = time.perf_counter()
        oracle.accel_rows(pos, vel, mass, G, c, eps, rows)
        t1 += time.perf_counter() - t0
        n1 += 1
    oracle.set_threads(threads)
    one = n1 * float(len(rows)) * float(N) / t1
    log(f"cpu oracle, 1 thread: {one:.4e} pair/s")
    return {"value": n_eval * float(N) * float(N) / t_used, "unit": "pair/s", "cores": threads,
            "kind": "oracle",
            "sample": f"{n_eval} full force evaluation(s) of the N={N} workload "
                      f"({t_used:.1f} s, {threads} OpenMP threads)",
            "one_thread": {"value": one, "unit": "pair/s", "cores": 1,
                           "sample": f"{n1} x {len(rows)} star rows (every 8th) x {N} bodies "
                                     f"({t1:.1f} s)"}}


if __name__ == "__main__":
    sys.exit(main())
