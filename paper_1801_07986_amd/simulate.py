"""Run a system forward with periodic diagnostics and checkpoints.

Every ``--every`` time units it records (one JSON line each): the 1PN total
energy and momentum (Eqs. (7)-(8)) and the energy error relative to the start,
the star nearest to the massive object and how many stars lie within
``--close`` Schwarzschild radii (2GM/c^2) of it, and the nearest star-star
pair -- the quantities the paper follows for its test model (Sec. 4: energy
error, nearest binary, nearest star to the massive object) -- and the largest
1PN/Newtonian ratio of a massive-object/star pair (Eq. (5)).  All arithmetic
runs in libpn (pn_step, pn_diagnostics, pn_encounters).

Checkpoints (``--checkpoint PATH``) hold the FP64 state and the run's
parameters; ``--resume PATH`` continues a run exactly (the continuation is
bitwise identical to an uninterrupted run of the same chunks).

Example, the paper's test model (cold collapse, N = 10^4 stars, M = 100 m,
c = G = 1, eps = 1e-3, dt = 2^-15, to t = 10):

    python -m paper_1801_07986_amd.simulate --model cold --n-stars 10000 \\
        --dt-log2 -15 --t-end 10 --every 0.125 --out cold.jsonl
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np


def _log(msg):
    print(f"[simulate] {msg}", file=sys.stderr, flush=True)


def save_checkpoint(path, pos, vel, mass, meta):
    tmp = path + ".tmp.npz"
    np.savez(tmp, pos=pos.cpu().numpy(), vel=vel.cpu().numpy(), mass=mass.cpu().numpy(),
             meta=np.frombuffer(json.dumps(meta).encode(), dtype=np.uint8))
    os.replace(tmp, path)


def load_checkpoint(path):
    z = np.load(path, allow_pickle=False)
    meta = json.loads(bytes(z["meta"]).decode())
    return z["pos"], z["vel"], z["mass"], meta


def run(pos, vel, mass, *, G, c, eps, dt, t_end, every, precision, out_path, t0=0.0, step0=0,
        E_ref=None, close=10.0, checkpoint=None, meta=None, stream=None, integrator="rk4"):
    """Advance (pos, vel) [torch, on the GPU] from t0 to t_end; returns the last record.

    integrator "rk4" (pn_step, FP64 or mixed) or "hermite" (pn_step_hermite,
    FP64; each chunk between records starts the scheme afresh from the
    acceleration and jerk of its first state)."""
    import paper_1801_07986_amd as pn

    prec = pn.PN_MIXED if precision == "mixed" else pn.PN_FP64
    M = float(mass[0].item())
    r_s = 2.0 * G * M / (c * c) if math.isfinite(c) else 0.0
    chunk = max(1, int(round(every / dt)))
    total = int(round((t_end - t0) / dt))
    d0 = pn.pn_diagnostics(pos, vel, mass, G, c, eps, stream=stream)
    if E_ref is None:
        E_ref = d0[0] + d0[1]
    meta = dict(meta or {})
    meta.update(G=G, c=c, eps=eps, dt=dt, precision=precision, E_ref=E_ref, every=every,
                close=close, integrator=integrator)
    done, step, rec = 0, step0, None
    mode = "a" if step0 > 0 else "w"
    with open(out_path, mode) as f:
        while True:
            d = pn.pn_diagnostics(pos, vel, mass, G, c, eps, stream=stream)
            enc = pn.pn_encounters(pos, vel, mass, G, c, close * r_s, stream=stream)
            E = d[0] + d[1]
            rec = {"t": t0 + done * dt, "step": step, "E": E, "E_N": d[0], "E_1PN": d[1],
                   "dE_rel": abs(E - E_ref) / abs(E_ref), "P": [d[2] + d[5], d[3] + d[6],
                                                             d[4] + d[7]],
                   **enc, "r_schwarzschild": r_s, "wall": time.time()}
            rec["pair"] = list(rec["pair"])
            f.write(json.dumps(rec) + "\n")
            f.flush()
            _log(f"t={rec['t']:.5f} dE/E={rec['dE_rel']:.3e} min_r_bh={enc['min_r_bh']:.4e} "
                 f"n_close={enc['n_close_bh']} min_r_pair={enc['min_r_pair']:.3e} "
                 f"max_1pn_ratio={enc['max_bh_pair_1pn_ratio']:.3e}")
            if done >= total:
                break
            n = min(chunk, total - done)
            if integrator == "hermite":
                pn.pn_step_hermite(pos, vel, mass, G, c, eps, dt, n, stream=stream)
            else:
                pn.pn_step(pos, vel, mass, G, c, eps, dt, n, prec, stream=stream)
            done += n
            step += n
            if checkpoint:
                save_checkpoint(checkpoint, pos, vel, mass,
                                dict(meta, t=t0 + done * dt, step=step))
    return rec


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--model", choices=("cold", "plummer"), default="cold")
    ap.add_argument("--n-stars", type=int, default=10000)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--bh-mass", type=float, default=None,
                    help="plummer: black-hole mass (cold: 100 m, as in the paper)")
    ap.add_argument("--c", type=float, default=None,
                    help="speed of light (default 1; on --resume, the checkpoint's unless given: "
                         "a different c restarts the energy reference at the resumed state)")
    ap.add_argument("--eps", type=float, default=1e-3)
    ap.add_argument("--dt-log2", type=float, default=-15.0)
    ap.add_argument("--t-end", type=float, default=1.0)
    ap.add_argument("--every", type=float, default=0.125)
    ap.add_argument("--close", type=float, default=10.0, help="count radius in 2GM/c^2")
    ap.add_argument("--precision", choices=("fp64", "mixed"), default="fp64")
    ap.add_argument("--integrator", choices=("rk4", "hermite"), default=None,
                    help="default rk4; on --resume, the checkpoint's unless given")
    ap.add_argument("--out", required=True)
    ap.add_argument("--checkpoint", default=None)
    ap.add_argument("--resume", default=None)
    args = ap.parse_args(argv)

    import torch

    from paper_1801_07986_amd import inputs

    dt = 2.0 ** args.dt_log2
    t0, step0, E_ref = 0.0, 0, None
    if args.resume:
        pos, vel, mass, meta = load_checkpoint(args.resume)
        t0, step0, E_ref = meta["t"], meta["step"], meta["E_ref"]
        args.eps, dt = meta["eps"], meta["dt"]
        if args.c is None or args.c == meta["c"]:
            args.c = meta["c"]
        else:
            E_ref = None
            _log(f"c = {args.c} instead of the checkpoint's {meta['c']}: energy reference restarts")
        if args.integrator is None:
            args.integrator = meta.get("integrator", "rk4")
        _log(f"resuming from t={t0} (step {step0})")
    else:
        args.c = 1.0 if args.c is None else args.c
        if args.model == "cold":
            pos, vel, mass = inputs.cold_sphere_bh(args.n_stars, args.seed)
        else:
            pos, vel, mass = inputs.plummer_bh(args.n_stars + 1, args.bh_mass or 0.1, args.seed)
    dev = torch.device("cuda:0")
    P = torch.from_numpy(np.ascontiguousarray(pos)).to(dev)
    V = torch.from_numpy(np.ascontiguousarray(vel)).to(dev)
    Mm = torch.from_numpy(np.ascontiguousarray(mass)).to(dev)
    _log(f"model={args.model} N={len(mass)} dt={dt:g} c={args.c} eps={args.eps} "
         f"integrator={args.integrator or 'rk4'} t: {t0} -> {args.t_end}")
    rec = run(P, V, Mm, G=1.0, c=args.c, eps=args.eps, dt=dt, t_end=args.t_end,
              every=args.every, precision=args.precision, out_path=args.out, t0=t0, step0=step0,
              E_ref=E_ref, close=args.close, checkpoint=args.checkpoint,
              meta={"model": args.model, "n_stars": args.n_stars, "seed": args.seed},
              integrator=args.integrator or "rk4")
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
