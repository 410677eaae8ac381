"""Every launch shape of the sweep, forced with pn_set_shape: 1 or 2 i-bodies
per lane, 1, 4 or 8 wavefronts per i-range, the default or an odd split count,
in both precisions.  Each shape runs one evaluation (pn_accel: k_pair) and
three RK4 steps (pn_step: the chained k_epilogue_chain / k_pair_bh sequence)
on a ragged N = 1000 system, against the oracle; in FP64 also the two-pass
entry points (pn_potential_accel, then pn_correction on its outputs: the
MODE_P1 and MODE_P2 sweeps).  The tuned table only ever
picks some of these shapes, so without this the others would not run on the
GPU.

Bounds as in the parity tests: FP64 per-body total within 1e-12 (floor 1e-3
of the summed Newtonian term magnitude), three steps within 1e-12 of the
oracle's; mixed total within 1e-6 (floor s / 2, the FP32 pair-term rounding
bound of the parity tests), three steps within 1e-8 (positions) and
1e-6 (velocities, per body against the largest) of the oracle's.
"""
import numpy as np
import pytest

import oracle
from paper_1801_07986_amd import inputs

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

G = 1.0
N, M_BH, C, EPS, DT = 1000, 0.1, 30.0, 1e-4, 1e-4
SHAPES = [(ipt, ws, ns) for ipt in (1, 2) for ws in (1, 4, 8) for ns in (0, 3)]


@pytest.fixture(scope="module")
def pn():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1801_07986_amd as pkg

    pkg.load()
    return pkg


@pytest.fixture(scope="module")
def system():
    pos, vel, mass = inputs.plummer_bh(N, M_BH, 910)
    ref = oracle.accel(pos, vel, mass, G, C, EPS)
    step = oracle.step(pos, vel, mass, G, C, EPS, DT, 3)
    d = pos[:, None, :] - pos[None, :, :]
    R2 = (d * d).sum(-1) + EPS * EPS
    np.fill_diagonal(R2, np.inf)
    scale = (G * mass[None, :] / R2).sum(1)
    return pos, vel, mass, ref, step, scale


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to("cuda:0")


def rel(a, b, s, floor=1e-3):
    return (np.linalg.norm(a - b, axis=-1) / np.maximum(np.linalg.norm(b, axis=-1), floor * s)).max()


@pytest.mark.parametrize("prec", [0, 1], ids=["fp64", "mixed"])
@pytest.mark.parametrize("shape", SHAPES, ids=[f"ipt{a}_ws{b}_ns{c}" for a, b, c in SHAPES])
def test_every_shape(pn, system, shape, prec):
    from paper_1801_07986_amd import _binding

    pos, vel, mass, (rN, rphi, r1), (rp, rv), scale = system
    print(f"[case] shape {shape} precision {prec}", flush=True)
    pn.pn_set_shape(-1, 0, 0, 0, 0, 0)
    pn.pn_set_stage_kernel(-1, 0, 0, 0)  # the chained stages, whose sweep takes the shape
    pn.pn_set_shape(prec, 2, 1 << 30, *shape)
    try:
        assert tuple(pn.pn_query_shape(prec, N)[:2]) == shape[:2]
        aN = torch.empty((N, 3), dtype=torch.float64, device="cuda:0")
        a1 = torch.empty_like(aN)
        phi = torch.empty(N, dtype=torch.float64, device="cuda:0")
        pn.pn_accel(dev(pos), dev(vel), dev(mass), G, C, EPS, prec, aN, phi, a1)
        if prec == 0:
            bN = torch.empty_like(aN)
            b1 = torch.empty_like(aN)
            bphi = torch.empty_like(phi)
            pn.pn_potential_accel(dev(pos), None, dev(mass), G, C, EPS, bN, bphi)
            pn.pn_correction(dev(pos), dev(vel), dev(mass), G, C, EPS, bphi, bN, b1)
        P, V = dev(pos), dev(vel)
        pn.pn_step(P, V, dev(mass), G, C, EPS, DT, 3, prec)
    finally:
        pn.pn_set_shape(-1, 0, 0, 0, 0, 0)
        _binding.install_tuned_shapes()
    e = rel(aN.cpu().numpy() + a1.cpu().numpy(), rN + r1, scale, 1e-3 if prec == 0 else 0.5)
    gp, gv = P.cpu().numpy(), V.cpu().numpy()
    dp = np.abs(gp - rp).max() / np.abs(rp).max()
    dv = (np.linalg.norm(gv - rv, axis=1) / np.linalg.norm(rv, axis=1).max()).max()
    print(f"evaluation {e:.2e}, three steps: x {dp:.2e}, v {dv:.2e}")
    if prec == 0:
        eN = rel(bN.cpu().numpy(), rN, scale)
        e1 = rel(b1.cpu().numpy(), r1, scale, 1e-6)
        ephi = (np.abs(bphi.cpu().numpy() - rphi) / np.abs(rphi)).max()
        print(f"two-pass: a^N {eN:.2e}, phi {ephi:.2e}, 1PN part {e1:.2e}")
        assert eN <= 1e-12 and ephi <= 1e-12 and e1 <= 1e-11
        assert e <= 1e-12 and dp <= 1e-12 and dv <= 1e-12
    else:
        assert e <= 1e-6 and dp <= 1e-8 and dv <= 1e-6


TINY = [(n, s) for n in (3, 17, 70) for s in ((1, 8, 1), (2, 8, 1), (1, 8, 0), (2, 4, 1))]


@pytest.mark.parametrize("prec", [0, 1], ids=["fp64", "mixed"])
@pytest.mark.parametrize("n,shape", TINY, ids=[f"n{n}_ipt{a}_ws{b}_ns{c}" for n, (a, b, c) in TINY])
def test_tiny_systems_in_wide_shapes(pn, n, shape, prec):
    """Systems smaller than a workgroup's i-range and j-ranges shorter than
    its wavefronts (some wavefronts get no j at all) in the 8-wavefront
    shapes: one evaluation and three RK4 steps against the oracle."""
    from paper_1801_07986_amd import _binding

    pos, vel, mass = inputs.plummer_bh(n, M_BH, 920 + n)
    rN, rphi, r1 = oracle.accel(pos, vel, mass, G, C, EPS)
    rp, rv = oracle.step(pos, vel, mass, G, C, EPS, DT, 3)
    d = pos[:, None, :] - pos[None, :, :]
    R2 = (d * d).sum(-1) + EPS * EPS
    np.fill_diagonal(R2, np.inf)
    scale = (G * mass[None, :] / R2).sum(1)
    print(f"[case] N={n} shape {shape} precision {prec}", flush=True)
    pn.pn_set_shape(-1, 0, 0, 0, 0, 0)
    pn.pn_set_stage_kernel(-1, 0, 0, 0)
    pn.pn_set_shape(prec, 2, 1 << 30, *shape)
    try:
        assert tuple(pn.pn_query_shape(prec, n)[:2]) == shape[:2]
        aN = torch.empty((n, 3), dtype=torch.float64, device="cuda:0")
        a1 = torch.empty_like(aN)
        phi = torch.empty(n, dtype=torch.float64, device="cuda:0")
        pn.pn_accel(dev(pos), dev(vel), dev(mass), G, C, EPS, prec, aN, phi, a1)
        P, V = dev(pos), dev(vel)
        pn.pn_step(P, V, dev(mass), G, C, EPS, DT, 3, prec)
    finally:
        pn.pn_set_shape(-1, 0, 0, 0, 0, 0)
        _binding.install_tuned_shapes()
    e = rel(aN.cpu().numpy() + a1.cpu().numpy(), rN + r1, scale, 1e-3 if prec == 0 else 0.5)
    ephi = (np.abs(phi.cpu().numpy() - rphi) / np.abs(rphi)).max()
    gp, gv = P.cpu().numpy(), V.cpu().numpy()
    dp = np.abs(gp - rp).max() / np.abs(rp).max()
    dv = (np.linalg.norm(gv - rv, axis=1) / np.linalg.norm(rv, axis=1).max()).max()
    print(f"N={n} {shape}: evaluation {e:.2e}, phi {ephi:.2e}, three steps: x {dp:.2e}, v {dv:.2e}")
    if prec == 0:
        assert e <= 1e-12 and ephi <= 1e-12 and dp <= 1e-12 and dv <= 1e-12
    else:
        assert e <= 1e-6 and ephi <= 1e-6 and dp <= 1e-8 and dv <= 1e-6
