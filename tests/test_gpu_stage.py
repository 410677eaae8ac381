"""pn_step's one-launch Runge-Kutta stages (k_stage) for small systems,
forced with pn_set_stage_kernel for every size and 2, 4, 8 or 16 stars per
workgroup, through the C ABI.

Against the oracle (classical RK4 on Eqs. (1)-(6), FP64): three steps of
ragged systems N = 2 ... 1000 within 1e-12 (positions, relative to the
largest) and 1e-12 (velocities, per body against the largest) in FP64,
1e-8 / 1e-6 mixed, the bounds of the chained stages in the shape tests; and
100 steps of the N = 1024 workload as its trajectory test holds the chained
stages.  Bitwise: the same call twice, graph replay against direct launches, a
run split over two calls or over single steps against one call.  Device-side
checks: a non-positive mass of the massive object and a non-finite
acceleration are reported as by the chained stages.
"""
import numpy as np
import pytest

import oracle
from paper_1801_07986_amd import inputs

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

G, C, EPS, DT = 1.0, 30.0, 1e-4, 1e-4
NS = (2, 4, 8, 16)


@pytest.fixture(scope="module")
def pn():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1801_07986_amd as pkg

    pkg.load()
    return pkg


@pytest.fixture
def stage(pn):
    """Force the one-launch stages with ns stars per workgroup at every size;
    the tuned table is restored afterwards."""
    from paper_1801_07986_amd import _binding

    def force(ns):
        pn.pn_set_stage_kernel(-1, 0, 0, 0)
        for prec in (pn.PN_FP64, pn.PN_MIXED):
            pn.pn_set_stage_kernel(prec, 2, 1 << 28, ns)

    yield force
    _binding.install_tuned_shapes()


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to("cuda:0")


def step(pn, pos, vel, mass, n, prec, flags=0, c=C, eps=EPS):
    P, V = dev(pos), dev(vel)
    pn.pn_step(P, V, dev(mass), G, c, eps, DT, n, prec, flags=flags)
    torch.cuda.synchronize()
    return P.cpu().numpy(), V.cpu().numpy()


@pytest.mark.parametrize("prec", [0, 1], ids=["fp64", "mixed"])
@pytest.mark.parametrize("N", [2, 3, 17, 100, 257, 1000])
def test_stage_parity(pn, stage, N, prec):
    if N == 2:  # a bound pair (the one-star sphere would sit on the massive object)
        pos = np.array([[0.0, 0.0, 0.0], [1.0, 0.2, -0.1]])
        vel = np.array([[0.0, -0.001, 0.0], [0.0, 0.3, 0.05]])
        mass = np.array([0.1, 0.001])
    else:
        pos, vel, mass = inputs.plummer_bh(N, 0.1, 500 + N)
    rp, rv = oracle.step(pos, vel, mass, G, C, EPS, DT, 3)
    for ns in NS:
        stage(ns)
        assert pn.pn_query_stage_kernel(prec, N) == ns
        print(f"[case] N={N} prec={prec} ns={ns}", flush=True)
        gp, gv = step(pn, pos, vel, mass, 3, prec)
        dp = np.abs(gp - rp).max() / np.abs(rp).max()
        dv = (np.linalg.norm(gv - rv, axis=1) / np.linalg.norm(rv, axis=1).max()).max()
        print(f"N={N} prec={prec} ns={ns}: x {dp:.2e} v {dv:.2e}", flush=True)
        if prec == 0:
            assert dp <= 1e-12 and dv <= 1e-12
        else:
            assert dp <= 1e-8 and dv <= 1e-6


@pytest.mark.parametrize("prec", [0, 1], ids=["fp64", "mixed"])
def test_stage_trajectory_n1024(pn, stage, prec):
    """The N = 1024 workload (M = 0.1, c = 50), 100 RK4 steps, 4 stars per
    workgroup, against the oracle's trajectory."""
    w = inputs.WORKLOADS["plummer_n1024_fp64"]
    pos, vel, mass = inputs.plummer_bh(w["N"], w["M_bh"], w["seed"])
    stage(4)
    P, V = dev(pos), dev(vel)
    pn.pn_step(P, V, dev(mass), G, w["c"], w["eps"], w["dt"], w["steps"], prec)
    rp, rv = oracle.step(pos, vel, mass, G, w["c"], w["eps"], w["dt"], w["steps"])
    gp, gv = P.cpu().numpy(), V.cpu().numpy()
    dp = np.abs(gp - rp).max() / np.abs(rp).max()
    dv = (np.linalg.norm(gv - rv, axis=1) / np.linalg.norm(rv, axis=1).max()).max()
    print(f"prec={prec} stage trajectory: x {dp:.3e}, v {dv:.3e}")
    if prec == 0:
        assert dp <= 1e-12 and dv <= 1e-10
    else:
        assert dp <= 1e-8 and dv <= 1e-6


@pytest.mark.parametrize("prec", [0, 1], ids=["fp64", "mixed"])
@pytest.mark.parametrize("N,ns", [(100, 2), (257, 4), (1000, 8), (2049, 16)])
def test_stage_bitwise(pn, stage, N, ns, prec):
    stage(ns)
    pos, vel, mass = inputs.plummer_bh(N, 0.1, 7)
    print(f"[case] bitwise N={N} ns={ns} prec={prec}", flush=True)
    a = step(pn, pos, vel, mass, 6, prec)
    b = step(pn, pos, vel, mass, 6, prec)
    d = step(pn, pos, vel, mass, 6, prec, flags=pn.PN_NOGRAPH)
    p2, v2 = step(pn, pos, vel, mass, 2, prec)
    r = step(pn, p2, v2, mass, 4, prec)
    s = step(pn, pos, vel, mass, 1, prec)
    for _ in range(5):
        s = step(pn, s[0], s[1], mass, 1, prec)
    same = lambda x, y: np.array_equal(x[0], y[0]) and np.array_equal(x[1], y[1])  # noqa: E731
    print(f"N={N} ns={ns} prec={prec}: repeat {same(a, b)}, direct {same(a, d)}, "
          f"2 + 4 {same(a, r)}, 6 x 1 {same(a, s)}")
    assert same(a, b) and same(a, d) and same(a, r) and same(a, s)


@pytest.mark.parametrize("prec", [0, 1], ids=["fp64", "mixed"])
def test_stage_long_graph_bitwise(pn, stage, prec):
    """41 steps: the first direct, then two replays of the 16-step graph and
    eight of the one-step graph; the same as direct launches and as 20 + 21."""
    stage(4)
    pos, vel, mass = inputs.plummer_bh(100, 0.1, 8)
    a = step(pn, pos, vel, mass, 41, prec)
    d = step(pn, pos, vel, mass, 41, prec, flags=pn.PN_NOGRAPH)
    p2, v2 = step(pn, pos, vel, mass, 20, prec)
    r = step(pn, p2, v2, mass, 21, prec)
    same = lambda x, y: np.array_equal(x[0], y[0]) and np.array_equal(x[1], y[1])  # noqa: E731
    print(f"prec={prec}: direct {same(a, d)}, 20 + 21 {same(a, r)}")
    assert same(a, d) and same(a, r)


def test_stage_device_checks(pn, stage):
    stage(4)
    pos, vel, mass = inputs.plummer_bh(64, 0.1, 14)
    bad = mass.copy()
    bad[0] = 0.0
    with pytest.raises(pn.PNError) as e:
        step(pn, pos, vel, bad, 2, pn.PN_FP64)
    assert e.value.code == pn.PN_EINVAL
    pos[5] = pos[9]  # two coincident stars without softening
    with pytest.raises(pn.PNError) as e:
        step(pn, pos, vel, mass, 2, pn.PN_FP64, eps=0.0)
    assert e.value.code == pn.PN_ENONFINITE
