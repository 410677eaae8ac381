"""Batched ensembles (pn_step_batched): every system advances exactly as it
would alone, whatever its neighbours in the batch.

Tolerances: FP64 positions/velocities within 1e-13 of the same system run
alone through pn_step (the two differ only in the summation order of the
j-splits) and within 1e-12 of the oracle; mixed within 1e-8 of the oracle's
positions.  Graph replay and direct launches agree bitwise; two runs agree
bitwise.
"""
import math

import numpy as np
import pytest

import oracle
from paper_1801_07986_amd import inputs

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

G = 1.0


@pytest.fixture(scope="module")
def pn():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1801_07986_amd as pkg

    pkg.load()
    return pkg


# (N, M_bh, c, eps, seed): uneven sizes, ragged tails, a Newtonian member (c = inf)
SYSTEMS = [(2, 0.1, 30.0, 1e-4, 1), (3, 0.05, 50.0, 1e-4, 2), (64, 0.1, 20.0, 1e-3, 3),
           (300, 0.02, 80.0, 1e-4, 4), (1000, 0.1, math.inf, 1e-4, 5), (2049, 0.07, 25.0, 1e-4, 6),
           (17, 0.1, 30.0, 0.0, 7)]


def build_ensemble(systems):
    ps, vs, ms, off = [], [], [], [0]
    for N, M, c, eps, seed in systems:
        p, v, m = inputs.plummer_bh(N, M, 500 + seed)
        ps.append(p)
        vs.append(v)
        ms.append(m)
        off.append(off[-1] + N)
    return np.concatenate(ps), np.concatenate(vs), np.concatenate(ms), off


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


def run_batched(pn, pos, vel, mass, off, systems, dt, steps, prec, flags=0):
    P, V = dev(pos), dev(vel)
    pn.pn_step_batched(off, [G] * len(systems), [s[2] for s in systems], [s[3] for s in systems],
                       P, V, dev(mass), dt, steps, prec, flags=flags)
    return P.cpu().numpy(), V.cpu().numpy()


@pytest.mark.parametrize("prec", [0, 1], ids=["fp64", "mixed"])
def test_batched_equals_each_system_alone(pn, prec):
    pos, vel, mass, off = build_ensemble(SYSTEMS)
    dt, steps = 1e-4, 3
    bp, bv = run_batched(pn, pos, vel, mass, off, SYSTEMS, dt, steps, prec)
    for k, (N, M, c, eps, seed) in enumerate(SYSTEMS):
        sl = slice(off[k], off[k + 1])
        print(f"[system] {k} N={N} c={c} eps={eps}", flush=True)
        P, V = dev(pos[sl]), dev(vel[sl])
        pn.pn_step(P, V, dev(mass[sl]), G, c, eps, dt, steps, prec)
        sp, sv = P.cpu().numpy(), V.cpu().numpy()
        rp, rv = oracle.step(pos[sl], vel[sl], mass[sl], G, c, eps, dt, steps)
        scale_p, scale_v = np.abs(rp).max(), np.abs(rv).max()
        if prec == 0:
            assert np.abs(bp[sl] - sp).max() <= 1e-13 * scale_p
            assert np.abs(bv[sl] - sv).max() <= 1e-13 * scale_v
            assert np.abs(bp[sl] - rp).max() <= 1e-12 * scale_p
            assert np.abs(bv[sl] - rv).max() <= 1e-12 * scale_v
        else:
            assert np.abs(bp[sl] - rp).max() <= 1e-8 * scale_p
            assert np.abs(bv[sl] - rv).max() <= 1e-6 * scale_v


def test_batched_graph_equals_direct_and_is_deterministic(pn):
    pos, vel, mass, off = build_ensemble(SYSTEMS)
    a = run_batched(pn, pos, vel, mass, off, SYSTEMS, 1e-4, 4, 0)
    b = run_batched(pn, pos, vel, mass, off, SYSTEMS, 1e-4, 4, 0, flags=pn.PN_NOGRAPH)
    c = run_batched(pn, pos, vel, mass, off, SYSTEMS, 1e-4, 4, 0)
    for x, y, z in zip(a, b, c):
        assert np.array_equal(x, y) and np.array_equal(x, z)


def step_alone_in_shape(pn, pos, vel, mass, c, eps, dt, steps, prec, ipt, ns):
    """pn_step of one system with the sweep shape forced to (ipt, 4 waves, ns)."""
    from paper_1801_07986_amd import _binding

    N = len(mass)
    pn.pn_set_shape(-1, 0, 0, 0, 0, 0)
    pn.pn_set_stage_kernel(-1, 0, 0, 0)  # the chained stages, whose sweep takes the shape
    pn.pn_set_shape(prec, N, N, ipt, 4, ns)
    try:
        P, V = dev(pos), dev(vel)
        pn.pn_step(P, V, dev(mass), G, c, eps, dt, steps, prec)
    finally:
        pn.pn_set_shape(-1, 0, 0, 0, 0, 0)
        _binding.install_tuned_shapes()
    return P.cpu().numpy(), V.cpu().numpy()


@pytest.mark.parametrize("prec", [0, 1], ids=["fp64", "mixed"])
@pytest.mark.parametrize("bshape", [(1, 0), (2, 0), (1, 3), (2, 5)],
                         ids=["ipt1_rule", "ipt2_rule", "ipt1_ns3", "ipt2_ns5"])
def test_batched_single_system_matches_pn_step_shape(pn, prec, bshape):
    """One system of N = 5000 in a batch of one, in each batched sweep shape
    (1 or 2 i per lane; the split rule or a forced count), against pn_step
    with the same shape (same i per lane, 4 wavefronts, same split count):
    bitwise."""
    from paper_1801_07986_amd import _binding

    N = 5000
    pos, vel, mass = inputs.plummer_bh(N, 0.1, 77)
    off = [0, N]
    pn.pn_set_batch_shape(prec, *bshape)
    try:
        ipt, splits = pn.pn_query_batch_shape(prec, off)
        assert ipt == bshape[0] and (bshape[1] == 0 or splits[0] == bshape[1])
        bp, bv = run_batched(pn, pos, vel, mass, off, [(N, 0.1, 30.0, 1e-4, 0)], 1e-4, 2, prec)
    finally:
        _binding.install_tuned_shapes()
    sp, sv = step_alone_in_shape(pn, pos, vel, mass, 30.0, 1e-4, 1e-4, 2, prec, ipt, splits[0])
    assert np.array_equal(bp, sp) and np.array_equal(bv, sv)


def test_batched_invalid_mass(pn):
    pos, vel, mass, off = build_ensemble(SYSTEMS[:3])
    mass[off[1]] = -1.0  # massive object of the second system
    with pytest.raises(pn.PNError) as e:
        run_batched(pn, pos, vel, mass, off, SYSTEMS[:3], 1e-4, 1, 0)
    assert e.value.code == pn.PN_EINVAL


def test_direct_call_of_another_ensemble_between_graph_replays(pn):
    """Graph replay of ensemble A, a direct-launch call of a smaller ensemble B
    (which rewrites the system descriptors in the shared batched scratch),
    then a replay of A with the same buffers: A must step exactly as before."""
    big, small = SYSTEMS[2:6], SYSTEMS[:3]
    pos, vel, mass, off = build_ensemble(big)
    P, V, Mm = dev(pos), dev(vel), dev(mass)
    Gs, cs, es = [G] * len(big), [s[2] for s in big], [s[3] for s in big]

    def step_big(flags):
        P.copy_(dev(pos))
        V.copy_(dev(vel))
        pn.pn_step_batched(off, Gs, cs, es, P, V, Mm, 1e-4, 2, 0, flags=flags)
        return P.cpu().numpy(), V.cpu().numpy()

    ref = step_big(pn.PN_NOGRAPH)
    first = step_big(0)  # captures A's step graph
    p2, v2, m2, off2 = build_ensemble(small)
    run_batched(pn, p2, v2, m2, off2, small, 1e-4, 2, 0, flags=pn.PN_NOGRAPH)
    again = step_big(0)  # same key as the cached graph
    for x, y, z in zip(ref, first, again):
        assert np.array_equal(x, y) and np.array_equal(x, z)


@pytest.fixture(scope="module")
def ensemble256():
    """The benchmark's ensemble: 256 systems, N ~ U{1024..16384},
    M ~ U[0.01, 0.1], c ~ U[20, 100], eps = 1e-4, system b seeded 10000 + b."""
    systems = inputs.ensemble()
    ps, vs, ms, off = [], [], [], [0]
    for s in systems:
        p, v, m = inputs.plummer_bh(s["N"], s["M_bh"], s["seed"])
        ps.append(p)
        vs.append(v)
        ms.append(m)
        off.append(off[-1] + s["N"])
    return systems, np.concatenate(ps), np.concatenate(vs), np.concatenate(ms), off


@pytest.mark.timeout(300)
@pytest.mark.parametrize("prec", [0, 1], ids=["fp64", "mixed"])
def test_ensemble256_members_equal_pn_step(pn, ensemble256, prec):
    """One batched RK4 step of the whole 256-system ensemble in its tuned shape;
    eight members (the largest, the second largest, the median, the two
    smallest, and three seeded random ones; the largest and the smallest are
    the first and the last in the plan's order of decreasing N) bitwise
    against pn_step of the member alone in the batched plan's shape (its i per
    lane, 4 wavefronts, the member's split count); the two smallest against
    the oracle's RK4 step too."""
    systems, pos, vel, mass, off = ensemble256
    Ns = np.array([s["N"] for s in systems])
    ipt, splits = pn.pn_query_batch_shape(prec, off)
    cs = [s["c"] for s in systems]
    print(f"[case] ensemble of {len(systems)}, {off[-1]} bodies, precision {prec}, "
          f"{ipt} i per lane, split counts {sorted(set(splits))}", flush=True)
    bp, bv = run_batched(pn, pos, vel, mass, off, [(s["N"], s["M_bh"], s["c"], s["eps"], 0)
                                                   for s in systems], 1e-4, 1, prec)
    order = np.argsort(-Ns, kind="stable")  # the plan's order: decreasing N
    rng = np.random.default_rng(256)
    pick = [order[0], order[1], order[len(order) // 2], order[-2], order[-1]]
    pick += [int(k) for k in rng.choice(np.setdiff1d(np.arange(len(systems)), pick), 3,
                                         replace=False)]
    worst = 0.0
    for k in pick:
        N, c = int(Ns[k]), cs[k]
        sl = slice(off[k], off[k + 1])
        print(f"[system] {k} N={N} c={c:.1f} splits={splits[k]}", flush=True)
        sp, sv = step_alone_in_shape(pn, pos[sl], vel[sl], mass[sl], c, 1e-4, 1e-4, 1, prec, ipt,
                                     splits[k])
        assert np.array_equal(bp[sl], sp) and np.array_equal(bv[sl], sv)
        if k in (order[-1], order[-2]):
            rp, rv = oracle.step(pos[sl], vel[sl], mass[sl], G, c, 1e-4, 1e-4, 1)
            dp = np.abs(bp[sl] - rp).max() / np.abs(rp).max()
            dv = np.abs(bv[sl] - rv).max() / np.abs(rv).max()
            print(f"  against the oracle: x {dp:.2e} v {dv:.2e}")
            worst = max(worst, dp)
            if prec == 0:
                assert dp <= 1e-12 and dv <= 1e-12
            else:
                assert dp <= 1e-8 and dv <= 1e-6
