"""Jerk and fourth-order Hermite scheme of the HIP path against the oracle.

The GPU jerk is the exact derivative of the evaluated force along the motion
(dual numbers); the oracle's is exact to rounding too (complex-step
differentiation of its own force, pinned against closed forms and difference
quotients).  Bounds per body, relative to max(|j_ref|, 1e-3 s_j) with
s_j = sum_b G m_b |v_ib| / R_ib^3 the summed magnitude of the Newtonian pair
jerk terms: total jerk <= 1e-12; its 1PN part j(c) - j(inf) <= 1e-10
relative to max(|j1_ref|, 1e-6 s_j).  The Newtonian jerk (c = inf) also has
a closed form, checked to 1e-12.

Hermite trajectories against the oracle's scheme with exact jerks: positions
<= 1e-12 of the largest, velocities <= 1e-11 per body of the largest.
"""
import numpy as np
import pytest

import oracle
from paper_1801_07986_amd import inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

G = 1.0
TOL_JERK, TOL_JERK_1PN = 1e-12, 1e-10


@pytest.fixture(scope="module")
def pn():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1801_07986_amd as pkg

    pkg.load()
    return pkg


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to("cuda:0")


def host(t):
    return t.detach().cpu().numpy()


def case(N, seed, M=0.1):
    """Plummer sphere + massive object; for N = 2 (where the recentred sphere
    would put the one star on the massive object, at rest) a bound pair."""
    print(f"[case] N={N} seed={seed} M={M}", flush=True)
    if N == 2:
        pos = np.array([[0.0, 0.0, 0.0], [0.7, -0.2, 0.3]])
        vel = np.array([[0.0, 0.0, 0.0], [0.1, 0.45, -0.2]])
        return pos, vel, np.array([M, 1e-3])
    return inputs.plummer_bh(N, M, seed)


def pair_terms(pos, vel, eps, rows, chunk=256):
    """Softened separations of the given rows to all bodies, self-pairs masked."""
    for k in range(0, len(rows), chunk):
        r = rows[k:k + chunk]
        d = pos[r][:, None, :] - pos[None, :, :]
        dv = vel[r][:, None, :] - vel[None, :, :]
        R2 = (d * d).sum(-1) + eps * eps
        R2[np.arange(len(r)), r] = np.inf
        yield k, r, d, dv, R2


def scales(pos, vel, mass, eps, rows=None):
    """(s_a, s_j): summed magnitudes of the Newtonian pair acceleration and jerk terms."""
    rows = np.arange(len(mass)) if rows is None else np.asarray(rows)
    sa, sj = np.empty(len(rows)), np.empty(len(rows))
    for k, r, d, dv, R2 in pair_terms(pos, vel, eps, rows):
        sa[k:k + len(r)] = (G * mass[None, :] / R2).sum(1)
        sj[k:k + len(r)] = (G * mass[None, :] * np.linalg.norm(dv, axis=-1) / R2 ** 1.5).sum(1)
    return sa, sj


def newton_jerk_closed_form(pos, vel, mass, eps, rows=None):
    """Textbook Newtonian jerk with Plummer softening (for the given rows):
    j_i = -sum_b G m_b [v_ib / R^3 - 3 (x_ib . v_ib) x_ib / R^5],  R^2 = r^2 + eps^2."""
    rows = np.arange(len(mass)) if rows is None else np.asarray(rows)
    out = np.empty((len(rows), 3))
    for k, r, d, dv, R2 in pair_terms(pos, vel, eps, rows):
        R3 = R2 ** 1.5
        xv = (d * dv).sum(-1)
        t = dv / R3[..., None] - 3.0 * (xv / (R3 * R2))[..., None] * d
        out[k:k + len(r)] = -(G * mass[None, :, None] * t).sum(1)
    return out


def body_rel(a, b, scale, floor=1e-3):
    """Per-body relative error; a body whose reference and scale are both
    exactly zero must match exactly (error 0, else inf)."""
    num = np.linalg.norm(a - b, axis=-1)
    den = np.maximum(np.linalg.norm(b, axis=-1), floor * scale)
    out = np.where(num == 0.0, 0.0, np.inf)
    np.divide(num, den, out=out, where=den > 0)
    return out


def gpu_jerk(pn, pos, vel, mass, c, eps):
    N = len(mass)
    acc = torch.empty((N, 3), dtype=torch.float64, device="cuda:0")
    jerk = torch.empty((N, 3), dtype=torch.float64, device="cuda:0")
    pn.pn_jerk(dev(pos), dev(vel), dev(mass), G, c, eps, acc, jerk)
    return host(acc), host(jerk)


def jerk_errors(j, j0, rj, rj0, sj):
    """(total, 1PN part) per-body errors of the GPU jerks j (at c) and j0 (at
    c = inf) against the oracle's rj, rj0."""
    return body_rel(j, rj, sj), body_rel(j - j0, rj - rj0, sj, 1e-6)


@pytest.mark.parametrize("N", [2, 3, 17, 64, 257, 1000, 2049])
def test_jerk_fp64(pn, N):
    pos, vel, mass = case(N, 700 + N)
    c, eps = 30.0, 1e-4
    a, j = gpu_jerk(pn, pos, vel, mass, c, eps)
    _, j0 = gpu_jerk(pn, pos, vel, mass, float("inf"), eps)
    ra, rj = oracle.jerk_exact(pos, vel, mass, G, c, eps)
    _, rj0 = oracle.jerk_exact(pos, vel, mass, G, float("inf"), eps)
    sa, sj = scales(pos, vel, mass, eps)
    ea = body_rel(a, ra, sa).max()
    ej, ej1 = jerk_errors(j, j0, rj, rj0, sj)
    print(f"N={N}: acc {ea:.2e} jerk {ej.max():.2e} 1PN jerk {ej1.max():.2e}")
    assert ea <= 1e-12
    assert ej.max() <= TOL_JERK and ej1.max() <= TOL_JERK_1PN


@pytest.mark.parametrize("N", [2, 64, 1000])
def test_newtonian_jerk_closed_form(pn, N):
    """c = inf: the jerk is the softened Newtonian closed form, to rounding."""
    pos, vel, mass = case(N, 800 + N)
    eps = 1e-3
    _, j = gpu_jerk(pn, pos, vel, mass, float("inf"), eps)
    ref = newton_jerk_closed_form(pos, vel, mass, eps)
    _, sj = scales(pos, vel, mass, eps)
    e = body_rel(j, ref, sj).max()
    print(f"N={N}: closed form {e:.2e}")
    assert e <= 1e-12


@pytest.mark.parametrize("c", [1.0, 3.0, 30.0])
def test_jerk_1pn_part(pn, c):
    """j(c) - j(inf) against the oracle's, per body: the derivative of the
    1PN terms alone, from c = 1 (1PN terms of the Newtonian size) to c = 30."""
    N = 1000
    pos, vel, mass = case(N, 901)
    eps = 1e-4
    _, j = gpu_jerk(pn, pos, vel, mass, c, eps)
    _, j0 = gpu_jerk(pn, pos, vel, mass, float("inf"), eps)
    _, rj = oracle.jerk_exact(pos, vel, mass, G, c, eps)
    _, rj0 = oracle.jerk_exact(pos, vel, mass, G, float("inf"), eps)
    _, sj = scales(pos, vel, mass, eps)
    ej, ej1 = jerk_errors(j, j0, rj, rj0, sj)
    share = np.median(np.linalg.norm(rj - rj0, axis=1) / np.linalg.norm(rj, axis=1))
    print(f"c={c}: 1PN share of the jerk (median) {share:.1e}; errors: total {ej.max():.2e}, "
          f"1PN {ej1.max():.2e} (median {np.median(ej1):.2e})")
    assert ej.max() <= TOL_JERK and ej1.max() <= TOL_JERK_1PN


def test_jerk_nonfinite_reported(pn):
    pos, vel, mass = case(64, 902)
    pos[5] = pos[7]  # coincident stars without softening
    with pytest.raises(pn.PNError) as ei:
        gpu_jerk(pn, pos, vel, mass, 30.0, 0.0)
    assert ei.value.code == pn.PN_ENONFINITE


def test_hermite_trajectory_n1024(pn):
    """Plummer N = 1024 (M = 0.1, c = 50, eps = 1e-4): 20 Hermite steps of 1e-3."""
    pos, vel, mass = case(1024, 903)
    c, eps, dt, n = 50.0, 1e-4, 1e-3, 20
    P, V = dev(pos), dev(vel)
    pn.pn_step_hermite(P, V, dev(mass), G, c, eps, dt, n)
    rp, rv = oracle.hermite(pos, vel, mass, G, c, eps, dt, n)
    dp = np.abs(host(P) - rp).max() / np.abs(rp).max()
    dv = (np.linalg.norm(host(V) - rv, axis=1) / np.linalg.norm(rv, axis=1).max()).max()
    print(f"hermite trajectory: max |dx|/max|x| {dp:.3e}, max per-body |dv|/max|v| {dv:.3e}")
    assert dp <= 1e-12 and dv <= 1e-11


@pytest.mark.parametrize("N", [2, 3, 257])
def test_hermite_small(pn, N):
    pos, vel, mass = case(N, 904 + N)
    c, eps, dt, n = 30.0, 1e-3, 2e-3, 5
    P, V = dev(pos), dev(vel)
    pn.pn_step_hermite(P, V, dev(mass), G, c, eps, dt, n)
    rp, rv = oracle.hermite(pos, vel, mass, G, c, eps, dt, n)
    dp = np.abs(host(P) - rp).max() / np.abs(rp).max()
    dv = np.abs(host(V) - rv).max() / np.abs(rv).max()
    print(f"N={N} hermite: x {dp:.2e} v {dv:.2e}")
    assert dp <= 1e-12 and dv <= 1e-11


def test_hermite_fourth_order(pn):
    """Position errors at t = 0.25 fall ~16x per halving of dt (reference: 2560
    steps).  N = 64, M = 0.5, c = 3 (a strong velocity-dependent force),
    eps = 0.05: the oracle's scheme gives ratios 15.7 and 15.8 here."""
    pos, vel, mass = case(64, 905, M=0.5)
    c, eps, T = 3.0, 5e-2, 0.25
    m = dev(mass)

    def run(nsteps):
        P, V = dev(pos), dev(vel)
        pn.pn_step_hermite(P, V, m, G, c, eps, T / nsteps, nsteps)
        return host(P)

    ref = run(2560)
    errs = [np.abs(run(n) - ref).max() for n in (80, 160, 320)]
    ratios = [errs[0] / errs[1], errs[1] / errs[2]]
    print(f"errors {errs}, ratios {ratios}")
    assert all(12.0 <= r <= 20.0 for r in ratios)


def test_hermite_graph_equals_direct_launches(pn):
    pos, vel, mass = case(777, 906)
    outs = []
    for flags in (0, pn.PN_NOGRAPH):
        P, V = dev(pos), dev(vel)
        pn.pn_step_hermite(P, V, dev(mass), G, 40.0, 1e-4, 1e-3, 6, flags=flags)
        outs.append((host(P), host(V)))
    assert np.array_equal(outs[0][0], outs[1][0]) and np.array_equal(outs[0][1], outs[1][1])


def test_hermite_long_graph_equals_direct_launches(pn):
    """35 steps: two replays of the 16-step graph and three of the one-step
    graph, bitwise the same as direct launches."""
    pos, vel, mass = case(777, 908)
    outs = []
    for flags in (0, pn.PN_NOGRAPH):
        P, V = dev(pos), dev(vel)
        pn.pn_step_hermite(P, V, dev(mass), G, 40.0, 1e-4, 1e-4, 35, flags=flags)
        outs.append((host(P), host(V)))
    assert np.array_equal(outs[0][0], outs[1][0]) and np.array_equal(outs[0][1], outs[1][1])


def test_hermite_zero_is_noop_and_rk4_graph_survives(pn):
    pos, vel, mass = case(100, 907)
    P, V = dev(pos), dev(vel)
    pn.pn_step_hermite(P, V, dev(mass), G, 40.0, 1e-4, 1e-3, 0)
    assert np.array_equal(host(P), pos) and np.array_equal(host(V), vel)
    # alternating schemes on one state recaptures each step graph; results stay exact
    m = dev(mass)
    P1, V1 = dev(pos), dev(vel)
    pn.pn_step(P1, V1, m, G, 40.0, 1e-4, 1e-4, 3, 0)
    pn.pn_step_hermite(P1, V1, m, G, 40.0, 1e-4, 1e-4, 3)
    pn.pn_step(P1, V1, m, G, 40.0, 1e-4, 1e-4, 3, 0)
    rp, rv = oracle.step(pos, vel, mass, G, 40.0, 1e-4, 1e-4, 3)
    rp, rv = oracle.hermite(rp, rv, mass, G, 40.0, 1e-4, 1e-4, 3)
    rp, rv = oracle.step(rp, rv, mass, G, 40.0, 1e-4, 1e-4, 3)
    dp = np.abs(host(P1) - rp).max() / np.abs(rp).max()
    dv = np.abs(host(V1) - rv).max() / np.abs(rv).max()
    print(f"RK4 / Hermite / RK4: x {dp:.2e} v {dv:.2e}")
    assert dp <= 1e-12 and dv <= 1e-11


def test_full_size_n16384_jerk_and_hermite_step(pn):
    """N = 16384 Plummer (M = 0.05, c = 30, eps = 1e-4): acceleration and jerk
    against the oracle's exact jerk on the massive object, the 64 bodies with
    the largest jerk scale and 1024 random bodies (a star row costs the oracle
    O(N) after one evaluation, the massive object's O(N^2)); the Newtonian
    jerk (c = inf) on the same rows against its closed form.  Then one Hermite
    step of 1e-4 against the oracle's."""
    w = inputs.WORKLOADS["plummer_n16384_fp64"]
    pos, vel, mass = inputs.plummer_bh(w["N"], w["M_bh"], w["seed"])
    c, eps = w["c"], w["eps"]
    a, j = gpu_jerk(pn, pos, vel, mass, c, eps)
    _, j0 = gpu_jerk(pn, pos, vel, mass, float("inf"), eps)
    rows = np.arange(len(mass))
    _, sj_all = scales(pos, vel, mass, eps, rows)
    rng = np.random.default_rng(16384)
    rows = np.unique(np.concatenate([[0], np.argsort(sj_all)[-64:],
                                     rng.choice(len(mass), 1024, replace=False)]))
    print(f"[case] N=16384 oracle jerk rows ({len(rows)})", flush=True)
    ra, rj = oracle.jerk_exact(pos, vel, mass, G, c, eps, rows)
    _, rj0 = oracle.jerk_exact(pos, vel, mass, G, float("inf"), eps, rows)
    sa, sj = scales(pos, vel, mass, eps, rows)
    ea = body_rel(a[rows], ra, sa).max()
    ej, ej1 = jerk_errors(j[rows], j0[rows], rj, rj0, sj)
    ref0 = newton_jerk_closed_form(pos, vel, mass, eps, rows)
    e0 = body_rel(j0[rows], ref0, sj).max()
    print(f"N=16384: acc {ea:.2e}, jerk {ej.max():.2e} (massive object {ej[0]:.2e}), "
          f"1PN jerk {ej1.max():.2e}, Newtonian jerk vs closed form {e0:.2e}", flush=True)
    assert ea <= 1e-12 and ej.max() <= TOL_JERK and ej1.max() <= TOL_JERK_1PN and e0 <= 1e-12
    P, V = dev(pos), dev(vel)
    pn.pn_step_hermite(P, V, dev(mass), G, c, eps, w["dt"], 1)
    print("[case] N=16384 oracle Hermite step", flush=True)
    rp, rv = oracle.hermite(pos, vel, mass, G, c, eps, w["dt"], 1)
    dp = np.abs(host(P) - rp).max() / np.abs(rp).max()
    dv = np.abs(host(V) - rv).max() / np.abs(rv).max()
    print(f"N=16384 Hermite step: x {dp:.2e} v {dv:.2e}")
    assert dp <= 1e-14 and dv <= 1e-12
