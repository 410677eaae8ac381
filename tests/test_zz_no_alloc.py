"""pn_accel_noalloc (scratch in a fixed device array, no allocation) against
pn_accel on the same inputs, through the C ABI.

Calls in a row on one GPU, each smaller than the one before, so that a call
finds the array holding a larger call's contents.  Where the fixed scratch
holds pn_accel's own launch shape the outputs must be bitwise identical.
Where it needs fewer j-splits (N = 65536: pn_accel's partial sums would not
fit in 64 MiB) the two differ by summation order only, so each is held to
the accuracy target of its precision: FP64 per-body relative difference
<= 1e-12 (1PN part <= 1e-11); mixed within 1e-6 of pn_accel's FP64 result
per body, with the mixed floor of the parity tests (1e-6 of max(|a|, s / 2),
s the summed magnitude of the body's Newtonian pair terms: the FP32
pair-term rounding bound; 1PN part 3e-5 with the floor 1e-6 s), and within
twice that of pn_accel's mixed result.
"""
import numpy as np
import pytest

from paper_1801_07986_amd import inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

G, C, EPS = 1.0, 30.0, 1e-4


@pytest.fixture(scope="module")
def pn():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1801_07986_amd as pkg

    pkg.load()
    return pkg


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to("cuda:0")


def _run(fn, pos, vel, mass, precision):
    N = len(mass)
    aN = torch.full((N, 3), float("nan"), dtype=torch.float64, device="cuda:0")
    phi = torch.full((N,), float("nan"), dtype=torch.float64, device="cuda:0")
    a1 = torch.full((N, 3), float("nan"), dtype=torch.float64, device="cuda:0")
    fn(_dev(pos), _dev(vel), _dev(mass), G, C, EPS, precision, aN, phi, a1)
    torch.cuda.synchronize()
    return aN.cpu().numpy(), phi.cpu().numpy(), a1.cpu().numpy()


def _newton_scale(pos, mass):
    """s_i = sum_{b != i} G m_b / R_ib^2 (plain torch FP64 on the GPU: only the
    floor of the error metric)."""
    P, M = _dev(pos), _dev(mass)
    N = len(mass)
    out = np.empty(N)
    for k in range(0, N, 1024):
        d = P[k:k + 1024, None, :] - P[None, :, :]
        t = G * M[None, :] / ((d * d).sum(-1) + EPS * EPS)
        idx = torch.arange(k, min(N, k + 1024), device="cuda:0")
        t[idx - k, idx] = 0.0
        out[k:k + 1024] = t.sum(1).cpu().numpy()
    return out


def _rel(a, b, scale=None, floor=0.0):
    den = np.linalg.norm(b, axis=-1)
    if scale is not None:
        den = np.maximum(den, floor * scale)
    return np.linalg.norm(a - b, axis=-1) / den


def _check(pn, N, precision, seed, bitwise):
    print(f"[no-alloc] N={N} precision={precision} seed={seed}", flush=True)
    pos, vel, mass = inputs.plummer_bh(N, 0.1, seed)
    got = _run(pn.pn_accel_noalloc, pos, vel, mass, precision)
    ref = _run(pn.pn_accel, pos, vel, mass, precision)
    for g in got:
        assert np.isfinite(g).all()
    same = all(np.array_equal(g, r) for g, r in zip(got, ref))
    e_tot = _rel(got[0] + got[2], ref[0] + ref[2]).max()
    e_1pn = _rel(got[2], ref[2]).max()
    e_phi = (np.abs(got[1] - ref[1]) / np.abs(ref[1])).max()
    print(f"[no-alloc] N={N} precision={precision}: against pn_accel total {e_tot:.2e} "
          f"1PN {e_1pn:.2e} phi {e_phi:.2e} bitwise {same}", flush=True)
    if bitwise:
        assert same
    if precision == pn.PN_FP64:
        assert e_tot <= 1e-12 and e_phi <= 1e-12 and e_1pn <= 1e-11
    else:
        s = _newton_scale(pos, mass)
        m_tot = _rel(got[0] + got[2], ref[0] + ref[2], s, 0.5).max()
        ref64 = _run(pn.pn_accel, pos, vel, mass, pn.PN_FP64)
        f_tot = _rel(got[0] + got[2], ref64[0] + ref64[2], s, 0.5).max()
        f_1pn = _rel(got[2], ref64[2], s, 1e-6).max()
        f_phi = (np.abs(got[1] - ref64[1]) / np.abs(ref64[1])).max()
        print(f"[no-alloc] N={N} mixed: against pn_accel mixed {m_tot:.2e} (floor s / 2); against "
              f"the FP64 path total {f_tot:.2e} 1PN {f_1pn:.2e} phi {f_phi:.2e}", flush=True)
        assert m_tot <= 2e-6 and e_phi <= 2e-6
        assert f_tot <= 1e-6 and f_phi <= 1e-6 and f_1pn <= 3e-5


def test_no_alloc_matches_pn_accel_fp64(pn):
    # N = 65536: fewer splits than pn_accel's; N = 16384: the tuned shape's 32
    # splits fit (48 MB), bitwise; then a smaller call
    _check(pn, 65536, pn.PN_FP64, 70, bitwise=False)
    _check(pn, 16384, pn.PN_FP64, 71, bitwise=True)
    _check(pn, 3001, pn.PN_FP64, 72, bitwise=True)


def test_no_alloc_matches_pn_accel_mixed(pn):
    # N = 65536: fewer splits than pn_accel's (its partials would need more
    # than 64 MiB); then smaller calls in pn_accel's own shapes
    _check(pn, 65536, pn.PN_MIXED, 73, bitwise=False)
    _check(pn, 16384, pn.PN_MIXED, 74, bitwise=True)
    _check(pn, 1000, pn.PN_FP64, 75, bitwise=True)
