"""pn_accel_noalloc (scratch in a fixed device array, no allocation) against
pn_accel on the same inputs, through the C ABI.

Two or three calls in a row on one GPU, each smaller than the one before, so
that a call finds the array holding a larger call's contents.  Where the
fixed scratch holds pn_accel's own launch shape the outputs must be bitwise
identical; where it needs fewer j-splits (the mixed N = 65536 case) they
differ by summation order only: per-body relative difference <= 1e-12 in
FP64, <= 1e-6 mixed (the accuracy targets of the two paths), 1PN part
<= 1e-11 / 1e-5.
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


def _rel(a, b):
    return np.linalg.norm(a - b, axis=-1) / np.linalg.norm(b, axis=-1)


def _check(pn, N, precision, seed, bitwise):
    print(f"[no-alloc] N={N} precision={precision} seed={seed}", flush=True)
    pos, vel, mass = inputs.plummer_bh(N, 0.1, seed)
    got = _run(pn.pn_accel_noalloc, pos, vel, mass, precision)
    ref = _run(pn.pn_accel, pos, vel, mass, precision)
    for g, r in zip(got, ref):
        assert np.isfinite(g).all()
    e_tot = _rel(got[0] + got[2], ref[0] + ref[2]).max()
    e_1pn = _rel(got[2], ref[2]).max()
    e_phi = (np.abs(got[1] - ref[1]) / np.abs(ref[1])).max()
    same = all(np.array_equal(g, r) for g, r in zip(got, ref))
    print(f"[no-alloc] N={N} precision={precision}: total {e_tot:.2e} 1PN {e_1pn:.2e} "
          f"phi {e_phi:.2e} bitwise {same}", flush=True)
    if bitwise:
        assert same
    tol, tol1 = (1e-12, 1e-11) if precision == 0 else (1e-6, 1e-5)
    assert e_tot <= tol and e_phi <= tol and e_1pn <= tol1


def test_no_alloc_matches_pn_accel_fp64(pn):
    # N = 16384: the tuned shape's 32 splits fit (48 MB); then a smaller call
    _check(pn, 16384, pn.PN_FP64, 71, bitwise=True)
    _check(pn, 3001, pn.PN_FP64, 72, bitwise=True)


def test_no_alloc_matches_pn_accel_mixed(pn):
    # N = 65536: fewer splits than pn_accel's (its partials would need 138 MB)
    _check(pn, 65536, pn.PN_MIXED, 73, bitwise=False)
    _check(pn, 16384, pn.PN_MIXED, 74, bitwise=True)
    _check(pn, 1000, pn.PN_FP64, 75, bitwise=True)
