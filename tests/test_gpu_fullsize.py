"""GPU parity at the full workload sizes (the benchmark's configurations).

- xi, 10^6 clustered points, weighted (the headline workload): binary64 (what
  both precision modes run by default) and the binary32 screen against the
  oracle over the whole catalogue.
- wp 2-D histogram, same generator: both precisions against the oracle.
- float32 cross count D(10^6) x R(10^7), non-periodic: the oracle on a random
  sample of D against all of R (the GPU counts the same sample against the
  same R grid), plus properties of the full count that hold at any size
  (binary32 == binary64; additivity over a split of D).
- 256 mocks of 2*10^5..2*10^6 points in one plan: binary32 == binary64 for
  every mock and every bin; the four smallest mocks against the oracle; every
  mock equal to its own single-call count (whose path the other parity tests
  pin to the oracle).
"""
import time
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

import oracle
from paper_1911_08275_amd import synth

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def native():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1911_08275_amd import native
    native.lib()
    return native


def test_headline_xi_weighted_full(native, monkeypatch):
    c = synth.config2()
    _say("headline xi weighted: oracle")
    t = time.time()
    ref = oracle.xi(c["cat"], c["edges"], periodic=True, box=420.0)
    _say(f"  oracle {time.time() - t:.1f}s")
    d = native.to_device(c["cat"])
    # binary64 (both modes by default), then the binary32 screen switched on
    for prec, screen in (("fp32", False), ("fp64", False), ("fp32", True)):
        if screen:
            monkeypatch.setenv("CP_XI_WEIGHTED_BINARY32", "1")
        g = native.countpairs_xi(d, c["edges"], precision=prec, periodic=True, boxsize=420.0,
                                 need_ravg=True)
        assert g.stats["precision"] == ("fp32" if screen else "fp64"), g.stats
        assert (g.npairs == ref.npairs).all(), (prec, g.npairs, ref.npairs)
        np.testing.assert_allclose(g.wsum, ref.wsum, rtol=1e-12, atol=0)
        np.testing.assert_allclose(g.ravg, ref.ravg, rtol=1e-12, atol=0)
        _say(f"  {prec} ok, rechecks {g.stats['rechecks']}, pair kernel "
             f"{g.stats['ms_pairs']:.3f} ms")


def test_headline_estimators(native):
    """xi(r) and w_p(r_p) of the 10^6-point Neyman-Scott catalogue from the GPU
    counts and the library's estimators (natural estimator, analytic random
    pairs of the periodic box, line-of-sight sum) against the generator's
    closed-form correlation function."""
    import math
    from neyman_scott import ns_tolerance, ns_wp, ns_xi
    c = synth.config2()
    n, parents, sigma, box = c["cat"].n, 20_000, 1.5, 420.0
    e = c["edges"]
    d = native.to_device(c["cat"])
    _say("headline estimators")
    g = native.countpairs_xi(d, e, precision="fp32", periodic=True, boxsize=box)
    rr = native.cp_rr_periodic_xi(n, box, e)
    xi = native.cp_xi_natural(g.npairs, rr)
    want = ns_xi(e, parents, sigma, box)
    vol = 4.0 / 3.0 * math.pi * (e[1:] ** 3 - e[:-1] ** 3)
    tol = ns_tolerance(want, rr, vol, parents, box)
    assert np.all(np.abs(xi - want) < tol), (xi, want, tol)
    pimax, npi = 40.0, 40
    g = native.countpairs_wp(d, e, pimax, npi, precision="fp32", periodic=True, boxsize=box)
    rr2 = native.cp_rr_periodic_wp(n, box, e, pimax, npi)
    wp = native.cp_wp_integrate(native.cp_xi_natural(g.npairs.reshape(rr2.shape), rr2), pimax)
    want = ns_wp(e, pimax, parents, sigma, box)
    vol = math.pi * (e[1:] ** 2 - e[:-1] ** 2) * 2 * pimax
    tol = 2 * pimax * ns_tolerance(want / (2 * pimax), rr2.sum(axis=1), vol, parents, box)
    assert np.all(np.abs(wp - want) < tol), (wp, want, tol)


def test_wp_full(native):
    c = synth.config3()
    _say("wp full: oracle")
    t = time.time()
    ref = oracle.wp(c["cat"], c["edges"], 40.0, 40, periodic=True, box=420.0)
    _say(f"  oracle {time.time() - t:.1f}s")
    d = native.to_device(c["cat"])
    for prec in ("fp32", "fp64"):
        g = native.countpairs_wp(d, c["edges"], 40.0, 40, precision=prec, periodic=True,
                                 boxsize=420.0)
        assert g.stats["precision"] == prec, g.stats
        assert (g.npairs == ref.npairs).all(), prec


def test_cross_full_sampled(native):
    c = synth.config4()
    rng = np.random.Generator(np.random.PCG64(77))
    idx = np.sort(rng.choice(c["d"].n, 20_000, replace=False))
    sub = c["d"].subset(idx)
    dr = native.to_device(c["r"])
    _say("cross sample: oracle")
    t = time.time()
    ref = oracle.xi(sub, c["edges"], periodic=False, other=c["r"])
    _say(f"  oracle {time.time() - t:.1f}s")
    for prec in ("fp32", "fp64"):
        g = native.countpairs_cross(native.to_device(sub), dr, c["edges"], precision=prec,
                                    periodic=False)
        assert g.stats["precision"] == prec, g.stats
        assert (g.npairs == ref.npairs).all(), prec
    # full size: binary32 == binary64, and counts add up over a split of D
    dd = native.to_device(c["d"])
    f32 = native.countpairs_cross(dd, dr, c["edges"], precision="fp32", periodic=False)
    f64 = native.countpairs_cross(dd, dr, c["edges"], precision="fp64", periodic=False)
    assert (f32.npairs == f64.npairs).all()
    half = c["d"].n // 2
    a = c["d"].subset(np.arange(half))
    b = c["d"].subset(np.arange(half, c["d"].n))
    ga = native.countpairs_cross(native.to_device(a), dr, c["edges"], periodic=False)
    gb = native.countpairs_cross(native.to_device(b), dr, c["edges"], periodic=False)
    assert (ga.npairs + gb.npairs == f32.npairs).all()


def test_batch_256_mocks(native):
    import torch
    specs = synth.mock_specs()
    with ThreadPoolExecutor(8) as ex:
        cats = list(ex.map(synth.mock, specs))
    _say(f"batch: {len(cats)} mocks, {sum(c.n for c in cats)} points")
    devs = [native.to_device(c) for c in cats]
    xe = synth.log_edges(0.1, 25.0, 14)
    res = {}
    for prec in ("fp32", "fp64"):
        plan = native.Plan(devs, xi_edges=xe, wp_edges=xe, pimax=40.0, npibins=40,
                           precision=prec, periodic=True, boxsize=420.0)
        plan.execute()
        res[prec] = plan.results()
        sx, sw = plan.stats()
        assert sx["precision"] == prec and sw["precision"] == prec, (sx, sw)
        plan.close()
        torch.cuda.synchronize()
    assert (res["fp32"][0] == res["fp64"][0]).all()
    assert (res["fp32"][1] == res["fp64"][1]).all()
    xi, wp = res["fp32"]
    order = np.argsort([c.n for c in cats])
    for m in order[:4]:
        _say(f"  mock {m} (n={cats[m].n}) vs oracle")
        assert (xi[m] == oracle.xi(cats[m], xe, True, 420.0).npairs).all()
        assert (wp[m] == oracle.wp(cats[m], xe, 40.0, 40, periodic=True, box=420.0).npairs).all()
    # every mock of the plan equals its own single call (a few ms each)
    _say("  every mock vs its single call")
    for m in range(len(devs)):
        s = native.countpairs_xi(devs[m], xe, periodic=True, boxsize=420.0)
        assert (s.npairs == xi[m]).all(), m
        s = native.countpairs_wp(devs[m], xe, 40.0, 40, periodic=True, boxsize=420.0)
        assert (s.npairs == wp[m]).all(), m
