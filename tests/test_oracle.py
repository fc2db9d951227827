"""Pins for the CPU FP64 oracle (no GPU).

Each test checks the oracle against something other than itself: exact integer
arithmetic on lattice inputs, hand-derived worked examples, closed-form totals,
the analytic expectation for uniform points, exact identities between auto and
cross counts, and high-precision (mpmath) sums for the weighted mean separation.
"""
import json
import math
import os

import mpmath
import numpy as np
import pytest

import oracle
from paper_1911_08275_amd import synth

HERE = os.path.dirname(os.path.abspath(__file__))


# ----------------------------------------------------------- worked examples

def _golden_cases():
    with open(os.path.join(HERE, "golden", "worked_examples.json")) as f:
        return json.load(f)["cases"]


@pytest.mark.parametrize("case", _golden_cases(), ids=lambda c: c["name"])
@pytest.mark.parametrize("grid", [False, True])
def test_worked_examples(case, grid):
    p = np.array(case["points"], dtype=np.float64)
    w = np.array(case["weights"]) if "weights" in case else None
    mode = oracle.XI if case["mode"] == "xi" else oracle.WP
    r = oracle.count(mode, p[:, 0], p[:, 1], p[:, 2], w, edges=case["edges"],
                     periodic=case["periodic"], box=case["box"],
                     pimax=case.get("pimax", 0.0), npibins=case.get("npibins", 1), grid=grid)
    assert r.npairs.tolist() == case["npairs"]
    if "wsum" in case:
        assert r.wsum.tolist() == case["wsum"]
        assert r.wrsum.tolist() == case["wrsum"]


# ------------------------------------------------------ exact lattice pins

Q = 2.0 ** -6                       # lattice quantum: all arithmetic below is exact
LQ = int(420.0 / Q)                 # box side in quanta (26880)
EDGE_M = [3, 16, 40, 65, 100, 160, 255, 400, 640, 1000, 1600, 2500, 5000, 13440, 16000]


def _lattice_points(n, seed, periodic=True):
    rng = np.random.Generator(np.random.PCG64(seed))
    k = rng.integers(0, LQ, (n, 3))
    # planted partners exactly on edges (axis-aligned and 3-4-5 triangles),
    # and exactly half a box away (the minimum-image tie)
    base = k[rng.integers(0, n, 60)]
    offs = []
    for m in (16, 65, 100, 400, 2500, 13440):
        offs.append([m, 0, 0])
        offs.append([0, 0, -m])
        if m % 5 == 0:
            t = m // 5
            offs.append([3 * t, 4 * t, 0])
            offs.append([0, -4 * t, 3 * t])
    offs = np.array(offs)
    extra = base[:, None, :] + offs[None, :, :]
    extra = extra.reshape(-1, 3)
    if periodic:
        extra %= LQ
    else:
        extra = extra[(extra >= 0).all(1) & (extra < LQ).all(1)]
    return np.concatenate([k, extra], 0)


def _int_sep(ki, kj, periodic):
    d = kj[None, :, :] - ki[:, None, :]
    if periodic:
        d = np.where(d > LQ // 2, d - LQ, d)
        d = np.where(d < -(LQ // 2), d + LQ, d)
    return d


def _int_counts_xi(ki, kj, auto, periodic, em):
    d = _int_sep(ki, kj, periodic)
    s = (d * d).sum(-1)
    e2 = np.array(em, dtype=np.int64) ** 2
    ok = np.ones(s.shape, bool)
    if auto:
        np.fill_diagonal(ok, False)
    out = []
    for a, b in zip(e2[:-1], e2[1:]):
        out.append(int(((s >= a) & (s < b) & ok).sum()))
    return np.array(out, dtype=np.uint64)


def _int_counts_wp(ki, kj, auto, periodic, em, pim, npi):
    d = _int_sep(ki, kj, periodic)
    rp2 = d[..., 0] ** 2 + d[..., 1] ** 2
    pi = np.abs(d[..., 2])
    e2 = np.array(em, dtype=np.int64) ** 2
    ok = pi < pim
    if auto:
        np.fill_diagonal(ok, False)
    dq = pim // npi
    out = np.zeros((len(em) - 1, npi), dtype=np.uint64)
    for k, (a, b) in enumerate(zip(e2[:-1], e2[1:])):
        sel = (rp2 >= a) & (rp2 < b) & ok
        out[k] = np.bincount((pi[sel] // dq).astype(np.int64), minlength=npi)[:npi]
    return out


@pytest.mark.parametrize("periodic", [True, False])
@pytest.mark.parametrize("grid", [False, True])
def test_lattice_xi_exact(periodic, grid):
    k = _lattice_points(500, 11, periodic)
    x, y, z = (k[:, a] * Q for a in range(3))
    edges = np.array(EDGE_M, dtype=np.float64) * Q
    r = oracle.count(oracle.XI, x, y, z, edges=edges, periodic=periodic, box=420.0, grid=grid)
    ref = _int_counts_xi(k, k, True, periodic, EDGE_M)
    assert (r.npairs == ref).all()
    # there must be exact ties on edges for this to pin the half-open rule
    d = _int_sep(k, k, periodic)
    s = (d * d).sum(-1)
    assert np.isin(s, np.array(EDGE_M[1:], dtype=np.int64) ** 2).sum() > 100


@pytest.mark.parametrize("periodic", [True, False])
def test_lattice_cross_exact(periodic):
    k1 = _lattice_points(300, 21, periodic)
    k2 = _lattice_points(400, 22, periodic)
    c1 = [k1[:, a] * Q for a in range(3)]
    c2 = [k2[:, a] * Q for a in range(3)]
    edges = np.array(EDGE_M, dtype=np.float64) * Q
    r = oracle.count(oracle.XI, *c1, None, *c2, None, edges=edges, periodic=periodic, box=420.0)
    assert (r.npairs == _int_counts_xi(k1, k2, False, periodic, EDGE_M)).all()


@pytest.mark.parametrize("periodic", [True, False])
@pytest.mark.parametrize("grid", [False, True])
def test_lattice_wp_exact(periodic, grid):
    k = _lattice_points(500, 12, periodic)
    # pi edges fall on the lattice: pi_max = 2560 quanta = 40, 40 bins of 1
    k[:40, 2] = k[40:80, 2] + 64 * (np.arange(40) % 7)   # ties on pi edges
    k %= LQ
    x, y, z = (k[:, a] * Q for a in range(3))
    edges = np.array(EDGE_M[:12], dtype=np.float64) * Q
    r = oracle.count(oracle.WP, x, y, z, edges=edges, periodic=periodic, box=420.0,
                     pimax=40.0, npibins=40, grid=grid)
    ref = _int_counts_wp(k, k, True, periodic, EDGE_M[:12], 2560, 40)
    assert (r.npairs == ref).all()


def test_lattice_weights_exact():
    cat = synth.lattice(400, 420.0, quantum=Q, seed=5, weights=True, duplicates=20)
    edges = np.array(EDGE_M, dtype=np.float64) * Q
    r = oracle.xi(cat, edges, periodic=True, box=420.0)
    k = np.stack([np.rint(v / Q).astype(np.int64) for v in (cat.x, cat.y, cat.z)], 1)
    d = _int_sep(k, k, True)
    s = (d * d).sum(-1)
    ww = cat.w[:, None] * cat.w[None, :]          # exact: multiples of 1/16
    np.fill_diagonal(ww, 0.0)
    e2 = np.array(EDGE_M, dtype=np.int64) ** 2
    off = ~np.eye(len(k), dtype=bool)
    for b in range(len(EDGE_M) - 1):
        sel = (s >= e2[b]) & (s < e2[b + 1]) & off
        assert r.npairs[b] == sel.sum()
        assert r.wsum[b] == ww[sel].sum()             # exact sum of exact terms
        # weighted separation: 50-digit reference
        mpmath.mp.dps = 50
        ref = mpmath.fsum(mpmath.mpf(float(a)) * mpmath.sqrt(mpmath.mpf(int(si)) * mpmath.mpf(Q) ** 2)
                          for a, si in zip(ww[sel], s[sel]))
        if sel.sum():
            assert abs(r.wrsum[b] - float(ref)) <= 2e-15 * abs(float(ref))


# ------------------------------------------------------- closed-form totals

def test_full_box_total_periodic():
    cat = synth.uniform(2000, 420.0, seed=3)
    n = cat.n
    # every minimum-image separation is at most sqrt(3) * 210 < 400
    r = oracle.xi(cat, [0.0, 100.0, 400.0], periodic=True, box=420.0)
    assert int(r.npairs.sum()) == n * (n - 1)
    r = oracle.wp(cat, [0.0, 300.0], pimax=211.0, npibins=7, periodic=True, box=420.0)
    assert int(r.npairs.sum()) == n * (n - 1)


def test_full_box_total_nonperiodic_cross():
    a = synth.uniform(700, 50.0, seed=8)
    b = synth.uniform(900, 50.0, seed=9)
    r = oracle.xi(a, [0.0, 5.0, 90.0], periodic=False, other=b)
    assert int(r.npairs.sum()) == a.n * b.n


def test_auto_equals_self_cross():
    """Auto ordered counts equal the cross count of A with itself when the
    first edge is positive (self pairs have separation 0): unique = half."""
    cat = synth.clustered(3000, 60, 2.0, 100.0, seed=4, weights=True)
    edges = synth.log_edges(0.05, 20.0, 12)
    a = oracle.xi(cat, edges, periodic=True, box=100.0)
    c = oracle.xi(cat, edges, periodic=True, box=100.0, other=cat)
    assert (a.npairs == c.npairs).all()
    assert (a.npairs % 2 == 0).all()
    np.testing.assert_allclose(a.wsum, c.wsum, rtol=1e-14)
    # with a zero first edge the cross count also holds the n self pairs
    c0 = oracle.xi(cat, np.r_[0.0, edges], periodic=True, box=100.0, other=cat)
    a0 = oracle.xi(cat, np.r_[0.0, edges], periodic=True, box=100.0)
    assert int(c0.npairs[0]) == int(a0.npairs[0]) + cat.n


# ----------------------------------------------- grid enumeration = loop

@pytest.mark.parametrize("seed", [0, 1, 2])
@pytest.mark.parametrize("mode", ["xi", "wp"])
@pytest.mark.parametrize("periodic", [True, False])
def test_grid_equals_naive_loop(seed, mode, periodic):
    rng = np.random.Generator(np.random.PCG64(100 + seed))
    box = float(rng.choice([60.0, 100.0, 420.0]))
    cat = synth.clustered(1500, 40, 1.0 + 2 * seed, box, seed=seed, weights=True)
    rmax = float(rng.choice([box / 2.2, box / 3.5, box / 9.0]))
    edges = np.sort(rng.uniform(0, rmax, 8))
    edges[-1] = rmax
    if seed == 1:
        edges[0] = 0.0
    kw = dict(periodic=periodic, box=box)
    if mode == "wp":
        pimax = float(rng.choice([box / 2.5, box / 10.0]))
        g = oracle.wp(cat, edges, pimax, 5, grid=True, **kw)
        b = oracle.wp(cat, edges, pimax, 5, grid=False, **kw)
    else:
        g = oracle.xi(cat, edges, grid=True, **kw)
        b = oracle.xi(cat, edges, grid=False, **kw)
    assert (g.npairs == b.npairs).all()
    np.testing.assert_allclose(g.wsum, b.wsum, rtol=1e-14)
    np.testing.assert_allclose(g.wrsum, b.wrsum, rtol=1e-14)


def test_grid_equals_naive_loop_cross():
    d = synth.to_float32(synth.clustered(800, 20, 1.5, 420.0, seed=3))
    r = synth.to_float32(synth.uniform(5000, 420.0, seed=4))
    edges = synth.log_edges(0.1, 25.0, 14)
    g = oracle.xi(d, edges, periodic=False, other=r, grid=True)
    b = oracle.xi(d, edges, periodic=False, other=r, grid=False)
    assert (g.npairs == b.npairs).all()
    # float32 input is promoted exactly
    d64 = d.astype(np.float64)
    r64 = r.astype(np.float64)
    g64 = oracle.xi(d64, edges, periodic=False, other=r64)
    assert (g64.npairs == g.npairs).all()


# ------------------------------------------------------ statistical pins

def test_uniform_shell_expectation():
    """Uniform points in a periodic cube: E[DD_k] = N(N-1) (4 pi / 3)
    (e_{k+1}^3 - e_k^3) / L^3 (the analytic RR of Section 1.1)."""
    c = synth.config1()
    r = oracle.xi(c["cat"], c["edges"], periodic=True, box=c["box"])
    n = c["cat"].n
    e = c["edges"]
    expct = n * (n - 1) * (4 * np.pi / 3) * (e[1:] ** 3 - e[:-1] ** 3) / c["box"] ** 3
    sel = expct >= 50
    z = (r.npairs[sel] - expct[sel]) / np.sqrt(2 * expct[sel])
    assert np.all(np.abs(z) < 4.5), z
    chi2 = float((z ** 2).sum())
    assert chi2 < sel.sum() + 6 * np.sqrt(2 * sel.sum())


def test_wp_cylinder_expectation():
    """Uniform points: E[DD_{k,l}] = N(N-1) pi (e_{k+1}^2 - e_k^2) 2 dpi / L^3."""
    cat = synth.uniform(20000, 420.0, seed=6)
    edges = synth.log_edges(1.0, 25.0, 8)
    r = oracle.wp(cat, edges, 40.0, 4, periodic=True, box=420.0)
    n = cat.n
    ring = np.pi * (edges[1:] ** 2 - edges[:-1] ** 2)
    expct = n * (n - 1) * ring[:, None] * 2 * 10.0 / 420.0 ** 3 * np.ones((1, 4))
    sel = expct >= 50
    z = (r.npairs[sel] - expct[sel]) / np.sqrt(2 * expct[sel])
    assert np.all(np.abs(z) < 4.5), z


def test_wp_pi_sum_is_filtered_rp_histogram():
    """Summing the 2-D histogram over pi bins gives the paper's 1-D rp
    histogram with the pi < pi_max filter (one pi bin)."""
    cat = synth.clustered(4000, 80, 1.5, 200.0, seed=9)
    edges = synth.log_edges(0.1, 25.0, 14)
    r40 = oracle.wp(cat, edges, 40.0, 40, periodic=True, box=200.0)
    r1 = oracle.wp(cat, edges, 40.0, 1, periodic=True, box=200.0)
    assert (r40.npairs.sum(1) == r1.npairs[:, 0]).all()


def test_weight_special_cases():
    cat = synth.clustered(2000, 40, 1.5, 100.0, seed=10)
    edges = synth.log_edges(0.1, 20.0, 10)
    r1 = oracle.xi(cat, edges, periodic=True, box=100.0)
    assert (r1.wsum == r1.npairs.astype(np.float64)).all()
    cat.w = np.full(cat.n, 2.0)
    r2 = oracle.xi(cat, edges, periodic=True, box=100.0)
    assert (r2.npairs == r1.npairs).all()
    assert (r2.wsum == 4.0 * r1.wsum).all()
    assert (r2.wrsum == 4.0 * r1.wrsum).all()
    np.testing.assert_array_equal(r2.ravg, r1.ravg)


# ------------------------------------------------------------ error codes

def test_errors():
    p = np.array([[1.0, 2.0, 3.0], [4.0, 5.0, 6.0]])
    args = (p[:, 0], p[:, 1], p[:, 2])
    with pytest.raises(oracle.OracleError) as e:
        oracle.count(oracle.XI, *args, edges=[1.0, 1.0], periodic=False)
    assert e.value.code == -1
    with pytest.raises(oracle.OracleError) as e:
        oracle.count(oracle.XI, *args, edges=[1.0, 2.0], periodic=True, box=5.0)
    assert e.value.code == -2
    bad = p.copy()
    bad[0, 1] = np.nan
    with pytest.raises(oracle.OracleError) as e:
        oracle.count(oracle.XI, bad[:, 0], bad[:, 1], bad[:, 2], edges=[1.0, 2.0],
                     periodic=False)
    assert e.value.code == -3
    with pytest.raises(oracle.OracleError):
        oracle.count(oracle.WP, *args, edges=[1.0, 2.0], periodic=False, pimax=0.0)
    # fewer than two points: zero counts
    r = oracle.count(oracle.XI, p[:1, 0], p[:1, 1], p[:1, 2], edges=[0.0, 2.0],
                     periodic=False)
    assert r.npairs.tolist() == [0]
