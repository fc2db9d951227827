"""The binary32 decision bound of the pair kernels, checked on the CPU.

The binary32 loops decide a pair against an edge E from d~, the binary32
value of s - E evaluated in the kernel's operation order; a pair with
|d~| >= eps goes to the side sign(d~) says, anything closer is re-evaluated
in binary64.  These tests replay that operation order in numpy binary32
(fused multiply-adds emulated through binary64, whose extra rounding is far
below the margins) on pairs placed within a few parts per million of the
edges, and check that

  * |d~ - (s - E)| stays below eps / 2 (the derived bound without its safety
    factor of two), for the two-slot form d~ = fl(fma chain from
    b = fl32(|r|^2 - E)) + |p|^2 and for the three-slot second difference
    d2 = fl(d1 + fl32(E_a - E_b)) against eps + 2 u E_B;
  * every pair with |d~| >= eps lands on the side of the binary64 reference
    value s (the canonical unfused ((dx^2 + dy^2) + dz^2));
  * the z-window of a unit (late entry / early exit) keeps every pair within
    reach.

eps follows the derivation of the decision bound: with u = 2^-24,
u64 = 2^-53, P the half diagonal of a cell, e_B = R_max, G = 2 P + e_B and M
the largest coordinate magnitude,
  eta = u G 1.01 + 4 sqrt(3) u64 M,
  eps = 2 [7.5 u G^2 + 2 e_B eta + eta^2 + 8 u64 (E_B + 2 e_B M)].
"""
import math

import numpy as np
import pytest

U = 2.0 ** -24
U64 = 2.0 ** -53


def f32(x):
    return np.asarray(x, dtype=np.float64).astype(np.float32)


def fmaf(a, b, c):
    """binary32 fma: exact product and sum in binary64, one rounding to binary32."""
    return f32(a.astype(np.float64) * b.astype(np.float64) + c.astype(np.float64))


def eps_xi(cell, rmax, box):
    P = 0.5 * math.sqrt(3.0) * cell * (1 + 1e-6)
    eB = rmax
    G = 2 * P + eB
    M = box
    eta = U * G * 1.01 + 4 * math.sqrt(3.0) * U64 * M
    return 2.0 * (7.5 * U * G * G + 2 * eB * eta + eta * eta + 8 * U64 * (eB * eB + 2 * eB * M))


def _pairs(rng, n, edges, cell, box, shift):
    """Tile points x_i in a cell of the box, partners x_j at squared
    separation within a few ppm of a random edge (only partners that stay in
    the box are kept), in a cell offset by up to two cells; optional periodic
    shift of the partner's cell by one box length along x."""
    E = np.asarray(edges, dtype=np.float64) ** 2
    k = rng.integers(1, len(edges), n)
    # half the pairs within 4 ppm of the edge (mostly inside the band), half
    # within 200 ppm (mostly decided in binary32)
    width = np.where(rng.random(n) < 0.5, 4e-6, 2e-4)
    target = E[k] * (1.0 + rng.uniform(-1.0, 1.0, n) * width)
    xi = rng.uniform(2 * cell, box - 2 * cell, (n, 3))
    v = rng.normal(size=(n, 3))
    v /= np.linalg.norm(v, axis=1)[:, None]
    xj = xi + v * np.sqrt(target)[:, None]
    ok = np.all((xj >= 0) & (xj < box), axis=1)
    xi, xj, k = xi[ok], xj[ok], k[ok]
    S = np.zeros_like(xi)
    if shift:
        # the partner's stored coordinate is x_j - L, its cell is shifted by +L
        xj = xj.copy()
        xj[:, 0] -= box
        S[:, 0] = box
        keep = xj[:, 0] >= -box
        xi, xj, k, S = xi[keep], xj[keep], k[keep], S[keep]
    return xi, xj, k, S, E


def _kernel_d(xi, xj, S, E_t, cell):
    """d~ in the two-slot loop's operation order."""
    O = (np.floor(xj / cell) + 0.5) * cell          # centre of the partner's cell
    p = f32(xj - O)
    r = f32(xi - (O + S))
    qx, qy, qz = -2.0 * p[:, 0], -2.0 * p[:, 1], -2.0 * p[:, 2]   # exact in binary32
    qw = fmaf(p[:, 2], p[:, 2], fmaf(p[:, 1], p[:, 1], f32(p[:, 0] * p[:, 0])))
    ra = fmaf(r[:, 2], r[:, 2], fmaf(r[:, 1], r[:, 1], f32(r[:, 0] * r[:, 0])))
    b = f32(ra.astype(np.float64) - E_t)
    v = fmaf(r[:, 0], qx, b)
    v = fmaf(r[:, 1], qy, v)
    v = fmaf(r[:, 2], qz, v)
    return f32(v.astype(np.float64) + qw.astype(np.float64))


def _s64(xi, xj, S):
    d = (xj - xi) + S
    return (d[:, 0] * d[:, 0] + d[:, 1] * d[:, 1]) + d[:, 2] * d[:, 2]


@pytest.mark.parametrize("refine,shift", [(2, False), (2, True), (3, False), (4, True)])
def test_two_slot_bound(refine, shift):
    rng = np.random.Generator(np.random.PCG64(11 + refine + 7 * shift))
    box, rmax = 420.0, 25.0
    edges = np.geomspace(0.1, rmax, 15)
    cell = box / math.floor(box / (rmax / refine))
    eps = eps_xi(cell, rmax, box)
    xi, xj, k, S, E = _pairs(rng, 400_000, edges, cell, box, shift)
    Et = E[k]
    d = _kernel_d(xi, xj, S, Et, cell)
    s = _s64(xi, xj, S)
    err = np.abs(d.astype(np.float64) - (s - Et))
    assert err.max() < eps / 2, (err.max(), eps)
    eps32 = np.nextafter(np.float32(eps), np.float32(np.inf))
    sure = np.abs(d) >= eps32
    assert sure.mean() > 0.1                      # the test does exercise decisions
    assert np.array_equal((d < 0)[sure], (s < Et)[sure])


def test_three_slot_second_difference():
    rng = np.random.Generator(np.random.PCG64(5))
    box, rmax = 420.0, 25.0
    edges = np.geomspace(0.1, rmax, 15)
    cell = box / math.floor(box / (rmax / 2))
    eps = eps_xi(cell, rmax, box)
    E = edges ** 2
    eps3 = eps + 2 * U * E[-1] * 1.01
    xi, xj, k, S, _ = _pairs(rng, 400_000, edges, cell, box, False)
    # the upper edge of the three-slot unit is the target edge: E_b = E[k],
    # E_a = E[k - 1]
    Ea, Eb = E[k - 1], E[k]
    d1 = _kernel_d(xi, xj, S, Ea, cell)
    c = f32(Ea - Eb)
    d2 = f32(d1.astype(np.float64) + c.astype(np.float64))
    s = _s64(xi, xj, S)
    err = np.abs(d2.astype(np.float64) - (s - Eb))
    assert err.max() < eps3 / 2, (err.max(), eps3)
    sure = np.abs(d2) >= np.float32(eps3)
    assert np.array_equal((d2 < 0)[sure], (s < Eb)[sure])


def test_z_window_keeps_pairs_within_reach():
    """Every pair with s < E_B lies inside the unit's z-window computed from
    the tile's z range and the x/y gaps (here the pair's own |dx|, |dy|, the
    tightest gaps a bounding box can give)."""
    rng = np.random.Generator(np.random.PCG64(9))
    rmax = 25.0
    EB = rmax * rmax
    n = 500_000
    xi = rng.uniform(0, 420, (n, 3))
    v = rng.normal(size=(n, 3))
    v /= np.linalg.norm(v, axis=1)[:, None]
    xj = xi + v * (rmax * np.sqrt(rng.uniform(0.999, 1.0, n)))[:, None]
    d = xj - xi
    s = (d[:, 0] * d[:, 0] + d[:, 1] * d[:, 1]) + d[:, 2] * d[:, 2]
    keep = s < EB
    xi, xj, d = xi[keep], xj[keep], d[keep]
    m0, m1 = np.abs(d[:, 0]), np.abs(d[:, 1])
    rp = m0 * m0 + m1 * m1
    hz = np.sqrt(f32(np.maximum(EB - rp, 0.0) + 1e-12 * EB)).astype(np.float64) * (1.0 + 1e-5)
    hz = hz + 1e-9 * (2 * np.abs(xi[:, 2]) + 1.0)
    zl = xi[:, 2] - hz
    zh = xi[:, 2] + hz
    lo = zl.astype(np.float32)
    lo = np.where(lo.astype(np.float64) > zl, np.nextafter(lo, np.float32(-np.inf)), lo)
    hi = zh.astype(np.float32)
    hi = np.where(hi.astype(np.float64) < zh, np.nextafter(hi, np.float32(np.inf)), hi)
    assert np.all(xj[:, 2] >= lo.astype(np.float64))
    assert np.all(xj[:, 2] <= hi.astype(np.float64))


def test_pi_bin_without_division():
    """The binary64 pi bin of the kernels: l0 = trunc(pi * fl(1 / dpi)) clamped
    to [0, npi), then one compare each way against q_l = fl(l dpi) and
    q_{l+1}; against the definition q_l <= pi < q_{l+1} (q_0 = 0, top pi_max)
    by search, on random and on edge-adjacent values of pi."""
    rng = np.random.Generator(np.random.PCG64(31))
    for _ in range(200):
        pimax = float(rng.uniform(0.5, 300.0))
        npi = int(rng.integers(1, 257))
        dpi = pimax / npi
        inv = 1.0 / dpi
        q = np.array([0.0] + [l * dpi for l in range(1, npi)] + [pimax])
        pz = list(rng.uniform(0.0, pimax, 200))
        for l in range(1, npi):
            for v in (q[l], np.nextafter(q[l], 0.0), np.nextafter(q[l], np.inf)):
                pz.append(float(v))
        pz = np.array([v for v in pz if 0.0 <= v < pimax])
        l0 = np.clip((pz * inv).astype(np.int64), 0, npi - 1)
        lq = np.array([l * dpi for l in range(npi + 1)])
        l1 = l0 - ((l0 > 0) & (pz < lq[l0])).astype(np.int64)
        l2 = l1 + ((l1 + 1 < npi) & (pz >= lq[np.minimum(l1 + 1, npi)])).astype(np.int64)
        want = np.searchsorted(q[1:npi], pz, side="right")
        assert np.array_equal(l2, want)


def _f32_up(x):
    """Smallest binary32 value >= x (elementwise)."""
    x = np.asarray(x, dtype=np.float64)
    r = x.astype(np.float32)
    return np.where(r.astype(np.float64) < x, np.nextafter(r, np.float32(np.inf)), r)


def _f32_down(x):
    """Largest binary32 value <= x (elementwise)."""
    x = np.asarray(x, dtype=np.float64)
    r = x.astype(np.float32)
    return np.where(r.astype(np.float64) > x, np.nextafter(r, np.float32(-np.inf)), r)


def pi_band(eta, dpi, npi):
    """The binary32 pi band of the w_p loops, in units of dpi."""
    return np.float32(eta / dpi + 8 * U * npi + 1e-12 * npi)


@pytest.mark.parametrize("seed", [41, 42])
def test_pi_binary32_decision(seed):
    """Binary32 pi decision of the w_p loops: a pair is counted at once when
    pi~ < pi_hi32 = up32(pi_max + eta) and the fraction of
    f = fl32(pi~ * fl32(1 / dpi)) lies in [pi_delta, fl32(1 - pi_delta)]; it
    goes to bin floor(f).  For every estimate within eta of |dz| that must be
    the bin of |dz| under the binary64 edges q_l = fl(l dpi), with |dz| below
    pi_max (the loops keep no separate test near pi_max).  |dz| is placed on
    and around every edge, pi_max included, with estimates at both ends of
    its error interval and at the nearest binary32 value."""
    rng = np.random.Generator(np.random.PCG64(seed))
    counted = 0
    for _ in range(150):
        pimax = float(rng.uniform(0.5, 300.0))
        npi = int(rng.integers(1, 257))
        dpi = pimax / npi
        eta = dpi * float(10.0 ** rng.uniform(-9.0, -4.0))
        inv = np.float32(1.0 / dpi)
        pd = pi_band(eta, dpi, npi)
        pd1 = np.float32(np.float32(1.0) - pd)
        phi = _f32_up(pimax + eta)
        q = np.array([l * dpi for l in range(1, npi)] + [pimax])
        base = np.concatenate([q, np.nextafter(q, 0.0), np.nextafter(q, np.inf),
                               rng.uniform(0.0, 1.02 * pimax, 300)])
        offs = np.array([-4.0, -2.0, -1.0, -0.6, -0.2, 0.0, 0.2, 0.6, 1.0, 2.0, 4.0]) * eta
        step = 8 * U * max(npi, 1) * dpi * np.array([-1.0, -0.5, 0.5, 1.0])
        dz = np.concatenate([(base[:, None] + offs[None, :]).ravel(),
                             (q[:, None] + step[None, :]).ravel()])
        dz = dz[dz >= 0.0]
        truebin = np.searchsorted(q[:-1], dz, side="right")
        for est in (dz.astype(np.float32), _f32_up(np.maximum(dz - eta, 0.0)), _f32_down(dz + eta)):
            ok = np.abs(est.astype(np.float64) - dz) <= eta
            f = est * inv                       # binary32 product
            fr = f - np.floor(f)                # exact: the kernels' v_fract
            certain = ok & (est < phi) & (fr >= pd) & (fr <= pd1)
            counted += int(certain.sum())
            assert np.all(dz[certain] < pimax)
            assert np.array_equal(np.floor(f[certain]).astype(np.int64), truebin[certain])
    assert counted > 10000


@pytest.mark.parametrize("seed", [43, 44])
def test_pi_bin_binary64_through_binary32(seed):
    """The binary64 w_p loops bin a binary64 |dz| < pi_max through binary32:
    f = fl32(fl32(|dz|) * fl32(1 / dpi)), bin floor(f) unless the fraction of
    f lies within pi_delta64 = 1.01 u pi_max / dpi + 8 u npi (+1e-12 npi) of
    an integer.  Every bin so taken must be the bin of |dz| under the binary64
    edges, on |dz| at and around every edge and just below pi_max."""
    rng = np.random.Generator(np.random.PCG64(seed))
    counted = 0
    for _ in range(150):
        pimax = float(rng.uniform(0.5, 300.0))
        npi = int(rng.integers(1, 257))
        dpi = pimax / npi
        inv = np.float32(1.0 / dpi)
        pd = np.float32(1.01 * U * pimax / dpi + 8 * U * npi + 1e-12 * npi)
        pd1 = np.float32(np.float32(1.0) - pd)
        q = np.array([l * dpi for l in range(1, npi)] + [pimax])
        base = np.concatenate([q, np.nextafter(q, 0.0), np.nextafter(q, np.inf),
                               rng.uniform(0.0, pimax, 300)])
        step = dpi * np.array([-1e-4, -1e-5, -1e-6, -1e-7, 0.0, 1e-7, 1e-6, 1e-5, 1e-4])
        dz = (base[:, None] + step[None, :]).ravel()
        dz = dz[(dz >= 0.0) & (dz < pimax)]
        truebin = np.searchsorted(q[:-1], dz, side="right")
        f = dz.astype(np.float32) * inv
        fr = f - np.floor(f)
        certain = (fr >= pd) & (fr <= pd1)
        counted += int(certain.sum())
        assert np.array_equal(np.floor(f[certain]).astype(np.int64), truebin[certain])
        assert np.all(np.floor(f[certain]) <= npi - 1)
    assert counted > 10000
