"""Pin of the oracle's rounding on inputs where the arithmetic is inexact.

The lattice pins make every operation exact, so they cannot tell the oracle's
operation order from another one.  Here an independent brute force written in
numpy binary64 evaluates the reading of Section 1.1 (eqn:separations) with the
order of Code 3: per axis d = p_j - p_i, then the minimum image in a periodic
box (d > L/2 -> d - L, d < -L/2 -> d + L), then s = (dx*dx + dy*dy) + dz*dz;
squared edges E_k = e_k * e_k; bin k iff E_k <= s < E_{k+1}.  numpy rounds
every elementwise product and sum once and never fuses a multiply-add, so the
brute force is the unfused left-to-right sequence by construction.  It shares
nothing with oracle.c.

The inputs are random (non-lattice) coordinates plus planted pairs whose
canonical s is a squared edge or one of its binary64 neighbours, planted pairs
that straddle the periodic boundary, and planted line-of-sight separations on a
pi edge or its neighbours, with pi edges q_l = l * (pi_max / n) that are not
exact.  The oracle's counts (plain loop of Code 1 and chaining mesh of Section
1.2) must equal the brute force bit for bit.

Each test also shows that the fixture can tell the reading from plausible
mistakes: summing in another order, fusing a multiply-add, shifting a
coordinate by the box before subtracting, comparing r instead of s against the
edges, forming the pi edges as (l * pi_max) / n, or accepting pi = pi_max.
Each of those gives different counts on the same points.
"""
import math
from fractions import Fraction

import numpy as np
import pytest

import oracle

I64 = np.int64


# --------------------------------------------------------------- helpers

def _step(v, k):
    """v (> 0, binary64) moved by k units in the last place."""
    return (np.asarray(v, dtype=np.float64).view(I64) + I64(k)).view(np.float64)


def _sep(a, b, box):
    """d = b - a per axis, minimum image when box is given (canonical order)."""
    d = b - a
    if box is not None:
        h = 0.5 * box
        d = np.where(d > h, d - box, np.where(d < -h, d + box, d))
    return d


def _sep_shift_first(a, b, box):
    """A plausible mistake: the periodic shift applied to the coordinate
    before the subtraction, d = (b -/+ L) - a."""
    d = b - a
    if box is None:
        return d
    h = 0.5 * box
    return np.where(d > h, (b - box) - a, np.where(d < -h, (b + box) - a, d))


def _s_canon(dx, dy, dz):
    return (dx * dx + dy * dy) + dz * dz


def _fma(a, b, c):
    """Correctly rounded a * b + c (exact rational arithmetic)."""
    return float(Fraction(a) * Fraction(b) + Fraction(c))


def _bins(E, s):
    """k with E[k] <= s < E[k+1], -1 outside [E[0], E[-1])."""
    k = np.searchsorted(E, s, side="right") - 1
    return np.where(k >= len(E) - 1, -1, k)


def _pairs(p1, p2, auto, box, chunk=256):
    """Yields (i, j, dx, dy, dz) blocks of every ordered pair (j != i for
    an auto-count), canonical separations."""
    n1 = p1.shape[0]
    for i0 in range(0, n1, chunk):
        i1 = min(n1, i0 + chunk)
        d = [_sep(p1[i0:i1, a][:, None], p2[None, :, a], box) for a in range(3)]
        ok = np.ones(d[0].shape, bool)
        if auto:
            ok[np.arange(i1 - i0), np.arange(i0, i1)] = False
        yield i0, i1, d, ok


def _hist_xi(p1, p2, auto, box, E, s_fn=None, sep_fn=_sep, w1=None, w2=None):
    nb = len(E) - 1
    cnt = np.zeros(nb, np.uint64)
    terms_w = [[] for _ in range(nb)]
    terms_wr = [[] for _ in range(nb)]
    for i0, i1, d, ok in _pairs(p1, p2, auto, box):
        if sep_fn is not _sep:
            d = [sep_fn(p1[i0:i1, a][:, None], p2[None, :, a], box) for a in range(3)]
        s = (s_fn or _s_canon)(*d)
        k = _bins(E, s)
        sel = ok & (k >= 0)
        cnt += np.bincount(k[sel], minlength=nb).astype(np.uint64)
        if w1 is not None:
            ww = w1[i0:i1, None] * w2[None, :]
            wr = ww * np.sqrt(s)
            for b in range(nb):
                m = sel & (k == b)
                terms_w[b].append(ww[m])
                terms_wr[b].append(wr[m])
    if w1 is None:
        return cnt
    ws = np.array([math.fsum(np.concatenate(t)) if t else 0.0 for t in terms_w])
    wrs = np.array([math.fsum(np.concatenate(t)) if t else 0.0 for t in terms_wr])
    return cnt, ws, wrs


def _pi_edges(pimax, npi):
    dpi = pimax / npi
    return np.array([l * dpi for l in range(1, npi)], dtype=np.float64)


def _hist_wp(p1, p2, auto, box, E, pimax, npi, qin=None):
    nb = len(E) - 1
    cnt = np.zeros((nb, npi), np.uint64)
    qin = _pi_edges(pimax, npi) if qin is None else qin
    for i0, i1, d, ok in _pairs(p1, p2, auto, box):
        rp2 = d[0] * d[0] + d[1] * d[1]
        pi = np.abs(d[2])
        k = _bins(E, rp2)
        l = np.searchsorted(qin, pi, side="right")
        sel = ok & (k >= 0) & (pi < pimax)
        np.add.at(cnt, (k[sel], l[sel]), 1)
    return cnt


# ------------------------------------------------------- planted inputs

def _plant_sep(rng, targets, box, lo, ext, wrap_axis=None, tries=400, K=96):
    """Pairs (p_i, p_j) whose canonical squared separation equals each
    target exactly.  A random direction is drawn, then one coordinate of p_j
    is walked through consecutive binary64 values until s hits the target.
    wrap_axis: the pair straddles the periodic boundary on that axis."""
    out_i, out_j = [], []
    for v in targets:
        e = math.sqrt(v)
        for _ in range(tries):
            u = rng.normal(size=3)
            u /= np.linalg.norm(u)
            d = u * e
            if wrap_axis is not None:
                d[wrap_axis] = -abs(d[wrap_axis])
                if abs(d[wrap_axis]) < 0.2 * e:
                    continue
            pi = lo + rng.uniform(0, 1, 3) * ext
            if wrap_axis is not None:
                pi[wrap_axis] = rng.uniform(0.01, 0.9) * abs(d[wrap_axis])
            pj = pi + d
            if box is not None:
                pj = np.mod(pj, box)
                if np.any(pj >= box) or np.any(pj <= 0):
                    continue
            # tune the axis whose step moves s least (not the wrapped one)
            cand = [a for a in range(3) if a != wrap_axis and abs(d[a]) > 1e-3 * e]
            a = min(cand, key=lambda a: abs(d[a]) * np.spacing(pj[a]))
            ks = np.arange(-K, K + 1)
            col = _step(pj[a], ks)
            P = np.repeat(pj[None, :], ks.size, 0)
            P[:, a] = col
            dd = [_sep(pi[b], P[:, b], box) for b in range(3)]
            s = _s_canon(*dd)
            hit = np.nonzero(s == v)[0]
            if hit.size and (box is None or (0 < P[hit[0]]).all() and (P[hit[0]] < box).all()):
                out_i.append(pi)
                out_j.append(P[hit[0]])
                break
    return np.array(out_i), np.array(out_j)


def _edge_targets(E, per=3):
    """Each squared edge and its two binary64 neighbours, `per` times."""
    t = []
    for v in E:
        if v <= 0:
            continue
        for k in (-1, 0, 1):
            t += [float(_step(v, k))] * per
    return t


# ----------------------------------------------------------------- xi

BOX = 97.3                                  # not a round number: inexact wraps
EDGES = np.geomspace(0.37, 23.9, 12)        # inexact edges and squares


def _xi_catalog(seed, periodic):
    rng = np.random.Generator(np.random.PCG64(seed))
    E = EDGES * EDGES
    if periodic:
        lo, ext, box = np.zeros(3), np.full(3, BOX), BOX
    else:
        # large coordinates: the subtraction rounds at a coarse step
        lo, ext, box = np.array([1000.0, -1200.0 + 1e3, 333.3]), np.full(3, 80.0), None
    bg = lo + rng.uniform(0, 1, (1500, 3)) * ext
    a, b = _plant_sep(rng, _edge_targets(E), box, lo, ext)
    parts = [bg, a, b]
    if periodic:
        for ax in range(3):
            a, b = _plant_sep(rng, _edge_targets(E, 1), box, lo, ext, wrap_axis=ax)
            parts += [a, b]
    p = np.concatenate(parts, 0)
    return p[rng.permutation(p.shape[0])], E


def _oracle_xi(p, E_edges, box, other=None, w=None, w2=None, grid=True):
    kw = dict(edges=E_edges, periodic=box is not None, box=box or 0.0, grid=grid)
    if other is None:
        return oracle.count(oracle.XI, p[:, 0], p[:, 1], p[:, 2], w, **kw)
    return oracle.count(oracle.XI, p[:, 0], p[:, 1], p[:, 2], w,
                        other[:, 0], other[:, 1], other[:, 2], w2, **kw)


def _near_edge_alt(p1, p2, auto, box, E, base_cnt, alt_s):
    """Histogram under an alternative s that differs from the canonical one
    by at most a couple of ulps: only pairs within 4 ulps of an edge can
    change bin, and those are re-binned with alt_s (python floats)."""
    cnt = base_cnt.astype(np.int64).copy()
    for i0, i1, d, ok in _pairs(p1, p2, auto, box):
        s = _s_canon(*d)
        k = _bins(E, s)
        near = np.zeros(s.shape, bool)
        for v in E:
            near |= np.abs(s - v) <= 4 * np.spacing(v)
        for ii, jj in zip(*np.nonzero(near & ok)):
            s2 = alt_s(float(d[0][ii, jj]), float(d[1][ii, jj]), float(d[2][ii, jj]))
            k1 = int(k[ii, jj])
            k2 = int(_bins(E, np.array([s2]))[0])
            if k1 >= 0:
                cnt[k1] -= 1
            if k2 >= 0:
                cnt[k2] += 1
    return cnt.astype(np.uint64)


@pytest.mark.parametrize("periodic", [True, False])
def test_xi_rounding_matches_brute_force(periodic):
    p, E = _xi_catalog(31 if periodic else 32, periodic)
    box = BOX if periodic else None
    ref = _hist_xi(p, p, True, box, E)
    for grid in (False, True):
        r = _oracle_xi(p, EDGES, box, grid=grid)
        assert (r.npairs == ref).all(), (grid, r.npairs, ref)
    # the planted pairs put many separations exactly on edges
    s_hits = 0
    for i0, i1, d, ok in _pairs(p, p, True, box):
        s = _s_canon(*d)
        s_hits += int((np.isin(s, E) & ok).sum())
    assert s_hits >= 2 * len(E)

    # the fixture tells the reading from plausible mistakes
    alts = {
        "reassociated": lambda dx, dy, dz: dx * dx + (dy * dy + dz * dz),
        "fused last add": lambda dx, dy, dz: _fma(dz, dz, dx * dx + dy * dy),
        "fused first add": lambda dx, dy, dz: (_fma(dy, dy, dx * dx)) + dz * dz,
    }
    for name, f in alts.items():
        alt = _near_edge_alt(p, p, True, box, E, ref, f)
        assert (alt != ref).any(), name
    # distance-space bins (r = sqrt(s) against e_k) instead of squared space
    dist = np.zeros_like(ref)
    for i0, i1, d, ok in _pairs(p, p, True, box):
        r_ = np.sqrt(_s_canon(*d))
        k = _bins(EDGES, r_)
        dist += np.bincount(k[ok & (k >= 0)], minlength=len(ref)).astype(np.uint64)
    assert (dist != ref).any()
    if periodic:
        alt = _hist_xi(p, p, True, box, E, sep_fn=_sep_shift_first)
        assert (alt != ref).any()


def test_xi_cross_rounding_and_weights():
    """Cross counts (set 1 against set 2) and the weighted sums on inexact
    values: counts bit for bit; sum of w_i w_j and of w_i w_j sqrt(s) against
    exactly rounded sums (math.fsum) of the same rounded terms."""
    rng = np.random.Generator(np.random.PCG64(33))
    p, E = _xi_catalog(34, True)
    n = p.shape[0]
    idx = rng.permutation(n)
    p1, p2 = p[idx[: n // 2]], p[idx[n // 2:]]
    w1 = rng.uniform(0.5, 1.5, p1.shape[0])
    w2 = rng.uniform(0.5, 1.5, p2.shape[0])
    cnt, ws, wrs = _hist_xi(p1, p2, False, BOX, E, w1=w1, w2=w2)
    for grid in (False, True):
        r = _oracle_xi(p1, EDGES, BOX, other=p2, w=w1, w2=w2, grid=grid)
        assert (r.npairs == cnt).all()
        np.testing.assert_allclose(r.wsum, ws, rtol=1e-15, atol=0)
        np.testing.assert_allclose(r.wrsum, wrs, rtol=1e-15, atol=0)


# ----------------------------------------------------------------- wp

PIMAX, NPI = 37.3, 13                         # l * (37.3 / 13) != (l * 37.3) / 13 for some l


def _plant_pi(rng, targets, box, tries=200, K=64):
    """Pairs with |dz| = fl(z_j - z_i) equal to each target exactly, r_p
    random within the largest r_p edge."""
    out_i, out_j = [], []
    for t in targets:
        for _ in range(tries):
            zi = rng.uniform(0.05, 3.0)
            zj0 = zi + t
            ks = np.arange(-K, K + 1)
            zj = _step(zj0, ks)
            hit = np.nonzero((zj - zi) == t)[0]
            if not hit.size:
                continue
            rp = rng.uniform(0.5, 0.95) * EDGES[-1]
            ang = rng.uniform(0, 2 * np.pi)
            xi_, yi_ = rng.uniform(30.0, 60.0, 2)
            pi = np.array([xi_, yi_, zi])
            pj = np.array([xi_ + rp * np.cos(ang), yi_ + rp * np.sin(ang), zj[hit[0]]])
            if rng.uniform() < 0.5:            # also the other sign of dz
                pi, pj = pj, pi
            out_i.append(pi)
            out_j.append(pj)
            break
    return np.array(out_i), np.array(out_j)


def _plant_rp(rng, targets, box, tries=400, K=96):
    """Pairs whose canonical r_p^2 = dx*dx + dy*dy equals each target
    exactly (|dz| below pi_max), found as in _plant_sep."""
    out_i, out_j = [], []
    for v in targets:
        rp = math.sqrt(v)
        for _ in range(tries):
            ang = rng.uniform(0, 2 * np.pi)
            d = np.array([rp * math.cos(ang), rp * math.sin(ang), rng.uniform(-0.8, 0.8) * PIMAX])
            pi = rng.uniform(0, box, 3)
            pj = np.mod(pi + d, box)
            if np.any(pj >= box) or np.any(pj <= 0):
                continue
            cand = [a for a in (0, 1) if abs(d[a]) > 1e-3 * rp]
            a = min(cand, key=lambda a: abs(d[a]) * np.spacing(pj[a]))
            ks = np.arange(-K, K + 1)
            P = np.repeat(pj[None, :], ks.size, 0)
            P[:, a] = _step(pj[a], ks)
            dx, dy = (_sep(pi[b], P[:, b], box) for b in (0, 1))
            hit = np.nonzero(dx * dx + dy * dy == v)[0]
            if hit.size and (0 < P[hit[0]]).all() and (P[hit[0]] < box).all():
                out_i.append(pi)
                out_j.append(P[hit[0]])
                break
    return np.array(out_i), np.array(out_j)


def _wp_catalog(seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    E = EDGES * EDGES
    bg = rng.uniform(0, BOX, (1300, 3))
    # r_p^2 on squared edges and their neighbours
    a, b = _plant_rp(rng, _edge_targets(E, 2), BOX)
    # pi on pi edges, on pi_max and their neighbours
    qin = _pi_edges(PIMAX, NPI)
    tq = []
    for q in list(qin) + [PIMAX]:
        tq += [float(_step(q, k)) for k in (-1, 0, 1)] * 3
    c, d = _plant_pi(rng, tq, BOX)
    p = np.concatenate([bg, a, b, c, d], 0)
    assert ((p >= 0) & (p < BOX)).all()
    return p[rng.permutation(p.shape[0])], E


def test_wp_rounding_matches_brute_force():
    p, E = _wp_catalog(41)
    ref = _hist_wp(p, p, True, BOX, E, PIMAX, NPI)
    for grid in (False, True):
        r = oracle.count(oracle.WP, p[:, 0], p[:, 1], p[:, 2], edges=EDGES, periodic=True,
                         box=BOX, pimax=PIMAX, npibins=NPI, grid=grid)
        assert (r.npairs == ref).all(), grid
    # there are exact ties on pi edges, on pi_max and on r_p^2 edges
    qin = _pi_edges(PIMAX, NPI)
    ties_pi = ties_rp = at_max = 0
    for i0, i1, d, ok in _pairs(p, p, True, BOX):
        pi = np.abs(d[2])
        rp2 = d[0] * d[0] + d[1] * d[1]
        ties_pi += int((np.isin(pi, qin) & ok).sum())
        at_max += int(((pi == PIMAX) & ok).sum())
        ties_rp += int((np.isin(rp2, E) & ok).sum())
    assert ties_pi >= 2 * len(qin) and at_max >= 2 and ties_rp >= 10

    # plausible mistakes change the counts
    alt_q = np.array([(l * PIMAX) / NPI for l in range(1, NPI)])
    assert (alt_q != qin).any()
    alt = _hist_wp(p, p, True, BOX, E, PIMAX, NPI, qin=alt_q)
    assert (alt != ref).any()
    # pi <= pi_max accepted instead of pi < pi_max
    alt = _hist_wp(p, p, True, BOX, E, PIMAX * (1 + 2 ** -52), NPI, qin=qin)
    assert alt.sum() != ref.sum()
