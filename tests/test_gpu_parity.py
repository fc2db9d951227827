"""GPU parity: the HIP path (through the C ABI) against the CPU FP64 oracle.

Counts must match exactly (both precisions); weighted sums and mean
separations within 1e-12 relative.  Sizes here let the oracle finish in
seconds while still spanning many tiles, ragged tiles and shifted periodic
cells; the full-size workloads are in test_gpu_fullsize.py.
"""
import os

import numpy as np
import pytest

import oracle
from paper_1911_08275_amd import synth

pytestmark = pytest.mark.gpu

RTOL_W = 1e-12


@pytest.fixture(scope="module")
def native():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1911_08275_amd import native
    native.lib()
    return native


def _say(*a):
    print(*a, flush=True)


def _check(g, r, weighted=False, prec=None, periodic=True):
    n = g.npairs.reshape(r.npairs.shape)
    bad = np.nonzero(n != r.npairs)
    assert (n == r.npairs).all(), (bad, n[bad], r.npairs[bad])
    if weighted:
        ws = g.wsum.reshape(r.wsum.shape)
        np.testing.assert_allclose(ws, r.wsum, rtol=RTOL_W, atol=0)
        np.testing.assert_allclose(g.ravg.reshape(r.wsum.shape), r.ravg, rtol=RTOL_W, atol=0)
    if prec is not None:
        # the precision the pair kernel ran: as asked, except on a periodic
        # grid with a single wrapped cell on some axis (per-pair minimum
        # images) and for weighted xi (unless the binary32 screen is asked
        # for), which run in binary64
        wrapped = periodic and 1 in list(g.stats["grid"])
        w_xi = weighted and r.npairs.ndim == 1 and os.environ.get("CP_XI_WEIGHTED_BINARY32") != "1"
        assert g.stats["precision"] == ("fp64" if (wrapped or w_xi) else prec), g.stats


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_config1_uniform(native, prec):
    c = synth.config1()
    _say("config1", prec)
    ref = oracle.xi(c["cat"], c["edges"], periodic=True, box=c["box"])
    d = native.to_device(c["cat"])
    g = native.countpairs_xi(d, c["edges"], precision=prec, periodic=True, boxsize=c["box"])
    _check(g, ref, prec=prec)
    assert g.stats["candidates"] > 0


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_clustered_xi_weighted(native, prec):
    cat = synth.clustered(60_000, 1200, 1.5, 420.0, seed=2, weights=True)
    edges = synth.log_edges(0.1, 25.0, 14)
    _say("clustered xi weighted", prec)
    ref = oracle.xi(cat, edges, periodic=True, box=420.0)
    d = native.to_device(cat)
    g = native.countpairs_xi(d, edges, precision=prec, periodic=True, boxsize=420.0,
                             need_ravg=True)
    _check(g, ref, weighted=True, prec=prec)
    # counts only, same call without weights requested
    g2 = native.countpairs_xi(d, edges, precision=prec, periodic=True, boxsize=420.0)
    _check(g2, ref, prec=prec)


def test_xi_weighted_binary32_screen(native, monkeypatch):
    """Weighted xi with the binary32 screen switched on
    (CP_XI_WEIGHTED_BINARY32=1): candidates screened in binary32, the pairs
    that survive evaluated in binary64 from the wave's list; counts equal the
    oracle, sums within 1e-12, on a clustered periodic catalogue at several
    refine factors and with pruning off, a non-periodic one and a cross
    count."""
    monkeypatch.setenv("CP_XI_WEIGHTED_BINARY32", "1")
    cat = synth.clustered(60_000, 1200, 1.5, 420.0, seed=2, weights=True)
    edges = synth.log_edges(0.1, 25.0, 14)
    ref = oracle.xi(cat, edges, periodic=True, box=420.0)
    d = native.to_device(cat)
    for refine in ((2, 2, 2), (1, 1, 1), (3, 3, 2)):
        for noprune in (False, True):
            _say("xi weighted binary32 screen", refine, noprune)
            g = native.countpairs_xi(d, edges, precision="fp32", periodic=True, boxsize=420.0,
                                     need_ravg=True, refine=refine, no_prune=noprune)
            _check(g, ref, weighted=True, prec="fp32")
    c = synth.clustered(8_000, 200, 2.0, 200.0, seed=51, weights=True)
    np_cat = synth.Catalog(c.x - 20.0, c.y * 0.75 + 5.0, c.z * 0.5, c.w)
    e2 = synth.log_edges(0.5, 20.0, 10)
    g = native.countpairs_xi(native.to_device(np_cat), e2, precision="fp32", periodic=False,
                             need_ravg=True)
    _check(g, oracle.xi(np_cat, e2, periodic=False), weighted=True, prec="fp32", periodic=False)
    b = synth.uniform(40_000, 420.0, seed=22, weights=True)
    g = native.countpairs_cross(d, native.to_device(b), edges, precision="fp32", periodic=True,
                                boxsize=420.0, need_ravg=True)
    _check(g, oracle.xi(cat, edges, periodic=True, box=420.0, other=b), weighted=True,
           prec="fp32")


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_clustered_wp(native, prec):
    cat = synth.clustered(60_000, 1200, 1.5, 420.0, seed=3)
    edges = synth.log_edges(0.1, 25.0, 14)
    _say("clustered wp", prec)
    ref = oracle.wp(cat, edges, 40.0, 40, periodic=True, box=420.0)
    d = native.to_device(cat)
    g = native.countpairs_wp(d, edges, 40.0, 40, precision=prec, periodic=True, boxsize=420.0)
    _check(g, ref, prec=prec)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_wp_weighted(native, prec):
    cat = synth.clustered(30_000, 600, 2.0, 200.0, seed=13, weights=True)
    edges = synth.log_edges(0.2, 20.0, 9)
    _say("wp weighted", prec)
    ref = oracle.wp(cat, edges, 25.0, 10, periodic=True, box=200.0)
    d = native.to_device(cat)
    g = native.countpairs_wp(d, edges, 25.0, 10, precision=prec, periodic=True, boxsize=200.0,
                             need_ravg=True)
    _check(g, ref, weighted=True, prec=prec)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_cross_nonperiodic_float32(native, prec):
    dcat = synth.to_float32(synth.clustered(20_000, 400, 1.5, 420.0, seed=2))
    rcat = synth.to_float32(synth.uniform(150_000, 420.0, seed=4))
    edges = synth.log_edges(0.1, 25.0, 14)
    _say("cross f32", prec)
    ref = oracle.xi(dcat, edges, periodic=False, other=rcat)
    g = native.countpairs_cross(native.to_device(dcat), native.to_device(rcat), edges,
                                precision=prec, periodic=False)
    _check(g, ref, prec=prec, periodic=False)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_cross_wp_periodic_weighted(native, prec):
    a = synth.clustered(15_000, 300, 1.5, 300.0, seed=21, weights=True)
    b = synth.uniform(40_000, 300.0, seed=22, weights=True)
    edges = synth.log_edges(0.5, 20.0, 8)
    _say("cross wp", prec)
    ref = oracle.wp(a, edges, 30.0, 6, periodic=True, box=300.0, other=b)
    g = native.countpairs_cross_wp(native.to_device(a), native.to_device(b), edges, 30.0, 6,
                                   precision=prec, periodic=True, boxsize=300.0, need_ravg=True)
    _check(g, ref, weighted=True, prec=prec)


Q = 2.0 ** -6


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("mode", ["xi", "wp"])
def test_lattice_edge_ties(native, prec, mode):
    """Lattice points with many separations exactly on bin edges: the binary32
    path must send them to binary64 and land on the reference side."""
    rng = np.random.Generator(np.random.PCG64(31))
    k = rng.integers(0, int(60 / Q), (3000, 3))
    base = k[rng.integers(0, len(k), 400)]
    offs = np.array([[64, 0, 0], [0, 192, 0], [0, 0, 320], [3 * 64, 4 * 64, 0],
                     [0, 3 * 128, 4 * 128], [640, 0, 0], [0, 0, 64 * 7]])
    extra = (base[:, None, :] + offs[None]).reshape(-1, 3) % int(60 / Q)
    k = np.concatenate([k, extra], 0)
    cat = synth.Catalog(*(np.ascontiguousarray(k[:, a] * Q) for a in range(3)))
    edges = np.array([0.5, 1.0, 2.0, 3.0, 5.0, 7.0, 10.0])
    _say("lattice", mode, prec)
    d = native.to_device(cat)
    if mode == "xi":
        ref = oracle.xi(cat, edges, periodic=True, box=60.0)
        g = native.countpairs_xi(d, edges, precision=prec, periodic=True, boxsize=60.0)
    else:
        ref = oracle.wp(cat, edges, 8.0, 8, periodic=True, box=60.0)
        g = native.countpairs_wp(d, edges, 8.0, 8, precision=prec, periodic=True, boxsize=60.0)
    _check(g, ref, prec=prec)
    if prec == "fp32":
        assert g.stats["rechecks"] > 0


@pytest.mark.parametrize("e0", [0.0, 0.25])
def test_coincident_points(native, e0):
    """Coincident distinct points (separation 0) on a grid without wrapped
    cells: with a first edge of 0 they land in bin 0 (half-open from 0), with
    a positive first edge they are dropped.  Binary32 estimates of a zero
    separation carry rounding of either sign, so near E_0 = 0 they must still
    land in bin 0; lattice partners planted exactly on edges (and on pi edges)
    force binary64 rechecks.  xi (weighted and not), w_p and cross, both
    precisions, against the oracle."""
    rng = np.random.Generator(np.random.PCG64(71))
    q = 2.0 ** -6
    lq = int(420.0 / q)
    k = rng.integers(0, lq, (20_000, 3))
    # partners at edge distances (axis and 3-4-5 offsets) and exact duplicates
    base = k[rng.integers(0, len(k), 600)]
    offs = np.array([[32, 0, 0], [0, 64, 0], [0, 0, 128], [3 * 64, 4 * 64, 0],
                     [0, 3 * 128, 4 * 128], [640, 0, 0], [0, 0, 64 * 5]])
    extra = (base[:, None, :] + offs[None]).reshape(-1, 3) % lq
    dups = k[rng.integers(0, len(k), 500)]
    kk = np.concatenate([k, extra, dups], 0)
    w = rng.integers(1, 8, len(kk)) * 0.25
    cat = synth.Catalog(*(np.ascontiguousarray(kk[:, a] * q) for a in range(3)), w=w)
    edges = np.array([e0, 0.5, 1.0, 2.0, 3.0, 5.0, 10.0, 20.0])
    d = native.to_device(cat)
    ref = oracle.xi(cat, edges, periodic=True, box=420.0)
    refw = oracle.wp(cat, edges, 16.0, 16, periodic=True, box=420.0)
    other = synth.Catalog(cat.x[:5000].copy(), cat.y[:5000].copy(), cat.z[:5000].copy(),
                          cat.w[:5000].copy())
    refc = oracle.xi(cat, edges, periodic=True, box=420.0, other=other)
    if e0 == 0.0:
        # each duplicate adds at least one coincident pair, counted both ways
        assert ref.npairs[0] >= 2 * len(dups)
    for prec in ("fp64", "fp32"):
        _say("coincident", e0, prec)
        g = native.countpairs_xi(d, edges, precision=prec, periodic=True, boxsize=420.0)
        _check(g, ref, prec=prec)
        assert min(g.stats["grid"]) > 1
        if prec == "fp32":
            assert g.stats["rechecks"] > 0
        g = native.countpairs_xi(d, edges, precision=prec, periodic=True, boxsize=420.0,
                                 need_ravg=True)
        _check(g, ref, weighted=True, prec=prec)
        g = native.countpairs_wp(d, edges, 16.0, 16, precision=prec, periodic=True,
                                 boxsize=420.0)
        _check(g, refw, prec=prec)
        if prec == "fp32":
            assert g.stats["rechecks"] > 0
        g = native.countpairs_cross(d, native.to_device(other), edges, precision=prec,
                                    periodic=True, boxsize=420.0)
        _check(g, refc, prec=prec)


def test_full_box_total(native):
    """R_max beyond half the box: per-pair minimum image, N(N-1) in total."""
    cat = synth.uniform(3000, 420.0, seed=3)
    _say("full box")
    for prec in ("fp64", "fp32"):
        g = native.countpairs_xi(native.to_device(cat), [0.0, 100.0, 400.0], precision=prec,
                                 periodic=True, boxsize=420.0)
        assert int(g.npairs.sum()) == cat.n * (cat.n - 1)
        ref = oracle.xi(cat, [0.0, 100.0, 400.0], periodic=True, box=420.0)
        _check(g, ref, prec=prec)
        g = native.countpairs_wp(native.to_device(cat), [0.0, 50.0, 300.0], 211.0, 3,
                                 precision=prec, periodic=True, boxsize=420.0)
        assert int(g.npairs.sum()) == cat.n * (cat.n - 1)


@pytest.mark.parametrize("refine", [(1, 1, 1), (2, 2, 2), (3, 3, 3), (3, 3, 1), (1, 2, 4), (8, 8, 8), (8, 1, 3)])
def test_refine_factors(native, refine):
    """Refine factors up to the cap of 8 cells per R_max (a half-shell of 145
    neighbour columns at (8, 8, 8), cut into the most chunks a tile may have),
    anisotropic ones included."""
    cat = synth.clustered(40_000, 800, 1.5, 420.0, seed=5)
    edges = synth.log_edges(0.1, 25.0, 14)
    _say("refine", refine)
    ref = oracle.xi(cat, edges, periodic=True, box=420.0)
    refw = oracle.wp(cat, edges, 40.0, 40, periodic=True, box=420.0)
    d = native.to_device(cat)
    for prec in ("fp32", "fp64"):
        g = native.countpairs_xi(d, edges, precision=prec, periodic=True, boxsize=420.0,
                                 refine=refine)
        _check(g, ref, prec=prec)
        g = native.countpairs_wp(d, edges, 40.0, 40, precision=prec, periodic=True,
                                 boxsize=420.0, refine=refine)
        _check(g, refw, prec=prec)


@pytest.mark.parametrize("refine", [(1, 1, 1), (2, 2, 2), (3, 1, 2)])
def test_nonperiodic_auto(native, refine):
    """Auto-counts without periodic wrap: the half-shell meets the edges of
    the catalogue's bounding box (columns and cells beyond it are skipped),
    on a clustered catalogue stretched to a non-cubic region."""
    c = synth.clustered(8_000, 200, 2.0, 200.0, seed=51, weights=True)
    cat = synth.Catalog(c.x - 20.0, c.y * 0.75 + 5.0, c.z * 0.5, c.w)
    edges = synth.log_edges(0.5, 20.0, 10)
    d = native.to_device(cat)
    ref = oracle.xi(cat, edges, periodic=False)
    refw = oracle.wp(cat, edges, 15.0, 5, periodic=False)
    for prec in ("fp64", "fp32"):
        _say("nonperiodic auto", refine, prec)
        g = native.countpairs_xi(d, edges, precision=prec, periodic=False, refine=refine,
                                 need_ravg=True)
        _check(g, ref, weighted=True, prec=prec, periodic=False)
        g = native.countpairs_wp(d, edges, 15.0, 5, precision=prec, periodic=False,
                                 refine=refine)
        _check(g, refw, prec=prec, periodic=False)


@pytest.mark.parametrize("rmax,refine,expect_r", [
    (120.0, (1, 1, 1), (1, 1, 1)),     # 3 cells per axis: exactly 2 r + 1
    (150.0, (2, 2, 2), (2, 2, 2)),     # 5 cells per axis: exactly 2 r + 1
    (150.0, (2, 1, 3), (2, 0, 3)),     # 5 cells, one wrapped cell, 8 cells
])
def test_minimal_periodic_grids(native, rmax, refine, expect_r):
    """Periodic grids at the edge of the no-aliasing condition (an axis with
    exactly 2 r + 1 cells, where the neighbour offsets -r..r reach every cell
    of the axis once), mixed with a single wrapped cell: the auto-count's
    half-shell must still meet every pair of cells once, and the cross count
    every pair."""
    a = synth.clustered(3_000, 60, 2.0, 420.0, seed=41, weights=True)
    b = synth.uniform(2_000, 420.0, seed=42, weights=True)
    edges = synth.log_edges(1.0, rmax, 8)
    da, db = native.to_device(a), native.to_device(b)
    for prec in ("fp64", "fp32"):
        _say("minimal grid", rmax, refine, prec)
        g = native.countpairs_xi(da, edges, precision=prec, periodic=True, boxsize=420.0,
                                 refine=refine, need_ravg=True)
        assert tuple(g.stats["refine"]) == expect_r
        _check(g, oracle.xi(a, edges, periodic=True, box=420.0), weighted=True, prec=prec)
        g = native.countpairs_wp(da, edges, 60.0, 6, precision=prec, periodic=True,
                                 boxsize=420.0, refine=refine)
        _check(g, oracle.wp(a, edges, 60.0, 6, periodic=True, box=420.0), prec=prec)
        g = native.countpairs_cross(da, db, edges, precision=prec, periodic=True, boxsize=420.0,
                                    refine=refine)
        _check(g, oracle.xi(a, edges, periodic=True, box=420.0, other=b), prec=prec)


@pytest.mark.parametrize("rmax", [80.0, 100.0])
def test_large_rmax(native, rmax):
    """R_max of 80 and 100 in a box of 420 (the top of the paper's R_max
    scaling range): 5 or 4 cells per axis at refine 1, so the neighbour reach
    of a cell wraps most of the periodic box; w_p with pi_max = R_max and
    1-wide pi bins."""
    cat = synth.clustered(20_000, 400, 1.5, 420.0, seed=31)
    edges = synth.log_edges(0.1, rmax, 14)
    npi = int(rmax)
    ref = oracle.xi(cat, edges, periodic=True, box=420.0)
    refw = oracle.wp(cat, edges, rmax, npi, periodic=True, box=420.0)
    d = native.to_device(cat)
    for refine in ((1, 1, 1), (2, 2, 2), (3, 3, 1)):
        for prec in ("fp64", "fp32"):
            _say("large rmax", rmax, refine, prec)
            g = native.countpairs_xi(d, edges, precision=prec, periodic=True, boxsize=420.0,
                                     refine=refine)
            _check(g, ref, prec=prec)
            g = native.countpairs_wp(d, edges, rmax, npi, precision=prec, periodic=True,
                                     boxsize=420.0, refine=refine)
            _check(g, refw, prec=prec)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_dense_cell_unsorted_path(native, prec):
    """A cluster of 9000 points inside one cell (more than the 4096 points up
    to which cells are z-sorted): that cell keeps its grouped order and is
    searched whole, its neighbours are sorted and cut to z-windows; counts and
    weighted sums still match the oracle."""
    rng = np.random.Generator(np.random.PCG64(41))
    n1, n2 = 9000, 6000
    c = np.array([200.0, 210.0, 220.0])
    dense = c + rng.normal(scale=1.2, size=(n1, 3))
    spread = rng.uniform(150.0, 270.0, (n2, 3))
    p = np.concatenate([dense, spread], 0) % 420.0
    w = rng.uniform(0.5, 1.5, len(p))
    cat = synth.Catalog(*(np.ascontiguousarray(p[:, a]) for a in range(3)), w=w)
    edges = synth.log_edges(0.1, 25.0, 14)
    _say("dense cell", prec)
    ref = oracle.xi(cat, edges, periodic=True, box=420.0)
    d = native.to_device(cat)
    for refine in [(1, 1, 1), (2, 2, 2)]:
        g = native.countpairs_xi(d, edges, precision=prec, periodic=True, boxsize=420.0,
                                 refine=refine, need_ravg=True)
        _check(g, ref, weighted=True, prec=prec)
        g = native.countpairs_xi(d, edges, precision=prec, periodic=True, boxsize=420.0,
                                 refine=refine)
        _check(g, ref, prec=prec)
    refw = oracle.wp(cat, edges, 40.0, 40, periodic=True, box=420.0)
    g = native.countpairs_wp(d, edges, 40.0, 40, precision=prec, periodic=True, boxsize=420.0,
                             refine=(1, 1, 1))
    _check(g, refw, prec=prec)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_dense_cell_sorted_path(native, prec):
    """Clusters of 700 and 2500 points, each inside one cell at refine 1 (below
    the 4096-point z-sort limit): their z order takes several LDS stages of
    the z-order pass and spans several position windows, some points share
    their z exactly (ties broken by grouped position); counts, weighted sums
    and the bounding-box tests agree with the oracle and with pruning off."""
    rng = np.random.Generator(np.random.PCG64(43))
    c1, c2 = np.array([212.5, 212.5, 212.5]), np.array([87.5, 312.5, 137.5])
    a = c1 + rng.normal(scale=0.8, size=(2500, 3))
    b = c2 + rng.normal(scale=0.5, size=(700, 3))
    b[::7, 2] = b[0, 2]                       # exact z ties inside one cell
    spread = rng.uniform(100.0, 330.0, (5000, 3))
    p = np.concatenate([a, b, spread], 0) % 420.0
    w = rng.uniform(0.5, 1.5, len(p))
    cat = synth.Catalog(*(np.ascontiguousarray(p[:, k]) for k in range(3)), w=w)
    edges = synth.log_edges(0.1, 25.0, 14)
    _say("dense sorted cell", prec)
    ref = oracle.xi(cat, edges, periodic=True, box=420.0)
    d = native.to_device(cat)
    for refine in [(1, 1, 1), (2, 2, 2)]:
        g = native.countpairs_xi(d, edges, precision=prec, periodic=True, boxsize=420.0,
                                 refine=refine, need_ravg=True)
        _check(g, ref, weighted=True, prec=prec)
        g = native.countpairs_xi(d, edges, precision=prec, periodic=True, boxsize=420.0,
                                 refine=refine)
        _check(g, ref, prec=prec)
        h = native.countpairs_xi(d, edges, precision=prec, periodic=True, boxsize=420.0,
                                 refine=refine, no_prune=True)
        _check(h, ref, prec=prec)
        assert g.stats["cell_pairs_pruned"] > 0
    refw = oracle.wp(cat, edges, 40.0, 40, periodic=True, box=420.0)
    for refine in [(1, 1, 1), (2, 2, 1)]:
        g = native.countpairs_wp(d, edges, 40.0, 40, precision=prec, periodic=True,
                                 boxsize=420.0, refine=refine)
        _check(g, refw, prec=prec)


def test_build_paths_agree(native, monkeypatch):
    """The two ways of grouping points by cell -- LDS column histograms (grids
    of up to 8192 columns) and one device-scope atomic per point (any grid) --
    give the same counts and weighted sums, for auto and cross counts,
    periodic and not, xi and w_p, float64 and float32 inputs."""
    cat = synth.clustered(40_000, 800, 1.5, 420.0, seed=12, weights=True)
    rnd = synth.to_float32(synth.uniform(30_000, 420.0, seed=13, weights=True))
    edges = synth.log_edges(0.1, 25.0, 14)
    d, r = native.to_device(cat), native.to_device(rnd)
    out = {}
    for path in ("1", "0"):
        monkeypatch.setenv("CP_BUILD_COLUMNS", path)
        _say("build path", path)
        res = [native.countpairs_xi(d, edges, precision="fp32", periodic=True, boxsize=420.0,
                                    need_ravg=True, refine=(2, 2, 2)),
               native.countpairs_wp(d, edges, 40.0, 40, precision="fp32", periodic=True,
                                    boxsize=420.0, refine=(2, 2, 1)),
               native.countpairs_xi(d, edges, precision="fp64", periodic=False, refine=(2, 2, 2)),
               native.countpairs_cross(d, r, edges, precision="fp32", periodic=False,
                                       need_ravg=True, refine=(2, 2, 2))]
        out[path] = res
    for a, b in zip(out["1"], out["0"]):
        assert (a.npairs == b.npairs).all()
        if a.wsum is not None:
            np.testing.assert_allclose(a.wsum, b.wsum, rtol=1e-12, atol=0)
            np.testing.assert_allclose(a.ravg, b.ravg, rtol=1e-12, atol=0)
    ref = oracle.xi(cat, edges, periodic=False, other=rnd)
    _check(out["1"][3], ref, weighted=True, prec="fp32", periodic=False)


def test_plan_build_paths_agree(native, monkeypatch):
    """Plans build all catalogues' cells with the column kernels at once
    (catalogue = blockIdx.y, a matrix and scan segment each, an empty
    catalogue among them); the atomic grouping (CP_BUILD_COLUMNS=0) gives the
    same counts, and both equal single calls."""
    cats = _mock_set()
    cats.append(synth.Catalog(np.zeros(0), np.zeros(0), np.zeros(0), None))
    xe = synth.log_edges(0.1, 25.0, 14)
    devs = [native.to_device(c) for c in cats]
    out = {}
    for path in ("1", "0"):
        monkeypatch.setenv("CP_BUILD_COLUMNS", path)
        _say("plan build path", path)
        for prec in ("fp32", "fp64"):
            plan = native.Plan(devs, xi_edges=xe, wp_edges=xe, pimax=40.0, npibins=40,
                               precision=prec, periodic=True, boxsize=420.0, refine=(2, 2, 2))
            plan.execute()
            out[path, prec] = plan.results()
            plan.close()
    for prec in ("fp32", "fp64"):
        for a, b in zip(out["1", prec], out["0", prec]):
            assert (a == b).all()
    xi, wp = out["1", "fp32"]
    assert xi[-1].sum() == 0 and wp[-1].sum() == 0
    for m in range(len(cats) - 1):
        s = native.countpairs_xi(devs[m], xe, precision="fp64", periodic=True, boxsize=420.0)
        assert (s.npairs == xi[m]).all()
        s = native.countpairs_wp(devs[m], xe, 40.0, 40, precision="fp64", periodic=True,
                                 boxsize=420.0)
        assert (s.npairs == wp[m]).all()


def test_unique_mode_and_pruning_stats(native):
    cat = synth.clustered(30_000, 600, 1.5, 420.0, seed=6)
    edges = synth.log_edges(0.1, 25.0, 14)
    d = native.to_device(cat)
    _say("unique")
    o = native.countpairs_xi(d, edges, periodic=True, boxsize=420.0)
    u = native.countpairs_xi(d, edges, periodic=True, boxsize=420.0, count_mode="unique")
    assert (o.npairs == 2 * u.npairs).all()
    assert o.stats["cell_pairs_pruned"] > 0


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_pruning_off_equals_on(native, prec):
    """The bounding-box tests of Section 2.2 (unit skipping, z-window, whole-unit
    counts) only leave out pairs that cannot be in range: with them switched
    off every count is unchanged and still equals the oracle."""
    cat = synth.clustered(40_000, 800, 1.5, 420.0, seed=12, weights=True)
    edges = synth.log_edges(0.1, 25.0, 14)
    d = native.to_device(cat)
    ref = oracle.xi(cat, edges, periodic=True, box=420.0)
    for refine in ((2, 2, 3), (1, 1, 1), (3, 3, 1)):
        _say("prune on/off xi", prec, refine)
        kw = dict(precision=prec, periodic=True, boxsize=420.0, refine=refine)
        on = native.countpairs_xi(d, edges, need_ravg=True, **kw)
        off = native.countpairs_xi(d, edges, need_ravg=True, no_prune=True, **kw)
        _check(on, ref, weighted=True, prec=prec)
        _check(off, ref, weighted=True, prec=prec)
        assert on.stats["cell_pairs_pruned"] > 0
        assert off.stats["cell_pairs_pruned"] == 0
        assert off.stats["candidates"] > on.stats["candidates"]
        u_on = native.countpairs_xi(d, edges, **kw)
        u_off = native.countpairs_xi(d, edges, no_prune=True, **kw)
        _check(u_on, ref, prec=prec)
        _check(u_off, ref, prec=prec)
    _say("prune on/off wp", prec)
    refw = oracle.wp(cat, edges, 40.0, 40, periodic=True, box=420.0)
    for flag in (False, True):
        g = native.countpairs_wp(d, edges, 40.0, 40, precision=prec, periodic=True,
                                 boxsize=420.0, no_prune=flag)
        _check(g, refw, prec=prec)
    _say("prune on/off cross", prec)
    rcat = synth.uniform(60_000, 420.0, seed=13)
    refc = oracle.xi(cat, edges, periodic=False, other=rcat)
    dr = native.to_device(rcat)
    for flag in (False, True):
        g = native.countpairs_cross(d, dr, edges, precision=prec, periodic=False, no_prune=flag)
        _check(g, refc, prec=prec, periodic=False)


def test_maximum_bins(native):
    """The largest histograms: 60 xi bins (weighted), a 60 x 256 w_p histogram
    (64 KB per wave, so the kernel runs fewer waves per workgroup), a weighted
    w_p of 20 x 100 bins (three waves per workgroup), and a weighted 60 x 256
    w_p, whose per-wave histograms cannot fit the LDS: a clean error."""
    cat = synth.clustered(30_000, 600, 1.5, 420.0, seed=44, weights=True)
    d = native.to_device(cat)
    e60 = synth.log_edges(0.1, 25.0, 60)
    ref = oracle.xi(cat, e60, periodic=True, box=420.0)
    for prec in ("fp64", "fp32"):
        _say("max bins xi", prec)
        g = native.countpairs_xi(d, e60, precision=prec, periodic=True, boxsize=420.0,
                                 need_ravg=True)
        _check(g, ref, weighted=True, prec=prec)
    refw = oracle.wp(cat, e60, 40.0, 256, periodic=True, box=420.0)
    for prec in ("fp64", "fp32"):
        _say("max bins wp", prec)
        g = native.countpairs_wp(d, e60, 40.0, 256, precision=prec, periodic=True, boxsize=420.0)
        _check(g, refw, prec=prec)
    e20 = synth.log_edges(0.1, 25.0, 20)
    refw = oracle.wp(cat, e20, 40.0, 100, periodic=True, box=420.0)
    for prec in ("fp64", "fp32"):
        _say("weighted wp 20 x 100", prec)
        g = native.countpairs_wp(d, e20, 40.0, 100, precision=prec, periodic=True,
                                 boxsize=420.0, need_ravg=True)
        _check(g, refw, weighted=True, prec=prec)
    with pytest.raises(native.CountpairsError, match="LDS"):
        native.countpairs_wp(d, e60, 40.0, 256, periodic=True, boxsize=420.0, need_ravg=True)


def test_tiny_inputs(native):
    import torch
    edges = [0.0, 1.0, 2.0]
    _say("tiny")
    for n in (0, 1, 2, 5):
        cat = synth.uniform(n, 3.0, seed=n)
        for prec in ("fp32", "fp64"):
            g = native.countpairs_xi(native.to_device(cat), edges, precision=prec,
                                     periodic=True, boxsize=3.0)
            ref = oracle.xi(cat, edges, periodic=True, box=3.0)
            _check(g, ref, prec=prec)
            g = native.countpairs_xi(native.to_device(cat), edges, precision=prec,
                                     periodic=False)
            ref = oracle.xi(cat, edges, periodic=False)
            _check(g, ref, prec=prec, periodic=False)


def test_device_errors(native):
    import torch
    cat = synth.uniform(1000, 10.0, seed=1)
    d = native.to_device(cat)
    d.x[5] = 10.0      # == box: outside [0, L)
    with pytest.raises(native.CountpairsError) as e:
        native.countpairs_xi(d, [0.1, 1.0], periodic=True, boxsize=10.0)
    assert e.value.code == -2
    d = native.to_device(cat)
    d.y[7] = float("nan")
    with pytest.raises(native.CountpairsError) as e:
        native.countpairs_xi(d, [0.1, 1.0], periodic=True, boxsize=10.0)
    assert e.value.code == -3
    with pytest.raises(native.CountpairsError) as e:
        native.countpairs_xi(d, [0.1, 1.0], periodic=False)
    assert e.value.code == -3
    # the library stays usable after an error
    d = native.to_device(cat)
    g = native.countpairs_xi(d, [0.1, 1.0], periodic=True, boxsize=10.0)
    _check(g, oracle.xi(cat, [0.1, 1.0], periodic=True, box=10.0))


def test_repeatable_counts(native):
    cat = synth.clustered(50_000, 1000, 1.5, 420.0, seed=8)
    edges = synth.log_edges(0.1, 25.0, 14)
    d = native.to_device(cat)
    a = native.countpairs_xi(d, edges, periodic=True, boxsize=420.0)
    b = native.countpairs_xi(d, edges, periodic=True, boxsize=420.0)
    c = native.countpairs_xi(d, edges, periodic=True, boxsize=420.0, precision="fp64")
    assert (a.npairs == b.npairs).all() and (a.npairs == c.npairs).all()


def _mock_set(nm=6, seed=40):
    rng = np.random.Generator(np.random.PCG64(seed))
    cats = []
    for m in range(nm):
        n = int(rng.integers(20_000, 80_000))
        cats.append(synth.clustered(n, max(1, n // 50), float(rng.uniform(0.5, 3.0)), 420.0,
                                    seed=seed + m))
    return cats


def test_plan_matches_oracle(native):
    cats = _mock_set()
    xe = synth.log_edges(0.1, 25.0, 14)
    we = synth.log_edges(0.1, 25.0, 14)
    devs = [native.to_device(c) for c in cats]
    _say("plan")
    for prec in ("fp32", "fp64"):
        plan = native.Plan(devs, xi_edges=xe, wp_edges=we, pimax=40.0, npibins=40,
                           precision=prec, periodic=True, boxsize=420.0)
        plan.execute()
        xi, wp = plan.results()
        for m in (0, 3, 5):
            _check(type("G", (), {"npairs": xi[m]})(), oracle.xi(cats[m], xe, True, 420.0))
            _check(type("G", (), {"npairs": wp[m]})(),
                   oracle.wp(cats[m], we, 40.0, 40, periodic=True, box=420.0))
        for m in range(len(cats)):
            s = native.countpairs_xi(devs[m], xe, precision=prec, periodic=True, boxsize=420.0)
            assert (s.npairs == xi[m]).all()
        plan.close()


@pytest.mark.parametrize("case", ["fused", "xi_beyond_pimax"])
def test_plan_fused_xi_wp(native, monkeypatch, case):
    """Binary32 plans count xi and w_p in one launch over the w_p search when
    every xi pair lies inside it (xi R_max <= r_p,max and <= pi_max): the
    results equal the two-launch plan (CP_PLAN_FUSED=0), the oracle and single
    calls, bit for bit, own cells and exact z ties included.  With xi R_max
    above pi_max the plan keeps two launches and agrees as well."""
    cats = _mock_set()
    # exact z ties and a dense cluster: own-cell pairs and the xi bands
    cats[0].z[::5] = cats[0].z[0]
    xe = synth.log_edges(0.1, 25.0, 14)
    we = synth.log_edges(0.1, 25.0, 14)
    pimax = 40.0 if case == "fused" else 20.0
    devs = [native.to_device(c) for c in cats]
    _say("plan fused", case)
    out = {}
    for fused in ("1", "0"):
        monkeypatch.setenv("CP_PLAN_FUSED", fused)
        plan = native.Plan(devs, xi_edges=xe, wp_edges=we, pimax=pimax, npibins=40,
                           precision="fp32", periodic=True, boxsize=420.0, refine=(2, 2, 2))
        plan.execute()
        out[fused] = plan.results()
        sx, sw = plan.stats()
        assert sx["precision"] == "fp32" and sw["precision"] == "fp32"
        plan.close()
    assert (out["1"][0] == out["0"][0]).all()
    assert (out["1"][1] == out["0"][1]).all()
    xi, wp = out["1"]
    for m in (0, 2, 5):
        _check(type("G", (), {"npairs": xi[m]})(), oracle.xi(cats[m], xe, True, 420.0))
        _check(type("G", (), {"npairs": wp[m]})(),
               oracle.wp(cats[m], we, pimax, 40, periodic=True, box=420.0))
    for m in range(len(cats)):
        s = native.countpairs_xi(devs[m], xe, precision="fp32", periodic=True, boxsize=420.0)
        assert (s.npairs == xi[m]).all(), m
        s = native.countpairs_wp(devs[m], we, pimax, 40, precision="fp32", periodic=True,
                                 boxsize=420.0)
        assert (s.npairs == wp[m]).all(), m


def test_plan_pruning_off_equals_on(native):
    """The plan path with the bounding-box tests switched off gives the same
    counts for every catalogue and statistic."""
    cats = _mock_set()
    xe = synth.log_edges(0.1, 25.0, 14)
    devs = [native.to_device(c) for c in cats]
    _say("plan prune on/off")
    res = []
    for flag in (False, True):
        plan = native.Plan(devs, xi_edges=xe, wp_edges=xe, pimax=40.0, npibins=40,
                           precision="fp32", periodic=True, boxsize=420.0, no_prune=flag)
        plan.execute()
        res.append(plan.results())
        plan.close()
    assert (res[0][0] == res[1][0]).all() and (res[0][1] == res[1][1]).all()


def test_plan_graph_replays(native):
    """Replays of the captured graph, with eager work in between, all equal
    the eager result."""
    import torch
    cats = _mock_set(4, seed=60)
    xe = synth.log_edges(0.1, 25.0, 14)
    devs = [native.to_device(c) for c in cats]
    eager = [native.countpairs_xi(d, xe, periodic=True, boxsize=420.0).npairs for d in devs]
    plan = native.Plan(devs, xi_edges=xe, wp_edges=xe, pimax=40.0, npibins=40, periodic=True,
                       boxsize=420.0)
    for rep in range(4):
        plan.execute()
        xi, _ = plan.results()
        for m in range(len(devs)):
            assert (xi[m] == eager[m]).all(), (rep, m)
        # eager work between replays
        native.countpairs_xi(devs[rep % len(devs)], xe, periodic=True, boxsize=420.0)
        torch.cuda.synchronize()
    # refill a catalogue in place: the next replay sees the new points
    new = synth.clustered(devs[1].n, 500, 2.5, 420.0, seed=99)
    devs[1].x.copy_(torch.from_numpy(new.x))
    devs[1].y.copy_(torch.from_numpy(new.y))
    devs[1].z.copy_(torch.from_numpy(new.z))
    plan.execute()
    xi, _ = plan.results()
    _check(type("G", (), {"npairs": xi[1]})(), oracle.xi(new, xe, True, 420.0))
    plan.close()


def test_autotuned_refine_same_counts(native, tmp_path, monkeypatch):
    """refine = 0 through the C ABI: the library times candidate settings on
    the call's data (refine factors, work-chunk target, waves per workgroup),
    writes its JSON cache, reuses the choice on the next call of the same
    signature; counts equal the oracle either way.  CP_AUTOTUNE=0 gives the
    library defaults; an explicit refine is used as given."""
    import json
    cache = tmp_path / "at.json"
    monkeypatch.setenv("CP_AUTOTUNE_CACHE", str(cache))
    cat = synth.clustered(40_000, 800, 1.5, 420.0, seed=12, weights=True)
    edges = synth.log_edges(0.1, 25.0, 14)
    d = native.to_device(cat)
    ref = oracle.xi(cat, edges, periodic=True, box=420.0)
    refw = oracle.wp(cat, edges, 40.0, 40, periodic=True, box=420.0)
    _say("autotune xi")
    g = native.countpairs_xi(d, edges, periodic=True, boxsize=420.0, need_ravg=True)
    _check(g, ref, weighted=True)
    assert g.stats["tuned"] == "tuned", g.stats
    text = cache.read_text()
    json.loads(text)                          # the cache file is valid JSON
    entries = [l for l in text.splitlines() if l.strip().startswith('"xi/')]
    assert len(entries) == 1 and "/w/p/" in entries[0]
    assert '"refine": [' in entries[0] and '"chunk_pct": ' in entries[0]
    g2 = native.countpairs_xi(d, edges, periodic=True, boxsize=420.0, need_ravg=True)
    _check(g2, ref, weighted=True)
    assert g2.stats["tuned"] == "cached"
    assert g2.stats["refine"] == g.stats["refine"] and g2.stats["chunk_pct"] == g.stats["chunk_pct"]
    _say("autotune wp")
    g = native.countpairs_wp(d, edges, 40.0, 40, periodic=True, boxsize=420.0)
    _check(g, refw, prec="fp32")
    assert g.stats["tuned"] == "tuned"
    monkeypatch.setenv("CP_AUTOTUNE", "0")
    g = native.countpairs_xi(d, edges, periodic=True, boxsize=420.0, precision="fp64")
    _check(g, ref)
    assert g.stats["tuned"] == "default" and g.stats["refine"] == [2, 2, 2]
    monkeypatch.delenv("CP_AUTOTUNE")
    g = native.countpairs_xi(d, edges, periodic=True, boxsize=420.0, refine=(3, 3, 1))
    _check(g, ref)
    assert g.stats["tuned"] == "given" and g.stats["refine"] == [3, 3, 1]
    _say("autotune plan")
    other = synth.clustered(30_000, 600, 2.0, 420.0, seed=13)
    plan = native.Plan([d, native.to_device(other)], xi_edges=edges, wp_edges=edges, pimax=40.0,
                       npibins=40, periodic=True, boxsize=420.0)
    plan.execute()
    xi, wp = plan.results()
    sx, sw = plan.stats()
    assert sx["tuned"] == "tuned" and sw["tuned"] == "tuned"
    assert (xi[0] == ref.npairs).all() and (wp[0] == refw.npairs).all()
    assert (xi[1] == oracle.xi(other, edges, periodic=True, box=420.0).npairs).all()
    plan.close()
    assert any(l.strip().startswith('"plan:') for l in cache.read_text().splitlines())


def test_caller_workspace(native):
    import torch
    cat = synth.clustered(30_000, 600, 1.5, 420.0, seed=14)
    r = synth.uniform(40_000, 420.0, seed=15)
    edges = synth.log_edges(0.1, 25.0, 14)
    d, dr = native.to_device(cat), native.to_device(r)
    nbytes = native.workspace_size("cross", cat.n, r.n, edges, periodic=False)
    ws = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    g = native.countpairs_cross(d, dr, edges, periodic=False, workspace=ws)
    _check(g, oracle.xi(cat, edges, periodic=False, other=r))
    nbytes = native.workspace_size("xi", cat.n, 0, edges, periodic=True, boxsize=420.0)
    ws = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    g = native.countpairs_xi(d, edges, periodic=True, boxsize=420.0, workspace=ws)
    _check(g, oracle.xi(cat, edges, periodic=True, box=420.0))
    small = torch.empty(4096, dtype=torch.uint8, device="cuda")
    with pytest.raises(native.CountpairsError) as e:
        native.countpairs_xi(d, edges, periodic=True, boxsize=420.0, workspace=small)
    assert e.value.code == -4
