"""countpairs_xi_noalloc (the entry point without allocation, on the library's
static device scratch) against countpairs_xi through the C ABI: identical
counts, weighted sums within 1e-12, over two calls in a row (the second on a
smaller catalogue, so stale scratch contents from the first must not leak),
in both precisions; no change in free device memory across calls; clean
errors for a call too large for the static scratch and for a workspace."""
import numpy as np
import pytest

from paper_1911_08275_amd import synth

pytestmark = pytest.mark.gpu

RTOL = 1e-12


@pytest.fixture(scope="module")
def native():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1911_08275_amd import native
    native.lib()
    return native


def _same(a, b, weighted):
    assert (a.npairs == b.npairs).all(), (a.npairs, b.npairs)
    if weighted:
        np.testing.assert_allclose(a.wsum, b.wsum, rtol=RTOL, atol=0)
        np.testing.assert_allclose(a.ravg, b.ravg, rtol=RTOL, atol=0)


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_noalloc_matches_xi(native, prec):
    import torch
    edges = synth.log_edges(0.1, 25.0, 14)
    big = synth.clustered(200_000, 4000, 1.5, 420.0, seed=61, weights=True)
    small = synth.clustered(30_000, 600, 2.5, 420.0, seed=62, weights=True)
    kw = dict(precision=prec, periodic=True, boxsize=420.0)
    db, ds = native.to_device(big), native.to_device(small)
    print("noalloc", prec, flush=True)
    # first a large call, then a smaller one on the same scratch
    for d in (db, ds):
        for w in (True, False):
            ref = native.countpairs_xi(d, edges, need_ravg=w, **kw)
            got = native.countpairs_xi_noalloc(d, edges, need_ravg=w, **kw)
            _same(got, ref, w)
            # weighted xi runs binary64 in either mode
            assert got.stats["precision"] == ("fp64" if w else prec)
            assert got.stats["candidates"] == ref.stats["candidates"]
    # a non-periodic call uses the scratch for the bounding-box reduction too
    ref = native.countpairs_xi(ds, edges, precision=prec, periodic=False, need_ravg=True)
    got = native.countpairs_xi_noalloc(ds, edges, precision=prec, periodic=False, need_ravg=True)
    _same(got, ref, True)
    # no device allocation across calls (after the calls above warmed up)
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    for d in (db, ds):
        native.countpairs_xi_noalloc(d, edges, need_ravg=True, **kw)
    torch.cuda.synchronize()
    assert torch.cuda.mem_get_info()[0] == free0


def test_noalloc_limits(native):
    import torch
    edges = synth.log_edges(0.1, 25.0, 14)
    cat = synth.uniform(2_000_000, 420.0, seed=63)
    d = native.to_device(cat)
    print("noalloc limits", flush=True)
    with pytest.raises(native.CountpairsError) as e:
        native.countpairs_xi_noalloc(d, edges, periodic=True, boxsize=420.0)
    assert e.value.code == -4 and "static scratch" in e.value.detail
    ws = torch.empty(1 << 20, dtype=torch.uint8, device="cuda")
    small = native.to_device(synth.uniform(1000, 420.0, seed=64))
    with pytest.raises(native.CountpairsError) as e:
        native.countpairs_xi_noalloc(small, edges, periodic=True, boxsize=420.0, workspace=ws)
    assert e.value.code == -1
    # the entry point still works after the failures
    ref = native.countpairs_xi(small, edges, periodic=True, boxsize=420.0)
    got = native.countpairs_xi_noalloc(small, edges, periodic=True, boxsize=420.0)
    assert (got.npairs == ref.npairs).all()
