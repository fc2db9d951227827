"""Seeded synthetic catalogues shared by the tests, the benchmark and the oracle.

This module only draws random numbers and lays them out; it holds none of the
pair-counting arithmetic.  Both the HIP path and the CPU oracle are fed from
here, so a difference between them can never come from their inputs.

The paper benchmarks on a 1.2-million-galaxy catalogue in a periodic box of
side 420 with R_max = 25 (Section 3.1, Section 3.2); that catalogue is not
available, so Neyman-Scott clustered points of the same box, size and scale
stand in for it (Poisson(mean) children around uniform parents, conditioned on
the exact total N, which makes the child counts multinomial).

All generators use numpy's PCG64 bit generator and return float64 SoA arrays.
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import Optional

import numpy as np

BOX = 420.0


@dataclass
class Catalog:
    x: np.ndarray
    y: np.ndarray
    z: np.ndarray
    w: Optional[np.ndarray] = None

    @property
    def n(self) -> int:
        return int(self.x.shape[0])

    def astype(self, dtype) -> "Catalog":
        return Catalog(self.x.astype(dtype), self.y.astype(dtype), self.z.astype(dtype),
                       None if self.w is None else self.w.copy())

    def subset(self, idx) -> "Catalog":
        return Catalog(self.x[idx].copy(), self.y[idx].copy(), self.z[idx].copy(),
                       None if self.w is None else self.w[idx].copy())


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def _wrap(v: np.ndarray, box: float) -> np.ndarray:
    v = np.mod(v, box)
    v[v >= box] = 0.0  # np.mod can round a tiny negative up to exactly box
    return v


def uniform(n: int, box: float = BOX, seed: int = 1, weights: bool = False) -> Catalog:
    """n points uniform in [0, box)^3."""
    rng = _rng(seed)
    p = rng.uniform(0.0, box, (n, 3))
    w = rng.uniform(0.5, 1.5, n) if weights else None
    return Catalog(np.ascontiguousarray(p[:, 0]), np.ascontiguousarray(p[:, 1]),
                   np.ascontiguousarray(p[:, 2]), w)


def clustered(n: int, nparents: int, sigma: float, box: float = BOX, seed: int = 2,
              weights: bool = False) -> Catalog:
    """Neyman-Scott process: nparents uniform centres, children offset by an
    isotropic Gaussian of width sigma, wrapped into the periodic box, shuffled.
    Weights, when asked for, are U(0.5, 1.5) and are drawn last."""
    rng = _rng(seed)
    parents = rng.uniform(0.0, box, (nparents, 3))
    counts = rng.multinomial(n, np.full(nparents, 1.0 / nparents))
    pts = np.repeat(parents, counts, axis=0) + rng.normal(0.0, sigma, (n, 3))
    pts = _wrap(pts, box)
    pts = pts[rng.permutation(n)]
    w = rng.uniform(0.5, 1.5, n) if weights else None
    return Catalog(np.ascontiguousarray(pts[:, 0]), np.ascontiguousarray(pts[:, 1]),
                   np.ascontiguousarray(pts[:, 2]), w)


def lattice(n: int, box: float = BOX, quantum: float = 2.0 ** -10, seed: int = 7,
            weights: bool = False, duplicates: int = 0) -> Catalog:
    """Points on the grid quantum * k (k integer) inside [0, box), so every
    coordinate difference and every squared separation below 2^53 quantum^2 is
    exact in binary64.  `duplicates` copies of earlier points are appended."""
    rng = _rng(seed)
    kmax = int(np.floor(box / quantum))
    k = rng.integers(0, kmax, (n, 3))
    if duplicates:
        k = np.concatenate([k, k[rng.integers(0, n, duplicates)]], axis=0)
    p = k.astype(np.float64) * quantum
    w = None
    if weights:
        w = rng.integers(1, 8, p.shape[0]).astype(np.float64) * 0.25
    return Catalog(np.ascontiguousarray(p[:, 0]), np.ascontiguousarray(p[:, 1]),
                   np.ascontiguousarray(p[:, 2]), w)


def to_float32(cat: Catalog, box: float = BOX) -> Catalog:
    """float32 copy of the positions; a coordinate that rounds up to the box
    side is moved to the largest float32 below it (stays inside [0, box))."""
    out = []
    top = np.float32(box)
    below = np.nextafter(top, np.float32(0))
    for v in (cat.x, cat.y, cat.z):
        f = v.astype(np.float32)
        f[f >= top] = below
        out.append(np.ascontiguousarray(f))
    return Catalog(out[0], out[1], out[2], None if cat.w is None else cat.w.copy())


def log_edges(lo: float, hi: float, nbins: int) -> np.ndarray:
    """nbins + 1 log-spaced separation edges (computed once, float64)."""
    return np.logspace(np.log10(lo), np.log10(hi), nbins + 1)


# ---------------------------------------------------------------- workloads

def config1() -> dict:
    """xi(r) auto-count: 10^4 uniform points, periodic L = 420, 20 log bins
    over [0.1, 20], unweighted, FP64."""
    return dict(cat=uniform(10_000, BOX, seed=1), edges=log_edges(0.1, 20.0, 20),
                periodic=True, box=BOX)


def config2(n: int = 1_000_000, nparents: int = 20_000, seed: int = 2) -> dict:
    """xi(r) auto-count: Neyman-Scott 10^6 points (2*10^4 parents, mean 50
    children, sigma 1.5), periodic L = 420, 14 log bins over [0.1, 25],
    weights U(0.5, 1.5) with the weighted mean separation per bin."""
    return dict(cat=clustered(n, nparents, 1.5, BOX, seed=seed, weights=True),
                edges=log_edges(0.1, 25.0, 14), periodic=True, box=BOX)


def config3(n: int = 1_000_000, nparents: int = 20_000, seed: int = 2) -> dict:
    """wp(rp) 2-D histogram on the config-2 catalogue (line of sight z),
    14 log rp bins over [0.1, 25], pi_max = 40 in 40 unit pi bins, unweighted."""
    cat = clustered(n, nparents, 1.5, BOX, seed=seed, weights=False)
    return dict(cat=cat, edges=log_edges(0.1, 25.0, 14), pimax=40.0, npibins=40,
                periodic=True, box=BOX)


def config4(nd: int = 1_000_000, nr: int = 10_000_000) -> dict:
    """cross count DR, non-periodic: D = float32 of the config-2 catalogue,
    R = float32 of 10^7 uniform points in the same cube."""
    d = to_float32(clustered(nd, max(1, nd // 50), 1.5, BOX, seed=2))
    r = to_float32(uniform(nr, BOX, seed=4))
    return dict(d=d, r=r, edges=log_edges(0.1, 25.0, 14), periodic=False, box=BOX)


def mock_specs(nmocks: int = 256, seed: int = 5, nmin: int = 200_000,
               nmax: int = 2_000_000) -> list:
    """(N_m, sigma_m, seed_m) for the batched workload: N ~ U{nmin..nmax},
    sigma ~ U(0.5, 3), parents = round(N / 50)."""
    rng = _rng(seed)
    ns = rng.integers(nmin, nmax + 1, nmocks)
    sig = rng.uniform(0.5, 3.0, nmocks)
    return [(int(ns[m]), float(sig[m]), 1000 + m) for m in range(nmocks)]


def mock(spec) -> Catalog:
    n, sigma, seed = spec
    return clustered(n, max(1, int(round(n / 50))), sigma, BOX, seed=seed)
