"""Correlation-function estimators of Section 1, written out in binary64.

TEST INFRASTRUCTURE ONLY, like the rest of this package: the tests, the smoke
check and the benchmark's CPU leg may use it; the library never does.

  rr_periodic_xi  random pairs of n points in a periodic cube: a partner of a
                  point is uniform over the cube, so an ordered pair lands in
                  the shell [e_k, e_k+1) with probability shell volume / L^3
                  (Section 1, analytic random counts for a periodic cube);
  rr_periodic_wp  the same for the (r_p, pi) bins: annulus area times the two
                  line-of-sight slabs of width dpi (pi = |dz|);
  xi_natural      eqn:xi, DD / RR - 1, each count over its own pair total;
  wp_integrate    twice the line-of-sight integral of xi(r_p, pi) (the w_p
                  equation of Section 1) as a sum over equal pi bins.

Pinned in tests/test_estimators.py against the closed-form correlation
function of the Neyman-Scott generator and against uniform catalogues.
"""
from __future__ import annotations

import math

import numpy as np


def _pairs(n: int, count_mode: str) -> float:
    total = float(n) * float(max(n - 1, 0))
    return total / 2.0 if count_mode == "unique" else total


def rr_periodic_xi(n: int, box: float, edges, count_mode: str = "ordered") -> np.ndarray:
    e = np.asarray(edges, dtype=np.float64)
    shell = np.array([4.0 / 3.0 * math.pi * (e[k + 1] ** 3 - e[k] ** 3)
                      for k in range(e.size - 1)])
    return _pairs(n, count_mode) * shell / box ** 3


def rr_periodic_wp(n: int, box: float, rp_edges, pimax: float, npibins: int,
                   count_mode: str = "ordered") -> np.ndarray:
    e = np.asarray(rp_edges, dtype=np.float64)
    dpi = pimax / npibins
    out = np.zeros((e.size - 1, npibins))
    for k in range(e.size - 1):
        annulus = math.pi * (e[k + 1] ** 2 - e[k] ** 2)
        for l in range(npibins):
            out[k, l] = _pairs(n, count_mode) * annulus * 2.0 * dpi / box ** 3
    return out


def xi_natural(dd, rr, dd_norm: float = 1.0, rr_norm: float = 1.0) -> np.ndarray:
    dd = np.asarray(dd, dtype=np.float64)
    rr = np.asarray(rr, dtype=np.float64)
    with np.errstate(divide="ignore", invalid="ignore"):
        out = (dd / dd_norm) / (rr / rr_norm) - 1.0
    return np.where(rr > 0, out, np.nan)


def wp_integrate(xi2d, pimax: float) -> np.ndarray:
    x = np.asarray(xi2d, dtype=np.float64)
    dpi = pimax / x.shape[1]
    return np.array([2.0 * sum(float(v) for v in row) * dpi for row in x])
