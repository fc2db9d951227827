"""Closed-form correlation function of the Neyman-Scott generator
(paper_1911_08275_amd.synth.clustered), used as a pin of the estimators.

With P parents uniform in a periodic cube of side L and N children split
among them by a multinomial draw, a fraction 1/P of the N(N-1) ordered pairs
are siblings, whose separation is Maxwell-distributed with scale
a = sigma sqrt(2) (each axis the difference of two Gaussians); all other
pairs are uniform over the cube.  Per bin:
    xi_k  = -1/P + L^3 (F(e_k+1) - F(e_k)) / (P V_k),
    w_p,k = -2 pi_max / P + L^3 (G(e_k) - G(e_k+1)) erf(pi_max / (a sqrt 2)) / (P A_k),
F the Maxwell CDF, G(r) = exp(-r^2 / 2a^2) the tail of the projected
(2-D Rayleigh) separation, V_k the shell volume, A_k the annulus area.
"""
import math

import numpy as np


def _maxwell_cdf(r, a):
    return math.erf(r / (a * math.sqrt(2.0))) - math.sqrt(2.0 / math.pi) * (r / a) * \
        math.exp(-r * r / (2.0 * a * a))


def ns_xi(edges, nparents, sigma, box):
    a = sigma * math.sqrt(2.0)
    out = []
    for lo, hi in zip(edges[:-1], edges[1:]):
        vol = 4.0 / 3.0 * math.pi * (hi ** 3 - lo ** 3)
        p = _maxwell_cdf(hi, a) - _maxwell_cdf(lo, a)
        out.append(-1.0 / nparents + box ** 3 * p / (nparents * vol))
    return np.array(out)


def ns_wp(edges, pimax, nparents, sigma, box):
    a = sigma * math.sqrt(2.0)
    out = []
    for lo, hi in zip(edges[:-1], edges[1:]):
        area = math.pi * (hi * hi - lo * lo)
        p = math.exp(-lo * lo / (2 * a * a)) - math.exp(-hi * hi / (2 * a * a))
        p *= math.erf(pimax / (a * math.sqrt(2.0)))
        out.append(-2.0 * pimax / nparents + box ** 3 * p / (nparents * area))
    return np.array(out)


def ns_tolerance(want, rr, vol, parents, box):
    """Allowed |measured - expected| of xi per bin: 3 % of xi (the sibling
    pair total fluctuates by ~1 %), five standard deviations of the bin's
    ordered pair count (variance ~2 E), and five of the count of distinct
    cluster pairs the bin samples (pairs of different clusters come in
    clumps of ~m^2)."""
    expect = rr * (1.0 + want)
    return (0.03 * np.abs(want) + 5.0 * np.sqrt(2.0 * expect) / rr +
            5.0 / np.sqrt(parents * parents * vol / box ** 3))
