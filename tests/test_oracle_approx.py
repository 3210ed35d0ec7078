"""Pins for the oracle's sign-function approximants.

* Jacobi elliptic functions and K against scipy (independent library routine).
* Closed forms: the degree-0 minimax polynomial and the one-pole Zolotarev
  approximant.
* Alternation certificates (Chebyshev / Zolotarev optimality): the minimax
  error 1 - sqrt(y) P(y) of Eq. 6 equioscillates at n+2 points; Zolotarev's
  1 - r(x) at 2n+1 points.
"""
import math

import numpy as np
import pytest
import scipy.special as ss

from oracle import approx


@pytest.mark.parametrize("u,m", [(0.3, 0.5), (1.7, 0.99), (2.5, 0.9917), (0.01, 0.999999), (3.0, 0.1)])
def test_elliptic_vs_scipy(u, m):
    sn, cn, dn = approx.ellipj(u, m)
    ref = ss.ellipj(u, m)
    assert abs(sn - ref[0]) < 1e-14 and abs(cn - ref[1]) < 1e-14 and abs(dn - ref[2]) < 1e-14
    assert abs(approx.ellipk(m) - ss.ellipk(m)) < 1e-13 * ss.ellipk(m)


def _alternation_levels(err, delta):
    """Peak |err| of each maximal run of equal sign among the grid points where
    |err| > delta/2 (robust to rounding noise near flat extrema).  Consecutive
    runs alternate in sign by construction; their number counts alternation
    points."""
    sel = np.abs(err) > 0.5 * delta
    e = err[sel]
    s = np.sign(e)
    cuts = np.nonzero(s[1:] != s[:-1])[0] + 1
    return np.array([np.abs(run).max() for run in np.split(e, cuts)])


def test_minimax_degree0_closed_form():
    # min_c max_{eps<=y<=1} |1 - c sqrt(y)|:  c = 2/(1+sqrt(eps)), delta = (1-sqrt(eps))/(1+sqrt(eps))
    eps = 0.01
    p = approx.minimax_polynomial(eps, 0)
    assert abs(p.c[0] - 2 / (1 + math.sqrt(eps))) < 1e-12
    assert abs(p.delta - (1 - math.sqrt(eps)) / (1 + math.sqrt(eps))) < 1e-12


@pytest.mark.parametrize("eps,n", [(0.0909 ** 2, 12), (0.0909 ** 2, 60), (0.05 ** 2, 40), (0.2 ** 2, 25)])
def test_minimax_equioscillation(eps, n):
    p = approx.minimax_polynomial(eps, n)
    th = np.linspace(0, np.pi, 200001)
    y = 0.5 * ((1 - eps) * np.cos(th) + 1 + eps)
    e = p.h(y)
    peaks = _alternation_levels(e, p.delta)
    assert len(peaks) >= n + 2, "fewer than n+2 alternation points"
    assert np.all(peaks > (1 - 1e-6) * p.delta)
    assert abs(np.abs(e).max() - p.delta) < 1e-6 * p.delta
    # optimality: beats Chebyshev interpolation of 1/sqrt(y) of the same degree
    z = np.cos(np.pi * (np.arange(n + 1) + 0.5) / (n + 1))
    yi = 0.5 * ((1 - eps) * z + 1 + eps)
    c_int = np.polynomial.chebyshev.chebfit(z, 1 / np.sqrt(yi), n)
    e_int = 1 - np.sqrt(y) * np.polynomial.chebyshev.chebval((2 * y - 1 - eps) / (1 - eps), c_int)
    assert p.delta < np.abs(e_int).max()


def test_minimax_converges_geometrically():
    eps = 0.0909 ** 2
    d = [approx.minimax_polynomial(eps, n).delta for n in (20, 40, 60)]
    assert d[0] > d[1] > d[2]
    rate = d[2] / d[1]
    assert rate < math.exp(-2 * 20 * math.sqrt(eps)) * 1.5


def test_zolotarev_one_pole_closed_form():
    # n = 1: sigma = k, r(x) = D x/(x^2 + k), delta = (1 - sqrt k)^2 / (1 + sqrt k)^2
    k = 0.09
    r = approx.zolotarev(k, 1)
    assert abs(r.sigma[0] - k) < 1e-14
    assert abs(r.delta - (1 - math.sqrt(k)) ** 2 / (1 + math.sqrt(k)) ** 2) < 1e-12


@pytest.mark.parametrize("k,n", [(0.0909, 5), (0.0909, 10), (0.05, 10), (0.3, 4), (0.0909, 6)])
def test_zolotarev_equioscillation(k, n):
    r = approx.zolotarev(k, n)
    x = np.geomspace(k, 1.0, 400001)
    e = 1 - r(x)
    peaks = _alternation_levels(e, r.delta)
    assert len(peaks) >= 2 * n + 1
    assert np.all(peaks > (1 - 1e-6) * r.delta - 1e-14)   # rounding of 1 - r(x) ~ 1e-15
    assert abs(np.abs(e).max() - r.delta) < 1e-6 * r.delta + 1e-14
    assert np.all(r.sigma > 0) and np.all(np.diff(r.sigma) > 0) and np.all(r.beta > 0)


def test_zolotarev_poles_vs_scipy():
    k, n = 0.0909, 8
    r = approx.zolotarev(k, n)
    m1 = 1 - k * k
    kk = ss.ellipk(m1)
    u = (2 * np.arange(1, n + 1) - 1) * kk / (2 * n)
    sn, cn, _, _ = ss.ellipj(u, m1)
    assert np.allclose(r.sigma, k * k * sn ** 2 / cn ** 2, rtol=1e-12, atol=0)


def test_zolotarev_error_decreases():
    d = [approx.zolotarev(0.0909, n).delta for n in (5, 6, 8, 10)]
    assert all(a > b for a, b in zip(d, d[1:]))
    assert d[-1] < 1e-10


@pytest.mark.parametrize("k,n", [(0.0932, 260), (0.0932, 400)])
def test_minimax_at_rounding_floor(k, n):
    """Degrees whose optimum error is below double-precision noise: the result
    must still approximate (regression: the exchange once chased noise extrema)."""
    p = approx.minimax_polynomial(k * k, n)
    y = np.linspace(k * k, 1.0, 200001)
    assert np.abs(p.h(y)).max() < 1e-13
