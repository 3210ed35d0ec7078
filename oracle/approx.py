"""Sign-function approximants -- oracle (test infrastructure only).

Two families, both for x = lambda / |Q| with sqrt(eps) <= |x| <= 1:

* Minimax polynomial (Sec. 2.2, Eq. 5 and Eq. 6): sign(x) ~ x P(x^2) with
  P(y) = sum_{k=0}^{n} c_k T_k(z),  z = (2y - 1 - eps) / (1 - eps),
  chosen to minimise delta = max_{eps <= y <= 1} |1 - sqrt(y) P(y)|.
  The paper writes P_n = sum c_k T_k without naming the interval map; the
  affine map of [eps, 1] onto [-1, 1] above is the reading used, and the sum
  uses the full c_0 (no halved first term).  Computed with the Remez exchange
  algorithm for the weight sqrt(y).
* Zolotarev's optimal rational approximant (not in the paper; used for the
  rational variant of the sign function):
  r(x) = x sum_{l=1}^{n} beta_l / (x^2 + sigma_l),
  sigma_l = k^2 sn^2(u; k') / cn^2(u; k') at u = (2l-1) K(k') / (2n),
  numerator zeros at u = 2l K(k') / (2n), k' = sqrt(1 - k^2), k = sqrt(eps),
  with the overall scale fixed so that the relative error equioscillates.

Jacobi elliptic functions and K are computed with the arithmetic-geometric
mean and descending Landen transformation (DLMF 22.20(ii), 19.8(i)).
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

# ----------------------------------------------------------------------------
# Elliptic functions
# ----------------------------------------------------------------------------


def _agm_sequence(m: float):
    """AGM sequence for parameter m = k^2: a_0 = 1, b_0 = sqrt(1 - m), c_0 = sqrt(m)."""
    a = [1.0]
    b = math.sqrt(1.0 - m)
    c = [math.sqrt(m)]
    while abs(c[-1]) > 1e-17 * a[-1] and len(a) < 64:
        an, bn = a[-1], b
        a.append(0.5 * (an + bn))
        c.append(0.5 * (an - bn))
        b = math.sqrt(an * bn)
    return a, c


def ellipk(m: float) -> float:
    """Complete elliptic integral of the first kind K(m) = pi / (2 AGM(1, sqrt(1-m)))."""
    a, _ = _agm_sequence(m)
    return math.pi / (2.0 * a[-1])


def ellipj(u: float, m: float):
    """Jacobi sn, cn, dn at argument u and parameter m = k^2 (descending Landen)."""
    a, c = _agm_sequence(m)
    n = len(a) - 1
    phi = (2.0 ** n) * a[n] * u
    for j in range(n, 0, -1):
        phi = 0.5 * (phi + math.asin(c[j] * math.sin(phi) / a[j]))
    sn = math.sin(phi)
    cn = math.cos(phi)
    dn = math.sqrt(1.0 - m * sn * sn)
    return sn, cn, dn


# ----------------------------------------------------------------------------
# Zolotarev rational approximant
# ----------------------------------------------------------------------------


@dataclass
class Rational:
    k: float            # lower end of the approximation interval [k, 1]
    sigma: np.ndarray   # shifts (poles in x^2), ascending
    beta: np.ndarray    # residues
    delta: float        # max |1 - r(x)| on [k, 1]

    def __call__(self, x):
        x = np.asarray(x, dtype=np.float64)
        return x * np.sum(self.beta / (x[..., None] ** 2 + self.sigma), axis=-1)


def _turning_points(d: np.ndarray) -> np.ndarray:
    """Interior grid indices i where the differences d = diff(values) turn:
    d[i-1] > 0 >= d[i] (maximum) or d[i-1] < 0 <= d[i] (minimum)."""
    a, b = d[:-1], d[1:]
    return np.nonzero(((a > 0) & (b <= 0)) | ((a < 0) & (b >= 0)))[0] + 1


def _local_extrema(f, lo: float, hi: float, npts: int = 20000, log: bool = True):
    """All local extrema of f on [lo, hi] (endpoints included), refined by golden section."""
    t = np.geomspace(lo, hi, npts) if log else np.linspace(lo, hi, npts)
    v = f(t)
    d = np.diff(v)
    idx = [0] + list(_turning_points(d)) + [len(t) - 1]
    pts = []
    gr = (math.sqrt(5) - 1) / 2
    for i in idx:
        if i in (0, len(t) - 1):
            pts.append(t[i])
            continue
        a, b = t[i - 1], t[i + 1]
        sgn = 1.0 if v[i] > v[i - 1] else -1.0  # maximum or minimum
        for _ in range(100):
            x1 = b - gr * (b - a)
            x2 = a + gr * (b - a)
            if sgn * f(np.array([x1]))[0] > sgn * f(np.array([x2]))[0]:
                b = x2
            else:
                a = x1
            if b - a < 1e-15 * max(1.0, abs(b)):
                break
        pts.append(0.5 * (a + b))
    return np.array(pts)


def zolotarev(k: float, n: int) -> Rational:
    """Optimal rational approximation of sign(x) on [k, 1] with n poles in x^2."""
    if not (0.0 < k < 1.0) or n < 1:
        raise ValueError("need 0 < k < 1 and n >= 1")
    kp2 = 1.0 - k * k
    big_k = ellipk(kp2)
    c = np.empty(2 * n)
    for j in range(1, 2 * n):
        sn, cn, _ = ellipj(j * big_k / (2 * n), kp2)
        c[j] = sn * sn / (cn * cn)
    sigma = k * k * c[1:2 * n:2]          # j = 1, 3, ..., 2n-1
    zeros = k * k * c[2:2 * n:2]          # j = 2, 4, ..., 2n-2

    def g(x):
        x = np.asarray(x, dtype=np.float64)[..., None]
        num = np.prod(x * x + zeros, axis=-1) if zeros.size else 1.0
        return x[..., 0] * num / np.prod(x * x + sigma, axis=-1)

    ext = _local_extrema(g, k, 1.0)
    gv = g(ext)
    gmax, gmin = gv.max(), gv.min()
    scale = 2.0 / (gmax + gmin)
    delta = (gmax - gmin) / (gmax + gmin)
    beta = np.empty(n)
    for l in range(n):
        num = np.prod(zeros - sigma[l]) if zeros.size else 1.0
        den = np.prod(np.delete(sigma, l) - sigma[l])
        beta[l] = scale * num / den
    return Rational(k=k, sigma=sigma, beta=beta, delta=float(delta))


# ----------------------------------------------------------------------------
# Minimax polynomial in the Chebyshev basis (Eq. 5, Eq. 6)
# ----------------------------------------------------------------------------


@dataclass
class Polynomial:
    eps: float          # approximation interval [eps, 1] in y = x^2
    c: np.ndarray       # Chebyshev coefficients c_0..c_n (full c_0)
    delta: float        # max |1 - sqrt(y) P(y)| on [eps, 1]

    def z(self, y):
        return (2.0 * np.asarray(y, dtype=np.float64) - 1.0 - self.eps) / (1.0 - self.eps)

    def P(self, y):
        return _cheb_eval(self.c, self.z(y))

    def h(self, y):
        """Eq. 6: h(y) = 1 - sqrt(y) P(y)."""
        y = np.asarray(y, dtype=np.float64)
        return 1.0 - np.sqrt(y) * self.P(y)

    def __call__(self, x):
        x = np.asarray(x, dtype=np.float64)
        return x * self.P(x * x)


def _cheb_matrix(n: int, z: np.ndarray) -> np.ndarray:
    """T_k(z) for k = 0..n, shape [len(z), n+1], by the defining recurrence."""
    t = np.empty((z.size, n + 1))
    t[:, 0] = 1.0
    if n >= 1:
        t[:, 1] = z
    for k in range(2, n + 1):
        t[:, k] = 2.0 * z * t[:, k - 1] - t[:, k - 2]
    return t


def _cheb_eval(c: np.ndarray, z) -> np.ndarray:
    z = np.atleast_1d(np.asarray(z, dtype=np.float64))
    return _cheb_matrix(len(c) - 1, z.ravel()) @ c


def _alternating_subset(pts: np.ndarray, vals: np.ndarray, count: int):
    """Reduce a sorted list of extrema to ``count`` points of alternating sign,
    keeping the largest |vals| (multiple-exchange Remez step)."""
    p, v = list(pts), list(vals)
    # merge consecutive points of equal sign, keep the larger magnitude
    i = 0
    while i < len(p) - 1:
        if np.sign(v[i]) == np.sign(v[i + 1]):
            drop = i if abs(v[i]) < abs(v[i + 1]) else i + 1
            del p[drop], v[drop]
        else:
            i += 1
    # drop from the ends (smaller end first) until the count fits
    while len(p) > count:
        if abs(v[0]) < abs(v[-1]):
            del p[0], v[0]
        else:
            del p[-1], v[-1]
    return np.array(p), np.array(v)


ROUNDING_FLOOR = 1e-13   # max |h| at which double-precision evaluation noise dominates


def _golden_refine(f, lo: np.ndarray, hi: np.ndarray, sgn: np.ndarray, iters: int = 60):
    """Golden-section search of sgn*f for a maximum inside each bracket [lo, hi],
    all brackets at once."""
    gr = (math.sqrt(5) - 1) / 2
    lo = lo.copy()
    hi = hi.copy()
    for _ in range(iters):
        x1 = hi - gr * (hi - lo)
        x2 = lo + gr * (hi - lo)
        left = sgn * f(x1) > sgn * f(x2)
        hi = np.where(left, x2, hi)
        lo = np.where(left, lo, x1)
    return 0.5 * (lo + hi)


def minimax_polynomial(eps: float, n: int, tol: float = 1e-7, max_iter: int = 60) -> Polynomial:
    """Weighted Remez exchange for min over P of max_{eps<=y<=1} |1 - sqrt(y) P(y)|.

    The error of the optimum equioscillates at n+2 points of [eps, 1] (the
    alternation theorem for the positive weight sqrt(y)).  Start: the
    reference points are the n+2 Chebyshev extrema of T_{n+1} mapped onto
    [eps, 1]; each step solves sqrt(y_i) P(y_i) + (-1)^i E = 1 for (c, E),
    locates all extrema of the new error on a fine grid in theta = arccos z
    with golden-section refinement, and exchanges the reference.  Stops when
    the largest error exceeds the levelled error |E| by less than ``tol``
    (relative).
    """
    if not (0.0 < eps < 1.0) or n < 0:
        raise ValueError("need 0 < eps < 1 and n >= 0")

    def y_of_theta(th):
        return 0.5 * ((1.0 - eps) * np.cos(th) + 1.0 + eps)

    m = n + 2
    theta_ref = np.pi * np.arange(m)[::-1] / (m - 1)
    yref = y_of_theta(theta_ref)
    poly = None
    best = None
    for _ in range(max_iter):
        zr = (2.0 * yref - 1.0 - eps) / (1.0 - eps)
        a = np.empty((m, m))
        a[:, : n + 1] = np.sqrt(yref)[:, None] * _cheb_matrix(n, zr)
        a[:, n + 1] = (-1.0) ** np.arange(m)
        sol = np.linalg.solve(a, np.ones(m))
        poly = Polynomial(eps=eps, c=sol[: n + 1], delta=abs(sol[n + 1]))
        lev = abs(sol[n + 1])

        def err_theta(th, poly=poly):
            return poly.h(y_of_theta(th))

        npts = max(4000, 40 * m)
        th = np.linspace(0.0, np.pi, npts)
        ev = err_theta(th)
        inner = _turning_points(np.diff(ev))
        t_in = _golden_refine(err_theta, th[inner - 1], th[inner + 1], np.sign(ev[inner]))
        pts = np.concatenate([[th[0]], t_in, [th[-1]]])
        vals = err_theta(pts)
        order = np.argsort(-pts)          # y ascending
        pts, vals = pts[order], vals[order]
        emax = float(np.max(np.abs(vals)))
        poly.delta = emax
        # Eq. 6 asks for the smallest max |h|: keep the best iterate.  Once the
        # error reaches the rounding floor of double precision the extrema are
        # rounding noise and further exchanges only degrade the reference.
        if best is None or emax < best.delta:
            best = poly
        if emax - lev <= tol * emax or emax <= ROUNDING_FLOOR:
            break
        sel_t, _ = _alternating_subset(pts, vals, m)
        if len(sel_t) < m:
            break
        yref = y_of_theta(sel_t)
    return best


def eval_forward_recurrence(poly: Polynomial, apply_z, psi: np.ndarray) -> np.ndarray:
    """sum_k c_k T_k(Z) psi with the forward three-term recurrence
    T_0 psi = psi, T_1 psi = Z psi, T_{k+1} psi = 2 Z T_k psi - T_{k-1} psi."""
    t_prev = psi
    out = poly.c[0] * psi
    if len(poly.c) == 1:
        return out
    t_cur = apply_z(psi)
    out = out + poly.c[1] * t_cur
    for k in range(2, len(poly.c)):
        t_next = 2.0 * apply_z(t_cur) - t_prev
        out = out + poly.c[k] * t_next
        t_prev, t_cur = t_cur, t_next
    return out
