"""Two-sided pins of the low-mode diagnostics of Sec. 2.3 (Eq. 8, Eq. 9, Eq. 10)
on a planted spectrum whose values are worked out by hand.

Q = W diag(lambda) W^H on C^8 with a fixed unitary W and the planted eigenvalues
lambda = (-4, -3, -0.35, 0.3, 2, 2.5, 5, 6); the two modes of smallest |lambda|
are the wanted ones and every other eigenvalue has |lambda| >= 2.  The
approximate subspace is spanned by

    v_+ = cos(t) w(0.3) + sin(t) w(5),        v_- = cos(f) w(-0.35) + sin(f) w(-3),

(w(x) the eigenvector of x).  Q maps span(w(0.3), w(5)) and span(w(-0.35), w(-3))
into themselves, so the Rayleigh-Ritz matrix on span(v_+, v_-) is diagonal and,
by hand:

    nu_+  = 0.3 cos^2 t + 5 sin^2 t,          rho_+ = |5 - 0.3| sin t cos t,
    nu_-  = -0.35 cos^2 f - 3 sin^2 f,        rho_- = |-3 + 0.35| sin f cos f,

(Eq. 8: rho = |(Q - nu) v| = |a - b| sin cos for v = cos w(a) + sin w(b)).  d_k
(the reading of the garbled sentence of Sec. 2.3) is the distance of nu_k from
the spectrum of Q on the complement of the exact projector of its own sign:
that spectrum holds the opposite-sign wanted eigenvalue and every |lambda| >= 2,
so with the Ritz estimates in place of the exact values

    d_k = min(2 - |nu_k|, |nu_k| + |nu_j|)  (j the opposite-sign mode).

With t = 0.01, f = 0.02 the opposite-sign distance |nu_+| + |nu_-| ~ 0.65 is the
smaller one for both modes, so a d_k that forgets it is off by a factor ~2.6.
kappa_+ = rho_+ / d_+ and kappa_- = rho_- / d_- (Eq. 9: one mode of each sign),
and |P_+ - (P_+)_exact| = sin t exactly (two rank-one projectors at angle t),
which Eq. 10 must bound.  A second planted case has two positive modes and no
negative one, where the gap term lam_next - |nu_k| decides.

Each pin is checked against the oracle, and plausible mistakes (the opposite-sign
distance dropped, kappa summed over both signs, d_k not squared, the (1 + 2 kappa)
factor of Eq. 10 dropped) are planted and must fail at least one pin.
"""
import numpy as np
import pytest

from oracle import lowmodes

LAM = np.array([-4.0, -3.0, -0.35, 0.3, 2.0, 2.5, 5.0, 6.0])
T, F = 0.01, 0.02


def _unitary(n, seed):
    rng = np.random.default_rng(seed)
    z = rng.normal(size=(n, n)) + 1j * rng.normal(size=(n, n))
    qm, r = np.linalg.qr(z)
    return qm * (np.diag(r) / np.abs(np.diag(r)))


def _planted(lam, pairs):
    """Q = W diag(lam) W^H and the basis vectors cos(a) w(x) + sin(a) w(y) for
    each (x, y, a) in pairs (columns of W are the eigenvectors w)."""
    w = _unitary(len(lam), 7)
    q = (w * lam) @ w.conj().T
    col = {x: w[:, i] for i, x in enumerate(lam)}
    basis = np.stack([np.cos(a) * col[x] + np.sin(a) * col[y] for x, y, a in pairs])
    return q, basis, col


def _case_two_signs():
    q, basis, col = _planted(LAM, [(0.3, 5.0, T), (-0.35, -3.0, F)])
    # mix the two basis vectors so that Rayleigh-Ritz has to undo the mixing
    mix = _unitary(2, 11)
    basis = mix.T @ basis
    c, s, cf, sf = np.cos(T), np.sin(T), np.cos(F), np.sin(F)
    nu_p = 0.3 * c * c + 5.0 * s * s
    nu_m = -0.35 * cf * cf - 3.0 * sf * sf
    rho_p = (5.0 - 0.3) * s * c
    rho_m = (3.0 - 0.35) * sf * cf
    d_p = min(2.0 - nu_p, nu_p - nu_m)
    d_m = min(2.0 + nu_m, nu_p - nu_m)
    hand = {"nu": {1: nu_p, -1: nu_m}, "rho": {1: rho_p, -1: rho_m}, "d": {1: d_p, -1: d_m},
            "kappa": {1: rho_p / d_p, -1: rho_m / d_m},
            "exact": {1: col[0.3], -1: col[-0.35]}, "dev": {1: s, -1: sf}}
    return q, basis, 2.0, hand


def _case_one_sign():
    lam = np.array([-4.0, -2.6, 0.3, 1.9, 2.2, 2.5, 5.0, 6.0])
    t2, f2 = 0.004, 0.006
    q, basis, col = _planted(lam, [(0.3, 5.0, t2), (1.9, -4.0, f2)])
    c, s, cf, sf = np.cos(t2), np.sin(t2), np.cos(f2), np.sin(f2)
    nu = np.array([0.3 * c * c + 5.0 * s * s, 1.9 * cf * cf - 4.0 * sf * sf])
    rho = np.array([4.7 * s * c, 5.9 * sf * cf])
    d = 2.2 - nu            # no negative mode: only the gap term
    return q, basis, 2.2, {"nu": nu, "rho": rho, "d": d, "kappa": float(np.sqrt(np.sum((rho / d) ** 2)))}


def _bound_hand(k):
    q = k * (1 + 2 * k)
    return q / (1 - 2 * q)


def _ritz(q, basis):
    nu, u = lowmodes.rayleigh_ritz(lambda v: q @ v, basis)
    rho = lowmodes.residues(lambda v: q @ v, u, nu)
    return nu, u, rho


def _pin_failures(gap, kap, bound):
    """Evaluate every pin with the given diagnostic functions; return the failing ones."""
    bad = []
    q, basis, lam_next, h = _case_two_signs()
    nu, u, rho = _ritz(q, basis)
    d = gap(nu, lam_next)
    kp, km = kap(nu, rho, d)
    for k, n in enumerate(nu):
        sg = 1 if n > 0 else -1
        if abs(d[k] - h["d"][sg]) > 1e-12:
            bad.append(f"d[{sg}]")
    if abs(kp - h["kappa"][1]) > 1e-12 * h["kappa"][1] or abs(km - h["kappa"][-1]) > 1e-12 * h["kappa"][-1]:
        bad.append("kappa two signs")
    for sg, kk in ((1, kp), (-1, km)):
        if abs(bound(kk) - _bound_hand(h["kappa"][sg])) > 1e-12 * _bound_hand(h["kappa"][sg]):
            bad.append(f"bound[{sg}]")
        if not h["dev"][sg] <= bound(kk):
            bad.append(f"Eq. 10 violated [{sg}]")
    q1, b1, ln1, h1 = _case_one_sign()
    nu1, _, rho1 = _ritz(q1, b1)
    d1 = gap(nu1, ln1)
    kp1, km1 = kap(nu1, rho1, d1)
    if np.abs(d1 - h1["d"]).max() > 1e-12:
        bad.append("d one sign")
    if abs(kp1 - h1["kappa"]) > 1e-12 * h1["kappa"] or km1 != 0.0:
        bad.append("kappa one sign")
    return bad


def test_rayleigh_ritz_closed_form():
    """Eq. 8 pin: Ritz values and residues of the planted subspace equal their hand values."""
    q, basis, _, h = _case_two_signs()
    nu, u, rho = _ritz(q, basis)
    for k, n in enumerate(nu):
        sg = 1 if n > 0 else -1
        assert abs(n - h["nu"][sg]) < 1e-14
        assert abs(rho[k] - h["rho"][sg]) < 1e-14
        # the Ritz vector is the planted v (up to a phase)
        ex = h["exact"][sg]
        assert abs(abs(np.vdot(ex, u[k])) - np.cos(T if sg > 0 else F)) < 1e-14


def test_diagnostics_hand_values():
    """Eq. 9 and Eq. 10 pins: d_k, kappa_+-, the bound and the true projector
    deviation on both planted cases."""
    assert _pin_failures(lowmodes.gap_distances, lowmodes.kappas, lowmodes.projector_bound) == []
    q, basis, _, h = _case_two_signs()
    nu, u, _ = _ritz(q, basis)
    for sg in (1, -1):
        sel = (np.sign(nu) == sg)
        p = u[sel].T @ u[sel].conj()
        ex = h["exact"][sg][:, None]
        dev = np.linalg.norm(p - ex @ ex.conj().T, 2)
        assert abs(dev - h["dev"][sg]) < 1e-13


def _gap_no_opposite(nu, lam_next):
    return lam_next - np.abs(np.asarray(nu))


def _gap_plus(nu, lam_next):
    return lam_next + 0.0 * np.abs(np.asarray(nu)) - np.abs(np.asarray(nu)).min()


def _kappa_both_signs(nu, rho, d):
    k = float(np.sqrt(np.sum((rho / d) ** 2)))
    return k, k


def _kappa_not_squared(nu, rho, d):
    pos = nu > 0
    return float(np.sqrt(np.sum(rho[pos] / d[pos] ** 2))), float(np.sqrt(np.sum(rho[~pos] / d[~pos] ** 2)))


def _kappa_max(nu, rho, d):
    pos = nu > 0
    r = rho / d
    return float(r[pos].max(initial=0.0)) * 1.5 if pos.sum() > 1 else float(r[pos].sum()), float(r[~pos].sum())


def _bound_no_factor(k):
    return k / (1 - 2 * k)


def _bound_wrong_den(k):
    q = k * (1 + 2 * k)
    return q / (1 - q)


@pytest.mark.parametrize("mutant", ["gap_no_opposite", "gap_plus", "kappa_both_signs", "kappa_not_squared",
                                    "kappa_max", "bound_no_factor", "bound_wrong_den"])
def test_planted_mistakes_are_caught(mutant):
    gap, kap, bound = lowmodes.gap_distances, lowmodes.kappas, lowmodes.projector_bound
    if mutant.startswith("gap"):
        gap = {"gap_no_opposite": _gap_no_opposite, "gap_plus": _gap_plus}[mutant]
    elif mutant.startswith("kappa"):
        kap = {"kappa_both_signs": _kappa_both_signs, "kappa_not_squared": _kappa_not_squared,
               "kappa_max": _kappa_max}[mutant]
    else:
        bound = {"bound_no_factor": _bound_no_factor, "bound_wrong_den": _bound_wrong_den}[mutant]
    assert _pin_failures(gap, kap, bound), f"mutant {mutant} passed every pin"


def test_certified_lower_gap_is_conservative():
    """With the rest of the spectrum known only as a Ritz value lam and residue r
    of a guard vector, Q has an eigenvalue in [lam - r, lam + r]; passing the
    lower end lam - r as lam_next can only shrink d_k and grow kappa, so the
    Eq. 10 bound stays valid.  Guard: cos(g) w(2) + sin(g) w(6)."""
    q, basis, _, h = _case_two_signs()
    nu, u, rho = _ritz(q, basis)
    lam = np.sort(np.abs(LAM))
    w = np.linalg.eigh(q)[1]
    vals = np.linalg.eigh(q)[0]
    g = 0.05
    guard = np.cos(g) * w[:, np.argmin(np.abs(vals - 2.0))] + np.sin(g) * w[:, np.argmin(np.abs(vals - 6.0))]
    lam_g = np.vdot(guard, q @ guard).real
    r_g = np.linalg.norm(q @ guard - lam_g * guard)
    assert abs(lam_g - (2.0 * np.cos(g) ** 2 + 6.0 * np.sin(g) ** 2)) < 1e-13
    assert abs(r_g - 4.0 * np.sin(g) * np.cos(g)) < 1e-13
    assert lam_g - r_g <= lam[2] <= lam_g + r_g
    d_lo = lowmodes.gap_distances(nu, lam_g - r_g)
    d_ex = lowmodes.gap_distances(nu, 2.0)
    assert np.all(d_lo <= d_ex + 1e-15)
    kp, km = lowmodes.kappas(nu, rho, d_lo)
    assert kp >= h["kappa"][1] - 1e-15 and km >= h["kappa"][-1] - 1e-15
