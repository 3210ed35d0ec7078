"""Pins for the oracle's sign(Q) (Eq. 5, Eq. 11), low-mode diagnostics (Eq. 7-10),
D_N (Eq. 4, Eq. 12) and the link force, all at 4^4 against dense linear algebra.
"""
import numpy as np
import pytest

import synthetic
from oracle import approx, dirac, force, geometry, lowmodes, overlap, sign

M = -1.4
S = 0.4
LMAX = 6.6


def _ops(d):
    dims = d.dims
    return lambda v: dirac.apply_Q(d.U, v.reshape(-1, 4, 3), M, dims).reshape(v.shape)


def test_exact_sign_properties(dense_random):
    sgn = sign.dense_sign_exact(dense_random.Q, eig=(dense_random.lam, dense_random.W))
    n = sgn.shape[0]
    assert np.abs(sgn @ sgn - np.eye(n)).max() < 1e-11
    assert np.abs(sgn - sgn.conj().T).max() < 1e-12
    assert np.abs(sgn @ dense_random.Q - dense_random.Q @ sgn).max() < 1e-11


def test_free_field_sign_closed_form(dense_cold):
    """For U = 1 and a plane wave, sign(Q) = Q(p)/|Q(p)| with Q(p) = gamma5 D_W(p)."""
    dims = dense_cold.dims
    g, g5 = dirac.gamma_matrices()
    x = geometry.coords(dims)
    nvec = np.array([1, 0, 3, 2])
    p = 2 * np.pi * nvec / np.array(dims)
    chi = np.arange(12).reshape(4, 3) + 1j
    psi = np.exp(1j * (x @ p))[:, None, None] * chi[None]
    dw = (M + np.sum(1 - np.cos(p))) * np.eye(4) + 1j * sum(np.sin(p[m]) * g[m] for m in range(4))
    qp = g5 @ dw
    mag = np.sqrt((M + np.sum(1 - np.cos(p))) ** 2 + np.sum(np.sin(p) ** 2))
    expect = np.einsum("st,vtc->vsc", qp / mag, psi).ravel()
    got = sign.dense_sign_exact(dense_cold.Q, eig=(dense_cold.lam, dense_cold.W)) @ psi.ravel()
    assert np.abs(got - expect).max() < 1e-11


@pytest.mark.parametrize("kind", ["rational", "polynomial"])
def test_sparse_sign_matches_dense(dense_tiny, kind):
    """Operator-form sign (stencil + CG per shift / forward recurrence) equals
    W f(Lambda) W^H, and is within delta |psi| of the exact sign (Sec. 2.2)."""
    d = dense_tiny
    eig = (d.lam, d.W)
    k = np.abs(d.lam[d.order[0]]) / LMAX
    appr = approx.zolotarev(k, 8) if kind == "rational" else approx.minimax_polynomial(k * k, 60)
    v = geometry.volume(d.dims)
    psi = synthetic.spinor(v)
    got = sign.sign_approx(_ops(d), psi, appr, LMAX)
    ref = sign.dense_sign_approx(d.Q, appr, LMAX, eig=eig) @ psi.ravel()
    assert np.linalg.norm(got.ravel() - ref) < 1e-11 * np.linalg.norm(psi)
    ex = sign.dense_sign_exact(d.Q, eig=eig) @ psi.ravel()
    assert np.linalg.norm(got.ravel() - ex) <= appr.delta * np.linalg.norm(psi) * (1 + 1e-6) + 1e-12


@pytest.mark.parametrize("form", ["literal", "sandwich"])
def test_projected_sign_exact_modes(dense_random, form):
    """Eq. 11 with exact eigenvectors equals W f(Lambda) W^H (f = sign on the l modes)."""
    l = 8
    eig = (dense_random.lam, dense_random.W)
    nu, modes = lowmodes.dense_lowmodes(dense_random.Q, l, eig=eig)
    lam_next = np.abs(dense_random.lam[dense_random.order[l]])
    rat = approx.zolotarev(lam_next / LMAX, 6)
    psi = synthetic.spinor(256)
    q = dense_random.Q
    ap = lambda v: sign.sign_rational(lambda w: (q @ w.ravel()).reshape(w.shape), v, rat, LMAX)
    fn = sign.project_literal if form == "literal" else sign.project_sandwich
    got = fn(ap, modes.reshape(l, 256, 4, 3), nu, psi).ravel()
    ref = sign.dense_sign_approx(q, rat, LMAX, n_low=l, eig=eig) @ psi.ravel()
    assert np.linalg.norm(got - ref) < 1e-9 * np.linalg.norm(psi)
    ex = sign.dense_sign_exact(q, eig=eig) @ psi.ravel()
    assert np.linalg.norm(got - ex) <= rat.delta * np.linalg.norm(psi) * 1.01 + 1e-9


@pytest.mark.parametrize("case", ["cold48", "random8"])
def test_rayleigh_ritz_and_projector_bound(dense_random, dense_cold, case):
    """Perturbed subspace: Eq. 10 bounds the deviation of P_+- from the exact projectors.

    cold48: the free field's 48 modes at |lambda| = 0.6 (gap to 1.077), noise 1e-5;
    random8: 8 lowest modes of the random field (no clear gap), noise 1e-9.
    """
    d = dense_cold if case == "cold48" else dense_random
    l, noise = (48, 1e-5) if case == "cold48" else (8, 1e-9)
    q = d.Q
    nu_ex, modes_ex = lowmodes.dense_lowmodes(q, l, eig=(d.lam, d.W))
    rng = np.random.default_rng(3)
    noisy = modes_ex + noise * (rng.normal(size=modes_ex.shape) + 1j * rng.normal(size=modes_ex.shape))
    apply_flat = lambda v: q @ v
    nu, u = lowmodes.rayleigh_ritz(apply_flat, noisy)
    rho = lowmodes.residues(apply_flat, u, nu)
    lam_next = np.abs(d.lam[d.order[l]])
    dist = lowmodes.gap_distances(nu, lam_next)
    kp, km = lowmodes.kappas(nu, rho, dist)
    assert 0 < kp < 0.1 and 0 < km < 0.1
    for sgn, kap in ((1, kp), (-1, km)):
        sel_ex = np.sign(nu_ex) == sgn
        p_ex = modes_ex[sel_ex].T @ modes_ex[sel_ex].conj()
        sel = np.sign(nu) == sgn
        p = u[sel].T @ u[sel].conj()
        dev = np.linalg.norm(p - p_ex, 2)
        assert 0 < dev <= lowmodes.projector_bound(kap)
    assert np.abs(np.sort(nu) - np.sort(nu_ex)).max() < 1e-5


def test_dn_bound_eq12(dense_random):
    """Eq. 12: |D~ - D| <= (2/a)(1 + s - m/2)(kappa_+ + kappa_-) with the exact sign on
    the complement, approximate projectors from a perturbed subspace."""
    l, mq = 8, 0.05
    q = dense_random.Q
    nu_ex, modes_ex = lowmodes.dense_lowmodes(q, l, eig=(dense_random.lam, dense_random.W))
    rng = np.random.default_rng(4)
    noisy = modes_ex + 1e-9 * (rng.normal(size=modes_ex.shape) + 1j * rng.normal(size=modes_ex.shape))
    nu, u = lowmodes.rayleigh_ritz(lambda v: q @ v, noisy)
    rho = lowmodes.residues(lambda v: q @ v, u, nu)
    lam_next = np.abs(dense_random.lam[dense_random.order[l]])
    kp, km = lowmodes.kappas(nu, rho, lowmodes.gap_distances(nu, lam_next))
    s_ex = sign.dense_sign_exact(q, eig=(dense_random.lam, dense_random.W))
    p = u.T @ u.conj()
    s_ap = (u.T * np.sign(nu)) @ u.conj() + (np.eye(q.shape[0]) - p) @ s_ex
    dm = overlap.dense_DN(s_ex, S, mq)
    dm_ap = overlap.dense_DN(s_ap, S, mq)
    dev = np.linalg.norm(dm_ap - dm, 2)
    assert dev <= lowmodes.dn_bound(kp, km, S, mq)


def test_ginsparg_wilson_and_circle(dense_random):
    s_ex = sign.dense_sign_exact(dense_random.Q, eig=(dense_random.lam, dense_random.W))
    d = overlap.dense_DN(s_ex, S)
    assert overlap.gw_residual(d, S) < 1e-10
    ev = np.linalg.eigvals(d)
    c = 1 / overlap.abar(S)
    assert np.abs(np.abs(ev - c) - c).max() < 1e-10
    n = d.shape[0]
    g5 = overlap.gamma5_dense(n // 12)
    assert np.abs(d.conj().T - g5 @ d @ g5).max() < 1e-11
    # approximate sign: GW holds to O(delta)
    lam_low = np.abs(dense_random.lam[dense_random.order[0]])
    rat = approx.zolotarev(lam_low / LMAX, 6)
    d_ap = overlap.dense_DN(sign.dense_sign_approx(dense_random.Q, rat, LMAX, eig=(dense_random.lam, dense_random.W)), S)
    r = overlap.gw_residual(d_ap, S)
    assert r < 10 * rat.delta * (1 + S) and r > 1e-3 * rat.delta


def test_free_field_dn_closed_form(dense_cold):
    """D_N(p) = (1/abar)(1 + D_W(p)/|D_W(p)|) for U = 1."""
    dims = dense_cold.dims
    g, _ = dirac.gamma_matrices()
    p = 2 * np.pi * np.array([2, 1, 0, 3]) / np.array(dims)
    x = geometry.coords(dims)
    chi = (np.arange(12) % 5).reshape(4, 3) - 2j
    psi = np.exp(1j * (x @ p))[:, None, None] * chi[None]
    dw = (M + np.sum(1 - np.cos(p))) * np.eye(4) + 1j * sum(np.sin(p[m]) * g[m] for m in range(4))
    mag = np.sqrt((M + np.sum(1 - np.cos(p))) ** 2 + np.sum(np.sin(p) ** 2))
    expect = np.einsum("st,vtc->vsc", (np.eye(4) + dw / mag) * (1 + S), psi).ravel()
    got = overlap.dense_DN(sign.dense_sign_exact(dense_cold.Q, eig=(dense_cold.lam, dense_cold.W)), S) @ psi.ravel()
    assert np.abs(got - expect).max() < 1e-11


def test_dn_operator_form_and_solve(dense_random):
    """apply_DN (operator form) equals the dense D_N^m; CGNE reaches the dense LU solution."""
    mq = 0.05
    s_ex = sign.dense_sign_exact(dense_random.Q, eig=(dense_random.lam, dense_random.W))
    dm = overlap.dense_DN(s_ex, S, mq)
    b = synthetic.spinor(256, seed=21)
    app = lambda v: overlap.apply_DN(lambda w: (s_ex @ w.ravel()).reshape(w.shape), v, S, mq)
    assert np.abs(app(b).ravel() - dm @ b.ravel()).max() < 1e-12
    g5 = lambda v: dirac.gamma5(v)
    x, it = overlap.cgne(app, lambda v: g5(app(g5(v))), b, tol=1e-11)
    x_lu = np.linalg.solve(dm, b.ravel())
    assert np.linalg.norm(x.ravel() - x_lu) < 1e-8 * np.linalg.norm(x_lu)
    assert np.linalg.norm(b.ravel() - dm @ x.ravel()) <= 1e-11 * np.linalg.norm(b) * 1.01


@pytest.mark.parametrize("dims", [(2, 2, 2, 2), (4, 2, 2, 4)])
def test_force_vs_central_fd(dims):
    v = geometry.volume(dims)
    u = synthetic.gauge_field(dims)
    psi = synthetic.spinor(v)
    f = force.force_action(u, psi, M, dims)
    om = synthetic.su3_directions(v, 8)
    h = 1e-5
    for w in om:
        sp = force.action(force.perturb_links(u, w, h), psi, M, dims)
        sm = force.action(force.perturb_links(u, w, -h), psi, M, dims)
        fd = (sp - sm) / (2 * h)
        an = float(np.sum(f * w))
        assert abs(fd - an) <= 1e-8 * max(1.0, abs(an))


def test_grad_psi_vs_fd():
    dims = (2, 2, 2, 4)
    v = geometry.volume(dims)
    u = synthetic.gauge_field(dims)
    psi = synthetic.spinor(v)
    g = force.grad_psi_action(u, psi, M, dims)
    eta = synthetic.spinor(v, seed=99)
    h = 1e-5
    fd = (force.action(u, psi + h * eta, M, dims) - force.action(u, psi - h * eta, M, dims)) / (2 * h)
    # dS = Re<grad, d psi> in the convention grad = 2 dS/d(psi-bar)
    assert abs(fd - np.vdot(g, eta).real) < 1e-7 * abs(fd)


def test_ritz_functional_lowmodes(dense_random):
    """The Ritz-functional minimisation reproduces the lowest eigenvalues of Q^2
    from dense diagonalisation, with orthonormal vectors and small residues;
    the Rayleigh-Ritz step of Q in their span gives the lowest |lambda| of Q."""
    q = dense_random.Q
    n = q.shape[0]
    a = q @ q
    rng = np.random.default_rng(3)
    starts = rng.normal(size=(6, n)) + 1j * rng.normal(size=(6, n))
    mu, x, g = lowmodes.ritz_lowmodes(lambda v: a @ v, starts, 6, tol=1e-10)
    lam2 = np.sort(dense_random.lam ** 2)[:6]
    assert np.allclose(mu, lam2, rtol=0, atol=1e-12)
    assert np.abs(x.conj() @ x.T - np.eye(6)).max() < 1e-12
    assert np.all(g <= 1e-10)
    for xi, mi in zip(x, mu):
        assert np.linalg.norm(a @ xi - mi * xi) <= 1e-9
    nu, u = lowmodes.rayleigh_ritz(lambda v: q @ v, x)
    order = np.argsort(np.abs(dense_random.lam), kind="stable")[:6]
    assert np.allclose(np.sort(np.abs(nu)), np.sort(np.abs(dense_random.lam[order])), atol=1e-10)


def test_ritz_functional_free_field_degenerate(dense_cold):
    """On the free field the lowest eigenvalue of Q^2 (0.36) is 48-fold: every
    minimisation lands in that eigenspace."""
    q = dense_cold.Q
    a = q @ q
    rng = np.random.default_rng(4)
    starts = rng.normal(size=(4, q.shape[0])) + 1j * rng.normal(size=(4, q.shape[0]))
    mu, x, _ = lowmodes.ritz_lowmodes(lambda v: a @ v, starts, 4, tol=1e-11)
    assert np.allclose(mu, 0.36, atol=1e-12)
    pe = dense_cold.W[:, np.abs(np.abs(dense_cold.lam) - 0.6) < 1e-9]
    assert np.linalg.norm(x.T - pe @ (pe.conj().T @ x.T)) < 1e-9


@pytest.mark.parametrize("form", ["literal", "sandwich"])
def test_projection_of_a_batch(dense_tiny, form):
    """Each field of a batch is projected exactly as when passed alone."""
    q = dense_tiny.Q
    nu, modes = lowmodes.dense_lowmodes(q, 5, eig=(dense_tiny.lam, dense_tiny.W))
    rng = np.random.default_rng(12)
    batch = rng.normal(size=(3, q.shape[0])) + 1j * rng.normal(size=(3, q.shape[0]))
    fn = sign.project_literal if form == "literal" else sign.project_sandwich
    r = sign.dense_sign_approx(q, approx.zolotarev(0.1, 6), LMAX, eig=(dense_tiny.lam, dense_tiny.W))
    got = fn(lambda t: t @ r.T, modes, nu, batch)
    for j in range(3):
        one = fn(lambda t: r @ t, modes, nu, batch[j])
        assert np.abs(got[j] - one).max() < 1e-13
