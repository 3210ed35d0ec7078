"""Pins for the oracle's Wilson-Dirac operator (Eq. 1, Eq. 2).

Each pin is fixed by mathematics independent of the oracle's code path:
Clifford algebra, the free-field momentum-space closed form, the free-field
spectrum, gamma5-Hermiticity, gauge covariance, the operator-norm bound and
the even/odd Schur complement built from dense blocks.  A final test plants
plausible mistakes in the oracle and checks that some pin catches each one.
"""
import numpy as np
import pytest

import synthetic
from oracle import dirac, geometry

M = -1.4


def _plane_wave(dims, nvec, chi):
    x = geometry.coords(dims)
    p = 2 * np.pi * np.asarray(nvec) / np.asarray(dims)
    phase = np.exp(1j * (x @ p))
    return phase[:, None, None] * chi[None], p


def test_gamma_clifford():
    g, g5 = dirac.gamma_matrices()
    for mu in range(4):
        assert np.allclose(g[mu], g[mu].conj().T)
        assert np.linalg.matrix_rank(np.eye(4) - g[mu]) == 2
        for nu in range(4):
            acomm = g[mu] @ g[nu] + g[nu] @ g[mu]
            assert np.allclose(acomm, 2 * np.eye(4) * (mu == nu))
        assert np.allclose(g5 @ g[mu] + g[mu] @ g5, 0)
    assert np.allclose(g5, np.diag([1, 1, -1, -1]))


def test_links_are_su3():
    u = synthetic.gauge_field((4, 4, 4, 4))
    uu = np.einsum("vmba,vmbc->vmac", u.conj(), u)
    assert np.abs(uu - np.eye(3)).max() < 1e-14
    assert np.abs(np.linalg.det(u) - 1).max() < 1e-14
    assert np.abs(np.linalg.inv(u) - np.swapaxes(u.conj(), -1, -2)).max() < 1e-14


@pytest.mark.parametrize("dims,nvec", [((4, 4, 4, 4), (0, 0, 0, 0)), ((4, 4, 4, 4), (1, 2, 3, 1)),
                                        ((8, 4, 6, 2), (3, 1, 5, 1)), ((6, 2, 4, 8), (2, 1, 1, 7))])
def test_free_field_closed_form(dims, nvec):
    """U = 1, psi = exp(i p.x) chi  =>  D_W psi = [m + sum(1 - cos p) + i sum gamma sin p] psi."""
    g, _ = dirac.gamma_matrices()
    rng = np.random.default_rng(7)
    chi = rng.normal(size=(4, 3)) + 1j * rng.normal(size=(4, 3))
    psi, p = _plane_wave(dims, nvec, chi)
    sym = (M + np.sum(1 - np.cos(p))) * np.eye(4)
    for mu in range(4):
        sym = sym + 1j * np.sin(p[mu]) * g[mu]
    expect = np.einsum("st,vtc->vsc", sym, psi)
    got = dirac.wilson_dirac(synthetic.cold_gauge(dims), psi, M, dims)
    assert np.abs(got - expect).max() < 1e-13


def test_free_field_spectrum(dense_cold):
    """|lambda(Q)| = sqrt((m + sum(1-cos p))^2 + sum sin^2 p), 12-fold per momentum."""
    dims = dense_cold.dims
    ps = np.array(np.meshgrid(*[2 * np.pi * np.arange(n) / n for n in dims], indexing="ij")).reshape(4, -1).T
    mags = np.sqrt((M + np.sum(1 - np.cos(ps), axis=1)) ** 2 + np.sum(np.sin(ps) ** 2, axis=1))
    expect = np.sort(np.repeat(mags, 12))
    got = np.sort(np.abs(dense_cold.lam))
    assert np.abs(got - expect).max() < 1e-12
    assert abs(got[0] - 0.6) < 1e-12 and np.sum(np.abs(got - 0.6) < 1e-9) == 48
    assert abs(got[-1] - 6.6) < 1e-12
    # Q is traceless per momentum: equal numbers of positive and negative eigenvalues
    assert np.sum(dense_cold.lam > 0) == np.sum(dense_cold.lam < 0)


def test_gamma5_hermiticity_and_norm(dense_random):
    q = dense_random.Q
    assert np.abs(q - q.conj().T).max() < 1e-14
    assert np.abs(dense_random.lam).max() <= dirac.lambda_max_bound(M) + 1e-12


@pytest.mark.parametrize("dims", [(4, 4, 4, 4), (8, 4, 6, 2)])
def test_gamma5_hermiticity_sparse(dims):
    u = synthetic.gauge_field(dims)
    v = geometry.volume(dims)
    chi = synthetic.spinor(v, seed=11)
    psi = synthetic.spinor(v, seed=12)
    a = np.vdot(chi, dirac.apply_Q(u, psi, M, dims))
    b = np.vdot(dirac.apply_Q(u, chi, M, dims), psi)
    assert abs(a - b) < 1e-12 * abs(a)
    assert np.linalg.norm(dirac.apply_Q(u, psi, M, dims)) <= 6.6 * np.linalg.norm(psi)


@pytest.mark.parametrize("dims", [(4, 4, 4, 4), (8, 4, 6, 2)])
def test_gauge_covariance(dims):
    """Q[U^Omega] (Omega psi) = Omega Q[U] psi with U^Omega_mu(x) = Omega(x) U_mu(x) Omega(x+mu)^H."""
    u = synthetic.gauge_field(dims)
    v = geometry.volume(dims)
    om = synthetic.haar_su3(v)
    nb = geometry.neighbour_table(dims)
    ug = np.einsum("vab,vmbc->vmac", om, u)
    for mu in range(4):
        ug[:, mu] = ug[:, mu] @ om[nb[:, mu]].conj().transpose(0, 2, 1)
    psi = synthetic.spinor(v)
    lhs = dirac.apply_Q(ug, np.einsum("vab,vsb->vsa", om, psi), M, dims)
    rhs = np.einsum("vab,vsb->vsa", om, dirac.apply_Q(u, psi, M, dims))
    assert np.abs(lhs - rhs).max() < 1e-13


class _Unit:
    """Links U = 1 at every site of any lattice, indexable like a gauge field."""

    def __getitem__(self, key):
        sites, _ = key
        return np.broadcast_to(np.eye(3, dtype=np.complex128), np.shape(sites) + (3, 3))


def test_apply_Q_at_free_field_large():
    """Per-site Q on the 32^3 x 64 lattice with U = 1 against the momentum-space closed form,
    at sites on every face of the lattice and in its interior."""
    dims = (64, 32, 32, 32)
    rng = np.random.default_rng(5)
    chi = rng.normal(size=(4, 3)) + 1j * rng.normal(size=(4, 3))
    nvec = (5, 3, 11, 1)
    p = 2 * np.pi * np.asarray(nvec) / np.asarray(dims)

    def psi_at(idx):
        x = np.stack(np.unravel_index(idx, dims), axis=-1)
        return np.exp(1j * (x @ p))[:, None, None] * chi[None]

    corners = np.array([[0, 0, 0, 0], [63, 31, 31, 31], [0, 31, 0, 31], [63, 0, 17, 0], [12, 5, 31, 0]])
    sites = np.concatenate([geometry.lex_of(dims, corners), rng.integers(0, geometry.volume(dims), 64)])
    _, g5 = dirac.gamma_matrices()
    expect = np.einsum("st,vtc->vsc", g5 @ dirac.free_field_symbol(p, M), psi_at(sites))
    got = dirac.apply_Q_at(_Unit(), psi_at, M, dims, sites)
    assert np.abs(got - expect).max() < 1e-13


@pytest.mark.parametrize("dims", [(4, 4, 4, 4), (8, 4, 6, 2)])
def test_apply_Q_at_gauge_covariance(dims):
    """Per-site Q: Q[U^Omega](Omega psi)(y) = Omega(y) (Q[U] psi)(y) at every site, two right-hand sides."""
    u = synthetic.gauge_field(dims)
    v = geometry.volume(dims)
    om = synthetic.haar_su3(v)
    nb = geometry.neighbour_table(dims)
    ug = np.einsum("vab,vmbc->vmac", om, u)
    for mu in range(4):
        ug[:, mu] = ug[:, mu] @ om[nb[:, mu]].conj().transpose(0, 2, 1)
    psi = synthetic.spinor(v, nrhs=2)
    psig = np.einsum("vab,rvsb->rvsa", om, psi)
    sites = np.arange(v)
    lhs = dirac.apply_Q_at(ug, lambda i: psig[:, i], M, dims, sites)
    rhs = np.einsum("vab,rvsb->rvsa", om, dirac.apply_Q_at(u, lambda i: psi[:, i], M, dims, sites))
    assert np.abs(lhs - rhs).max() < 1e-13
    # and the per-site form agrees with the whole-lattice form
    assert np.abs(dirac.apply_Q_at(u, lambda i: psi[:, i], M, dims, sites) - dirac.apply_Q(u, psi, M, dims)).max() < 1e-13


def test_eo_schur_complement(dense_random):
    """Qhat_ee = gamma5 (D_ee - D_eo D_oo^{-1} D_oe), blocks taken from the dense D_W."""
    dims = dense_random.dims
    v = geometry.volume(dims)
    leo = geometry.lex_of_eo(dims)
    g5 = np.tile(np.repeat([1.0, 1.0, -1.0, -1.0], 3), v)
    d = g5[:, None] * dense_random.Q                    # D_W = gamma5 Q
    idx = lambda p: (leo[p][:, None] * 12 + np.arange(12)).ravel()
    e, o = idx(0), idx(1)
    schur = d[np.ix_(e, e)] - d[np.ix_(e, o)] @ np.linalg.solve(d[np.ix_(o, o)], d[np.ix_(o, e)])
    g5e = np.tile(np.repeat([1.0, 1.0, -1.0, -1.0], 3), v // 2)
    psi_e = synthetic.spinor(v // 2, seed=5)
    expect = (g5e[:, None] * schur) @ psi_e.ravel()
    got = dirac.qhat_ee(dense_random.U, psi_e, M, dims).ravel()
    assert np.abs(got - expect).max() < 1e-12
    # the off-diagonal blocks are -H/2
    psi_o = synthetic.spinor(v // 2, seed=6)
    h_eo = dirac.dslash(dense_random.U, psi_o, dims, 0).ravel()
    assert np.abs(-0.5 * h_eo - d[np.ix_(e, o)] @ psi_o.ravel()).max() < 1e-13


# ----------------------------------------------------------------------------
# planted mistakes: every mutant must fail at least one of the pins above
# ----------------------------------------------------------------------------

def _mutant_hopping(kind):
    g, _ = dirac.gamma_matrices()
    i4 = np.eye(4)

    def hop(U, psi, dims):
        ul = U.reshape(tuple(dims) + (4, 3, 3))
        pl = psi.reshape(psi.shape[:-3] + tuple(dims) + (4, 3))
        base = pl.ndim - 6
        out = np.zeros_like(pl)
        for mu in range(4):
            sp = -1 if kind != "roll_sign" else 1
            fwd = np.roll(pl, sp, axis=base + mu)
            pf = i4 - g[mu] if kind != "proj_swap" else i4 + g[mu]
            pb = i4 + g[mu] if kind != "proj_swap" else i4 - g[mu]
            uf = ul[..., mu, :, :]
            ub = np.roll(ul[..., mu, :, :], 1, axis=mu)
            if kind == "no_inverse":
                ub_use = ub
            elif kind == "back_link_site":
                ub_use = np.swapaxes(uf.conj(), -1, -2)
            else:
                ub_use = np.swapaxes(ub.conj(), -1, -2)
            if kind == "transpose_fwd":
                uf = np.swapaxes(uf, -1, -2)
            out += np.einsum("...ab,...sb->...sa", uf, np.einsum("st,...tc->...sc", pf, fwd))
            if kind == "drop_backward" and mu == 2:
                continue
            bwd = np.roll(pl, -sp, axis=base + mu)
            out += np.einsum("...ab,...sb->...sa", ub_use, np.einsum("st,...tc->...sc", pb, bwd))
        return out.reshape(psi.shape)
    return hop


@pytest.mark.parametrize("kind", ["proj_swap", "no_inverse", "back_link_site", "transpose_fwd",
                                  "drop_backward", "roll_sign"])
def test_planted_mistakes_are_caught(kind, monkeypatch):
    monkeypatch.setattr(dirac, "hopping", _mutant_hopping(kind))
    failures = 0
    checks = [test_gamma5_hermiticity_sparse, test_gauge_covariance]
    for chk in checks:
        try:
            chk((8, 4, 6, 2))
        except AssertionError:
            failures += 1
    try:
        test_free_field_closed_form((8, 4, 6, 2), (3, 1, 5, 1))
    except AssertionError:
        failures += 1
    assert failures > 0, f"mutant {kind} passed every pin"
