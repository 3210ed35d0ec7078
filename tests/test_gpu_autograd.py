"""GPU derivatives of y = Q[U] psi (not in the paper; they follow from Eq. 1).

* the su(3) link force for a random cotangent vs the oracle's formula;
* the tangent-space gradient satisfies Re<grad, i w T_a U> = w F^a;
* S = psi^H Q^2 psi = |Q psi|^2 through torch.autograd on the 16^3 x 32 lattice:
  dS/dpsi vs the oracle's 2 Q^2 psi, and dS/dU along 8 random su(3) directions
  vs central finite differences (step 1e-5) of the oracle's action.
"""
import numpy as np
import pytest

import synthetic
from oracle import dirac, force, geometry

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_1010_5636_amd as ndq  # noqa: E402

M = -1.4


def cu(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda")


@pytest.mark.parametrize("dims,recon", [((4, 4, 4, 4), 18), ((8, 4, 6, 2), 18), ((8, 4, 6, 2), 12)])
def test_force_vs_oracle(dims, recon):
    v = geometry.volume(dims)
    u = synthetic.gauge_field(dims)
    psi = synthetic.spinor(v, seed=3)
    g = synthetic.spinor(v, seed=4)
    ref = force.force_vjp(u, psi, g, dims)
    G = ndq.Geometry(dims)
    U = ndq.GaugeField.pack(G, cu(u), ndq.F64, recon)
    x = ndq.SpinorField.pack(G, cu(psi), ndq.F64, ndq.FULL)
    gy = ndq.SpinorField.pack(G, cu(g), ndq.F64, ndq.FULL)
    f, grad = ndq.gauge_force(G, U, x, gy, want_force=True, want_grad=True)
    f = f.cpu().numpy()
    assert np.abs(f - ref).max() <= 1e-12 * np.abs(ref).max()
    # tangent gradient: Re<grad, i w T U> = w . F for random su(3) directions w
    grad = grad.cpu().numpy()
    om = synthetic.su3_directions(v, 2)
    T = force.su3_generators()
    for w in om:
        du = 1j * np.einsum("vma,aij,vmjk->vmik", w, T, u)
        assert abs(np.vdot(grad, du).real - np.sum(w * f)) <= 1e-10 * np.abs(np.sum(w * f))


def test_autograd_16c32():
    dims = (32, 16, 16, 16)
    v = geometry.volume(dims)
    u = synthetic.gauge_field(dims)
    psi = synthetic.spinor(v)
    G = ndq.Geometry(dims)
    psi_t = cu(psi).requires_grad_(True)
    u_t = cu(u).requires_grad_(True)
    y = ndq.QFunction.apply(psi_t, u_t, G, M)
    S = (y.conj() * y).real.sum()
    S.backward()
    s_ref = force.action(u, psi, M, dims)
    assert abs(S.item() - s_ref) <= 1e-12 * s_ref
    gpsi_ref = force.grad_psi_action(u, psi, M, dims)
    gpsi = psi_t.grad.cpu().numpy()
    assert np.linalg.norm(gpsi - gpsi_ref) <= 1e-12 * np.linalg.norm(gpsi_ref)
    grad_u = u_t.grad.cpu().numpy()
    T = force.su3_generators()
    h = 1e-5
    for w in synthetic.su3_directions(v, 8):
        du = 1j * np.einsum("vma,aij,vmjk->vmik", w, T, u)
        an = np.vdot(grad_u, du).real
        # central difference (S(h) - S(-h)) / 2h, evaluated as Re<y+ - y-, y+ + y-> / 2h:
        # S ~ 3e7 here, so the naive difference of two sums would carry rounding noise
        # ~ eps S / h ~ 1e-8 relative; this form has only element-wise rounding
        yp = dirac.apply_Q(force.perturb_links(u, w, h), psi, M, dims)
        ym = dirac.apply_Q(force.perturb_links(u, w, -h), psi, M, dims)
        fd = np.vdot(yp - ym, yp + ym).real / (2 * h)
        assert abs(an - fd) <= 1e-8 * abs(fd), (an, fd)
