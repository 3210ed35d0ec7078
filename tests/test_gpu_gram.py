"""Gram matrices of blocks of FP64 spinor fields on the matrix cores
(G = A^H B, the inner products of the Rayleigh-Ritz step of Sec. 2.3) against
the plain definition (numpy vdot of the canonical fields)."""
import numpy as np
import pytest

import synthetic
from oracle import geometry

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_1010_5636_amd as ndq  # noqa: E402


@pytest.mark.parametrize("dims", [(8, 4, 6, 2), (4, 4, 4, 4), (32, 16, 16, 16)])
@pytest.mark.parametrize("na,nb", [(1, 1), (5, 3), (16, 16), (17, 33), (28, 28), (64, 64), (64, 1)])
def test_gram_vs_definition(dims, na, nb):
    if dims == (32, 16, 16, 16) and na * nb > 28 * 28:
        pytest.skip("large blocks checked on the small lattices")
    v = geometry.volume(dims)
    a = synthetic.spinor(v, nrhs=na, seed=81)
    b = synthetic.spinor(v, nrhs=nb, seed=82)
    g = ndq.Geometry(dims)
    A = ndq.SpinorField.pack(g, torch.from_numpy(a).cuda(), ndq.F64, ndq.FULL)
    B = ndq.SpinorField.pack(g, torch.from_numpy(b).cuda(), ndq.F64, ndq.FULL)
    G = ndq.spinor_gram(g, A, B).cpu().numpy()
    ref = a.reshape(na, -1).conj() @ b.reshape(nb, -1).T
    scale = np.sqrt(12 * v)   # |A_i| |B_j| for unit-variance components
    assert np.abs(G - ref).max() <= 1e-13 * scale * scale, np.abs(G - ref).max()


def test_gram_same_block_is_hermitian():
    dims = (8, 8, 8, 8)
    v = geometry.volume(dims)
    a = synthetic.spinor(v, nrhs=20, seed=83)
    g = ndq.Geometry(dims)
    A = ndq.SpinorField.pack(g, torch.from_numpy(a).cuda(), ndq.F64, ndq.FULL)
    G = ndq.spinor_gram(g, A, A).cpu().numpy()
    assert np.abs(G - G.conj().T).max() <= 1e-12 * np.abs(G).max()
    assert np.allclose(np.diag(G).real, np.linalg.norm(a.reshape(20, -1), axis=1) ** 2, rtol=1e-13)
