"""sign(Q) and its approximations -- oracle (test infrastructure only).

* Eq. 5 (Sec. 2.2): sign(Q) ~ X P_n(X^2), X = Q / |Q|.
* Rational variant: sign(Q) ~ X sum_l beta_l (X^2 + sigma_l)^{-1}.
* Eq. 11 (Sec. 2.3): with the low-mode projectors P_+ and P_- of Eq. 7,
  sign(Q) ~ P_+ - P_- + (1 - P_+ - P_-) X P_n(X^2), applied literally: the
  approximant acts on the full input and the complement projector acts after
  it.  The "sandwich" form (1 - P) r(X) (1 - P) is provided as an option; the
  two agree when the u_k are exact eigenvectors.

Plain definitions used here:

* dense matrices: spectral decomposition Q = W diag(lambda) W^H and
  f(Q) = W diag(f(lambda)) W^H;
* sparse rational: one independent conjugate-gradient solve per shift
  (textbook Hestenes-Stiefel CG), tolerance 1e-13;
* sparse polynomial: the forward three-term Chebyshev recurrence.
"""
from __future__ import annotations

import numpy as np

from . import approx as _approx


def _vdot(a: np.ndarray, b: np.ndarray) -> complex:
    return complex(np.vdot(a.ravel(), b.ravel()))


def _norm(a: np.ndarray) -> float:
    return float(np.linalg.norm(a.ravel()))


# ----------------------------------------------------------------------------
# dense (small lattices)
# ----------------------------------------------------------------------------


def dense_eig(q_dense: np.ndarray):
    """Eigenvalues (ascending) and eigenvectors of a Hermitian dense Q."""
    return np.linalg.eigh(q_dense)


def dense_sign_exact(q_dense: np.ndarray, eig=None) -> np.ndarray:
    """W sign(Lambda) W^H; ``eig`` = (lambda, W) if already known."""
    lam, w = dense_eig(q_dense) if eig is None else eig
    return (w * np.sign(lam)) @ w.conj().T


def dense_sign_approx(q_dense: np.ndarray, approximant, lam_max: float, n_low: int = 0,
                      eig=None) -> np.ndarray:
    """W f(Lambda) W^H with f = sign on the n_low eigenvalues of smallest |lambda|
    and f(lambda) = approximant(lambda / lam_max) elsewhere: Eq. 11 in closed
    form for exact eigenvectors."""
    lam, w = dense_eig(q_dense) if eig is None else eig
    f = approximant(lam / lam_max)
    if n_low:
        low = np.argsort(np.abs(lam), kind="stable")[:n_low]
        f[low] = np.sign(lam[low])
    return (w * f) @ w.conj().T


# ----------------------------------------------------------------------------
# sparse (operator form)
# ----------------------------------------------------------------------------


def cg(apply_a, b: np.ndarray, tol: float = 1e-13, max_iter: int = 100000):
    """Textbook conjugate gradients for a Hermitian positive-definite A.

    Stops when |b - A x| <= tol |b| (recursive residual).  Returns (x, iterations).
    """
    x = np.zeros_like(b)
    r = b.copy()
    p = r.copy()
    rr = _vdot(r, r).real
    bnorm = _norm(b)
    if bnorm == 0.0:
        return x, 0
    for it in range(1, max_iter + 1):
        ap = apply_a(p)
        alpha = rr / _vdot(p, ap).real
        x = x + alpha * p
        r = r - alpha * ap
        rr_new = _vdot(r, r).real
        if np.sqrt(rr_new) <= tol * bnorm:
            return x, it
        p = r + (rr_new / rr) * p
        rr = rr_new
    raise RuntimeError("CG did not converge")


def sign_rational(apply_q, psi: np.ndarray, rat: _approx.Rational, lam_max: float,
                  tol: float = 1e-13) -> np.ndarray:
    """X sum_l beta_l (X^2 + sigma_l)^{-1} psi, one CG solve per shift."""
    acc = np.zeros_like(psi)
    for sigma, beta in zip(rat.sigma, rat.beta):
        x, _ = cg(lambda v, s=sigma: apply_q(apply_q(v)) / lam_max ** 2 + s * v, psi, tol)
        acc = acc + beta * x
    return apply_q(acc) / lam_max


def sign_polynomial(apply_q, psi: np.ndarray, poly: _approx.Polynomial, lam_max: float) -> np.ndarray:
    """X P(X^2) psi with the forward Chebyshev recurrence in
    Z = (2 X^2 - (1 + eps)) / (1 - eps)."""
    eps = poly.eps

    def apply_z(v):
        return (2.0 * apply_q(apply_q(v)) / lam_max ** 2 - (1.0 + eps) * v) / (1.0 - eps)

    return apply_q(_approx.eval_forward_recurrence(poly, apply_z, psi)) / lam_max


def sign_approx(apply_q, psi, approximant, lam_max, tol: float = 1e-13):
    if isinstance(approximant, _approx.Rational):
        return sign_rational(apply_q, psi, approximant, lam_max, tol)
    return sign_polynomial(apply_q, psi, approximant, lam_max)


def _field_dot(u: np.ndarray, psi: np.ndarray):
    """<u, psi> summed over the field axes of u; psi may carry leading batch axes
    (one inner product per field of the batch)."""
    axes = tuple(range(-u.ndim, 0))
    return np.sum(u.conj() * psi, axis=axes)


def _times_mode(c, u: np.ndarray) -> np.ndarray:
    """c u for a scalar or a batch of coefficients c (one per field of a batch)."""
    c = np.asarray(c)
    return c.reshape(c.shape + (1,) * u.ndim) * u


def project_literal(apply_approx, modes: np.ndarray, nu: np.ndarray, psi: np.ndarray) -> np.ndarray:
    """Eq. 11 as printed: (P_+ - P_-) psi + (1 - P_+ - P_-) [X P(X^2) psi].

    ``modes`` is [l, ...field shape] with orthonormal rows u_k; ``nu`` the
    Rayleigh-Ritz eigenvalues (P Q u_k = nu_k u_k).  ``psi`` is one field or a
    batch of fields (leading axes); each is projected on its own.
    """
    if np.any(nu == 0):
        raise ValueError("a low mode with nu_k = 0 has no sign")
    t = apply_approx(psi)
    out = t.copy()
    for u, n in zip(modes, nu):
        out = out + _times_mode(np.sign(n) * _field_dot(u, psi) - _field_dot(u, t), u)
    return out


def project_sandwich(apply_approx, modes: np.ndarray, nu: np.ndarray, psi: np.ndarray) -> np.ndarray:
    """(P_+ - P_-) psi + (1 - P) r(X) (1 - P) psi (exactly Hermitian variant);
    ``psi`` one field or a batch of fields as in ``project_literal``."""
    if np.any(nu == 0):
        raise ValueError("a low mode with nu_k = 0 has no sign")
    rest = psi.copy()
    for u in modes:
        rest = rest - _times_mode(_field_dot(u, psi), u)
    t = apply_approx(rest)
    out = t.copy()
    for u, n in zip(modes, nu):
        out = out + _times_mode(np.sign(n) * _field_dot(u, psi), u) - _times_mode(_field_dot(u, t), u)
    return out
