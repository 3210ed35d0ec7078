"""Write the stored expected values under tests/golden/ from the FP64 oracle.

    python tests/golden/make_golden.py

Only ``oracle`` and the seeded inputs of ``synthetic`` are used; nothing here
touches the GPU library.  Each fixture records its inputs (lattice, seeds,
parameters), the passage of the paper it follows, and the values.
"""
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import synthetic  # noqa: E402
from oracle import approx, dirac, overlap, sign  # noqa: E402

M = -1.4
LMAX = 6.6


def cplx(a):
    a = np.asarray(a).ravel()
    return [[float(z.real), float(z.imag)] for z in a]


def q_apply():
    dims = (4, 2, 2, 2)
    u = synthetic.gauge_field(dims, seed=77)
    psi = synthetic.spinor(32, seed=78)
    y = dirac.apply_Q(u, psi, M, dims)
    return {"what": "Q psi = gamma5 D_W psi (Sec. 2.1, Eq. 1, Eq. 2), chiral gamma matrices, periodic",
            "dims": list(dims), "m": M, "gauge": "synthetic.gauge_field(dims, seed=77)",
            "spinor": "synthetic.spinor(32, seed=78)", "layout": "canonical [V][4 spin][3 colour], lexicographic",
            "Q_psi": cplx(y), "norm2": float(np.vdot(y, y).real)}


def approximants():
    z = approx.zolotarev(0.1, 8)
    p = approx.minimax_polynomial(0.01, 20)
    return {"zolotarev": {"what": "Zolotarev's optimal rational approximation of sign(x) on [k, 1], "
                                  "x sum_l beta_l / (x^2 + sigma_l)", "k": 0.1, "n": 8,
                          "sigma": z.sigma.tolist(), "beta": z.beta.tolist(), "delta": z.delta},
            "minimax": {"what": "minimax polynomial of 1/sqrt(y) on [eps, 1] in the Chebyshev basis "
                                "(Sec. 2.2, Eq. 5, Eq. 6)", "eps": 0.01, "n": 20, "c": p.c.tolist(),
                        "delta": p.delta}}


def dn_apply():
    dims = (2, 2, 2, 4)
    u = synthetic.gauge_field(dims, seed=79)
    v = 32
    psi = synthetic.spinor(v, seed=80)
    q = dirac.dense_Q(u, M, dims)
    lam, w = sign.dense_eig(q)
    eps = sign.dense_sign_exact(q, eig=(lam, w))
    s = overlap.s_of_wilson_mass(M)
    d = overlap.dense_DN(eps, s, 0.05)
    y = d @ psi.ravel()
    return {"what": "D_N^m psi with the exact sign of Q (Sec. 2.2, Eq. 4; massive form of Eq. 12), "
                    "mq = 0.05, dense 384 x 384", "dims": list(dims), "m": M, "mq": 0.05,
            "gauge": "synthetic.gauge_field(dims, seed=79)", "spinor": "synthetic.spinor(32, seed=80)",
            "min_abs_lambda_Q": float(np.abs(lam).min()), "DN_psi": cplx(y)}


if __name__ == "__main__":
    for name, fn in (("q_apply_4x2x2x2.json", q_apply), ("approximants.json", approximants),
                     ("dn_apply_2x2x2x4.json", dn_apply)):
        with open(os.path.join(HERE, name), "w") as fh:
            json.dump(fn(), fh, indent=1)
        print("wrote", name)
