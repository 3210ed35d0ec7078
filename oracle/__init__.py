"""FP64 CPU oracle for the Neuberger-Dirac hot path -- TEST INFRASTRUCTURE ONLY.

This package is a plain, slow, deliberately unoptimised restatement of what
the paper (Walk, Wittig, Dranischnikow, Schoemer, "Implementation of the
Neuberger-Dirac operator on GPUs", Lattice 2010) defines:

* the gamma5-Hermitian Wilson-Dirac operator Q = gamma5 D_W (Sec. 2.1, Eq. 1
  and Eq. 2), evaluated with full 4x4 spin matrices and full 3x3 links;
* the sign-function approximants: the minimax polynomial in a Chebyshev basis
  (Sec. 2.2, Eq. 5 and Eq. 6) and a Zolotarev rational approximant;
* the low-mode projection (Sec. 2.3, Eq. 7-11) and its diagnostics;
* the Neuberger-Dirac operator D_N and its massive form (Eq. 4, Eq. 12);
* the su(3) link force of S = |Q psi|^2;
* the index of the massless D_N by zero-mode counting (outlook of Sec. 4).

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import it.  It shares no code with the GPU library
(``paper_1010_5636_amd``) and never imports it; the seeded input generators
in ``synthetic`` are the one common dependency.

Precision: numpy float64/complex128 throughout.

Parity status of each function is stated in its docstring; functions pinned
only by their own invariants say "parity unpinned".
"""
from . import geometry, dirac, approx, sign, lowmodes, overlap, force, index  # noqa: F401
