"""MI355X-native hot path of the Neuberger-Dirac operator (HIP kernels behind a C ABI).

The compute lives in ``libndq.so`` (built from ``csrc/`` by ``build.py``);
``ndq`` is its ctypes binding.
"""
from . import ndq  # noqa: F401
from .ndq import (F16, F32, F64, EVEN, ODD, FULL, LITERAL, SANDWICH, MINMAX_POLY, ZOLOTAREV,  # noqa: F401
                  Approx, GaugeField, Geometry, NdqError, Overlap, SpinorField, apply_DN, apply_dslash, apply_Q, apply_Q_multi,
                  apply_Qhat_ee, apply_sign, autotune, gauge_force, index_DN, lowmodes_compute, set_launch, set_launch_for, solve_DN, spinor_gram,
                  QFunction)
