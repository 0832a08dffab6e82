"""FP64 CPU oracle for the adaptive-FMM photoionization path.  TEST INFRASTRUCTURE ONLY.

This package is the plain, slow, obviously correct definition of what the
GPU path computes: the discrete quadrature of the Zheleznyak integral
(Lin & Zhuang, Sec. 2.1 eqs. (1)-(3) and Sec. 2.4 eq. (15)) restricted to
the source and target sets of the adaptive strategies (Sec. 3, eq. (18);
Sec. 4.3, eq. (22); the field rule of Sec. 5), plus the learned selector's
reference MLP.  It never approximates: no tree, no expansion.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import, call, link or execute anything in this package.
It shares no code, header, table or constant generator with the HIP path
in ``paper_2112_10059_amd/``; neither imports the other.

Functions with no independent pin say "parity unpinned" in their docstring.
"""
from .physics import (  # noqa: F401
    GasConstants,
    gas_constants,
    g_absorption,
    kernel_K,
    absorbed_fraction,
    cube_self_coefficient,
)
from .selection import source_mask, target_mask  # noqa: F401
from .direct import direct_sum, direct_sum_numpy, photoionization  # noqa: F401
from .metrics import rel_l2, local_ball_error  # noqa: F401
