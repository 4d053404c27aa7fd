"""MI355X (gfx950) coupled phase-field lattice Boltzmann step.

The conservative Allen-Cahn phase-field LBM of arXiv:2206.11637 (sec.
"Conservative Allen-Cahn model"): D3Q15 phase-field populations coupled to
D3Q27 velocity-based hydrodynamic populations with surface-tension,
pressure, viscous and body forces and bounce-back walls, advanced by
hand-written HIP kernels behind a C ABI (include/pflbm.h).  This package is
the thin Python binding: it marshals torch device buffers and the current
HIP stream into those calls.  Every step of the method runs in the library;
there is no CPU fallback.
"""
from ._lib import PFLBMError, load  # noqa: F401
from .sim import Simulation, lattice  # noqa: F401
from .rollout import PFLBMRollout, amplitude_rollout  # noqa: F401
