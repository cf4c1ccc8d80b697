"""MI355X (gfx950) static autotuning model of Lim, Norris and Malony,
"Autotuning GPU Kernels via Static and Predictive Analysis" (arXiv:1701.08547).

The compute path is the C-ABI library ``libsa.so`` (``include/sa.h``); this
package holds its thin ctypes binding (``api``), the seeded input generators
(``workloads``) and the build script (``build``).
"""
from . import workloads  # noqa: F401
from .api import (  # noqa: F401
    Plan, SAError, Surrogate, Workspace, arch_default, arch_gfx950, arch_validate, autotune, device_batch, features,
    occupancy, plan_layout, score, set_tile, topk, workspace_bytes,
)
