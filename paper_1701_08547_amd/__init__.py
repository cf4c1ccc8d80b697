"""MI355X (gfx950) static autotuning model of Lim, Norris and Malony,
"Autotuning GPU Kernels via Static and Predictive Analysis" (arXiv:1701.08547).

The compute path is the C-ABI library ``libsa.so`` (``include/sa.h``,
``include/sa_runtime.h``, ``include/sa_workload.h``); this package holds its
thin ctypes binding (``api``), the seeded input generators (``workloads``),
the build script (``build``) and command-line drivers of the measurements
(``streamed``, ``report``, ``runtime_dataset``, ``correction``,
``calibration``, ``imix``).
"""
from . import workloads  # noqa: F401
from .api import (  # noqa: F401
    Plan, SAError, Surrogate, Workspace, arch_default, arch_gfx950, arch_validate, autotune, device_batch, features,
    headroom, occupancy, plan_layout, product_size, score, score_product, score_suggested, set_tile, suggest, topk,
    workspace_bytes,
)
