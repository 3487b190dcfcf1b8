"""Plain FP64 CPU oracle for the IMRT fluence-map optimiser.

TEST INFRASTRUCTURE, NOT PART OF THE PRODUCT.  Only ``tests/``, the smoke
check in ``__graft_entry__`` and the CPU-baseline leg of ``bench.py`` may
import anything from here.  It shares no code with the HIP library: it reads
only the workload specifications in ``workloads`` and builds every input
itself.

Modules:
  phantom   synthetic structures and dose-deposition matrix D (brute force)
  model     dose, one-sided quadratic penalties, objective, gradient, projection
  solver    gradient projection with Armijo's line search, lambda_0, KKT residual
  quantize  D stored in bfloat16 / binary16 codes with per-beamlet scales

Parity status of each function is recorded with the pins in ``tests/``.
"""
from . import model, phantom, quantize, solver  # noqa: F401
