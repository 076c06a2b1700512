"""MI355X-native NNP energy/force evaluation and MD (gas phase or periodic
boxes; velocity Verlet or Langevin dynamics).

The compute path is the HIP library ``libnnp_hip.so`` behind the C ABI of
``include/nnp.h``; this package only marshals arguments to it.  PyTorch is
used for device memory and streams (``autograd.NNPEnergy``), never for the
computation.
"""

from ._lib import NNPError, EXPORTS, LIB_PATH, load  # noqa: F401
from .context import Context  # noqa: F401

__all__ = ["Context", "NNPError", "load", "LIB_PATH", "EXPORTS"]
