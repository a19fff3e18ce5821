"""MI355X (gfx950) piCholesky cross-validation.

The compute path lives in the HIP library ``libpichol.so`` (sources in
``csrc/``, C-ABI in ``include/pichol.h``); ``binding`` marshals torch
tensors into its entry points.  Importing this package loads nothing: the
library is loaded on the first call, and a missing library raises.
"""

__all__ = ["binding"]
