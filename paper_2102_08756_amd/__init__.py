"""MI355X-native spectral boundary integral (SBIM) traction update.

The compute path is the HIP library ``_lib/libsbim.so`` (sources in ``csrc/``,
C ABI in ``include/sbim.h``); ``sbim`` is its Python binding.
"""
from .sbim import (SBIM, Config, Fault, Plane, SBIMError, SBIMRun, Strip, checkpointed_loss,  # noqa: F401
                   load_library, EXPORTS, LIB_PATH)
