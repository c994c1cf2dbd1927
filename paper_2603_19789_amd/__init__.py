"""MI355X-native SSLBM SEIRD solver (arXiv 2603.19789).

The solver itself lives in the HIP library ``libsslbm.so`` built from
``csrc/``; ``binding`` is a thin ctypes layer over its C ABI. Importing this
package loads nothing: the library is opened on first use of ``Solver``,
``BGK``, ``Ensemble``, ``Model`` or ``library()``. ``adjoint`` (reverse-mode
gradients for torch.autograd) and ``surrogate`` (the learned surrogate) are
modules of their own.
"""
from __future__ import annotations

__all__ = ["Solver", "BGK", "Ensemble", "Model", "SSLBMError", "library"]


def __getattr__(name):
    if name in ("Solver", "BGK", "Ensemble", "Model", "SSLBMError", "library"):
        from . import binding
        return getattr(binding, name)
    raise AttributeError(name)
