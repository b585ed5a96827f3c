"""MI355X (gfx950) MPS-VQE energy engine.

The hot path -- UCCSD energy <psi(theta)|H|psi(theta)> of a Jordan-Wigner
Hamiltonian on a matrix product state -- runs in hand-written HIP kernels
behind the C ABI of ``include/q2c.h``; ``q2c`` is its ctypes binding.  The
binding (and with it libq2c.so) is loaded on first use, so that the build
step does not depend on an earlier build; using it without a built library
raises ImportError.
"""
import importlib

_EXPORTS = ("MPS", "Context", "Problem", "Server", "Q2C_FP64", "Q2C_MIXED", "Q2CError")


def __getattr__(name):
    if name == "q2c":
        return importlib.import_module(".q2c", __name__)
    if name in _EXPORTS:
        return getattr(importlib.import_module(".q2c", __name__), name)
    raise AttributeError(f"module {__name__!r} has no attribute {name!r}")
