"""MI355X (gfx950) MPS-VQE energy engine.

The hot path -- UCCSD energy <psi(theta)|H|psi(theta)> of a Jordan-Wigner
Hamiltonian on a matrix product state -- runs in hand-written HIP kernels
behind the C ABI of ``include/q2c.h``; ``q2c`` is its ctypes binding.
"""
from . import q2c  # noqa: F401  (loads libq2c.so; raises ImportError if it is not built)
from .q2c import (  # noqa: F401
    MPS,
    Context,
    Problem,
    Q2C_FP64,
    Q2C_MIXED,
    Q2CError,
)
