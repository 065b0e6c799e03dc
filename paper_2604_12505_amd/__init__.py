"""MI355X-native sloshing simulator: body-frame WCSPH coupled to rigid-body
attitude dynamics, and an MLP surrogate of the slosh wrench.

The compute lives in ``libslosh.so`` (HIP kernels for gfx950 behind the C ABI
of ``include/slosh.h``).  This package is the thin binding: it marshals
arguments and uses PyTorch for device memory and streams only.
"""
from ._lib import LibraryMissing, load  # noqa: F401
