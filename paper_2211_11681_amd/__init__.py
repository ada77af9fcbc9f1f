"""Samplet (S-format) kernel matrix arithmetic on AMD Instinct MI355X.

The pattern-restricted product C = P_S(A B) of samplet-compressed matrices
(Harbrecht, Multerer, Schenk, Schwab, "Multiresolution kernel matrix algebra",
Section 4.1) and the operations built on it, as hand-written HIP kernels for
gfx950 behind the C ABI of include/spm.h.  ``spm`` is the thin Python binding;
``autograd`` wires the hand-written adjoints into torch.autograd.
"""
from . import _lib  # noqa: F401


def load():
    """Load libspm.so; raises ImportError if it has not been built."""
    return _lib.load()
