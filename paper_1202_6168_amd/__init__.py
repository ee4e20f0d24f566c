"""D-iteration fluid diffusion on AMD Instinct MI355X (gfx950).

The solver is the C-ABI library libditr.so (include/ditr.h) built from
csrc/*.hip; ``paper_1202_6168_amd.ditr`` is its thin ctypes binding.
"""
from . import ditr  # noqa: F401

__all__ = ["ditr"]
