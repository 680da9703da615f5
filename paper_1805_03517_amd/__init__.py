"""MI355X (gfx950) Flow Fields dense correspondence search (FlowFields++,
Sec. 3.1 "Matches") behind the C ABI in include/ff.h.

The HIP library libff.so is built in-tree by ``python -m
paper_1805_03517_amd.build``; ``ff`` is its ctypes binding and ``synth``
the seeded synthetic pair generators.
"""
from . import ff  # noqa: F401
from .ff import FFError, Matcher  # noqa: F401

__all__ = ["ff", "FFError", "Matcher"]
