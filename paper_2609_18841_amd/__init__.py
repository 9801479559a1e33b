"""MI355X (gfx950) batched TEBD-Lindblad hot path: HIP library + thin Python binding.

The compute path lives in lib/libtebd.so (sources in csrc/, C ABI in include/tebd.h);
api.py only marshals arguments.  Importing api fails loudly if the library is missing.
"""
from . import api  # noqa: F401
