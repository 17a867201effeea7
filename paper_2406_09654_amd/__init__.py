"""MI355X (gfx950) implementation of the Coralai per-step ecosystem update.

The compute lives in ``libcoralai.so`` (hand-written HIP, C ABI declared in
``include/coralai.h``); ``binding`` mirrors that ABI one function per entry
point and ``world`` adds owning wrappers whose device memory comes from
PyTorch.
"""
from .binding import (CORALAI_BF16, CORALAI_FP32, CoralaiError, coralai_stats,  # noqa: F401
                      coralai_world_desc, lib)

__all__ = ["lib", "CoralaiError", "coralai_world_desc", "coralai_stats", "CORALAI_FP32",
           "CORALAI_BF16", "World", "Batch", "make_desc"]


def __getattr__(name):
    if name in ("World", "Batch", "make_desc", "desc_from_spec"):
        from . import world
        return getattr(world, name)
    raise AttributeError(name)
