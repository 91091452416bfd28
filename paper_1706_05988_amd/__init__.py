"""MI355X-native shifted pipelined CG (Cools & Vanroose, Alg. 3).

``paper_1706_05988_amd.pcg`` binds the C ABI of ``libpcg.so`` (declared in
``include/pcg.h``); ``paper_1706_05988_amd.build`` compiles it for gfx950.
"""
from . import pcg  # noqa: F401

__all__ = ["pcg"]
