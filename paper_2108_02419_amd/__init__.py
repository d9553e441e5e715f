"""MI355X-native Monte-Carlo of the BBE track-race model.

The library ``libbbe.so`` (HIP kernels for gfx950 behind the C ABI in
``include/bbe.h``) runs many independent simulations of a race from the start
or from an in-play state and tallies the finish orders into win
probabilities (Cliff, Hawkins, Keen & Lau-Soto, EMSS 2021, Sections 3 and 6).

``api`` holds the tensor-level helpers used by the tests and the benchmark.
"""
from . import _bbe  # noqa: F401
from ._bbe import BBEError, Race  # noqa: F401

__all__ = ["BBEError", "Race"]
