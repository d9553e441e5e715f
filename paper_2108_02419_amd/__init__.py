"""MI355X-native Monte-Carlo of the BBE track-race model.

The library ``libbbe.so`` (HIP kernels for gfx950 behind the C ABI in
``include/bbe.h``) runs many independent simulations of a race from the start
or from an in-play state and tallies the finish orders into win
probabilities (Cliff, Hawkins, Keen & Lau-Soto, EMSS 2021, Sections 3 and 6).

Modules: ``_bbe`` (ctypes binding of every ABI function, argument
marshalling only), ``api`` (tensor-level helpers that allocate outputs),
``inputs`` (seeded synthetic workloads), ``build`` (hipcc build of the
library), and the applications built on the library: ``surrogate``
(training and judging the surrogate network), ``query_loop`` (in-play
queries answered by the surrogate with a Monte-Carlo gate and audit) and
``bettors`` (RP(d) and cheap bettor populations through a race in play).
"""
from . import _bbe  # noqa: F401
from ._bbe import BBEError, Race  # noqa: F401

__all__ = ["BBEError", "Race"]
