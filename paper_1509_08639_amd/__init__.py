"""MI355X-native comparable-corpus sentence miner (HIP, gfx950).

The miner of Section 4 of arXiv:1509.08639 -- sentence-pair scores from a
lexicon-overlap classifier, Needleman-Wunsch alignment, threshold -- as a C
ABI shared library (include/ymine.h, libymine.so) with a thin ctypes binding
in :mod:`paper_1509_08639_amd.ymine`.
"""
from . import ymine  # noqa: F401

__all__ = ["ymine"]
