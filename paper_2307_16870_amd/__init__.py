"""Entanglement-aware MPS / MPO two-site gate update for AMD MI355X.

The HIP library (``_lib/libeamps.so``, C ABI in ``include/ea_mps.h``) does
the work; this package binds it (``_binding``) and offers a small driver
(``EAState``) that walks a circuit layer by layer.
"""
from ._binding import *  # noqa: F401,F403
from ._binding import SYMBOLS, LIB_PATH, EAError  # noqa: F401
from .driver import EAState, run_batched  # noqa: F401
