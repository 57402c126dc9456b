"""Entanglement-aware MPS / MPO two-site gate update for AMD MI355X.

The HIP library (``_lib/libeamps.so``, C ABI in ``include/ea_mps.h``) does
the work; this package binds it (``_binding``) and offers a small driver
(``EAState``) that walks a circuit layer by layer.
"""
from ._binding import *  # noqa: F401,F403
from ._binding import SYMBOLS, LIB_PATH, EAError  # noqa: F401
from .driver import EAState, capture_batched, run_batched  # noqa: F401

# Jacobi launch shapes chosen by the autotuner (``autotune.py``) for this
# GPU, if present; EA_MPS_TUNING names another table, or "none" for the
# built-in shapes.
import os as _os

_tuning = _os.environ.get("EA_MPS_TUNING") or _os.path.join(
    _os.path.dirname(_os.path.abspath(__file__)), "tuning_gfx950.json")
if _tuning != "none" and _os.path.exists(_tuning):
    load_tuning(_tuning)  # noqa: F405
TUNING_TABLE = _tuning if _tuning != "none" and _os.path.exists(_tuning) else None
