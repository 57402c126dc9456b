"""CPU-side checks of the C ABI: the library loads and exports every function
the header declares (no compute calls, no GPU needed)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ea_mps.h")
LIB = os.path.join(ROOT, "paper_2307_16870_amd", "_lib", "libeamps.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[a-z_]+\s*\*?\s*([a-z_][a-z0-9_]*)\s*\(", text, flags=re.M)
    return sorted(set(n for n in names if n.startswith(("mps_", "ea_"))))


def test_header_parses():
    names = declared_functions()
    for must in ["mps_init_product", "mps_apply_1q", "mps_apply_2q", "mps_apply_layer",
                 "mps_fidelity_estimate", "mps_expect", "mps_to_statevector"]:
        assert must in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    for name in declared_functions():
        assert hasattr(lib, name), name


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_binding_names_match_header():
    import paper_2307_16870_amd as P
    assert sorted(P.SYMBOLS) == declared_functions()
    for name in P.SYMBOLS:
        assert callable(getattr(P, name))


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_null_handle_and_last_error():
    """Argument validation happens on the host before any HIP call."""
    import paper_2307_16870_amd as P
    lib = P._binding._lib
    assert lib.mps_set_schedule(None, 0.9, 10, 1) == P.EA_EINVAL
    assert "null" in P.ea_last_error()
    assert lib.mps_fidelity_estimate(None, None, None) == P.EA_EINVAL
    h = ctypes.c_void_p()
    assert lib.mps_init_product(1, 0, 0, 0, None, None, None, ctypes.byref(h)) == P.EA_EINVAL
    assert lib.mps_init_product(4, 7, 0, 0, None, None, None, ctypes.byref(h)) == P.EA_EINVAL
    assert lib.mps_init_product(4, 0, 9, 0, None, None, None, ctypes.byref(h)) == P.EA_EINVAL
    assert lib.mps_init_product(4, 0, 0, -1, None, None, None, ctypes.byref(h)) == P.EA_EINVAL
    half = P._binding.Allocator()  # alloc without free
    half.alloc = P._binding._ALLOC_FN(lambda c, n, s: None)
    assert lib.mps_init_product(4, 0, 0, 0, None, ctypes.byref(half), None,
                                ctypes.byref(h)) == P.EA_EINVAL
    assert "allocator" in P.ea_last_error()
    assert lib.mps_set_schedule(None, 0.9, 10, P.EA_FIXED) == P.EA_EINVAL
    assert lib.mps_apply_layer_ranks(None, 0, None, None, None, None) == P.EA_EINVAL
    lib.mps_free(None)


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_tuning_table_validation_and_order():
    """The launch-shape table is host state: validated, copied and sorted
    without touching a device."""
    import paper_2307_16870_amd as P
    saved = P.mps_get_tuning()
    try:
        good = [{"f64": 1, "n_max": 2048, "block": 32, "rot_threads": 1024, "chunk_wgs": 256},
                {"f64": 0, "n_max": 512, "block": 16, "rot_threads": 256, "chunk_wgs": 128},
                {"f64": 1, "n_max": 256, "block": 16, "rot_threads": 512, "chunk_wgs": 512}]
        P.mps_set_tuning(good)
        got = P.mps_get_tuning()
        assert [(e["f64"], e["n_max"]) for e in got] == [(0, 512), (1, 256), (1, 2048)]
        assert got[2] == good[0]
        bad = [dict(good[0], block=8), dict(good[0], rot_threads=300), dict(good[0], f64=2),
               dict(good[0], n_max=0), dict(good[0], chunk_wgs=32), dict(good[0], chunk_wgs=8192)]
        for e in bad:
            with pytest.raises(P.EAError) as ei:
                P.mps_set_tuning([e])
            assert ei.value.code == P.EA_EINVAL
        with pytest.raises(P.EAError):
            P.mps_set_tuning([good[0], dict(good[0], block=16)])  # same (f64, n_max)
        assert P.mps_get_tuning() == got  # unchanged by the rejected calls
        P.mps_set_tuning([])
        assert P.mps_get_tuning() == []
    finally:
        P.mps_set_tuning(saved)
