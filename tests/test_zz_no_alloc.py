"""The allocation-free two-site update (mps_apply_2q_noalloc) against
mps_apply_2q through the C ABI: the same kernels on the same inputs, so every
output must be bit-identical (kept rank, f, T, sweeps, both site tensors).
Two calls in a row share the library's device array, the second on smaller
matrices; a centre move inside the call; a site buffer too small is refused
before the state changes; and the 2048 x 2048 factorisation of a bond-1024
update fits the array."""
import numpy as np
import pytest

import circuits as C

pytestmark = pytest.mark.gpu
P = pytest.importorskip("paper_2307_16870_amd")


def _update(prec, chis, seed, noalloc, center=1, site=1, reserve=None, chi_max=0):
    n = len(chis) + 1
    tens = C.random_mps_tensors([1, *chis, 1], 2, seed=seed)
    G = C.haar_unitary(np.random.default_rng(seed))
    with P.EAState(n, "pure", prec, chi_max=chi_max) as st:
        st.load(tens, center)
        if reserve:
            st.set_option(P.EA_OPT_RESERVE_BOND, reserve)
        fn = P.mps_apply_2q_noalloc if noalloc else P.mps_apply_2q
        rc, f = fn(st.h, site, G, 0.98)
        return rc, f, st.gate_log()[-1], [st.site(i) for i in range(n)], st.bond_dims()


def _same(a, b):
    rca, fa, ga, sa, ba = a
    rcb, fb, gb, sb, bb = b
    assert rca == rcb and fa == fb
    for key in ("k", "k_f", "f", "total", "sweeps", "capped", "chi_l", "chi_r"):
        assert ga[key] == gb[key], key
    assert ba == bb
    for x, y in zip(sa, sb):
        assert x.shape == y.shape and np.array_equal(x, y)


@pytest.mark.parametrize("prec", ["c128", "c64"])
def test_noalloc_two_calls_in_a_row(prec):
    print("case: noalloc two calls", prec, flush=True)
    big, small = (300, 260, 333), (100, 128, 90)
    r_big = _update(prec, big, 11, True, reserve=600)
    r_small = _update(prec, small, 12, True, reserve=200)
    _same(r_big, _update(prec, big, 11, False, reserve=600))
    _same(r_small, _update(prec, small, 12, False, reserve=200))


@pytest.mark.parametrize("center,site", [(0, 6), (13, 4)])
@pytest.mark.parametrize("prec", ["c128", "c64"])
def test_noalloc_with_centre_moves(prec, center, site):
    """The centre several sites away from the gate: the call first moves it
    (Cholesky QR moves, right or left, on site matrices up to 128 x 64)."""
    print("case: noalloc centre moves", prec, center, site, flush=True)
    chis = (2, 4, 8, 16, 32, 64, 128, 64, 32, 16, 8, 4, 2)
    a = _update(prec, chis, 21, True, center=center, site=site, reserve=256)
    b = _update(prec, chis, 21, False, center=center, site=site, reserve=256)
    _same(a, b)


def test_noalloc_refuses_small_site_buffer():
    """Without reserved bond capacity the kept rank does not fit the loaded
    site buffers: EA_ETOOBIG, nothing written, the state as before."""
    print("case: noalloc refusal", flush=True)
    chis = (40, 30, 40)
    tens = C.random_mps_tensors([1, *chis, 1], 2, seed=5)
    G = C.haar_unitary(np.random.default_rng(5))
    with P.EAState(4, "pure", "c128") as st:
        st.load(tens, 1)
        before = st.statevector()
        with pytest.raises(P.EAError) as e:
            P.mps_apply_2q_noalloc(st.h, 1, G, 1.0)
        assert e.value.code == P.EA_ETOOBIG
        assert st.gate_log() == []
        np.testing.assert_allclose(st.statevector(), before, atol=1e-13)


@pytest.mark.parametrize("prec", ["c64", "c128"])
def test_noalloc_full_size_bond_1024(prec):
    """chi = 1024 (Theta 2048 x 2048, kept rank capped at 1024 as in the
    50-qubit workload) fits the 256 MiB array."""
    print("case: noalloc chi=1024", prec, flush=True)
    chis = (1024, 1024, 1024)
    a = _update(prec, chis, 31, True, reserve=1024, chi_max=1024)
    b = _update(prec, chis, 31, False, reserve=1024, chi_max=1024)
    assert a[2]["capped"] and a[2]["k"] == 1024
    _same(a, b)
