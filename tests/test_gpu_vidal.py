"""GPU parity of the layer-parallel gauge (Vidal form, Hastings update)
through the C ABI against the oracle's layer-parallel mode: FP64 within
1e-10 (kept ranks, f, targets, ln P, amplitudes), FP32 within 1e-4; exact
against brute force without truncation; leaving the gauge for expectation
values; refusals.  Seeds are ones whose every cut lies between distinct
singular values (asserted from the oracle's spectra), where the kept vectors
are unique."""
import sys

import numpy as np
import pytest

import circuits as C
from oracle import brute
from oracle.vidal import OracleVidal
from tests.gpu_util import protected

pytestmark = pytest.mark.gpu
P = pytest.importorskip("paper_2307_16870_amd")

X, Y, Z = C.pauli_matrices()[1:]


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _oracle(prog, f_min, kind=None):
    o = OracleVidal(prog.n_sites, kind or prog.kind, keep_spectra=True)
    return o.run(prog, f_min)


def _gap(o):
    return min(((r.s[r.k - 1] - r.s[r.k]) / r.s[0] if r.k < len(r.s) else 1.0) for r in o.log)


def _run(prog, f_min, prec, kind=None):
    st = P.EAState(prog.n_sites, kind or prog.kind, prec)
    st.set_option(P.EA_OPT_GAUGE, 1)
    st.run(prog, f_min)
    return st


def test_vidal_exact_config1_vs_bruteforce():
    _say("case: vidal exact")
    prog, c = C.config_program(1)
    st = _run(prog, 1.0, "c128")
    try:
        psi = st.statevector()
        F, _ = st.fidelity_estimate()
    finally:
        st.close()
    np.testing.assert_allclose(psi, brute.run_statevector(prog), atol=1e-10)
    assert abs(F - 1.0) < 1e-12


@pytest.mark.parametrize("prec", ["c128", "c64"])
def test_vidal_truncating_pure_vs_oracle(prec):
    _say("case: vidal truncating pure", prec)
    prog = C.brickwork_program(12, 12, 57)
    o = _oracle(prog, 0.95)
    assert _gap(o) > 1e-3
    st = _run(prog, 0.95, prec)
    try:
        glog, psi, (F, lnF) = st.gate_log(), st.statevector(), st.fidelity_estimate()
    finally:
        st.close()
    tol = 1e-10 if prec == "c128" else 1e-4
    tol_w = 1e-12 if prec == "c128" else 1e-6
    assert len(glog) == len(o.log)
    for g, r in zip(glog, o.log):
        assert g["site"] == r.site
        if protected(r, r.f_t, tol_w):
            assert g["k"] == r.k
        assert abs(g["f_t"] - r.f_t) < tol
        assert abs(g["f"] - r.f) < tol
    assert abs(lnF - o.lnP) < tol
    np.testing.assert_allclose(psi, o.to_statevector(), atol=1e-10 if prec == "c128" else 3e-4)
    # every gate of a layer took the same target
    pos = 0
    for layer in prog.layers:
        fts = [g["f_t"] for g in glog[pos:pos + len(layer)]]
        assert max(fts) - min(fts) == 0.0
        pos += len(layer)


def test_vidal_larger_bonds_fp64_vs_oracle():
    """16 qubits, depth 12, F_min 0.99: bonds above 32 (three-kernel Jacobi)."""
    _say("case: vidal larger bonds")
    prog = C.brickwork_program(16, 12, 61)
    o = _oracle(prog, 0.99)
    assert max(r.k for r in o.log) > 40
    st = _run(prog, 0.99, "c128")
    try:
        glog, (F, lnF) = st.gate_log(), st.fidelity_estimate()
        psi = st.statevector()
    finally:
        st.close()
    for g, r in zip(glog, o.log):
        if protected(r, r.f_t, 1e-12):
            assert g["k"] == r.k
        assert abs(g["f"] - r.f) < 1e-10
    assert abs(lnF - o.lnP) < 1e-10
    if _gap(o) > 1e-6:
        np.testing.assert_allclose(psi, o.to_statevector(), atol=1e-9)


def test_vidal_mixed_fp64_vs_oracle():
    _say("case: vidal mixed")
    prog = C.brickwork_program(7, 6, 53, kind="mixed", noise_p=1e-2)
    o = _oracle(prog, 0.95)
    assert _gap(o) > 1e-3
    st = _run(prog, 0.95, "c128")
    try:
        glog, (F, lnF) = st.gate_log(), st.fidelity_estimate()
        rho = st.density()
    finally:
        st.close()
    for g, r in zip(glog, o.log):
        assert g["k"] == r.k
        assert abs(g["f"] - r.f) < 1e-10
        assert abs(g["lnS"] - r.lnS) < 1e-10
    assert abs(lnF - o.lnP) < 1e-10
    np.testing.assert_allclose(rho, o.to_density(), atol=1e-10)


def test_vidal_one_site_gates_and_leaving_the_gauge():
    """One-site rotations between layers (RY RZ + CZ ansatz, F_min 0.999);
    after leaving the gauge, <Z_i> and <X_i> agree with the oracle's state."""
    _say("case: vidal 1q + leave")
    angles = C.hea_angles(10, 4, seed=13)
    prog = C.hea_program(angles)
    o = _oracle(prog, 0.999)
    st = _run(prog, 0.999, "c128")
    try:
        glog = st.gate_log()
        with pytest.raises(P.EAError):
            st.expect([0], [1], [Z])
        st.set_option(P.EA_OPT_GAUGE, 0)
        ev = st.expect(list(range(10)) * 2, [1] * 20, [Z] * 10 + [X] * 10)
        psi = st.statevector()
    finally:
        st.close()
    for g, r in zip(glog, o.log):
        assert g["k"] == r.k and abs(g["f"] - r.f) < 1e-10
    phi = o.to_statevector()
    ref = [brute.expect_pure(phi, 10, i, 1, Z) for i in range(10)] + \
          [brute.expect_pure(phi, 10, i, 1, X) for i in range(10)]
    np.testing.assert_allclose(ev, np.real(ref) / np.vdot(phi, phi).real, atol=1e-10)
    np.testing.assert_allclose(psi / np.linalg.norm(psi), phi / np.linalg.norm(phi), atol=1e-10)


def test_vidal_refusals():
    _say("case: vidal refusals")
    with P.EAState(6, "pure", "c128") as st:
        st.apply_2q(0, C.haar_unitary(np.random.default_rng(1)), 1.0)
        with pytest.raises(P.EAError):  # not a product state
            st.set_option(P.EA_OPT_GAUGE, 1)
        st.reset()
        st.set_option(P.EA_OPT_GAUGE, 1)
        st.apply_2q(0, C.haar_unitary(np.random.default_rng(1)), 1.0)
        with pytest.raises(P.EAError):
            P.mps_apply_2q_noalloc(st.h, 2, C.haar_unitary(np.random.default_rng(2)), 1.0)


@pytest.mark.parametrize("prec", ["c128", "c64"])
def test_vidal_side_by_side_layer_is_bit_identical(prec):
    """A layer's gates on their own streams and threads give the same bits as
    one after another on the state's stream (16 qubits, F_min 0.99)."""
    _say("case: vidal side by side", prec)
    prog = C.brickwork_program(16, 10, 71)
    res = []
    for par in (1, 0):
        st = P.EAState(16, "pure", prec)
        try:
            st.set_option(P.EA_OPT_GAUGE_PARALLEL, par)
            st.set_option(P.EA_OPT_GAUGE, 1)
            st.run(prog, 0.99)
            res.append((st.statevector(), [(g["k"], g["f"], g["sweeps"]) for g in st.gate_log()]))
        finally:
            st.close()
    assert res[0][1] == res[1][1]
    assert np.array_equal(res[0][0], res[1][0])
