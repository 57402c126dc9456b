"""Device-resident small-bond layers (one workgroup walks a state's layer with
every size read on the device) against the host-orchestrated path, the
oracle and brute force.  Circuits are chosen so that bonds outgrow the small
limit part-way through, which exercises the hand-over between the two paths."""
import sys

import numpy as np
import pytest

import circuits as C
from oracle import brute
from tests.gpu_util import oracle_run, protected

pytestmark = pytest.mark.gpu
P = pytest.importorskip("paper_2307_16870_amd")


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _run(prog, prec, f_min, small, kind="pure"):
    with P.EAState(prog.n_sites, kind, prec) as st:
        st.set_option(P.EA_OPT_SMALL_LAYERS, small if small is not True else 64)
        st.run(prog, f_min)
        out = (st.statevector() if kind == "pure" else st.density(), st.fidelity_estimate()[0],
               st.gate_log(), st.bond_dims())
    return out


@pytest.mark.parametrize("n,depth,seed,cols", [(14, 12, 11, 64), (11, 9, 12, 64),
                                               (16, 15, 13, 64), (16, 15, 13, 128)])
def test_small_path_fp64_matches_host_path_and_oracle(n, depth, seed, cols):
    _say("case: small fp64", n, depth, seed, cols)
    prog = C.brickwork_program(n, depth, seed)
    psi_s, F_s, log_s, b_s = _run(prog, "c128", 0.97, cols)
    psi_h, F_h, log_h, b_h = _run(prog, "c128", 0.97, 0)
    o = oracle_run(prog, 0.97)
    for g, r in zip(log_s, o.log):
        if protected(r, r.f_t, 1e-12):
            assert g["k"] == r.k
        assert abs(g["f"] - r.f) < 1e-10
    assert [g["k"] for g in log_s] == [g["k"] for g in log_h]
    np.testing.assert_allclose(psi_s, psi_h, atol=1e-10)
    np.testing.assert_allclose(psi_s, o.to_statevector(), atol=1e-10)
    assert abs(F_s - o.fidelity_estimate()[0]) < 1e-10
    _say("largest bond", max(b_s))


def test_small_path_exact_vs_bruteforce():
    """12 qubits, depth 8, F_min = 1: every amplitude against the state vector."""
    _say("case: small exact")
    prog, c = C.config_program(1)
    psi, F, log, _ = _run(prog, "c128", 1.0, True)
    ref = brute.run_statevector(prog)
    np.testing.assert_allclose(psi, ref, atol=1e-12)
    assert abs(F - 1.0) < 1e-12


def test_small_path_fp32_and_bf16x3():
    prog = C.brickwork_program(12, 8, 21)
    ref, _, _, _ = _run(prog, "c128", 0.98, 0)
    for prec in ("c64", "bf16x3"):
        _say("case: small", prec)
        psi, F, log, _ = _run(prog, prec, 0.98, True)
        psi_h, F_h, _, _ = _run(prog, prec, 0.98, 0)
        assert np.abs(psi - ref).max() < 2e-4
        assert abs(F - F_h) < 1e-5


def test_small_path_mpo_vs_bruteforce():
    """Noisy MPO (d = 4), 6 qubits, whole layers of fused unitary +
    depolarising superoperators, no truncation: the density matrix."""
    _say("case: small mpo")
    n = 6
    rng = np.random.default_rng(31)
    gates = []
    with P.EAState(n, "mixed", "c128") as st:
        st.set_option(P.EA_OPT_SMALL_LAYERS, 64)
        for t in range(5):
            pairs = list(C.brickwork_pairs(n, t))
            ops = []
            for i in pairs:
                u = C.haar_unitary(rng)
                ops.append(C.depolarizing2_superop(0.02) @ C.unitary_superop(u))
                gates.append((i, 2, u, 0.02))
            st.apply_layer(pairs, np.stack(ops))
        rho_g = st.density()
    rho = brute.run_density(n, gates)
    np.testing.assert_allclose(rho_g, rho, atol=1e-10)


@pytest.mark.parametrize("cols", [64, 128])
def test_small_batched_many_states_one_launch(cols):
    """Twenty states of different sizes in one launch per layer, against each
    state run alone on the host-orchestrated path."""
    _say("case: small batched", cols)
    rng = np.random.default_rng(5)
    progs = [C.brickwork_program(int(rng.integers(6, 16)), int(rng.integers(3, 13)), 500 + b)
             for b in range(20)]
    states = [P.EAState(p.n_sites, "pure", "c128") for p in progs]
    for st, p in zip(states, progs):
        st.set_option(P.EA_OPT_SMALL_LAYERS, cols)
        st.set_schedule(0.98, p.n_2q)
    depth = max(len(p.layers) for p in progs)
    for t in range(depth):
        sites, ops = [], []
        for p in progs:
            layer = p.layers[t] if t < len(p.layers) else []
            sites.append([op.site for op in layer])
            ops.append(np.stack([op.mat for op in layer]) if layer else np.zeros((0, 4, 4), complex))
        rc, codes, _ = P.mps_apply_layer_batched([s.h for s in states], sites, ops)
        assert rc >= 0 and all(c >= 0 for c in codes)
    for st, p in zip(states, progs):
        psi = st.statevector()
        ks = [r["k"] for r in st.gate_log()]
        st.close()
        psi_h, F_h, log_h, _ = _run(p, "c128", 0.98, 0)
        assert ks == [r["k"] for r in log_h]
        np.testing.assert_allclose(psi, psi_h, atol=1e-10)


@pytest.mark.parametrize("prec", ["c128", "c64"])
def test_persistent_launch_then_layer_batches(prec):
    """The leading small-bond layers of sixteen circuits in one launch, the
    rest layer by layer, against each circuit run alone on the
    host-orchestrated path; some circuits outgrow the limit part-way."""
    _say("case: persistent batched", prec)
    rng = np.random.default_rng(8)
    progs = [C.brickwork_program(int(rng.integers(8, 17)), int(rng.integers(4, 15)), 700 + b)
             for b in range(16)]
    states = [P.EAState(p.n_sites, "pure", prec) for p in progs]
    layers = [[[(op.site, op.mat) for op in layer] for layer in p.layers] for p in progs]
    for st, p in zip(states, progs):
        st.set_schedule(0.98, p.n_2q)
    rc, codes, done = P.mps_run_layers_batched([s.h for s in states], layers)
    assert rc >= 0 and all(c >= 0 for c in codes)
    _say("layers done on the device:", done, "of", [len(p.layers) for p in progs])
    assert any(d < len(p.layers) for d, p in zip(done, progs))
    assert any(d == len(p.layers) for d, p in zip(done, progs))
    for t in range(max(len(p.layers) for p in progs)):
        idx = [b for b, p in enumerate(progs) if done[b] <= t < len(p.layers)]
        if idx:
            P.mps_apply_layer_batched([states[b].h for b in idx],
                                      [[op.site for op in progs[b].layers[t]] for b in idx],
                                      [np.stack([op.mat for op in progs[b].layers[t]]) for b in idx])
    for st, p in zip(states, progs):
        psi = st.statevector()
        F = st.fidelity_estimate()[0]
        log = st.gate_log()
        st.close()
        psi_h, F_h, log_h, _ = _run(p, prec, 0.98, 0)
        assert len(log) == len(log_h) == p.n_2q
        if prec == "c128":
            assert [r["k"] for r in log] == [r["k"] for r in log_h]
            np.testing.assert_allclose(psi, psi_h, atol=1e-10)
            assert abs(F - F_h) < 1e-10
        else:
            assert np.abs(psi - psi_h).max() < 1e-3
            assert abs(F - F_h) < 1e-4


def test_run_batched_driver():
    progs = [C.brickwork_program(10, 6, 900 + b) for b in range(4)]
    states = [P.EAState(p.n_sites, "pure", "c128") for p in progs]
    P.run_batched(states, progs, 0.99)
    for st, p in zip(states, progs):
        psi = st.statevector()
        st.close()
        psi_h, _, _, _ = _run(p, "c128", 0.99, 0)
        np.testing.assert_allclose(psi, psi_h, atol=1e-10)


def test_run_batched_driver_with_captured_program():
    """The driver's replay of a captured program equals its eager launch."""
    progs = [C.brickwork_program(12, 9, 950 + b) for b in range(4)]
    ref = []
    for b, p in enumerate(progs):
        with P.EAState(p.n_sites, "pure", "c128") as st:
            P.run_batched([st], [p], 0.99)
            ref.append(st.statevector())
    states = [P.EAState(p.n_sites, "pure", "c128") for p in progs]
    graph = P.capture_batched(states, progs)
    for _ in range(2):
        for st in states:
            st.reset()
        P.run_batched(states, progs, 0.99, captured=graph)
        for st, r in zip(states, ref):
            np.testing.assert_allclose(st.statevector(), r, atol=1e-12)
    graph.close()
    for st in states:
        st.close()

