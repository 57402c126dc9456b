"""Captured programs: the device-resident small-bond launch of many circuits
as one HIP graph (mps_program_capture / mps_program_launch), against the same
launch made eagerly (mps_run_layers_batched) and against the
host-orchestrated path.  The graph is replayed several times, with other
work on the same states and synchronisations between the replays, and every
replay is checked."""
import sys

import numpy as np
import pytest

import circuits as C

pytestmark = pytest.mark.gpu
P = pytest.importorskip("paper_2307_16870_amd")


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _progs(seed, count, nmin, nmax, dmin, dmax):
    rng = np.random.default_rng(seed)
    return [C.brickwork_program(int(rng.integers(nmin, nmax + 1)), int(rng.integers(dmin, dmax + 1)),
                                1000 * seed + b) for b in range(count)]


def _layers(p):
    return [[(op.site, op.mat) for op in layer] for layer in p.layers]


def _snapshot(states):
    return [(st.statevector(), [(r["k"], r["f"], r["sweeps"]) for r in st.gate_log()],
             st.fidelity_estimate()[0], st.bond_dims(), st.center()) for st in states]


def _assert_same(a, b):
    for (psi1, log1, F1, bd1, c1), (psi2, log2, F2, bd2, c2) in zip(a, b):
        assert log1 == log2
        assert F1 == F2 and bd1 == bd2 and c1 == c2
        assert np.array_equal(psi1, psi2)


@pytest.mark.parametrize("mixed_prec", [False, True])
def test_program_equals_eager_launch_over_replays(mixed_prec):
    """Ten circuits (FP64, or FP64 and FP32 mixed) captured once and replayed
    three times from the product state; each replay bit-identical to the
    eager persistent launch on twin states.  Between replays the states run
    other work (a host-path layer) and are reset."""
    _say("case: program replays, mixed precisions" if mixed_prec else "case: program replays")
    progs = _progs(3, 10, 6, 12, 3, 9)
    precs = [("c64" if (mixed_prec and b % 2) else "c128") for b in range(len(progs))]
    twins = [P.EAState(p.n_sites, "pure", q) for p, q in zip(progs, precs)]
    for st, p in zip(twins, progs):
        st.set_schedule(0.98, p.n_2q)
    rc, codes, done_ref = P.mps_run_layers_batched([s.h for s in twins], [_layers(p) for p in progs])
    ref = _snapshot(twins)
    for st in twins:
        st.close()
    states = [P.EAState(p.n_sites, "pure", q) for p, q in zip(progs, precs)]
    prog = P.mps_program_capture([s.h for s in states], [_layers(p) for p in progs])
    try:
        for rep in range(3):
            _say("replay", rep)
            for st, p in zip(states, progs):
                st.reset()
                st.set_schedule(0.98, p.n_2q)
            rc, codes, done = P.mps_program_launch(prog)
            assert rc >= 0 and all(c >= 0 for c in codes)
            assert done == done_ref
            _assert_same(_snapshot(states), ref)
            # other work on the same states between replays
            layer = progs[0].layers[0]
            states[0].apply_layer([op.site for op in layer], np.stack([op.mat for op in layer]))
    finally:
        prog.close()
        for st in states:
            st.close()


def test_program_hands_over_to_host_path():
    """Circuits that outgrow the small limit stop on the device; the host
    path continues from there, and the result matches each circuit run
    alone on the host-orchestrated path."""
    _say("case: program hand-over")
    progs = _progs(4, 8, 10, 16, 6, 13)
    states = [P.EAState(p.n_sites, "pure", "c128") for p in progs]
    for st, p in zip(states, progs):
        st.set_schedule(0.98, p.n_2q)
    prog = P.mps_program_capture([s.h for s in states], [_layers(p) for p in progs])
    try:
        rc, codes, done = P.mps_program_launch(prog)
    finally:
        prog.close()
    assert rc >= 0
    _say("layers done:", done, "of", [len(p.layers) for p in progs])
    assert any(d < len(p.layers) for d, p in zip(done, progs))
    for t in range(max(len(p.layers) for p in progs)):
        idx = [b for b, p in enumerate(progs) if done[b] <= t < len(p.layers)]
        if idx:
            P.mps_apply_layer_batched([states[b].h for b in idx],
                                      [[op.site for op in progs[b].layers[t]] for b in idx],
                                      [np.stack([op.mat for op in progs[b].layers[t]]) for b in idx])
    for st, p in zip(states, progs):
        psi, F, log = st.statevector(), st.fidelity_estimate()[0], st.gate_log()
        st.close()
        with P.EAState(p.n_sites, "pure", "c128") as h:
            h.set_option(P.EA_OPT_SMALL_LAYERS, 0)
            h.run(p, 0.98)
            assert [r["k"] for r in log] == [r["k"] for r in h.gate_log()]
            np.testing.assert_allclose(psi, h.statevector(), atol=1e-10)
            assert abs(F - h.fidelity_estimate()[0]) < 1e-10


def test_program_argument_errors():
    progs = _progs(5, 2, 6, 8, 2, 4)
    a = P.EAState(progs[0].n_sites, "pure", "c128")
    b = P.EAState(progs[1].n_sites, "pure", "c128")
    try:
        with pytest.raises(P.EAError) as ei:
            P.mps_program_capture([a.h, a.h], [_layers(progs[0])] * 2)
        assert ei.value.code == P.EA_EINVAL
        b.set_option(P.EA_OPT_SMALL_LAYERS, 0)
        with pytest.raises(P.EAError) as ei:
            P.mps_program_capture([a.h, b.h], [_layers(progs[0]), _layers(progs[1])])
        assert ei.value.code == P.EA_EINVAL
        bad = _layers(progs[0])
        bad[0] = [(progs[0].n_sites - 1, bad[0][0][1])]  # pair off the chain's end
        with pytest.raises(P.EAError) as ei:
            P.mps_program_capture([a.h], [bad])
        assert ei.value.code == P.EA_ERANGE
    finally:
        a.close()
        b.close()
