"""Object wrapper over the C ABI handle and a circuit walker.

``EAState`` owns one ``ea_mps`` handle.  ``run`` hands a circuit to the
library layer by layer (one-qubit operators one by one, then all two-qubit
operators of the layer in one ``mps_apply_layer`` call); it does no
arithmetic of its own.
"""
from __future__ import annotations

import numpy as np

from . import _binding as B


class EAState:
    def __init__(self, n_sites, kind="pure", prec="c128", chi_max=0, local=None, stream=None,
                 allocator=None):
        """allocator: None (hipMalloc) or "torch" (torch's caching allocator)."""
        self.n = int(n_sites)
        self.kind = kind
        self.d = 2 if kind == "pure" else 4
        k = B.EA_PURE if kind == "pure" else B.EA_MIXED
        p = {"c128": B.EA_C128, "c64": B.EA_C64, "bf16x3": B.EA_C64_BF16X3}[prec]
        self.h = B.mps_init_product(self.n, k, p, chi_max, local, stream, allocator)
        self.warnings = 0

    def close(self):
        if getattr(self, "h", None) is not None:
            B.mps_free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    # ---------------------------------------------------------------- calls
    def set_option(self, opt, val):
        return B.mps_set_option(self.h, opt, val)

    def set_schedule(self, f_min, n_total, strategy=B.EA_GLOBAL):
        return B.mps_set_schedule(self.h, f_min, n_total, strategy)

    def apply_1q(self, site, op):
        return B.mps_apply_1q(self.h, site, op)

    def apply_2q(self, site, op, budget=-1.0):
        return B.mps_apply_2q(self.h, site, op, budget)

    def apply_layer(self, sites, ops, budgets=None):
        return B.mps_apply_layer(self.h, sites, ops, budgets)

    def apply_layer_ranks(self, sites, ops, ranks):
        return B.mps_apply_layer_ranks(self.h, sites, ops, ranks)

    def fidelity_estimate(self):
        return B.mps_fidelity_estimate(self.h)

    def expect(self, sites, widths, ops):
        return B.mps_expect(self.h, sites, widths, ops)

    def statevector(self):
        return B.mps_to_statevector(self.h, 2 ** self.n)

    def density(self):
        dim = 2 ** self.n
        return B.mps_to_statevector(self.h, dim * dim).reshape(dim, dim)

    def bond_dims(self):
        return B.mps_bond_dims(self.h, self.n)

    def center(self):
        return B.mps_center(self.h)

    def gate_log(self):
        return B.mps_gate_log(self.h)

    def load(self, tensors, center):
        return B.mps_load(self.h, tensors, center)

    def site(self, i):
        return B.mps_get_site(self.h, i)

    def reset(self, local=None):
        self.warnings = 0
        return B.mps_reset_product(self.h, local)

    def profile(self, enable):
        return B.mps_profile(self.h, enable)

    def profile_read(self, family):
        return B.mps_profile_read(self.h, family)

    # -------------------------------------------------------------- circuit
    def run(self, program, f_min=1.0, strategy=B.EA_GLOBAL, schedule=True):
        """Apply a ``circuits.Program``; returns the number of warnings."""
        if schedule:
            self.set_schedule(f_min, max(1, program.n_2q), strategy)
        for layer in program.layers:
            self.run_layer(layer)
        return self.warnings

    def run_layer(self, layer, visit_ranks=None):
        """One-qubit ops of the layer in order, then its two-qubit ops, with
        their kept ranks forced if ``visit_ranks`` lists one per two-qubit op
        in the order the library visits them (as ``gate_log`` records it)."""
        for op in layer:
            if op.width == 1:
                self.apply_1q(op.site, op.mat)
        twos = [op for op in layer if op.width == 2]
        if twos:
            sites, mats = [op.site for op in twos], np.stack([op.mat for op in twos])
            if visit_ranks is None:
                rc, _ = self.apply_layer(sites, mats)
            else:
                # the library visits ascending if the centre is nearer the
                # lowest site, else descending
                c = self.center()
                asc = abs(c - min(sites)) <= abs(c - max(sites))
                order = sorted(range(len(twos)), key=lambda j: sites[j], reverse=not asc)
                ranks = [0] * len(twos)
                for t, j in enumerate(order):
                    ranks[j] = int(visit_ranks[t])
                rc, _ = self.apply_layer_ranks(sites, mats, ranks)
            if rc > 0:
                self.warnings += 1

    def replay(self, program, ranks, f_min=1.0, strategy=B.EA_GLOBAL):
        """Apply a program with the kept rank of every two-qubit gate given
        (``ranks`` in visiting order, as ``gate_log`` lists them): the
        forced-rank replay of a recorded run."""
        self.set_schedule(f_min, max(1, program.n_2q), strategy)
        pos = 0
        for layer in program.layers:
            n2 = sum(1 for op in layer if op.width == 2)
            self.run_layer(layer, list(ranks[pos:pos + n2]) if n2 else None)
            pos += n2
        return self.warnings


def capture_batched(states, programs):
    """Capture the leading device-resident launch of ``run_batched`` for these
    states and programs as a replayable HIP graph (``mps_program_capture``)."""
    layers = [[[(op.site, op.mat) for op in layer] for layer in p.layers] for p in programs]
    return B.mps_program_capture([s.h for s in states], layers)


def run_batched(states, programs, f_min=1.0, strategy=B.EA_GLOBAL, persistent=True,
                captured=None, progress=None):
    """Advance independent states through their programs together.  With
    ``persistent`` the leading small-bond layers of all states run in one
    device-resident launch (``mps_run_layers_batched``, or a replay of
    ``captured`` from ``capture_batched`` on the same states and programs);
    then every remaining layer is one ``mps_apply_layer_batched`` call over
    the states that still have it.  Programs must hold two-qubit gates only.
    ``progress(t)``, if given, is called after each such layer.  Returns the
    worst status seen."""
    for st, p in zip(states, programs):
        st.set_schedule(f_min, max(1, p.n_2q), strategy)
    done = [0] * len(states)
    worst = 0
    if captured is not None:
        rc, _, done = B.mps_program_launch(captured)
        worst = max(worst, rc)
    elif persistent:
        layers = [[[(op.site, op.mat) for op in layer] for layer in p.layers] for p in programs]
        rc, _, done = B.mps_run_layers_batched([s.h for s in states], layers)
        worst = max(worst, rc)
    depth = max((len(p.layers) for p in programs), default=0)
    for t in range(min(done, default=0), depth):
        idx = [b for b, p in enumerate(programs) if done[b] <= t < len(p.layers)]
        if not idx:
            continue
        sites = [[op.site for op in programs[b].layers[t]] for b in idx]
        ops = [np.stack([op.mat for op in programs[b].layers[t]]) for b in idx]
        rc, _, _ = B.mps_apply_layer_batched([states[b].h for b in idx], sites, ops)
        worst = max(worst, rc)
        if progress is not None:
            progress(t)
    return worst
