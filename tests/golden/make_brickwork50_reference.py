"""Write the oracle's record of the 50-qubit, depth-20 brickwork workload
(Haar two-qubit gates, global fidelity schedule with F_min = 0.99, bond cap
1024) to ``brickwork50_depth20_oracle.json``.

Calls only the oracle (FP64; its SVD step is the LAPACK routine, which the CPU
tests pin to the oracle's own Jacobi) and the seeded circuit generator.  Per
two-qubit gate it stores the kept rank, the truncation fidelity, the running
log-fidelity, the total weight and the discarded weights at the chosen rank and
one below it relative to the threshold (so a test can tell which rank
decisions are protected by a margin); at the end it stores one- and two-site
expectation values.  Takes about an hour on 8 cores.

    python tests/golden/make_brickwork50_reference.py
"""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import circuits as C  # noqa: E402
from oracle.mps import OracleMPS  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "brickwork50_depth20_oracle.json")
Z = np.diag([1.0, -1.0]).astype(complex)
X = np.array([[0, 1], [1, 0]], dtype=complex)
OBS = ([("Z", s, 1) for s in (0, 7, 13, 24, 25, 36, 49)] + [("X", s, 1) for s in (3, 24, 40)]
       + [("ZZ", s, 2) for s in (0, 12, 24, 48)])


def main():
    prog, c = C.config_program(2)
    o = OracleMPS(prog.n_sites, "pure", chi_max=c["chi_max"], svd="lapack", keep_spectra=True)
    o.set_schedule(c["f_min"], prog.n_2q)
    t0 = time.time()
    gates = []
    for li, layer in enumerate(prog.layers):
        for op in layer:
            if op.width == 1:
                o.apply_1q(op.site, op.mat)
        recs = o.apply_layer([op for op in layer if op.width == 2])
        for r in recs:
            w = r.s * r.s
            T = float(w.sum())
            thr = (1.0 - r.f_t) * T
            gates.append(dict(gate=r.gate, site=r.site, chi=[r.chi_l, r.chi_m, r.chi_r], k=r.k,
                              f_t=r.f_t, f=r.f, lnP=r.lnP, total=T, capped=bool(r.capped),
                              margin_k=float((w[r.k:].sum() - thr) / T),
                              margin_km1=float((w[r.k - 1:].sum() - thr) / T)))
            r.s = None
        print(f"layer {li} done at {time.time() - t0:.0f}s, max bond {max(o.bond_dims())}", flush=True)
    obs = []
    for name, s, w in OBS:
        op = {"Z": Z, "X": X, "ZZ": np.kron(Z, Z)}[name]
        v = o.expect(s, w, op)
        obs.append(dict(name=name, site=s, width=w, re=float(v.real), im=float(v.imag)))
    out = dict(workload=dict(n=prog.n_sites, depth=c["depth"], f_min=c["f_min"],
                             chi_max=c["chi_max"], seed=c["seed"]),
               lnP=o.lnP, bonds=o.bond_dims(), center=o.center, gates=gates, observables=obs)
    with open(OUT, "w") as fh:
        json.dump(out, fh, indent=0)
    print("wrote", OUT, flush=True)


if __name__ == "__main__":
    main()
