"""Autotuner of the three-kernel Jacobi launch shape.

For each working precision (complex FP32, complex FP64) and factorisation
width n (the columns of Theta = 2 chi for a pure-state update at bond chi,
4 chi for an MPO update), it times one two-site update on seeded random
site tensors with each candidate shape and keeps the fastest:

* block width and rotation-kernel threads, with 256 row-chunk workgroups;
* then the row-chunk workgroup target, with the best of the above.

The winners form the table of ``mps_set_tuning`` (an entry per width, each
covering the widths above the previous one), written as JSON.  Every update
runs through the library; the script only chooses among launch shapes whose
results differ by rounding alone.

    python -m paper_2307_16870_amd.autotune [--out FILE] [--reps R] [--widths 128,256,...]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

from . import _binding as B
from .driver import EAState

DEFAULT_OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuning_gfx950.json")
BLOCK_THREADS = [(32, 1024), (32, 512), (32, 256), (16, 512), (16, 256), (16, 1024)]
CHUNK_WGS = [128, 256, 512]


def _tensors(chi, d, seed):
    """Three random site tensors (chi, d, chi) between unit outer bonds."""
    rng = np.random.default_rng(seed)
    dims = [1, chi, chi, chi, 1]
    out = []
    for i in range(4):
        a = rng.standard_normal((dims[i], d, dims[i + 1])) + 1j * rng.standard_normal(
            (dims[i], d, dims[i + 1]))
        out.append(a / np.linalg.norm(a))
    return out


def _haar4(seed):
    rng = np.random.default_rng(seed)
    z = (rng.standard_normal((4, 4)) + 1j * rng.standard_normal((4, 4))) / np.sqrt(2)
    q, r = np.linalg.qr(z)
    return q * (np.diag(r) / np.abs(np.diag(r)))


def time_update(prec, n, block, threads, wgs, reps, log):
    """Median wall time (s) of one two-site update whose Theta has n columns."""
    chi = n // 2
    tens = _tensors(chi, 2, seed=n)
    gate = _haar4(n + 1)
    B.mps_set_tuning([{"f64": int(prec == "c128"), "n_max": 1 << 30, "block": block,
                       "rot_threads": threads, "chunk_wgs": wgs}])
    times = []
    with EAState(4, "pure", prec) as st:
        st.load(tens, 1)
        st.apply_2q(1, gate, 0.99)  # code objects and buffers
        for _ in range(reps):
            st.load(tens, 1)
            t0 = time.perf_counter()
            st.apply_2q(1, gate, 0.99)  # returns after the decision is read back
            times.append(time.perf_counter() - t0)
    t = float(np.median(times))
    log(f"{prec} n={n} block={block} threads={threads} wgs={wgs}: {1e3 * t:.2f} ms")
    return t


def tune(widths, precs=("c64", "c128"), reps=3, log=print):
    entries, timings = [], []
    saved = B.mps_get_tuning()
    try:
        for prec in precs:
            for n in widths:
                best = None
                for block, threads in BLOCK_THREADS:
                    t = time_update(prec, n, block, threads, 256, reps, log)
                    timings.append({"prec": prec, "n": n, "block": block, "rot_threads": threads,
                                    "chunk_wgs": 256, "ms": 1e3 * t})
                    if best is None or t < best[0]:
                        best = (t, block, threads, 256)
                for wgs in CHUNK_WGS:
                    if wgs == 256:
                        continue
                    t = time_update(prec, n, best[1], best[2], wgs, reps, log)
                    timings.append({"prec": prec, "n": n, "block": best[1],
                                    "rot_threads": best[2], "chunk_wgs": wgs, "ms": 1e3 * t})
                    if t < best[0]:
                        best = (t, best[1], best[2], wgs)
                entries.append({"f64": int(prec == "c128"), "n_max": n, "block": best[1],
                                "rot_threads": best[2], "chunk_wgs": best[3]})
    finally:
        B.mps_set_tuning(saved)
    # the widest entry of each precision also covers anything wider
    for f64 in (0, 1):
        mine = [e for e in entries if e["f64"] == f64]
        if mine:
            max(mine, key=lambda e: e["n_max"])["n_max"] = 1 << 30
    return entries, timings


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--out", default=DEFAULT_OUT)
    ap.add_argument("--reps", type=int, default=3)
    ap.add_argument("--widths", default="128,256,512,1024,2048")
    args = ap.parse_args(argv)
    widths = [int(x) for x in args.widths.split(",")]

    def log(*a):
        print(*a, file=sys.stderr, flush=True)

    entries, timings = tune(widths, reps=args.reps, log=log)
    with open(args.out, "w") as fh:
        json.dump({"device": "MI355X (gfx950)", "widths": widths, "reps": args.reps,
                   "entries": entries,
                   "timings": timings}, fh, indent=1)
    log(f"wrote {args.out}")
    print(json.dumps(entries))


if __name__ == "__main__":
    main()
