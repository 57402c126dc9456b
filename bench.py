#!/usr/bin/env python3
"""Throughput of the entanglement-aware two-site gate update on one MI355X.

Workload (one "step"): the noiseless 1D brickwork circuit of 50 qubits and
depth 20 with seeded Haar-random U(4) gates, started from |0...0>, run with
the global target schedule for F_min = 0.99 and a bond cap of 1024 -- 490
two-site updates (contract, gate, SVD, truncate, fidelity product), plus the
orthogonality-centre moves between them.  Default arithmetic: complex FP32
contraction and Jacobi rotations, FP64 singular-value sums, kept-rank search
and fidelity product.

Prints one JSON line.  ``value`` is two-site updates per second over the
timed steps (inputs are generated on the host before timing; the state lives
in device memory throughout).  ``roofline`` reports the kernel family with
the largest device time.  During the timed steps every launch is counted
with its algorithmic flops and bytes, and one launch in PROF_EVERY of each
family is timed with a HIP event pair on the library's stream (timing every
launch adds about a fifth to the FP32 circuit); the family's average launch
time is that of the timed launches.  ``cpu_baseline`` times the CPU oracle
on the first layers of the same circuit.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAKS = {  # MI355X published peaks
    "hbm_GBs": 8000.0,
    "f32_vector_TF": 157.3, "f64_vector_TF": 78.6,
    "f32_mfma_TF": 157.3, "f64_mfma_TF": 78.6, "bf16_mfma_TF": 2500.0,
}


PROF_EVERY = 16  # one launch in 16 of each kernel family is timed with events


def log(*a):
    print(*a, file=sys.stderr, flush=True)


# ---------------------------------------------------------------- HBM traffic
# roofline.traffic comes from rocprofv3 counter runs (FETCH_SIZE, then
# WRITE_SIZE, KiB per dispatch) of this script, each scaled by what the same
# counter reads for a device copy of known size (--calibrate-copy), and is
# stored in profiles/traffic.json together with a digest of the kernel
# sources; it is reported only while the sources are unchanged.
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic.json")
CSRC = os.path.join(ROOT, "paper_2307_16870_amd", "csrc")
COPY_BYTES = 256 << 20


def source_digest():
    import hashlib
    h = hashlib.sha256()
    for f in sorted(os.listdir(CSRC)):
        if f.endswith((".hip", ".h")):
            with open(os.path.join(CSRC, f), "rb") as fh:
                h.update(f.encode() + b"\0" + fh.read())
    return h.hexdigest()


def traffic_for(kernel):
    try:
        with open(TRAFFIC_FILE) as fh:
            d = json.load(fh)
    except (OSError, ValueError):
        return None
    e = d.get("kernels", {}).get(kernel)
    if e is None or d.get("source_sha256") != source_digest():
        return None
    return e["hbm_bytes_per_launch"]


def calibrate_copy():
    """A plain device copy of COPY_BYTES, five times (profiled with --pmc)."""
    import torch
    a = torch.empty(COPY_BYTES // 4, dtype=torch.float32, device="cuda").fill_(1.0)
    b = torch.empty_like(a)
    for _ in range(5):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes": COPY_BYTES, "repeats": 5}))


def summarize_pmc(run_dir):
    """Write run_dir/traffic.json (the content of profiles/traffic.json) from
    counter CSVs under run_dir: fetch/ and write/ (bench run), copy_fetch/
    and copy_write/ (calibration)."""
    import csv
    import glob

    def per_kernel(sub, counter):
        vals = {}
        for f in glob.glob(os.path.join(run_dir, sub, "**", "*counter_collection.csv"),
                           recursive=True):
            for r in csv.DictReader(open(f)):
                if r["Counter_Name"] != counter:
                    continue
                name = r["Kernel_Name"].split("(")[0].split("<")[0].replace("void ", "").strip()
                vals.setdefault(name, []).append(float(r["Counter_Value"]))
        return {k: sum(v) / len(v) for k, v in vals.items()}, {k: len(v) for k, v in vals.items()}

    cf, _ = per_kernel("copy_fetch", "FETCH_SIZE")
    cw, _ = per_kernel("copy_write", "WRITE_SIZE")
    copy_k = max(cf, key=cf.get)
    f_fetch = COPY_BYTES / (cf[copy_k] * 1024.0)
    f_write = COPY_BYTES / (cw[copy_k] * 1024.0)
    fe, nf = per_kernel("fetch", "FETCH_SIZE")
    wr, _ = per_kernel("write", "WRITE_SIZE")
    out = {"source_sha256": source_digest(),
           "calibration": {"copy_kernel": copy_k, "copy_bytes": COPY_BYTES,
                           "fetch_KiB": cf[copy_k], "write_KiB": cw[copy_k],
                           "fetch_factor": f_fetch, "write_factor": f_write},
           "kernels": {}}
    for k in fe:
        fb = fe[k] * 1024.0 * f_fetch
        wb = wr.get(k, 0.0) * 1024.0 * f_write
        out["kernels"][k] = {"launches": nf[k], "fetch_bytes_per_launch": fb,
                             "write_bytes_per_launch": wb, "hbm_bytes_per_launch": fb + wb}
    with open(os.path.join(run_dir, "traffic.json"), "w") as fh:
        json.dump(out, fh, indent=1)
    print(json.dumps(out, indent=1))


def run_circuit(st, prog, f_min, progress=False):
    st.reset()
    st.set_schedule(f_min, prog.n_2q)
    t0 = time.perf_counter()
    for li, layer in enumerate(prog.layers):
        st.run_layer(layer)
        if progress:
            log(f"  layer {li} done at {time.perf_counter() - t0:.1f}s")


def _timed_oracle(prog, chi_max, svd):
    """The oracle with every two-site update (its centre moves included)
    timed: records (seconds, d, chi_l, chi_r)."""
    from oracle.mps import OracleMPS

    class TimedOracle(OracleMPS):
        def apply_2q(self, i, G, f_t=None, direction="right", forced_k=None):
            t0 = time.perf_counter()
            rec = super().apply_2q(i, G, f_t, direction, forced_k)
            self.times.append((time.perf_counter() - t0, self.d, rec.chi_l, rec.chi_r))
            return rec

    o = TimedOracle(prog.n_sites, "pure", chi_max=chi_max, svd=svd)
    o.times = []
    return o


def _update_cost(d, chi_l, chi_r):
    """Cost model of one update on the CPU: the SVD of the (d chi_l) x
    (d chi_r) two-site matrix, m n min(m, n) (the contraction and the move
    scale the same way at equal bonds)."""
    m, n = d * chi_l, d * chi_r
    return float(m) * n * min(m, n)


def cpu_baseline(prog, f_min, chi_max, n_layers, budget_s, gpu_log=None, gpu_prefix_s=None):
    """The oracle (complex128, its own one-sided Jacobi SVD, all host cores)
    on the first layers of the same circuit, and beside it the same oracle
    with LAPACK's SVD (the fair CPU speed baseline) on the same layers.  The
    GPU's time for the same layers is reported next to it.  From the
    per-update times, binned by (d, chi_l, chi_r), a fitted a + b m n min(m, n)
    model extrapolates the oracle to the whole circuit (labelled as such)."""
    import numpy as np
    legs = {}
    used = 0
    for svd in ("auto", "lapack"):
        o = _timed_oracle(prog, chi_max, svd)
        o.set_schedule(f_min, prog.n_2q)
        t0 = time.perf_counter()
        n_upd = 0
        layers = prog.layers[:n_layers] if svd == "auto" else prog.layers[:used]
        for layer in layers:
            o.apply_layer(layer)
            n_upd += len(layer)
            if svd == "auto":
                used += 1
                if time.perf_counter() - t0 > budget_s:
                    break
        dt = time.perf_counter() - t0
        legs[svd] = {"seconds": dt, "updates": n_upd, "times": o.times,
                     "max_bond": max(o.bond_dims())}
    jac = legs["auto"]
    cores = len(os.sched_getaffinity(0))
    out = {
        "value": jac["updates"] / jac["seconds"], "unit": "updates/s", "cores": cores,
        "kind": "oracle",
        "sample": (f"first {used} of {len(prog.layers)} layers ({jac['updates']} of {prog.n_2q} "
                   f"updates, bonds up to {jac['max_bond']}) of the same circuit; complex128 "
                   f"oracle with its own one-sided Jacobi SVD; {jac['seconds']:.1f} s"),
        "lapack": {"value": legs["lapack"]["updates"] / legs["lapack"]["seconds"],
                   "unit": "updates/s",
                   "sample": f"the same {used} layers, the oracle with LAPACK's SVD "
                             f"(numpy.linalg.svd); {legs['lapack']['seconds']:.1f} s"},
    }
    if gpu_prefix_s is not None:
        out["gpu_same_sample"] = {"value": jac["updates"] / gpu_prefix_s, "unit": "updates/s",
                                  "seconds": gpu_prefix_s,
                                  "sample": f"the GPU path on the same {used} layers"}
    if gpu_log:
        # per-update CPU cost extrapolated to the whole circuit with the GPU
        # run's bonds (same schedule, same ranks up to rounding)
        for name, leg in (("extrapolated_oracle", jac), ("extrapolated_lapack", legs["lapack"])):
            t = np.array([x[0] for x in leg["times"]])
            c = np.array([_update_cost(*x[1:]) for x in leg["times"]])
            # least squares t = a + b c over per-(d, chi_l, chi_r) bin means
            bins = {}
            for ti, x in zip(t, leg["times"]):
                bins.setdefault(x[1:], []).append(ti)
            cb = np.array([_update_cost(*k) for k in bins])
            tb = np.array([np.mean(v) for v in bins.values()])
            A = np.stack([np.ones_like(cb), cb], axis=1)
            (a, b), *_ = np.linalg.lstsq(A, tb, rcond=None)
            a, b = max(a, 0.0), max(b, 1e-30)
            full = sum(a + b * _update_cost(2, r["chi_l"], r["chi_r"]) for r in gpu_log)
            out[name] = {"value": len(gpu_log) / full, "unit": "updates/s",
                         "circuit_s": full, "label": "extrapolated",
                         "model": f"t = {a:.3e} s + {b:.3e} s * m n min(m, n), fitted on "
                                  f"{len(bins)} (d, chi_l, chi_r) bins of the sample, "
                                  f"m = d chi_l, n = d chi_r, applied to every update of the "
                                  f"GPU run (sweep counts growing with n not modelled)"}
    return out


def bench_batched(args, torch, C, P):
    """Independent circuits of the batched workload (N ~ U{20..80}, depth ~
    U{10..40}, capped at --max-depth, F_min = 0.99, chi <= 1024), advanced
    together (leading small-bond layers in one device-resident launch,
    captured once in a HIP graph and replayed by each step, then one batched
    call per layer) and, for comparison, one after the other."""
    import numpy as np
    progs = C.batched_programs(64)[: args.circuits]
    for p in progs:
        p.layers = p.layers[: args.max_depth]
    n_upd = sum(p.n_2q for p in progs)

    states = [P.EAState(p.n_sites, "pure", args.prec, chi_max=1024) for p in progs]
    if args.topk:
        for st in states:
            st.set_option(P.EA_OPT_TOPK, 1)
            st.set_option(P.EA_OPT_TOPK_POWER, args.topk_power)
    depth = max(len(p.layers) for p in progs)

    graph = P.capture_batched(states, progs)

    t_start = [0.0]

    def progress(t):
        log(f"  layer {t} done at {time.perf_counter() - t_start[0]:.1f}s")

    def run_batched():
        # leading small-bond layers of all circuits: a replay of the captured
        # device-resident launch; then one batched call per remaining layer
        for st in states:
            st.reset()
        t_start[0] = time.perf_counter()
        P.run_batched(states, progs, 0.99, captured=graph, progress=progress)

    def run_sequential():
        for st, p in zip(states, progs):
            st.reset()
            st.run(p, 0.99)

    if not args.single_pass:
        run_batched()  # loads code objects, sizes buffers
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    run_batched()
    torch.cuda.synchronize()
    tb = time.perf_counter() - t0
    log(f"batched {tb:.2f}s")
    ts = None
    if not args.no_sequential:
        t0 = time.perf_counter()
        run_sequential()
        torch.cuda.synchronize()
        ts = time.perf_counter() - t0
        log(f"sequential {ts:.2f}s")
    Fs = [s.fidelity_estimate()[0] for s in states]
    out = {
        "metric": "2-site gate updates/s, independent circuits advanced together, 1 GPU",
        "value": n_upd / tb, "unit": "updates/s", "n_gpus": 1, "steps": 1, "warmup": 1,
        "ms_per_step": 1000 * tb, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64" if args.prec == "c128" else "f32",
        "data": "synthetic",
        "config": {"workload": f"batched-{len(progs)}-circuits-N20to80-depth<= {args.max_depth}",
                   "circuits": len(progs), "updates": n_upd, "f_min": 0.99, "chi_max": 1024,
                   **({"topk": True} if args.topk else {})},
        "sequential_updates_per_s": None if ts is None else n_upd / ts,
        "speedup_batched_vs_sequential": None if ts is None else ts / tb,
        "circuits_with_P_ge_0.99": int(sum(F >= 0.99 for F in Fs)),
        "final_fidelity_estimates": [round(F, 6) for F in Fs],
        "capped_updates": int(sum(sum(r["capped"] for r in s.gate_log()) for s in states)),
        "partial_factorisations": int(sum(sum(r["subspace"] > 0 for r in s.gate_log())
                                          for s in states)),
        "first_pass_includes_code_loading": bool(args.single_pass),
    }
    graph.close()
    for s in states:
        s.close()
    print(json.dumps(out), flush=True)


def bench_mpo40(args, torch, C, P):
    """Noisy MPO workload: 40 qubits, depth 30, Haar U(4) gates each followed
    by two-qubit depolarising noise p = 1e-3 (one fused 16x16 superoperator),
    F_min = 0.95, chi <= 1024, d = 4 per site."""
    prog, cfg = C.config_program(3, depth=args.depth if args.depth != 20 else 30)
    stream = torch.cuda.current_stream()
    st = P.EAState(prog.n_sites, "mixed", args.prec, chi_max=cfg["chi_max"], stream=stream)
    if args.topk:
        st.set_option(P.EA_OPT_TOPK, 1)
        st.set_option(P.EA_OPT_TOPK_POWER, args.topk_power)
    tiny = C.config_program(3, depth=2)[0]
    run_circuit(st, tiny, 1.0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    run_circuit(st, prog, cfg["f_min"], progress=True)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    F, _ = st.fidelity_estimate()
    glog = st.gate_log()
    out = {
        "metric": "2-site gate updates/s & circuit time, noisy MPO (d = 4), 1 GPU",
        "value": prog.n_2q / dt, "unit": "updates/s", "n_gpus": 1, "steps": 1, "warmup": 0,
        "ms_per_step": 1000 * dt, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64" if args.prec == "c128" else "f32",
        "data": "synthetic",
        "config": {"workload": f"mpo-brickwork-haar-40q-depth{len(prog.layers)}-p1e-3-Fmin0.95-chi1024",
                   "updates_per_step": prog.n_2q, "prec": args.prec},
        "final_fidelity_estimate": F,
        "capped_updates": int(sum(r["capped"] for r in glog)),
        "max_bond": int(max(st.bond_dims())),
        "partial_factorisations": int(sum(r["subspace"] > 0 for r in glog)),
    }
    if args.topk:
        out["config"]["topk"] = True
    # the running estimate after each layer, and where the bond cap first bites
    per_layer, pos, first_cap = [], 0, None
    for li, layer in enumerate(prog.layers):
        recs = glog[pos:pos + len(layer)]
        pos += len(layer)
        if recs:
            per_layer.append(round(math.exp(recs[-1]["lnP"]), 6))
            if first_cap is None and any(r["capped"] for r in recs):
                first_cap = li + 1
    out["estimate_after_layer"] = per_layer
    out["first_layer_with_capped_update"] = first_cap
    out["layers_with_estimate_ge_f_min"] = sum(1 for v in per_layer if v >= cfg["f_min"])
    st.close()
    print(json.dumps(out), flush=True)


def bench_hea32(args, torch, C, P):
    """Energy and all 640 angle derivatives of the 32-qubit, 10-layer
    hardware-efficient ansatz (F_min = 0.999) through the adjoint; the CPU
    oracle's adjoint on the same problem is timed beside it."""
    import numpy as np
    n, L = 32, 10
    angles = C.hea_angles(n, L, seed=5)
    terms = C.hea_hamiltonian(n)
    dops = P.make_dops(P.hea_dops(n, L))
    st = P.EAState(n, "pure", args.prec)
    P.mps_energy_grad(st.h, dops, angles, terms, f_min=0.999)  # loads code objects
    torch.cuda.synchronize()
    reps = max(1, args.steps)
    t0 = time.perf_counter()
    for _ in range(reps):
        E, g, lnP = P.mps_energy_grad(st.h, dops, angles, terms, f_min=0.999)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / reps
    n_upd = len(st.gate_log())
    st.close()
    out = {
        "metric": "energy + 640-angle gradient evaluations/s (adjoint through truncation), 1 GPU",
        "value": 1.0 / dt, "unit": "gradients/s", "n_gpus": 1, "steps": reps, "warmup": 1,
        "ms_per_step": 1000 * dt, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64" if args.prec == "c128" else "f32",
        "data": "synthetic",
        "config": {"workload": "hea-32q-10layers-RyRz-CZ-640angles-Fmin0.999",
                   "two_site_updates_forward": n_upd, "prec": args.prec},
        "energy": E, "lnP": lnP, "grad_norm": float(np.linalg.norm(g)),
    }
    if not args.no_cpu:
        from oracle.adjoint import hea_energy_and_grad
        t1 = time.perf_counter()
        hea_energy_and_grad(angles, terms, f_min=0.999)
        tc = time.perf_counter() - t1
        out["cpu_baseline"] = {"value": 1.0 / tc, "unit": "gradients/s",
                               "cores": len(os.sched_getaffinity(0)), "kind": "oracle",
                               "sample": f"one full energy + gradient evaluation, {tc:.1f} s"}
    print(json.dumps(out), flush=True)


def _exact_statevector_torch(torch, prog):
    """Reference |psi> of a noiseless program by plain dense state-vector
    simulation (torch complex128 on the GPU), for the true fidelity of the
    strategy study: not part of the simulator under test."""
    n = prog.n_sites
    psi = torch.zeros(2 ** n, dtype=torch.complex128, device="cuda")
    psi[0] = 1.0
    for op in prog.ops():
        g = torch.as_tensor(op.mat, dtype=torch.complex128, device="cuda")
        w = 2 ** op.width
        left = 2 ** op.site
        v = psi.view(left, w, -1)
        psi = torch.einsum("ab,lbr->lar", g, v).reshape(-1)
    return psi


def bench_fig1(args, torch, C, P):
    """Strategy study (Sec. VI, Fig. 1 analogue): 25 qubits, brickwork Haar
    depth 20, complex FP64; per F_min in {0.9, 0.99} and per strategy (naive,
    nearest, global) the final estimate P against the true fidelity
    |<psi_exact|psi>|^2 from a dense state vector, with the peak bond and the
    wall time."""
    import numpy as np
    n, depth = 25, 20
    prog = C.brickwork_program(n, depth, 2307)
    t0 = time.perf_counter()
    ref = _exact_statevector_torch(torch, prog)
    torch.cuda.synchronize()
    t_ref = time.perf_counter() - t0
    ref = ref.cpu().numpy()
    rows = []
    names = {P.EA_NAIVE: "naive", P.EA_NEAREST: "nearest", P.EA_GLOBAL: "global"}
    for f_min in (0.9, 0.99):
        for strat in (P.EA_NAIVE, P.EA_NEAREST, P.EA_GLOBAL):
            with P.EAState(n, "pure", "c128") as st:
                torch.cuda.synchronize()
                t1 = time.perf_counter()
                st.run(prog, f_min, strategy=strat)
                torch.cuda.synchronize()
                dt = time.perf_counter() - t1
                F, _ = st.fidelity_estimate()
                psi = st.statevector()
                bonds = [max(r["chi_l"], r["k"]) for r in st.gate_log()]
            psi = psi / np.linalg.norm(psi)
            true = float(abs(np.vdot(ref, psi)) ** 2)
            rows.append({"f_min": f_min, "strategy": names[strat], "estimate": F,
                         "true_fidelity": true, "peak_bond": int(max(bonds)),
                         "seconds": dt, "updates": prog.n_2q})
            log(f"fig1 F_min={f_min} {names[strat]}: P={F:.5f} true={true:.5f} "
                f"peak bond {max(bonds)} {dt:.2f}s")
    print(json.dumps({"study": "fig1-strategies-25q-depth20", "reference_seconds": t_ref,
                      "rows": rows}), flush=True)


def bench_fig2a(args, torch, C, P):
    """Mirror circuit (Sec. VI, Fig. 2a analogue): 40 qubits, a brickwork Haar
    circuit of depth 10 followed by its inverse, complex FP64, F_min in
    {1 - 1e-6, 0.99}: the largest bond after every layer (entanglement grows,
    then falls back), the final estimate and <Z_i> at the end (all 1 for the
    exact identity)."""
    import numpy as np
    n, depth = 40, 10
    prog = C.mirror_program(n, depth, 40)
    rows = []
    for f_min in (1 - 1e-6, 0.99):
        with P.EAState(n, "pure", "c128") as st:
            st.set_schedule(f_min, prog.n_2q)
            peaks = []
            t1 = time.perf_counter()
            for layer in prog.layers:
                st.run_layer(layer)
                peaks.append(int(max(st.bond_dims())))
            dt = time.perf_counter() - t1
            F, _ = st.fidelity_estimate()
            z = np.real(st.expect(list(range(n)), [1] * n, [np.diag([1.0, -1.0])] * n))
        rows.append({"f_min": f_min, "max_bond_per_layer": peaks, "estimate": F,
                     "min_Z": float(z.min()), "final_max_bond": peaks[-1], "seconds": dt})
        log(f"fig2a F_min={f_min}: peaks {peaks} P={F:.6f} min<Z>={z.min():.6f}")
    print(json.dumps({"study": "fig2a-mirror-40q-depth10x2", "rows": rows}), flush=True)


def bench_fig4(args, torch, C, P):
    """Entanglement-aware against fixed-bond-dimension simulation (Sec. VI,
    Fig. 4 analogue, scaled down): the EA run with F_min (bond cap 1024), then
    the standard run (every target 1, only the cap truncates) with chi_max =
    the largest bond of the EA run.  Noiseless: 32 qubits, depth 16, F_min
    0.99.  Noisy MPO: 16 qubits, depth 12, two-qubit depolarising p = 1e-3,
    F_min 0.95.  Complex FP32 (--prec).  Wall time, final estimate, peak
    bond, capped updates and the sum over updates of chi_l chi_r."""
    rows = []
    for kind, n, depth, f_min, noise in (("pure", 32, 16, 0.99, 0.0),
                                         ("mixed", 16, 12, 0.95, 1e-3)):
        prog = C.brickwork_program(n, depth, 75, kind=kind, noise_p=noise)
        res = {}
        chi_ea = None
        for mode in ("ea", "fixed"):
            chi_max = 1024 if mode == "ea" else chi_ea
            with P.EAState(n, kind, args.prec, chi_max=chi_max) as st:
                run_circuit(st, C.brickwork_program(n, 2, 1, kind=kind, noise_p=noise), 1.0)
                st.reset()
                torch.cuda.synchronize()
                t1 = time.perf_counter()
                st.run(prog, f_min, strategy=P.EA_GLOBAL if mode == "ea" else P.EA_FIXED)
                torch.cuda.synchronize()
                dt = time.perf_counter() - t1
                F, _ = st.fidelity_estimate()
                glog = st.gate_log()
            peak = max(r["k"] for r in glog)
            if mode == "ea":
                chi_ea = peak
            res[mode] = {"seconds": dt, "estimate": F, "peak_bond": int(peak),
                         "chi_work": float(sum(r["chi_l"] * r["chi_r"] for r in glog)),
                         "capped_updates": int(sum(r["capped"] for r in glog))}
            log(f"fig4 {kind} {mode}: {dt:.2f}s P={F:.5f} peak {peak}")
        rows.append({"kind": kind, "n_qubits": n, "depth": depth, "f_min": f_min,
                     "noise_p": noise, "chi_max_fixed": chi_ea, **res,
                     "speedup_ea_vs_fixed": res["fixed"]["seconds"] / res["ea"]["seconds"]})
    print(json.dumps({"study": "fig4-ea-vs-fixed-chi", "prec": args.prec, "rows": rows}),
          flush=True)


def bench_vidal50(args, torch, C, P):
    """The 50-qubit depth-20 circuit (F_min 0.99, chi <= 1024) in the
    layer-parallel gauge (Vidal form, Hastings update; a layer's gates side by
    side on their own streams), against the single-centre run of the same
    build: wall time and final estimate of each."""
    prog, cfg = C.config_program(2, depth=args.depth)
    out_modes = {}
    for mode in ("layer_parallel", "single_centre"):
        st = P.EAState(prog.n_sites, "pure", args.prec, chi_max=cfg["chi_max"])
        if mode == "layer_parallel":
            st.set_option(P.EA_OPT_GAUGE, 1)
        run_circuit(st, C.brickwork_program(prog.n_sites, 2, 99), 1.0)
        st.reset()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        run_circuit(st, prog, cfg["f_min"], progress=True)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        F, _ = st.fidelity_estimate()
        glog = st.gate_log()
        out_modes[mode] = {"seconds": dt, "updates_per_s": prog.n_2q / dt, "estimate": F,
                           "capped_updates": int(sum(r["capped"] for r in glog)),
                           "max_bond": int(max(st.bond_dims()))}
        log(f"{mode}: {dt:.2f}s P={F:.5f}")
        st.close()
    lp = out_modes["layer_parallel"]
    print(json.dumps({
        "metric": "2-site gate updates/s, layer-parallel gauge, 1 GPU", "value": lp["updates_per_s"],
        "unit": "updates/s", "n_gpus": 1, "steps": 1, "warmup": 0, "ms_per_step": 1000 * lp["seconds"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if args.prec == "c128" else "f32", "data": "synthetic",
        "config": {"workload": f"brickwork-haar-50q-depth{args.depth}-Fmin0.99-chi1024-layer-parallel",
                   "prec": args.prec},
        "modes": out_modes,
        "speedup_vs_single_centre": out_modes["single_centre"]["seconds"] / lp["seconds"]}),
        flush=True)


def bench_contraction(args, torch, C, P):
    """The two-site contraction with the gate (one launch per update) alone, at
    chi = 256, 512 and 1024 (Theta up to 2048 x 2048, K = chi), in every
    precision: device time per launch from HIP events and the fraction of the
    matrix-core peak of its arithmetic type.  The SVD after it is cut to one
    sweep (its time is not counted)."""
    import numpy as np
    peak = {"c64": PEAKS["f32_mfma_TF"], "c128": PEAKS["f64_mfma_TF"],
            "bf16x3": PEAKS["f32_mfma_TF"]}
    rows = []
    G = C.haar_unitary(np.random.default_rng(1))
    for prec in ("c64", "c128", "bf16x3"):
        for chi in (256, 512, 1024):
            tens = C.random_mps_tensors([1, chi, chi, chi, 1], 2, seed=chi)
            st = P.EAState(4, "pure", prec)
            st.set_option(P.EA_OPT_MAX_SWEEPS, 1)
            st.load(tens, 1)
            st.apply_2q(1, G, 0.99)  # loads the code objects
            st.profile(True)
            for _ in range(max(1, args.steps)):
                st.load(tens, 1)
                st.apply_2q(1, G, 0.99)
            f = st.profile_read(P.EA_K_THETA)
            st.close()
            tf = f["flops"] / f["ms"] / 1e9
            rows.append({"prec": prec, "chi": chi, "us_per_launch": 1000 * f["ms"] / f["launches"],
                         "algorithmic_TFLOPs": tf, "frac_of_mfma_peak": tf / peak[prec]})
            log(f"{prec} chi={chi}: {tf:.1f} TFLOP/s")
    big = [r for r in rows if r["chi"] == 1024 and r["prec"] == args.prec][0]
    out = {
        "metric": "two-site contraction + gate, TFLOP/s at chi = 1024 (Theta 2048 x 2048)",
        "value": big["algorithmic_TFLOPs"], "unit": "TFLOP/s", "n_gpus": 1,
        "steps": max(1, args.steps), "warmup": 1, "ms_per_step": big["us_per_launch"] / 1000,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if args.prec == "c128" else "f32", "data": "synthetic",
        "config": {"workload": "theta-contraction-chi256-512-1024", "prec": args.prec},
        "roofline": {"bound": "mfma", "achieved": big["algorithmic_TFLOPs"], "peak": peak[args.prec],
                     "unit": "TFLOP/s", "frac": big["frac_of_mfma_peak"], "traffic": None},
        "sizes": rows,
    }
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1)
    ap.add_argument("--warmup", type=int, default=0)
    ap.add_argument("--prec", default="c64", choices=["c64", "c128", "bf16x3"])
    ap.add_argument("--depth", type=int, default=20)
    ap.add_argument("--no-fp64", action="store_true",
                    help="skip the untimed-by-contract FP64 comparison circuit")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--topk", action="store_true",
                    help="partial (top-k) factorisation of eligible updates (EA_OPT_TOPK)")
    ap.add_argument("--topk-power", type=int, default=1,
                    help="subspace iterations of the partial factorisation (EA_OPT_TOPK_POWER)")
    ap.add_argument("--no-variants", "--no-topk-variant", dest="no_variants", action="store_true",
                    help="skip the untimed runs of the circuit with the partial factorisation "
                         "and in the layer-parallel gauge")
    ap.add_argument("--cpu-layers", type=int, default=10)
    ap.add_argument("--cpu-budget", type=float, default=30.0)
    ap.add_argument("--workload", default="brickwork50",
                    choices=["brickwork50", "batched", "mpo40", "hea32", "contraction",
                             "fig1", "fig2a", "fig4", "vidal50"],
                    help="brickwork50: the 50-qubit depth-20 circuit (default); batched: "
                         "independent circuits of the batched workload advanced together; "
                         "mpo40: the noisy 40-qubit MPO circuit; hea32: adjoint gradients; "
                         "contraction: the two-site contraction alone at chi <= 1024; "
                         "fig1 / fig2a / fig4: the paper's strategy, mirror-circuit and "
                         "EA-against-fixed-bond studies at reduced sizes")
    ap.add_argument("--circuits", type=int, default=16, help="batched: number of circuits")
    ap.add_argument("--max-depth", type=int, default=12, help="batched: depth cap per circuit")
    ap.add_argument("--no-sequential", action="store_true",
                    help="batched: skip the one-circuit-after-another comparison")
    ap.add_argument("--single-pass", action="store_true",
                    help="batched: time the first pass (no untimed warm-up pass)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a device copy of known size (counter calibration)")
    ap.add_argument("--summarize-pmc", metavar="DIR",
                    help="only write DIR/traffic.json from counter CSVs under DIR")
    args = ap.parse_args()
    if args.summarize_pmc:
        return summarize_pmc(args.summarize_pmc)
    if args.calibrate_copy:
        return calibrate_copy()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import torch
    import circuits as C
    import paper_2307_16870_amd as P

    assert torch.cuda.is_available(), "no GPU visible"
    torch.cuda.init()
    if args.workload == "batched":
        return bench_batched(args, torch, C, P)
    if args.workload == "mpo40":
        return bench_mpo40(args, torch, C, P)
    if args.workload == "hea32":
        return bench_hea32(args, torch, C, P)
    if args.workload == "contraction":
        return bench_contraction(args, torch, C, P)
    if args.workload == "vidal50":
        return bench_vidal50(args, torch, C, P)
    if args.workload in ("fig1", "fig2a", "fig4"):
        return {"fig1": bench_fig1, "fig2a": bench_fig2a, "fig4": bench_fig4}[args.workload](
            args, torch, C, P)
    stream = torch.cuda.current_stream()
    prog, cfg = C.config_program(2, depth=args.depth)
    f_min, chi_max = cfg["f_min"], cfg["chi_max"]

    st = P.EAState(prog.n_sites, "pure", args.prec, chi_max=chi_max, stream=stream)
    if args.topk:
        st.set_option(P.EA_OPT_TOPK, 1)
        st.set_option(P.EA_OPT_TOPK_POWER, args.topk_power)
    # load the kernels' code objects before anything is timed (not a step)
    tiny = C.brickwork_program(prog.n_sites, 2, 99)
    run_circuit(st, tiny, 1.0)
    for w in range(args.warmup):
        log(f"warmup step {w}")
        run_circuit(st, prog, f_min, progress=True)

    st.profile(PROF_EVERY)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        log(f"timed step {k}")
        run_circuit(st, prog, f_min, progress=True)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    fams = {name: st.profile_read(i) for i, name in enumerate(P._binding.K_FAMILY_NAMES)}
    st.profile(False)

    F, lnF = st.fidelity_estimate()
    glog = st.gate_log()
    glog_full = glog[-prog.n_2q:]  # the last timed step's updates
    n_upd = prog.n_2q * args.steps
    ms_step = 1000.0 * elapsed / args.steps
    log(f"elapsed {elapsed:.2f}s  P={F:.5f}")

    # dominant kernel family and its roofline
    f64 = args.prec == "c128"
    mfma_peak = PEAKS["f64_mfma_TF"] if f64 else PEAKS["f32_mfma_TF"]
    alu_peak = PEAKS["f64_vector_TF"] if f64 else PEAKS["f32_vector_TF"]
    bound_of = {"jacobi_gram": "mfma", "jacobi_apply": "mfma", "theta": "mfma"}
    kernel_of = {"jacobi_rot": "k_jeig", "jacobi_gram": "k_jgram", "jacobi_apply": "k_japply",
                 "theta": "k_theta_mfma", "jacobi_fused": "k_jacobi_block"}

    def roof(name):
        fd = fams[name]
        ms = max(fd["ms"], 1e-12)  # average timed launch x all launches
        bound = bound_of.get(name, "alu")
        achieved = fd["flops"] / (ms * 1e-3) / 1e12
        peak = mfma_peak if bound == "mfma" else alu_peak
        return {
            "kernel": kernel_of.get(name, name), "family": name, "bound": bound,
            "achieved": achieved, "peak": peak, "unit": "TFLOP/s", "frac": achieved / peak,
            "traffic": traffic_for(kernel_of.get(name, name)),
            "avg_launch_ms": fd["avg_ms"], "launches": fd["launches"],
            "timed_launches": fd["timed"],
            "algorithmic_flops_per_launch": fd["flops"] / max(1, fd["launches"]),
            "algorithmic_bytes_per_launch": fd["bytes"] / max(1, fd["launches"]),
            "achieved_GBs_algorithmic": fd["bytes"] / (ms * 1e-3) / 1e9,
        }

    dom = max((k for k in fams if k != "centre_move"), key=lambda k: fams[k]["ms"])
    roofline = roof(dom)

    out = {
        "metric": "2-site gate updates/s & circuit time at F>=0.99, mixed-prec vs FP64, 1 GPU",
        "value": n_upd / elapsed,
        "unit": "updates/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if f64 else "f32",
        "data": "synthetic",
        "config": {"workload": f"brickwork-haar-50q-depth{args.depth}-Fmin0.99-chi1024",
                   "n_qubits": prog.n_sites, "depth": args.depth, "updates_per_step": prog.n_2q,
                   "f_min": f_min, "chi_max": chi_max, "schedule": "global", "prec": args.prec,
                   **({"topk": True} if args.topk else {})},
        "circuit_time_s": ms_step / 1000.0,
        "final_fidelity_estimate": F,
        "capped_updates": int(sum(r["capped"] for r in glog_full)),
        "meets_f_min": bool(F >= f_min),
        "f_min_note": ("the bond cap of 1024 binds before the end of this circuit: capped "
                       "updates keep less weight than their target, so the estimate ends "
                       "below F_min" if F < f_min else "estimate at or above F_min"),
        "max_bond": int(max(st.bond_dims())),
        "partial_factorisations": int(sum(r["subspace"] > 0 for r in glog_full)),
        "partial_attempts_not_accepted": int(sum(r["attempts"] > (1 if r["subspace"] else 0)
                                                 for r in glog_full)),
        "jacobi_sweeps": {
            "mean": sum(r["sweeps"] for r in glog_full) / max(1, len(glog_full)),
            "mean_at_width_ge_1024": (lambda L: sum(L) / max(1, len(L)))(
                [r["sweeps"] for r in glog_full if 2 * min(r["chi_l"], r["chi_r"]) >= 1024]),
            "max": max((r["sweeps"] for r in glog_full), default=0)},
        "kernels_ms": {k: round(v["ms"], 3) for k, v in fams.items()},
        "roofline": roofline,
        "rooflines_other": {k: roof(k) for k in ["jacobi_apply", "jacobi_gram", "theta"]
                            if fams[k]["launches"] > 0 and k != dom},
    }
    # the Jacobi SVD of the two-site updates as a whole: (18 m n^2 + 14 n^3)
    # flops per sweep (the per-sweep count of a one-sided Jacobi in its
    # real-arithmetic form; complex arithmetic executes about four times as
    # many), m x n the factored matrix, over every update's sweeps, against
    # the time of all Jacobi kernel families
    jac_fl = 0.0
    for r in glog_full:
        mw, nw = 2 * max(r["chi_l"], r["chi_r"]), 2 * min(r["chi_l"], r["chi_r"])
        jac_fl += r["sweeps"] * (18.0 * mw * nw * nw + 14.0 * nw ** 3)
    jac_fl *= args.steps
    jac_ms = sum(fams[k]["ms"] for k in ("jacobi_gram", "jacobi_rot", "jacobi_apply",
                                         "jacobi_small", "jacobi_fused"))
    if jac_ms > 0:
        ach = jac_fl / (jac_ms * 1e-3) / 1e12
        out["rooflines_other"]["jacobi_svd_all"] = {
            "kernels": "k_jgram + k_jeig + k_japply + k_jacobi_block", "bound": "mfma",
            "achieved": ach, "peak": mfma_peak, "unit": "TFLOP/s", "frac": ach / mfma_peak,
            "count": "sum over updates of sweeps x (18 m n^2 + 14 n^3)",
            "device_ms": jac_ms}
    if not args.no_fp64 and args.prec != "c128":
        log("fp64 comparison step")
        st64 = P.EAState(prog.n_sites, "pure", "c128", chi_max=chi_max, stream=stream)
        run_circuit(st64, tiny, 1.0)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        run_circuit(st64, prog, f_min, progress=True)
        torch.cuda.synchronize()
        t64 = time.perf_counter() - t1
        F64, _ = st64.fidelity_estimate()
        out["fp64"] = {"ms_per_step": 1000 * t64, "updates_per_s": prog.n_2q / t64,
                       "final_fidelity_estimate": F64,
                       "speedup_mixed_vs_fp64": t64 / (ms_step / 1000.0)}
        st64.close()
    if not args.topk and not args.no_variants:
        # the same circuit with the partial (top-k) factorisation: a variant
        # beside the contract's number, not part of it
        log("partial-factorisation variant")
        stk = P.EAState(prog.n_sites, "pure", args.prec, chi_max=chi_max, stream=stream)
        stk.set_option(P.EA_OPT_TOPK, 1)
        stk.set_option(P.EA_OPT_TOPK_POWER, args.topk_power)
        run_circuit(stk, tiny, 1.0)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        run_circuit(stk, prog, f_min, progress=True)
        torch.cuda.synchronize()
        tk = time.perf_counter() - t1
        Fk, _ = stk.fidelity_estimate()
        gk = stk.gate_log()[-prog.n_2q:]
        out["topk_variant"] = {
            "option": f"EA_OPT_TOPK (oversampling 64, {args.topk_power} subspace iteration(s))",
            "ms_per_step": 1000 * tk, "updates_per_s": prog.n_2q / tk,
            "final_fidelity_estimate": Fk,
            "capped_updates": int(sum(r["capped"] for r in gk)),
            "partial_factorisations": int(sum(r["subspace"] > 0 for r in gk)),
            "partial_attempts_not_accepted": int(sum(r["attempts"] > (1 if r["subspace"] else 0)
                                                     for r in gk)),
            "speedup_vs_full_svd": tk and (ms_step / 1000.0) / tk}
        stk.close()
    if not args.no_variants:
        # the same circuit in the layer-parallel gauge (Vidal form, Hastings
        # update): another variant beside the contract's number
        log("layer-parallel variant")
        stg = P.EAState(prog.n_sites, "pure", args.prec, chi_max=chi_max, stream=stream)
        stg.set_option(P.EA_OPT_GAUGE, 1)
        run_circuit(stg, tiny, 1.0)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        run_circuit(stg, prog, f_min, progress=True)
        torch.cuda.synchronize()
        tg = time.perf_counter() - t1
        Fg, _ = stg.fidelity_estimate()
        out["layer_parallel_variant"] = {
            "option": "EA_OPT_GAUGE (Vidal form, a layer's gates side by side; the estimate "
                      "is approximate after truncations)",
            "ms_per_step": 1000 * tg, "updates_per_s": prog.n_2q / tg,
            "final_fidelity_estimate": Fg, "speedup_vs_full_svd": (ms_step / 1000.0) / tg}
        stg.close()
    st.close()
    if not args.no_cpu:
        # the GPU on the oracle's sample: the first cpu_layers layers
        st2 = P.EAState(prog.n_sites, "pure", args.prec, chi_max=chi_max, stream=stream)
        run_circuit(st2, tiny, 1.0)
        st2.reset()
        st2.set_schedule(f_min, prog.n_2q)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for layer in prog.layers[:args.cpu_layers]:
            st2.run_layer(layer)
        torch.cuda.synchronize()
        tpre = time.perf_counter() - t1
        st2.close()
        log("cpu baseline")
        out["cpu_baseline"] = cpu_baseline(prog, f_min, chi_max, args.cpu_layers, args.cpu_budget,
                                           gpu_log=glog_full, gpu_prefix_s=tpre)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
