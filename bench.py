"""Benchmark of the full hot path on one MI355X.

One step = cd_decompose (pairs, diagonal, screening, pivot selection,
all-row solve) + cd_build_jk (J and K, with the AO->MO transform of every
vector by the occupied coefficients on both sides fused into it, or as a
separate cd_transform call where the precision does not fuse it).  The default
workload is the 1200-function one (300 centres in a 24 angstrom box,
exponents 0.1 .. 10 bohr^-2, 150 occupied orbitals, Schwarz screening 1e-12)
at tau = 1e-6, the largest single-GPU configuration.  Inputs are resident in
device memory before the timed region.

Prints one JSON line.  value = Cholesky vectors per second of the whole FP64
step (M / step time).  The same line carries the step and the J/K build with
FP32 and with 3 x BF16 exchange products against FP64 (times and errors), the
64-molecule batched workload against the same molecules one by one at equal
precision, per-phase device times from HIP events recorded on the library's
stream, the roofline of the dominant kernel and the CPU oracle's rate.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK = {"fp64": 78.6, "fp32": 157.3, "bf16": 2500.0}   # dense TFLOP/s, MI355X
HBM_TBPS = 8.0
METRIC = "Cholesky vectors/s + J/K build TFLOP/s at tau=1e-6; mixed/batched vs plain FP64"
PRECISIONS = ("fp64", "fp32", "bf16x3")
#: precisions whose J/K build also writes C^T L C (the transform fused into it)
FUSED = ("fp64", "fp32", "bf16x3")

# HBM bytes per launch of a kernel on a workload, from two rocprofv3 --pmc runs
# of the bench (FETCH_SIZE, then WRITE_SIZE, KiB per dispatch; commands in
# profiles/hbm_bytes_1200fn_tau1e-6.md), each scaled by what the same counter
# reads for a plain 1 GiB device copy (`bench.py --copy-probe 1024`): FETCH_SIZE
# reads 524 302 KiB there (factor 2.0), WRITE_SIZE 1 048 576 KiB (factor 1.0).
# The figures belong to the kernel sources they were taken on; once those
# change the traffic is reported as null until the counters are taken again.
DECOMP_SOURCES = ["paper_2609_00306_amd/csrc/cd_decompose.hip",
                  "paper_2609_00306_amd/csrc/cd_mfma.hpp",
                  "paper_2609_00306_amd/csrc/cd_device.hpp",
                  "paper_2609_00306_amd/csrc/cd_kernels.hpp"]
LP_SOURCES = ["paper_2609_00306_amd/csrc/cd_jk_lp.hip",
                "paper_2609_00306_amd/csrc/cd_device.hpp",
                "paper_2609_00306_amd/csrc/cd_mfma.hpp"]
FETCH_SCALE, WRITE_SCALE = 1048576.0 / 524302.25, 1048576.0 / 1048576.0
_DECOMP_SHA = "1446673a140d255bd8993e8e60526ad7b5f4bbc861702a2271d9d17a60e869d6"
_LP_SHA = "1f0a970e247f971c4ba77365c789fa8d62b7bb1ff504d2293d3acd5e2d2fa1fb"
COUNTERS = {
    ("C5", 1e-6): {
        "k_step2": {"sources": DECOMP_SOURCES, "sha256": _DECOMP_SHA,
                    "fetch_kib": 36124221.8, "write_kib": 2679898.1},
        "k_step1": {"sources": DECOMP_SOURCES, "sha256": _DECOMP_SHA,
                    "fetch_kib": 3718871.4, "write_kib": 355229.4},
        "k_syrk_bf16x3": {"sources": LP_SOURCES, "sha256": _LP_SHA,
                          "fetch_kib": 13626673.3, "write_kib": 198720.0},
        "k_syrk_f32": {"sources": LP_SOURCES, "sha256": _LP_SHA,
                       "fetch_kib": 9473423.2, "write_kib": 94752.0},
    },
}


def sources_sha256(files):
    import hashlib
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def counter_traffic(kernel, config, tau):
    """HBM bytes per launch of 'kernel' from the recorded counters, or None."""
    c = COUNTERS.get((config, tau), {}).get(kernel)
    if c is None or sources_sha256(c["sources"]) != c["sha256"]:
        return None
    return 1024.0 * (c["fetch_kib"] * FETCH_SCALE + c["write_kib"] * WRITE_SCALE)


def cpu_baseline(m, tau, schwarz, M_full, prefix):
    """The CPU oracle timed on the host cores: the first 'prefix' vectors of the
    same decomposition (the oracle's cost per vector grows with the vector
    index, about n K operations for vector K, so the full run is estimated
    from the prefix by that model)."""
    import oracle
    rp, _ = oracle.rows(m.xyz, m.alpha, schwarz)
    P = int(min(prefix, M_full))
    t0 = time.perf_counter()
    ref = oracle.decompose(m.xyz, m.alpha, rp, tau, max_vectors=P)
    t1 = time.perf_counter()
    cores = int(os.environ.get("OMP_NUM_THREADS") or os.cpu_count() or 1)
    est_full = (t1 - t0) * (M_full / max(1, ref.M)) ** 2
    return {"value": ref.M / (t1 - t0), "unit": "vectors/s", "cores": cores, "kind": "oracle",
            "sample": f"the oracle's decomposition of the same workload stopped after its first "
                      f"{ref.M} of {M_full} vectors (capacity), {t1 - t0:.2f} s; its cost per "
                      f"vector grows linearly with the vector index, so the full run would take "
                      f"about {est_full:.0f} s",
            "seconds": t1 - t0, "vectors": int(ref.M),
            "full_run_vectors_per_s_estimate": M_full / est_full}


def copy_probe(mib):
    """A plain device-to-device copy of a known size, three times: the reference
    against which the HBM byte counters of a profiled run are scaled."""
    import torch
    n = mib * (1 << 20) // 8
    src = torch.ones(n, dtype=torch.float64, device="cuda:0")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes_read": n * 8, "copy_probe_bytes_written": n * 8,
                      "launches": 3}), flush=True)


def _timed(fn, steps, warmup):
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) * 1e3 / steps


def batched_c4(steps, warmup, tuned=True):
    """64 molecules of uneven size (52..400 functions), tau = 1e-5: one batched
    cd_decompose call plus one batched cd_build_jk call per step, against the
    same molecules one by one (one call per molecule), each at FP64 and at FP32
    K, so batching and precision are reported as separate factors."""
    import torch

    from paper_2609_00306_amd import cdlib
    from paper_2609_00306_amd.inputs import BATCH_C4, batch_c4

    dev = torch.device("cuda:0")
    mols = batch_c4()
    tau, schwarz = BATCH_C4["tau"], BATCH_C4["schwarz"]
    pairs = [(m.xyz, m.alpha) for m in mols]
    probe, pws = cdlib.allocate_many(pairs, tau, schwarz, device=dev)
    cdlib.run_decompose(probe, tau, schwarz, workspace=pws)
    torch.cuda.synchronize()
    Ms = [max(1, d.M()) for d in probe]
    assert all(int(d.status.item()) == 0 for d in probe)
    del probe, pws
    decs, ws = cdlib.allocate_many(pairs, tau, schwarz, max_vectors=Ms, device=dev)
    singles = [cdlib.allocate(m.xyz, m.alpha, tau, schwarz, M, device=dev) for m, M in zip(mols, Ms)]
    tuning = cdlib.autotune(decs, tau, schwarz, workspace=ws) if tuned else None
    out = {"workload": f"{len(mols)} molecules, N {min(m.n_basis for m in mols)}.."
                       f"{max(m.n_basis for m in mols)} s-Gaussians, tau={tau:g}, O=N/8",
           "n_molecules": len(mols), "n_vectors": sum(Ms)}
    res = {}
    jk_out = {}
    for prec in ("fp64", "fp32"):
        jks, jws = cdlib.prepare_jk_many(decs, [m.C for m in mols], prec)
        sjks = [cdlib.prepare_jk(d, m.C, prec) for d, m in zip(singles, mols)]

        def batched():
            cdlib.run_decompose(decs, tau, schwarz, workspace=ws, tuning=tuning)
            cdlib.run_jk_many(jks, jws, prec)

        def plain():
            for d, j in zip(singles, sjks):
                cdlib.run_decompose([d], tau, schwarz)
                cdlib.run_jk(j, prec)

        ms_b = _timed(batched, steps, warmup)
        ms_p = _timed(plain, steps, warmup)
        graph = {"captured": False}
        try:
            g = torch.cuda.CUDAGraph()
            side = torch.cuda.Stream()
            side.wait_stream(torch.cuda.current_stream())
            with torch.cuda.stream(side):
                batched()
            torch.cuda.current_stream().wait_stream(side)
            with torch.cuda.graph(g):
                batched()
            ms_g = _timed(g.replay, steps, warmup)
            graph = {"captured": True, "ms_per_step": ms_g}
            del g
        except Exception as e:  # noqa: BLE001
            graph = {"captured": False, "reason": str(e)[:200]}
        res[prec] = {"batched_ms": ms_b, "one_by_one_ms": ms_p, "graph": graph,
                     "batched_vectors_per_s": sum(Ms) / (ms_b * 1e-3),
                     "speedup_batched_vs_one_by_one": ms_p / ms_b}
        cdlib.run_jk_many(jks, jws, prec)
        torch.cuda.synchronize()
        jk_out[prec] = [(j.J.clone(), j.K.clone()) for j in jks]
        del jks, jws, sjks
    err = {"max_abs_dJ": 0.0, "max_abs_dK": 0.0, "max_abs_dE2": 0.0}
    for m, (J64, K64), (J32, K32) in zip(mols, jk_out["fp64"], jk_out["fp32"]):
        Ct = torch.as_tensor(m.C, device=dev)
        Dm = Ct @ Ct.T
        e2 = lambda J, K: float(2.0 * (Dm * J).sum() - (Dm * K).sum())  # noqa: E731
        err["max_abs_dJ"] = max(err["max_abs_dJ"], float((J32 - J64).abs().max()))
        err["max_abs_dK"] = max(err["max_abs_dK"], float((K32 - K64).abs().max()))
        err["max_abs_dE2"] = max(err["max_abs_dE2"], abs(e2(J32, K32) - e2(J64, K64)))
    out.update({
        "fp64": res["fp64"], "fp32_K": res["fp32"],
        "speedup_batched_vs_one_by_one_fp64": res["fp64"]["speedup_batched_vs_one_by_one"],
        "speedup_batched_vs_one_by_one_fp32": res["fp32"]["speedup_batched_vs_one_by_one"],
        "speedup_fp32_vs_fp64_batched": res["fp64"]["batched_ms"] / res["fp32"]["batched_ms"],
        "fp32_K_error_vs_fp64": err,
        "tuning": None if tuning is None else {"step2_row_tiles": tuning.step2_row_tiles,
                                               "step1_min_rows": tuning.step1_min_rows,
                                               "step1_q": tuning.step1_q},
    })
    return out


def bench_batched(args):
    """--config C4: the batched workload alone, one JSON line."""
    import torch
    torch.cuda.set_device(0)
    b = batched_c4(args.steps, args.warmup)
    ms = b["fp64"]["batched_ms"]
    out = {"metric": METRIC, "value": b["n_vectors"] / (ms * 1e-3), "unit": "vectors/s",
           "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "f64", "data": "synthetic",
           "config": {"workload": "batched: " + b["workload"], "n_molecules": b["n_molecules"],
                      "n_vectors": b["n_vectors"]},
           "batched": b}
    print(json.dumps(out), flush=True)


def run_scf(cdlib, d, m, prec, e_tol=1e-10, d_tol=1e-8):
    """One converged SCF on decomposition d; returns (result, ms)."""
    import torch
    from paper_2609_00306_amd.inputs import scf_charges
    cx, Z = scf_charges(m)
    S, H = cdlib.one_electron(m.xyz, m.alpha, cx, Z)
    e_ch = float(sum(Z[i] * Z[j] / ((((cx[i] - cx[j]) ** 2).sum()) ** 0.5)
                     for i in range(len(Z)) for j in range(i)))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    r = cdlib.scf(d, S, H, m.n_occ, e_ch, prec=prec, e_tol=e_tol, d_tol=d_tol)
    torch.cuda.synchronize()
    return r, (time.perf_counter() - t0) * 1e3


def scf_sweep(args):
    """Converged SCF energies on the workload over tau and J/K precision; the
    error is taken against the FP64 SCF at the smallest tau."""
    import torch

    from paper_2609_00306_amd import cdlib
    from paper_2609_00306_amd.inputs import CONFIGS, config_molecule
    torch.cuda.set_device(0)
    cfg = CONFIGS[args.config]
    m = config_molecule(args.config)
    taus = [1e-3, 1e-4, 1e-5, 1e-6, 1e-8]
    rows = []
    ref = None
    for tau in reversed(taus):
        d = cdlib.decompose(m.xyz, m.alpha, tau, schwarz=cfg["schwarz"])
        for prec in PRECISIONS:
            tol = (1e-10, 1e-8) if prec == "fp64" else (1e-6, 1e-6)
            r, ms = run_scf(cdlib, d, m, prec, *tol)
            E = float(r.energies[-1])
            if ref is None:
                ref = E
            rows.append({"tau": tau, "precision": prec, "M": d.M(), "iterations": len(r.energies),
                         "converged": r.converged, "energy": E, "error_vs_fp64_tau1e-8": E - ref,
                         "ms": ms})
        del d
    print(json.dumps({"scf_sweep": args.config, "n_basis": m.n_basis, "n_occ": m.n_occ,
                      "rows": rows}), flush=True)


def bench_hermitian(args):
    """The Hermitian decomposition of the seeded finite-field stand-in
    (n rows, n/2 Gaussians) at tau: time per decomposition (HIP events on the
    launch stream), vectors/s, and the bandwidth of the reads it must make
    (each vector K re-reads the K earlier vectors of every row)."""
    import torch

    from paper_2609_00306_amd import cdlib
    from paper_2609_00306_amd.inputs import hermitian_gram
    torch.cuda.set_device(0)
    n = args.hermitian
    A = torch.from_numpy(hermitian_gram(n, n // 2, seed=5)).to("cuda")
    tau = args.tau
    z = cdlib.zdecompose(A, tau)
    M = z.M()
    st = torch.cuda.current_stream()
    for _ in range(args.warmup):
        cdlib.zdecompose(A, tau, sync=False)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    torch.cuda.synchronize()
    ev[0].record(st)
    for _ in range(args.steps):
        cdlib.zdecompose(A, tau, sync=False)
    ev[1].record(st)
    torch.cuda.synchronize()
    ms = ev[0].elapsed_time(ev[1]) / args.steps
    # algorithmic bytes: earlier vectors of every row (16 n K for vector K),
    # the pivot row of A, the new vector and the residual update
    traffic = 16.0 * n * M * (M - 1) / 2.0 + M * n * (16.0 + 16.0 + 16.0)
    print(json.dumps({"hermitian": {"n": n, "n_fun": n // 2, "tau": tau, "n_vectors": M,
                                    "ms": ms, "vectors_per_s": M / (ms * 1e-3),
                                    "roofline": {"bound": "hbm",
                                                 "achieved": traffic / (ms * 1e-3) / 1e9,
                                                 "peak": HBM_TBPS * 1e3, "unit": "GB/s",
                                                 "frac": traffic / (ms * 1e-3) / 1e9 / (HBM_TBPS * 1e3)},
                                    "steps": args.steps}}), flush=True)


def jk_work(N, O, n, M, n_diag, fused):
    """Flops of one J/K build.  Executed: J (two passes over the vectors,
    4 n M), the half transform over the kept pairs (2 deg O M with deg = 2n -
    the kept diagonal pairs, the number of (mu, sigma) entries of the unpacked
    vectors), the exchange product over the lower triangle (N (N+1) O M) and,
    when fused, the second half of C^T L C (2 N O^2 M).  Dense equivalent: the
    unpacked half transform 2 N^2 O M instead of the neighbour lists."""
    deg = 2.0 * n - n_diag
    ex = 4.0 * n * M + 2.0 * deg * O * M + float(N) * (N + 1) * O * M
    if fused:
        ex += 2.0 * N * O * O * M
    dense = 4.0 * n * M + 2.0 * N * N * O * M + float(N) * (N + 1) * O * M
    return ex, dense


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--config", default="C5")
    ap.add_argument("--tau", type=float, default=1e-6)
    ap.add_argument("--precision", default="fp64", choices=list(PRECISIONS),
                    help="J/K precision of the headline step (the others are timed beside it "
                         "unless --no-compare)")
    ap.add_argument("--no-compare", action="store_true",
                    help="time only the headline precision")
    ap.add_argument("--eta", type=float, default=1.0,
                    help="span factor of the pivot selection (1 = exact pivoting)")
    ap.add_argument("--pivot-block", default=None, metavar="I,J,..",
                    help="restricted candidates (Sec. 6.2): pivots only from rows of two "
                         "functions whose exponent index is listed")
    ap.add_argument("--scf-sweep", action="store_true",
                    help="only run converged SCFs over tau and J/K precision and print the "
                         "energy errors (one JSON line)")
    ap.add_argument("--hermitian", type=int, default=0, metavar="N",
                    help="only time the Hermitian (finite-field) decomposition of the N-row "
                         "stand-in matrix (one JSON line)")
    ap.add_argument("--tuning", default="builtin", choices=["auto", "builtin"],
                    help="launch shapes of the decomposition: measured by cd_autotune before "
                         "the warm-up (auto) or the built-in choice")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-prefix", type=int, default=2400,
                    help="vectors of the oracle's decomposition timed for cpu_baseline")
    ap.add_argument("--no-batched", action="store_true",
                    help="leave out the 64-molecule batched comparison")
    ap.add_argument("--no-extras", action="store_true",
                    help="leave out the SCF and the second-order energy (profiling runs)")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="only run a plain copy of MIB MiB (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported "
              "(the multi-GPU form is design only)", file=sys.stderr)
        sys.exit(2)

    if args.copy_probe:
        copy_probe(args.copy_probe)
        return
    if args.config == "C4":
        bench_batched(args)
        return
    if args.scf_sweep:
        scf_sweep(args)
        return
    if args.hermitian:
        bench_hermitian(args)
        return

    import numpy as np
    import torch

    from paper_2609_00306_amd import cdlib
    from paper_2609_00306_amd.inputs import CONFIGS, config_molecule

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    cfg = CONFIGS[args.config]
    m = config_molecule(args.config)
    tau, schwarz = args.tau, cfg["schwarz"]
    N, O = m.n_basis, m.n_occ

    fn = None
    if args.pivot_block is not None:
        from paper_2609_00306_amd.inputs import exponent_block
        fn = exponent_block(m, [int(x) for x in args.pivot_block.split(",") if x != ""])

    # size the outputs with the measured number of vectors
    probe = cdlib.decompose(m.xyz, m.alpha, tau, schwarz=schwarz, eta=args.eta, pivot_fn=fn)
    M = probe.M()
    assert int(probe.status.item()) == 0
    del probe
    torch.cuda.empty_cache()
    d = cdlib.allocate(m.xyz, m.alpha, tau, schwarz, max(1, M), device=dev, pivot_fn=fn)
    n = d.n_rows
    precs = [args.precision] + ([] if args.no_compare else
                                [p for p in PRECISIONS if p != args.precision])
    jks = {p: cdlib.prepare_jk(d, m.C, p, lmo=p in FUSED) for p in precs}
    stream = torch.cuda.current_stream()

    # launch shapes: measured once on this workload (untimed), or the built-in ones
    tuning = cdlib.autotune([d], tau, schwarz) if args.tuning == "auto" else None

    def step(prec, phase_ev, jk_ev):
        cdlib.run_decompose([d], tau, schwarz, events=phase_ev, eta=args.eta, tuning=tuning)
        jk_ev[0].record(stream)
        cdlib.run_jk(jks[prec], prec)
        jk_ev[1].record(stream)
        if prec not in FUSED:
            cdlib.transform(d, m.C, m.C, sync=False)
        jk_ev[2].record(stream)

    mk = lambda: torch.cuda.Event(enable_timing=True)  # noqa: E731

    def avg(evs, i, j, which):
        vals = [(pe if which == "p" else je)[i].elapsed_time((pe if which == "p" else je)[j])
                for pe, je in evs]
        return sum(vals) / len(vals)

    runs = {}
    for prec in precs:
        for _ in range(args.warmup):
            step(prec, [mk() for _ in range(4)], [mk() for _ in range(3)])
        evs = [([mk() for _ in range(4)], [mk() for _ in range(3)]) for _ in range(args.steps)]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for pe, je in evs:
            step(prec, pe, je)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / args.steps
        assert d.M() == M and int(d.status.item()) == 0
        runs[prec] = {"ms_per_step": ms, "setup": avg(evs, 0, 1, "p"),
                      "pivot_selection": avg(evs, 1, 2, "p"), "all_row_solve": avg(evs, 2, 3, "p"),
                      "cd": avg(evs, 0, 3, "p"), "jk": avg(evs, 0, 1, "j"),
                      "transform": avg(evs, 1, 2, "j")}
    head = runs[args.precision]

    # J/K of every precision from the same vectors (the last step's), against FP64
    rp_host = d.row_pair.cpu().numpy()
    mu = np.floor((np.sqrt(8.0 * rp_host + 1.0) - 1.0) / 2.0).astype(np.int64)
    n_diag = int(np.count_nonzero(rp_host == mu * (mu + 1) // 2 + mu))
    Ct = torch.as_tensor(m.C, device=dev)
    Dm = Ct @ Ct.T

    def e2(J, K):
        return float(2.0 * (Dm * J).sum() - (Dm * K).sum())

    for p in precs:
        cdlib.run_jk(jks[p], p)
    torch.cuda.synchronize()
    ref = jks["fp64"] if "fp64" in jks else None
    precision = {}
    for p in precs:
        r = runs[p]
        w_ex, w_dense = jk_work(N, O, n, M, n_diag, p in FUSED)
        e = {"step_ms": r["ms_per_step"], "jk_ms": r["jk"],
             "transform": "fused into the J/K build" if p in FUSED else "separate call",
             "transform_ms": None if p in FUSED else r["transform"],
             "jk_plus_transform_ms": r["jk"] + (0.0 if p in FUSED else r["transform"]),
             "jk_tflops": w_ex / ((r["jk"] + (0.0 if p in FUSED else r["transform"])) * 1e-3) / 1e12}
        if ref is not None and p != "fp64":
            e["error_vs_fp64"] = {"max_abs_dJ": float((jks[p].J - ref.J).abs().max()),
                                  "max_abs_dK": float((jks[p].K - ref.K).abs().max()),
                                  "abs_dE2": abs(e2(jks[p].J, jks[p].K) - e2(ref.J, ref.K))}
            if p in FUSED:
                e["error_vs_fp64"]["max_abs_dLmo"] = float(
                    (jks[p].Lmo[:M] - ref.Lmo[:M]).abs().max())
            e["speedup_step_vs_fp64"] = runs["fp64"]["ms_per_step"] / r["ms_per_step"]
            e["speedup_jk_vs_fp64"] = ((runs["fp64"]["jk"] + 0.0) /
                                       (r["jk"] + (0.0 if p in FUSED else r["transform"])))
        if p in ("bf16x3", "fp32"):
            # HBM bytes of the exchange product against the bytes of its operand
            # (the k-blocked X over N padded to 128-row tiles: 3 BF16 planes or FP32)
            kern = "k_syrk_bf16x3" if p == "bf16x3" else "k_syrk_f32"
            e["exchange_product_hbm_bytes"] = counter_traffic(kern, args.config, tau)
            e["exchange_product_operand_bytes"] = ((6.0 if p == "bf16x3" else 4.0) *
                                                   (-(-N // 128) * 128) * M * O)
        precision[p] = e

    # per-batch device-clock stamps of the pivot selection (one untimed run)
    cap = 4096
    timeline = torch.zeros(1 + 16 * cap, dtype=torch.int64, device=dev)
    cdlib.run_decompose([d], tau, schwarz, timeline=timeline, eta=args.eta, tuning=tuning)
    torch.cuda.synchronize()
    tl = timeline.cpu().numpy()
    nbatch = int(tl[0])
    st = tl[1:1 + 8 * min(nbatch, cap)].reshape(-1, 8)[:, :7].astype(float) / 100.0  # 100 MHz -> us
    stages = ["nominate+exchange", "union+select", "candidate_columns", "exchange_columns",
              "block_factor", "row_update"]
    st = st[np.all(st > 0, axis=1)]          # batches that ran every stage
    breakdown = {k: float((st[:, i + 1] - st[:, i]).sum()) for i, k in enumerate(stages)
                 if st.shape[0]}
    nblk = (M + 127) // 128
    s2 = tl[1 + 8 * cap:1 + 8 * cap + 8 * min(nblk, cap)].reshape(-1, 8)[:, :6].astype(float) / 100.0
    s2_stages = ["off_block_product", "integrals", "substitution", "residuals", "store"]
    s2 = s2[np.all(s2 > 0, axis=1)]
    s2_breakdown = {k: float((s2[:, i + 1] - s2[:, i]).sum()) for i, k in enumerate(s2_stages)
                    if s2.shape[0]}

    extras = {}
    if not args.no_extras:
        # a converged SCF on the step's vectors (outside the step)
        scf_res, scf_ms = run_scf(cdlib, d, m, args.precision,
                                  *((1e-10, 1e-8) if args.precision == "fp64" else (1e-6, 1e-6)))
        extras["scf"] = {"ms": scf_ms, "iterations": len(scf_res.energies),
                         "converged": scf_res.converged,
                         "ms_per_iteration": scf_ms / max(1, len(scf_res.energies)),
                         "energy": float(scf_res.energies[-1]), "jk_precision": args.precision}
        del scf_res
        # second-order energy from the step's vectors (outside the step, once):
        # the transform with occupied and virtual orbitals, then the contraction
        from paper_2609_00306_amd.inputs import mp2_orbitals
        Co, Cv, eo, ev = mp2_orbitals(m)
        V = Cv.shape[1]
        Bmo = cdlib.transform(d, Co, Cv)
        cdlib.mp2_energy(Bmo, d.n_vectors, eo, ev)   # warm-up
        e0, e1 = mk(), mk()
        e0.record(stream)
        E_mp2 = cdlib.mp2_energy(Bmo, d.n_vectors, eo, ev, sync=False)
        e1.record(stream)
        torch.cuda.synchronize()
        t_mp2 = e0.elapsed_time(e1)
        w_mp2 = O * (O + 1) / 2.0 * V * V * 2.0 * M   # (ia|jb), i <= j, all a, b
        extras["mp2"] = {"ms": t_mp2, "energy": float(E_mp2.item()), "n_virt": V,
                         "tflops": w_mp2 / (t_mp2 * 1e-3) / 1e12,
                         "frac_fp64_peak": w_mp2 / (t_mp2 * 1e-3) / 1e12 / PEAK["fp64"],
                         "work": "O(O+1)/2 V^2 2M (integrals of pairs i <= j)", "runs": 1}
        del Bmo

    restricted = None
    if fn is not None:
        # against the unrestricted decomposition of the same molecule: the
        # residual left outside the candidate block and the J/K energy change
        full = cdlib.decompose(m.xyz, m.alpha, tau, schwarz=schwarz)
        Jf, Kf = cdlib.build_jk(full, m.C, "fp64")
        Jr, Kr = cdlib.build_jk(d, m.C, "fp64")
        restricted = {"flagged_functions": int(fn.sum()), "n_active": d.n_active,
                      "n_active_unrestricted": full.n_active, "M_unrestricted": full.M(),
                      "max_residual": float(d.diag.max()),
                      "abs_dE2_vs_unrestricted": abs(e2(Jr, Kr) - e2(Jf, Kf)), "E2": e2(Jr, Kr)}
        del full, Jf, Kf, Jr, Kr

    batched = None
    if not args.no_batched:
        del jks
        torch.cuda.empty_cache()
        batched = batched_c4(max(1, min(args.steps, 3)), 1)

    t_sel, t_solve = head["pivot_selection"], head["all_row_solve"]
    w_cd = float(n) * M * (M - 1)                       # Schur / triangular-solve contraction
    w_sel = float(d.n_active) * M * (M - 1)             # the same contraction on the active rows
    roof = {
        "k_step2": {"kernel": "k_step2 (all-row blocked forward substitution, FP64 MFMA)",
                    "bound": "mfma", "achieved": w_cd / (t_solve * 1e-3) / 1e12,
                    "peak": PEAK["fp64"], "unit": "TFLOP/s",
                    "traffic": counter_traffic("k_step2", args.config, tau),
                    "work": "n M (M - 1) FP64 flops per launch", "launch_ms": t_solve},
        "k_step1": {"kernel": "k_step1 (pivot selection on the active rows, one cooperative "
                              "launch of candidate batches; launch_ms is the phase, which also "
                              "holds the pivot-block inverses and the solve's integral pass)",
                    "bound": "mfma", "achieved": w_sel / (t_sel * 1e-3) / 1e12,
                    "peak": PEAK["fp64"], "unit": "TFLOP/s",
                    "traffic": counter_traffic("k_step1", args.config, tau),
                    "work": "n_active M (M - 1) FP64 flops per launch", "launch_ms": t_sel},
    }
    for r in roof.values():
        r["frac"] = r["achieved"] / r["peak"]
    dominant = "k_step1" if t_sel > t_solve else "k_step2"
    other = "k_step2" if dominant == "k_step1" else "k_step1"
    ms = head["ms_per_step"]
    w_ex, w_dense = jk_work(N, O, n, M, n_diag, args.precision in FUSED)
    out = {
        "metric": METRIC,
        "value": M / (ms * 1e-3),
        "unit": "vectors/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else f"f64 decomposition, {args.precision} K",
        "data": "synthetic",
        "config": {"workload": f"{args.config}: {N} s-Gaussians ({cfg['n_centres']} centres, "
                               f"{cfg['box']:.1f} A box, {len(cfg['exponents'])} exponents), "
                               f"tau={tau:g}, Schwarz {schwarz:g}, O={O}",
                   "n_basis": N, "n_rows": n, "n_active": d.n_active, "n_vectors": M,
                   "tau": tau, "n_occ": O, "jk_precision": args.precision, "eta": args.eta,
                   "pivot_block": args.pivot_block,
                   "tuning": None if tuning is None else
                   {"step2_row_tiles": tuning.step2_row_tiles,
                    "step1_min_rows": tuning.step1_min_rows, "step1_q": tuning.step1_q}},
        "cd_ms": head["cd"],
        "cd_vectors_per_s": M / (head["cd"] * 1e-3),
        "jk_ms": head["jk"],
        "jk_tflops": w_ex / ((head["jk"] + (0.0 if args.precision in FUSED else
                                            head["transform"])) * 1e-3) / 1e12,
        "jk_tflops_dense_equivalent": w_dense / (head["jk"] * 1e-3) / 1e12,
        "jk_work": "executed: 4nM (J) + 2 deg O M (half transform over kept pairs, deg = 2n - "
                   "kept diagonal pairs) + N(N+1) O M (exchange product) + 2 N O^2 M (fused "
                   "C^T L C); dense equivalent: 4nM + 2N^2 O M + N(N+1) O M",
        "precision": precision,
        "batched_c4": batched,
        "phases_ms": {"setup": head["setup"], "pivot_selection": t_sel, "all_row_solve": t_solve},
        "pivot_selection": {"batches": nbatch, "vectors_per_batch": M / max(1, nbatch),
                            "stage_us_total": breakdown},
        "all_row_solve_wg0_stage_us_total": s2_breakdown,
        "restricted_candidates": restricted,
        "roofline": {k: v for k, v in roof[dominant].items()},
        "roofline_other_kernel": roof[other],
    }
    out.update(extras)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(m, tau, schwarz, M, args.cpu_prefix)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
