"""Benchmark of the full hot path on one MI355X.

One step = cd_decompose (pairs, diagonal, screening, pivot selection,
all-row solve) + cd_build_jk (J and K) + cd_transform (AO->MO transform of
every vector with the occupied coefficients on both sides), on the
400-function workload (100 centres in a 16 angstrom box, exponents 0.1 ..
10 bohr^-2, 50 occupied orbitals, Schwarz screening 1e-12) at tau = 1e-6.
Inputs are resident in device memory before the timed region.

Prints one JSON line.  value = Cholesky vectors per second of the whole step
(M / step time).  Extra fields give the decomposition alone, J/K TFLOP/s,
per-phase device times from HIP events recorded on the library's stream, the
roofline of the dominant kernel and the CPU oracle's rate.
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

# HBM bytes per launch of the two decomposition kernels on the default workload
# (400 functions, tau = 1e-6), from two rocprofv3 --pmc runs of
# `bench.py --steps 1 --warmup 0` (FETCH_SIZE, then WRITE_SIZE, KiB per
# dispatch), each scaled by what the same counter reads for a plain 1 GiB
# device copy (`bench.py --copy-probe 1024`): FETCH_SIZE reads 524 302 KiB
# there (factor 2.0), WRITE_SIZE 1 048 576 KiB (factor 1.0).  The figures
# belong to the kernel sources they were taken on; once those change the
# traffic is reported as null until the counters are taken again.
KERNEL_SOURCES = ["paper_2609_00306_amd/csrc/cd_decompose.hip",
                  "paper_2609_00306_amd/csrc/cd_mfma.hpp",
                  "paper_2609_00306_amd/csrc/cd_device.hpp",
                  "paper_2609_00306_amd/csrc/cd_kernels.hpp"]
FETCH_SCALE, WRITE_SCALE = 1048576.0 / 524302.2, 1048576.0 / 1048576.0
COUNTERS = {
    "sources_sha256": "759c7b00a436e790c22cb8ab041cca7fbabadcfe2e0e7788284f191b6d398992",
    "workload": ("C2", 1e-6),
    "fetch_kib": {"k_step2": 2348599.5, "k_step1": 73105.5},
    "write_kib": {"k_step2": 259291.5, "k_step1": 30159.5},
}


def kernel_sources_sha256():
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def counter_traffic(kernel, config, tau):
    """HBM bytes per launch of 'kernel' from the recorded counters, or None."""
    if (config, tau) != COUNTERS["workload"]:
        return None
    if kernel_sources_sha256() != COUNTERS["sources_sha256"]:
        return None
    return 1024.0 * (COUNTERS["fetch_kib"][kernel] * FETCH_SCALE
                     + COUNTERS["write_kib"][kernel] * WRITE_SCALE)


def cpu_baseline(m, tau, schwarz):
    """The CPU oracle timed on the host cores: one full decomposition + FP64 J/K."""
    import oracle
    rp, _ = oracle.rows(m.xyz, m.alpha, schwarz)
    t0 = time.perf_counter()
    ref = oracle.decompose(m.xyz, m.alpha, rp, tau)
    t1 = time.perf_counter()
    oracle.jk_cd(m.n_basis, rp, ref.L, m.C)
    t2 = time.perf_counter()
    cores = int(os.environ.get("OMP_NUM_THREADS") or os.cpu_count() or 1)
    return {"value": ref.M / (t2 - t0), "unit": "vectors/s", "cores": cores, "kind": "oracle",
            "sample": f"one full step of the same workload: decomposition (M={ref.M}) "
                      f"{t1 - t0:.2f} s + FP64 J/K {t2 - t1:.2f} s"}


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


def bench_batched(args):
    """64 molecules of uneven size (52..400 functions), tau = 1e-5: one batched
    cd_decompose call plus one cd_build_jk call (FP32 K) per step, against the
    same molecules run one by one on the plain path (FP64 J/K)."""
    import torch

    from paper_2609_00306_amd import cdlib
    from paper_2609_00306_amd.inputs import BATCH_C4, batch_c4

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
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
    jks, jws = cdlib.prepare_jk_many(decs, [m.C for m in mols], "fp32")
    singles = [cdlib.allocate(m.xyz, m.alpha, tau, schwarz, M, device=dev) for m, M in zip(mols, Ms)]
    sjks = [cdlib.prepare_jk(d, m.C, "fp64") for d, m in zip(singles, mols)]

    # launch shapes of the batched decomposition chosen by measurement (untimed)
    tuning = cdlib.autotune(decs, tau, schwarz, workspace=ws)

    def batched():
        cdlib.run_decompose(decs, tau, schwarz, workspace=ws, tuning=tuning)
        cdlib.run_jk_many(jks, jws, "fp32")

    def batched_builtin():
        cdlib.run_decompose(decs, tau, schwarz, workspace=ws)
        cdlib.run_jk_many(jks, jws, "fp32")

    def plain():
        for d, j in zip(singles, sjks):
            cdlib.run_decompose([d], tau, schwarz)
            cdlib.run_jk(j, "fp64")

    def timed(fn):
        for _ in range(args.warmup):
            fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) * 1e3 / args.steps

    ms_b = timed(batched)
    ms_bb = timed(batched_builtin)
    ms_p = timed(plain)
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
        ms_g = timed(g.replay)
        graph = {"captured": True, "ms_per_step": ms_g, "vectors_per_s": sum(Ms) / (ms_g * 1e-3)}
    except Exception as e:  # a cooperative launch may not be capturable
        graph = {"captured": False, "reason": str(e)[:200]}
    M_tot = sum(Ms)
    out = {
        "metric": "Cholesky vectors/s + J/K build TFLOP/s at tau=1e-6; mixed/batched vs plain FP64",
        "value": M_tot / (ms_b * 1e-3),
        "unit": "vectors/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_b,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64 decomposition, fp32 K", "data": "synthetic",
        "config": {"workload": f"batched: {len(mols)} molecules, N {min(m.n_basis for m in mols)}"
                               f"..{max(m.n_basis for m in mols)} s-Gaussians, tau={tau:g}, "
                               f"O=N/8, FP32 K", "n_molecules": len(mols), "n_vectors": M_tot},
        "plain_one_by_one": {"ms_per_step": ms_p, "vectors_per_s": M_tot / (ms_p * 1e-3),
                             "jk_precision": "fp64"},
        "speedup_vs_plain": ms_p / ms_b,
        "tuning": {"step2_row_tiles": tuning.step2_row_tiles,
                   "step1_min_rows": tuning.step1_min_rows,
                   "builtin_shapes_ms_per_step": ms_bb},
        "graph": graph,
    }
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
        for prec in ("fp64", "fp32", "bf16x3"):
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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--config", default="C2")
    ap.add_argument("--tau", type=float, default=1e-6)
    ap.add_argument("--precision", default="fp64", choices=["fp64", "fp32", "bf16x3"])
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
    # in FP64 and 3 x BF16 the J/K build also writes the transformed vectors
    # C^T L C from the FP64 half transform it already forms; in FP32 the
    # transform is its own call
    fused = args.precision in ("fp64", "bf16x3")
    jk = cdlib.prepare_jk(d, m.C, args.precision, lmo=fused)
    stream = torch.cuda.current_stream()

    # launch shapes: measured once on this workload (untimed), or the built-in ones
    tuning = cdlib.autotune([d], tau, schwarz) if args.tuning == "auto" else None

    def step(phase_ev, jk_ev):
        cdlib.run_decompose([d], tau, schwarz, events=phase_ev, eta=args.eta, tuning=tuning)
        jk_ev[0].record(stream)
        cdlib.run_jk(jk, args.precision)
        jk_ev[1].record(stream)
        if not fused:
            cdlib.transform(d, m.C, m.C, sync=False)
        jk_ev[2].record(stream)

    mk = lambda: torch.cuda.Event(enable_timing=True)  # noqa: E731
    for _ in range(args.warmup):
        step([mk() for _ in range(4)], [mk() for _ in range(3)])
    torch.cuda.synchronize()

    # per-batch device-clock stamps of the pivot selection (one untimed step)
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
    nblk = (M + 63) // 64
    s2 = tl[1 + 8 * cap:1 + 8 * cap + 8 * min(nblk, cap)].reshape(-1, 8)[:, :6].astype(float) / 100.0
    s2_stages = ["off_block_product", "stage", "integrals", "substitution", "store"]
    s2 = s2[np.all(s2 > 0, axis=1)]
    s2_breakdown = {k: float((s2[:, i + 1] - s2[:, i]).sum()) for i, k in enumerate(s2_stages)
                    if s2.shape[0]}

    evs = [([mk() for _ in range(4)], [mk() for _ in range(3)]) for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for pe, je in evs:
        step(pe, je)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms = (t1 - t0) * 1e3 / args.steps
    assert d.M() == M and int(d.status.item()) == 0

    prec_err = None
    if args.precision != "fp64":
        # the reduced-precision J/K of the last step against the FP64 build from
        # the same vectors; E2 = 2 tr(DJ) - tr(DK), D = C C^T
        J64, K64 = cdlib.build_jk(d, m.C, "fp64")
        Ct = torch.as_tensor(m.C, device=dev)
        Dm = Ct @ Ct.T

        def e2(J, K):
            return float(2.0 * (Dm * J).sum() - (Dm * K).sum())

        prec_err = {"against": "FP64 J/K from the same vectors",
                    "max_abs_dJ": float((jk.J - J64).abs().max()),
                    "max_abs_dK": float((jk.K - K64).abs().max()),
                    "abs_dE2": abs(e2(jk.J, jk.K) - e2(J64, K64))}

    # a converged SCF on the step's vectors (outside the step)
    scf_res, scf_ms = run_scf(cdlib, d, m, args.precision,
                              *((1e-10, 1e-8) if args.precision == "fp64" else (1e-6, 1e-6)))
    scf = {"ms": scf_ms, "iterations": len(scf_res.energies), "converged": scf_res.converged,
           "ms_per_iteration": scf_ms / max(1, len(scf_res.energies)),
           "energy": float(scf_res.energies[-1]), "jk_precision": args.precision}
    del scf_res

    restricted = None
    if fn is not None:
        # against the unrestricted decomposition of the same molecule: the
        # residual left outside the candidate block and the J/K energy change
        full = cdlib.decompose(m.xyz, m.alpha, tau, schwarz=schwarz)
        Jf, Kf = cdlib.build_jk(full, m.C, "fp64")
        Jr, Kr = cdlib.build_jk(d, m.C, "fp64")
        Ct = torch.as_tensor(m.C, device=dev)
        Dm = Ct @ Ct.T
        e2f = float(2.0 * (Dm * Jf).sum() - (Dm * Kf).sum())
        e2r = float(2.0 * (Dm * Jr).sum() - (Dm * Kr).sum())
        restricted = {"flagged_functions": int(fn.sum()), "n_active": d.n_active,
                      "n_active_unrestricted": full.n_active, "M_unrestricted": full.M(),
                      "max_residual": float(d.diag.max()),
                      "abs_dE2_vs_unrestricted": abs(e2r - e2f), "E2": e2r}
        del full, Jf, Kf, Jr, Kr

    # second-order energy from the step's vectors (outside the step): the
    # transform with occupied and virtual orbitals, then the contraction
    from paper_2609_00306_amd.inputs import mp2_orbitals
    Co, Cv, eo, ev = mp2_orbitals(m)
    V = Cv.shape[1]
    Bmo = cdlib.transform(d, Co, Cv)
    E_mp2 = cdlib.mp2_energy(Bmo, d.n_vectors, eo, ev)
    mp2_ev = [mk() for _ in range(args.steps + 1)]
    mp2_ev[0].record(stream)
    for k in range(args.steps):
        cdlib.mp2_energy(Bmo, d.n_vectors, eo, ev, sync=False)
        mp2_ev[k + 1].record(stream)
    torch.cuda.synchronize()
    t_mp2 = mp2_ev[0].elapsed_time(mp2_ev[-1]) / args.steps
    w_mp2 = O * (O + 1) / 2.0 * V * V * 2.0 * M   # (ia|jb), i <= j, all a, b
    mp2 = {"ms": t_mp2, "energy": float(E_mp2.item()), "n_virt": V,
           "tflops": w_mp2 / (t_mp2 * 1e-3) / 1e12,
           "frac_fp64_peak": w_mp2 / (t_mp2 * 1e-3) / 1e12 / PEAK["fp64"],
           "work": "O(O+1)/2 V^2 2M (integrals of pairs i <= j)"}
    del Bmo

    def avg(i, j, which):
        vals = []
        for pe, je in evs:
            e = pe if which == "p" else je
            vals.append(e[i].elapsed_time(e[j]))
        return sum(vals) / len(vals)

    t_setup = avg(0, 1, "p")
    t_sel = avg(1, 2, "p")
    t_solve = avg(2, 3, "p")
    t_cd = avg(0, 3, "p")
    t_jk = avg(0, 1, "j")
    t_tr = avg(1, 2, "j")
    w_cd = float(n) * M * (M - 1)                       # Schur / triangular-solve contraction
    w_sel = float(d.n_active) * M * (M - 1)             # the same contraction on the active rows
    w_j = 4.0 * n * M
    w_k = 2.0 * N * N * O * M + float(N) * (N + 1) * O * M
    roof = {
        "k_step2": {"kernel": "k_step2 (all-row blocked forward substitution, FP64 MFMA)",
                    "bound": "mfma", "achieved": w_cd / (t_solve * 1e-3) / 1e12,
                    "peak": PEAK["fp64"], "unit": "TFLOP/s",
                    "traffic": counter_traffic("k_step2", args.config, tau)},
        "k_step1": {"kernel": "k_step1 (pivot selection on the active rows, one cooperative "
                              "launch of candidate batches)",
                    "bound": "mfma", "achieved": w_sel / (t_sel * 1e-3) / 1e12,
                    "peak": PEAK["fp64"], "unit": "TFLOP/s",
                    "traffic": counter_traffic("k_step1", args.config, tau)},
    }
    for r in roof.values():
        r["frac"] = r["achieved"] / r["peak"]
    dominant = "k_step1" if t_sel > t_solve else "k_step2"
    other = "k_step2" if dominant == "k_step1" else "k_step1"
    out = {
        "metric": "Cholesky vectors/s + J/K build TFLOP/s at tau=1e-6; mixed/batched vs plain FP64",
        "value": M / (ms * 1e-3),
        "unit": "vectors/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else f"f64 decomposition, {args.precision} J/K",
        "data": "synthetic",
        "config": {"workload": f"{N} s-Gaussians ({cfg['n_centres']} centres, "
                               f"{cfg['box']:.1f} A box, {len(cfg['exponents'])} exponents), "
                               f"tau={tau:g}, Schwarz {schwarz:g}, O={O}",
                   "n_basis": N, "n_rows": n, "n_active": d.n_active, "n_vectors": M,
                   "tau": tau, "n_occ": O, "jk_precision": args.precision, "eta": args.eta,
                   "pivot_block": args.pivot_block,
                   "tuning": None if tuning is None else
                   {"step2_row_tiles": tuning.step2_row_tiles,
                    "step1_min_rows": tuning.step1_min_rows}},
        "cd_ms": t_cd,
        "cd_vectors_per_s": M / (t_cd * 1e-3),
        "jk_ms": t_jk,
        "jk_tflops": (w_j + w_k) / (t_jk * 1e-3) / 1e12,
        "transform_ms": None if fused else t_tr,
        "transform": "fused into the J/K build (C^T L C from its half transform)" if fused
                     else "separate call",
        "mp2": mp2,
        "scf": scf,
        "restricted_candidates": restricted,
        "phases_ms": {"setup": t_setup, "pivot_selection": t_sel, "all_row_solve": t_solve},
        "pivot_selection": {"batches": nbatch, "vectors_per_batch": M / max(1, nbatch),
                            "stage_us_total": breakdown},
        "all_row_solve_wg0_stage_us_total": s2_breakdown,
        "jk_tflops_work": "dense-equivalent 4nM + 2N^2 O M + N(N+1) O M",
        "precision_error": prec_err,
        "roofline": roof[dominant],
        "roofline_other_kernel": roof[other],
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(m, tau, schwarz)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
