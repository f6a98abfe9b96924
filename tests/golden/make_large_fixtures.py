"""Write the oracle's results on the two large workloads to tests/golden/.

The oracle's decomposition of the 1000- and 1200-function workloads (and its
J/K from its own vectors) takes minutes, too long for a GPU test, so this
script runs it once and stores what the GPU tests compare with.  It calls
only the CPU oracle (``oracle/``) and the seeded input generators; nothing
here comes from the GPU library.

    python tests/golden/make_large_fixtures.py C3 C5

Stored per workload (``<name>_tau1e-6.npz``), all from one oracle run at
tau = 1e-6, Schwarz screening 1e-12:

* the pivot sequence and the pivot values d_K (Sec. 2: the residual diagonal
  at the pivot when vector K is formed);
* the final residual diagonal at 4096 sampled rows, and its maximum;
* L at 4096 sampled (vector, row) entries, and L^K at its own pivot row for
  every K;
* J and K (Sec. 4.1, D = C C^T, from the oracle's vectors) on six full rows
  and on the diagonal, and E2 = 2 tr(DJ) - tr(DK) with both traces.

The sample indices are drawn from PCG64(2026) and stored with the values.
"""
from __future__ import annotations

import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2609_00306_amd.inputs import CONFIGS, config_molecule  # noqa: E402

TAU = 1e-6
SCHWARZ = 1e-12
N_SAMPLE = 4096
N_ROWS_JK = 6


def fixture_path(name: str) -> str:
    return os.path.join(HERE, f"{name}_tau1e-6.npz")


def make(name: str) -> None:
    m = config_molecule(name)
    assert CONFIGS[name]["schwarz"] == SCHWARZ
    N, O = m.n_basis, m.n_occ
    rp, _ = oracle.rows(m.xyz, m.alpha, SCHWARZ)
    n = len(rp)
    t0 = time.time()
    ref = oracle.decompose(m.xyz, m.alpha, rp, TAU, max_vectors=min(n, 8192))
    t1 = time.time()
    assert ref.rc == 0, f"oracle status {ref.rc}"
    M = ref.M
    print(f"{name}: n={n} M={M} decomposition {t1 - t0:.1f} s", flush=True)
    J, K = oracle.jk_cd(N, rp, ref.L, m.C)
    t2 = time.time()
    print(f"{name}: J/K {t2 - t1:.1f} s", flush=True)
    Dm = m.C @ m.C.T
    e2 = oracle.e2(m.C, J, K)

    rng = np.random.Generator(np.random.PCG64(2026))
    d_idx = np.sort(rng.choice(n, size=min(N_SAMPLE, n), replace=False))
    l_k = rng.integers(0, M, size=N_SAMPLE)
    l_r = rng.integers(0, n, size=N_SAMPLE)
    mu_sel = np.sort(rng.choice(N, size=N_ROWS_JK, replace=False))
    piv = ref.pivots
    np.savez_compressed(
        fixture_path(name),
        name=name, tau=TAU, schwarz=SCHWARZ, n_basis=N, n_occ=O, n_rows=n, M=M,
        row_pair_first=rp[:16], row_pair_last=rp[-16:],
        pivots=piv.astype(np.int64), dpiv=ref.dpiv,
        d_idx=d_idx.astype(np.int64), d_val=ref.D[d_idx], d_max=float(ref.D.max()),
        l_k=l_k.astype(np.int64), l_r=l_r.astype(np.int64), l_val=ref.L[l_k, l_r],
        l_at_pivot=ref.L[np.arange(M), piv],
        mu_sel=mu_sel.astype(np.int64), J_rows=J[mu_sel], K_rows=K[mu_sel],
        J_diag=np.diag(J).copy(), K_diag=np.diag(K).copy(),
        e2=e2, tr_DJ=float(np.sum(Dm * J)), tr_DK=float(np.sum(Dm * K)),
        oracle_seconds=np.array([t1 - t0, t2 - t1]))
    print(f"{name}: wrote {fixture_path(name)}", flush=True)


if __name__ == "__main__":
    for a in sys.argv[1:] or ["C3", "C5"]:
        make(a)
