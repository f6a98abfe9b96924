"""GPU parity on the two large workloads (1000 and 1200 functions, tau = 1e-6)
against the oracle's stored results (tests/golden/, written by
make_large_fixtures.py, which calls only the oracle).

The decomposition is held to the oracle pivot for pivot, with the pivot
values, sampled vectors and sampled final residuals within 1e-10.  J and K,
built by the GPU in FP64, FP32 and 3xBF16 from the GPU's vectors, are held on
six full rows and on the diagonal to the oracle's J and K from the oracle's
vectors: 1e-10 in FP64, 1e-6 Eh with reduced-precision K (J is FP64 in every
mode), and E2 = 2 tr(DJ) - tr(DK) likewise.  The launch configuration is the
one the benchmark times (built-in shapes, one problem per call).
"""
import os

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

import oracle  # noqa: E402
from paper_2609_00306_amd import cdlib  # noqa: E402
from paper_2609_00306_amd.inputs import config_molecule  # noqa: E402

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
TOL_L = 1e-10
TOL_JK = 1e-10
TOL_K_LP = 1e-6
TOL_E2_LP = 1e-6


def _fixture(name):
    path = os.path.join(GOLDEN, f"{name}_tau1e-6.npz")
    assert os.path.exists(path), f"missing {path}: run tests/golden/make_large_fixtures.py"
    return np.load(path, allow_pickle=False)


@pytest.fixture(scope="module", autouse=True)
def gpu():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    cdlib.load()
    return torch.device("cuda:0")


@pytest.mark.parametrize("name", ["C3", "C5"])
def test_large_workload_against_oracle_fixture(name):
    f = _fixture(name)
    m = config_molecule(name)
    tau, schwarz = float(f["tau"]), float(f["schwarz"])
    d = cdlib.decompose(m.xyz, m.alpha, tau, schwarz=schwarz)
    M = d.M()
    assert int(d.status.item()) == 0
    assert d.n_rows == int(f["n_rows"])
    rp = d.row_pair.cpu().numpy()
    assert np.array_equal(rp[:16], f["row_pair_first"]) and np.array_equal(rp[-16:],
                                                                           f["row_pair_last"])
    rp_o, _ = oracle.rows(m.xyz, m.alpha, schwarz)
    assert np.array_equal(rp, rp_o)
    # pivot for pivot, with the pivot values
    assert M == int(f["M"])
    assert np.array_equal(d.pivots[:M].cpu().numpy(), f["pivots"])
    assert np.abs(d.pivot_values[:M].cpu().numpy() - f["dpiv"]).max() <= TOL_L
    # sampled vectors, vectors at their own pivots, sampled final residuals
    lk = torch.as_tensor(f["l_k"], device=d.L.device)
    lr = torch.as_tensor(f["l_r"], device=d.L.device)
    assert np.abs(d.L[lk, lr].cpu().numpy() - f["l_val"]).max() <= TOL_L
    ar = torch.arange(M, device=d.L.device)
    assert np.abs(d.L[ar, d.pivots[:M]].cpu().numpy() - f["l_at_pivot"]).max() <= TOL_L
    diag = d.diag.cpu().numpy()
    assert np.abs(diag[f["d_idx"]] - f["d_val"]).max() <= TOL_L
    assert diag.max() < tau and abs(diag.max() - float(f["d_max"])) <= TOL_L

    # J and K in each precision against the oracle's J/K from the oracle's vectors
    mu = f["mu_sel"]
    Ct = torch.as_tensor(m.C, device=d.L.device)
    Dm = (Ct @ Ct.T).cpu().numpy()
    for prec in ("fp64", "fp32", "bf16x3"):
        J, K = cdlib.build_jk(d, m.C, prec)
        J, K = J.cpu().numpy(), K.cpu().numpy()
        tol_k = TOL_JK if prec == "fp64" else TOL_K_LP
        assert np.abs(J[mu] - f["J_rows"]).max() <= TOL_JK, prec
        assert np.abs(np.diag(J) - f["J_diag"]).max() <= TOL_JK, prec
        assert np.abs(K[mu] - f["K_rows"]).max() <= tol_k, prec
        assert np.abs(np.diag(K) - f["K_diag"]).max() <= tol_k, prec
        assert np.array_equal(K, K.T) and np.array_equal(J, J.T)
        tr_dj, tr_dk = float(np.sum(Dm * J)), float(np.sum(Dm * K))
        e2 = 2.0 * tr_dj - tr_dk
        if prec == "fp64":
            assert abs(e2 - float(f["e2"])) <= 1e-12 * abs(float(f["e2"])) + 1e-9
        else:
            assert abs(e2 - float(f["e2"])) <= TOL_E2_LP, prec
        del J, K
