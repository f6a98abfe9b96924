"""GPU parity: the HIP path (through the C ABI) against the CPU oracle on the
same seeded inputs.

Bar: row sets and pivot sequences identical (or, where the sequences part at
a near-tie, every GPU pivot a valid argmax of the oracle's own residuals
within 1e-12 max D1, with the oracle replaying the GPU's pivots); vectors
and final residual diagonal within 1e-10 absolute; J and K (FP64) within
1e-10.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

import oracle  # noqa: E402
from paper_2609_00306_amd import cdlib  # noqa: E402
from paper_2609_00306_amd.inputs import config_molecule, make_molecule, random_small  # noqa: E402

TOL_L = 1e-10
TOL_JK = 1e-10


@pytest.fixture(scope="module", autouse=True)
def gpu():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    cdlib.load()
    return torch.device("cuda:0")


def run_gpu(m, tau, schwarz, max_vectors=None):
    # asynchronous call; the device status word is checked by the caller
    d = cdlib.decompose(m.xyz, m.alpha, tau, schwarz=schwarz, max_vectors=max_vectors,
                        sync=False)
    torch.cuda.synchronize()
    M = d.M()
    return d, M


_ORACLE_CACHE = {}


def gpu_e2(C, J, K):
    """E2 = 2 tr(DJ) - tr(DK), D = C C^T, of GPU results (numpy on the host; the
    oracle's own E2 is taken only from the oracle's J and K)."""
    Dm = np.asarray(C) @ np.asarray(C).T
    return float(2.0 * np.sum(Dm * J) - np.sum(Dm * K))


def oracle_cd(m, rp, tau, cap, pivot_fn=None):
    fk = None if pivot_fn is None else bytes(np.asarray(pivot_fn, dtype=np.uint8))
    key = (m.name, m.seed, m.n_basis, tau, len(rp), cap, fk)
    if key not in _ORACLE_CACHE:
        _ORACLE_CACHE[key] = oracle.decompose(m.xyz, m.alpha, rp, tau, max_vectors=cap,
                                              pivot_fn=pivot_fn)
    return _ORACLE_CACHE[key]


def check_against_oracle(m, tau, schwarz, d, M, expect_status=0, pivot_fn=None):
    """Compare one GPU decomposition with the oracle; returns the oracle result used."""
    assert int(d.status.item()) == expect_status
    rp, _ = oracle.rows(m.xyz, m.alpha, schwarz)
    rp_g = d.row_pair.cpu().numpy()
    assert np.array_equal(rp, rp_g), "screened row sets differ"
    piv = d.pivots[:M].cpu().numpy()
    cap = d.max_vectors
    ref = oracle_cd(m, rp, tau, cap, pivot_fn)
    if not (ref.M == M and np.array_equal(ref.pivots, piv)):
        D1max = float(np.max(oracle.diagonal_all(m.xyz, m.alpha))) if m.n_basis else 0.0
        ref = oracle.decompose(m.xyz, m.alpha, rp, tau, max_vectors=cap, given=piv,
                               tie_tol=1e-12 * D1max, pivot_fn=pivot_fn)
        assert ref.bad == -1, f"GPU pivot {ref.bad} is not a valid argmax"
        assert ref.M == M
    L = d.L[:M].cpu().numpy()
    if M:
        err = np.abs(L - ref.L).max()
        assert err <= TOL_L, f"max |dL| = {err:.3e}"
    diag = d.diag.cpu().numpy()
    if len(diag):
        assert np.abs(diag - ref.D).max() <= TOL_L
    return rp, ref


@pytest.mark.parametrize("seed,tau", [(1, 1e-3), (2, 1e-6), (3, 1e-9), (4, 0.0), (5, 1e-6)])
def test_tiny_molecules(seed, tau):
    m = random_small(seed, n_centres=3 + seed % 3, exps=(0.25, 1.0, 4.0))
    d, M = run_gpu(m, tau, 0.0)
    check_against_oracle(m, tau, 0.0, d, M)


def test_c1_full_matrix():
    m = config_molecule("C1")
    d, M = run_gpu(m, 1e-6, 0.0)
    assert d.n_rows == 1830
    rp, ref = check_against_oracle(m, 1e-6, 0.0, d, M)
    assert M == 235


def test_ragged_sizes_several_tiles():
    # 37 functions: 703 rows, not a multiple of any tile; small tau -> many batches
    m = make_molecule(37, 6.0, (0.5,), 3, seed=77)
    d, M = run_gpu(m, 1e-10, 1e-12)
    check_against_oracle(m, 1e-10, 1e-12, d, M)


@pytest.mark.parametrize("tau", [1e-4, 1e-6])
def test_c2_parity(tau):
    m = config_molecule("C2")
    d, M = run_gpu(m, tau, 1e-12)
    check_against_oracle(m, tau, 1e-12, d, M)


def test_capacity_limit():
    m = config_molecule("C1")
    d, M = run_gpu(m, 1e-6, 0.0, max_vectors=50)
    assert M == 50
    check_against_oracle(m, 1e-6, 0.0, d, M, expect_status=cdlib.CD_ERR_CAPACITY)


def test_empty_and_single_function():
    m0 = make_molecule(0, 1.0, (1.0,), 0, seed=1)
    d, M = run_gpu(m0, 1e-6, 1e-12, max_vectors=1)
    assert M == 0 and d.n_rows == 0 and int(d.status.item()) == 0
    xyz = np.zeros((1, 3))
    alpha = np.array([0.8])
    d = cdlib.decompose(xyz, alpha, 1e-6, schwarz=0.0)
    assert d.M() == 1
    assert d.L[0, 0].item() == pytest.approx(np.sqrt(2.0 * np.sqrt(0.8 / np.pi)), rel=1e-14)


def test_deterministic_repeat():
    m = config_molecule("C2")
    d1, M1 = run_gpu(m, 1e-5, 1e-12)
    d2, M2 = run_gpu(m, 1e-5, 1e-12)
    assert M1 == M2
    assert torch.equal(d1.pivots[:M1], d2.pivots[:M2])
    assert torch.equal(d1.L[:M1], d2.L[:M2])


@pytest.mark.parametrize("name,schwarz", [("C1", 0.0), ("C2", 1e-12)])
def test_jk_fp64_parity(name, schwarz):
    m = config_molecule(name)
    tau = 1e-6
    d, M = run_gpu(m, tau, schwarz)
    rp, ref = check_against_oracle(m, tau, schwarz, d, M)
    J, K = cdlib.build_jk(d, m.C, "fp64")
    Jr, Kr = oracle.jk_cd(m.n_basis, rp, ref.L, m.C)
    J = J.cpu().numpy()
    K = K.cpu().numpy()
    assert np.abs(J - Jr).max() <= TOL_JK
    assert np.abs(K - Kr).max() <= TOL_JK
    assert np.array_equal(J, J.T) and np.array_equal(K, K.T)


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3"])
@pytest.mark.parametrize("name", ["C1", "C2"])
def test_jk_with_fused_transform(name, prec):
    """The J/K build with the optional MO-basis output (FP64, and FP32 and
    3 x BF16, whose half transform is FP64 before rounding or splitting): J and
    K as without it, and C^T L^P C equal to the stand-alone transform with
    C1 = C2 = C and to the oracle's."""
    m = config_molecule(name)
    d, M = run_gpu(m, 1e-6, 1e-12)
    rp, ref = check_against_oracle(m, 1e-6, 1e-12, d, M)
    jk = cdlib.prepare_jk(d, m.C, prec, lmo=True)
    cdlib.run_jk(jk, prec, sync=True)
    J0, K0 = cdlib.build_jk(d, m.C, prec)
    assert torch.equal(jk.J, J0) and torch.equal(jk.K, K0)
    T = cdlib.transform(d, m.C, m.C)
    assert torch.equal(jk.Lmo[:M], T[:M])
    exp = oracle.transform(m.n_basis, rp, ref.L, m.C, m.C)
    assert np.abs(jk.Lmo[:M].cpu().numpy() - exp).max() <= TOL_L
    # the FP32 build with the MO output needs the FP64 copy of the half
    # transform: a workspace sized for FP64 is refused
    with pytest.raises(cdlib.CDError) as e:
        cdlib.run_jk(cdlib.prepare_jk(d, m.C, "fp64", lmo=True), "fp32", sync=True)
    assert e.value.status == cdlib.CD_ERR_WORKSPACE


def test_transform_parity():
    m = config_molecule("C1")
    d, M = run_gpu(m, 1e-6, 0.0)
    rp, ref = check_against_oracle(m, 1e-6, 0.0, d, M)
    C1 = m.C[:, :7]
    C2 = m.C[:, 2:10]
    out = cdlib.transform(d, C1, C2)[:M].cpu().numpy()
    exp = oracle.transform(m.n_basis, rp, ref.L, C1, C2)
    assert np.abs(out - exp).max() <= TOL_L


# Reduced-precision J/K (FP32 and split 3xBF16 on matrix cores, FP32 inside
# k-slabs of 32, FP64 across): J is FP64 in every mode; K and the two-electron
# energy against the oracle's FP64 build from the oracle's vectors.
TOL_K = {"fp32": 1e-6, "bf16x3": 1e-6}
TOL_E2 = {"fp32": 1e-6, "bf16x3": 1e-6}


@pytest.mark.parametrize("prec", ["fp32", "bf16x3"])
@pytest.mark.parametrize("name,schwarz", [("C1", 0.0), ("C2", 1e-12)])
def test_jk_reduced_precision(name, schwarz, prec):
    m = config_molecule(name)
    d, M = run_gpu(m, 1e-6, schwarz)
    rp, ref = check_against_oracle(m, 1e-6, schwarz, d, M)
    Jr, Kr = oracle.jk_cd(m.n_basis, rp, ref.L, m.C)
    J, K = cdlib.build_jk(d, m.C, prec)
    J = J.cpu().numpy()
    K = K.cpu().numpy()
    assert np.abs(J - Jr).max() <= TOL_JK
    assert np.abs(K - Kr).max() <= TOL_K[prec]
    assert np.array_equal(K, K.T)
    assert abs(gpu_e2(m.C, J, K) - oracle.e2(m.C, Jr, Kr)) <= TOL_E2[prec]


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3"])
@pytest.mark.parametrize("n_occ", [100, 170])
def test_jk_wide_occupied_sets(n_occ, prec):
    """J/K with more occupied orbitals than the C1/C2 sets: 100 (one column range
    of 160, whose reduced-precision planes are staged through LDS) and 170 (two
    column ranges, whose planes are written value by value), 200 functions, against
    the oracle's FP64 build from the oracle's vectors, and C^T L C against the
    oracle's transform."""
    m = make_molecule(50, 10.0, (0.3, 1.5, 7.0, 30.0), n_occ, seed=91)
    d, M = run_gpu(m, 1e-6, 1e-12)
    rp, ref = check_against_oracle(m, 1e-6, 1e-12, d, M)
    Jr, Kr = oracle.jk_cd(m.n_basis, rp, ref.L, m.C)
    J, K = cdlib.build_jk(d, m.C, prec)
    J = J.cpu().numpy()
    K = K.cpu().numpy()
    assert np.abs(J - Jr).max() <= TOL_JK
    assert np.abs(K - Kr).max() <= (TOL_JK if prec == "fp64" else TOL_K[prec])
    assert np.array_equal(K, K.T)
    # with the MO-basis output (a transform product of two row ranges at 170)
    jk = cdlib.prepare_jk(d, m.C, prec, lmo=True)
    cdlib.run_jk(jk, prec, sync=True)
    assert np.array_equal(jk.K.cpu().numpy(), K)
    exp = oracle.transform(m.n_basis, rp, ref.L, m.C, m.C)
    assert np.abs(jk.Lmo[:M].cpu().numpy() - exp).max() <= TOL_L


def test_jk_large_tile_product():
    """600 functions (150 centres), where the FP64 exchange product runs on
    128 x 128 tile pairs: five tiles, the last holding 88 functions, so the
    second 64-row half of that tile is partly padding (the 1200-function
    workload, checked against stored oracle rows, has a fully padded half).
    J and K in every precision against the oracle's FP64 build from the
    oracle's vectors."""
    m = make_molecule(150, 16.0 * 1.5 ** (1.0 / 3.0), (0.3, 1.5, 7.0, 30.0), 75, seed=17)
    assert m.n_basis == 600
    d, M = run_gpu(m, 1e-5, 1e-12)
    rp, ref = check_against_oracle(m, 1e-5, 1e-12, d, M)
    Jr, Kr = oracle.jk_cd(m.n_basis, rp, ref.L, m.C)
    for prec in ("fp64", "fp32", "bf16x3"):
        J, K = cdlib.build_jk(d, m.C, prec)
        J = J.cpu().numpy()
        K = K.cpu().numpy()
        assert np.abs(J - Jr).max() <= TOL_JK, prec
        assert np.abs(K - Kr).max() <= (TOL_JK if prec == "fp64" else TOL_K[prec]), prec
        assert np.array_equal(K, K.T), prec


@pytest.mark.parametrize("name,eta", [("C1", 0.5), ("C1", 0.05), ("ragged", 0.1), ("C2", 0.1)])
def test_span_factor_gives_a_valid_decomposition(name, eta):
    """Span factor eta < 1 (Sec. 3, Table 1): pivots are taken from the qualified
    set without the exact argmax, so the pivot sequence differs from Sec. 2.
    Checked by what holds for every valid pivoted CD: all final residuals < tau;
    the residual matrix R = A - L L^T is positive semidefinite, so on any block of
    rows its diagonal is the reported residual and |R_rs| <= sqrt(R_rr R_ss);
    a pivot row vanishes in every later vector; and the rank stays close to
    exact pivoting's (greedy exact pivoting does not minimise the rank, so it
    can come out a little above or below)."""
    if name == "ragged":
        m, tau, schwarz = make_molecule(37, 6.0, (0.5,), 3, seed=77), 1e-8, 1e-12
    else:
        m, tau, schwarz = config_molecule(name), 1e-6, (0.0 if name == "C1" else 1e-12)
    d = cdlib.decompose(m.xyz, m.alpha, tau, schwarz=schwarz, sync=False, eta=eta)
    ex = cdlib.decompose(m.xyz, m.alpha, tau, schwarz=schwarz, sync=False)
    torch.cuda.synchronize()
    assert int(d.status.item()) == 0 and int(ex.status.item()) == 0
    M, Mx = d.M(), ex.M()
    assert 0.8 * Mx - 8 <= M <= 1.25 * Mx + 8
    L = d.L[:M].cpu().numpy()
    D = d.diag.cpu().numpy()
    piv = d.pivots[:M].cpu().numpy()
    assert D.max() < tau
    assert len(set(piv.tolist())) == M
    for k in range(M):
        assert L[k, piv[k]] > 0.0
        if k + 1 < M:
            assert np.abs(L[k + 1:, piv[k]]).max() <= 1e-9
    rp = d.row_pair.cpu().numpy()
    rng = np.random.default_rng(5)
    idx = np.arange(len(rp)) if len(rp) <= 800 else np.sort(rng.choice(len(rp), 400, replace=False))
    A = oracle.eri_matrix(m.xyz, m.alpha, rp[idx])
    Ls = L[:, idx]
    R = A - Ls.T @ Ls
    assert np.abs(np.diag(R) - D[idx]).max() <= 1e-10
    Dp = np.maximum(D[idx], 0.0)
    assert (np.abs(R) - np.sqrt(np.outer(Dp, Dp))).max() <= 1e-10


def test_batched_decomposition_matches_single_and_oracle():
    # 20 molecules of uneven size in one call: more than one shared launch
    mols = [make_molecule(3 + (7 * i) % 9, 3.0 + 0.4 * (i % 5), (0.3, 1.1, 4.0), 2, seed=500 + i)
            for i in range(20)]
    tau = 1e-6
    decs, ws = cdlib.allocate_many([(m.xyz, m.alpha) for m in mols], tau, 0.0)
    cdlib.run_decompose(decs, tau, 0.0, workspace=ws)
    torch.cuda.synchronize()
    for m, d in zip(mols, decs):
        M = d.M()
        check_against_oracle(m, tau, 0.0, d, M)
        single, M1 = run_gpu(m, tau, 0.0)
        assert M1 == M
        assert torch.equal(single.pivots[:M], d.pivots[:M])
        assert (single.L[:M] - d.L[:M]).abs().max().item() <= 1e-12


def test_autotune_shapes_give_the_same_decomposition():
    # the measured launch shapes change only how rows are split over
    # workgroups, not the arithmetic of any row
    mols = [make_molecule(6 + 3 * i, 5.0, (0.3, 1.1, 4.0), 2, seed=900 + i) for i in range(6)]
    tau = 1e-6
    pairs = [(m.xyz, m.alpha) for m in mols]
    ref, rws = cdlib.allocate_many(pairs, tau, 1e-12)
    cdlib.run_decompose(ref, tau, 1e-12, workspace=rws)
    decs, ws = cdlib.allocate_many(pairs, tau, 1e-12)
    t = cdlib.autotune(decs, tau, 1e-12, workspace=ws)
    assert 2 <= t.step2_row_tiles <= 7 and t.step1_min_rows in (16, 32, 48, 64)
    assert t.step1_q in (32, 48, 64)
    torch.cuda.synchronize()
    for d, r in zip(decs, ref):
        assert d.M() == r.M() and int(d.status.item()) == 0
        assert torch.equal(d.pivots[:d.M()], r.pivots[:r.M()])
        assert (d.L[:d.M()] - r.L[:r.M()]).abs().max().item() <= 1e-12
    # explicit shapes at the ends of both ranges
    for shape in [cdlib.cd_tuning(2, 16, 8), cdlib.cd_tuning(7, 64, 64)]:
        cdlib.run_decompose(decs, tau, 1e-12, workspace=ws, tuning=shape)
        torch.cuda.synchronize()
        for d, r in zip(decs, ref):
            assert torch.equal(d.pivots[:d.M()], r.pivots[:r.M()])
            assert (d.L[:d.M()] - r.L[:r.M()]).abs().max().item() <= 1e-12
    # the same shapes again: the kept result, no new measurement
    t2 = cdlib.autotune(decs, tau, 1e-12, workspace=ws)
    assert (t2.step2_row_tiles, t2.step1_min_rows, t2.step1_q) == (
        t.step2_row_tiles, t.step1_min_rows, t.step1_q)
    torch.cuda.synchronize()
    for d, r in zip(decs, ref):
        assert torch.equal(d.pivots[:d.M()], r.pivots[:r.M()])


@pytest.mark.parametrize("prec,lmo", [("fp64", False), ("fp64", True), ("fp32", False),
                                      ("fp32", True), ("bf16x3", False), ("bf16x3", True)])
def test_batched_jk_matches_single(prec, lmo):
    """Several problems in one call (on the library's two streams) give the
    single-problem results bit for bit, with and without the MO output, and
    the oracle's J/K from the oracle's vectors within the precision's bar."""
    mols = [make_molecule(4 + i, 4.0, (0.3, 1.1, 4.0), 3, seed=700 + i) for i in range(5)]
    decs, ws = cdlib.allocate_many([(m.xyz, m.alpha) for m in mols], 1e-6, 1e-12)
    cdlib.run_decompose(decs, 1e-6, 1e-12, workspace=ws)
    jks, jws = cdlib.prepare_jk_many(decs, [m.C for m in mols], prec, lmo=lmo)
    cdlib.run_jk_many(jks, jws, prec)
    torch.cuda.synchronize()
    for m, d, jk in zip(mols, decs, jks):
        J, K = cdlib.build_jk(d, m.C, prec)
        assert torch.equal(J, jk.J) and torch.equal(K, jk.K)
        if lmo:
            M = d.M()
            assert torch.equal(jk.Lmo[:M], cdlib.transform(d, m.C, m.C)[:M])
        rp, ref = check_against_oracle(m, 1e-6, 1e-12, d, d.M())
        Jr, Kr = oracle.jk_cd(m.n_basis, rp, ref.L, m.C)
        Jg, Kg = jk.J.cpu().numpy(), jk.K.cpu().numpy()
        assert np.abs(Jg - Jr).max() <= TOL_JK
        assert np.abs(Kg - Kr).max() <= (TOL_JK if prec == "fp64" else TOL_K[prec])
        e2r = oracle.e2(m.C, Jr, Kr)
        assert abs(gpu_e2(m.C, Jg, Kg) - e2r) <= (1e-10 if prec == "fp64" else TOL_E2[prec])


def test_batched_c4_sizes_against_oracle():
    """Molecules of the 64-molecule batch (52..400 functions, tau = 1e-5): the
    four largest and the two smallest in one call.  Their pivot-selection
    workgroups (one per 32 active rows) exceed the co-resident capacity of one
    cooperative launch, so the call scales every problem's share down; each
    problem's decomposition is held to the oracle, and its FP32 and FP64 J/K
    (batched) to the oracle's J/K."""
    from paper_2609_00306_amd.inputs import BATCH_C4, batch_c4
    allm = batch_c4()
    order = sorted(range(len(allm)), key=lambda i: allm[i].n_basis)
    mols = [allm[i] for i in order[-4:] + order[:2]]
    tau, schwarz = BATCH_C4["tau"], BATCH_C4["schwarz"]
    decs, ws = cdlib.allocate_many([(m.xyz, m.alpha) for m in mols], tau, schwarz)
    n_cu = torch.cuda.get_device_properties(0).multi_processor_count
    assert sum(min(n_cu, -(-d.n_active // 32)) for d in decs) > n_cu   # the scaling branch
    cdlib.run_decompose(decs, tau, schwarz, workspace=ws)
    torch.cuda.synchronize()
    refs = []
    for m, d in zip(mols, decs):
        refs.append(check_against_oracle(m, tau, schwarz, d, d.M()))
    for prec in ("fp32", "fp64"):
        jks, jws = cdlib.prepare_jk_many(decs, [m.C for m in mols], prec)
        cdlib.run_jk_many(jks, jws, prec)
        torch.cuda.synchronize()
        for m, jk, (rp, ref) in zip(mols, jks, refs):
            Jr, Kr = oracle.jk_cd(m.n_basis, rp, ref.L, m.C)
            Jg, Kg = jk.J.cpu().numpy(), jk.K.cpu().numpy()
            assert np.abs(Jg - Jr).max() <= TOL_JK
            assert np.abs(Kg - Kr).max() <= (TOL_JK if prec == "fp64" else TOL_K[prec])
            assert abs(gpu_e2(m.C, Jg, Kg) - oracle.e2(m.C, Jr, Kr)) <= TOL_E2["fp32"]


@pytest.mark.parametrize("name,tau1,tau2", [("C1", 1e-3, 1e-6), ("C2", 1e-4, 1e-6)])
def test_resume_continues_to_a_smaller_tau(name, tau1, tau2):
    """CD_RESUME: a decomposition stopped at tau1 continued to tau2 (the Sec. 2
    pivot order does not depend on tau; Table 5: more vectors as tau falls).
    The first M1 vectors and pivot values stay bit for bit; the whole pivot
    sequence equals a direct run at tau2; the vectors, pivot values and
    residuals agree with it to TOL_L, and the result passes the oracle check."""
    m = config_molecule(name)
    schwarz = 0.0 if name == "C1" else 1e-12
    d = cdlib.decompose(m.xyz, m.alpha, tau1, schwarz=schwarz)
    M1 = d.M()
    L1 = d.L[:M1].clone()
    pv1 = d.pivot_values[:M1].clone()
    piv1 = d.pivots[:M1].clone()
    cdlib.resume(d, tau2, schwarz)
    direct = cdlib.decompose(m.xyz, m.alpha, tau2, schwarz=schwarz)
    M2 = d.M()
    assert int(d.status.item()) == 0 and M2 == direct.M() and M2 > M1
    assert torch.equal(d.L[:M1], L1)
    assert torch.equal(d.pivot_values[:M1], pv1) and torch.equal(d.pivots[:M1], piv1)
    assert torch.equal(d.pivots[:M2], direct.pivots[:M2])
    assert (d.L[:M2] - direct.L[:M2]).abs().max().item() <= TOL_L
    assert (d.pivot_values[:M2] - direct.pivot_values[:M2]).abs().max().item() <= TOL_L
    assert (d.diag - direct.diag).abs().max().item() <= TOL_L
    check_against_oracle(m, tau2, schwarz, d, M2)


def test_resume_after_capacity_and_invalid_state():
    """A decomposition that hit its capacity continues once a larger L is given
    (equal to a direct run); a stored state that cannot be continued (status
    CD_ERR_DEVICE) is refused with CD_ERR_INVALID_ARG and leaves the outputs."""
    m = config_molecule("C1")
    d = cdlib.decompose(m.xyz, m.alpha, 1e-6, schwarz=0.0, max_vectors=50, sync=False)
    torch.cuda.synchronize()
    assert int(d.status.item()) == cdlib.CD_ERR_CAPACITY and d.M() == 50
    cdlib.resume(d, 1e-6, 0.0)
    direct = cdlib.decompose(m.xyz, m.alpha, 1e-6, schwarz=0.0)
    M = d.M()
    assert int(d.status.item()) == 0 and M == direct.M() == 235
    assert torch.equal(d.pivots[:M], direct.pivots[:M])
    assert (d.L[:M] - direct.L[:M]).abs().max().item() <= TOL_L
    L0, diag0 = d.L[:M].clone(), d.diag.clone()
    d.status.fill_(cdlib.CD_ERR_DEVICE)
    cdlib.resume(d, 1e-8, 0.0, sync=False)
    torch.cuda.synchronize()
    assert int(d.status.item()) == cdlib.CD_ERR_INVALID_ARG and d.M() == M
    assert torch.equal(d.L[:M], L0) and torch.equal(d.diag, diag0)


def test_poisoned_diagonal_reports_not_psd():
    """CD_DEBUG_POISON_DIAG: a NaN initial residual must end the decomposition
    with CD_ERR_NOT_PSD in the status word (Sec. 2 needs a positive
    semidefinite matrix), in one problem and in a batched call, and CD_SYNC
    folds it into the return value."""
    m = config_molecule("C1")
    d = cdlib.allocate(m.xyz, m.alpha, 1e-6, 0.0)
    cdlib.run_decompose([d], 1e-6, 0.0, poison=True)
    torch.cuda.synchronize()
    assert int(d.status.item()) == cdlib.CD_ERR_NOT_PSD and d.M() == 0
    with pytest.raises(cdlib.CDError) as e:
        cdlib.run_decompose([d], 1e-6, 0.0, poison=True, sync=True)
    assert e.value.status == cdlib.CD_ERR_NOT_PSD
    mols = [make_molecule(5 + i, 4.0, (0.3, 1.1, 4.0), 2, seed=810 + i) for i in range(3)]
    decs, ws = cdlib.allocate_many([(x.xyz, x.alpha) for x in mols], 1e-6, 1e-12)
    cdlib.run_decompose(decs, 1e-6, 1e-12, workspace=ws, poison=True)
    torch.cuda.synchronize()
    assert all(int(x.status.item()) == cdlib.CD_ERR_NOT_PSD for x in decs)
    # the same buffers decompose normally afterwards
    cdlib.run_decompose([d], 1e-6, 0.0)
    torch.cuda.synchronize()
    check_against_oracle(m, 1e-6, 0.0, d, d.M())


@pytest.mark.parametrize("name", ["C5"])
def test_large_workload_properties(name):
    """At the 1200-function size the full oracle run is too slow for a test;
    check what holds at any size (Sec. 2): every final residual < tau, the
    reconstruction error of sampled integrals <= tau (Cauchy-Schwarz), and
    each vector vanishing at earlier pivot rows; sampled rows against the
    oracle's exact integrals."""
    m = config_molecule(name)
    tau = 1e-6
    d, M = run_gpu(m, tau, 1e-12)
    assert int(d.status.item()) == 0 and M > 0
    rp, _ = oracle.rows(m.xyz, m.alpha, 1e-12)
    assert np.array_equal(rp, d.row_pair.cpu().numpy())
    diag = d.diag.cpu().numpy()
    assert diag.max() < tau and diag.min() >= -1e-12
    L = d.L[:M].cpu().numpy()
    piv = d.pivots[:M].cpu().numpy()
    assert len(np.unique(piv)) == M
    rng = np.random.default_rng(12)
    rows = rng.integers(0, d.n_rows, 64)
    cols = np.concatenate([rng.integers(0, d.n_rows, 32), piv[rng.integers(0, M, 32)]])
    for r in rows[:16]:
        for c in cols:
            mu, nu = oracle.unpack_pair(int(rp[r]))
            sg, rh = oracle.unpack_pair(int(rp[c]))
            a = oracle.eri(m.xyz, m.alpha, mu, nu, sg, rh)
            assert abs(a - float(L[:, r] @ L[:, c])) <= tau
    for K in rng.integers(1, M, 50):
        assert np.abs(L[K, piv[:K]]).max() <= 1e-9
    # the pivot values L^K at its own pivot row squared are non-increasing
    dk = np.array([L[K, piv[K]] ** 2 for K in range(M)])
    assert np.all(np.diff(dk) <= 1e-9 * dk[:-1])
    # row-sampled replay of the all-row solve (Sec. 3, Eq. CVsLT): with B the
    # pivot rows, the vectors of any row r solve  L_B x = A(B, r), L_B[K][J] =
    # L^J at P_K (lower triangular); A from the oracle's integrals
    from scipy.linalg import solve_triangular
    sel = rng.integers(0, d.n_rows, 12)
    A = oracle.eri_matrix(m.xyz, m.alpha, np.concatenate([rp[piv], rp[sel]]))
    LB = np.ascontiguousarray(L[:, piv].T)
    X = solve_triangular(LB, A[:M, M:], lower=True)
    assert np.abs(X - L[:, sel]).max() <= 1e-9


def test_unscreened_large_workload():
    """The 1200-function molecule with no screening: all 720 600 pairs are rows
    and L holds 32 GB.  The rows screened out at 1e-12 have D1 far below tau,
    so the active rows, the pivots and every kept row's arithmetic are those of
    the screened run: pivots, pivot values and the vectors of the rows both runs
    share agree bit for bit.  The extra rows obey what holds at any size
    (Sec. 2): final residual < tau, |A - L L^T| <= tau on sampled entries, and
    the row-sampled replay of Eq. CVsLT with the oracle's integrals."""
    from scipy.linalg import solve_triangular
    m = config_molecule("C5")
    tau = 1e-6
    ref, Mr = run_gpu(m, tau, 1e-12)
    d = cdlib.allocate(m.xyz, m.alpha, tau, 0.0, max_vectors=Mr + 8)
    assert d.n_rows == 720600 and d.n_active == ref.n_active
    cdlib.run_decompose([d], tau, 0.0)
    torch.cuda.synchronize()
    M = d.M()
    assert int(d.status.item()) == 0 and M == Mr
    rp_s = ref.row_pair
    pos = torch.searchsorted(d.row_pair, rp_s)
    assert torch.equal(d.row_pair[pos], rp_s)
    piv_u = d.row_pair[d.pivots[:M]]
    assert torch.equal(piv_u, rp_s[ref.pivots[:M]])
    assert torch.equal(d.pivot_values[:M], ref.pivot_values[:M])
    for k0 in range(0, M, 512):   # vectors of the shared rows, in slabs (bit for bit)
        k1 = min(M, k0 + 512)
        assert torch.equal(d.L[k0:k1].index_select(1, pos), ref.L[k0:k1])
    assert torch.equal(d.diag[pos], ref.diag)
    assert float(d.diag.max()) < tau and float(d.diag.min()) >= -1e-12
    # the rows only the unscreened run has
    extra = torch.ones(d.n_rows, dtype=torch.bool, device=d.L.device)
    extra[pos] = False
    ex = torch.nonzero(extra).flatten()
    assert ex.numel() == 720600 - ref.n_rows
    rng = np.random.default_rng(31)
    sel = torch.as_tensor(np.sort(rng.choice(ex.numel(), 12, replace=False)), device=ex.device)
    rows = ex[sel]
    rp = d.row_pair.cpu().numpy()
    piv = d.pivots[:M].cpu().numpy()
    Lsel = d.L[:M].index_select(1, rows).cpu().numpy()
    LB = d.L[:M].index_select(1, d.pivots[:M]).cpu().numpy().T.copy()
    r_np = rows.cpu().numpy()
    A = oracle.eri_matrix(m.xyz, m.alpha, np.concatenate([rp[piv], rp[r_np]]))
    X = solve_triangular(LB, A[:M, M:], lower=True)
    assert np.abs(X - Lsel).max() <= 1e-9
    Aext = A[M:, M:]
    assert np.abs(Aext - Lsel.T @ Lsel).max() <= tau
    assert np.abs(np.diag(Aext) - (Lsel ** 2).sum(0) - d.diag[rows].cpu().numpy()).max() <= 1e-12


def test_active_rows_beyond_the_selection_capacity_are_refused():
    """The pivot selection holds at most 256 active rows per workgroup and 256
    workgroups (65 536 rows); beyond that cd_decompose refuses on the host with
    CD_ERR_UNSUPPORTED before any device work: the 400-function molecule with
    no screening at tau = 0 has all 80 200 rows active."""
    m = config_molecule("C2")
    d = cdlib.allocate(m.xyz, m.alpha, 0.0, 0.0, max_vectors=16)
    assert d.n_active == 80200
    st0 = d.status.clone()
    with pytest.raises(cdlib.CDError) as e:
        cdlib.run_decompose([d], 0.0, 0.0)
    assert e.value.status == cdlib.CD_ERR_UNSUPPORTED
    assert b"capacity" in cdlib.load().cd_last_error()
    torch.cuda.synchronize()
    assert torch.equal(d.status, st0)


# Second-order energy from transformed vectors (CD-based MP2, Secs. 5 and 7).
# Both sides add the same terms in different orders (FP64 matrix-core
# products over P, tile-wise sums over a, b): with |terms| summed in S, the
# rounding difference is below (M + V^2) * 2^-52 * S; 1e-10 relative to the
# largest magnitude covers it for every shape here.
TOL_MP2 = 1e-10


def _mp2_gpu(B, M, eo, ev, dev, pad_rows=0):
    """GPU energy and pairs for B [M][O][V], padded with NaN rows the kernels
    must not read."""
    M0, O, V = B.shape
    Bd = torch.full((M0 + pad_rows, O, V), float("nan"), dtype=torch.float64, device=dev)
    Bd[:M0] = torch.from_numpy(B).to(dev)
    nv = torch.tensor([M], dtype=torch.int64, device=dev)
    E, pe = cdlib.mp2_energy(Bd, nv, eo, ev, pair_energy=True)
    return float(E.item()), pe.cpu().numpy()


@pytest.mark.parametrize("M,O,V", [(37, 5, 50), (70, 9, 130), (64, 1, 64), (200, 12, 200),
                                   (50, 4, 100), (33, 3, 40), (90, 6, 180),
                                   (5, 3, 1), (0, 4, 70), (16, 0, 40), (16, 3, 0)])
def test_mp2_parity(gpu, M, O, V):
    """Several virtual tiles with a ragged tail (last tile with 2, 8, 36, 40,
    50 and 52 virtuals: 1, 3 and 4 row tiles), one exact tile, a single
    virtual, and the empty cases (no vectors: E = 0; no occupied or no
    virtual orbitals: E = 0)."""
    from paper_2609_00306_amd.inputs import random_mo_vectors
    B = random_mo_vectors(M, O, V, seed=100 + M + O + V)
    rng = np.random.default_rng(M * 7 + O)
    eo = np.sort(rng.uniform(-1.5, -0.3, O))
    ev = np.sort(rng.uniform(0.2, 2.5, V))
    E, pe = _mp2_gpu(B, M, eo, ev, gpu, pad_rows=3)
    Er, per = oracle.mp2(B, eo, ev)
    scale = max(1e-300, np.abs(per).max() if per.size else 0.0)
    assert abs(E - Er) <= TOL_MP2 * max(abs(Er), scale)
    assert pe.shape == (O, O)
    if O > 0:
        assert np.abs(pe - per).max() <= TOL_MP2 * scale
        assert np.array_equal(pe, pe.T)
    if M == 0 or O == 0 or V == 0:
        assert E == 0.0


def test_mp2_chain_c1(gpu):
    """Decomposition, transform with the occupied and virtual orbitals, and
    the energy, all on the GPU, against the same chain in the oracle.  The
    vectors agree to 1e-10 absolute, so the integrals (ia|jb) agree to about
    2 M 1e-10 max|B|; 1e-7 relative on E covers that bound."""
    from paper_2609_00306_amd.inputs import mp2_orbitals
    m = config_molecule("C1")
    d, M = run_gpu(m, 1e-6, 0.0)
    rp, ref = check_against_oracle(m, 1e-6, 0.0, d, M)
    Co, Cv, eo, ev = mp2_orbitals(m)
    Bg = cdlib.transform(d, Co, Cv)
    E = float(cdlib.mp2_energy(Bg, d.n_vectors, eo, ev).item())
    Br = oracle.transform(m.n_basis, rp, ref.L, Co, Cv)
    Er, _ = oracle.mp2(Br, eo, ev)
    assert Er < 0.0
    assert abs(E - Er) <= 1e-7 * abs(Er)


def test_mp2_c2_shape_sampled_pairs(gpu):
    """The 400-function workload's shape at tau = 1e-6 (M = 1930 vectors,
    O = 50, V = 350): sampled pair energies against the oracle's pair by
    pair, and E against the sum of the GPU's own pairs."""
    from paper_2609_00306_amd.inputs import random_mo_vectors
    M, O, V = 1930, 50, 350
    B = random_mo_vectors(M, O, V, seed=2)
    rng = np.random.default_rng(22)
    eo = np.sort(rng.uniform(-1.5, -0.3, O))
    ev = np.sort(rng.uniform(0.2, 2.5, V))
    E, pe = _mp2_gpu(B, M, eo, ev, gpu)
    for i, j in [(0, 0), (O - 1, O - 1), (0, O - 1), (17, 33), (25, 26)]:
        r = oracle.mp2_pair(B, eo, ev, i, j)
        assert abs(pe[i, j] - r) <= TOL_MP2 * abs(r)
        assert pe[j, i] == pe[i, j]
    iu = np.triu_indices(O, 1)
    s = np.trace(pe) + 2.0 * pe[iu].sum()
    assert abs(E - s) <= 1e-12 * abs(s)


def test_mp2_rejects_bad_vector_count(gpu):
    """A vector count above the buffer's capacity is reported through the
    status word (the kernels then read no vectors)."""
    B = torch.zeros((4, 2, 3), dtype=torch.float64, device=gpu)
    nv = torch.tensor([5], dtype=torch.int64, device=gpu)
    with pytest.raises(cdlib.CDError) as e:
        cdlib.mp2_energy(B, nv, [-1.0, -0.5], [0.5, 1.0, 2.0])
    assert e.value.status == cdlib.CD_ERR_INVALID_ARG


# Restricted candidates (Sec. 6.2): the Cholesky basis from the rows of two
# flagged functions only (stand-in for the LL,LL block: the functions of the
# flagged exponents); every row still gets its vectors and final residual.
@pytest.mark.parametrize("name,schwarz,flagged", [("C1", 0.0, (0, 1)), ("C1", 0.0, (1, 2)),
                                                  ("C2", 1e-12, (0, 1, 2))])
def test_restricted_candidates_parity(name, schwarz, flagged):
    from paper_2609_00306_amd.inputs import exponent_block
    m = config_molecule(name)
    fn = exponent_block(m, flagged)
    tau = 1e-6
    d = cdlib.decompose(m.xyz, m.alpha, tau, schwarz=schwarz, pivot_fn=fn, sync=False)
    torch.cuda.synchronize()
    M = d.M()
    rp, ref = check_against_oracle(m, tau, schwarz, d, M, pivot_fn=fn)
    cand = oracle.candidate_rows(rp, fn).astype(bool)
    D1 = oracle.diagonal_all(m.xyz, m.alpha)[rp]
    assert d.n_active == int(np.count_nonzero(cand & (D1 >= tau)))
    piv = d.pivots[:M].cpu().numpy()
    assert cand[piv].all()
    diag = d.diag.cpu().numpy()
    assert diag[cand].max() < tau
    assert diag[~cand].max() > tau        # the restriction leaves large residuals elsewhere


def test_restricted_candidates_edge_flags():
    """All functions flagged: the unrestricted decomposition, bit for bit.
    None flagged: no active rows, no vectors, the residual is the diagonal."""
    m = make_molecule(37, 6.0, (0.5, 2.0), 3, seed=78)
    tau = 1e-8
    d0, M0 = run_gpu(m, tau, 1e-12)
    d1 = cdlib.decompose(m.xyz, m.alpha, tau, schwarz=1e-12,
                         pivot_fn=np.ones(m.n_basis, np.uint8))
    assert d1.M() == M0 and torch.equal(d1.pivots[:M0], d0.pivots[:M0])
    assert torch.equal(d1.L[:M0], d0.L[:M0]) and torch.equal(d1.diag, d0.diag)
    dz = cdlib.decompose(m.xyz, m.alpha, tau, schwarz=1e-12,
                         pivot_fn=np.zeros(m.n_basis, np.uint8), max_vectors=4)
    assert dz.n_active == 0 and dz.M() == 0 and int(dz.status.item()) == 0
    check_against_oracle(m, tau, 1e-12, dz, 0, pivot_fn=np.zeros(m.n_basis, np.uint8))


# SCF on Cholesky J/K (Sec. 4.1).  Both sides take the same steps (core guess,
# then F_k = H + 2J - K, E_k = tr(D_k (H + F_k)) + charge repulsion, D_(k+1)
# the projector on the O lowest levels of F_k); the GPU reaches the projector
# by purification, the oracle by diagonalisation.  J and K agree to 1e-10
# elementwise, so each E_k agrees to about 3e-10 sum|D|; the projectors agree
# to the purification's idempotency tolerance.
def _scf_case(m, tau, schwarz, prec="fp64", e_tol=1e-10, d_tol=1e-8, diis=8):
    from paper_2609_00306_amd.inputs import scf_charges
    cx, Z = scf_charges(m)
    d, M = run_gpu(m, tau, schwarz)
    S, H = cdlib.one_electron(m.xyz, m.alpha, cx, Z)
    e_ch = oracle.charge_repulsion(cx, Z)
    res = cdlib.scf(d, S, H, m.n_occ, e_ch, prec=prec, e_tol=e_tol, d_tol=d_tol, diis=diis)
    return d, M, cx, Z, S, H, e_ch, res


def test_one_electron_parity():
    from paper_2609_00306_amd.inputs import scf_charges
    for m in (config_molecule("C1"), make_molecule(13, 5.0, (0.3, 1.2, 6.0), 6, seed=31)):
        cx, Z = scf_charges(m)
        S, H = cdlib.one_electron(m.xyz, m.alpha, cx, Z)
        Sr, Tr, Vr = oracle.one_electron(m.xyz, m.alpha, cx, Z)
        Hr = Tr + Vr
        assert np.abs(S.cpu().numpy() - Sr).max() <= 1e-14 * np.abs(Sr).max()
        assert np.abs(H.cpu().numpy() - Hr).max() <= 1e-13 * np.abs(Hr).max()


@pytest.mark.parametrize("case,diis", [("C1", 8), ("C1", 0), ("ragged", 8)])
def test_scf_parity(case, diis):
    if case == "C1":
        m, tau, schwarz = config_molecule("C1"), 1e-6, 0.0
    else:
        m, tau, schwarz = make_molecule(13, 5.0, (0.3, 1.2, 6.0), 6, seed=31), 1e-7, 1e-12
    d, M, cx, Z, S, H, e_ch, res = _scf_case(m, tau, schwarz, diis=diis)
    rp, ref = check_against_oracle(m, tau, schwarz, d, M)
    Sr, Tr, Vr = oracle.one_electron(m.xyz, m.alpha, cx, Z)
    exp = oracle.scf(Sr, Tr + Vr, e_ch, m.n_occ,
                     lambda C: oracle.jk_cd(m.n_basis, rp, ref.L, C), diis=diis)
    assert res.converged and exp.converged
    E = res.energies.cpu().numpy()
    assert len(E) == len(exp.energies)
    tol = 3e-10 * np.abs(exp.D).sum() + 1e-12 * abs(exp.energies[-1])
    assert np.abs(E - exp.energies).max() <= tol
    D = res.D.cpu().numpy()
    assert np.abs(D - exp.D).max() <= 1e-8
    C = res.C.cpu().numpy()
    assert np.abs(C @ C.T - D).max() <= 1e-12
    # converged-SCF invariants on the GPU's own result
    Sn = S.cpu().numpy()
    assert np.trace(D @ Sn) == pytest.approx(m.n_occ, abs=1e-9)
    F = res.F.cpu().numpy()
    assert np.abs(F @ D @ Sn - Sn @ D @ F).max() < 1e-8


def test_scf_c2_converges_with_valid_density():
    """The 400-function workload (50 charge-2 sites, 50 ghost centres): the
    oracle's SCF takes minutes here, so the converged result is checked for
    what holds at any size (idempotency in the S metric, electron count,
    Brillouin condition, D = C C^T)."""
    m = config_molecule("C2")
    d, M, cx, Z, S, H, e_ch, res = _scf_case(m, 1e-6, 1e-12)
    assert res.converged and len(res.energies) <= 40
    Sn = S.cpu().numpy()
    D = res.D.cpu().numpy()
    F = res.F.cpu().numpy()
    C = res.C.cpu().numpy()
    assert np.abs(D @ Sn @ D - D).max() < 1e-9
    assert np.trace(D @ Sn) == pytest.approx(m.n_occ, abs=1e-9)
    assert np.abs(F @ D @ Sn - Sn @ D @ F).max() < 1e-8
    assert np.abs(C @ C.T - D).max() < 1e-12


def test_scf_reduced_precision_energy_error():
    """FP32 and 3xBF16 K in the SCF: the converged energy moves by at most
    1e-5 Eh from the FP64 one (the J/K energy bar).  The energy change per
    iteration and the commutator cannot fall below what the K rounding leaves
    (about 1e-7 here), so both tolerances are 1e-6."""
    m = config_molecule("C1")
    base = _scf_case(m, 1e-6, 0.0)[-1]
    for prec in ("fp32", "bf16x3"):
        r = _scf_case(m, 1e-6, 0.0, prec, e_tol=1e-6, d_tol=1e-6)[-1]
        assert r.converged
        assert abs(float(r.energies[-1]) - float(base.energies[-1])) <= 1e-5


def test_scf_rejects_a_singular_overlap():
    """Two identical functions make S singular: the orthogonaliser does not
    converge and the call says so (no vectors of the SCF are touched)."""
    m = make_molecule(5, 4.0, (0.5, 2.0), 2, seed=41)
    xyz = np.concatenate([m.xyz, m.xyz[:1]])
    alpha = np.concatenate([m.alpha, m.alpha[:1]])
    d = cdlib.decompose(xyz, alpha, 1e-8, schwarz=1e-12)
    S, H = cdlib.one_electron(xyz, alpha, m.xyz[:2], [2.0, 2.0])
    with pytest.raises(cdlib.CDError) as e:
        cdlib.scf(d, S, H, 2, 0.0, max_iter=5)
    assert e.value.status == cdlib.CD_ERR_NOT_PSD


# Hermitian decomposition (Sec. 7) on the seeded stand-in for finite-field
# integrals.  The pivot sequences must be equal; rounding in a residual is
# divided by sqrt(d_K) in vector K, so vectors are compared as L_K sqrt(d_K)
# (1e-13 of max|A|), residual diagonals to 1e-12 of max|A|.
def _zcheck(A, tau, max_vectors=None, expect_status=0):
    Ad = torch.from_numpy(A).to("cuda")
    z = cdlib.zdecompose(Ad, tau, max_vectors=max_vectors, sync=False)
    torch.cuda.synchronize()
    assert int(z.status.item()) == expect_status
    M = z.M()
    ref = oracle.zdecompose(A, tau, max_vectors=max_vectors)
    assert M == ref.M
    piv = z.pivots[:M].cpu().numpy()
    assert np.array_equal(piv, ref.pivots)
    L = z.L[:M].cpu().numpy()
    amax = np.abs(A).max()
    if M:
        dk = np.array([ref.L[K, ref.pivots[K]].real for K in range(M)])
        assert (np.abs(L - ref.L) * dk[:, None]).max() <= 1e-13 * amax
    assert np.abs(z.diag.cpu().numpy()[:A.shape[0]] - ref.D).max() <= 1e-12 * amax
    return z, ref


@pytest.mark.parametrize("n,q,tau,field", [(300, 250, 1e-6, 0.5), (1200, 900, 1e-8, 0.5),
                                           (777, 500, 1e-6, 0.0), (64, 80, 0.0, 0.3)])
def test_zdecompose_parity(n, q, tau, field):
    from paper_2609_00306_amd.inputs import hermitian_gram
    A = hermitian_gram(n, q, seed=n + q, field=field)
    z, ref = _zcheck(A, tau)
    assert ref.rc == 0


def test_zdecompose_capacity_and_single_row():
    from paper_2609_00306_amd.inputs import hermitian_gram
    A = hermitian_gram(500, 400, seed=21)
    _zcheck(A, 1e-8, max_vectors=50, expect_status=cdlib.CD_ERR_CAPACITY)
    one = np.array([[2.25 + 0.0j]])
    z = cdlib.zdecompose(torch.from_numpy(one).to("cuda"), 1e-6)
    assert z.M() == 1 and z.L[0, 0].item() == 1.5 + 0.0j


def test_zdecompose_large_properties():
    """4096 rows (the measured size): every final residual < tau, sampled
    entries of A - sum L L^H within tau, pivot rows vanishing in later
    vectors, distinct pivots."""
    from paper_2609_00306_amd.inputs import hermitian_gram
    A = hermitian_gram(4096, 2048, seed=5)
    tau = 1e-6
    z = cdlib.zdecompose(torch.from_numpy(A).to("cuda"), tau)
    M = z.M()
    assert int(z.status.item()) == 0 and M > 500
    assert float(z.diag.max()) < tau
    L = z.L[:M].cpu().numpy()
    piv = z.pivots[:M].cpu().numpy()
    assert len(np.unique(piv)) == M
    rng = np.random.default_rng(4)
    rows, cols = rng.integers(0, 4096, 200), rng.integers(0, 4096, 200)
    rec = np.einsum("kr,kr->r", L[:, rows], L[:, cols].conj())
    assert np.abs(A[rows, cols] - rec).max() <= tau
    for K in rng.integers(1, M, 40):
        assert np.abs(L[K, piv[:K]]).max() <= 1e-9



def test_scf_energy_from_span_factor_vectors():
    """The span-factor decomposition (eta = 0.1) is a different but valid
    Cholesky basis: the SCF on its J/K lands within the decomposition error
    (order tau) of the SCF on the exact-pivoting vectors."""
    from paper_2609_00306_amd.inputs import scf_charges
    m = config_molecule("C2")
    tau = 1e-6
    cx, Z = scf_charges(m)
    S, H = cdlib.one_electron(m.xyz, m.alpha, cx, Z)
    e_ch = oracle.charge_repulsion(cx, Z)
    E = []
    for eta in (1.0, 0.1):
        d = cdlib.decompose(m.xyz, m.alpha, tau, schwarz=1e-12, eta=eta)
        r = cdlib.scf(d, S, H, m.n_occ, e_ch)
        assert r.converged
        E.append(float(r.energies[-1]))
    assert abs(E[0] - E[1]) <= 50 * tau


def test_mp2_on_restricted_candidate_vectors():
    """The energy kernels take any vectors: on a restricted-candidate
    decomposition of C1 the GPU chain (transform, energy) equals the oracle's
    chain on the oracle's restricted decomposition."""
    from paper_2609_00306_amd.inputs import exponent_block, mp2_orbitals
    m = config_molecule("C1")
    fn = exponent_block(m, (0, 1))
    d = cdlib.decompose(m.xyz, m.alpha, 1e-6, schwarz=0.0, pivot_fn=fn)
    M = d.M()
    rp, ref = check_against_oracle(m, 1e-6, 0.0, d, M, pivot_fn=fn)
    Co, Cv, eo, ev = mp2_orbitals(m)
    E = float(cdlib.mp2_energy(cdlib.transform(d, Co, Cv), d.n_vectors, eo, ev).item())
    Er, _ = oracle.mp2(oracle.transform(m.n_basis, rp, ref.L, Co, Cv), eo, ev)
    assert abs(E - Er) <= 1e-7 * abs(Er)


def test_graph_replay_of_batched_step_matches_eager():
    """The batched step (decomposition of six molecules + FP64 J/K of all of
    them, with the library's side streams) captured in a graph: every replay,
    with eager work and synchronisation in between and the outputs poisoned
    before it, reproduces the eager results bit for bit."""
    from paper_2609_00306_amd.inputs import BATCH_C4, batch_c4
    mols = batch_c4(count=6)
    tau, schwarz = BATCH_C4["tau"], BATCH_C4["schwarz"]
    pairs = [(m.xyz, m.alpha) for m in mols]
    decs, ws = cdlib.allocate_many(pairs, tau, schwarz, device="cuda")
    jks, jws = cdlib.prepare_jk_many(decs, [m.C for m in mols], "fp64")

    def step():
        cdlib.run_decompose(decs, tau, schwarz, workspace=ws)
        cdlib.run_jk_many(jks, jws, "fp64")

    step()
    torch.cuda.synchronize()
    ref = [(d.M(), d.pivots[:d.M()].clone(), d.L[:d.M()].clone(), j.J.clone(), j.K.clone())
           for d, j in zip(decs, jks)]
    assert all(int(d.status.item()) == 0 for d in decs)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        step()
    torch.cuda.current_stream().wait_stream(side)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        step()
    for rep in range(3):
        for d, j in zip(decs, jks):            # eager work between replays
            d.L.fill_(float("nan"))
            d.pivots.fill_(-1)
            j.J.fill_(float("nan"))
            j.K.fill_(float("nan"))
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for (M, piv, L, J, K), d, j in zip(ref, decs, jks):
            assert d.M() == M and int(d.status.item()) == 0
            assert torch.equal(d.pivots[:M], piv)
            assert torch.equal(d.L[:M], L)
            assert torch.equal(j.J, J) and torch.equal(j.K, K)
