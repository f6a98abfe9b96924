"""cd_decompose_noalloc (the allocation-free decomposition on the library's
static device scratch) against cd_decompose through the C ABI: bit for bit
on two calls in a row, the second with a smaller input, then a batch; inputs
beyond the scratch are refused on the host."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from paper_2609_00306_amd import cdlib  # noqa: E402
from paper_2609_00306_amd.inputs import config_molecule, make_molecule  # noqa: E402


@pytest.fixture(scope="module", autouse=True)
def gpu():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    cdlib.load()
    return torch.device("cuda:0")


def _same(a, b):
    M = a.M()
    assert M == b.M() and int(a.status.item()) == int(b.status.item()) == 0
    assert torch.equal(a.row_pair, b.row_pair)
    assert torch.equal(a.pivots[:M], b.pivots[:M])
    assert torch.equal(a.pivot_values[:M], b.pivot_values[:M])
    assert torch.equal(a.L[:M], b.L[:M])
    assert torch.equal(a.diag, b.diag)


def _pair(m, tau, schwarz, max_vectors=None):
    ref = cdlib.allocate(m.xyz, m.alpha, tau, schwarz, max_vectors)
    out = cdlib.allocate(m.xyz, m.alpha, tau, schwarz, ref.max_vectors)
    out.workspace = torch.empty(0, dtype=torch.uint8, device=ref.L.device)  # not used
    return ref, out


def test_noalloc_matches_cd_decompose_twice_then_smaller():
    # first call: the 400-function workload, capacity 2000 vectors (about 90 MB of scratch)
    m2 = config_molecule("C2")
    ref, out = _pair(m2, 1e-6, 1e-12, max_vectors=2000)
    cdlib.run_decompose([ref], 1e-6, 1e-12)
    cdlib.run_decompose_noalloc([out], 1e-6, 1e-12)
    torch.cuda.synchronize()
    assert out.M() == 1927
    _same(ref, out)
    # second call, smaller: the 60-function workload (the array keeps the first
    # call's contents; the call must not depend on them)
    m1 = config_molecule("C1")
    ref1, out1 = _pair(m1, 1e-6, 0.0)
    cdlib.run_decompose([ref1], 1e-6, 0.0)
    cdlib.run_decompose_noalloc([out1], 1e-6, 0.0, sync=True)
    _same(ref1, out1)
    assert out1.M() == 235
    # several problems in one call (all on the caller's stream)
    mols = [make_molecule(4 + 3 * i, 4.0, (0.3, 1.1, 4.0), 2, seed=950 + i) for i in range(4)]
    refs, rws = cdlib.allocate_many([(x.xyz, x.alpha) for x in mols], 1e-6, 1e-12)
    outs, _ = cdlib.allocate_many([(x.xyz, x.alpha) for x in mols], 1e-6, 1e-12)
    cdlib.run_decompose(refs, 1e-6, 1e-12, workspace=rws)
    cdlib.run_decompose_noalloc(outs, 1e-6, 1e-12)
    torch.cuda.synchronize()
    for a, b in zip(refs, outs):
        _same(a, b)


def test_noalloc_refuses_problems_beyond_the_scratch():
    m = config_molecule("C3")
    d = cdlib.allocate(m.xyz, m.alpha, 1e-6, 1e-12)
    assert d.workspace.numel() > cdlib.NOALLOC_SCRATCH_BYTES
    st0 = d.status.clone()
    with pytest.raises(cdlib.CDError) as e:
        cdlib.run_decompose_noalloc([d], 1e-6, 1e-12)
    assert e.value.status == cdlib.CD_ERR_WORKSPACE
    assert b"static scratch" in cdlib.load().cd_last_error()
    torch.cuda.synchronize()
    assert torch.equal(d.status, st0)
