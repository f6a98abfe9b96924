"""Host-side checks of the C-ABI library (no GPU needed): it loads, exports
every function include/cd.h declares, and the binding mirrors the header's
structs."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "cd.h")


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"\b(cd_[a-z0-9_]+)\s*\(", text)
    return sorted(set(names))


@pytest.fixture(scope="module")
def lib():
    from paper_2609_00306_amd import build, cdlib
    if not os.path.exists(cdlib.LIB_PATH):
        build.build()
    return cdlib.load()


def test_header_declares_the_three_calls():
    names = _declared_functions()
    for f in ("cd_decompose", "cd_build_jk", "cd_transform", "cd_query", "cd_last_error"):
        assert f in names


def test_library_exports_every_declared_symbol(lib):
    from paper_2609_00306_amd import cdlib
    names = _declared_functions()
    assert sorted(cdlib.EXPORTS) == names
    for f in names:
        assert hasattr(lib, f), f


def test_version_string(lib):
    assert b"gfx950" in lib.cd_version()


def _struct_sizes_from_c():
    """Compile a tiny host program that prints sizeof/offsetof of the ABI structs."""
    import subprocess
    import tempfile
    src = r'''
#include <stdio.h>
#include <stddef.h>
#include "cd.h"
int main(void) {
  printf("%zu %zu %zu %zu %zu %zu\n", sizeof(cd_molecule), sizeof(cd_decomp_opts),
         sizeof(cd_sizes), sizeof(cd_problem), sizeof(cd_jk_problem),
         sizeof(cd_transform_problem));
  printf("%zu %zu %zu %zu %zu\n", offsetof(cd_problem, status), offsetof(cd_jk_problem, status),
         offsetof(cd_transform_problem, status), offsetof(cd_decomp_opts, events), offsetof(cd_decomp_opts, timeline_cap));
  printf("%zu %zu %zu %zu %zu\n", sizeof(cd_tuning), offsetof(cd_tuning, step1_min_rows),
         offsetof(cd_tuning, step1_q), offsetof(cd_decomp_opts, tuning),
         offsetof(cd_decomp_opts, eta));
  printf("%zu %zu %zu\n", sizeof(cd_mp2_problem), offsetof(cd_mp2_problem, n_vectors),
         offsetof(cd_mp2_problem, status));
  printf("%zu %zu\n", sizeof(cd_zproblem), offsetof(cd_zproblem, status));
  printf("%zu %zu\n", offsetof(cd_jk_problem, Lmo), offsetof(cd_problem, pivot_values));
  printf("%zu %zu %zu %zu %zu\n", sizeof(cd_one_electron_problem),
         offsetof(cd_one_electron_problem, H), sizeof(cd_scf_problem),
         offsetof(cd_scf_problem, e_tol), offsetof(cd_scf_problem, converged));
  return 0;
}
'''
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "t.c")
        exe = os.path.join(d, "t")
        open(c, "w").write(src)
        subprocess.check_call(["gcc", "-std=c11", "-I", os.path.dirname(HEADER), "-o", exe, c])
        out = subprocess.check_output([exe]).decode().split()
    return [int(x) for x in out]


def test_binding_structs_match_header():
    from paper_2609_00306_amd import cdlib
    got = _struct_sizes_from_c()
    mine = [ctypes.sizeof(cdlib.cd_molecule), ctypes.sizeof(cdlib.cd_decomp_opts),
            ctypes.sizeof(cdlib.cd_sizes), ctypes.sizeof(cdlib.cd_problem),
            ctypes.sizeof(cdlib.cd_jk_problem), ctypes.sizeof(cdlib.cd_transform_problem),
            cdlib.cd_problem.status.offset, cdlib.cd_jk_problem.status.offset,
            cdlib.cd_transform_problem.status.offset, cdlib.cd_decomp_opts.events.offset,
            cdlib.cd_decomp_opts.timeline_cap.offset, ctypes.sizeof(cdlib.cd_tuning),
            cdlib.cd_tuning.step1_min_rows.offset, cdlib.cd_tuning.step1_q.offset,
            cdlib.cd_decomp_opts.tuning.offset,
            cdlib.cd_decomp_opts.eta.offset, ctypes.sizeof(cdlib.cd_mp2_problem),
            cdlib.cd_mp2_problem.n_vectors.offset, cdlib.cd_mp2_problem.status.offset,
            ctypes.sizeof(cdlib.cd_zproblem), cdlib.cd_zproblem.status.offset,
            cdlib.cd_jk_problem.Lmo.offset, cdlib.cd_problem.pivot_values.offset,
            ctypes.sizeof(cdlib.cd_one_electron_problem), cdlib.cd_one_electron_problem.H.offset,
            ctypes.sizeof(cdlib.cd_scf_problem), cdlib.cd_scf_problem.e_tol.offset,
            cdlib.cd_scf_problem.converged.offset]
    assert mine == got


def test_argument_validation_without_device(lib):
    from paper_2609_00306_amd import cdlib
    # null opts / negative count are rejected before any device work
    assert lib.cd_query(None, -1, None, None, None, None) == cdlib.CD_ERR_INVALID_ARG
    mol = cdlib.cd_molecule(-3, None, None)
    opts = cdlib.cd_decomp_opts(1e-6, 1e-12, 0, None, None, 0)
    caps = (ctypes.c_int64 * 1)(10)
    sizes = (cdlib.cd_sizes * 1)()
    assert lib.cd_query(ctypes.byref(mol), 1, ctypes.byref(opts), caps, sizes,
                        None) == cdlib.CD_ERR_INVALID_ARG
    assert b"n_basis" in lib.cd_last_error()
    bad = cdlib.cd_decomp_opts(-1.0, 1e-12, 0, None, None, 0)
    mol = cdlib.cd_molecule(0, None, None)
    assert lib.cd_query(ctypes.byref(mol), 1, ctypes.byref(bad), caps, sizes,
                        None) == cdlib.CD_ERR_INVALID_ARG
    nan = cdlib.cd_decomp_opts(float("nan"), 1e-12, 0, None, None, 0)
    assert lib.cd_decompose(None, 0, ctypes.byref(nan), None, 0, None) == cdlib.CD_ERR_INVALID_ARG
    # an N = 0 molecule needs no device work: zero rows
    assert lib.cd_query(ctypes.byref(mol), 1, ctypes.byref(opts), caps, sizes, None) == 0
    assert sizes[0].n_rows == 0 and sizes[0].n_active == 0
    # a problem whose workspace is too small is rejected on the host
    p = cdlib.cd_problem(cdlib.cd_molecule(0, None, None), 0, 0, 4, None, None, None, None,
                         1, 1)
    assert lib.cd_decompose(ctypes.byref(p), 1, ctypes.byref(opts), None, 0,
                            None) == cdlib.CD_ERR_WORKSPACE
    p.n_active = 5
    assert lib.cd_decompose(ctypes.byref(p), 1, ctypes.byref(opts), None, 0,
                            None) == cdlib.CD_ERR_INVALID_ARG
    # a workspace that is large enough but not 256-byte aligned is rejected on the host
    p.n_active = 0
    assert lib.cd_decompose(ctypes.byref(p), 1, ctypes.byref(opts), ctypes.c_void_p(0x1008),
                            1 << 30, None) == cdlib.CD_ERR_INVALID_ARG
    assert b"aligned" in lib.cd_last_error()
    # launch shapes outside their ranges are rejected on the host
    for rt, mr, q in [(1, 0, 0), (8, 0, 0), (0, 8, 0), (0, 1024, 0), (0, 0, 4), (0, 0, 65)]:
        t = cdlib.cd_tuning(rt, mr, q)
        o = cdlib.cd_decomp_opts(1e-6, 1e-12, 0, None, None, 0, ctypes.pointer(t))
        assert lib.cd_decompose(ctypes.byref(p), 1, ctypes.byref(o), None, 0,
                                None) == cdlib.CD_ERR_INVALID_ARG
        assert b"tuning" in lib.cd_last_error()
    # flags other than CD_SYNC, CD_RESUME and CD_DEBUG_POISON_DIAG are rejected on the host
    o = cdlib.cd_decomp_opts(1e-6, 1e-12, 8, None, None, 0, None)
    assert lib.cd_decompose(ctypes.byref(p), 1, ctypes.byref(o), None, 0,
                            None) == cdlib.CD_ERR_INVALID_ARG
    assert b"flags" in lib.cd_last_error()
    # span factors outside [0, 1] (or NaN) are rejected on the host
    for eta in [-0.1, 1.5, float("nan")]:
        o = cdlib.cd_decomp_opts(1e-6, 1e-12, 0, None, None, 0, None, eta)
        assert lib.cd_decompose(ctypes.byref(p), 1, ctypes.byref(o), None, 0,
                                None) == cdlib.CD_ERR_INVALID_ARG
        assert b"eta" in lib.cd_last_error()
    # second-order energy: negative sizes, null pointers, a short workspace
    ws = ctypes.c_size_t()
    assert lib.cd_query_mp2(None, 1, ctypes.byref(ws)) == cdlib.CD_ERR_INVALID_ARG
    mp = cdlib.cd_mp2_problem(-1, 4, 8)
    assert lib.cd_query_mp2(ctypes.byref(mp), 1, ctypes.byref(ws)) == cdlib.CD_ERR_INVALID_ARG
    mp = cdlib.cd_mp2_problem(3, 70, 8)
    assert lib.cd_query_mp2(ctypes.byref(mp), 1, ctypes.byref(ws)) == 0
    # 6 occupied pairs x 3 virtual tile pairs of partials, 6 pair sums, 1 total
    assert ws.value >= (6 * 3 + 6 + 1) * 8
    assert lib.cd_mp2_energy(ctypes.byref(mp), 1, 0, None, 0, None) == cdlib.CD_ERR_WORKSPACE
    assert lib.cd_mp2_energy(ctypes.byref(mp), 1, 0, ctypes.c_void_p(0x1000), ws.value,
                             None) == cdlib.CD_ERR_INVALID_ARG
    assert b"null pointer" in lib.cd_last_error()
    # Hermitian decomposition: sizes, tau, workspace and pointers on the host
    zp = cdlib.cd_zproblem(-1)
    assert lib.cd_query_zdecompose(ctypes.byref(zp), ctypes.byref(ws)) == cdlib.CD_ERR_INVALID_ARG
    zp = cdlib.cd_zproblem(10, None, 5)
    assert lib.cd_query_zdecompose(ctypes.byref(zp), ctypes.byref(ws)) == 0 and ws.value > 0
    assert lib.cd_zdecompose(ctypes.byref(zp), float("nan"), 0, None, 0,
                             None) == cdlib.CD_ERR_INVALID_ARG
    assert lib.cd_zdecompose(ctypes.byref(zp), 1e-6, 0, None, 0, None) == cdlib.CD_ERR_WORKSPACE
    assert lib.cd_zdecompose(ctypes.byref(zp), 1e-6, 0, ctypes.c_void_p(0x1008), ws.value,
                             None) == cdlib.CD_ERR_INVALID_ARG
    assert lib.cd_zdecompose(ctypes.byref(zp), 1e-6, 0, ctypes.c_void_p(0x1000), ws.value,
                             None) == cdlib.CD_ERR_INVALID_ARG
    # J/K: an unknown precision is refused before any device work
    jp = cdlib.cd_jk_problem(4, 0, 0, None, None, ctypes.c_void_p(0x1000), 2,
                             ctypes.c_void_p(0x1000), ctypes.c_void_p(0x1000),
                             ctypes.c_void_p(0x1000), ctypes.c_void_p(0x1000),
                             ctypes.c_void_p(0x1000))
    assert lib.cd_query_jk(ctypes.byref(jp), 1, 7, ctypes.byref(ws)) == cdlib.CD_ERR_INVALID_ARG
    assert b"precision" in lib.cd_last_error()
    # SCF: sizes and pointers are checked on the host
    sp = cdlib.cd_scf_problem(n_basis=4, n_occ=5, max_iter=10)
    assert lib.cd_query_scf(ctypes.byref(sp), 0, ctypes.byref(ws)) == cdlib.CD_ERR_INVALID_ARG
    sp = cdlib.cd_scf_problem(n_basis=4, n_occ=2, max_iter=0)
    assert lib.cd_query_scf(ctypes.byref(sp), 0, ctypes.byref(ws)) == cdlib.CD_ERR_INVALID_ARG
    sp = cdlib.cd_scf_problem(n_basis=4, n_occ=2, max_iter=5)
    assert lib.cd_scf(ctypes.byref(sp), 0, None, 0, None) == cdlib.CD_ERR_INVALID_ARG
    assert b"null pointer" in lib.cd_last_error()
    op = cdlib.cd_one_electron_problem(cdlib.cd_molecule(2, None, None))
    assert lib.cd_one_electron(ctypes.byref(op), 0, None) == cdlib.CD_ERR_INVALID_ARG
    best = cdlib.cd_tuning()
    assert lib.cd_autotune(None, 0, ctypes.byref(opts), None, 0, None,
                           None) == cdlib.CD_ERR_INVALID_ARG


def test_product_path_refuses_missing_library(tmp_path):
    from paper_2609_00306_amd import cdlib
    saved = cdlib._lib
    cdlib._lib = None
    try:
        with pytest.raises(RuntimeError, match="not built"):
            cdlib.load(str(tmp_path / "nope.so"))
    finally:
        cdlib._lib = saved
