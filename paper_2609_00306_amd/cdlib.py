"""Thin ctypes binding of the C ABI in include/cd.h.

Argument marshalling only: every step of the computation runs in the HIP
library.  PyTorch provides device memory and the stream.  The library must
have been built (``paper_2609_00306_amd.build.build()``); there is no CPU
fallback, and a missing library raises.
"""
from __future__ import annotations

import ctypes
import dataclasses
import os
from typing import List, Optional, Sequence

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libcd.so")

CD_OK, CD_ERR_INVALID_ARG, CD_ERR_WORKSPACE, CD_ERR_CAPACITY, CD_ERR_NOT_PSD, \
    CD_ERR_DEVICE, CD_ERR_UNSUPPORTED = range(7)
CD_FP64, CD_FP32, CD_BF16X3 = 0, 1, 2
CD_SYNC = 1
CD_RESUME = 2
CD_DEBUG_POISON_DIAG = 4
PRECISIONS = {"fp64": CD_FP64, "fp32": CD_FP32, "bf16x3": CD_BF16X3}

_vp = ctypes.c_void_p


class cd_molecule(ctypes.Structure):
    _fields_ = [("n_basis", ctypes.c_int32), ("xyz", _vp), ("alpha", _vp), ("pivot_fn", _vp)]


class cd_tuning(ctypes.Structure):
    _fields_ = [("step2_row_tiles", ctypes.c_int32), ("step1_min_rows", ctypes.c_int32),
                ("step1_q", ctypes.c_int32)]


class cd_decomp_opts(ctypes.Structure):
    _fields_ = [("tau", ctypes.c_double), ("schwarz", ctypes.c_double),
                ("flags", ctypes.c_uint32), ("events", ctypes.POINTER(ctypes.c_void_p)),
                ("timeline", _vp), ("timeline_cap", ctypes.c_int64),
                ("tuning", ctypes.POINTER(cd_tuning)), ("eta", ctypes.c_double)]


class cd_sizes(ctypes.Structure):
    _fields_ = [("n_rows", ctypes.c_int64), ("n_active", ctypes.c_int64),
                ("ws_bytes", ctypes.c_size_t)]


class cd_problem(ctypes.Structure):
    _fields_ = [("mol", cd_molecule), ("n_rows", ctypes.c_int64),
                ("n_active", ctypes.c_int64), ("max_vectors", ctypes.c_int64), ("row_pair", _vp), ("L", _vp),
                ("pivots", _vp), ("diag", _vp), ("n_vectors", _vp), ("status", _vp),
                ("pivot_values", _vp)]


class cd_jk_problem(ctypes.Structure):
    _fields_ = [("n_basis", ctypes.c_int32), ("n_rows", ctypes.c_int64),
                ("max_vectors", ctypes.c_int64), ("row_pair", _vp), ("L", _vp),
                ("n_vectors", _vp), ("n_occ", ctypes.c_int32), ("C", _vp), ("J", _vp),
                ("K", _vp), ("status", _vp), ("Lmo", _vp)]


class cd_transform_problem(ctypes.Structure):
    _fields_ = [("n_basis", ctypes.c_int32), ("n_rows", ctypes.c_int64),
                ("max_vectors", ctypes.c_int64), ("row_pair", _vp), ("L", _vp),
                ("n_vectors", _vp), ("p", ctypes.c_int32), ("C1", _vp), ("q", ctypes.c_int32),
                ("C2", _vp), ("Lmo", _vp), ("status", _vp)]


class cd_mp2_problem(ctypes.Structure):
    _fields_ = [("n_occ", ctypes.c_int32), ("n_virt", ctypes.c_int32),
                ("max_vectors", ctypes.c_int64), ("n_vectors", _vp), ("B", _vp), ("e_occ", _vp),
                ("e_virt", _vp), ("energy", _vp), ("pair_energy", _vp), ("status", _vp)]



class cd_one_electron_problem(ctypes.Structure):
    _fields_ = [("mol", cd_molecule), ("n_charges", ctypes.c_int32), ("charge_xyz", _vp),
                ("charge", _vp), ("S", _vp), ("H", _vp)]


class cd_scf_problem(ctypes.Structure):
    _fields_ = [("n_basis", ctypes.c_int32), ("n_rows", ctypes.c_int64),
                ("max_vectors", ctypes.c_int64), ("row_pair", _vp), ("L", _vp),
                ("n_vectors", _vp), ("n_occ", ctypes.c_int32), ("S", _vp), ("H", _vp),
                ("e_charges", ctypes.c_double), ("max_iter", ctypes.c_int32),
                ("e_tol", ctypes.c_double), ("d_tol", ctypes.c_double),
                ("diis", ctypes.c_int32), ("C", _vp), ("D", _vp),
                ("F", _vp), ("energies", _vp), ("status", _vp), ("n_iter", ctypes.c_int32),
                ("converged", ctypes.c_int32)]



class cd_zproblem(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("A", _vp), ("max_vectors", ctypes.c_int64), ("L", _vp),
                ("pivots", _vp), ("diag", _vp), ("n_vectors", _vp), ("status", _vp)]


#: every function include/cd.h declares
EXPORTS = ("cd_query", "cd_decompose", "cd_decompose_noalloc", "cd_autotune", "cd_query_jk", "cd_build_jk", "cd_query_transform",
           "cd_transform", "cd_query_mp2", "cd_mp2_energy", "cd_one_electron", "cd_query_scf",
           "cd_scf", "cd_query_zdecompose", "cd_zdecompose", "cd_last_error", "cd_version")

_lib = None


class CDError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"cd status {status}: {msg}")
        self.status = status


def load(path: str = LIB_PATH):
    """Load libcd.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"HIP library not built: {path} is missing; run "
                           "paper_2609_00306_amd.build.build()")
    L = ctypes.CDLL(path)
    P = ctypes.POINTER
    L.cd_query.argtypes = [P(cd_molecule), ctypes.c_int32, P(cd_decomp_opts),
                           P(ctypes.c_int64), P(cd_sizes), _vp]
    L.cd_decompose.argtypes = [P(cd_problem), ctypes.c_int32, P(cd_decomp_opts), _vp,
                               ctypes.c_size_t, _vp]
    L.cd_decompose_noalloc.argtypes = [P(cd_problem), ctypes.c_int32, P(cd_decomp_opts), _vp]
    L.cd_autotune.argtypes = [P(cd_problem), ctypes.c_int32, P(cd_decomp_opts), _vp,
                              ctypes.c_size_t, P(cd_tuning), _vp]
    L.cd_query_jk.argtypes = [P(cd_jk_problem), ctypes.c_int32, ctypes.c_int,
                              P(ctypes.c_size_t)]
    L.cd_build_jk.argtypes = [P(cd_jk_problem), ctypes.c_int32, ctypes.c_int, ctypes.c_uint32,
                              _vp, ctypes.c_size_t, _vp]
    L.cd_query_transform.argtypes = [P(cd_transform_problem), ctypes.c_int32,
                                     P(ctypes.c_size_t)]
    L.cd_transform.argtypes = [P(cd_transform_problem), ctypes.c_int32, ctypes.c_uint32, _vp,
                               ctypes.c_size_t, _vp]
    L.cd_query_mp2.argtypes = [P(cd_mp2_problem), ctypes.c_int32, P(ctypes.c_size_t)]
    L.cd_mp2_energy.argtypes = [P(cd_mp2_problem), ctypes.c_int32, ctypes.c_uint32, _vp,
                                ctypes.c_size_t, _vp]
    L.cd_one_electron.argtypes = [P(cd_one_electron_problem), ctypes.c_uint32, _vp]
    L.cd_query_scf.argtypes = [P(cd_scf_problem), ctypes.c_int, P(ctypes.c_size_t)]
    L.cd_scf.argtypes = [P(cd_scf_problem), ctypes.c_int, _vp, ctypes.c_size_t, _vp]
    L.cd_query_zdecompose.argtypes = [P(cd_zproblem), P(ctypes.c_size_t)]
    L.cd_zdecompose.argtypes = [P(cd_zproblem), ctypes.c_double, ctypes.c_uint32, _vp,
                                ctypes.c_size_t, _vp]
    for f in ("cd_query", "cd_decompose", "cd_decompose_noalloc", "cd_autotune", "cd_query_jk", "cd_build_jk",
              "cd_query_transform", "cd_transform", "cd_query_mp2", "cd_mp2_energy",
              "cd_one_electron", "cd_query_scf", "cd_scf", "cd_query_zdecompose",
              "cd_zdecompose"):
        getattr(L, f).restype = ctypes.c_int
    L.cd_last_error.restype = ctypes.c_char_p
    L.cd_last_error.argtypes = []
    L.cd_version.restype = ctypes.c_char_p
    L.cd_version.argtypes = []
    _lib = L
    return L


def _check(st: int):
    if st != CD_OK:
        raise CDError(st, load().cd_last_error().decode())


def _ptr(t: Optional[torch.Tensor]) -> Optional[int]:
    return None if t is None or t.numel() == 0 else t.data_ptr()


def _stream(stream) -> Optional[int]:
    s = torch.cuda.current_stream() if stream is None else stream
    return s.cuda_stream


def _dev_f64(a, device) -> torch.Tensor:
    if isinstance(a, torch.Tensor):
        return a.to(device=device, dtype=torch.float64).contiguous()
    return torch.as_tensor(a, dtype=torch.float64).to(device).contiguous()


@dataclasses.dataclass
class Decomposition:
    """Device-resident result of cd_decompose for one molecule."""
    n_basis: int
    n_rows: int
    n_active: int
    max_vectors: int
    xyz: torch.Tensor
    alpha: torch.Tensor
    row_pair: torch.Tensor   # [n_rows] int64
    L: torch.Tensor          # [max_vectors][n_rows] float64
    pivots: torch.Tensor     # [max_vectors] int64
    diag: torch.Tensor       # [n_rows] float64
    n_vectors: torch.Tensor  # [1] int64
    status: torch.Tensor     # [1] int32
    workspace: torch.Tensor
    pivot_fn: Optional[torch.Tensor] = None   # [N] uint8 restricted candidates, or None
    pivot_values: Optional[torch.Tensor] = None   # [max_vectors] float64 d_K

    def M(self) -> int:
        return int(self.n_vectors.item())


def molecule(xyz: torch.Tensor, alpha: torch.Tensor,
             pivot_fn: Optional[torch.Tensor] = None) -> cd_molecule:
    return cd_molecule(int(alpha.shape[0]), _ptr(xyz), _ptr(alpha), _ptr(pivot_fn))


def _dev_flags(pivot_fn, n: int, device) -> Optional[torch.Tensor]:
    if pivot_fn is None:
        return None
    f = torch.as_tensor(pivot_fn).reshape(-1).to(device=device)
    if f.numel() != n:
        raise ValueError("pivot_fn needs one flag per basis function")
    return (f != 0).to(torch.uint8).contiguous()


def query(mols: Sequence[cd_molecule], tau: float, schwarz: float,
          max_vectors: Sequence[int], stream=None) -> List[cd_sizes]:
    L = load()
    n = len(mols)
    arr = (cd_molecule * n)(*mols)
    caps = (ctypes.c_int64 * n)(*[int(c) for c in max_vectors])
    out = (cd_sizes * n)()
    opts = cd_decomp_opts(float(tau), float(schwarz), 0, None, None, 0, None)
    _check(L.cd_query(arr, n, ctypes.byref(opts), caps, out, _stream(stream)))
    return list(out)


def allocate(xyz, alpha, tau: float, schwarz: float, max_vectors: Optional[int] = None,
             device="cuda", stream=None, pivot_fn=None) -> Decomposition:
    """Allocate outputs and workspace for one molecule (sizes from cd_query).

    Without ``max_vectors`` the capacity is the number of active rows, which
    bounds the number of vectors (every pivot is an active row).  ``pivot_fn``:
    optional per-function flags of restricted-candidate pivoting (Sec. 6.2)."""
    xyz = _dev_f64(xyz, device).reshape(-1, 3)
    alpha = _dev_f64(alpha, device).reshape(-1)
    fn = _dev_flags(pivot_fn, int(alpha.shape[0]), device)
    if max_vectors is None:
        sz = query([molecule(xyz, alpha, fn)], tau, schwarz, [0], stream)[0]
        max_vectors = max(1, int(sz.n_active))
    sz = query([molecule(xyz, alpha, fn)], tau, schwarz, [max_vectors], stream)[0]
    n, mv = int(sz.n_rows), int(max_vectors)
    i64 = dict(dtype=torch.int64, device=device)
    f64 = dict(dtype=torch.float64, device=device)
    return Decomposition(
        n_basis=int(alpha.shape[0]), n_rows=n, n_active=int(sz.n_active), max_vectors=mv,
        xyz=xyz, alpha=alpha,
        row_pair=torch.empty(n, **i64), L=torch.empty((mv, n), **f64),
        pivots=torch.empty(mv, **i64), diag=torch.empty(n, **f64),
        n_vectors=torch.zeros(1, **i64), status=torch.zeros(1, dtype=torch.int32, device=device),
        workspace=torch.empty(max(1, int(sz.ws_bytes)), dtype=torch.uint8, device=device),
        pivot_fn=fn, pivot_values=torch.empty(mv, **f64))


def allocate_many(mols, tau: float, schwarz: float, max_vectors=None, device="cuda",
                  stream=None):
    """Outputs for several molecules plus one shared workspace (batched call).

    ``mols``: sequence of (xyz, alpha).  Returns (decompositions, workspace)."""
    decs = [allocate(x, a, tau, schwarz, None if max_vectors is None else max_vectors[i],
                     device, stream) for i, (x, a) in enumerate(mols)]
    total = sum(int(d.workspace.numel()) for d in decs)
    for d in decs:
        d.workspace = torch.empty(0, dtype=torch.uint8, device=device)
    ws = torch.empty(max(1, total), dtype=torch.uint8, device=device)
    return decs, ws


def problem(d: Decomposition) -> cd_problem:
    return cd_problem(molecule(d.xyz, d.alpha, d.pivot_fn), d.n_rows, d.n_active, d.max_vectors,
                      _ptr(d.row_pair),
                      _ptr(d.L), _ptr(d.pivots), _ptr(d.diag), _ptr(d.n_vectors),
                      _ptr(d.status), _ptr(d.pivot_values))


def run_decompose(decs: Sequence[Decomposition], tau: float, schwarz: float, sync: bool = False,
                  stream=None, workspace: Optional[torch.Tensor] = None,
                  events: Optional[Sequence] = None, timeline: Optional[torch.Tensor] = None,
                  tuning: Optional[cd_tuning] = None, eta: float = 1.0,
                  resume: bool = False, poison: bool = False):
    """cd_decompose on already allocated problems (one workspace per call).

    ``events``: optional four torch.cuda.Event(enable_timing=True) that the
    library records at its phase boundaries on the stream.  ``tuning``: launch
    shapes (from autotune), or None for the built-in ones.  ``eta``: span
    factor of the two-step first step (1 = exact pivoting).  ``resume``:
    CD_RESUME (continue the stored decompositions to ``tau``; see ``resume``).
    ``poison``: CD_DEBUG_POISON_DIAG (tests of the device error path)."""
    L = load()
    n = len(decs)
    arr = (cd_problem * n)(*[problem(d) for d in decs])
    ev = None
    if events is not None:
        for e in events:
            if not e.cuda_event:        # torch creates the event on its first record
                e.record(torch.cuda.current_stream() if stream is None else stream)
        ev = (ctypes.c_void_p * 4)(*[e.cuda_event for e in events])
    tl, cap = (None, 0) if timeline is None else (timeline.data_ptr(),
                                                   (timeline.numel() - 1) // 16)
    flags = ((CD_SYNC if sync else 0) | (CD_RESUME if resume else 0)
             | (CD_DEBUG_POISON_DIAG if poison else 0))
    opts = cd_decomp_opts(float(tau), float(schwarz), flags, ev, tl, cap,
                          ctypes.pointer(tuning) if tuning is not None else None, float(eta))
    if workspace is None:
        if n != 1:
            raise ValueError("pass a shared workspace for more than one molecule")
        workspace = decs[0].workspace
    _check(L.cd_decompose(arr, n, ctypes.byref(opts), _ptr(workspace), workspace.numel(),
                          _stream(stream)))


NOALLOC_SCRATCH_BYTES = 128 << 20


def run_decompose_noalloc(decs: Sequence[Decomposition], tau: float, schwarz: float,
                          sync: bool = False, stream=None, eta: float = 1.0):
    """cd_decompose_noalloc: the decomposition with the library's static device
    scratch instead of a workspace (no device allocation in the call; calls
    that overlap on one GPU race).  The problems' own workspaces are unused."""
    L = load()
    n = len(decs)
    arr = (cd_problem * n)(*[problem(d) for d in decs])
    opts = cd_decomp_opts(float(tau), float(schwarz), CD_SYNC if sync else 0, None, None, 0,
                          None, float(eta))
    _check(L.cd_decompose_noalloc(arr, n, ctypes.byref(opts), _stream(stream)))


def autotune(decs: Sequence[Decomposition], tau: float, schwarz: float, stream=None,
             workspace: Optional[torch.Tensor] = None) -> cd_tuning:
    """cd_autotune: measure launch shapes for these problems (blocking); the
    outputs are left as the chosen shape's decomposition."""
    L = load()
    n = len(decs)
    arr = (cd_problem * n)(*[problem(d) for d in decs])
    opts = cd_decomp_opts(float(tau), float(schwarz), 0, None, None, 0, None)
    if workspace is None:
        if n != 1:
            raise ValueError("pass a shared workspace for more than one molecule")
        workspace = decs[0].workspace
    best = cd_tuning(0, 0, 0)
    _check(L.cd_autotune(arr, n, ctypes.byref(opts), _ptr(workspace), workspace.numel(),
                         ctypes.byref(best), _stream(stream)))
    return best


def resume(d: Decomposition, tau: float, schwarz: float, max_vectors: Optional[int] = None,
           sync: bool = True, stream=None, eta: float = 1.0) -> Decomposition:
    """Continue the decomposition in ``d`` (made at a larger threshold with the
    same ``schwarz``) to ``tau`` with CD_RESUME, in place.  The capacity becomes
    ``max_vectors`` (default: the active rows at ``tau``); if that is larger
    than ``d``'s, L, the pivots and the pivot values move into larger buffers
    first (vector K stays at L[K]).  The workspace is sized at the new
    threshold."""
    sz = query([molecule(d.xyz, d.alpha, d.pivot_fn)], tau, schwarz, [0], stream)[0]
    mv = int(max_vectors) if max_vectors is not None else max(1, int(sz.n_active))
    if mv > d.max_vectors:
        dev = d.L.device
        L = torch.empty((mv, d.n_rows), dtype=torch.float64, device=dev)
        L[:d.max_vectors].copy_(d.L)
        piv = torch.empty(mv, dtype=torch.int64, device=dev)
        piv[:d.max_vectors].copy_(d.pivots)
        pv = torch.empty(mv, dtype=torch.float64, device=dev)
        pv[:d.max_vectors].copy_(d.pivot_values)
        d.L, d.pivots, d.pivot_values, d.max_vectors = L, piv, pv, mv
    sz = query([molecule(d.xyz, d.alpha, d.pivot_fn)], tau, schwarz, [d.max_vectors], stream)[0]
    if int(sz.n_rows) != d.n_rows:
        raise ValueError("resume needs the same rows (same molecule and schwarz)")
    d.n_active = int(sz.n_active)
    d.workspace = torch.empty(max(1, int(sz.ws_bytes)), dtype=torch.uint8, device=d.L.device)
    run_decompose([d], tau, schwarz, sync=sync, stream=stream, eta=eta, resume=True)
    return d


def decompose(xyz, alpha, tau: float, schwarz: float = 1e-12, max_vectors: Optional[int] = None,
              sync: bool = True, device="cuda", stream=None, eta: float = 1.0,
              pivot_fn=None) -> Decomposition:
    d = allocate(xyz, alpha, tau, schwarz, max_vectors, device, stream, pivot_fn)
    run_decompose([d], tau, schwarz, sync=sync, stream=stream, eta=eta)
    return d


@dataclasses.dataclass
class JK:
    J: torch.Tensor
    K: torch.Tensor
    status: torch.Tensor
    workspace: torch.Tensor
    problem: cd_jk_problem
    C: torch.Tensor
    Lmo: Optional[torch.Tensor] = None   # [max_vectors][O][O] when asked for


def prepare_jk(d: Decomposition, C, prec: str = "fp64", lmo: bool = False) -> JK:
    """Outputs and workspace of one J/K build; with ``lmo`` the build also
    writes C^T L^P C from its FP64 half transform (fp64 and bf16x3)."""
    dev = d.L.device
    C = _dev_f64(C, dev)
    N = d.n_basis
    J = torch.empty((N, N), dtype=torch.float64, device=dev)
    K = torch.empty((N, N), dtype=torch.float64, device=dev)
    st = torch.zeros(1, dtype=torch.int32, device=dev)
    O = int(C.shape[1]) if C.ndim == 2 else 0
    Lmo = (torch.empty((d.max_vectors, O, O), dtype=torch.float64, device=dev) if lmo else None)
    p = cd_jk_problem(N, d.n_rows, d.max_vectors, _ptr(d.row_pair), _ptr(d.L), _ptr(d.n_vectors),
                      O, _ptr(C), _ptr(J), _ptr(K), _ptr(st), _ptr(Lmo))
    ws = ctypes.c_size_t()
    _check(load().cd_query_jk(ctypes.byref(p), 1, PRECISIONS[prec], ctypes.byref(ws)))
    w = torch.empty(max(1, ws.value), dtype=torch.uint8, device=dev)
    return JK(J, K, st, w, p, C, Lmo)


def prepare_jk_many(decs: Sequence[Decomposition], Cs, prec: str = "fp64", lmo: bool = False):
    """J/K outputs for several decompositions plus one shared workspace (with
    ``lmo`` each problem also gets its C^T L^P C output)."""
    jks = [prepare_jk(d, C, prec, lmo=lmo) for d, C in zip(decs, Cs)]
    total = sum(int(j.workspace.numel()) for j in jks)
    dev = decs[0].L.device
    for j in jks:
        j.workspace = torch.empty(0, dtype=torch.uint8, device=dev)
    return jks, torch.empty(max(1, total), dtype=torch.uint8, device=dev)


def run_jk_many(jks: Sequence[JK], workspace: torch.Tensor, prec: str = "fp64",
                sync: bool = False, stream=None):
    n = len(jks)
    arr = (cd_jk_problem * n)(*[j.problem for j in jks])
    _check(load().cd_build_jk(arr, n, PRECISIONS[prec], CD_SYNC if sync else 0,
                              _ptr(workspace), workspace.numel(), _stream(stream)))


def run_jk(jk: JK, prec: str = "fp64", sync: bool = False, stream=None):
    _check(load().cd_build_jk(ctypes.byref(jk.problem), 1, PRECISIONS[prec],
                              CD_SYNC if sync else 0, _ptr(jk.workspace), jk.workspace.numel(),
                              _stream(stream)))


def build_jk(d: Decomposition, C, prec: str = "fp64", sync: bool = True, stream=None):
    jk = prepare_jk(d, C, prec)
    run_jk(jk, prec, sync, stream)
    return jk.J, jk.K


def transform(d: Decomposition, C1, C2, sync: bool = True, stream=None) -> torch.Tensor:
    dev = d.L.device
    C1 = _dev_f64(C1, dev)
    C2 = _dev_f64(C2, dev)
    p, q = int(C1.shape[1]), int(C2.shape[1])
    out = torch.empty((d.max_vectors, p, q), dtype=torch.float64, device=dev)
    st = torch.zeros(1, dtype=torch.int32, device=dev)
    prob = cd_transform_problem(d.n_basis, d.n_rows, d.max_vectors, _ptr(d.row_pair), _ptr(d.L),
                                _ptr(d.n_vectors), p, _ptr(C1), q, _ptr(C2), _ptr(out), _ptr(st))
    ws = ctypes.c_size_t()
    L = load()
    _check(L.cd_query_transform(ctypes.byref(prob), 1, ctypes.byref(ws)))
    w = torch.empty(max(1, ws.value), dtype=torch.uint8, device=dev)
    _check(L.cd_transform(ctypes.byref(prob), 1, CD_SYNC if sync else 0, _ptr(w), w.numel(),
                          _stream(stream)))
    return out


def mp2_energy(B, n_vectors, e_occ, e_virt, pair_energy: bool = False, sync: bool = True,
               stream=None):
    """Closed-shell second-order energy from transformed vectors B[max_vectors][O][V].

    ``n_vectors`` is a device int64 tensor of one element (a decomposition's
    count).  Returns the energy as a device tensor of one element and, when
    asked, the pair energies e_ij as an [O][O] device tensor.
    """
    dev = B.device
    if B.dtype != torch.float64 or B.dim() != 3 or not B.is_contiguous():
        raise ValueError("B must be a contiguous float64 [max_vectors][O][V] tensor")
    mv, O, V = (int(x) for x in B.shape)
    eo = _dev_f64(e_occ, dev)
    ev = _dev_f64(e_virt, dev)
    if eo.numel() != O or ev.numel() != V:
        raise ValueError("orbital energies do not match B's shape")
    if n_vectors.dtype != torch.int64 or n_vectors.device != dev:
        raise ValueError("n_vectors must be an int64 tensor on B's device")
    E = torch.empty(1, dtype=torch.float64, device=dev)
    pe = torch.empty((O, O), dtype=torch.float64, device=dev) if pair_energy else None
    st = torch.zeros(1, dtype=torch.int32, device=dev)
    prob = cd_mp2_problem(O, V, mv, _ptr(n_vectors), _ptr(B), _ptr(eo), _ptr(ev), _ptr(E),
                          _ptr(pe), _ptr(st))
    ws = ctypes.c_size_t()
    L = load()
    _check(L.cd_query_mp2(ctypes.byref(prob), 1, ctypes.byref(ws)))
    w = torch.empty(max(1, ws.value), dtype=torch.uint8, device=dev)
    _check(L.cd_mp2_energy(ctypes.byref(prob), 1, CD_SYNC if sync else 0, _ptr(w), w.numel(),
                           _stream(stream)))
    return (E, pe) if pair_energy else E


def one_electron(xyz, alpha, charge_xyz, charge, device="cuda", sync: bool = True, stream=None):
    """Overlap S and one-electron Hamiltonian H (kinetic + point-charge
    attraction) as device [N][N] tensors."""
    xyz = _dev_f64(xyz, device).reshape(-1, 3)
    alpha = _dev_f64(alpha, device).reshape(-1)
    cx = _dev_f64(charge_xyz, device).reshape(-1, 3)
    Z = _dev_f64(charge, device).reshape(-1)
    N = int(alpha.shape[0])
    S = torch.empty((N, N), dtype=torch.float64, device=device)
    H = torch.empty((N, N), dtype=torch.float64, device=device)
    prob = cd_one_electron_problem(molecule(xyz, alpha), int(Z.numel()), _ptr(cx), _ptr(Z),
                                   _ptr(S), _ptr(H))
    _check(load().cd_one_electron(ctypes.byref(prob), CD_SYNC if sync else 0, _stream(stream)))
    return S, H


@dataclasses.dataclass
class SCFResult:
    energies: torch.Tensor   # [n_iter] E_k
    C: torch.Tensor          # [N][O], D = C C^T
    D: torch.Tensor
    F: torch.Tensor
    converged: bool


def scf(d: Decomposition, S: torch.Tensor, H: torch.Tensor, n_occ: int, e_charges: float,
        prec: str = "fp64", max_iter: int = 100, e_tol: float = 1e-10, d_tol: float = 1e-8,
        diis: int = 8, stream=None) -> SCFResult:
    """Closed-shell SCF on the decomposition's J/K (cd_scf; blocking)."""
    dev = d.L.device
    N = d.n_basis
    f64 = dict(dtype=torch.float64, device=dev)
    C = torch.empty((N, n_occ), **f64)
    D = torch.empty((N, N), **f64)
    F = torch.empty((N, N), **f64)
    E = torch.zeros(max_iter, **f64)
    st = torch.zeros(1, dtype=torch.int32, device=dev)
    S = S.contiguous()
    H = H.contiguous()
    prob = cd_scf_problem(N, d.n_rows, d.max_vectors, _ptr(d.row_pair), _ptr(d.L),
                          _ptr(d.n_vectors), int(n_occ), _ptr(S), _ptr(H), float(e_charges),
                          int(max_iter), float(e_tol), float(d_tol), int(diis), _ptr(C),
                          _ptr(D), _ptr(F),
                          _ptr(E), _ptr(st), 0, 0)
    L = load()
    ws = ctypes.c_size_t()
    _check(L.cd_query_scf(ctypes.byref(prob), PRECISIONS[prec], ctypes.byref(ws)))
    w = torch.empty(max(1, ws.value), dtype=torch.uint8, device=dev)
    _check(L.cd_scf(ctypes.byref(prob), PRECISIONS[prec], _ptr(w), w.numel(), _stream(stream)))
    return SCFResult(E[:prob.n_iter].clone(), C, D, F, bool(prob.converged))


@dataclasses.dataclass
class ZDecomposition:
    """Device-resident result of cd_zdecompose."""
    L: torch.Tensor          # [max_vectors][n] complex128
    pivots: torch.Tensor     # [max_vectors] int64
    diag: torch.Tensor       # [n] float64
    n_vectors: torch.Tensor  # [1] int64
    status: torch.Tensor     # [1] int32
    workspace: Optional[torch.Tensor] = None

    def M(self) -> int:
        return int(self.n_vectors.item())


def zdecompose(A: torch.Tensor, tau: float, max_vectors: Optional[int] = None,
               sync: bool = True, stream=None) -> ZDecomposition:
    """Pivoted Cholesky decomposition of a Hermitian PSD complex128 device
    matrix [n][n] (Sec. 7): A ~ sum_K L_K L_K^H."""
    if A.dtype != torch.complex128 or A.dim() != 2 or A.shape[0] != A.shape[1]:
        raise ValueError("A must be a square complex128 tensor")
    A = A.contiguous()
    dev = A.device
    n = int(A.shape[0])
    mv = n if max_vectors is None else int(max_vectors)
    out = ZDecomposition(L=torch.empty((max(1, mv), max(1, n)), dtype=torch.complex128, device=dev),
                         pivots=torch.empty(max(1, mv), dtype=torch.int64, device=dev),
                         diag=torch.empty(max(1, n), dtype=torch.float64, device=dev),
                         n_vectors=torch.zeros(1, dtype=torch.int64, device=dev),
                         status=torch.zeros(1, dtype=torch.int32, device=dev))
    prob = cd_zproblem(n, _ptr(A), mv, _ptr(out.L), _ptr(out.pivots), _ptr(out.diag),
                       _ptr(out.n_vectors), _ptr(out.status))
    L = load()
    ws = ctypes.c_size_t()
    _check(L.cd_query_zdecompose(ctypes.byref(prob), ctypes.byref(ws)))
    w = torch.empty(max(1, ws.value) + 256, dtype=torch.uint8, device=dev)
    off = (-w.data_ptr()) % 256
    _check(L.cd_zdecompose(ctypes.byref(prob), float(tau), CD_SYNC if sync else 0,
                           w.data_ptr() + off, w.numel() - off, _stream(stream)))
    out.workspace = w
    return out

