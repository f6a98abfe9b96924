"""CPU oracle (plain FP64 C, OpenMP over rows) for the Cholesky path.

TEST INFRASTRUCTURE ONLY: imported by the test suite, by the smoke check and
by the benchmark's CPU-baseline leg, never by the GPU library.  It shares no
code with the GPU library.  ``build()`` compiles ``cd_oracle.c`` with gcc.

Every function follows the paper's Sec. 2 (decomposition), Sec. 4.1 (J/K
from the vectors, AO->MO transform); see ``cd_oracle.c`` for the formulas.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import NamedTuple, Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "cd_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

_d = ctypes.POINTER(ctypes.c_double)
_i64 = ctypes.POINTER(ctypes.c_int64)
_i32 = ctypes.POINTER(ctypes.c_int32)


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O2, OpenMP)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = ctypes.CDLL(_LIB)
        L.or_boys0.restype = ctypes.c_double
        L.or_boys0.argtypes = [ctypes.c_double]
        L.or_eri.restype = ctypes.c_double
        L.or_eri.argtypes = [_d, _d, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int]
        L.or_unpack_pair.restype = None
        L.or_unpack_pair.argtypes = [ctypes.c_int64, _i32, _i32]
        L.or_diagonal_all.restype = None
        L.or_diagonal_all.argtypes = [ctypes.c_int, _d, _d, _d]
        L.or_rows.restype = ctypes.c_int64
        L.or_rows.argtypes = [ctypes.c_int, _d, _d, ctypes.c_double, _i64, _d]
        L.or_eri_matrix.restype = None
        L.or_eri_matrix.argtypes = [_d, _d, ctypes.c_int64, _i64, _d]
        L.or_one_electron.restype = None
        L.or_one_electron.argtypes = [ctypes.c_int, _d, _d, ctypes.c_int, _d, _d, _d, _d, _d]
        L.or_charge_repulsion.restype = ctypes.c_double
        L.or_charge_repulsion.argtypes = [ctypes.c_int, _d, _d]
        L.or_zdecompose.restype = ctypes.c_int
        L.or_zdecompose.argtypes = [ctypes.c_int64, _d, ctypes.c_double, ctypes.c_int64, _d,
                                    _i64, _d, _i64]
        L.or_decompose.restype = ctypes.c_int
        L.or_decompose.argtypes = [_d, _d, ctypes.c_int64, _i64, ctypes.c_double, ctypes.c_int64,
                                   _d, _i64, _d, _d, _i64, _i64, ctypes.c_int64,
                                   ctypes.c_double, _i64, ctypes.c_void_p]
        L.or_jk_cd.restype = None
        L.or_jk_cd.argtypes = [ctypes.c_int, ctypes.c_int64, _i64, _d, ctypes.c_int64, _d,
                               ctypes.c_int, _d, _d]
        L.or_jk_exact.restype = None
        L.or_jk_exact.argtypes = [ctypes.c_int, _d, _d, _d, ctypes.c_int, _d, _d]
        L.or_e2.restype = ctypes.c_double
        L.or_e2.argtypes = [ctypes.c_int, _d, ctypes.c_int, _d, _d]
        L.or_mp2_pair.restype = ctypes.c_double
        L.or_mp2_pair.argtypes = [ctypes.c_int64, ctypes.c_int, ctypes.c_int, _d, _d, _d,
                                  ctypes.c_int, ctypes.c_int]
        L.or_mp2.restype = ctypes.c_double
        L.or_mp2.argtypes = [ctypes.c_int64, ctypes.c_int, ctypes.c_int, _d, _d, _d, _d]
        L.or_transform.restype = None
        L.or_transform.argtypes = [ctypes.c_int, ctypes.c_int64, _i64, _d, ctypes.c_int64, _d,
                                   ctypes.c_int, _d, ctypes.c_int, _d]
        _lib = L
    return _lib


def _p(a: np.ndarray, t):
    return a.ctypes.data_as(t)


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def boys0(T: float) -> float:
    return lib().or_boys0(float(T))


def eri(xyz, alpha, mu, nu, sg, rh) -> float:
    xyz, alpha = _f64(xyz), _f64(alpha)
    return lib().or_eri(_p(xyz, _d), _p(alpha, _d), mu, nu, sg, rh)


def unpack_pair(pq: int):
    a, b = ctypes.c_int32(), ctypes.c_int32()
    lib().or_unpack_pair(int(pq), ctypes.byref(a), ctypes.byref(b))
    return a.value, b.value


def diagonal_all(xyz, alpha) -> np.ndarray:
    xyz, alpha = _f64(xyz), _f64(alpha)
    N = alpha.shape[0]
    out = np.empty(N * (N + 1) // 2)
    lib().or_diagonal_all(N, _p(xyz, _d), _p(alpha, _d), _p(out, _d))
    return out


def rows(xyz, alpha, schwarz: float):
    """Screened row list (packed pair indices, ascending) and max D^1."""
    xyz, alpha = _f64(xyz), _f64(alpha)
    N = alpha.shape[0]
    rp = np.empty(max(1, N * (N + 1) // 2), dtype=np.int64)
    mx = ctypes.c_double()
    n = lib().or_rows(N, _p(xyz, _d), _p(alpha, _d), float(schwarz), _p(rp, _i64),
                      ctypes.byref(mx))
    return rp[:n].copy(), mx.value


def eri_matrix(xyz, alpha, row_pair) -> np.ndarray:
    xyz, alpha = _f64(xyz), _f64(alpha)
    rp = np.ascontiguousarray(row_pair, dtype=np.int64)
    n = rp.shape[0]
    A = np.empty((n, n))
    lib().or_eri_matrix(_p(xyz, _d), _p(alpha, _d), n, _p(rp, _i64), _p(A, _d))
    return A


class CD(NamedTuple):
    rc: int
    M: int
    L: np.ndarray        # [M][n]
    pivots: np.ndarray   # [M] row indices
    dpiv: np.ndarray     # [M] pivot values d_K
    D: np.ndarray        # [n] final residual diagonal
    bad: int             # replay: first pivot that was not a valid argmax (or -1)


def candidate_rows(row_pair, pivot_fn) -> np.ndarray:
    """Row mask of restricted-candidate pivoting (Sec. 6.2): row (mu nu) may be
    a pivot iff both functions are flagged in ``pivot_fn`` [N]."""
    fn = np.asarray(pivot_fn).astype(bool)
    out = np.zeros(len(row_pair), dtype=np.uint8)
    for r, pq in enumerate(np.asarray(row_pair, dtype=np.int64)):
        mu, nu = unpack_pair(int(pq))
        out[r] = 1 if (fn[mu] and fn[nu]) else 0
    return out


def decompose(xyz, alpha, row_pair, tau: float, max_vectors: Optional[int] = None,
              given: Optional[np.ndarray] = None, tie_tol: float = 0.0,
              pivot_fn=None) -> CD:
    """Sec. 2 decomposition over the given rows.  With ``pivot_fn`` (flags per
    function) only rows of two flagged functions may be pivots (Sec. 6.2)."""
    xyz, alpha = _f64(xyz), _f64(alpha)
    rp = np.ascontiguousarray(row_pair, dtype=np.int64)
    n = rp.shape[0]
    cand = None if pivot_fn is None else candidate_rows(rp, pivot_fn)
    if max_vectors is None:
        max_vectors = n
    L = np.zeros((max(1, max_vectors), max(1, n)))
    piv = np.zeros(max(1, max_vectors), dtype=np.int64)
    dp = np.zeros(max(1, max_vectors))
    D = np.zeros(max(1, n))
    M = ctypes.c_int64()
    bad = ctypes.c_int64()
    if given is not None:
        g = np.ascontiguousarray(given, dtype=np.int64)
        gp, ng = _p(g, _i64), g.shape[0]
    else:
        g, gp, ng = None, None, 0
    rc = lib().or_decompose(_p(xyz, _d), _p(alpha, _d), n, _p(rp, _i64), float(tau),
                            int(max_vectors), _p(L, _d), _p(piv, _i64), _p(dp, _d), _p(D, _d),
                            ctypes.byref(M), gp, ng, float(tie_tol), ctypes.byref(bad),
                            None if cand is None else cand.ctypes.data)
    m = M.value
    return CD(rc, m, L[:m, :n].copy(), piv[:m].copy(), dp[:m].copy(), D[:n].copy(), bad.value)


def jk_cd(N: int, row_pair, L, C):
    rp = np.ascontiguousarray(row_pair, dtype=np.int64)
    L = _f64(L)
    C = _f64(C)
    M = L.shape[0] if L.ndim == 2 else 0
    O = C.shape[1]
    J = np.empty((N, N))
    K = np.empty((N, N))
    lib().or_jk_cd(N, rp.shape[0], _p(rp, _i64), _p(L, _d), M, _p(C, _d), O, _p(J, _d),
                   _p(K, _d))
    return J, K


def jk_exact(xyz, alpha, C):
    xyz, alpha, C = _f64(xyz), _f64(alpha), _f64(C)
    N = alpha.shape[0]
    J = np.empty((N, N))
    K = np.empty((N, N))
    lib().or_jk_exact(N, _p(xyz, _d), _p(alpha, _d), _p(C, _d), C.shape[1], _p(J, _d),
                      _p(K, _d))
    return J, K


def e2(C, J, K) -> float:
    C, J, K = _f64(C), _f64(J), _f64(K)
    return lib().or_e2(C.shape[0], _p(C, _d), C.shape[1], _p(J, _d), _p(K, _d))


def transform(N: int, row_pair, L, C1, C2) -> np.ndarray:
    rp = np.ascontiguousarray(row_pair, dtype=np.int64)
    L, C1, C2 = _f64(L), _f64(C1), _f64(C2)
    M = L.shape[0]
    p, q = C1.shape[1], C2.shape[1]
    out = np.empty((M, p, q))
    lib().or_transform(N, rp.shape[0], _p(rp, _i64), _p(L, _d), M, _p(C1, _d), p, _p(C2, _d),
                       q, _p(out, _d))
    return out


def mp2(B, e_occ, e_virt):
    """Closed-shell second-order energy from transformed vectors B [M][O][V]
    (CD-based MP2, Secs. 5 and 7): returns (E, pair energies [O][O])."""
    B, eo, ev = _f64(B), _f64(e_occ), _f64(e_virt)
    M, O, V = B.shape
    pair = np.zeros((max(1, O), max(1, O)))
    e = lib().or_mp2(M, O, V, _p(B, _d), _p(eo, _d), _p(ev, _d), _p(pair, _d))
    return e, pair[:O, :O].copy()


def mp2_pair(B, e_occ, e_virt, i: int, j: int) -> float:
    """One pair energy e_ij of ``mp2``."""
    B, eo, ev = _f64(B), _f64(e_occ), _f64(e_virt)
    M, O, V = B.shape
    return lib().or_mp2_pair(M, O, V, _p(B, _d), _p(eo, _d), _p(ev, _d), int(i), int(j))


def one_electron(xyz, alpha, charge_xyz, charge):
    """Overlap S, kinetic T and point-charge attraction V, each [N][N]."""
    xyz, alpha = _f64(xyz), _f64(alpha)
    cx, Z = _f64(np.reshape(charge_xyz, (-1, 3))), _f64(charge)
    N, nc = alpha.shape[0], Z.shape[0]
    S, T, V = (np.zeros((max(1, N), max(1, N))) for _ in range(3))
    lib().or_one_electron(N, _p(xyz, _d), _p(alpha, _d), nc, _p(cx, _d), _p(Z, _d),
                          _p(S, _d), _p(T, _d), _p(V, _d))
    return S[:N, :N].copy(), T[:N, :N].copy(), V[:N, :N].copy()


def charge_repulsion(charge_xyz, charge) -> float:
    cx, Z = _f64(np.reshape(charge_xyz, (-1, 3))), _f64(charge)
    return lib().or_charge_repulsion(Z.shape[0], _p(cx, _d), _p(Z, _d))


class SCF(NamedTuple):
    energies: np.ndarray     # E_k for k = 0, 1, .. (density D_k, Fock matrix F(D_k))
    C: np.ndarray            # [N][O] occupied orbitals of the last density
    eps: np.ndarray          # orbital energies of the last Fock matrix
    F: np.ndarray
    D: np.ndarray
    converged: bool


def scf(S, H, e_charges: float, n_occ: int, jk, max_iter: int = 100,
        e_tol: float = 1e-10, d_tol: float = 1e-8, diis: int = 8) -> SCF:
    """Closed-shell Roothaan-Hall SCF (Sec. 4.1 builds its J and K from the
    Cholesky vectors).  ``jk(C)`` returns J and K of D = C C^T.

    D_0 is the projector on the n_occ lowest solutions of H C = S C e (core
    guess).  Iteration k: F_k = H + 2 J(D_k) - K(D_k),
    E_k = tr(D_k (H + F_k)) + e_charges, e_k = F_k D_k S - S D_k F_k.  Stops
    when |E_k - E_{k-1}| < e_tol and max |e_k| < d_tol.  Otherwise D_{k+1}
    comes from the n_occ lowest solutions of F C = S C e, with F = F_k
    (``diis`` = 0) or Pulay's extrapolation over the last ``diis`` iterations
    (Chem. Phys. Lett. 73, 393 (1980)): F = sum_i c_i F_i with sum_i c_i = 1
    minimising |sum_i c_i e_i| (Frobenius), i.e. the bordered system
    [B 1; 1^T 0] [c; -l] = [0; 1] with B_ij = sum e_i o e_j."""
    import scipy.linalg
    e, V = scipy.linalg.eigh(H, S)
    C = np.ascontiguousarray(V[:, :n_occ])
    energies = []
    conv = False
    F = H.copy()
    Fs, es = [], []
    for _ in range(max_iter):
        D = C @ C.T
        J, K = jk(C)
        F = H + 2.0 * J - K
        E = float(np.sum(D * (H + F))) + e_charges
        energies.append(E)
        comm = F @ D @ S - S @ D @ F
        if len(energies) > 1 and abs(E - energies[-2]) < e_tol and np.abs(comm).max() < d_tol:
            conv = True
            break
        Fx = F
        if diis > 0:
            Fs.append(F)
            es.append(comm)
            if len(Fs) > diis:
                Fs.pop(0)
                es.pop(0)
            n = len(Fs)
            A = np.zeros((n + 1, n + 1))
            for i in range(n):
                for j in range(n):
                    A[i, j] = float(np.sum(es[i] * es[j]))
            A[:n, n] = 1.0
            A[n, :n] = 1.0
            rhs = np.zeros(n + 1)
            rhs[n] = 1.0
            c = np.linalg.solve(A, rhs)[:n]
            Fx = sum(ci * Fi for ci, Fi in zip(c, Fs))
        e, V = scipy.linalg.eigh(Fx, S)
        C = np.ascontiguousarray(V[:, :n_occ])
    return SCF(np.array(energies), C, e, F, C @ C.T, conv)


class ZCD(NamedTuple):
    rc: int
    M: int
    L: np.ndarray        # [M][n] complex
    pivots: np.ndarray   # [M]
    D: np.ndarray        # [n] final residual diagonal (real)


def zdecompose(A, tau: float, max_vectors: Optional[int] = None) -> ZCD:
    """Pivoted Cholesky decomposition of a Hermitian PSD matrix (Sec. 2 in
    complex algebra, the finite-field case of Sec. 7): A ~ sum_K L_K L_K^H."""
    A = np.ascontiguousarray(A, dtype=np.complex128)
    n = A.shape[0]
    if max_vectors is None:
        max_vectors = n
    L = np.zeros((max(1, max_vectors), max(1, n)), dtype=np.complex128)
    piv = np.zeros(max(1, max_vectors), dtype=np.int64)
    D = np.zeros(max(1, n))
    M = ctypes.c_int64()
    rc = lib().or_zdecompose(n, A.ctypes.data_as(_d), float(tau), int(max_vectors),
                             L.ctypes.data_as(_d), _p(piv, _i64), _p(D, _d), ctypes.byref(M))
    m = M.value
    return ZCD(rc, m, L[:m, :n].copy(), piv[:m].copy(), D[:n].copy())

