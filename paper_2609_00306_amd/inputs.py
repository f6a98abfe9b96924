"""Seeded synthetic inputs: molecules made of normalised s-type Gaussians.

This module only draws random numbers and lays them out; it holds none of the
decomposition's arithmetic (no pair data, no integrals, no screening), so both
the CPU oracle and the GPU library can be fed from it.

Recipe (the paper's workloads are real molecules in real basis sets; these
synthetic stand-ins keep their basis sizes, occupied-orbital counts and
thresholds):

* Centres are drawn one at a time, uniform in the cube [0, L)^3 (L given in
  angstrom, converted with 1 bohr = 0.529177210903 angstrom, CODATA 2018); a
  draw closer than ``min_sep`` bohr to an earlier centre is rejected and drawn
  again.
* Every centre carries one primitive per exponent; functions are ordered
  centre-major, exponent-minor.
* The occupied coefficients C [N][O] are the Q factor of the QR decomposition
  of an N x O matrix of standard normal deviates, drawn after the centres from
  the same generator.
* The generator is ``numpy.random.Generator(PCG64(seed))``.
* For the second-order energy (``mp2_orbitals``): virtual coefficients are
  columns O .. O+V-1 of the Q factor of [C | G], G an N x V matrix of standard
  normal deviates (so they are orthonormal and orthogonal to C); orbital
  energies are sorted uniform deviates, occupied in [-1.5, -0.3] and virtual
  in [0.2, 2.5] hartree; all from ``PCG64(seed + 7919)``.
* Point charges for the SCF (``scf_charges``): charge 2 on each of the first O
  centres, none on the others (their functions are ghost functions), so the
  2 O electrons fill closed-shell He-like sites.
* Complex Hermitian stand-in for finite-field integrals (``hermitian_gram``):
  the Gram matrix F F^H of complex Gaussians with London-like plane-wave
  phases, F[r][q] = s_q exp(-b_q |P_r - c_q|^2) exp(i k_q . P_r) with
  k_q = (B x c_q) / 2; see the function for the distributions.
* Stand-alone transformed vectors for the second-order energy
  (``random_mo_vectors``): B[P][i][a] standard normal deviates scaled by
  sqrt(d_P), d_P falling geometrically from 1 to 1e-6 over P (the shape of a
  decomposition's pivot values), from ``PCG64(seed)``.
"""
from __future__ import annotations

import dataclasses
from typing import Dict, List, Sequence, Tuple

import numpy as np

BOHR_ANGSTROM = 0.529177210903
ANGSTROM_TO_BOHR = 1.0 / BOHR_ANGSTROM

#: four exponents in geometric progression from 0.1 to 10 bohr^-2
GEOMETRIC4 = tuple(float(x) for x in 10.0 ** np.linspace(-1.0, 1.0, 4))


@dataclasses.dataclass
class Molecule:
    """One synthetic molecule; all arrays are C-contiguous float64."""

    name: str
    seed: int
    xyz: np.ndarray      # [N][3] bohr, one row per basis function
    alpha: np.ndarray    # [N] bohr^-2
    C: np.ndarray        # [N][O] occupied coefficients (orthonormal columns)

    @property
    def n_basis(self) -> int:
        return int(self.alpha.shape[0])

    @property
    def n_occ(self) -> int:
        return int(self.C.shape[1])


def draw_centres(rng: np.random.Generator, n_centres: int, box_bohr: float,
                 min_sep: float = 1.0, max_tries: int = 1_000_000) -> np.ndarray:
    """Uniform centres in [0, box)^3 with rejection of close pairs."""
    out = np.empty((n_centres, 3))
    k = 0
    tries = 0
    while k < n_centres:
        tries += 1
        if tries > max_tries:
            raise RuntimeError("could not place centres; box too small for min_sep")
        c = rng.uniform(0.0, box_bohr, size=3)
        if k and np.min(np.sum((out[:k] - c) ** 2, axis=1)) < min_sep * min_sep:
            continue
        out[k] = c
        k += 1
    return out


def make_molecule(n_centres: int, box_angstrom: float, exponents: Sequence[float],
                  n_occ: int, seed: int, min_sep: float = 1.0, name: str = "",
                  rng: np.random.Generator | None = None) -> Molecule:
    if rng is None:
        rng = np.random.Generator(np.random.PCG64(seed))
    centres = draw_centres(rng, n_centres, box_angstrom * ANGSTROM_TO_BOHR, min_sep)
    ne = len(exponents)
    xyz = np.ascontiguousarray(np.repeat(centres, ne, axis=0))
    alpha = np.ascontiguousarray(np.tile(np.asarray(exponents, dtype=np.float64), n_centres))
    n = n_centres * ne
    if n_occ > 0:
        g = rng.standard_normal((n, n_occ))
        q, _ = np.linalg.qr(g)
        C = np.ascontiguousarray(q[:, :n_occ])
    else:
        C = np.zeros((n, 0))
    return Molecule(name=name or f"s{n}", seed=seed, xyz=xyz, alpha=alpha, C=C)


def random_small(seed: int, n_centres: int = 3, exps: Tuple[float, ...] = (0.3, 1.7),
                 box_angstrom: float = 3.0, n_occ: int = 2) -> Molecule:
    """Tiny molecules for brute-force checks."""
    return make_molecule(n_centres, box_angstrom, exps, n_occ, seed,
                         min_sep=0.5, name=f"tiny{seed}")


# Workloads. The thresholds are the ones each workload is run at; 'schwarz'
# is the pair-screening threshold.
CONFIGS: Dict[str, dict] = {
    # the full 1830 x 1830 unique-pair matrix: no screening
    "C1": dict(n_centres=20, box=8.0, exponents=(0.2, 1.0, 5.0), n_occ=10, seed=1,
               taus=(1e-6,), schwarz=0.0),
    "C2": dict(n_centres=100, box=16.0, exponents=GEOMETRIC4, n_occ=50, seed=2,
               taus=(1e-4, 1e-5, 1e-6), schwarz=1e-12),
    "C3": dict(n_centres=250, box=16.0 * (250 / 100) ** (1.0 / 3.0), exponents=GEOMETRIC4,
               n_occ=120, seed=3, taus=(1e-6,), schwarz=1e-12),
    "C5": dict(n_centres=300, box=24.0, exponents=GEOMETRIC4, n_occ=150, seed=5,
               taus=(1e-6,), schwarz=1e-12),
    # the same molecule with every one of the N(N+1)/2 = 720 600 pairs kept
    "C5u": dict(n_centres=300, box=24.0, exponents=GEOMETRIC4, n_occ=150, seed=5,
                taus=(1e-6,), schwarz=0.0),
}

#: batched workload: 64 molecules, seeds 4000+i, c ~ U{13..100} centres,
#: box 16 (c/100)^(1/3) angstrom, O = N // 8, tau = 1e-5
BATCH_C4 = dict(count=64, seed0=4000, cmin=13, cmax=100, exponents=GEOMETRIC4,
                tau=1e-5, schwarz=1e-12)


def config_molecule(name: str) -> Molecule:
    c = CONFIGS[name]
    return make_molecule(c["n_centres"], c["box"], c["exponents"], c["n_occ"], c["seed"],
                         name=name)


def batch_c4(count: int | None = None) -> List[Molecule]:
    b = BATCH_C4
    cnt = b["count"] if count is None else count
    mols = []
    for i in range(cnt):
        seed = b["seed0"] + i
        rng = np.random.Generator(np.random.PCG64(seed))
        c = int(rng.integers(b["cmin"], b["cmax"] + 1))
        nb = c * len(b["exponents"])
        mols.append(make_molecule(c, 16.0 * (c / 100.0) ** (1.0 / 3.0), b["exponents"],
                                  nb // 8, seed, name=f"C4_{i}", rng=rng))
    return mols


def mp2_orbitals(m: Molecule, n_virt: int | None = None):
    """Synthetic orbitals for the second-order energy of molecule ``m``:
    (C_occ [N][O], C_virt [N][V], e_occ [O], e_virt [V]); V defaults to N - O."""
    n, o = m.n_basis, m.n_occ
    v = n - o if n_virt is None else int(n_virt)
    if v < 0 or o + v > n:
        raise ValueError("need n_occ + n_virt <= n_basis")
    rng = np.random.Generator(np.random.PCG64(m.seed + 7919))
    g = rng.standard_normal((n, v))
    q, _ = np.linalg.qr(np.concatenate([m.C, g], axis=1))
    c_virt = np.ascontiguousarray(q[:, o:o + v])
    e_occ = np.sort(rng.uniform(-1.5, -0.3, o))
    e_virt = np.sort(rng.uniform(0.2, 2.5, v))
    return np.ascontiguousarray(m.C), c_virt, e_occ, e_virt


def exponent_block(m: Molecule, flagged: Sequence[int]) -> np.ndarray:
    """Per-function flags [N] (uint8): 1 for the functions whose exponent index
    (position within their centre) is in ``flagged``.  A stand-in for one block
    of a larger basis (restricted-candidate pivoting)."""
    n = m.n_basis
    n_exp = 1
    while n_exp < n and np.array_equal(m.xyz[n_exp], m.xyz[0]):   # functions on centre 0
        n_exp += 1
    keep = set(int(f) for f in flagged)
    return np.array([1 if (k % n_exp) in keep else 0 for k in range(m.n_basis)], dtype=np.uint8)


def scf_charges(m: Molecule, n_occ: int | None = None):
    """Synthetic point charges for the SCF: charge 2 on each of the first
    ``n_occ`` centres (closed-shell He-like sites, 2 n_occ electrons in all)
    and none on the rest, whose functions stay as ghost functions.
    Returns (charge_xyz [n_occ][3], charge [n_occ])."""
    o = m.n_occ if n_occ is None else int(n_occ)
    n = m.n_basis
    n_exp = 1
    while n_exp < n and np.array_equal(m.xyz[n_exp], m.xyz[0]):   # functions on centre 0
        n_exp += 1
    centres = m.xyz[::n_exp]
    if o > centres.shape[0]:
        raise ValueError("more occupied orbitals than centres")
    return np.ascontiguousarray(centres[:o]), np.full(o, 2.0)


def hermitian_gram(n_rows: int, n_fun: int, seed: int, field: float = 0.5,
                   box_bohr: float = 20.0) -> np.ndarray:
    """Seeded complex Hermitian positive semidefinite stand-in for the integral
    matrix of a finite magnetic field: A = F F^H with
    F[r][q] = s_q exp(-b_q |P_r - c_q|^2) exp(i k_q . P_r), k_q = (B x c_q) / 2
    for a field B = (0, 0, field): row "pair centres" P_r and function centres
    c_q uniform in the box, exponents b_q uniform in [0.05, 0.5] bohr^-2,
    weights s_q falling geometrically from 1 to 1e-4.  Returns [n][n] complex128."""
    rng = np.random.Generator(np.random.PCG64(seed))
    P = rng.uniform(0.0, box_bohr, (n_rows, 3))
    c = rng.uniform(0.0, box_bohr, (n_fun, 3))
    b = rng.uniform(0.05, 0.5, n_fun)
    s = np.geomspace(1.0, 1e-4, n_fun) if n_fun > 0 else np.zeros(0)
    k = 0.5 * np.cross(np.array([0.0, 0.0, field]), c)
    d2 = ((P[:, None, :] - c[None, :, :]) ** 2).sum(axis=2)
    F = s[None, :] * np.exp(-b[None, :] * d2) * np.exp(1j * (P @ k.T))
    A = F @ F.conj().T
    A = 0.5 * (A + A.conj().T)            # exactly Hermitian in floating point
    return np.ascontiguousarray(A)


def random_mo_vectors(n_vectors: int, n_occ: int, n_virt: int, seed: int) -> np.ndarray:
    """Seeded stand-in for transformed vectors B [n_vectors][n_occ][n_virt]."""
    rng = np.random.Generator(np.random.PCG64(seed))
    b = rng.standard_normal((n_vectors, n_occ, n_virt))
    if n_vectors > 0:
        d = np.geomspace(1.0, 1e-6, n_vectors)
        b *= np.sqrt(d)[:, None, None]
    return np.ascontiguousarray(b)
