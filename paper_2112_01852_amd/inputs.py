"""Seeded synthetic inputs for the domain-wall Dirac operator and its solver.

This module is shared by the HIP path, the CPU oracle tests and the benchmark.
It holds no arithmetic of the operator or the solver: it only draws random
gauge links and sources and lays them out in the canonical host layout.

Canonical layouts (row-major numpy arrays):

* gauge field ``U[mu][t][z][y][x][a][b]``: ``mu`` = 0..3 for x, y, z, t;
  ``a`` is the row and ``b`` the column of the 3x3 colour matrix.
* spinor field ``psi[rhs][s][t][z][y][x][spin][colour]`` (``rhs`` omitted for a
  single right-hand side): 4 spin and 3 colour components per 5D site.

The paper (Sections 4.2 and 4.3) measures its kernels on lattices filled by
Grid; those datasets are not available, so random links and Gaussian or point
sources of the same shapes stand in for them.

Random numbers come from NumPy's counter-based Philox bit generator keyed by
the seed, so each (seed, shape) pair always yields the same bytes.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "rng", "haar_su3", "smoothed_su3", "gauge_field", "gaussian_spinor",
    "point_source", "random_gauge_transform", "lattice_volume",
]


def rng(seed: int) -> np.random.Generator:
    """Philox4x32-10 stream for ``seed`` (Salmon et al., SC'11)."""
    return np.random.Generator(np.random.Philox(key=int(seed)))


def lattice_volume(L) -> int:
    return int(L[0]) * int(L[1]) * int(L[2]) * int(L[3])


def _complex_gaussian(g: np.random.Generator, shape, dtype=np.complex128):
    real = np.float64 if dtype == np.complex128 else np.float32
    z = g.standard_normal(tuple(shape) + (2,), dtype=real)
    return z.view(dtype)[..., 0]


def haar_su3(n: int, seed: int, dtype=np.complex128) -> np.ndarray:
    """``n`` Haar-random SU(3) matrices, shape (n, 3, 3).

    Rows 1 and 2 of a complex Gaussian matrix are Gram-Schmidt orthonormalised;
    row 3 is the complex conjugate of their cross product, so the determinant
    is exactly 1 and the distribution is the Haar measure on SU(3).
    """
    g = rng(seed)
    m = _complex_gaussian(g, (n, 2, 3), np.complex128)
    r1 = m[:, 0, :]
    r1 = r1 / np.linalg.norm(r1, axis=1, keepdims=True)
    r2 = m[:, 1, :]
    r2 = r2 - np.sum(np.conj(r1) * r2, axis=1, keepdims=True) * r1
    r2 = r2 / np.linalg.norm(r2, axis=1, keepdims=True)
    r3 = np.conj(np.cross(r1, r2))
    out = np.stack([r1, r2, r3], axis=1)
    return out.astype(dtype, copy=False)


# Gell-Mann matrices lambda_1..lambda_8
_GELL_MANN = np.zeros((8, 3, 3), dtype=np.complex128)
_GELL_MANN[0][0, 1] = _GELL_MANN[0][1, 0] = 1
_GELL_MANN[1][0, 1] = -1j
_GELL_MANN[1][1, 0] = 1j
_GELL_MANN[2][0, 0] = 1
_GELL_MANN[2][1, 1] = -1
_GELL_MANN[3][0, 2] = _GELL_MANN[3][2, 0] = 1
_GELL_MANN[4][0, 2] = -1j
_GELL_MANN[4][2, 0] = 1j
_GELL_MANN[5][1, 2] = _GELL_MANN[5][2, 1] = 1
_GELL_MANN[6][1, 2] = -1j
_GELL_MANN[6][2, 1] = 1j
_GELL_MANN[7][0, 0] = _GELL_MANN[7][1, 1] = 1 / np.sqrt(3)
_GELL_MANN[7][2, 2] = -2 / np.sqrt(3)


def smoothed_su3(n: int, seed: int, eps: float = 0.3, dtype=np.complex128) -> np.ndarray:
    """``n`` matrices U = exp(i*eps*H), H = sum_a h_a lambda_a / 2, h_a ~ N(0,1).

    H is traceless Hermitian, so U is special unitary up to rounding. The
    exponential is taken through the Hermitian eigendecomposition of H.
    """
    g = rng(seed)
    h = g.standard_normal((n, 8))
    H = np.einsum("na,aij->nij", h, _GELL_MANN) * 0.5
    w, v = np.linalg.eigh(H)
    ph = np.exp(1j * eps * w)
    U = np.einsum("nij,nj,nkj->nik", v, ph, np.conj(v))
    return U.astype(dtype, copy=False)


def gauge_field(L, kind: str = "haar", seed: int = 0, eps: float = 0.3,
                dtype=np.complex128) -> np.ndarray:
    """Gauge field in canonical layout ``U[4][T][Z][Y][X][3][3]``.

    ``kind`` is ``"haar"`` (Haar-random links), ``"smooth"`` (exp(i*eps*H)) or
    ``"unit"`` (all links the identity: the free field).
    """
    Lx, Ly, Lz, Lt = (int(v) for v in L)
    n = 4 * lattice_volume(L)
    if kind == "haar":
        U = haar_su3(n, seed, dtype=dtype)
    elif kind == "smooth":
        U = smoothed_su3(n, seed, eps=eps, dtype=dtype)
    elif kind == "unit":
        U = np.broadcast_to(np.eye(3, dtype=dtype), (n, 3, 3)).copy()
    else:
        raise ValueError(f"unknown gauge kind {kind!r}")
    return U.reshape(4, Lt, Lz, Ly, Lx, 3, 3)


def gaussian_spinor(L, Ls: int, seed: int, nrhs: int | None = None,
                    dtype=np.complex128) -> np.ndarray:
    """Complex Gaussian spinor (re, im ~ N(0,1) i.i.d.) on every 5D site.

    Shape ``[Ls][T][Z][Y][X][4][3]``, or ``[nrhs][Ls][...]`` when ``nrhs`` is
    given.
    """
    Lx, Ly, Lz, Lt = (int(v) for v in L)
    shape = (int(Ls), Lt, Lz, Ly, Lx, 4, 3)
    if nrhs is not None:
        shape = (int(nrhs),) + shape
    return _complex_gaussian(rng(seed), shape, dtype)


def point_source(L, Ls: int, spin: int, colour: int, dtype=np.complex128) -> np.ndarray:
    """Unit source at the 4D origin for one spin and colour.

    The 5D slice follows the chiral wall injection: spins 0 and 1 (upper
    chirality) are placed on s = Ls-1, spins 2 and 3 (lower chirality) on s = 0.
    """
    Lx, Ly, Lz, Lt = (int(v) for v in L)
    psi = np.zeros((int(Ls), Lt, Lz, Ly, Lx, 4, 3), dtype=dtype)
    s = int(Ls) - 1 if spin < 2 else 0
    psi[s, 0, 0, 0, 0, spin, colour] = 1.0
    return psi


def random_gauge_transform(L, seed: int, dtype=np.complex128) -> np.ndarray:
    """A Haar-random SU(3) matrix per 4D site, shape ``[T][Z][Y][X][3][3]``."""
    Lx, Ly, Lz, Lt = (int(v) for v in L)
    return haar_su3(lattice_volume(L), seed, dtype=dtype).reshape(Lt, Lz, Ly, Lx, 3, 3)
