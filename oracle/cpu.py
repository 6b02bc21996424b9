"""ctypes front end of the FP64 C++ oracle (``dwf_oracle.cpp``).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Every function takes canonical complex128 numpy arrays:
``U[4][T][Z][Y][X][3][3]`` and ``psi[Ls][T][Z][Y][X][4][3]``. Half-lattice
quantities are full-size arrays that are zero on the other 4D parity.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "dwf_oracle.cpp")
_LIB = os.path.join(_HERE, "liboracle_dwf.so")


def build(force: bool = True) -> str:
    """Compile the oracle with g++ (OpenMP, no FMA contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call([
            "g++", "-O2", "-std=c++17", "-fopenmp", "-ffp-contract=off", "-fPIC", "-shared",
            _SRC, "-o", tmp])
        os.replace(tmp, _LIB)
    return _LIB


class _Action(ctypes.Structure):
    _fields_ = [("L", ctypes.c_int32 * 4), ("Ls", ctypes.c_int32), ("bc", ctypes.c_int32 * 4),
                ("M5", ctypes.c_double), ("mf", ctypes.c_double),
                ("b", ctypes.c_double), ("c", ctypes.c_double)]


@dataclass(frozen=True)
class Action:
    """Lattice extents (x, y, z, t), Ls, boundary factors and Mobius parameters."""
    L: tuple
    Ls: int
    M5: float = 1.8
    mf: float = 0.01
    b: float = 1.0
    c: float = 0.0
    bc: tuple = (1, 1, 1, -1)

    def c_struct(self) -> _Action:
        a = _Action()
        a.L[:] = [int(v) for v in self.L]
        a.Ls = int(self.Ls)
        a.bc[:] = [int(v) for v in self.bc]
        a.M5, a.mf, a.b, a.c = float(self.M5), float(self.mf), float(self.b), float(self.c)
        return a

    @property
    def V(self) -> int:
        return int(np.prod(self.L))

    def spinor_shape(self):
        Lx, Ly, Lz, Lt = self.L
        return (self.Ls, Lt, Lz, Ly, Lx, 4, 3)

    def alpha(self) -> float:
        return self.b * (4.0 - self.M5) + 1.0

    def beta(self) -> float:
        return self.c * (4.0 - self.M5) - 1.0


_lib = None


def load(path: str):
    """ctypes handle of an oracle library at ``path`` with its signatures set."""
    L = ctypes.CDLL(path)
    P = ctypes.c_void_p
    A = ctypes.POINTER(_Action)
    I = ctypes.c_int
    L.or_gammas.argtypes = [P]
    L.or_hop.argtypes = [A, P, P, P, I]
    L.or_dwf.argtypes = [A, P, P, P, I]
    L.or_dwf_sites.argtypes = [A, P, P, P, ctypes.c_int64, P, I]
    L.or_local.argtypes = [A, P, P, ctypes.c_double, ctypes.c_double, I]
    L.or_mee.argtypes = [A, P, P, I, I]
    L.or_deo.argtypes = [A, P, P, P, I, I]
    L.or_mpc.argtypes = [A, P, P, P, I]
    L.or_cg.argtypes = [A, P, P, P, ctypes.c_double, I, ctypes.POINTER(ctypes.c_double)]
    L.or_cg.restype = I
    return L


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        _lib = load(_LIB)
    return _lib


def _c128(x) -> np.ndarray:
    return np.ascontiguousarray(x, dtype=np.complex128)


def _ptr(x: np.ndarray):
    return ctypes.c_void_p(x.ctypes.data)


def gammas() -> np.ndarray:
    """(5, 4, 4): gamma_x, gamma_y, gamma_z, gamma_t, gamma5 as the oracle uses them."""
    out = np.zeros((5, 4, 4), dtype=np.complex128)
    lib().or_gammas(_ptr(out))
    return out


def hop(a: Action, U, psi, dagger: bool = False) -> np.ndarray:
    """D_h psi (or D_h^dag psi) on every slice s."""
    U, psi = _c128(U), _c128(psi)
    out = np.empty_like(psi)
    lib().or_hop(ctypes.byref(a.c_struct()), _ptr(U), _ptr(psi), _ptr(out), int(dagger))
    return out


def wilson(a: Action, U, psi, mass: float, dagger: bool = False) -> np.ndarray:
    """Wilson operator (4 + mass) psi - D_h psi / 2 on every slice s, or with
    D_h^dag: the standalone Wilson Dslash operator (Section 4.1, Table 1).
    Only a.L and a.bc are used."""
    return (4.0 + float(mass)) * _c128(psi) - 0.5 * hop(a, U, psi, dagger)


def dwf(a: Action, U, psi, dagger: bool = False) -> np.ndarray:
    """Mobius domain-wall operator D psi = D_W A psi + B psi (or D^dag psi)."""
    U, psi = _c128(U), _c128(psi)
    out = np.empty_like(psi)
    lib().or_dwf(ctypes.byref(a.c_struct()), _ptr(U), _ptr(psi), _ptr(out), int(dagger))
    return out


def dwf_sites(a: Action, U, psi, idx, dagger: bool = False) -> np.ndarray:
    """D psi (or D^dag psi) at 5D sites ``idx = s*V + lex``; returns (n, 4, 3)."""
    U, psi = _c128(U), _c128(psi)
    idx = np.ascontiguousarray(idx, dtype=np.int64)
    out = np.empty((idx.size, 4, 3), dtype=np.complex128)
    lib().or_dwf_sites(ctypes.byref(a.c_struct()), _ptr(U), _ptr(psi), _ptr(idx),
                       ctypes.c_int64(idx.size), _ptr(out), int(dagger))
    return out


def local(a: Action, psi, x0: float, x1: float, dagger: bool = False) -> np.ndarray:
    """x0 psi + x1 C psi (or with C^dag)."""
    psi = _c128(psi)
    out = np.empty_like(psi)
    lib().or_local(ctypes.byref(a.c_struct()), _ptr(psi), _ptr(out), float(x0), float(x1),
                   int(dagger))
    return out


def mee(a: Action, psi, dagger: bool = False, inverse: bool = False) -> np.ndarray:
    """M_ee psi, M_ee^-1 psi, or their adjoints, at every 4D site."""
    psi = _c128(psi)
    out = np.empty_like(psi)
    lib().or_mee(ctypes.byref(a.c_struct()), _ptr(psi), _ptr(out), int(dagger), int(inverse))
    return out


def deo(a: Action, U, psi, out_parity: int, dagger: bool = False) -> np.ndarray:
    """Off-diagonal block into parity ``out_parity`` from parity ``1-out_parity``.

    dagger=False: M_{p,q} psi; dagger=True: (M_{q,p})^dag psi.
    """
    U, psi = _c128(U), _c128(psi)
    out = np.empty_like(psi)
    lib().or_deo(ctypes.byref(a.c_struct()), _ptr(U), _ptr(psi), _ptr(out), int(out_parity),
                 int(dagger))
    return out


def mpc(a: Action, U, psi, dagger: bool = False) -> np.ndarray:
    """Schur complement M_pc = M_oo - M_oe M_ee^-1 M_eo (or adjoint) on odd sites."""
    U, psi = _c128(U), _c128(psi)
    out = np.empty_like(psi)
    lib().or_mpc(ctypes.byref(a.c_struct()), _ptr(U), _ptr(psi), _ptr(out), int(dagger))
    return out


def cg(a: Action, U, b, tol: float = 1e-13, max_iter: int = 100000):
    """CG on M_pc^dag M_pc x = b (odd sites). Returns (x, iterations, true residual)."""
    U, b = _c128(U), _c128(b)
    x = np.empty_like(b)
    res = ctypes.c_double(0.0)
    it = lib().or_cg(ctypes.byref(a.c_struct()), _ptr(U), _ptr(b), _ptr(x), float(tol),
                     int(max_iter), ctypes.byref(res))
    return x, int(it), float(res.value)


def parity_mask(L) -> np.ndarray:
    """Boolean [T][Z][Y][X] array: True on odd sites ((x+y+z+t) odd)."""
    Lx, Ly, Lz, Lt = L
    t, z, y, x = np.meshgrid(np.arange(Lt), np.arange(Lz), np.arange(Ly), np.arange(Lx),
                             indexing="ij")
    return ((x + y + z + t) % 2) == 1


def restrict(psi: np.ndarray, L, parity: int) -> np.ndarray:
    """Copy of ``psi`` with the sites of the other parity set to zero."""
    odd = parity_mask(L)
    keep = odd if parity == 1 else ~odd
    out = np.array(psi, copy=True)
    out[..., ~keep, :, :] = 0
    return out


def system_solve(a: Action, U, b_full, tol: float = 1e-13, max_iter: int = 100000):
    """Solve D x = b on the full lattice by the even-odd Schur complement.

    b'_o = b_o - M_oe M_ee^-1 b_e; CG on M_pc^dag M_pc x_o = M_pc^dag b'_o;
    x_e = M_ee^-1 (b_e - M_eo x_o).
    """
    be = restrict(b_full, a.L, 0)
    bo = restrict(b_full, a.L, 1)
    t = restrict(mee(a, be, inverse=True), a.L, 0)
    bprime = bo - deo(a, U, t, 1)
    rhs = mpc(a, U, bprime, dagger=True)
    xo, it, res = cg(a, U, rhs, tol=tol, max_iter=max_iter)
    xe = restrict(mee(a, be - deo(a, U, xo, 0), inverse=True), a.L, 0)
    return xe + xo, it, res
