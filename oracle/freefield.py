"""Unit-link (free-field) closed forms in momentum space.

TEST INFRASTRUCTURE ONLY (see the package docstring).

With all links equal to 1 the 4D hop is diagonal in momentum: acting on
psi(x) = exp(i p.x) u it gives exp(i p.x) sum_mu [2 cos p_mu - 2 i g_mu sin p_mu] u,
so D_W = (4 - M5) - D_h/2 becomes the 4x4 matrix
W(p) = (4 - M5 - sum_mu cos p_mu) + i sum_mu g_mu sin p_mu.
Allowed momenta are p_mu = 2 pi n / L_mu in periodic directions and
(2n + 1) pi / L_mu in antiperiodic ones. The domain-wall operator at momentum
p is the (4 Ls) x (4 Ls) matrix D(p) = W(p) (b + c C) + (1 - C) on (s, spin).
"""
from __future__ import annotations

import numpy as np

from .dense import gamma_matrices, shift_matrices, chiral_projectors


def momenta(L, bc, n):
    """Momentum vector for integer mode numbers n = (nx, ny, nz, nt)."""
    return np.array([(2 * np.pi * n[mu] + (np.pi if bc[mu] < 0 else 0.0)) / L[mu]
                     for mu in range(4)])


def wilson_momentum(p, M5: float) -> np.ndarray:
    g, _ = gamma_matrices()
    W = (4.0 - M5 - np.sum(np.cos(p))) * np.eye(4, dtype=complex)
    for mu in range(4):
        W = W + 1j * np.sin(p[mu]) * g[mu]
    return W


def c_momentum(Ls: int, mf: float) -> np.ndarray:
    Su, Sd = shift_matrices(Ls, mf)
    Pp, Pm = chiral_projectors()
    return np.kron(Su, Pm) + np.kron(Sd, Pp)


def dwf_momentum(a, p, C=None) -> np.ndarray:
    """D(p) on (s, spin), shape (4 Ls, 4 Ls). C (which does not depend on p)
    may be passed in when many momenta are evaluated."""
    W = wilson_momentum(p, a.M5)
    if C is None:
        C = c_momentum(a.Ls, a.mf)
    I = np.eye(4 * a.Ls)
    return np.kron(np.eye(a.Ls), W) @ (a.b * I + a.c * C) + (I - C)


def plane_wave(L, Ls, p, u) -> np.ndarray:
    """psi[s][t][z][y][x][spin][colour] = exp(i p.x) u[s][spin][colour]."""
    Lx, Ly, Lz, Lt = L
    t, z, y, x = np.meshgrid(np.arange(Lt), np.arange(Lz), np.arange(Ly), np.arange(Lx),
                             indexing="ij")
    ph = np.exp(1j * (p[0] * x + p[1] * y + p[2] * z + p[3] * t))
    return ph[None, :, :, :, :, None, None] * np.asarray(u)[:, None, None, None, None, :, :]


def fft_solve(a, b: np.ndarray) -> np.ndarray:
    """Exact solution of D x = b for unit links, by Fourier transform.

    Antiperiodic directions are made periodic by the twist exp(-i pi x_mu / L_mu);
    each momentum then needs one (4 Ls) x (4 Ls) solve per colour. b may carry
    a leading axis of several right-hand sides, which share each momentum's
    D(p).
    """
    if b.ndim == 8:
        n = b.shape[0]
        cols = np.moveaxis(b, 0, -1).reshape(b.shape[1:-1] + (3 * n,))
        x = _fft_solve_cols(a, cols)
        return np.moveaxis(x.reshape(b.shape[1:-1] + (3, n)), -1, 0)
    return _fft_solve_cols(a, b)


def _fft_solve_cols(a, b: np.ndarray) -> np.ndarray:
    Lx, Ly, Lz, Lt = a.L
    L = a.L
    grids = np.meshgrid(np.arange(Lt), np.arange(Lz), np.arange(Ly), np.arange(Lx), indexing="ij")
    coord = {3: grids[0], 2: grids[1], 1: grids[2], 0: grids[3]}
    tw = np.ones((Lt, Lz, Ly, Lx), dtype=complex)
    for mu in range(4):
        if a.bc[mu] < 0:
            tw = tw * np.exp(-1j * np.pi * coord[mu] / L[mu])
    bt = b * tw[None, :, :, :, :, None, None]
    B = np.fft.fftn(bt, axes=(1, 2, 3, 4))
    X = np.empty_like(B)
    C = c_momentum(a.Ls, a.mf)
    nc = B.shape[-1]
    for kt in range(Lt):
        for kz in range(Lz):
            for ky in range(Ly):
                for kx in range(Lx):
                    p = momenta(L, a.bc, (kx, ky, kz, kt))
                    D = dwf_momentum(a, p, C)
                    rhs = B[:, kt, kz, ky, kx, :, :].reshape(4 * a.Ls, nc)
                    X[:, kt, kz, ky, kx, :, :] = np.linalg.solve(D, rhs).reshape(a.Ls, 4, nc)
    xt = np.fft.ifftn(X, axes=(1, 2, 3, 4))
    return xt / tw[None, :, :, :, :, None, None]
