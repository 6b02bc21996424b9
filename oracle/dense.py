"""Sparse-matrix construction of the domain-wall operators for small lattices.

TEST INFRASTRUCTURE ONLY (see the package docstring).

A second, independent construction of the operators that ``dwf_oracle.cpp``
applies with loops: here every operator is an explicit (scipy.sparse) matrix
assembled from Kronecker products, with the gamma matrices built from Pauli
matrices, neighbours from ``numpy.roll`` of the coordinate grid, and every
adjoint taken as the conjugate transpose of the matrix (so it checks the
oracle's separately written dagger paths).

Vector index = ((s*V + lex)*4 + spin)*3 + colour, i.e. the canonical spinor
array ``psi[s][t][z][y][x][spin][colour]`` flattened.

Conventions (the same readings as the oracle): DeGrand-Rossi basis,
D_W = (4 - M5) - D_h/2 with D_h = sum_mu [(1-g_mu) U_mu(x) T_+mu + (1+g_mu)
U_mu(x-mu)^dag T_-mu], C = P- S_u + P+ S_d, D = D_W (b + cC) + (1 - C),
M_ee = the 4D-local part of D, Schur complement on odd sites.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

SIGMA = [np.array([[0, 1], [1, 0]], dtype=complex),
         np.array([[0, -1j], [1j, 0]], dtype=complex),
         np.array([[1, 0], [0, -1]], dtype=complex)]


def gamma_matrices():
    """DeGrand-Rossi chiral basis built from Pauli matrices.

    gamma_k = [[0, s_k i sigma_k], [-s_k i sigma_k, 0]] with s = (+1, -1, +1)
    for k = x, y, z; gamma_t = [[0, 1], [1, 0]]; gamma5 = gx gy gz gt.
    """
    Z = np.zeros((2, 2), dtype=complex)
    I2 = np.eye(2, dtype=complex)
    g = []
    for k, sk in zip(range(3), (1, -1, 1)):
        m = sk * 1j * SIGMA[k]
        g.append(np.block([[Z, m], [-m, Z]]))
    g.append(np.block([[Z, I2], [I2, Z]]))
    g5 = g[0] @ g[1] @ g[2] @ g[3]
    return g, g5


def _grid(L):
    Lx, Ly, Lz, Lt = L
    t, z, y, x = np.meshgrid(np.arange(Lt), np.arange(Lz), np.arange(Ly), np.arange(Lx),
                             indexing="ij")
    return (x, y, z, t)


_AXIS = {0: 3, 1: 2, 2: 1, 3: 0}   # numpy axis of direction mu in [t][z][y][x]


def hop_matrix(L, U, bc=(1, 1, 1, -1)) -> sp.csr_matrix:
    """Sparse 12V x 12V matrix of D_h on one slice."""
    L = tuple(int(v) for v in L)
    V = int(np.prod(L))
    g, _ = gamma_matrices()
    lex = np.arange(V).reshape(L[3], L[2], L[1], L[0])
    coords = _grid(L)
    U = np.asarray(U, dtype=complex).reshape(4, L[3], L[2], L[1], L[0], 3, 3)
    rows, cols, vals = [], [], []
    I4 = np.eye(4, dtype=complex)
    shape = (V, 12, 12)
    for mu in range(4):
        ax = _AXIS[mu]
        fwd = np.roll(lex, -1, axis=ax)          # lex of x + mu
        bwd = np.roll(lex, +1, axis=ax)          # lex of x - mu
        eta_f = np.where(coords[mu] == L[mu] - 1, bc[mu], 1).astype(float)
        eta_b = np.where(coords[mu] == 0, bc[mu], 1).astype(float)
        Uf = U[mu]                                   # U_mu(x)
        Ub = np.conj(np.swapaxes(np.roll(U[mu], +1, axis=ax), -1, -2))  # U_mu(x-mu)^dag
        for nb, eta, link, proj in ((fwd, eta_f, Uf, I4 - g[mu]), (bwd, eta_b, Ub, I4 + g[mu])):
            blk = np.einsum("ab,...cd->...acbd", proj, link).reshape(-1, 12, 12)
            blk = blk * eta.reshape(-1)[:, None, None]
            r = np.broadcast_to(lex.reshape(-1)[:, None, None] * 12
                                + np.arange(12)[None, :, None], shape)
            c = np.broadcast_to(nb.reshape(-1)[:, None, None] * 12
                                + np.arange(12)[None, None, :], shape)
            rows.append(r.reshape(-1))
            cols.append(c.reshape(-1))
            vals.append(blk.reshape(-1))
    return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                         shape=(12 * V, 12 * V))


def shift_matrices(Ls: int, mf: float):
    """S_u and S_d as dense Ls x Ls matrices (wall entries -mf)."""
    Su = np.zeros((Ls, Ls))
    Sd = np.zeros((Ls, Ls))
    for s in range(Ls):
        if s + 1 < Ls:
            Su[s, s + 1] = 1.0
        else:
            Su[s, 0] = -mf
        if s - 1 >= 0:
            Sd[s, s - 1] = 1.0
        else:
            Sd[s, Ls - 1] = -mf
    return Su, Sd


def chiral_projectors():
    _, g5 = gamma_matrices()
    I4 = np.eye(4)
    return (I4 + g5) / 2, (I4 - g5) / 2


def c_matrix(V: int, Ls: int, mf: float) -> sp.csr_matrix:
    """C = P- S_u + P+ S_d on the 5D space."""
    Su, Sd = shift_matrices(Ls, mf)
    Pp, Pm = chiral_projectors()
    IV3 = sp.identity(V, format="csr")
    I3 = np.eye(3)
    return (sp.kron(Su, sp.kron(IV3, np.kron(Pm, I3))) +
            sp.kron(Sd, sp.kron(IV3, np.kron(Pp, I3)))).tocsr()


def dwf_matrix(a, U) -> sp.csr_matrix:
    """D = D_W (b + cC) + (1 - C) as a sparse 12 V Ls square matrix."""
    V = int(np.prod(a.L))
    n4 = 12 * V
    Dh = hop_matrix(a.L, U, a.bc)
    DW = (4.0 - a.M5) * sp.identity(n4) - 0.5 * Dh
    C = c_matrix(V, a.Ls, a.mf)
    I5 = sp.identity(n4 * a.Ls)
    A = a.b * I5 + a.c * C
    return (sp.kron(sp.identity(a.Ls), DW) @ A + (I5 - C)).tocsr()


def hop5_matrix(a, U) -> sp.csr_matrix:
    """D_h on every slice: kron(1_Ls, D_h)."""
    return sp.kron(sp.identity(a.Ls), hop_matrix(a.L, U, a.bc)).tocsr()


def parity_projector(a, parity: int) -> sp.csr_matrix:
    Lx, Ly, Lz, Lt = a.L
    x, y, z, t = _grid(a.L)
    on = (((x + y + z + t) % 2) == parity).reshape(-1).astype(float)
    d = np.tile(np.repeat(on, 12), a.Ls)
    return sp.diags(d).tocsr()


def mee_matrix(a) -> sp.csr_matrix:
    """4D-local part of D: alpha + beta C (acts site by site)."""
    V = int(np.prod(a.L))
    n = 12 * V * a.Ls
    C = c_matrix(V, a.Ls, a.mf)
    return (a.alpha() * sp.identity(n) + a.beta() * C).tocsr()


def eo_blocks(a, U):
    """The four parity blocks of D: dict keyed by (p, q) -> P_p D P_q."""
    D = dwf_matrix(a, U)
    P = [parity_projector(a, 0), parity_projector(a, 1)]
    return {(p, q): (P[p] @ D @ P[q]).tocsr() for p in (0, 1) for q in (0, 1)}


def mpc_matrix(a, U) -> np.ndarray:
    """Dense M_pc = M_oo - M_oe M_ee^-1 M_eo restricted to odd-site indices.

    Returns (M_pc, odd_index) where odd_index selects the odd rows/columns of
    the full vector.
    """
    B = eo_blocks(a, U)
    P1 = parity_projector(a, 1).diagonal().astype(bool)
    P0 = ~P1
    Mee = B[(0, 0)].toarray()[np.ix_(P0, P0)]
    Moo = B[(1, 1)].toarray()[np.ix_(P1, P1)]
    Moe = B[(1, 0)].toarray()[np.ix_(P1, P0)]
    Meo = B[(0, 1)].toarray()[np.ix_(P0, P1)]
    return Moo - Moe @ np.linalg.solve(Mee, Meo), np.nonzero(P1)[0]
