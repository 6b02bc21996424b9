"""Pins of the FP64 CPU oracle against facts fixed by mathematics.

None of these checks re-types the oracle's own formulas: each compares the
oracle's loop implementation with something built another way -- an explicit
sparse matrix from Kronecker products, a momentum-space closed form, an exact
symmetry, a textbook solve, or the overlap-operator identity satisfied by the
domain-wall operator's effective 4D operator.
"""
import dataclasses

import numpy as np
import scipy.sparse as sp
import pytest

from oracle import cpu, dense, freefield
from oracle import geometry
from paper_2112_01852_amd import inputs as I

SHAMIR = dict(M5=1.8, mf=0.01, b=1.0, c=0.0)
MOBIUS = dict(M5=1.8, mf=0.01, b=1.5, c=0.5)


def _rel(x, y):
    return np.linalg.norm(np.ravel(x - y)) / np.linalg.norm(np.ravel(y))


def _inner(u, v):
    return np.vdot(np.ravel(u), np.ravel(v))


@pytest.fixture(scope="module")
def tiny(oracle_lib):
    a = cpu.Action(L=(2, 2, 2, 2), Ls=4, **MOBIUS)
    U = I.gauge_field(a.L, "haar", 11)
    psi = I.gaussian_spinor(a.L, a.Ls, 12)
    return a, U, psi


# ---------------------------------------------------------------- gamma basis
def test_gamma_clifford_and_chirality(oracle_lib):
    g = cpu.gammas()
    for mu in range(4):
        assert np.allclose(g[mu], g[mu].conj().T), "gamma must be hermitian"
        for nu in range(4):
            anti = g[mu] @ g[nu] + g[nu] @ g[mu]
            assert np.allclose(anti, 2 * np.eye(4) * (mu == nu))
    assert np.allclose(g[4], np.diag([1, 1, -1, -1]))
    gd, g5d = dense.gamma_matrices()
    for mu in range(4):
        assert np.array_equal(g[mu], gd[mu])


# ------------------------------------------------------------- index tables
@pytest.mark.parametrize("L", [(2, 2, 2, 2), (4, 2, 2, 6), (4, 4, 4, 4), (6, 4, 2, 8)])
def test_geometry_invariants(L):
    cb, par, nbr, sign = geometry.tables(L)
    V = int(np.prod(L))
    # cb is a bijection onto 0..V/2-1 within each parity
    for p in (0, 1):
        assert np.array_equal(np.sort(cb[par == p]), np.arange(V // 2))
    # each site is the neighbour of exactly 8 (site, dir) pairs; back-and-forth is identity
    for p in (0, 1):
        q = 1 - p
        counts = np.bincount(nbr[p].ravel(), minlength=V // 2)
        assert np.all(counts == 8)
        for d in range(8):
            back = (d + 4) % 8
            assert np.array_equal(nbr[q][nbr[p][:, d], back], np.arange(V // 2))
            assert np.array_equal(sign[q][nbr[p][:, d], back], sign[p][:, d])
    # the sign is -1 exactly on hops across the t boundary
    assert set(np.unique(sign)) <= {-1, 1}
    n_wrap_t = 2 * (V // L[3])  # forward from t=Lt-1 and backward from t=0
    assert int((sign == -1).sum()) == n_wrap_t


# ------------------------------------------------- brute force (sparse matrix)
def test_dwf_matches_sparse_matrix(tiny):
    a, U, psi = tiny
    D = dense.dwf_matrix(a, U)
    assert _rel(cpu.dwf(a, U, psi).ravel(), D @ psi.ravel()) < 1e-14
    assert _rel(cpu.dwf(a, U, psi, dagger=True).ravel(), D.conj().T @ psi.ravel()) < 1e-14
    H = dense.hop5_matrix(a, U)
    assert _rel(cpu.hop(a, U, psi).ravel(), H @ psi.ravel()) < 1e-14
    assert _rel(cpu.hop(a, U, psi, dagger=True).ravel(), H.conj().T @ psi.ravel()) < 1e-14


def test_eo_blocks_match_sparse_matrix(tiny):
    a, U, psi = tiny
    B = dense.eo_blocks(a, U)
    for p in (0, 1):
        assert _rel(cpu.deo(a, U, psi, p).ravel(), B[(p, 1 - p)] @ psi.ravel()) < 1e-14
        assert _rel(cpu.deo(a, U, psi, p, dagger=True).ravel(),
                    B[(1 - p, p)].conj().T @ psi.ravel()) < 1e-14
        Pp = dense.parity_projector(a, p)
        assert _rel((Pp @ cpu.mee(a, psi).ravel()), B[(p, p)] @ psi.ravel()) < 1e-14
    Mpc, odd = dense.mpc_matrix(a, U)
    po = cpu.restrict(psi, a.L, 1)
    for dag, M in ((False, Mpc), (True, Mpc.conj().T)):
        y = cpu.mpc(a, U, po, dagger=dag).ravel()
        assert _rel(y[odd], M @ po.ravel()[odd]) < 1e-13
        assert np.all(np.delete(y, odd) == 0)


def test_eo_reassembly_equals_full_operator(tiny):
    a, U, psi = tiny
    full = cpu.dwf(a, U, psi)
    pe, po = cpu.restrict(psi, a.L, 0), cpu.restrict(psi, a.L, 1)
    even = cpu.restrict(cpu.mee(a, pe), a.L, 0) + cpu.deo(a, U, po, 0)
    odd = cpu.restrict(cpu.mee(a, po), a.L, 1) + cpu.deo(a, U, pe, 1)
    assert _rel(even + odd, full) < 1e-14


# ------------------------------------------------------------- free field
@pytest.mark.parametrize("n", [(0, 0, 0, 0), (1, 2, 3, 0), (3, 1, 0, 2), (2, 2, 2, 3)])
def test_free_field_wilson_plane_wave(oracle_lib, n):
    """Unit links: D_h on exp(ip.x)u is exp(ip.x) sum_mu [2cos p - 2i g sin p] u."""
    a = cpu.Action(L=(4, 4, 4, 4), Ls=2, **SHAMIR)
    U = I.gauge_field(a.L, "unit", 0)
    p = freefield.momenta(a.L, a.bc, n)
    g, _ = dense.gamma_matrices()
    u = I.gaussian_spinor((1, 1, 1, 1), a.Ls, 21).reshape(a.Ls, 4, 3)
    pw = freefield.plane_wave(a.L, a.Ls, p, u)
    K = sum(2 * np.cos(p[mu]) * np.eye(4) - 2j * np.sin(p[mu]) * g[mu] for mu in range(4))
    expect = freefield.plane_wave(a.L, a.Ls, p, np.einsum("ab,sbc->sac", K, u))
    assert _rel(cpu.hop(a, U, pw), expect) < 1e-14


@pytest.mark.parametrize("n", [(1, 2, 3, 0), (0, 3, 1, 2)])
def test_free_field_wilson_plane_wave_4d(oracle_lib, n):
    """Ls = 1 (4D Wilson fields): D_W(m) on exp(ip.x)u is
    exp(ip.x) [(4 + m - sum_mu cos p) + i sum_mu g sin p] u."""
    a = cpu.Action(L=(4, 6, 4, 4), Ls=1, **SHAMIR)
    U = I.gauge_field(a.L, "unit", 0)
    p = freefield.momenta(a.L, a.bc, n)
    g, _ = dense.gamma_matrices()
    u = I.gaussian_spinor((1, 1, 1, 1), 1, 22).reshape(1, 4, 3)
    pw = freefield.plane_wave(a.L, 1, p, u)
    m = 0.37
    K = (4 + m - sum(np.cos(p))) * np.eye(4) + 1j * sum(np.sin(p[mu]) * g[mu] for mu in range(4))
    expect = freefield.plane_wave(a.L, 1, p, np.einsum("ab,sbc->sac", K, u))
    assert _rel(cpu.wilson(a, U, pw, m), expect) < 1e-14


def test_wilson_matches_sparse_matrix(oracle_lib):
    """The 4D Wilson operator and its adjoint equal (4 + m) - D_h/2 built as a
    sparse Kronecker matrix (adjoint = conjugate transpose)."""
    a = cpu.Action(L=(4, 2, 2, 4), Ls=1, **SHAMIR)
    U = I.gauge_field(a.L, "haar", 61)
    psi = I.gaussian_spinor(a.L, 1, 62)
    m = -0.25
    W = (4 + m) * sp.identity(a.V * 12) - 0.5 * dense.hop_matrix(a.L, U, a.bc)
    for dag in (False, True):
        M = W.conj().T if dag else W
        expect = (M @ psi.ravel()).reshape(psi.shape)
        assert _rel(cpu.wilson(a, U, psi, m, dagger=dag), expect) < 1e-14


def test_wilson_gamma5_hermiticity(oracle_lib):
    """g5 D_W g5 = D_W^dag (an exact symmetry, on Haar links)."""
    a = cpu.Action(L=(4, 4, 2, 2), Ls=1, **SHAMIR)
    U = I.gauge_field(a.L, "haar", 63)
    psi = I.gaussian_spinor(a.L, 1, 64)
    g5 = lambda x: np.concatenate([x[..., :2, :], -x[..., 2:, :]], axis=-2)
    lhs = g5(cpu.wilson(a, U, g5(psi), 0.1))
    assert _rel(lhs, cpu.wilson(a, U, psi, 0.1, dagger=True)) < 1e-14


@pytest.mark.parametrize("params", [SHAMIR, MOBIUS])
def test_free_field_5d_momentum_closed_form(oracle_lib, params):
    a = cpu.Action(L=(4, 4, 2, 6), Ls=6, **params)
    U = I.gauge_field(a.L, "unit", 0)
    rng = np.random.default_rng(5)
    for n in [(1, 3, 0, 2), (0, 1, 1, 5)]:
        p = freefield.momenta(a.L, a.bc, n)
        u = rng.standard_normal((a.Ls, 4, 3)) + 1j * rng.standard_normal((a.Ls, 4, 3))
        pw = freefield.plane_wave(a.L, a.Ls, p, u)
        Dp = freefield.dwf_momentum(a, p)
        expect = freefield.plane_wave(a.L, a.Ls, p, (Dp @ u.reshape(-1, 3)).reshape(a.Ls, 4, 3))
        assert _rel(cpu.dwf(a, U, pw), expect) < 1e-13
        expect_d = freefield.plane_wave(a.L, a.Ls, p,
                                        (Dp.conj().T @ u.reshape(-1, 3)).reshape(a.Ls, 4, 3))
        assert _rel(cpu.dwf(a, U, pw, dagger=True), expect_d) < 1e-13


def test_free_field_wall_modes(oracle_lib):
    """Unit links, periodic boundaries, zero momentum, Shamir, mf = 0: D_W = -M5,
    so D = (1 - M5) - C. Then psi_s = (1 - M5)^(-s) u with u of upper chirality
    (P+) satisfies (D psi)_s = 0 for every s >= 1 and grows towards s = Ls-1,
    while the lower-chirality (P-) vector psi_s = (1 - M5)^s u decays from s = 0
    and is annihilated except on s = Ls-1. This fixes the 5D orientation of C."""
    a = cpu.Action(L=(2, 2, 2, 4), Ls=10, M5=1.8, mf=0.0, b=1.0, c=0.0, bc=(1, 1, 1, 1))
    U = I.gauge_field(a.L, "unit", 0)
    shape = a.spinor_shape()
    rng = np.random.default_rng(7)
    col = rng.standard_normal((2, 3)) + 1j * rng.standard_normal((2, 3))
    up = np.zeros(shape, complex)
    lo = np.zeros(shape, complex)
    for s in range(a.Ls):
        up[s, ..., 0:2, :] = (1 - a.M5) ** (-s) * col
        lo[s, ..., 2:4, :] = (1 - a.M5) ** s * col
    r_up = cpu.dwf(a, U, up)
    r_lo = cpu.dwf(a, U, lo)
    scale = np.abs(up).max()
    assert np.abs(r_up[1:]).max() < 1e-13 * scale
    assert np.abs(r_up[0]).max() > 0.1 * np.abs(up[0]).max()
    assert np.abs(r_lo[:-1]).max() < 1e-13
    assert np.abs(r_lo[-1]).max() > 0.1 * np.abs(lo[-1]).max()
    # the residual norms relative to the vectors are (M5-1)^(Ls-1)-small: wall modes
    assert np.linalg.norm(r_up) / np.linalg.norm(up) < 2 * 0.8 ** (a.Ls - 1)


# -------------------------------------------------------- exact symmetries
def test_gauge_covariance(oracle_lib):
    """D[U^g](g psi) = g D[U] psi with U^g_mu(x) = g(x) U_mu(x) g(x+mu)^dag."""
    a = cpu.Action(L=(4, 2, 2, 4), Ls=4, **MOBIUS)
    U = I.gauge_field(a.L, "haar", 31)
    psi = I.gaussian_spinor(a.L, a.Ls, 32)
    g = I.random_gauge_transform(a.L, 33)
    axis = {0: 3, 1: 2, 2: 1, 3: 0}
    Ug = np.empty_like(U)
    for mu in range(4):
        gfwd = np.roll(g, -1, axis=axis[mu])
        Ug[mu] = g @ U[mu] @ np.conj(np.swapaxes(gfwd, -1, -2))
    gpsi = np.einsum("tzyxab,stzyxsb->stzyxsa".replace("stzyxsb", "stzyxcb").replace(
        "stzyxsa", "stzyxca"), g, psi)
    for dag in (False, True):
        lhs = cpu.dwf(a, Ug, gpsi, dagger=dag)
        rhs = np.einsum("tzyxab,stzyxcb->stzyxca", g, cpu.dwf(a, U, psi, dagger=dag))
        assert _rel(lhs, rhs) < 1e-14


def _gamma5_R5(psi):
    out = psi[::-1].copy()
    out[..., 2:, :] *= -1
    return out


def test_shamir_gamma5_R5_hermiticity(oracle_lib):
    """Shamir: Gamma D Gamma = D^dag with Gamma = gamma5 R5 (R5: s -> Ls-1-s)."""
    a = cpu.Action(L=(4, 2, 2, 4), Ls=6, **SHAMIR)
    U = I.gauge_field(a.L, "haar", 41)
    psi = I.gaussian_spinor(a.L, a.Ls, 42)
    lhs = _gamma5_R5(cpu.dwf(a, U, _gamma5_R5(psi)))
    assert _rel(lhs, cpu.dwf(a, U, psi, dagger=True)) < 1e-14


def test_mobius_gamma5_R5_hermiticity_of_D_Ainv(oracle_lib):
    """Mobius: D A^-1 is Gamma-hermitian (A = b + cC)."""
    a = cpu.Action(L=(2, 2, 2, 2), Ls=4, **MOBIUS)
    U = I.gauge_field(a.L, "haar", 43)
    D = dense.dwf_matrix(a, U).toarray()
    V = int(np.prod(a.L))
    C = dense.c_matrix(V, a.Ls, a.mf).toarray()
    A = a.b * np.eye(D.shape[0]) + a.c * C
    # Gamma from its action on basis vectors through the canonical layout
    n = D.shape[0]
    G = np.stack([_gamma5_R5(e.reshape(a.spinor_shape())).ravel() for e in np.eye(n)], axis=1)
    # the oracle's D must agree with the dense one for the identity to say anything about it
    psi = I.gaussian_spinor(a.L, a.Ls, 44)
    assert _rel(cpu.dwf(a, U, psi).ravel(), D @ psi.ravel()) < 1e-14
    DA = D @ np.linalg.inv(A)
    assert np.abs(G @ DA @ G - DA.conj().T).max() < 1e-12


@pytest.mark.parametrize("params", [SHAMIR, MOBIUS])
def test_adjoint_identities(oracle_lib, params):
    """<chi, O psi> = <O^dag chi, psi> for every operator with a dagger path."""
    a = cpu.Action(L=(4, 2, 2, 4), Ls=4, **params)
    U = I.gauge_field(a.L, "haar", 51)
    psi = I.gaussian_spinor(a.L, a.Ls, 52)
    chi = I.gaussian_spinor(a.L, a.Ls, 53)
    pairs = [
        (lambda v: cpu.dwf(a, U, v), lambda v: cpu.dwf(a, U, v, dagger=True)),
        (lambda v: cpu.hop(a, U, v), lambda v: cpu.hop(a, U, v, dagger=True)),
        (lambda v: cpu.mee(a, v), lambda v: cpu.mee(a, v, dagger=True)),
        (lambda v: cpu.mee(a, v, inverse=True), lambda v: cpu.mee(a, v, dagger=True, inverse=True)),
        (lambda v: cpu.mpc(a, U, cpu.restrict(v, a.L, 1)),
         lambda v: cpu.mpc(a, U, cpu.restrict(v, a.L, 1), dagger=True)),
    ]
    for p in (0, 1):
        pairs.append((lambda v, p=p: cpu.deo(a, U, v, 1 - p),
                      lambda v, p=p: cpu.deo(a, U, v, p, dagger=True)))
    for O, Od in pairs:
        lhs = _inner(chi, O(psi))
        rhs = _inner(Od(chi), psi)
        assert abs(lhs - rhs) < 1e-12 * abs(lhs)


def test_mobius_b1_c0_is_shamir(oracle_lib):
    a = cpu.Action(L=(4, 2, 2, 4), Ls=4, **SHAMIR)
    U = I.gauge_field(a.L, "haar", 61)
    psi = I.gaussian_spinor(a.L, a.Ls, 62)
    # Shamir written out: D = D_W + 1 - C
    dw = (4 - a.M5) * psi - 0.5 * cpu.hop(a, U, psi)
    assert _rel(cpu.dwf(a, U, psi), dw + cpu.local(a, psi, 1.0, -1.0)) < 1e-14


def test_effective_4d_operator_is_polar_overlap(oracle_lib):
    """Mobius domain-wall fermions: with (P^-1 psi)_s = P- psi_s + P+ psi_{s-1},
    [P^-1 D(1)^-1 D(mf) P]_{00} = (1+mf)/2 + (1-mf)/2 g5 eps_Ls(H),
    H = g5 (b+c) D_W (2 + (b-c) D_W)^-1, eps_Ls(H) = [(1+H)^Ls - (1-H)^Ls] /
    [(1+H)^Ls + (1-H)^Ls] (Brower, Neff, Orginos). It fixes the 5D orientation,
    the wall factor and where b and c enter, independently of how D is built."""
    a = cpu.Action(L=(2, 2, 2, 2), Ls=6, M5=1.8, mf=0.05, b=1.5, c=0.5)
    U = I.gauge_field(a.L, "haar", 71)
    shape = a.spinor_shape()
    n = int(np.prod(shape))
    n4 = n // a.Ls

    def matrix(act):
        cols = [cpu.dwf(act, U, e.reshape(shape)).ravel() for e in np.eye(n)]
        return np.stack(cols, axis=1)

    Dm = matrix(a)
    D1 = matrix(dataclasses.replace(a, mf=1.0))
    _, g5 = dense.gamma_matrices()
    V = n4 // 12
    G5 = np.kron(np.eye(V), np.kron(g5, np.eye(3)))
    Pp, Pm = (np.eye(n4) + G5) / 2, (np.eye(n4) - G5) / 2
    Pinv = np.zeros((n, n), complex)
    for s in range(a.Ls):
        Pinv[s * n4:(s + 1) * n4, s * n4:(s + 1) * n4] += Pm
        sm = (s - 1) % a.Ls
        Pinv[s * n4:(s + 1) * n4, sm * n4:(sm + 1) * n4] += Pp
    K = Pinv @ np.linalg.solve(D1, Dm) @ np.linalg.inv(Pinv)
    Deff = K[:n4, :n4]
    # D_W from the hop (the oracle's 4D part is pinned separately above)
    Dh = np.stack([cpu.hop(dataclasses.replace(a, Ls=1), U, e.reshape((1,) + shape[1:])).ravel()
                   for e in np.eye(n4)], axis=1)
    DW = (4 - a.M5) * np.eye(n4) - 0.5 * Dh
    H = G5 @ ((a.b + a.c) * DW) @ np.linalg.inv(2 * np.eye(n4) + (a.b - a.c) * DW)
    Ap = np.linalg.matrix_power(np.eye(n4) + H, a.Ls)
    Am = np.linalg.matrix_power(np.eye(n4) - H, a.Ls)
    eps = np.linalg.solve(Ap + Am, Ap - Am)
    Dov = (1 + a.mf) / 2 * np.eye(n4) + (1 - a.mf) / 2 * G5 @ eps
    assert np.abs(Deff - Dov).max() < 1e-12


# ----------------------------------------------------------- M_ee inverse
@pytest.mark.parametrize("params", [SHAMIR, MOBIUS, dict(M5=1.4, mf=0.1, b=2.0, c=1.0)])
def test_mee_inverse_closed_form(oracle_lib, params):
    """M_ee = alpha + beta C per chirality is alpha + beta S (S = S_d on P+, S_u on
    P-), whose inverse is (1/alpha) sum_k rho^k S^k / (1 + mf rho^Ls), rho = -beta/alpha."""
    a = cpu.Action(L=(2, 2, 2, 2), Ls=8, **params)
    psi = I.gaussian_spinor(a.L, a.Ls, 81)
    Su, Sd = dense.shift_matrices(a.Ls, a.mf)
    al, be = a.alpha(), a.beta()
    rho = -be / al
    out = np.empty_like(psi)
    for S, spins in ((Sd, slice(0, 2)), (Su, slice(2, 4))):
        K = sum(rho ** k * np.linalg.matrix_power(S, k) for k in range(a.Ls)) / (
            al * (1 + a.mf * rho ** a.Ls))
        out[..., spins, :] = np.einsum("st,t...->s...", K, psi[..., spins, :])
    assert _rel(cpu.mee(a, psi, inverse=True), out) < 1e-14
    assert _rel(cpu.mee(a, cpu.mee(a, psi, inverse=True)), psi) < 1e-14
    assert _rel(cpu.mee(a, cpu.mee(a, psi, dagger=True, inverse=True), dagger=True), psi) < 1e-14


# ------------------------------------------------------------------ solver
def test_cg_matches_dense_solve(tiny):
    a, U, psi = tiny
    Mpc, odd = dense.mpc_matrix(a, U)
    b = cpu.restrict(psi, a.L, 1)
    x, it, res = cpu.cg(a, U, b, tol=1e-13, max_iter=1000)
    A = Mpc.conj().T @ Mpc
    xs = np.linalg.solve(A, b.ravel()[odd])
    assert res < 1e-12
    assert _rel(x.ravel()[odd], xs) < 1e-10
    assert it < 200


def test_schur_solve_free_field_matches_fft(oracle_lib):
    a = cpu.Action(L=(4, 4, 4, 4), Ls=4, **MOBIUS)
    U = I.gauge_field(a.L, "unit", 0)
    b = I.gaussian_spinor(a.L, a.Ls, 91)
    x_fft = freefield.fft_solve(a, b)
    assert _rel(cpu.dwf(a, U, x_fft), b) < 1e-13
    x, it, res = cpu.system_solve(a, U, b, tol=1e-12)
    assert res < 1e-12
    assert _rel(x, x_fft) < 1e-10


def test_fft_solve_several_rhs(oracle_lib):
    """The batched form (right-hand sides sharing each momentum's D(p)) solves
    each column: residual through the C++ oracle's D, and equal to the
    one-column form."""
    a = cpu.Action(L=(4, 2, 2, 4), Ls=4, **MOBIUS)
    U = I.gauge_field(a.L, "unit", 0)
    bs = np.stack([I.point_source(a.L, a.Ls, 2, 1), I.gaussian_spinor(a.L, a.Ls, 93)])
    xs = freefield.fft_solve(a, bs)
    assert xs.shape == bs.shape
    for j in range(2):
        assert _rel(cpu.dwf(a, U, xs[j]), bs[j]) < 1e-13
        assert _rel(xs[j], freefield.fft_solve(a, bs[j])) < 1e-14


def test_schur_solve_haar(oracle_lib):
    a = cpu.Action(L=(4, 2, 2, 4), Ls=4, **MOBIUS)
    U = I.gauge_field(a.L, "haar", 92)
    b = I.gaussian_spinor(a.L, a.Ls, 93)
    x, it, res = cpu.system_solve(a, U, b, tol=1e-12)
    assert _rel(cpu.dwf(a, U, x), b) < 1e-9


# --------------------------------------------------------- sampled outputs
@pytest.mark.parametrize("dagger", [False, True])
def test_sampled_sites_match_full_field(oracle_lib, dagger):
    a = cpu.Action(L=(4, 4, 2, 6), Ls=6, **MOBIUS)
    U = I.gauge_field(a.L, "haar", 101)
    psi = I.gaussian_spinor(a.L, a.Ls, 102)
    full = cpu.dwf(a, U, psi, dagger=dagger).reshape(a.Ls * a.V, 4, 3)
    idx = np.random.default_rng(3).choice(a.Ls * a.V, 64, replace=False)
    idx = np.concatenate([idx, [0, a.V - 1, (a.Ls - 1) * a.V, a.Ls * a.V - 1]])
    assert np.abs(cpu.dwf_sites(a, U, psi, idx, dagger=dagger) - full[idx]).max() < 1e-13


# ------------------------------------------------------- streaming probes
def test_su3_product_pins():
    """Brute-force triple loop on a few matrices; SU(3) closure (unitary,
    det 1); the identity is neutral; the product is not commutative."""
    from oracle import streaming
    A = I.haar_su3(6, 81)
    B = I.haar_su3(6, 82)
    C = streaming.su3_mul(A, B)
    for n in range(6):
        for i in range(3):
            for k in range(3):
                ref = sum(A[n, i, j] * B[n, j, k] for j in range(3))
                assert abs(C[n, i, k] - ref) < 1e-15
    eye = np.broadcast_to(np.eye(3), A.shape)
    assert np.allclose(np.conj(np.swapaxes(C, 1, 2)) @ C, eye, atol=1e-14)
    assert np.allclose(np.linalg.det(C), 1.0, atol=1e-14)
    assert np.array_equal(streaming.su3_mul(eye, B), B)
    assert np.abs(streaming.su3_mul(B, A) - C).max() > 1e-3
    assert streaming.FLOPS_PER_SU3_MUL == 27 * 6 + 18 * 2


def test_triad_pins():
    from oracle import streaming
    b = np.arange(7, dtype=np.float64)
    c = np.full(7, 0.5)
    assert np.array_equal(streaming.triad(b, c, 2.0), b + 1.0)
    assert np.array_equal(streaming.triad(b, c, 0.0), b)
