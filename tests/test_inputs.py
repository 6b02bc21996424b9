"""The seeded input generators: shapes, determinism and the group properties
that the link recipes promise."""
import numpy as np

from paper_2112_01852_amd import inputs as I


def test_haar_su3_is_special_unitary():
    U = I.haar_su3(500, 1)
    eye = np.einsum("nab,ncb->nac", U, np.conj(U))
    assert np.abs(eye - np.eye(3)).max() < 1e-14
    assert np.abs(np.linalg.det(U) - 1).max() < 1e-14


def test_haar_su3_is_left_invariant_in_distribution():
    # Haar: E[U] = 0 and E[|U_ab|^2] = 1/3 for every entry
    U = I.haar_su3(40000, 2)
    assert np.abs(U.mean(axis=0)).max() < 0.02
    assert np.abs((np.abs(U) ** 2).mean(axis=0) - 1 / 3).max() < 0.01


def test_smoothed_links_are_special_unitary_and_near_identity():
    U = I.smoothed_su3(2000, 3, eps=0.3)
    eye = np.einsum("nab,ncb->nac", U, np.conj(U))
    assert np.abs(eye - np.eye(3)).max() < 1e-13
    assert np.abs(np.linalg.det(U) - 1).max() < 1e-13
    # exp(i 0.3 H) with |H| ~ 1: mean trace well above the Haar value 0
    assert np.real(np.trace(U, axis1=1, axis2=2)).mean() / 3 > 0.8


def test_determinism_and_shapes():
    L = (4, 2, 2, 6)
    a = I.gauge_field(L, "haar", 5)
    b = I.gauge_field(L, "haar", 5)
    assert a.shape == (4, 6, 2, 2, 4, 3, 3) and np.array_equal(a, b)
    s = I.gaussian_spinor(L, 8, 9, nrhs=3)
    assert s.shape == (3, 8, 6, 2, 2, 4, 4, 3)
    assert np.array_equal(s, I.gaussian_spinor(L, 8, 9, nrhs=3))
    assert not np.array_equal(s, I.gaussian_spinor(L, 8, 10, nrhs=3))
    f = I.gaussian_spinor(L, 8, 9, dtype=np.complex64)
    assert f.dtype == np.complex64


def test_point_source_chiral_wall_injection():
    L, Ls = (4, 4, 4, 4), 8
    for spin in range(4):
        for col in range(3):
            p = I.point_source(L, Ls, spin, col)
            nz = np.argwhere(p != 0)
            assert nz.shape == (1, 7)
            s = Ls - 1 if spin < 2 else 0
            assert tuple(nz[0]) == (s, 0, 0, 0, 0, spin, col)
