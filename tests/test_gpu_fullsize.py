"""The benchmark workload itself: Mobius D and D^dag on the full 32^4 x 16
lattice, with the benchmark's inputs (Haar links seed 2000, Gaussian spinor
seed 2001, drawn in single precision as the benchmark draws them) and the
launch configuration it times (default shape, RIRI: the t-sweep for FP32
and FP16 storage), with the checkerboard kernel forced as extra cases,
read back on sampled 5D sites and compared with the FP64 oracle evaluated
site by site on the same inputs widened to FP64.

Sampled sites: every combination of the lattice edges (coordinate 0 and
L - 1 in each direction, slices 0 and Ls - 1, where the boundary phase and
the walls act) plus uniformly random sites. Tolerance: relative L2 over the
sampled reals, FP64 1e-13, FP32 1e-6, FP16 storage 5e-3.
"""
import itertools

import numpy as np
import pytest

from oracle import cpu
from paper_2112_01852_amd import inputs as I

pytestmark = pytest.mark.gpu

L, LS = (32, 32, 32, 32), 16
MOBIUS = dict(M5=1.8, mf=0.01, b=1.5, c=0.5)
TOL = {0: 1e-13, 1: 1e-6, 2: 5e-3}


def _sample_sites(n_random=2048, seed=7):
    Lx, Ly, Lz, Lt = L
    V = Lx * Ly * Lz * Lt
    edges = []
    for x, y, z, t, s in itertools.product((0, Lx - 1), (0, Ly - 1), (0, Lz - 1), (0, Lt - 1),
                                           (0, LS - 1)):
        edges.append(s * V + ((t * Lz + z) * Ly + y) * Lx + x)
    rng = np.random.default_rng(seed)
    rand = rng.integers(0, LS * V, size=n_random)
    return np.unique(np.concatenate([np.array(edges, dtype=np.int64), rand]))


@pytest.fixture(scope="module")
def full():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2112_01852_amd import qdwf as q
    q.lib()
    a = cpu.Action(L=L, Ls=LS, **MOBIUS)
    U = I.gauge_field(L, "haar", 2000, dtype=np.complex64).astype(np.complex128)
    psi = I.gaussian_spinor(L, LS, 2001, dtype=np.complex64)
    psi_d = torch.from_numpy(psi).cuda()
    psi = psi.astype(np.complex128)
    D = q.Dirac(L, LS, **MOBIUS)
    D.set_gauge(U)
    idx = _sample_sites()
    yield q, torch, a, U, psi, psi_d, D, idx
    D.close()


@pytest.mark.parametrize("prec,dagger,form", [(1, 0, ""), (1, 1, ""), (1, 0, "0"), (1, 1, "0"),
                                              (0, 0, ""), (2, 0, ""), (2, 0, "0")])
def test_full_lattice_sampled_sites(full, prec, dagger, form, monkeypatch):
    """form: "" the library's default (the t-sweep for FP32 and FP16 storage
    at this size, the checkerboard kernel for FP64), "0" / "1" the
    checkerboard kernel / the t-sweep forced."""
    q, torch, a, U, psi, psi_d, D, idx = full
    if form:
        monkeypatch.setenv("QDWF_SWEEP", form)
    fin = D.field(prec, q.QDWF_FULL, zero=False)
    q.qdwf_pack_spinor(D.ctx, fin, prec, q.QDWF_RIRI, psi_d, q.QDWF_FULL)
    fout = D.field(prec, q.QDWF_FULL, zero=False)
    q.qdwf_apply_D(D.ctx, fout, fin, dagger, prec, q.QDWF_RIRI)
    del fin
    dt = torch.complex128 if prec == 0 else torch.complex64
    out = D.unpack(fout, prec, q.QDWF_RIRI, q.QDWF_FULL, dtype=dt)
    del fout
    got = out.reshape(-1, 4, 3)[torch.from_numpy(idx).cuda()].cpu().numpy().astype(np.complex128)
    del out
    torch.cuda.empty_cache()
    ref = cpu.dwf_sites(a, U, psi, idx, dagger=bool(dagger))
    rel = np.linalg.norm((got - ref).ravel()) / np.linalg.norm(ref.ravel())
    assert rel < TOL[prec], (prec, dagger, rel)
