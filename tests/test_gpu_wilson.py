"""The Wilson Dslash kernel (qdwf_apply_Dh) and Wilson operator
(qdwf_apply_Dw) against the FP64 oracle, element by element, on 4D fields
(Ls = 1) and on every slice of 5D fields.

Tolerances (relative L2 over all reals, oracle on the original FP64 inputs):
FP64 1e-13, FP32 1e-6, FP16/BF16 storage 5e-3. The lattices leave a partial
last block of 256 lanes and, at 6x6x8x6, partial traversal tiles; 4D fields
(Ls = 1) are blocked over 16 sites in the RIRI layout.
"""
import numpy as np
import pytest

from oracle import cpu
from paper_2112_01852_amd import inputs as I

pytestmark = pytest.mark.gpu

TOL = {0: 1e-13, 1: 1e-6, 2: 5e-3, 3: 5e-3}
SHAMIR = dict(M5=1.8, mf=0.01, b=1.0, c=0.0)
CASES = [((6, 4, 4, 6), 1), ((6, 6, 8, 6), 1), ((4, 4, 2, 6), 8), ((4, 2, 4, 4), 16)]


def _rel(x, y):
    return float(np.linalg.norm((x - y).ravel()) / np.linalg.norm(y.ravel()))


@pytest.fixture(scope="module")
def q():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2112_01852_amd import qdwf
    qdwf.lib()
    return qdwf


@pytest.fixture(scope="module", params=range(len(CASES)))
def case(q, request):
    L, Ls = CASES[request.param]
    a = cpu.Action(L=L, Ls=Ls, **SHAMIR)
    U = I.gauge_field(L, "haar", 700 + request.param)
    psi = I.gaussian_spinor(L, Ls, 710 + request.param)
    D = q.Dirac(L, Ls, **SHAMIR)
    D.set_gauge(U)
    yield q, a, U, psi, D
    D.close()


@pytest.mark.parametrize("prec", [0, 1, 2, 3])
@pytest.mark.parametrize("layout", [0, 1])
@pytest.mark.parametrize("dagger", [0, 1])
def test_hop_full(case, prec, layout, dagger):
    q, a, U, psi, D = case
    f = D.pack(psi, prec, layout, q.QDWF_FULL)
    out = D.field(prec, q.QDWF_FULL)
    q.qdwf_apply_Dh(D.ctx, out, f, q.QDWF_FULL, dagger, prec, layout)
    got = D.unpack(out, prec, layout, q.QDWF_FULL).cpu().numpy()
    assert _rel(got, cpu.hop(a, U, psi, dagger=bool(dagger))) < TOL[prec]


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("parity", [0, 1])
@pytest.mark.parametrize("dagger", [0, 1])
def test_hop_one_parity(case, prec, parity, dagger):
    q, a, U, psi, D = case
    src = cpu.restrict(psi, a.L, 1 - parity)
    fin = D.pack(src, prec, q.QDWF_RIRI, 1 - parity)
    out = D.field(prec, parity)
    q.qdwf_apply_Dh(D.ctx, out, fin, parity, dagger, prec, q.QDWF_RIRI)
    got = D.unpack(out, prec, q.QDWF_RIRI, parity).cpu().numpy()
    ref = cpu.restrict(cpu.hop(a, U, src, dagger=bool(dagger)), a.L, parity)
    assert _rel(got, ref) < TOL[prec]


@pytest.mark.parametrize("prec", [0, 1, 3])
@pytest.mark.parametrize("dagger", [0, 1])
def test_wilson_operator(case, prec, dagger):
    q, a, U, psi, D = case
    mass = -0.3
    f = D.pack(psi, prec, q.QDWF_RIRI, q.QDWF_FULL)
    out = D.field(prec, q.QDWF_FULL)
    q.qdwf_apply_Dw(D.ctx, out, f, mass, dagger, prec, q.QDWF_RIRI)
    got = D.unpack(out, prec, q.QDWF_RIRI, q.QDWF_FULL).cpu().numpy()
    assert _rel(got, cpu.wilson(a, U, psi, mass, dagger=bool(dagger))) < TOL[prec]


def test_multi_rhs_columns(q):
    L, Ls, nrhs = (6, 4, 4, 6), 1, 3
    a = cpu.Action(L=L, Ls=Ls, **SHAMIR)
    U = I.gauge_field(L, "haar", 720)
    psis = I.gaussian_spinor(L, Ls, 721, nrhs=nrhs)
    D = q.Dirac(L, Ls, **SHAMIR)
    D.set_gauge(U)
    f = D.pack(psis, q.QDWF_F64, q.QDWF_RIRI, q.QDWF_FULL, nrhs)
    out = D.field(q.QDWF_F64, q.QDWF_FULL, nrhs)
    q.qdwf_apply_Dw(D.ctx, out, f, 0.2, 0, q.QDWF_F64, q.QDWF_RIRI, nrhs)
    got = D.unpack(out, q.QDWF_F64, q.QDWF_RIRI, q.QDWF_FULL, nrhs).cpu().numpy()
    for r in range(nrhs):
        assert _rel(got[r], cpu.wilson(a, U, psis[r], 0.2)) < TOL[0]
    D.close()


def test_gauge_update_reaches_lane_major_links(q):
    """4D contexts read lane-major copies of the links, rebuilt by every
    qdwf_set_gauge: a second gauge field must replace the first."""
    L = (8, 4, 4, 6)
    a = cpu.Action(L=L, Ls=1, **SHAMIR)
    psi = I.gaussian_spinor(L, 1, 741)
    D = q.Dirac(L, 1, **SHAMIR)
    for seed in (742, 743):
        U = I.gauge_field(L, "haar", seed)
        D.set_gauge(U)
        for prec in (0, 1, 3):
            f = D.pack(psi, prec, q.QDWF_RIRI, q.QDWF_FULL)
            out = D.field(prec, q.QDWF_FULL)
            q.qdwf_apply_Dw(D.ctx, out, f, 0.1, 1, prec, q.QDWF_RIRI)
            got = D.unpack(out, prec, q.QDWF_RIRI, q.QDWF_FULL).cpu().numpy()
            assert _rel(got, cpu.wilson(a, U, psi, 0.1, dagger=True)) < TOL[prec]
    D.close()


def test_invalid_arguments(q):
    D = q.Dirac((4, 4, 4, 4), 1, **SHAMIR)
    D.set_gauge(I.gauge_field((4, 4, 4, 4), "haar", 730))
    f = D.field(q.QDWF_F32, q.QDWF_FULL)
    with pytest.raises(q.QdwfError):
        q.qdwf_apply_Dh(D.ctx, f, f, q.QDWF_FULL, 0, q.QDWF_F32, q.QDWF_RIRI)   # aliasing
    g = D.field(q.QDWF_F32, q.QDWF_FULL)
    with pytest.raises(q.QdwfError):
        q.qdwf_apply_Dh(D.ctx, g, f, 5, 0, q.QDWF_F32, q.QDWF_RIRI)             # bad subset
    with pytest.raises(q.QdwfError):
        q.qdwf_apply_Dw(D.ctx, g, f, float("nan"), 0, q.QDWF_F32, q.QDWF_RIRI)
    D.close()
    with pytest.raises(q.QdwfError):
        q.qdwf_create(q.make_action((6, 6, 10, 6), 1))   # 1080 sites per parity: not a multiple of 16
