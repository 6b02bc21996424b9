"""The solver's operators on a whole benchmark-size lattice: the one-parity
hop D_eo (one and two right-hand sides) and the Schur operator M_pc (and
M_pc^dag M_pc) of the Mobius action on 16^4 x 16, the multi-right-hand-side
benchmark's volume, with smoothed links (eps 0.3) and Gaussian spinors.
Every element of the output half field is compared with the FP64 oracle on
the same inputs (at this size the oracle takes about a second per operator):
FP64 1e-13, FP32 1e-6, FP16 storage (the mixed solver's inner precision)
5e-3, relative L2 over all reals.
"""
import numpy as np
import pytest

from oracle import cpu
from paper_2112_01852_amd import inputs as I

pytestmark = pytest.mark.gpu

L, LS = (16, 16, 16, 16), 16
MOBIUS = dict(M5=1.8, mf=0.01, b=1.5, c=0.5)
TOL = {0: 1e-13, 1: 1e-6, 2: 5e-3}


def _rel(x, y):
    return float(np.linalg.norm((x - y).ravel()) / np.linalg.norm(y.ravel()))


@pytest.fixture(scope="module")
def big():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2112_01852_amd import qdwf as q
    q.lib()
    a = cpu.Action(L=L, Ls=LS, **MOBIUS)
    U = I.gauge_field(L, "smooth", 3100, eps=0.3)
    psi = I.gaussian_spinor(L, LS, 3101)
    D = q.Dirac(L, LS, **MOBIUS)
    D.set_gauge(U)
    refs = {}
    yield q, a, U, psi, D, refs
    D.close()


def _ref(refs, key, fn):
    if key not in refs:
        refs[key] = fn()
    return refs[key]


@pytest.mark.parametrize("prec,p,dagger", [(1, 0, 0), (1, 1, 0), (1, 0, 1), (1, 1, 1),
                                           (2, 1, 0), (2, 0, 1), (0, 1, 0)])
def test_deo_full_half_field(big, prec, p, dagger):
    q, a, U, psi, D, refs = big
    src = _ref(refs, ("src", 1 - p), lambda: cpu.restrict(psi, L, 1 - p))
    f = D.pack(src, prec, q.QDWF_RIRI, 1 - p)
    out = D.field(prec, p)
    q.qdwf_apply_Deo(D.ctx, out, f, p, dagger, prec, q.QDWF_RIRI)
    got = D.unpack(out, prec, q.QDWF_RIRI, p).cpu().numpy()
    ref = _ref(refs, ("deo", p, dagger), lambda: cpu.deo(a, U, src, p, dagger=bool(dagger)))
    assert _rel(got, ref) < TOL[prec], (prec, p, dagger)


def test_deo_two_right_hand_sides(big):
    q, a, U, psi, D, refs = big
    psi2 = I.gaussian_spinor(L, LS, 3102)
    srcs = np.stack([cpu.restrict(psi, L, 0), cpu.restrict(psi2, L, 0)])
    f = D.pack(srcs, q.QDWF_F32, q.QDWF_RIRI, q.QDWF_EVEN, 2)
    out = D.field(q.QDWF_F32, q.QDWF_ODD, 2)
    q.qdwf_apply_Deo(D.ctx, out, f, q.QDWF_ODD, 0, q.QDWF_F32, q.QDWF_RIRI, 2)
    got = D.unpack(out, q.QDWF_F32, q.QDWF_RIRI, q.QDWF_ODD, 2).cpu().numpy()
    ref0 = _ref(refs, ("deo", 1, 0), lambda: cpu.deo(a, U, srcs[0], 1))
    assert _rel(got[0], ref0) < TOL[1]
    assert _rel(got[1], cpu.deo(a, U, srcs[1], 1)) < TOL[1]


@pytest.mark.parametrize("prec", [1, 2, 0])
def test_mpc_and_normal_operator_full_half_field(big, prec):
    q, a, U, psi, D, refs = big
    src = _ref(refs, ("src", 1), lambda: cpu.restrict(psi, L, 1))
    f = D.pack(src, prec, q.QDWF_RIRI, q.QDWF_ODD)
    ws = D.workspace(q.QDWF_OP_MDAGM, prec)
    for dagger in (0, 1):
        out = D.field(prec, q.QDWF_ODD)
        q.qdwf_apply_Mpc(D.ctx, out, f, dagger, prec, q.QDWF_RIRI, 1, ws)
        got = D.unpack(out, prec, q.QDWF_RIRI, q.QDWF_ODD).cpu().numpy()
        ref = _ref(refs, ("mpc", dagger), lambda: cpu.mpc(a, U, src, dagger=bool(dagger)))
        assert _rel(got, ref) < TOL[prec], (prec, dagger)
    out = D.field(prec, q.QDWF_ODD)
    q.qdwf_apply_MdagM(D.ctx, out, f, prec, q.QDWF_RIRI, 1, ws)
    got = D.unpack(out, prec, q.QDWF_RIRI, q.QDWF_ODD).cpu().numpy()
    ref = _ref(refs, ("mdagm",), lambda: cpu.mpc(a, U, refs[("mpc", 0)], dagger=True))
    assert _rel(got, ref) < TOL[prec], (prec, "MdagM")
