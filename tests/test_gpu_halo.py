"""Domain decomposition emulated on one GPU (qdwf_apply_D_split): D applied
through face packing, half-spinor exchange, an interior hop with the cut
links zeroed and a boundary update, for several slab counts, against the
FP64 oracle (same tolerances as the operator parity tests) and against the
undivided qdwf_apply_D.
"""
import numpy as np
import pytest

from oracle import cpu
from paper_2112_01852_amd import inputs as I

pytestmark = pytest.mark.gpu

TOL = {0: 1e-13, 1: 1e-6, 2: 5e-3, 3: 5e-3}
MOBIUS = dict(M5=1.8, mf=0.01, b=1.5, c=0.5)
CASES = [((4, 4, 4, 8), 8, (1, 2, 4)), ((6, 2, 4, 12), 16, (2, 3, 6)), ((4, 2, 2, 6), 12, (3,))]


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


@pytest.mark.parametrize("case", range(len(CASES)))
@pytest.mark.parametrize("prec", [0, 1, 3])
@pytest.mark.parametrize("layout", [0, 1])
def test_split_equals_oracle(q, case, prec, layout):
    import torch
    L, Ls, rank_list = CASES[case]
    a = cpu.Action(L=L, Ls=Ls, **MOBIUS)
    U = I.gauge_field(L, "haar", 800 + case)
    psi = I.gaussian_spinor(L, Ls, 810 + case)
    ref = cpu.dwf(a, U, psi)
    D = q.Dirac(L, Ls, **MOBIUS)
    D.set_gauge(U)
    f = D.pack(psi, prec, layout, q.QDWF_FULL)
    whole = D.field(prec, q.QDWF_FULL)
    q.qdwf_apply_D(D.ctx, whole, f, 0, prec, layout)
    for ranks in rank_list:
        ws = torch.empty(q.qdwf_split_workspace_bytes(D.ctx, ranks, prec), dtype=torch.uint8,
                         device="cuda")
        q.qdwf_split_prepare(D.ctx, ranks, prec, ws)
        out = D.field(prec, q.QDWF_FULL)
        q.qdwf_apply_D_split(D.ctx, out, f, ranks, prec, layout, ws)
        got = D.unpack(out, prec, layout, q.QDWF_FULL).cpu().numpy()
        assert _rel(got, ref) < TOL[prec], (ranks, _rel(got, ref))
        if prec == 0:
            w = D.unpack(whole, prec, layout, q.QDWF_FULL).cpu().numpy()
            assert _rel(got, w) < 1e-14
    D.close()


def test_split_arguments(q):
    D = q.Dirac((4, 4, 4, 6), 8, **MOBIUS)
    assert q.qdwf_split_workspace_bytes(D.ctx, 4, q.QDWF_F32) == 0      # 4 does not divide 6
    assert q.qdwf_split_workspace_bytes(D.ctx, 6, q.QDWF_F32) == 0      # slabs of one slice
    f = D.field(q.QDWF_F32, q.QDWF_FULL)
    import torch
    ws = torch.empty(q.qdwf_split_workspace_bytes(D.ctx, 3, q.QDWF_F32), dtype=torch.uint8,
                     device="cuda")
    with pytest.raises(q.QdwfError):
        q.qdwf_split_prepare(D.ctx, 3, q.QDWF_F32, ws)                # gauge not set
    D.set_gauge(I.gauge_field((4, 4, 4, 6), "haar", 820))
    with pytest.raises(q.QdwfError):
        q.qdwf_apply_D_split(D.ctx, f, f, 3, q.QDWF_F32, q.QDWF_RIRI, ws)   # aliasing
    with pytest.raises(q.QdwfError):
        q.qdwf_apply_D_split(D.ctx, D.field(q.QDWF_F32, q.QDWF_FULL), f, 4, q.QDWF_F32,
                             q.QDWF_RIRI, ws)                           # ranks
    D.close()
