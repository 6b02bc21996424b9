"""The t-sweep traversal of the full operator D and D^dag (Ls = 16, interleaved
layout, 32- and 16-bit storage, Lx in {8, 16, 24, 32}) against the FP64
oracle, element by element, through the C ABI.

The lattices cover every row width the sweep takes, the degenerate Lt = 2
(the -t and +t neighbours are the same site), rows whose t extent is split
into chunks (few rows: each chunk starts its own window), (y, z) extents that
do not fill a whole patch of rows, and several right-hand sides. The sweep
is forced on (QDWF_SWEEP=1; by default it serves 16- and 32-wide rows). The
same calls with it switched off (QDWF_SWEEP=0, the checkerboard kernel) must
agree with the oracle too, and with the sweep to rounding.

Tolerances (relative L2 over all reals): FP32 1e-6, FP16/BF16 storage 5e-3.
"""
import numpy as np
import pytest

from oracle import cpu
from paper_2112_01852_amd import inputs as I

pytestmark = pytest.mark.gpu

TOL = {1: 1e-6, 2: 5e-3, 3: 5e-3}
MOBIUS = dict(M5=1.8, mf=0.01, b=1.5, c=0.5)
SHAMIR = dict(M5=1.8, mf=0.01, b=1.0, c=0.0)
CASES = [
    ((8, 4, 2, 4), MOBIUS, 1),
    ((16, 2, 4, 6), MOBIUS, 1),
    ((24, 2, 2, 2), SHAMIR, 1),    # Lt = 2: -t and +t are the same site
    ((8, 2, 2, 16), MOBIUS, 1),    # few rows: t split into chunks of 4
    ((32, 2, 2, 4), MOBIUS, 2),    # widest row, two right-hand sides
    ((8, 6, 6, 4), MOBIUS, 1),     # (y, z) patches of 2 x 2 rows
]


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
    L, params, nrhs = CASES[request.param]
    a = cpu.Action(L=L, Ls=16, **params)
    U = I.gauge_field(L, "haar", 900 + request.param)
    psi = I.gaussian_spinor(L, 16, 910 + request.param, nrhs=nrhs)
    D = q.Dirac(L, 16, **params)
    D.set_gauge(U)
    yield q, a, U, psi, D, nrhs
    D.close()


@pytest.fixture(autouse=True)
def force_sweep(monkeypatch):
    """The sweep is the default only for FP32 in 16- and 32-wide rows and FP16
    in 32-wide rows: force it."""
    monkeypatch.setenv("QDWF_SWEEP", "1")


def _apply(q, D, psi, prec, dagger, nrhs):
    f = D.pack(psi, prec, q.QDWF_RIRI, q.QDWF_FULL, nrhs)
    out = D.field(prec, q.QDWF_FULL, nrhs)
    q.qdwf_apply_D(D.ctx, out, f, dagger, prec, q.QDWF_RIRI, nrhs)
    return D.unpack(out, prec, q.QDWF_RIRI, q.QDWF_FULL, nrhs).cpu().numpy()


@pytest.mark.parametrize("prec", [1, 2, 3])
@pytest.mark.parametrize("dagger", [0, 1])
def test_sweep_matches_oracle(case, prec, dagger):
    q, a, U, psi, D, nrhs = case
    got = _apply(q, D, psi, prec, dagger, nrhs)
    if nrhs == 1:
        assert _rel(got, cpu.dwf(a, U, psi, dagger=bool(dagger))) < TOL[prec]
    else:
        for j in range(nrhs):
            assert _rel(got[j], cpu.dwf(a, U, psi[j], dagger=bool(dagger))) < TOL[prec]


@pytest.mark.parametrize("dagger", [0, 1])
def test_sweep_agrees_with_checkerboard_kernel(case, dagger, monkeypatch):
    q, a, U, psi, D, nrhs = case
    sweep = _apply(q, D, psi, 1, dagger, nrhs)
    monkeypatch.setenv("QDWF_SWEEP", "0")
    cbk = _apply(q, D, psi, 1, dagger, nrhs)
    monkeypatch.setenv("QDWF_SWEEP", "1")
    # same arithmetic in another order: FP32 rounding apart
    assert _rel(sweep, cbk) < 1e-6
    ref = cpu.dwf(a, U, psi if nrhs == 1 else psi[0], dagger=bool(dagger))
    assert _rel(cbk if nrhs == 1 else cbk[0], ref) < TOL[1]


def test_sweep_repeatable_and_gauge_update(q):
    """Two launches give identical bits; a new gauge field is picked up (the
    doubled links are rebuilt by qdwf_set_gauge)."""
    L = (16, 2, 2, 4)
    a = cpu.Action(L=L, Ls=16, **MOBIUS)
    psi = I.gaussian_spinor(L, 16, 931)
    D = q.Dirac(L, 16, **MOBIUS)
    D.set_gauge(I.gauge_field(L, "haar", 930))
    r1 = _apply(q, D, psi, 1, 0, 1)
    r2 = _apply(q, D, psi, 1, 0, 1)
    assert np.array_equal(r1, r2)
    U2 = I.gauge_field(L, "haar", 932)
    D.set_gauge(U2)
    r3 = _apply(q, D, psi, 1, 0, 1)
    assert _rel(r3, cpu.dwf(a, U2, psi)) < TOL[1]
    D.close()
