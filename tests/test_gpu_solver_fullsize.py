"""Solves at the benchmark's own volumes, checked against the oracle rather
than against the library's own residual:

* 24^4 x 16, smoothed links (eps 0.3, seed 3000), Gaussian odd-site source
  (seed 3001), the even-odd normal equations at tol 1e-10 with each inner
  precision, the launch configuration the benchmark times (graph replay,
  8 iterations per check): the residual of the returned x is recomputed with
  the oracle's M_pc and M_pc^dag in FP64 and must be <= 1.5e-10;
* 16^4 x 16 with unit links, the full system D x = b for a point source and
  a Gaussian source in one batched call: x must match the exact free-field
  solution (Fourier transform, one dense solve per momentum) to 1e-8
  relative;
* the multi-right-hand-side workload exactly (16^4 x 16, Haar links seed
  4000, 12 point sources plus 12 Gaussian sources seeds 4001..4012, the full
  system, FP32 inner): every column's |D x - b| / |b| recomputed with the
  oracle's D must be <= 1.5e-10.
"""
import numpy as np
import pytest

from oracle import cpu
from oracle import freefield
from paper_2112_01852_amd import inputs as I

pytestmark = pytest.mark.gpu

MOBIUS = dict(M5=1.8, mf=0.01, b=1.5, c=0.5)
_EXACT = {}   # free-field solutions, shared by the inner precisions (about 30 s each)


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


@pytest.fixture(scope="module")
def cg24(q):
    L, Ls = (24, 24, 24, 24), 16
    a = cpu.Action(L=L, Ls=Ls, **MOBIUS)
    U = I.gauge_field(L, "smooth", 3000, eps=0.3)
    b = cpu.restrict(I.gaussian_spinor(L, Ls, 3001), L, 1)
    D = q.Dirac(L, Ls, **MOBIUS)
    D.set_gauge(U)
    sols = {}
    yield q, a, U, b, D, sols
    D.close()


@pytest.mark.parametrize("inner", [0, 1, 2, 3])
def test_cg_24x24x24x24x16_oracle_residual(cg24, inner):
    q, a, U, b, D, sols = cg24
    print(f"24^4x16 NORMAL_PC solve, inner {q.PREC_NAME[inner]}", flush=True)
    bo = D.pack(b, q.QDWF_F64, q.QDWF_RIRI, q.QDWF_ODD)
    x = D.field(q.QDWF_F64, q.QDWF_ODD)
    ws = D.workspace(q.QDWF_OP_SOLVE, inner)
    prm = q.solve_params(inner_prec=inner, layout=q.QDWF_RIRI, tol=1e-10, check_every=8,
                         use_graph=1)
    rc, st = q.qdwf_solve(D.ctx, x, bo, 1, prm, ws)
    assert rc == q.QDWF_OK, q.qdwf_last_error()
    xs = D.unpack(x, q.QDWF_F64, q.QDWF_RIRI, q.QDWF_ODD).cpu().numpy()
    del ws, x, bo
    r = b - cpu.mpc(a, U, cpu.mpc(a, U, xs), dagger=True)
    res = float(np.linalg.norm(r) / np.linalg.norm(b))
    print(f"  iterations {st.iterations}, reliable updates {st.reliable_updates}, "
          f"library residual {st.true_residual:.3e}, oracle residual {res:.3e}", flush=True)
    assert st.true_residual <= 1e-10
    assert res <= 1.5e-10, res
    sols[inner] = xs
    if 0 in sols and inner != 0:
        # two solutions at residual 1e-10 differ by at most cond(A) * 2e-10;
        # recorded, not asserted (the condition number here is not pinned)
        print(f"  |x - x_fp64| / |x_fp64| = {_rel(xs, sols[0]):.3e}", flush=True)


@pytest.mark.parametrize("inner", [0, 1])
def test_full_solve_free_field_16x16x16x16x16(q, inner):
    L, Ls = (16, 16, 16, 16), 16
    a = cpu.Action(L=L, Ls=Ls, **MOBIUS)
    U = I.gauge_field(L, "unit")
    srcs = np.stack([I.point_source(L, Ls, 0, 0), I.point_source(L, Ls, 3, 2),
                     I.gaussian_spinor(L, Ls, 4101)])
    print(f"16^4x16 unit links, FULL system, 3 rhs, inner {q.PREC_NAME[inner]}", flush=True)
    D = q.Dirac(L, Ls, **MOBIUS)
    D.set_gauge(U)
    nrhs = srcs.shape[0]
    bf = D.pack(srcs, q.QDWF_F64, q.QDWF_RIRI, q.QDWF_FULL, nrhs)
    x = D.field(q.QDWF_F64, q.QDWF_FULL, nrhs)
    ws = D.workspace(q.QDWF_OP_SOLVE, inner, nrhs)
    prm = q.solve_params(system=q.QDWF_SYS_FULL, inner_prec=inner, tol=1e-10, check_every=8,
                         use_graph=1)
    rc, st = q.qdwf_solve(D.ctx, x, bf, nrhs, prm, ws)
    assert rc == q.QDWF_OK, q.qdwf_last_error()
    xs = D.unpack(x, q.QDWF_F64, q.QDWF_RIRI, q.QDWF_FULL, nrhs).cpu().numpy()
    D.close()
    assert st.full_residual <= 1e-10
    if "free16" not in _EXACT:
        _EXACT["free16"] = freefield.fft_solve(a, srcs)
    exact = _EXACT["free16"]
    for j in range(nrhs):
        rel = _rel(xs[j], exact[j])
        print(f"  rhs {j}: |x - x_exact| / |x_exact| = {rel:.3e}", flush=True)
        assert rel <= 1e-8, (j, rel)


def test_multi_rhs_workload_oracle_residual(q):
    L, Ls = (16, 16, 16, 16), 16
    a = cpu.Action(L=L, Ls=Ls, **MOBIUS)
    U = I.gauge_field(L, "haar", 4000)
    srcs = [I.point_source(L, Ls, sp, c) for sp in range(4) for c in range(3)]
    srcs += [I.gaussian_spinor(L, Ls, 4001 + j) for j in range(12)]
    b = np.stack(srcs)
    del srcs
    nrhs = b.shape[0]
    print("16^4x16 Haar, 12 point + 12 Gaussian sources, FULL system, FP32 inner", flush=True)
    D = q.Dirac(L, Ls, **MOBIUS)
    D.set_gauge(U)
    bf = D.pack(b, q.QDWF_F64, q.QDWF_RIRI, q.QDWF_FULL, nrhs)
    x = D.field(q.QDWF_F64, q.QDWF_FULL, nrhs)
    ws = D.workspace(q.QDWF_OP_SOLVE, q.QDWF_F32, nrhs)
    prm = q.solve_params(system=q.QDWF_SYS_FULL, inner_prec=q.QDWF_F32, tol=1e-10,
                         check_every=8, use_graph=1)
    rc, st = q.qdwf_solve(D.ctx, x, bf, nrhs, prm, ws)
    assert rc == q.QDWF_OK, q.qdwf_last_error()
    assert st.converged == nrhs
    xs = D.unpack(x, q.QDWF_F64, q.QDWF_RIRI, q.QDWF_FULL, nrhs).cpu().numpy()
    D.close()
    worst = 0.0
    for j in range(nrhs):
        r = cpu.dwf(a, U, xs[j]) - b[j]
        worst = max(worst, float(np.linalg.norm(r) / np.linalg.norm(b[j])))
    print(f"  iterations {st.iterations}, worst oracle |Dx-b|/|b| {worst:.3e}", flush=True)
    assert worst <= 1.5e-10, worst
