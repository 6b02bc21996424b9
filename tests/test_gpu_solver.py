"""CG solves on the GPU against the oracle's CG and the FP64 true residual.

Every solve must reach an FP64 true residual <= 1e-10 and agree with the
oracle's solution (solved to 1e-13) to 1e-8 relative; the lattices and links
used here have condition numbers of a few hundred, so 1e-10 in the residual
bounds the solution error well below 1e-8.
"""
import numpy as np
import pytest

from oracle import cpu
from paper_2112_01852_amd import inputs as I

pytestmark = pytest.mark.gpu

MOBIUS = dict(M5=1.8, mf=0.01, b=1.5, c=0.5)


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
def setup(q):
    L, Ls = (4, 4, 4, 6), 8
    a = cpu.Action(L=L, Ls=Ls, **MOBIUS)
    U = I.gauge_field(L, "smooth", 3000, eps=0.3)
    b = cpu.restrict(I.gaussian_spinor(L, Ls, 3001), L, 1)
    x_ref, it, res = cpu.cg(a, U, b, tol=1e-13)
    assert res < 1e-12
    D = q.Dirac(L, Ls, **MOBIUS)
    D.set_gauge(U)
    yield q, a, U, b, x_ref, D
    D.close()


def _solve(q, D, b, inner, layout=1, nrhs=1, **kw):
    bf = D.pack(b, q.QDWF_F64, layout, q.QDWF_ODD, nrhs)
    x = D.field(q.QDWF_F64, q.QDWF_ODD, nrhs)
    ws = D.workspace(q.QDWF_OP_SOLVE, inner, nrhs)
    prm = q.solve_params(inner_prec=inner, layout=layout, tol=1e-10, **kw)
    rc, st = q.qdwf_solve(D.ctx, x, bf, nrhs, prm, ws)
    return rc, st, D.unpack(x, q.QDWF_F64, layout, q.QDWF_ODD, nrhs).cpu().numpy()


@pytest.mark.parametrize("inner", [0, 1, 2, 3])
@pytest.mark.parametrize("layout", [0, 1])
def test_solve_normal_pc(setup, inner, layout):
    q, a, U, b, x_ref, D = setup
    rc, st, x = _solve(q, D, b, inner, layout)
    assert rc == q.QDWF_OK, q.qdwf_last_error()
    assert st.true_residual <= 1e-10
    # independent FP64 residual with the oracle operator
    r = b - cpu.mpc(a, U, cpu.mpc(a, U, x), dagger=True)
    assert np.linalg.norm(r) / np.linalg.norm(b) <= 1.5e-10
    assert _rel(x, x_ref) <= 1e-8
    if inner != 0:
        assert st.reliable_updates >= 1
        # the inner iteration must track the FP64 one: an inner operator that
        # disagreed with the outer one would still end at the true residual,
        # but only after many restarts
        rc0, st0, _ = _solve(q, D, b, 0, layout)
        assert st.iterations <= 1.5 * st0.iterations + 10, (st.iterations, st0.iterations)


def test_multi_rhs_solve_matches_single(setup):
    q, a, U, b, x_ref, D = setup
    nrhs = 3
    bs = np.stack([b, 2.0 * cpu.restrict(I.gaussian_spinor(a.L, a.Ls, 9), a.L, 1), 0.5 * b])
    rc, st, xs = _solve(q, D, bs, 1, nrhs=nrhs)
    assert rc == q.QDWF_OK and st.converged == nrhs
    for j in range(nrhs):
        rc1, st1, x1 = _solve(q, D, bs[j], 1)
        assert np.array_equal(xs[j], x1), f"rhs {j} differs between batched and alone"


@pytest.mark.parametrize("inner", [0, 1, 2, 3])
def test_graph_replay_matches_eager_and_oracle(setup, inner):
    q, a, U, b, x_ref, D = setup
    rc0, st0, x0 = _solve(q, D, b, inner, use_graph=0, check_every=5)
    rc1, st1, x1 = _solve(q, D, b, inner, use_graph=1, check_every=5)
    assert rc0 == rc1 == q.QDWF_OK
    assert st0.iterations == st1.iterations
    assert np.array_equal(x0, x1)
    # the replayed solve against the oracle: its CG solution and its operator
    assert _rel(x1, x_ref) <= 1e-8
    r = b - cpu.mpc(a, U, cpu.mpc(a, U, x1), dagger=True)
    assert np.linalg.norm(r) / np.linalg.norm(b) <= 1.5e-10
    # a second solve reuses nothing stale
    rc2, st2, x2 = _solve(q, D, b, inner, use_graph=1, check_every=5)
    assert np.array_equal(x1, x2)


def test_full_system_point_source(q):
    L, Ls = (4, 4, 4, 4), 8
    a = cpu.Action(L=L, Ls=Ls, **MOBIUS)
    U = I.gauge_field(L, "smooth", 4000, eps=0.3)
    src = I.point_source(L, Ls, 2, 1)
    D = q.Dirac(L, Ls, **MOBIUS)
    D.set_gauge(U)
    for inner in (0, 1):
        bf = D.pack(src, q.QDWF_F64, 1, q.QDWF_FULL)
        x = D.field(q.QDWF_F64, q.QDWF_FULL)
        ws = D.workspace(q.QDWF_OP_SOLVE, inner)
        prm = q.solve_params(system=q.QDWF_SYS_FULL, inner_prec=inner, tol=1e-10)
        rc, st = q.qdwf_solve(D.ctx, x, bf, 1, prm, ws)
        assert rc == q.QDWF_OK, q.qdwf_last_error()
        xs = D.unpack(x, q.QDWF_F64, 1, q.QDWF_FULL).cpu().numpy()
        assert st.full_residual <= 1e-10
        r = cpu.dwf(a, U, xs) - src
        assert np.linalg.norm(r) / np.linalg.norm(src) <= 1.5e-10
    D.close()


def test_not_converged_and_nan_are_reported(setup):
    q, a, U, b, x_ref, D = setup
    rc, st, x = _solve(q, D, b, 0, max_iter=3, check_every=1)
    assert rc == q.QDWF_ENOTCONV
    assert st.iterations == 3 and st.true_residual > 1e-10
    bad = b.copy()
    bad[np.unravel_index(np.argmax(np.abs(b)), b.shape)] = np.nan
    rc, st, x = _solve(q, D, bad, 1)
    assert rc == q.QDWF_ENAN


@pytest.mark.parametrize("inner", [0, 2])
def test_solve_bitwise_same_for_any_round_length(setup, inner):
    """x takes the steps of up to eight iterations in one pass, and a group
    of iterations never spans two rounds of check_every: rounds of 1, 3, 8
    and 13 iterations (groups cut at every length from 1 to 8), replayed
    from graphs or launched eagerly, must take the same iterations and
    reliable updates and give bitwise the same solution."""
    q, a, U, b, x_ref, D = setup
    runs = [_solve(q, D, b, inner, use_graph=g, check_every=ce)
            for ce, g in ((1, 0), (3, 1), (8, 1), (13, 1), (13, 0))]
    rc0, st0, x0 = runs[0]
    assert rc0 == q.QDWF_OK, q.qdwf_last_error()
    for rc, st, x in runs[1:]:
        assert rc == q.QDWF_OK
        assert (st.iterations, st.reliable_updates) == (st0.iterations, st0.reliable_updates)
        assert np.array_equal(x, x0)
    assert _rel(x0, x_ref) <= 1e-8


@pytest.mark.parametrize("check_every", [1, 8, 13])
@pytest.mark.parametrize("inner", [0, 2])
def test_max_iter_not_whole_groups(setup, inner, check_every):
    """A solve stopped by max_iter = 11, a whole number neither of groups of
    iterations nor of rounds, holds exactly 11 CG steps: in FP64 its x is the
    oracle's CG stopped after 11 iterations, and the reported true residual
    is that of the returned x."""
    q, a, U, b, x_ref, D = setup
    rc, st, x = _solve(q, D, b, inner, max_iter=11, check_every=check_every)
    assert rc == q.QDWF_ENOTCONV
    assert st.iterations == 11
    if inner == 0:
        x11, it, res11 = cpu.cg(a, U, b, tol=1e-30, max_iter=11)
        assert it == 11
        assert _rel(x, x11) <= 1e-10
    r = b - cpu.mpc(a, U, cpu.mpc(a, U, x), dagger=True)
    res = np.linalg.norm(r) / np.linalg.norm(b)
    assert res > 1e-10
    assert abs(res - st.true_residual) <= 1e-6 * res


@pytest.mark.parametrize("inner", [0, 2])
def test_fused_cg_step_independent_of_hop_shape(q, tmp_path, inner):
    """The hops carry the CG step's sums as one value per checkerboard site,
    so the solve must be bitwise the same for every launch shape of the hop:
    fewer threads per block, and blocks that hold two or four right-hand
    sides (whose lanes update r only while their own right-hand side runs;
    the three sources below pause for reliable updates at different
    iterations). Checked against the oracle's residual as well."""
    import os
    import torch
    L, Ls, nrhs = (4, 4, 4, 8), 16, 3
    a = cpu.Action(L=L, Ls=Ls, **MOBIUS)
    U = I.gauge_field(L, "smooth", 3100, eps=0.3)
    bs = np.stack([cpu.restrict(I.gaussian_spinor(L, Ls, 3101 + j), L, 1) for j in range(nrhs)])
    arch = torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]

    def run(cache_shape=None, threads=None):
        env = {}
        if cache_shape is not None:
            env["QDWF_TUNE_CACHE"] = str(tmp_path / f"shape_{cache_shape[0]}_{cache_shape[1]}.jsonl")
        if threads is not None:
            env["QDWF_HOP_THREADS"] = str(threads)
        old = {k: os.environ.get(k) for k in env}
        os.environ.update(env)
        try:
            D = q.Dirac(L, Ls, **MOBIUS)
            if cache_shape is not None:
                tr = q.qdwf_traversal(D.ctx)
                t = tr["tile"]
                with open(env["QDWF_TUNE_CACHE"], "w") as f:
                    for prec in {inner, q.QDWF_F64}:
                        for dag in (0, 1):
                            key = (f"{L[0]}x{L[1]}x{L[2]}x{L[3]}_Ls{Ls}_p{prec}_l{q.QDWF_RIRI}_d{dag}"
                                   f"_n{nrhs}_t{t[0]}.{t[1]}.{t[2]}.{t[3]}_o{tr['split']}.{tr['sweep']}_{arch}")
                            f.write(f'{{"key": "{key}", "threads": {cache_shape[0]}, "nrb": {cache_shape[1]}, '
                                    f'"xcd": 1, "lds_pad": 0, "sweep": 0, "ms": 1.0}}\n')
                got = q.qdwf_tuned_shape(D.ctx, inner, q.QDWF_RIRI, 1, nrhs)
                assert (got["threads"], got["nrb"]) == cache_shape, got
            D.set_gauge(U)
            rc, st, x = _solve(q, D, bs, inner, layout=q.QDWF_RIRI, nrhs=nrhs, use_graph=0)
            D.close()
        finally:
            for k, v in old.items():
                if v is None:
                    del os.environ[k]
                else:
                    os.environ[k] = v
        assert rc == q.QDWF_OK and st.converged == nrhs
        return st, x

    st0, x0 = run()
    for j in range(nrhs):
        r = bs[j] - cpu.mpc(a, U, cpu.mpc(a, U, x0[j]), dagger=True)
        assert np.linalg.norm(r) / np.linalg.norm(bs[j]) <= 1.5e-10
    for kw in (dict(threads=128), dict(cache_shape=(256, 2)), dict(cache_shape=(256, 4))):
        st, x = run(**kw)
        assert st.iterations == st0.iterations, kw
        assert np.array_equal(x, x0), f"the solve depends on the hop launch shape {kw}"
