"""Serving pool: continuous batching of heterogeneous solves.

Each served result must equal the same request solved alone (bitwise: the
per-request arithmetic and round schedule do not depend on the batch), every
solve must reach the FP64 true residual, and the pool must never hold more
than its HBM budget.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2112_01852_amd import qdwf as q
    from paper_2112_01852_amd import serve
    q.lib()
    return q, serve, torch


def _specs(serve):
    S = serve.Spec
    return [S((4, 4, 4, 4), 8, 0.05, 11, 12), S((4, 4, 4, 6), 12, 0.01, 13, 14),
            S((6, 6, 6, 6), 8, 0.003, 15, 16), S((4, 4, 4, 4), 16, 0.1, 17, 18),
            S((8, 8, 8, 8), 8, 0.02, 19, 20)]


def test_served_equals_alone_and_respects_budget(env):
    q, serve, torch = env
    params = q.solve_params(inner_prec=q.QDWF_F32, layout=q.QDWF_RIRI, tol=1e-10, check_every=4)
    prepared = serve.prepare(_specs(serve))
    sizes = [q.qdwf_request_bytes(p.spec.action(), params) for p in prepared]
    budget = sorted(sizes)[-1] + sorted(sizes)[-2]      # at most two big ones at a time
    arrivals = np.zeros(len(prepared))                   # all at once: exercises the queue
    res = serve.run_pool(prepared, arrivals, params, budget, max_slots=3)
    assert res["peak_bytes"] <= budget
    for i, p in enumerate(prepared):
        assert res["status"][i] == q.QDWF_OK
        assert res["stats"][i]["true_residual"] <= 1e-10
        rc, st, dt, alone = serve.solo_solve(p, params)
        assert rc == q.QDWF_OK
        assert torch.equal(p.x, alone), f"request {i} differs between served and alone"
        assert _oracle_residual(p) <= 1.5e-10, i


def _oracle_residual(p):
    """|b_o - M_pc^dag M_pc x_o| / |b_o| of a served result, with the oracle's
    FP64 operator on the request's own links, mass and source."""
    from oracle import cpu
    sp = p.spec
    a = cpu.Action(L=sp.L, Ls=sp.Ls, mf=sp.mf, M5=1.8, b=1.5, c=0.5)
    U = p.U.cpu().numpy()
    b = cpu.restrict(p.b.cpu().numpy(), sp.L, 1)
    x = cpu.restrict(p.x.cpu().numpy(), sp.L, 1)
    r = b - cpu.mpc(a, U, cpu.mpc(a, U, x), dagger=True)
    return float(np.linalg.norm(r) / np.linalg.norm(b))


def test_mixed_inner_precisions_converge(env):
    q, serve, torch = env
    prepared = serve.prepare(_specs(serve)[:3])
    for inner in (q.QDWF_F16, q.QDWF_BF16):
        params = q.solve_params(inner_prec=inner, tol=1e-10, check_every=8)
        budget = sum(q.qdwf_request_bytes(p.spec.action(), params) for p in prepared)
        res = serve.run_pool(prepared, np.zeros(3), params, budget, max_slots=4)
        for i in range(3):
            assert res["status"][i] == q.QDWF_OK
            assert res["stats"][i]["true_residual"] <= 1e-10
            assert _oracle_residual(prepared[i]) <= 1.5e-10, (inner, i)


def test_pool_rejects_what_can_never_fit_and_unknown_ids(env):
    q, serve, torch = env
    params = q.solve_params(inner_prec=q.QDWF_F32, tol=1e-10)
    p = serve.prepare(_specs(serve)[:1])[0]
    need = q.qdwf_request_bytes(p.spec.action(), params)
    pool = q.qdwf_pool_create(0, need - 1, 2)
    try:
        with pytest.raises(q.QdwfError) as e:
            q.qdwf_pool_submit(pool, p.spec.action(), p.U, p.b, p.x, params)
        assert e.value.code == q.QDWF_EINVAL
        with pytest.raises(q.QdwfError):
            q.qdwf_pool_poll(pool, 12345)
    finally:
        q.qdwf_pool_destroy(pool)
