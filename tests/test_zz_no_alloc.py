"""qdwf_dot_noalloc (the allocation-free form of qdwf_dot, its scratch in a
static device array) against qdwf_dot with a workspace, through the C ABI:
two calls in a row, the second on a smaller field, each bitwise equal to
qdwf_dot (the same kernels and reduction tree) and within 1e-12 of the same
inner products taken in FP64 by torch. A request for more scratch than the
array holds is refused before anything is launched.
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
    q.lib()
    return q, torch


def _fields(q, torch, D, prec, subset, nrhs, seed):
    g = torch.Generator(device="cuda")
    g.manual_seed(seed)
    n = q.qdwf_field_reals(D.ctx, subset) * nrhs
    x = torch.randn(n, generator=g, device="cuda", dtype=torch.float64).to(q.TORCH_DTYPE[prec])
    y = torch.randn(n, generator=g, device="cuda", dtype=torch.float64).to(q.TORCH_DTYPE[prec])
    return x, y


def _check_call(q, torch, D, prec, layout, subset, nrhs, seed):
    print(f"noalloc dot: L={D.L} Ls={D.Ls} prec={q.PREC_NAME[prec]} subset={subset} "
          f"nrhs={nrhs}", flush=True)
    x, y = _fields(q, torch, D, prec, subset, nrhs, seed)
    got = q.qdwf_dot_noalloc(D.ctx, x, y, subset, prec, layout, nrhs)
    ws = D.workspace(q.QDWF_OP_REDUCE, prec, nrhs)
    ref = q.qdwf_dot(D.ctx, x, y, subset, prec, layout, nrhs, ws)
    assert got == ref, (got, ref)
    # real parts against torch's FP64 dot of the same stored values
    xr = x.to(torch.float64).reshape(nrhs, -1)
    yr = y.to(torch.float64).reshape(nrhs, -1)
    for r in range(nrhs):
        re = float(torch.dot(xr[r], yr[r]))
        scale = float(torch.linalg.vector_norm(xr[r]) * torch.linalg.vector_norm(yr[r]))
        assert abs(got[r].real - re) <= 1e-12 * scale, (r, got[r].real, re)


def test_noalloc_dot_two_calls_second_smaller(env):
    q, torch = env
    big = q.Dirac((8, 8, 8, 8), 16, M5=1.8, mf=0.01, b=1.5, c=0.5)
    small = q.Dirac((4, 4, 4, 4), 8, M5=1.8, mf=0.05, b=1.5, c=0.5)
    try:
        _check_call(q, torch, big, q.QDWF_F32, q.QDWF_RIRI, q.QDWF_FULL, 4, 11)
        _check_call(q, torch, small, q.QDWF_F64, q.QDWF_RRII, q.QDWF_ODD, 1, 12)
        # back to a larger one in another precision: nothing stale is read
        _check_call(q, torch, big, q.QDWF_F16, q.QDWF_RIRI, q.QDWF_EVEN, 2, 13)
    finally:
        big.close()
        small.close()


def test_noalloc_dot_refuses_more_than_its_scratch(env):
    q, torch = env
    D = q.Dirac((8, 8, 8, 8), 16, M5=1.8, mf=0.01, b=1.5, c=0.5)
    try:
        x = D.field(q.QDWF_F32, q.QDWF_FULL)
        nrhs = 4096    # 4096 x (reduction blocks + 2) doubles: far beyond the scratch
        assert q.qdwf_workspace_bytes(D.ctx, q.QDWF_OP_REDUCE, q.QDWF_F32, nrhs) \
            > q.QDWF_NOALLOC_SCRATCH_BYTES
        with pytest.raises(q.QdwfError) as e:
            q.qdwf_dot_noalloc(D.ctx, x, x, q.QDWF_FULL, q.QDWF_F32, q.QDWF_RIRI, nrhs)
        assert e.value.code == q.QDWF_EINVAL
        assert "scratch" in q.qdwf_last_error()
    finally:
        D.close()
