"""Streaming probes (qdwf_su3_mul, qdwf_triad) against their FP64 oracle.

SU(3) products: relative L2 1e-13 (FP64) and 1e-6 (FP32 storage and
arithmetic, inputs rounded to FP32 on both sides). Sizes cover one partial
block, exact multiples of the 128/256-matrix tiles, ragged tails and a large
case; the triad also runs on arrays offset by one element (the unaligned
scalar path).
"""
import numpy as np
import pytest

from oracle import streaming
from paper_2112_01852_amd import inputs as I

pytestmark = pytest.mark.gpu


def _rel(x, y):
    return float(np.linalg.norm((x - y).ravel()) / np.linalg.norm(y.ravel()))


@pytest.fixture(scope="module")
def env():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2112_01852_amd import qdwf as q
    q.lib()
    return q, torch


@pytest.mark.parametrize("n", [1, 127, 128, 256, 1000, (1 << 20) + 3])
@pytest.mark.parametrize("prec", [0, 1])
def test_su3_mul(env, n, prec):
    q, torch = env
    cdt = np.complex128 if prec == 0 else np.complex64
    A = I.haar_su3(n, 90).astype(cdt)
    B = I.haar_su3(n, 91).astype(cdt)
    At, Bt = torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda()
    Ct = torch.empty_like(At)
    q.qdwf_su3_mul(Ct, At, Bt, n, prec)
    got = Ct.cpu().numpy()
    ref = streaming.su3_mul(A, B)
    assert _rel(got, ref) < (1e-13 if prec == 0 else 1e-6)


@pytest.mark.parametrize("n", [1, 5, 4096, 1000003])
@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("offset", [0, 1])
def test_triad(env, n, prec, offset):
    q, torch = env
    dt = np.float64 if prec == 0 else np.float32
    rng = np.random.default_rng(92)
    b = rng.standard_normal(n + offset).astype(dt)
    c = rng.standard_normal(n + offset).astype(dt)
    bt, ct = torch.from_numpy(b).cuda(), torch.from_numpy(c).cuda()
    at = torch.zeros_like(bt)
    q.qdwf_triad(at[offset:], bt[offset:], ct[offset:], 0.75, n, prec)
    got = at.cpu().numpy()
    ref = streaming.triad(b[offset:], c[offset:], 0.75)
    assert _rel(got[offset:], ref) < (1e-15 if prec == 0 else 1e-7)
    assert np.all(got[:offset] == 0)


def test_arguments(env):
    q, torch = env
    A = torch.zeros(18, dtype=torch.float64, device="cuda")
    with pytest.raises(q.QdwfError):
        q.qdwf_su3_mul(A, A, A, 1, 0)            # aliasing
    with pytest.raises(q.QdwfError):
        q.qdwf_su3_mul(A, A, A, -1, 0)           # negative size
    with pytest.raises(q.QdwfError):
        q.qdwf_triad(A, A, A, 1.0, 1, 2)         # precision
    q.qdwf_su3_mul(torch.zeros_like(A), A, A, 0, 0)   # n = 0: nothing launched
