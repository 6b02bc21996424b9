"""Autotuner: picks a launch shape, keeps results correct, round-trips its cache."""
import os

import numpy as np
import pytest

from oracle import cpu
from paper_2112_01852_amd import inputs as I

pytestmark = pytest.mark.gpu
MOBIUS = dict(M5=1.8, mf=0.01, b=1.5, c=0.5)


@pytest.fixture(scope="module")
def q():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2112_01852_amd import qdwf
    qdwf.lib()
    return qdwf


def test_tuned_operator_matches_oracle_and_cache_roundtrips(q, tmp_path):
    cache = tmp_path / "tune.jsonl"
    os.environ["QDWF_TUNE_CACHE"] = str(cache)
    try:
        L, Ls, nrhs = (8, 4, 4, 6), 16, 3
        a = cpu.Action(L=L, Ls=Ls, **MOBIUS)
        U = I.gauge_field(L, "haar", 7)
        psi = I.gaussian_spinor(L, Ls, 8, nrhs=nrhs)
        D = q.Dirac(L, Ls, **MOBIUS)
        D.set_gauge(U)
        ws = D.workspace(q.QDWF_OP_TUNE, q.QDWF_F32, nrhs)
        tD, tDd = q.qdwf_tune(D.ctx, q.QDWF_F32, q.QDWF_RIRI, nrhs, ws)
        assert tD > 0 and tDd > 0
        shape = q.qdwf_tuned_shape(D.ctx, q.QDWF_F32, q.QDWF_RIRI, 0, nrhs)
        f = D.pack(psi, q.QDWF_F32, q.QDWF_RIRI, q.QDWF_FULL, nrhs)
        for dag in (0, 1):
            out = D.field(q.QDWF_F32, q.QDWF_FULL, nrhs)
            q.qdwf_apply_D(D.ctx, out, f, dag, q.QDWF_F32, q.QDWF_RIRI, nrhs)
            got = D.unpack(out, q.QDWF_F32, q.QDWF_RIRI, q.QDWF_FULL, nrhs).cpu().numpy()
            for j in range(nrhs):
                ref = cpu.dwf(a, U, psi[j], dagger=bool(dag))
                assert np.linalg.norm(got[j] - ref) / np.linalg.norm(ref) < 1e-6
        D.close()
        lines = cache.read_text().strip().splitlines()
        assert len(lines) == 2
        # a new context of the same shape picks the cached shape up
        D2 = q.Dirac(L, Ls, **MOBIUS)
        assert q.qdwf_tuned_shape(D2.ctx, q.QDWF_F32, q.QDWF_RIRI, 0, nrhs) == shape
        D2.close()
    finally:
        del os.environ["QDWF_TUNE_CACHE"]


def test_traversal_search_roundtrips_and_matches_oracle(q, tmp_path):
    """qdwf_tune_traversal picks a site order and layout on throwaway
    contexts; a context created afterwards takes that order from the cache,
    and D and D^dag in the chosen layout match the oracle."""
    cache = tmp_path / "tune.jsonl"
    os.environ["QDWF_TUNE_CACHE"] = str(cache)
    try:
        L, Ls = (16, 8, 8, 8), 16
        act = q.make_action(L, Ls, **MOBIUS)
        choice, ms = q.qdwf_tune_traversal(act, 0, q.QDWF_F32, 1)
        assert ms > 0
        assert choice["layout"] in (q.QDWF_RIRI, q.QDWF_RRII)
        assert choice["split"] != choice["sweep"] and choice["tile"][choice["sweep"]] == 1
        lines = cache.read_text().strip().splitlines()
        assert len(lines) == 1 and '"key": "trav_16x8x8x8_Ls16_' in lines[0]
        D = q.Dirac(L, Ls, **MOBIUS)
        got_order = q.qdwf_traversal(D.ctx)
        assert got_order == {k: choice[k] for k in ("split", "sweep", "tile")}
        a = cpu.Action(L=L, Ls=Ls, **MOBIUS)
        U = I.gauge_field(L, "haar", 9)
        psi = I.gaussian_spinor(L, Ls, 10)
        D.set_gauge(U)
        lay = choice["layout"]
        f = D.pack(psi, q.QDWF_F32, lay)
        for dag in (0, 1):
            out = D.field(q.QDWF_F32)
            q.qdwf_apply_D(D.ctx, out, f, dag, q.QDWF_F32, lay)
            got = D.unpack(out, q.QDWF_F32, lay).cpu().numpy()
            ref = cpu.dwf(a, U, psi, dagger=bool(dag))
            assert np.linalg.norm(got - ref) / np.linalg.norm(ref) < 1e-6
        D.close()
        # a forced order (environment) still wins over the cache
        os.environ["QDWF_ORDER"] = "1,3"
        try:
            D3 = q.Dirac(L, Ls, **MOBIUS)
            o3 = q.qdwf_traversal(D3.ctx)
            assert (o3["split"], o3["sweep"]) == (1, 3)
            D3.close()
        finally:
            del os.environ["QDWF_ORDER"]
    finally:
        del os.environ["QDWF_TUNE_CACHE"]
