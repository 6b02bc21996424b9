"""Served solve stream: Poisson arrivals of even-odd Mobius domain-wall CG
solves of mixed volume, Ls and mass, run through the library's pool
(continuous batching, admission by HBM footprint), with latency percentiles.

The request inputs (a smoothed-link ensemble and a Gaussian source per
request) are drawn on the GPU from seeded torch generators so that a stream of
hundreds of requests can be prepared in seconds; they play the role of the
gauge configurations a production run would read from storage.
"""
from __future__ import annotations

import math
import time
from dataclasses import dataclass, field

import numpy as np
import torch

from . import qdwf as q

VOLUMES = (8, 12, 16, 24)
LS_CHOICES = (8, 12, 16)
MOBIUS = dict(M5=1.8, b=1.5, c=0.5)

_GELL_MANN = None


def _gell_mann(device):
    global _GELL_MANN
    if _GELL_MANN is None or _GELL_MANN.device != device:
        from .inputs import _GELL_MANN as G
        _GELL_MANN = torch.from_numpy(np.ascontiguousarray(G)).to(device)
    return _GELL_MANN


def smoothed_gauge_torch(L, seed: int, eps: float = 0.3, device="cuda"):
    """U = exp(i eps H), H = sum_a h_a lambda_a / 2 with h_a ~ N(0,1), per link,
    canonical layout [4][T][Z][Y][X][3][3] complex128, drawn on the GPU."""
    g = torch.Generator(device=device)
    g.manual_seed(int(seed))
    V = int(np.prod(L))
    h = torch.randn((4 * V, 8), generator=g, device=device, dtype=torch.float64)
    H = torch.einsum("na,aij->nij", h.to(torch.complex128), _gell_mann(torch.device(device))) * 0.5
    U = torch.linalg.matrix_exp(1j * eps * H)
    Lx, Ly, Lz, Lt = L
    return U.reshape(4, Lt, Lz, Ly, Lx, 3, 3).contiguous()


def gaussian_source_torch(L, Ls: int, seed: int, device="cuda"):
    g = torch.Generator(device=device)
    g.manual_seed(int(seed))
    Lx, Ly, Lz, Lt = L
    z = torch.randn((Ls, Lt, Lz, Ly, Lx, 4, 3, 2), generator=g, device=device, dtype=torch.float64)
    return torch.view_as_complex(z).contiguous()


@dataclass
class Spec:
    L: tuple
    Ls: int
    mf: float
    link_seed: int
    src_seed: int

    def action(self):
        return q.make_action(self.L, self.Ls, mf=self.mf, **MOBIUS)


def make_specs(n: int, master_seed: int = 5000):
    """Request mix: volume uniform over 8^4..24^4, Ls uniform over {8,12,16},
    mf log-uniform in [1e-3, 1e-1], one link and one source seed each."""
    rng = np.random.Generator(np.random.Philox(key=master_seed))
    specs = []
    for i in range(n):
        l = int(rng.choice(VOLUMES))
        Ls = int(rng.choice(LS_CHOICES))
        mf = float(10 ** rng.uniform(-3, -1))
        specs.append(Spec((l, l, l, l), Ls, mf, master_seed * 1000 + 2 * i + 1,
                          master_seed * 1000 + 2 * i + 2))
    return specs


@dataclass
class Prepared:
    spec: Spec
    U: torch.Tensor
    b: torch.Tensor
    x: torch.Tensor = field(default=None)


def prepare(specs, device="cuda", with_x: bool = True):
    """Links and source of every request on the GPU (and a zeroed solution
    buffer each when with_x)."""
    out = []
    for sp in specs:
        U = smoothed_gauge_torch(sp.L, sp.link_seed, device=device)
        b = gaussian_source_torch(sp.L, sp.Ls, sp.src_seed, device=device)
        out.append(Prepared(sp, U, b, torch.zeros_like(b) if with_x else None))
    torch.cuda.synchronize()
    return out


def solo_solve(p: Prepared, params):
    """One request solved alone through qdwf_solve (odd-site solution)."""
    sp = p.spec
    D = q.Dirac(sp.L, sp.Ls, mf=sp.mf, **MOBIUS)
    D.set_gauge(p.U)
    bo = D.field(q.QDWF_F64, q.QDWF_ODD)
    q.qdwf_pack_spinor(D.ctx, bo, q.QDWF_F64, params.layout, p.b, q.QDWF_ODD)
    x = D.field(q.QDWF_F64, q.QDWF_ODD)
    ws = D.workspace(q.QDWF_OP_SOLVE, params.inner_prec)
    t0 = time.perf_counter()
    rc, st = q.qdwf_solve(D.ctx, x, bo, 1, params, ws)
    dt = time.perf_counter() - t0
    out = torch.zeros_like(p.b)
    q.qdwf_unpack_spinor(D.ctx, out, x, q.QDWF_F64, params.layout, q.QDWF_ODD)
    torch.cuda.synchronize()
    D.close()
    return rc, st, dt, out


def poisson_arrivals(n: int, rate: float, seed: int):
    rng = np.random.Generator(np.random.Philox(key=seed))
    return np.cumsum(rng.exponential(1.0 / rate, size=n))


def run_pool(prepared, arrivals, params, arena_bytes: int, max_slots: int, device: int = 0,
             keep_x: bool = True):
    """Drive a pool in real time on torch's current stream: submit each
    request at its arrival time, step, poll. The pool's whole device memory
    is one arena tensor of arena_bytes. Returns per-request latency
    (completion - arrival), statuses, stats, the pool's peak arena use, the
    makespan and the device memory the process lost between the first and the
    last step (the pool allocates none after creation). keep_x: leave each
    solution in its request's x buffer (otherwise the buffer is released
    after the request finishes)."""
    n = len(prepared)
    arena = torch.empty(int(arena_bytes), dtype=torch.uint8, device=torch.device("cuda", device))
    pool = q.qdwf_pool_create(device, arena, max_slots, params)
    ids = [None] * n
    done_at = [None] * n
    status = [None] * n
    stats = [None] * n
    xbuf = [None] * n
    torch.cuda.synchronize(device)
    free0 = torch.cuda.mem_get_info(device)[0]
    free_min = free0
    t0 = time.perf_counter()
    nxt = 0
    finished = 0
    pending = []
    try:
        while finished < n:
            now = time.perf_counter() - t0
            while nxt < n and arrivals[nxt] <= now:
                p = prepared[nxt]
                xbuf[nxt] = p.x if keep_x else torch.empty_like(p.b)
                ids[nxt] = q.qdwf_pool_submit(pool, p.spec.action(), p.U, p.b, xbuf[nxt], params)
                pending.append(nxt)
                nxt += 1
            info = q.qdwf_pool_info(pool)
            if info["active"] == 0 and info["queued"] == 0:
                if nxt < n:
                    time.sleep(max(0.0, min(arrivals[nxt] - now, 0.01)))
                continue
            q.qdwf_pool_step(pool)
            now = time.perf_counter() - t0
            still = []
            for i in pending:
                ok, rc, st = q.qdwf_pool_poll(pool, ids[i])
                if ok:
                    done_at[i] = now
                    status[i] = rc
                    stats[i] = st.as_dict()
                    finished += 1
                    if not keep_x:
                        xbuf[i] = None
                else:
                    still.append(i)
            pending = still
            free_min = min(free_min, torch.cuda.mem_get_info(device)[0])
        torch.cuda.synchronize(device)
        info = q.qdwf_pool_info(pool)
    finally:
        q.qdwf_pool_destroy(pool)
        del arena
    lat = np.array(done_at) - np.array(arrivals)
    return {"latency": lat, "status": status, "stats": stats, "peak_bytes": info["peak"],
            "in_use_end": info["in_use"], "makespan": float(max(done_at)),
            "device_bytes_taken_while_serving": int(free0 - free_min)}


def percentiles(lat):
    return {"p50_s": float(np.percentile(lat, 50)), "p99_s": float(np.percentile(lat, 99)),
            "mean_s": float(np.mean(lat))}
