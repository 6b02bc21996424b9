"""ctypes binding of libqdwf.so (C ABI in include/qdwf.h).

Argument marshalling only: every step runs in the library's HIP kernels.
Functions carry the C names; device buffers are torch CUDA tensors (their
data pointers are passed), streams default to torch's current stream.
Loading fails loudly if the library has not been built.
"""
from __future__ import annotations

import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libqdwf.so")

QDWF_OK, QDWF_EINVAL, QDWF_ENOMEM, QDWF_EDEVICE, QDWF_ENOTCONV, QDWF_ENAN, QDWF_EBUSY = range(7)
QDWF_F64, QDWF_F32, QDWF_F16, QDWF_BF16 = 0, 1, 2, 3
QDWF_RRII, QDWF_RIRI = 0, 1
QDWF_EVEN, QDWF_ODD, QDWF_FULL = 0, 1, 2
QDWF_MEE_FWD, QDWF_MEE_INV = 0, 1
QDWF_SYS_NORMAL_PC, QDWF_SYS_FULL = 0, 1
QDWF_OP_MPC, QDWF_OP_MDAGM, QDWF_OP_SOLVE, QDWF_OP_REDUCE, QDWF_OP_TUNE = 0, 1, 2, 3, 4
QDWF_NOALLOC_SCRATCH_BYTES = 540672   # static scratch of qdwf_dot_noalloc per GPU

TORCH_DTYPE = {QDWF_F64: torch.float64, QDWF_F32: torch.float32,
               QDWF_F16: torch.float16, QDWF_BF16: torch.bfloat16}
PREC_NAME = {QDWF_F64: "f64", QDWF_F32: "f32", QDWF_F16: "f16", QDWF_BF16: "bf16"}


class QdwfError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"qdwf error {code}: {msg}")
        self.code = code


class qdwf_action(ctypes.Structure):
    _fields_ = [("L", ctypes.c_int32 * 4), ("Ls", ctypes.c_int32), ("bc", ctypes.c_int32 * 4),
                ("M5", ctypes.c_double), ("mf", ctypes.c_double),
                ("b", ctypes.c_double), ("c", ctypes.c_double)]


class qdwf_solve_params(ctypes.Structure):
    _fields_ = [("system", ctypes.c_int32), ("inner_prec", ctypes.c_int32),
                ("layout", ctypes.c_int32), ("max_iter", ctypes.c_int32),
                ("tol", ctypes.c_double), ("delta", ctypes.c_double),
                ("x0_is_guess", ctypes.c_int32), ("check_every", ctypes.c_int32),
                ("use_graph", ctypes.c_int32)]


class qdwf_solve_stats(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int32), ("reliable_updates", ctypes.c_int32),
                ("converged", ctypes.c_int32), ("restarts", ctypes.c_int32),
                ("true_residual", ctypes.c_double), ("full_residual", ctypes.c_double),
                ("seconds", ctypes.c_double), ("flops", ctypes.c_int64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class qdwf_request(ctypes.Structure):
    _fields_ = [("act", qdwf_action), ("U", ctypes.c_void_p), ("b", ctypes.c_void_p),
                ("x_out", ctypes.c_void_p), ("params", qdwf_solve_params)]


_P = ctypes.c_void_p
_I = ctypes.c_int
_SIG = {
    "qdwf_last_error": ([], ctypes.c_char_p),
    "qdwf_create": ([ctypes.POINTER(qdwf_action), _I, ctypes.POINTER(_P)], _I),
    "qdwf_destroy": ([_P], _I),
    "qdwf_set_gauge": ([_P, _P, _I, _P], _I),
    "qdwf_field_reals": ([_P, _I], ctypes.c_size_t),
    "qdwf_pack_spinor": ([_P, _P, _I, _I, _P, _I, _I, _I, _P], _I),
    "qdwf_unpack_spinor": ([_P, _P, _I, _P, _I, _I, _I, _I, _P], _I),
    "qdwf_apply_D": ([_P, _P, _P, _I, _I, _I, _I, _P], _I),
    "qdwf_apply_Mee": ([_P, _P, _P, _I, _I, _I, _I, _I, _I, _P], _I),
    "qdwf_apply_Deo": ([_P, _P, _P, _I, _I, _I, _I, _I, _P], _I),
    "qdwf_split_workspace_bytes": ([_P, _I, _I], ctypes.c_size_t),
    "qdwf_split_prepare": ([_P, _I, _I, _P, _P], _I),
    "qdwf_apply_D_split": ([_P, _P, _P, _I, _I, _I, _P, _P], _I),
    "qdwf_su3_mul": ([_P, _P, _P, ctypes.c_int64, _I, _I, _P], _I),
    "qdwf_triad": ([_P, _P, _P, ctypes.c_double, ctypes.c_int64, _I, _I, _P], _I),
    "qdwf_apply_Dh": ([_P, _P, _P, _I, _I, _I, _I, _I, _P], _I),
    "qdwf_apply_Dw": ([_P, _P, _P, ctypes.c_double, _I, _I, _I, _I, _P], _I),
    "qdwf_apply_Mpc": ([_P, _P, _P, _I, _I, _I, _I, _P, _P], _I),
    "qdwf_apply_MdagM": ([_P, _P, _P, _I, _I, _I, _P, _P], _I),
    "qdwf_workspace_bytes": ([_P, _I, _I, _I], ctypes.c_size_t),
    "qdwf_dot": ([_P, _P, _P, _P, _I, _I, _I, _I, _P, _P], _I),
    "qdwf_dot_noalloc": ([_P, _P, _P, _P, _I, _I, _I, _I, _P], _I),
    "qdwf_solve": ([_P, _P, _P, _I, ctypes.POINTER(qdwf_solve_params),
                    ctypes.POINTER(qdwf_solve_stats), _P, _P], _I),
    "qdwf_geometry_tables": ([_P, _P, _P, _P], _I),
    "qdwf_tune": ([_P, _I, _I, _I, _P, _P, _P], _I),
    "qdwf_tuned_shape": ([_P, _I, _I, _I, _I, _P], _I),
    "qdwf_tune_traversal": ([ctypes.POINTER(qdwf_action), _I, _I, _I, _P, _P, _P], _I),
    "qdwf_traversal": ([_P, _P], _I),
    "qdwf_request_bytes": ([ctypes.POINTER(qdwf_action), ctypes.POINTER(qdwf_solve_params)],
                           ctypes.c_size_t),
    "qdwf_pool_overhead_bytes": ([_I], ctypes.c_size_t),
    "qdwf_pool_create": ([_I, _P, ctypes.c_size_t, _I, ctypes.POINTER(qdwf_solve_params),
                          ctypes.POINTER(_P)], _I),
    "qdwf_pool_destroy": ([_P], _I),
    "qdwf_pool_submit": ([_P, ctypes.POINTER(qdwf_request), ctypes.POINTER(ctypes.c_uint64)], _I),
    "qdwf_pool_step": ([_P, _P, ctypes.POINTER(_I)], _I),
    "qdwf_pool_poll": ([_P, ctypes.c_uint64, ctypes.POINTER(qdwf_solve_stats)], _I),
    "qdwf_pool_info": ([_P, ctypes.POINTER(ctypes.c_size_t), ctypes.POINTER(ctypes.c_size_t),
                        ctypes.POINTER(_I), ctypes.POINTER(_I)], _I),
}

_lib = None


def lib() -> ctypes.CDLL:
    """Loads libqdwf.so; raises if it is missing (there is no fallback path)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run python -m paper_2112_01852_amd.build")
        L = ctypes.CDLL(LIB_PATH)
        for name, (args, res) in _SIG.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = res
        _lib = L
    return _lib


def declared_symbols():
    return list(_SIG)


def _check(rc):
    if rc != QDWF_OK:
        raise QdwfError(rc, lib().qdwf_last_error().decode())
    return rc


def _stream(stream):
    if stream is None:
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, torch.cuda.Stream):
        return ctypes.c_void_p(stream.cuda_stream)
    return ctypes.c_void_p(int(stream))


def _ptr(t, what="tensor"):
    if t is None:
        return None
    if isinstance(t, int):
        return ctypes.c_void_p(t)
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{what} must be a CUDA tensor")
    if not t.is_contiguous():
        raise ValueError(f"{what} must be contiguous")
    return ctypes.c_void_p(t.data_ptr())


def make_action(L, Ls, M5=1.8, mf=0.01, b=1.0, c=0.0, bc=(1, 1, 1, -1)) -> qdwf_action:
    a = qdwf_action()
    a.L[:] = [int(v) for v in L]
    a.Ls = int(Ls)
    a.bc[:] = [int(v) for v in bc]
    a.M5, a.mf, a.b, a.c = float(M5), float(mf), float(b), float(c)
    return a


# ---- C names ----------------------------------------------------------------
def qdwf_last_error() -> str:
    return lib().qdwf_last_error().decode()


def qdwf_create(act: qdwf_action, device: int = 0):
    h = ctypes.c_void_p()
    _check(lib().qdwf_create(ctypes.byref(act), int(device), ctypes.byref(h)))
    return h


def qdwf_destroy(ctx):
    _check(lib().qdwf_destroy(ctx))


def qdwf_set_gauge(ctx, U: torch.Tensor, stream=None):
    if U.dtype == torch.complex128:
        prec = QDWF_F64
    elif U.dtype == torch.complex64:
        prec = QDWF_F32
    else:
        raise TypeError("gauge field must be complex128 or complex64")
    _check(lib().qdwf_set_gauge(ctx, _ptr(U, "U"), prec, _stream(stream)))


def qdwf_field_reals(ctx, subset: int) -> int:
    return int(lib().qdwf_field_reals(ctx, int(subset)))


def _canon_prec(t):
    if t.dtype == torch.complex128:
        return QDWF_F64
    if t.dtype == torch.complex64:
        return QDWF_F32
    raise TypeError("canonical spinors must be complex128 or complex64")


def qdwf_pack_spinor(ctx, dst, prec, layout, src, subset, nrhs=1, stream=None):
    _check(lib().qdwf_pack_spinor(ctx, _ptr(dst, "dst"), int(prec), int(layout), _ptr(src, "src"),
                                  _canon_prec(src), int(subset), int(nrhs), _stream(stream)))


def qdwf_unpack_spinor(ctx, dst, src, prec, layout, subset, nrhs=1, stream=None):
    _check(lib().qdwf_unpack_spinor(ctx, _ptr(dst, "dst"), _canon_prec(dst), _ptr(src, "src"),
                                    int(prec), int(layout), int(subset), int(nrhs),
                                    _stream(stream)))


def qdwf_apply_D(ctx, out, inp, dagger, prec, layout, nrhs=1, stream=None):
    _check(lib().qdwf_apply_D(ctx, _ptr(out, "out"), _ptr(inp, "in"), int(dagger), int(prec),
                              int(layout), int(nrhs), _stream(stream)))


def qdwf_apply_Mee(ctx, out, inp, subset, dagger, which, prec, layout, nrhs=1, stream=None):
    _check(lib().qdwf_apply_Mee(ctx, _ptr(out, "out"), _ptr(inp, "in"), int(subset), int(dagger),
                                int(which), int(prec), int(layout), int(nrhs), _stream(stream)))


def qdwf_apply_Deo(ctx, out, inp, out_parity, dagger, prec, layout, nrhs=1, stream=None):
    _check(lib().qdwf_apply_Deo(ctx, _ptr(out, "out"), _ptr(inp, "in"), int(out_parity),
                                int(dagger), int(prec), int(layout), int(nrhs), _stream(stream)))


def qdwf_apply_Dh(ctx, out, inp, subset, dagger, prec, layout, nrhs=1, stream=None):
    _check(lib().qdwf_apply_Dh(ctx, _ptr(out, "out"), _ptr(inp, "in"), int(subset), int(dagger),
                               int(prec), int(layout), int(nrhs), _stream(stream)))


def qdwf_apply_Dw(ctx, out, inp, mass, dagger, prec, layout, nrhs=1, stream=None):
    _check(lib().qdwf_apply_Dw(ctx, _ptr(out, "out"), _ptr(inp, "in"), float(mass), int(dagger),
                               int(prec), int(layout), int(nrhs), _stream(stream)))


def qdwf_split_workspace_bytes(ctx, ranks, prec) -> int:
    return int(lib().qdwf_split_workspace_bytes(ctx, int(ranks), int(prec)))


def qdwf_split_prepare(ctx, ranks, prec, ws, stream=None):
    _check(lib().qdwf_split_prepare(ctx, int(ranks), int(prec), _ptr(ws, "ws"), _stream(stream)))


def qdwf_apply_D_split(ctx, out, inp, ranks, prec, layout, ws, stream=None):
    _check(lib().qdwf_apply_D_split(ctx, _ptr(out, "out"), _ptr(inp, "in"), int(ranks), int(prec),
                                    int(layout), _ptr(ws, "ws"), _stream(stream)))


def qdwf_su3_mul(C, A, B, n, prec, device=0, stream=None):
    _check(lib().qdwf_su3_mul(_ptr(C, "C"), _ptr(A, "A"), _ptr(B, "B"), int(n), int(prec),
                              int(device), _stream(stream)))


def qdwf_triad(a, b, c, s, n, prec, device=0, stream=None):
    _check(lib().qdwf_triad(_ptr(a, "a"), _ptr(b, "b"), _ptr(c, "c"), float(s), int(n), int(prec),
                            int(device), _stream(stream)))


def qdwf_workspace_bytes(ctx, op, prec, nrhs=1) -> int:
    return int(lib().qdwf_workspace_bytes(ctx, int(op), int(prec), int(nrhs)))


def qdwf_apply_Mpc(ctx, out, inp, dagger, prec, layout, nrhs, ws, stream=None):
    _check(lib().qdwf_apply_Mpc(ctx, _ptr(out, "out"), _ptr(inp, "in"), int(dagger), int(prec),
                                int(layout), int(nrhs), _ptr(ws, "ws"), _stream(stream)))


def qdwf_apply_MdagM(ctx, out, inp, prec, layout, nrhs, ws, stream=None):
    _check(lib().qdwf_apply_MdagM(ctx, _ptr(out, "out"), _ptr(inp, "in"), int(prec), int(layout),
                                  int(nrhs), _ptr(ws, "ws"), _stream(stream)))


def qdwf_dot(ctx, x, y, subset, prec, layout, nrhs, ws, stream=None):
    out = (ctypes.c_double * (2 * int(nrhs)))()
    _check(lib().qdwf_dot(ctx, ctypes.cast(out, ctypes.c_void_p), _ptr(x, "x"), _ptr(y, "y"),
                          int(subset), int(prec), int(layout), int(nrhs), _ptr(ws, "ws"),
                          _stream(stream)))
    return [complex(out[2 * i], out[2 * i + 1]) for i in range(int(nrhs))]


def qdwf_dot_noalloc(ctx, x, y, subset, prec, layout, nrhs, stream=None):
    out = (ctypes.c_double * (2 * int(nrhs)))()
    _check(lib().qdwf_dot_noalloc(ctx, ctypes.cast(out, ctypes.c_void_p), _ptr(x, "x"),
                                  _ptr(y, "y"), int(subset), int(prec), int(layout), int(nrhs),
                                  _stream(stream)))
    return [complex(out[2 * i], out[2 * i + 1]) for i in range(int(nrhs))]


def qdwf_solve(ctx, x, b, nrhs, params: qdwf_solve_params, ws, stream=None):
    """Returns (status code, stats). ENOTCONV / ENAN are returned, not raised."""
    st = qdwf_solve_stats()
    rc = lib().qdwf_solve(ctx, _ptr(x, "x"), _ptr(b, "b"), int(nrhs), ctypes.byref(params),
                          ctypes.byref(st), _ptr(ws, "ws"), _stream(stream))
    if rc not in (QDWF_OK, QDWF_ENOTCONV, QDWF_ENAN):
        _check(rc)
    return rc, st


def qdwf_geometry_tables(ctx, V: int):
    import numpy as np
    cb = np.empty(V, dtype=np.int32)
    nbr = np.empty((2, V // 2, 8), dtype=np.int32)
    sign = np.empty((2, V // 2, 8), dtype=np.int8)
    _check(lib().qdwf_geometry_tables(ctx, cb.ctypes.data_as(ctypes.c_void_p),
                                      nbr.ctypes.data_as(ctypes.c_void_p),
                                      sign.ctypes.data_as(ctypes.c_void_p)))
    return cb, nbr, sign


def qdwf_tune(ctx, prec, layout, nrhs, ws, stream=None):
    """Tunes the hop launch shape; returns (best D ms, best D^dag ms)."""
    best = (ctypes.c_double * 2)()
    _check(lib().qdwf_tune(ctx, int(prec), int(layout), int(nrhs), _ptr(ws, "ws"), _stream(stream),
                           ctypes.cast(best, ctypes.c_void_p)))
    return best[0], best[1]


def qdwf_tuned_shape(ctx, prec, layout, dagger, nrhs):
    out = (ctypes.c_int32 * 4)()
    _check(lib().qdwf_tuned_shape(ctx, int(prec), int(layout), int(dagger), int(nrhs),
                                  ctypes.cast(out, ctypes.c_void_p)))
    return dict(threads=out[0], nrb=out[1], xcd=out[2], lds_pad=out[3])


def qdwf_tune_traversal(act: qdwf_action, device, prec, nrhs, stream=None):
    """Searches site traversal orders and layouts on throwaway contexts;
    returns (dict(split, sweep, tile, layout), best ms)."""
    out = (ctypes.c_int32 * 7)()
    best = ctypes.c_double(0.0)
    _check(lib().qdwf_tune_traversal(ctypes.byref(act), int(device), int(prec), int(nrhs),
                                     _stream(stream), ctypes.cast(out, ctypes.c_void_p),
                                     ctypes.cast(ctypes.byref(best), ctypes.c_void_p)))
    return dict(split=out[0], sweep=out[1], tile=tuple(out[2:6]), layout=out[6]), best.value


def qdwf_traversal(ctx):
    """{split, sweep, tile} of a context's site traversal order."""
    out = (ctypes.c_int32 * 6)()
    _check(lib().qdwf_traversal(ctx, ctypes.cast(out, ctypes.c_void_p)))
    return dict(split=out[0], sweep=out[1], tile=tuple(out[2:6]))


def qdwf_request_bytes(act: qdwf_action, params: qdwf_solve_params) -> int:
    return int(lib().qdwf_request_bytes(ctypes.byref(act), ctypes.byref(params)))


def qdwf_pool_overhead_bytes(max_slots: int) -> int:
    return int(lib().qdwf_pool_overhead_bytes(int(max_slots)))


def qdwf_pool_create(device: int, arena: torch.Tensor, max_slots: int,
                     params: qdwf_solve_params):
    """The arena (a uint8 CUDA tensor, 256-byte aligned) is the pool's whole
    device memory; the caller keeps it alive until qdwf_pool_destroy."""
    h = ctypes.c_void_p()
    nbytes = arena.numel() * arena.element_size()
    _check(lib().qdwf_pool_create(int(device), _ptr(arena, "arena"), ctypes.c_size_t(nbytes),
                                  int(max_slots), ctypes.byref(params), ctypes.byref(h)))
    return h


def qdwf_pool_destroy(pool):
    _check(lib().qdwf_pool_destroy(pool))


def qdwf_pool_submit(pool, act: qdwf_action, U, b, x_out, params: qdwf_solve_params) -> int:
    r = qdwf_request()
    r.act = act
    r.U, r.b, r.x_out = _ptr(U, "U"), _ptr(b, "b"), _ptr(x_out, "x_out")
    r.params = params
    rid = ctypes.c_uint64()
    _check(lib().qdwf_pool_submit(pool, ctypes.byref(r), ctypes.byref(rid)))
    return int(rid.value)


def qdwf_pool_step(pool, stream=None) -> int:
    n = ctypes.c_int()
    _check(lib().qdwf_pool_step(pool, _stream(stream), ctypes.byref(n)))
    return int(n.value)


def qdwf_pool_poll(pool, rid: int):
    """(done, status, stats): done is False while the request is queued or running."""
    st = qdwf_solve_stats()
    rc = lib().qdwf_pool_poll(pool, ctypes.c_uint64(rid), ctypes.byref(st))
    if rc == QDWF_EBUSY:
        return False, rc, None
    if rc not in (QDWF_OK, QDWF_ENOTCONV, QDWF_ENAN):
        _check(rc)
    return True, rc, st


def qdwf_pool_info(pool):
    a, b_ = ctypes.c_size_t(), ctypes.c_size_t()
    na, nq = ctypes.c_int(), ctypes.c_int()
    _check(lib().qdwf_pool_info(pool, ctypes.byref(a), ctypes.byref(b_), ctypes.byref(na),
                                ctypes.byref(nq)))
    return {"in_use": a.value, "peak": b_.value, "active": na.value, "queued": nq.value}


def solve_params(system=QDWF_SYS_NORMAL_PC, inner_prec=QDWF_F64, layout=QDWF_RIRI, tol=1e-10,
                 max_iter=20000, delta=0.1, x0_is_guess=0, check_every=8, use_graph=0):
    p = qdwf_solve_params()
    p.system, p.inner_prec, p.layout, p.max_iter = system, inner_prec, layout, max_iter
    p.tol, p.delta, p.x0_is_guess = tol, delta, x0_is_guess
    p.check_every, p.use_graph = check_every, use_graph
    return p


# ---- convenience wrapper used by the tests and the benchmark -------------------
class Dirac:
    """One qdwf context plus allocation helpers for its fields (torch tensors)."""

    def __init__(self, L, Ls, M5=1.8, mf=0.01, b=1.0, c=0.0, bc=(1, 1, 1, -1), device=0):
        self.L, self.Ls = tuple(int(v) for v in L), int(Ls)
        self.params = dict(M5=M5, mf=mf, b=b, c=c, bc=tuple(bc))
        self.device = device
        self.ctx = qdwf_create(make_action(L, Ls, M5, mf, b, c, bc), device)
        self.V = self.L[0] * self.L[1] * self.L[2] * self.L[3]
        self.n5h = self.V // 2 * self.Ls

    def close(self):
        if self.ctx is not None:
            qdwf_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def field(self, prec, subset=QDWF_FULL, nrhs=1, zero=True):
        n = qdwf_field_reals(self.ctx, subset) * nrhs
        dev = torch.device("cuda", self.device)
        t = torch.zeros(n, dtype=TORCH_DTYPE[prec], device=dev) if zero else \
            torch.empty(n, dtype=TORCH_DTYPE[prec], device=dev)
        return t

    def workspace(self, op, prec, nrhs=1):
        nb = qdwf_workspace_bytes(self.ctx, op, prec, nrhs)
        return torch.empty(max(nb, 1), dtype=torch.uint8, device=torch.device("cuda", self.device))

    def set_gauge(self, U):
        Ut = U if isinstance(U, torch.Tensor) else torch.from_numpy(U)
        Ut = Ut.to(torch.device("cuda", self.device)).contiguous()
        qdwf_set_gauge(self.ctx, Ut)
        torch.cuda.synchronize(self.device)

    def pack(self, psi, prec, layout, subset=QDWF_FULL, nrhs=1):
        src = psi if isinstance(psi, torch.Tensor) else torch.from_numpy(psi)
        src = src.to(torch.device("cuda", self.device)).contiguous()
        dst = self.field(prec, subset, nrhs, zero=False)
        qdwf_pack_spinor(self.ctx, dst, prec, layout, src, subset, nrhs)
        return dst

    def unpack(self, f, prec, layout, subset=QDWF_FULL, nrhs=1, dtype=torch.complex128):
        Lx, Ly, Lz, Lt = self.L
        shape = (nrhs, self.Ls, Lt, Lz, Ly, Lx, 4, 3)
        dst = torch.zeros(shape, dtype=dtype, device=torch.device("cuda", self.device))
        qdwf_unpack_spinor(self.ctx, dst, f, prec, layout, subset, nrhs)
        return dst if nrhs > 1 else dst[0]
