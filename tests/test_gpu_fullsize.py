"""The benchmark workload itself, whole: every operator variant the benchmark
times on the 32^4 x 16 lattice, applied to the benchmark's inputs (Haar links
seed 2000, Gaussian spinor seed 2001, drawn in single precision as the
benchmark draws them) in the launch configuration it times, read back over
the entire output field and compared with the FP64 oracle on the same inputs
widened to FP64.

Variants: Mobius D and D^dag in FP32 interleaved (the t-sweep, the
library's default at this size, and the checkerboard kernel forced), FP32
split planes (RRII), FP64, FP16 and BF16 storage; the even-odd hop D_eo
(M_{p,q} and (M_{q,p})^dag) into each parity, FP32, both layouts.

Tolerance: relative L2 over all reals of the output field, FP64 1e-13, FP32
1e-6, FP16/BF16 storage 5e-3 (FP16/BF16 fields are compared against the
oracle on the unrounded inputs, so the storage rounding counts). The oracle
outputs are computed once per operator on the host and moved to the GPU,
where the norm of the difference is taken (test arithmetic in torch, not the
library). A fault confined to any row, plane or slice of the lattice changes
the norm of the difference by far more than these bounds.
"""
import numpy as np
import pytest

from oracle import cpu
from paper_2112_01852_amd import inputs as I

pytestmark = pytest.mark.gpu

L, LS = (32, 32, 32, 32), 16
MOBIUS = dict(M5=1.8, mf=0.01, b=1.5, c=0.5)
TOL = {0: 1e-13, 1: 1e-6, 2: 5e-3, 3: 5e-3}


@pytest.fixture(scope="module")
def full():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2112_01852_amd import qdwf as q
    q.lib()
    a = cpu.Action(L=L, Ls=LS, **MOBIUS)
    U = I.gauge_field(L, "haar", 2000, dtype=np.complex64).astype(np.complex128)
    psi = I.gaussian_spinor(L, LS, 2001, dtype=np.complex64)
    psi_d = torch.from_numpy(psi).cuda()
    D = q.Dirac(L, LS, **MOBIUS)
    D.set_gauge(U)
    refs = {}
    yield q, torch, a, U, psi, psi_d, D, refs
    D.close()
    refs.clear()
    torch.cuda.empty_cache()


def _ref_dev(ctx, key):
    """Oracle output for `key`, computed once and kept on the GPU (complex128)."""
    q, torch, a, U, psi, psi_d, D, refs = ctx
    if key not in refs:
        psi64 = psi.astype(np.complex128)
        if key[0] == "D":
            ref = cpu.dwf(a, U, psi64, dagger=bool(key[1]))
        else:                       # ("eo", out_parity, dagger): input is the other parity
            p, dagger = key[1], key[2]
            ref = cpu.deo(a, U, cpu.restrict(psi64, L, 1 - p), p, dagger=bool(dagger))
        del psi64
        refs[key] = torch.from_numpy(ref).cuda()
        del ref
    return refs[key]


def _rel_dev(torch, got, ref):
    d = got.to(torch.complex128) - ref
    return float(torch.linalg.vector_norm(d) / torch.linalg.vector_norm(ref))


@pytest.mark.parametrize("prec,layout,dagger,form", [
    (1, 1, 0, ""), (1, 1, 1, ""),          # FP32 RIRI: the t-sweep (headline)
    (1, 1, 0, "0"), (1, 1, 1, "0"),        # FP32 RIRI: checkerboard kernel
    (1, 0, 0, ""), (1, 0, 1, ""),          # FP32 RRII
    (0, 1, 0, ""), (0, 1, 1, ""),          # FP64
    (2, 1, 0, ""), (2, 1, 1, ""),          # FP16 storage (packed checkerboard kernel)
    (2, 1, 0, "1"), (2, 1, 1, "1"),        # FP16 storage, t-sweep forced
    (3, 1, 0, ""), (3, 1, 1, ""),          # BF16 storage
])
def test_D_whole_field(full, prec, layout, dagger, form, monkeypatch):
    """form: "" the library's default launch (what the benchmark times), "0"
    the checkerboard kernel forced, "1" the t-sweep forced."""
    q, torch = full[0], full[1]
    D, psi_d = full[6], full[5]
    if form:
        monkeypatch.setenv("QDWF_SWEEP", form)
    print(f"32^4x16 D prec={q.PREC_NAME[prec]} layout={layout} dagger={dagger} form={form!r}",
          flush=True)
    fin = D.field(prec, q.QDWF_FULL, zero=False)
    q.qdwf_pack_spinor(D.ctx, fin, prec, layout, psi_d, q.QDWF_FULL)
    fout = D.field(prec, q.QDWF_FULL, zero=False)
    q.qdwf_apply_D(D.ctx, fout, fin, dagger, prec, layout)
    del fin
    dt = torch.complex128 if prec == 0 else torch.complex64
    got = D.unpack(fout, prec, layout, q.QDWF_FULL, dtype=dt)
    del fout
    rel = _rel_dev(torch, got, _ref_dev(full, ("D", dagger)))
    del got
    torch.cuda.empty_cache()
    print(f"  rel {rel:.3e}", flush=True)
    assert rel < TOL[prec], (prec, layout, dagger, form, rel)


@pytest.mark.parametrize("layout", [1, 0])
@pytest.mark.parametrize("p,dagger", [(1, 0), (0, 0), (1, 1)])
def test_Deo_whole_half_field(full, layout, p, dagger):
    q, torch = full[0], full[1]
    D, psi_d = full[6], full[5]
    print(f"32^4x16 D_eo f32 layout={layout} out_parity={p} dagger={dagger}", flush=True)
    fin = D.field(q.QDWF_F32, 1 - p, zero=False)
    q.qdwf_pack_spinor(D.ctx, fin, q.QDWF_F32, layout, psi_d, 1 - p)
    fout = D.field(q.QDWF_F32, p, zero=False)
    q.qdwf_apply_Deo(D.ctx, fout, fin, p, dagger, q.QDWF_F32, layout)
    del fin
    got = D.unpack(fout, q.QDWF_F32, layout, p, dtype=torch.complex64)
    del fout
    rel = _rel_dev(torch, got, _ref_dev(full, ("eo", p, dagger)))
    del got
    torch.cuda.empty_cache()
    print(f"  rel {rel:.3e}", flush=True)
    assert rel < TOL[1], (layout, p, dagger, rel)
