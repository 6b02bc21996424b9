"""HIP path vs the FP64 oracle, element by element, through the C ABI.

Tolerances (relative L2 over all reals of the output field, oracle evaluated
on the original FP64 inputs): FP64 1e-13, FP32 1e-6, FP16/BF16 storage 5e-3.
Lattices are chosen so that the number of 4D sites per parity is not a
multiple of the sites per block (ragged last block) and so that Ls = 12
leaves idle lanes in every wavefront.
"""
import numpy as np
import pytest

from oracle import cpu, geometry
from paper_2112_01852_amd import inputs as I

pytestmark = pytest.mark.gpu

TOL = {0: 1e-13, 1: 1e-6, 2: 5e-3, 3: 5e-3}
MOBIUS = dict(M5=1.8, mf=0.01, b=1.5, c=0.5)
SHAMIR = dict(M5=1.8, mf=0.01, b=1.0, c=0.0)


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


class Case:
    def __init__(self, q, L, Ls, params, seed=100, kind="haar", nrhs=1):
        self.q = q
        self.a = cpu.Action(L=L, Ls=Ls, **params)
        self.U = I.gauge_field(L, kind, seed)
        self.psi = I.gaussian_spinor(L, Ls, seed + 1)
        self.D = q.Dirac(L, Ls, **params)
        self.D.set_gauge(self.U)

    def run_full(self, op, prec, layout, dagger):
        q, D = self.q, self.D
        f = D.pack(self.psi, prec, layout, q.QDWF_FULL)
        out = D.field(prec, q.QDWF_FULL)
        op(D.ctx, out, f, dagger, prec, layout)
        return D.unpack(out, prec, layout, q.QDWF_FULL).cpu().numpy()


CASES = [
    ((4, 6, 2, 6), 8, MOBIUS),     # Vh = 144 over 32 sites per block: ragged
    ((6, 2, 2, 6), 16, MOBIUS),    # Vh = 72 over 16: ragged
    ((4, 2, 4, 6), 12, MOBIUS),    # Ls = 12: 4 idle lanes per wavefront
    ((4, 4, 4, 4), 8, SHAMIR),     # the Shamir FP64 workload shape
    ((6, 6, 10, 6), 16, MOBIUS),   # partial traversal tiles and uneven XCD slabs; Vh = 1080
]


@pytest.fixture(scope="module", params=range(len(CASES)))
def case(q, request):
    L, Ls, params = CASES[request.param]
    c = Case(q, L, Ls, params, seed=1000 + request.param)
    yield c
    c.D.close()


def test_geometry_tables_bit_exact(q):
    """The kernels' tables equal the enumerated ones under the library's site
    numbering (a bijection per parity, exported with the tables)."""
    for L in [(4, 6, 2, 6), (2, 2, 2, 2), (8, 4, 6, 2), (4, 4, 16, 4)]:
        D = q.Dirac(L, 4)
        idx, nbr, sign = q.qdwf_geometry_tables(D.ctx, D.V)
        cb0, par, nbr0, sign0 = geometry.tables(L)
        Vh = D.V // 2
        perm = np.zeros((2, Vh), dtype=np.int64)   # lex//2 order -> internal index
        for p in (0, 1):
            assert np.array_equal(np.sort(idx[par == p]), np.arange(Vh))
            perm[p][cb0[par == p]] = idx[par == p]
        for p in (0, 1):
            exp_nbr = np.empty_like(nbr0[p])
            exp_sign = np.empty_like(sign0[p])
            exp_nbr[perm[p]] = perm[1 - p][nbr0[p]]
            exp_sign[perm[p]] = sign0[p]
            assert np.array_equal(nbr[p], exp_nbr)
            assert np.array_equal(sign[p], exp_sign)
        D.close()


@pytest.mark.parametrize("layout", [0, 1])
def test_pack_unpack_roundtrip_exact(case, layout):
    q, D = case.q, case.D
    for subset in (q.QDWF_EVEN, q.QDWF_ODD, q.QDWF_FULL):
        f = D.pack(case.psi, q.QDWF_F64, layout, subset)
        back = D.unpack(f, q.QDWF_F64, layout, subset).cpu().numpy()
        expect = case.psi if subset == q.QDWF_FULL else cpu.restrict(case.psi, case.a.L, subset)
        assert np.array_equal(back, expect)


@pytest.mark.parametrize("prec", [0, 1, 2, 3])
@pytest.mark.parametrize("layout", [0, 1])
@pytest.mark.parametrize("dagger", [0, 1])
def test_apply_D(case, prec, layout, dagger):
    ref = cpu.dwf(case.a, case.U, case.psi, dagger=bool(dagger))
    got = case.run_full(case.q.qdwf_apply_D, prec, layout, dagger)
    assert _rel(got, ref) < TOL[prec]


@pytest.mark.parametrize("prec", [0, 1, 3])
@pytest.mark.parametrize("dagger", [0, 1])
@pytest.mark.parametrize("which", [0, 1])
def test_apply_Mee(case, prec, dagger, which):
    q, D, a = case.q, case.D, case.a
    layout = q.QDWF_RIRI
    for subset in (q.QDWF_EVEN, q.QDWF_ODD, q.QDWF_FULL):
        f = D.pack(case.psi, prec, layout, subset)
        out = D.field(prec, subset)
        q.qdwf_apply_Mee(D.ctx, out, f, subset, dagger, which, prec, layout)
        got = D.unpack(out, prec, layout, subset).cpu().numpy()
        src = case.psi if subset == q.QDWF_FULL else cpu.restrict(case.psi, a.L, subset)
        ref = cpu.mee(a, src, dagger=bool(dagger), inverse=bool(which))
        if subset != q.QDWF_FULL:
            ref = cpu.restrict(ref, a.L, subset)
        assert _rel(got, ref) < TOL[prec]


@pytest.mark.parametrize("prec", [0, 1, 2])
@pytest.mark.parametrize("layout", [0, 1])
def test_apply_Deo(case, prec, layout):
    q, D, a = case.q, case.D, case.a
    for p in (0, 1):
        for dagger in (0, 1):
            f = D.pack(case.psi, prec, layout, 1 - p)
            out = D.field(prec, p)
            q.qdwf_apply_Deo(D.ctx, out, f, p, dagger, prec, layout)
            got = D.unpack(out, prec, layout, p).cpu().numpy()
            ref = cpu.deo(a, case.U, cpu.restrict(case.psi, a.L, 1 - p), p, dagger=bool(dagger))
            assert _rel(got, ref) < TOL[prec]


@pytest.mark.parametrize("prec", [0, 1, 2, 3])
@pytest.mark.parametrize("layout", [0, 1])
def test_apply_Mpc_and_MdagM(case, prec, layout):
    # M_pc's second hop takes chi = (A/b) M_ee^-1 M_eo in from its first stage;
    # FP16 in the interleaved layout runs the packed-FP16 hop
    q, D, a = case.q, case.D, case.a
    src = cpu.restrict(case.psi, a.L, 1)
    f = D.pack(src, prec, layout, q.QDWF_ODD)
    ws = D.workspace(q.QDWF_OP_MDAGM, prec)
    for dagger in (0, 1):
        out = D.field(prec, q.QDWF_ODD)
        q.qdwf_apply_Mpc(D.ctx, out, f, dagger, prec, layout, 1, ws)
        got = D.unpack(out, prec, layout, q.QDWF_ODD).cpu().numpy()
        assert _rel(got, cpu.mpc(a, case.U, src, dagger=bool(dagger))) < TOL[prec]
    out = D.field(prec, q.QDWF_ODD)
    q.qdwf_apply_MdagM(D.ctx, out, f, prec, layout, 1, ws)
    got = D.unpack(out, prec, layout, q.QDWF_ODD).cpu().numpy()
    ref = cpu.mpc(a, case.U, cpu.mpc(a, case.U, src), dagger=True)
    assert _rel(got, ref) < TOL[prec]


def test_dot_matches_numpy(case):
    q, D, a = case.q, case.D, case.a
    chi = I.gaussian_spinor(a.L, a.Ls, 77)
    ws = D.workspace(q.QDWF_OP_REDUCE, q.QDWF_F64)
    for layout in (0, 1):
        x = D.pack(chi, q.QDWF_F64, layout, q.QDWF_FULL)
        y = D.pack(case.psi, q.QDWF_F64, layout, q.QDWF_FULL)
        got = q.qdwf_dot(D.ctx, x, y, q.QDWF_FULL, q.QDWF_F64, layout, 1, ws)[0]
        ref = np.vdot(chi.ravel(), case.psi.ravel())
        assert abs(got - ref) < 1e-12 * abs(ref) + 1e-12 * np.linalg.norm(chi) * np.linalg.norm(case.psi)


def test_multi_rhs_columns_equal_single_rhs(q):
    L, Ls, nrhs = (4, 6, 2, 6), 8, 5
    a = cpu.Action(L=L, Ls=Ls, **MOBIUS)
    U = I.gauge_field(L, "haar", 5)
    psi = I.gaussian_spinor(L, Ls, 6, nrhs=nrhs)
    D = q.Dirac(L, Ls, **MOBIUS)
    D.set_gauge(U)
    for prec in (0, 1):
        for dagger in (0, 1):
            f = D.pack(psi, prec, 1, q.QDWF_FULL, nrhs)
            out = D.field(prec, q.QDWF_FULL, nrhs)
            q.qdwf_apply_D(D.ctx, out, f, dagger, prec, 1, nrhs)
            got = D.unpack(out, prec, 1, q.QDWF_FULL, nrhs).cpu().numpy()
            for j in range(nrhs):
                f1 = D.pack(psi[j], prec, 1, q.QDWF_FULL)
                o1 = D.field(prec, q.QDWF_FULL)
                q.qdwf_apply_D(D.ctx, o1, f1, dagger, prec, 1, 1)
                one = D.unpack(o1, prec, 1, q.QDWF_FULL).cpu().numpy()
                assert np.array_equal(got[j], one)
                if prec == 0:
                    assert _rel(got[j], cpu.dwf(a, U, psi[j], dagger=bool(dagger))) < 1e-13
    D.close()


def test_deterministic_bitwise(case):
    q = case.q
    a1 = case.run_full(q.qdwf_apply_D, 1, 1, 0)
    a2 = case.run_full(q.qdwf_apply_D, 1, 1, 0)
    assert np.array_equal(a1, a2)


def test_free_field_plane_wave_on_gpu(q):
    """Unit links and a plane wave: the GPU D matches the momentum-space form."""
    from oracle import freefield
    a = cpu.Action(L=(4, 4, 4, 4), Ls=6, **MOBIUS)
    U = I.gauge_field(a.L, "unit", 0)
    p = freefield.momenta(a.L, a.bc, (1, 2, 0, 3))
    rng = np.random.default_rng(1)
    u = rng.standard_normal((a.Ls, 4, 3)) + 1j * rng.standard_normal((a.Ls, 4, 3))
    pw = freefield.plane_wave(a.L, a.Ls, p, u)
    expect = freefield.plane_wave(a.L, a.Ls, p, (freefield.dwf_momentum(a, p) @ u.reshape(-1, 3)
                                                ).reshape(a.Ls, 4, 3))
    D = q.Dirac(a.L, a.Ls, **MOBIUS)
    D.set_gauge(U)
    f = D.pack(pw, 0, 0, q.QDWF_FULL)
    out = D.field(0, q.QDWF_FULL)
    q.qdwf_apply_D(D.ctx, out, f, 0, 0, 0)
    got = D.unpack(out, 0, 0, q.QDWF_FULL).cpu().numpy()
    assert _rel(got, expect) < 1e-13
    D.close()


def test_invalid_arguments_raise_before_launch(q):
    D = q.Dirac((4, 4, 4, 4), 8)
    f = D.field(1)
    with pytest.raises(q.QdwfError) as e:
        q.qdwf_apply_D(D.ctx, f, f, 0, 1, 1)        # aliasing
    assert e.value.code == q.QDWF_EINVAL
    with pytest.raises(q.QdwfError):
        q.qdwf_apply_D(D.ctx, D.field(1), f, 0, 1, 1)  # gauge not set
    D.set_gauge(I.gauge_field((4, 4, 4, 4), "unit", 0))
    with pytest.raises(q.QdwfError):
        q.qdwf_apply_D(D.ctx, D.field(1), f, 0, 7, 1)  # precision
    with pytest.raises(q.QdwfError):
        q.qdwf_apply_D(D.ctx, D.field(1), f, 0, 1, 5)  # layout
    with pytest.raises(q.QdwfError):
        q.qdwf_create(q.make_action((3, 4, 4, 4), 8))   # odd extent
    with pytest.raises(q.QdwfError):
        q.qdwf_create(q.make_action((4, 4, 4, 4), 0))   # Ls below 1
    with pytest.raises(q.QdwfError):
        q.qdwf_create(q.make_action((4, 4, 4, 4), 65))  # Ls above 64
    D.close()
