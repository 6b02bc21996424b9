"""The flop convention of the benchmark against the paper's Table 3.

The hop on one 5D site is written here with the half-spinor projection
(project (1 -+ g_mu) psi to two spin components, multiply by the link,
reconstruct), using a complex type that counts real operations. The result
must equal the oracle's full 4x4 gamma-matrix hop, and the count must equal
the 1320 real flops per site update quoted in Table 3 (1416 when each complex
product is issued as 0 + z2*z3, as with the RIRI layout).
"""
import json
import os

import numpy as np

from oracle import cpu
from paper_2112_01852_amd import inputs as I

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "table3_flops.json")


class Counter:
    n = 0
    riri = False


class Z:
    """Complex number that counts real flops."""
    __slots__ = ("v",)

    def __init__(self, v):
        self.v = complex(v)

    def __add__(self, o):
        Counter.n += 2
        return Z(self.v + o.v)

    def __sub__(self, o):
        Counter.n += 2
        return Z(self.v - o.v)

    def __mul__(self, o):
        Counter.n += 6
        return Z(self.v * o.v)

    def times_i(self, sign):   # multiply by +-i: a register swap, no flop
        return Z(sign * 1j * self.v)

    def neg(self):
        return Z(-self.v)

    def conj(self):
        return Z(self.v.conjugate())


def mat_vec(U, h, dag):
    """3x3 complex matrix times colour vector: 9 products + 6 additions = 66 flops."""
    out = []
    for a in range(3):
        acc = None
        for b in range(3):
            m = U[b][a].conj() if dag else U[a][b]
            t = m * h[b]
            if acc is None:
                if Counter.riri:
                    Counter.n += 2       # fcmla computes 0 + z2*z3
                acc = t
            else:
                acc = acc + t
        out.append(acc)
    return out


# (1 - g_mu) psi = (h0, h1, r2, r3): h from psi, rows 2 and 3 from h.
# Entry format per mu: h0 = psi0 + c0 * psi[k0], h1 = psi1 + c1 * psi[k1];
# r2 = d2 * h[j2], r3 = d3 * h[j3]; c, d in {+-1, +-i}. (1 + g_mu) flips c and d.
PROJ = {
    0: ((3, -1j), (2, -1j), (1, 1j), (0, 1j)),
    1: ((3, 1), (2, -1), (1, -1), (0, 1)),
    2: ((2, -1j), (3, 1j), (0, 1j), (1, -1j)),
    3: ((2, -1), (3, -1), (0, -1), (1, -1)),
}


def scale(z, c):
    if c == 1:
        return z
    if c == -1:
        return z.neg()
    return z.times_i(1 if c == 1j else -1)


def project(psi, mu, sgn):
    (k0, c0), (k1, c1), _, _ = PROJ[mu]
    c0, c1 = sgn * c0, sgn * c1
    h0 = [psi[0][a] + scale(psi[k0][a], c0) for a in range(3)]
    h1 = [psi[1][a] + scale(psi[k1][a], c1) for a in range(3)]
    return h0, h1


def reconstruct_acc(acc, uh, mu, sgn, first):
    _, _, (j2, d2), (j3, d3) = PROJ[mu]
    d2, d3 = sgn * d2, sgn * d3
    rows = [uh[0], uh[1], [scale(z, d2) for z in uh[j2]], [scale(z, d3) for z in uh[j3]]]
    if first:
        return rows
    return [[acc[s][a] + rows[s][a] for a in range(3)] for s in range(4)]


def hop_one_site(U, psi_nb, dagger):
    """U[mu][fwd/bwd] 3x3 lists; psi_nb[mu][fwd/bwd] 4x3 lists of Z."""
    acc = None
    first = True
    fs = 1 if not dagger else -1       # sign multiplying the table for the forward hop
    for mu in range(4):
        for d, (dag, sg) in enumerate(((False, fs), (True, -fs))):
            h0, h1 = project(psi_nb[mu][d], mu, sg)
            uh = [mat_vec(U[mu][d], h0, dag), mat_vec(U[mu][d], h1, dag)]
            acc = reconstruct_acc(acc, uh, mu, sg, first)
            first = False
    return acc


def _site_inputs(seed):
    a = cpu.Action(L=(4, 4, 4, 4), Ls=1, M5=1.8, mf=0.01, b=1.0, c=0.0, bc=(1, 1, 1, 1))
    U = I.gauge_field(a.L, "haar", seed)
    psi = I.gaussian_spinor(a.L, 1, seed + 1)
    x = (1, 2, 3, 1)
    Ux, Uy = [], []
    for mu in range(4):
        f = list(x); f[mu] = (x[mu] + 1) % 4
        b = list(x); b[mu] = (x[mu] - 1) % 4
        Ux.append([[[Z(v) for v in row] for row in U[mu, x[3], x[2], x[1], x[0]]],
                   [[Z(v) for v in row] for row in U[mu, b[3], b[2], b[1], b[0]]]])
        Uy.append([[[Z(v) for v in sp] for sp in psi[0, f[3], f[2], f[1], f[0]]],
                   [[Z(v) for v in sp] for sp in psi[0, b[3], b[2], b[1], b[0]]]])
    return a, U, psi, x, Ux, Uy


def test_half_spinor_hop_equals_oracle_and_counts_1320(oracle_lib):
    golden = json.load(open(GOLDEN))
    for dagger in (False, True):
        a, U, psi, x, Ul, pl = _site_inputs(7)
        Counter.n, Counter.riri = 0, False
        out = hop_one_site(Ul, pl, dagger)
        assert Counter.n == golden["rrii_flops_per_site"]
        ref = cpu.hop(a, U, psi, dagger=dagger)[0, x[3], x[2], x[1], x[0]]
        got = np.array([[z.v for z in row] for row in out])
        assert np.abs(got - ref).max() < 1e-13


def test_riri_issue_count_is_1416(oracle_lib):
    golden = json.load(open(GOLDEN))
    a, U, psi, x, Ul, pl = _site_inputs(9)
    Counter.n, Counter.riri = 0, True
    hop_one_site(Ul, pl, False)
    Counter.riri = False
    assert Counter.n == golden["riri_flops_per_site"]
