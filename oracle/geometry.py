"""Checkerboard and neighbour tables by enumeration of lattice coordinates.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Definitions: lex = ((t*Lz+z)*Ly+y)*Lx+x; parity = (x+y+z+t) mod 2;
checkerboard index cb = lex // 2 (a bijection within each parity because Lx is
even); directions 0..7 = +x, +y, +z, +t, -x, -y, -z, -t; the neighbour table
holds the checkerboard index (in the opposite parity) of the neighbour, and the
sign table the boundary factor of that hop (bc[mu] when the hop wraps).
"""
from __future__ import annotations

import numpy as np


def tables(L, bc=(1, 1, 1, -1)):
    """Returns (cb_of_lex[V], parity_of_lex[V], nbr[2][V/2][8], sign[2][V/2][8])."""
    Lx, Ly, Lz, Lt = (int(v) for v in L)
    V = Lx * Ly * Lz * Lt
    cb_of_lex = np.empty(V, dtype=np.int32)
    par_of_lex = np.empty(V, dtype=np.int32)
    nbr = np.full((2, V // 2, 8), -1, dtype=np.int32)
    sign = np.zeros((2, V // 2, 8), dtype=np.int8)
    ext = (Lx, Ly, Lz, Lt)
    for t in range(Lt):
        for z in range(Lz):
            for y in range(Ly):
                for x in range(Lx):
                    c = (x, y, z, t)
                    lex = ((t * Lz + z) * Ly + y) * Lx + x
                    p = (x + y + z + t) % 2
                    cb_of_lex[lex] = lex // 2
                    par_of_lex[lex] = p
                    for d in range(8):
                        mu, step = d % 4, (1 if d < 4 else -1)
                        n = list(c)
                        n[mu] += step
                        f = 1
                        if n[mu] == ext[mu]:
                            n[mu] = 0
                            f = bc[mu]
                        elif n[mu] < 0:
                            n[mu] = ext[mu] - 1
                            f = bc[mu]
                        nl = ((n[3] * Lz + n[2]) * Ly + n[1]) * Lx + n[0]
                        nbr[p, lex // 2, d] = nl // 2
                        sign[p, lex // 2, d] = f
    return cb_of_lex, par_of_lex, nbr, sign
