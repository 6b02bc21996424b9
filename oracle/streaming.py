"""Oracle of the streaming probes: the per-site SU(3) product of the
Benchmark_su3 study (Section 4.2) and the STREAM triad (Section 3).

TEST INFRASTRUCTURE ONLY (see the package docstring). Both are their plain
definitions in FP64: a batched 3x3 complex matrix product and an axpy.
"""
from __future__ import annotations

import numpy as np

FLOPS_PER_SU3_MUL = 198   # 27 complex multiplies (6 flops) + 18 complex adds (2 flops)


def su3_mul(A, B) -> np.ndarray:
    """C[i] = A[i] @ B[i] for arrays of 3x3 complex matrices, shape (n, 3, 3)."""
    A = np.asarray(A, dtype=np.complex128)
    B = np.asarray(B, dtype=np.complex128)
    return np.matmul(A, B)


def triad(b, c, s: float) -> np.ndarray:
    """a = b + s c, elementwise, in FP64."""
    return np.asarray(b, dtype=np.float64) + float(s) * np.asarray(c, dtype=np.float64)
