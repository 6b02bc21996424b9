"""Static check of the grouped DPP FMAs of the hop kernels in the gfx950
assembly.

The t-sweep and the checkerboard kernel apply the shifts of the fifth
dimension (s +- 1, and s +- 2^j in the M_ee^-1 scan) with v_fmac_f32_dpp
(row rotates), written as inline assembly in groups of six behind one
`s_nop 1`: the two wait states a DPP read needs after a VALU write
of its source cover the whole group only if no FMA in a group reads (through
DPP or as its multiplier) a register that an earlier FMA of the same group
wrote. The helper guarantees that by construction (distinct live values get
distinct registers); this test compiles sweep.hip and hop.hip for gfx950
exactly as the build does and checks every group in the generated code, so that a compiler
that allocated registers otherwise would be caught on the CPU.
"""
import os
import re
import subprocess

import pytest

from paper_2112_01852_amd import build as B


def _hipcc():
    try:
        return B.hipcc()
    except RuntimeError:
        return None


PAT = re.compile(r"v_fmac_f32_dpp\s+(v\d+),\s*(v\d+),\s*(v\d+)")


def _groups(lines):
    """Number of DPP FMA runs; AssertionError on a run that does not follow
    an s_nop 1, is longer than six, or reads a register written earlier in
    the run."""
    groups, i = 0, 0
    while i < len(lines):
        if lines[i].startswith("v_fmac_f32_dpp"):
            assert i > 0 and lines[i - 1] == "s_nop 1", (i, lines[i - 1], lines[i])
            written = set()
            while i < len(lines) and lines[i].startswith("v_fmac_f32_dpp"):
                dst, src, mul = PAT.match(lines[i]).groups()
                assert src not in written and mul not in written, (i, lines[i], sorted(written))
                written.add(dst)
                i += 1
            assert len(written) <= 6
            groups += 1
        else:
            i += 1
    return groups


def test_checker_catches_a_hazard():
    ok = ["s_nop 1", "v_fmac_f32_dpp v10, v20, v1 row_ror:1", "v_fmac_f32_dpp v11, v21, v1 row_ror:1"]
    assert _groups(ok) == 1
    with pytest.raises(AssertionError):
        _groups(["s_nop 1", "v_fmac_f32_dpp v10, v20, v1 row_ror:1", "v_fmac_f32_dpp v11, v10, v1 row_ror:1"])
    with pytest.raises(AssertionError):
        _groups(["v_add_f32_e32 v20, v2, v3", "v_fmac_f32_dpp v10, v20, v1 row_ror:1"])


_ASM = {}


def _asm(tmp_path_factory, src):
    """The gfx950 assembly of one source, built with the library's device
    flags (compiled once per test session)."""
    if src not in _ASM:
        out = tmp_path_factory.mktemp("asm") / (src + ".s")
        cmd = [_hipcc(), "-x", "hip", f"--offload-arch={B.ARCH}", "-O3", "-std=c++17",
               "-I", B.INCLUDE, "-I", B.CSRC, *B.DEVICE_FLAGS, "--cuda-device-only", "-S",
               os.path.join(B.CSRC, src), "-o", str(out)]
        r = subprocess.run(cmd, capture_output=True, text=True)
        assert r.returncode == 0, r.stderr[-2000:]
        _ASM[src] = [l.strip() for l in out.read_text().splitlines()]
    return _ASM[src]


@pytest.mark.skipif(_hipcc() is None, reason="hipcc not available")
@pytest.mark.parametrize("src", ["sweep.hip", "hop.hip"])
def test_grouped_dpp_fmas_read_no_register_written_in_their_group(tmp_path_factory, src):
    assert _groups(_asm(tmp_path_factory, src)) > 0


@pytest.mark.skipif(_hipcc() is None, reason="hipcc not available")
@pytest.mark.parametrize("src", ["sweep.hip", "hop.hip", "group.hip"])
def test_no_packed_fp32_and_no_accumulating_dot2(tmp_path_factory, src):
    """The device flags keep packed-FP32 arithmetic out of every kernel and
    select the three-operand dot products: no v_pk_{add,mul,fma}_f32 and no
    two-operand v_dot2c_f32_{f16,bf16} in the hop kernels' code, while the
    16-bit paths do use v_dot2_f32_f16 / v_dot2_f32_bf16."""
    lines = _asm(tmp_path_factory, src)
    ops = [l.split()[0] for l in lines if l.startswith("v_")]
    bad = sorted({o for o in ops if re.match(r"v_pk_(add|mul|fma)_f32", o)})
    assert not bad, bad
    acc = sorted({o for o in ops if o.startswith("v_dot2c_f32_")})
    assert not acc, acc
    if src != "sweep.hip":
        assert "v_dot2_f32_f16" in ops and "v_dot2_f32_bf16" in ops
