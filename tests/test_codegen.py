"""Checks on the gfx950 code the compiler generates for the hot kernels.

A buffer store wider than 64 bits reads its data VGPRs after it issues.
The compiler keeps VALU writes to those VGPRs two instructions away only
when the store's scalar offset is not a register; with a register scalar
offset, stale data reached memory on gfx950 (wrong first component of a
float4 in a few lanes).  Every wide buffer store must therefore use a
literal scalar offset, and no VALU op may overwrite its data VGPRs within
two instructions.
"""
from __future__ import annotations

import os
import re
import shutil
import subprocess
import sys
import tempfile
from functools import lru_cache

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

from paper_1702_08159_amd import build as hip_build  # noqa: E402

WIDE_STORE = re.compile(r"^(buffer|global|flat)_store_dwordx[34]\b")
VRANGE = re.compile(r"v\[(\d+):(\d+)\]")


@lru_cache(maxsize=None)
def _assembly(src: str, extra=()) -> str:
    try:
        cc = hip_build.hipcc()
    except RuntimeError:
        pytest.skip("hipcc not available")
    with tempfile.TemporaryDirectory() as tmp:
        out = os.path.join(tmp, "k.s")
        cmd = [cc, *hip_build.COMMON, *extra, "-S", "--offload-device-only", os.path.join(hip_build.CSRC, src),
               "-o", out]
        res = subprocess.run(cmd, capture_output=True, text=True)
        assert res.returncode == 0, res.stderr[-2000:]
        with open(out) as f:
            return f.read()


def _regs(operand: str):
    m = VRANGE.match(operand)
    if m:
        return set(range(int(m.group(1)), int(m.group(2)) + 1))
    m = re.match(r"v(\d+)$", operand)
    return {int(m.group(1))} if m else set()


def _exposed_stores(asm: str):
    lines = [l.strip() for l in asm.splitlines()]
    bad = []
    n_wide = 0
    for i, s in enumerate(lines):
        if not WIDE_STORE.match(s):
            continue
        n_wide += 1
        ops = [o.strip() for o in s.split(None, 1)[1].split(",")]
        data = ops[0] if s.startswith("buffer") else ops[1]
        if s.startswith("buffer"):
            soff = ops[3].split()[0]
            if soff.startswith("s"):
                bad.append(("register scalar offset", s))
                continue
        regs = _regs(data)
        waits = 0
        for t in lines[i + 1:i + 10]:
            if not t or t.startswith(";") or t.endswith(":") or t.startswith("."):
                continue
            if t.startswith("s_nop"):
                waits += int(t.split()[1]) + 1
                continue
            if waits >= 2:
                break
            if t.startswith("v_") and _regs(t.split()[1].rstrip(",")) & regs:
                bad.append(("data VGPR rewritten after %d wait states" % waits, s + "  ->  " + t))
                break
            waits += 1
    return n_wide, bad


def _hip_sources():
    return sorted(f for f in os.listdir(hip_build.CSRC) if f.endswith(".hip"))


def test_every_hip_source_is_checked():
    # the check below covers every HIP translation unit of the library
    assert set(_hip_sources()) == {s for s in hip_build.SOURCES if s.endswith(".hip")}


@pytest.mark.skipif(shutil.which("hipcc") is None and not os.path.exists("/opt/rocm/bin/hipcc"),
                    reason="hipcc not available")
@pytest.mark.parametrize("src", _hip_sources())
def test_wide_buffer_stores_have_no_data_hazard(src):
    extra = tuple(hip_build.SOURCES.get(src, []))
    n_wide, bad = _exposed_stores(_assembly(src, extra))
    if src in ("kernels.hip", "longn.hip", "head.hip", "train.hip"):
        assert n_wide > 0, src  # these issue 128-bit stores: the check must see them
    assert not bad, "\n".join("%s: %s" % b for b in bad[:10])


def test_checker_flags_register_soffset_and_early_rewrite():
    # the checker itself, on hand-written snippets
    asm = "\n".join([
        "buffer_store_dwordx4 v[4:7], v1, s[8:11], s12 offen nt",
        "v_mov_b32 v4, 0",
        "buffer_store_dwordx4 v[4:7], v1, s[8:11], 0 offen",
        "v_add_f32_e32 v5, v2, v3",
        "buffer_store_dwordx4 v[4:7], v1, s[8:11], 0 offen",
        "v_add_f32_e32 v9, v2, v3",
        "v_add_f32_e32 v8, v2, v3",
        "v_add_f32_e32 v4, v2, v3",
        "buffer_store_dword v4, v1, s[8:11], s12 offen",
    ])
    n_wide, bad = _exposed_stores(asm)
    assert n_wide == 3
    assert [b[0].split()[0] for b in bad] == ["register", "data"]


# Kernels of the measured paths that must keep every value in registers: a
# spill puts scratch traffic into the transform loops.  Patterns are on the
# mangled names (k_forward at n = 1024, every aligned-row backward with
# parameter gradients, the fused training-step kernels).
NO_SCRATCH = {
    "kernels.hip": [r"9k_forwardILi10ELi4E", r"15k_backward_rowsILi\d+ELb1ELb1E"],
    "train.hip": [r"16k_forward_logitsILi10ELb1E", r"16k_head_bwd_fusedILi10ELb1E"],
}


def _private_segment_sizes(asm: str):
    sizes, cur = {}, None
    for line in asm.splitlines():
        t = line.strip()
        if t.startswith(".amdhsa_kernel "):
            cur = t.split()[1]
        elif cur and t.startswith(".amdhsa_private_segment_fixed_size "):
            sizes[cur] = int(t.split()[1])
            cur = None
    return sizes


@pytest.mark.skipif(shutil.which("hipcc") is None and not os.path.exists("/opt/rocm/bin/hipcc"),
                    reason="hipcc not available")
@pytest.mark.parametrize("src", sorted(NO_SCRATCH))
def test_hot_kernels_use_no_scratch(src):
    sizes = _private_segment_sizes(_assembly(src, tuple(hip_build.SOURCES.get(src, []))))
    for pat in NO_SCRATCH[src]:
        hit = {k: v for k, v in sizes.items() if re.search(pat, k)}
        assert hit, pat
        assert all(v == 0 for v in hit.values()), {k: v for k, v in hit.items() if v}


def test_private_segment_parser():
    asm = "\n".join([
        "\t.amdhsa_kernel _Z1a", "\t\t.amdhsa_private_segment_fixed_size 0", "\t.end_amdhsa_kernel",
        "\t.amdhsa_kernel _Z1b", "\t\t.amdhsa_private_segment_fixed_size 36", "\t.end_amdhsa_kernel",
    ])
    assert _private_segment_sizes(asm) == {"_Z1a": 0, "_Z1b": 36}
