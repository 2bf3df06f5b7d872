"""Regression checks on the generated gfx950 assembly of the contraction
kernels (CPU only: hipcc cross-compiles).

The pivoted LU exchanges rows with inline-asm blocks that narrow EXEC and
move registers (row k <- row m, row m <- saved row k).  Properties that
must hold in every such block:
* no scalar-condition (SCC) value of the surrounding code is live across it
  (the block writes SCC);
* no register the block reads was already written earlier in the block;
* the block restores EXEC from the value it saved.
"""
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "paper_1411_3691_amd", "csrc", "contract_kernels.hip")
HIPCC = "/opt/rocm/bin/hipcc"

SCC_DEF = ("s_cmp", "s_and_b", "s_or_b", "s_xor_b", "s_andn2", "s_orn2", "s_add_u32",
           "s_sub_u32", "s_lshl", "s_lshr", "s_ashr", "s_bfe", "s_min", "s_max", "s_add_i32",
           "s_sub_i32", "s_and_saveexec", "s_or_saveexec", "s_not", "s_bitcmp")
SCC_USE = ("s_cbranch_scc", "s_cselect", "s_cmovk", "s_cmov_", "s_addc_u32", "s_subb_u32")


@pytest.fixture(scope="module")
def asm(tmp_path_factory):
    if not os.path.exists(HIPCC):
        pytest.skip("hipcc not available")
    out = tmp_path_factory.mktemp("asm") / "k.s"
    cmd = [HIPCC, "-O3", "-std=c++17", "--offload-arch=gfx950", "-I", os.path.join(ROOT, "include"),
           "-I", os.path.dirname(SRC), "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "-x", "hip", "-S", "--cuda-device-only", SRC, "-o", str(out)]
    subprocess.run(cmd, check=True, capture_output=True)
    return out.read_text().split("\n")


def asm_blocks(lines):
    i = 0
    while i < len(lines):
        if "ASMSTART" in lines[i]:
            j = i + 1
            body = []
            while "ASMEND" not in lines[j]:
                t = lines[j].strip()
                if t and not t.startswith(";"):
                    body.append(t)
                j += 1
            yield i, j, body
            i = j
        i += 1


def vregs(tok):
    m = re.match(r"v\[(\d+):(\d+)\]", tok)
    if m:
        return set(range(int(m.group(1)), int(m.group(2)) + 1))
    m = re.match(r"v(\d+)$", tok)
    return {int(m.group(1))} if m else set()


def test_exchange_blocks_read_nothing_they_already_wrote(asm):
    n = 0
    for i, _, body in asm_blocks(asm):
        moves = [ins for ins in body if ins.startswith("v_mov")]
        if not moves:
            continue
        assert body[0].startswith("s_and_saveexec_b64") and body[-1].startswith("s_mov_b64 exec")
        saved = body[0].split(None, 1)[1].split(",")[0].strip()
        assert body[-1].split(",")[1].strip() == saved, f"line {i}: {body}"
        written = set()
        for ins in moves:
            dst, src = [p.strip() for p in ins.split(None, 1)[1].split(",")[:2]]
            assert not (vregs(src) & written), f"line {i}: {body}"
            written |= vregs(dst)
            n += 1
    assert n > 1000


def test_no_scc_value_lives_across_an_exchange_block(asm):
    # Empty asm statements (the ties that keep a solve inside its loop) emit
    # no instruction and do not write SCC; every block with an instruction
    # is taken to write it.
    last_def = None
    crossed = False
    in_asm = False
    nonempty = False
    for n, line in enumerate(asm):
        t = line.strip()
        if "ASMSTART" in t:
            in_asm = True
            nonempty = False
            continue
        if "ASMEND" in t:
            in_asm = False
            if nonempty:
                crossed = last_def is not None
            continue
        if in_asm:
            if t and not t.startswith(";"):
                nonempty = True
            continue
        if not t or t.startswith((".", ";")):
            continue
        op = t.split()[0]
        assert not (op.startswith(SCC_USE) and crossed), f"line {n}: {t} after {last_def}"
        if op.startswith(SCC_DEF):
            last_def = (n, t)
            crossed = False
