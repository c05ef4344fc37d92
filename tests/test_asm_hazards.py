"""CPU: the compiled gfx950 assembly keeps the scalar condition code intact
across the library's inline-assembly blocks.

The binned vote's emission narrows the exec mask around its staging store in
one assembly block (s_and_saveexec / ds_write / s_or); both scalar
instructions write SCC.  The block declares the clobber, so the compiler must
not keep a comparison's SCC live across it.  Without the declaration it did:
a loop-exit compare before the block and its conditional branch after it, so
the wide vote left its loop early (13 % of the votes at G = 360).  This test
compiles the kernels to assembly and checks every instruction that reads SCC
after an inline block has an SCC write between the two, and that every
barrier after such a block's LDS store is preceded by a wait for all LDS
operations (the compiler does not count the store itself).
"""
import re
import shutil
import subprocess

import pytest

from paper_2506_11547_amd import build

HIPCC = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"

# scalar ALU instructions that write SCC (compares, arithmetic with carry out,
# logic, shifts, bit counts, min/max); s_mov / s_cselect / s_load do not
_WRITES = re.compile(
    r"^\s*(s_cmp|s_cmpk|s_bitcmp|s_add_|s_addk|s_sub_|s_and_|s_or_|s_xor_|s_andn2|s_orn2|"
    r"s_nand|s_nor|s_xnor|s_lshl|s_lshr|s_ashr|s_bfe|s_bcnt|s_min_|s_max_|s_not_|s_abs|"
    r"s_absdiff|s_mul_hi|s_andn1|s_orn1|s_quadmask|s_wqm)")
# instructions that read SCC
_READS = re.compile(r"^\s*(s_cbranch_scc|s_cselect|s_addc|s_subb|s_cmov)")


def scc_reads_after_asm(asm_text: str) -> list[str]:
    """Instructions that read SCC after an inline-assembly block with no SCC
    write in between (in textual order, which is the order within a block;
    a label or branch ends the search)."""
    bad = []
    inside = pending = False
    for line in asm_text.split("\n"):
        if "ASMSTART" in line:
            inside = True
            continue
        if "ASMEND" in line:
            inside, pending = False, True
            continue
        if inside or not pending:
            continue
        s = line.strip()
        if _READS.match(s):
            bad.append(s)
            pending = False
        elif _WRITES.match(s) or s.startswith(".LBB") or s.startswith("s_branch") \
                or s.startswith("s_endpgm"):
            pending = False
    return bad


def barriers_after_asm_stores(asm_text: str) -> int:
    """Barriers reached while a staging store written in an inline-assembly
    block may still be in flight: the compiler does not count that store, so
    only its own lgkmcnt(0) wait before a barrier (which waits for every LDS
    operation of the wave) makes the store visible to the other waves."""
    bad = 0
    inside = pending = False
    for line in asm_text.split("\n"):
        s = line.strip()
        if "ASMSTART" in s:
            inside = True
            continue
        if "ASMEND" in s:
            inside = False
            continue
        if inside and s.startswith("ds_write"):
            pending = True
        elif s.startswith("s_waitcnt") and "lgkmcnt(0)" in s:
            pending = False
        elif s.startswith("s_barrier") and pending:
            bad += 1
    return bad


def test_scanner_finds_a_planted_hazard():
    text = "\n".join([
        "s_cmp_ge_i32 s22, s91",
        ";;#ASMSTART",
        "s_and_saveexec_b64 s[22:23], s[0:1]",
        "ds_write_b32 v4, v14",
        "s_or_b64 exec, exec, s[22:23]",
        ";;#ASMEND",
        "s_cbranch_scc1 .LBB8_141",
    ])
    assert scc_reads_after_asm(text) == ["s_cbranch_scc1 .LBB8_141"]
    fixed = text.replace(";;#ASMEND", ";;#ASMEND\ns_cmp_ge_i32 s22, s91")
    assert scc_reads_after_asm(fixed) == []
    assert barriers_after_asm_stores(text + "\ns_barrier") == 1
    assert barriers_after_asm_stores(text + "\ns_waitcnt lgkmcnt(0)\ns_barrier") == 0


@pytest.mark.skipif(not shutil.which(HIPCC) and not __import__("os").path.exists(HIPCC),
                    reason="hipcc not found")
def test_no_scc_read_after_inline_asm(tmp_path):
    src = build.CSRC / "rv_bin.hip"
    out = tmp_path / "rv_bin.s"
    flags = [f for f in build.HIPCC_FLAGS if f not in ("-shared", "-fPIC")]
    subprocess.run([HIPCC, *flags, "--cuda-device-only", "-S", str(src), "-o", str(out)],
                   check=True, capture_output=True)
    text = out.read_text()
    assert "s_and_saveexec_b64" in text and "ASMSTART" in text
    assert scc_reads_after_asm(text) == []
    assert barriers_after_asm_stores(text) == 0
