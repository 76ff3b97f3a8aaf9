"""Guard against a miscompilation seen with this toolchain: a select on a
vector compare (v_cmp ... vcc) lowered to s_cselect, which reads SCC -- a
flag left by unrelated scalar arithmetic -- instead of VCC.  It appeared in
single-lane loops over LDS data and silently produced wrong compaction
indices.  The kernels are written to avoid that shape; this test compiles
them to gfx950 assembly and fails if the pattern reappears."""
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2506_09611_amd", "csrc")
HIPCC = "/opt/rocm/bin/hipcc"

SCC_WRITERS = re.compile(r"^\s*s_(cmp|bitcmp|and|or|xor|andn2|orn2|nand|nor|xnor|add|addc|sub|subb|"
                         r"lshl|lshr|ashr|bfe|not|abs|min|max|bcnt|cselect_never)")


def suspicious_selects(asm: str):
    out = []
    lines = asm.splitlines()
    prev = []   # recent meaningful instructions
    for ln, line in enumerate(lines):
        s = line.strip()
        if not s or s.startswith((";", ".", "s_waitcnt")) or s.endswith(":"):
            continue
        if s.startswith("s_cselect"):
            # the instruction just before (ignoring v_mov) is a VALU compare writing VCC,
            # and the one before that does not set SCC
            p = [q for q in prev if not q.startswith("v_mov")]
            if p and re.match(r"v_cmp\w*_e32 vcc", p[-1]) and not (len(p) > 1 and SCC_WRITERS.match(p[-2])):
                out.append((ln + 1, s))
        prev = (prev + [s])[-6:]
    return out


@pytest.mark.parametrize("src", ["update.hip", "dense.hip", "gemm.hip"])
def test_no_vcc_select_via_scc(src, tmp_path):
    if not os.path.exists(HIPCC):
        pytest.skip("hipcc not available")
    out = tmp_path / (src + ".s")
    cmd = [HIPCC, "--offload-arch=gfx950", "-O3", "-std=c++17", "-x", "hip", "--offload-device-only",
           "-S", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           os.path.join(CSRC, src), "-o", str(out)]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    bad = suspicious_selects(out.read_text())
    assert not bad, f"{src}: s_cselect fed by a VCC compare at {bad[:5]}"


def test_guard_detects_the_pattern():
    asm = "\tds_read_b32 v3, v2 offset:512\n\ts_waitcnt lgkmcnt(0)\n\tv_cmp_eq_u32_e32 vcc, 0, v3\n\ts_cselect_b32 s9, -1, s8\n"
    assert suspicious_selects(asm)
    ok = "\ts_cmp_lg_u64 s[88:89], 0\n\tv_cmp_lt_i64_e32 vcc, s[48:49], v[2:3]\n\ts_cselect_b64 s[38:39], -1, 0\n"
    assert not suspicious_selects(ok)
