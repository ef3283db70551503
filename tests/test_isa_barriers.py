"""Every loop that executes a workgroup barrier must be uniform in the gfx950 code.

When the compiler cannot prove a loop's trip count (or exit condition) uniform
across a wave, it structures the loop per lane: lanes are masked out of it
one by one ("s_andn2_b64 exec, exec, ...") while the wave keeps iterating.
Barriers inside such a loop stop pairing up between the waves of a
workgroup -- a dependency-flag kernel hung that way, and a residual kernel
raced on its LDS staging.  This test compiles each HIP source to gfx950
assembly and checks, for every loop that (with its nested loops) contains
s_barrier, that the loop's own blocks never mask lanes out.  No GPU needed.
"""
import os
import re
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1607_06303_amd", "csrc")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


def divergent_barrier_loops(asm: str):
    """(function, loop header) pairs of divergent loops containing s_barrier."""
    out = []
    for fn in re.split(r"\n(?=_Z\S*:)", asm):
        m = re.match(r"(_Z\S*):", fn)
        if not m:
            continue
        lines = fn.splitlines()
        blocks, cur = [], None
        for i, line in enumerate(lines):
            b = re.match(r"^(\.LBB\d+_\d+|; %bb\.\d+):", line)
            if b:
                if cur:
                    blocks.append(cur)
                name = b.group(1)
                hdr = None
                h = re.search(r"Header=(BB\d+_\d+)", line)
                if h:
                    hdr = h.group(1)
                nxt = lines[i + 1] if i + 1 < len(lines) else ""
                if "Loop Header" in line or ("Loop Header" in nxt and nxt.strip().startswith(";")):
                    hdr = "BB" + name.split("LBB")[1] if "LBB" in name else name
                cur = [i, i, hdr]
            elif cur:
                cur[1] = i
        if cur:
            blocks.append(cur)
        loops = {}
        for i, line in enumerate(lines):
            h = re.match(r"^\.(LBB\d+_\d+):", line)
            if not h:
                continue
            name = "BB" + h.group(1).split("LBB")[1]
            kids, j = [], i + 1
            while j < len(lines) and lines[j].strip().startswith(";"):
                c = re.search(r"Child Loop (BB\d+_\d+)", lines[j])
                if c:
                    kids.append(c.group(1))
                j += 1
            if kids or "Loop Header" in "".join(lines[i:i + 2]):
                loops[name] = kids
        for hdr, kids in loops.items():
            members = [hdr] + kids
            body = [x for b in blocks if b[2] in members for x in range(b[0], b[1] + 1)]
            own = [x for b in blocks if b[2] == hdr for x in range(b[0], b[1] + 1)]
            barriers = sum("s_barrier" in lines[x] for x in body)
            masked = sum(bool(re.search(r"s_andn2_b64 exec, exec", lines[x])) for x in own)
            if barriers and masked:
                out.append((m.group(1), hdr))
    return out


def test_checker_flags_a_divergent_barrier_loop():
    # a loop whose lanes leave one by one, with a barrier inside
    asm = """_Zfoo:
.LBB0_1:                                ; =>This Loop Header: Depth=1
	s_barrier
	s_andn2_b64 exec, exec, s[4:5]
	s_cbranch_execnz .LBB0_1
	s_endpgm
"""
    assert divergent_barrier_loops(asm) == [("_Zfoo", "BB0_1")]
    assert divergent_barrier_loops(asm.replace("s_barrier", "s_nop 0")) == []


@pytest.mark.skipif(not shutil.which(HIPCC) and not os.path.exists(HIPCC), reason="no hipcc")
@pytest.mark.parametrize("src", sorted(f for f in os.listdir(CSRC) if f.endswith(".hip")))
def test_no_divergent_barrier_loops(src):
    cmd = [HIPCC, "-std=c++17", "-O3", "--offload-arch=gfx950", "--cuda-device-only", "-S",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "-I" + os.path.join(ROOT, "include"), "-o", "-", os.path.join(CSRC, src)]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stderr[-2000:]
    bad = divergent_barrier_loops(r.stdout)
    assert not bad, "loops with barriers compiled as divergent: %s" % bad
