"""Register allocation of the inline-assembly LDS read blocks of the Gram
trainer (csrc/train.hip). Each block issues several ds_read_b128 from one
address register before it waits; if the compiler gave an output range the
address register, a read returning while the later ones are still being
issued would redirect them. The outputs are declared early-clobber; this
compiles the file for gfx950 and checks every such block of the result."""
import re
import subprocess
from pathlib import Path

import pytest

ROOT = Path(__file__).resolve().parents[1]
HIPCC = Path("/opt/rocm/bin/hipcc")


def overlapping_blocks(asm: str):
    """(number of asm blocks with ds_read_b128, blocks where an output range
    contains an address register)."""
    n, bad = 0, []
    for blk in re.findall(r";;#ASMSTART(.*?);;#ASMEND", asm, re.S):
        reads = re.findall(r"ds_read_b128 v\[(\d+):(\d+)\], v(\d+)", blk)
        if not reads:
            continue
        n += 1
        addrs = {int(a) for _, _, a in reads}
        if any(lo <= a <= hi for lo, hi in ((int(x), int(y)) for x, y, _ in reads) for a in addrs):
            bad.append(blk.strip().splitlines()[0])
    return n, bad


def test_checker_flags_an_overlap():
    ok = ";;#ASMSTART\n ds_read_b128 v[8:11], v4\n ds_read_b128 v[12:15], v4 offset:1024\n;;#ASMEND"
    bad = ";;#ASMSTART\n ds_read_b128 v[4:7], v4\n ds_read_b128 v[12:15], v4 offset:1024\n;;#ASMEND"
    assert overlapping_blocks(ok) == (1, [])
    assert overlapping_blocks(bad)[1] != []


@pytest.mark.skipif(not HIPCC.exists(), reason="hipcc not installed")
def test_lds_read_blocks_keep_addresses(tmp_path):
    out = tmp_path / "train.s"
    subprocess.run([str(HIPCC), "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-Xclang",
                    "-target-feature", "-Xclang", "-packed-fp32-ops", "-I", "include", "-x", "hip",
                    "--cuda-device-only", "-S", "paper_1504_01883_amd/csrc/train.hip", "-o",
                    str(out)], check=True, cwd=ROOT, capture_output=True, timeout=300)
    n, bad = overlapping_blocks(out.read_text())
    assert n >= 1, "no LDS read block found"
    assert bad == [], f"output ranges over the address register: {bad}"
