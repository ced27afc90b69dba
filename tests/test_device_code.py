"""Properties of the generated gfx950 device code (no GPU needed).

Every kernel addresses LDS with DS instructions and global memory with
global instructions: no FLAT memory instructions.  A pointer that may point
to either LDS or global memory makes the compiler emit FLAT accesses to the
LDS aperture, which the kernels here are not written to need.
"""
import glob
import os
import re
import subprocess

import pytest

from paper_2502_17632_amd import build_lib

SOURCES = sorted(glob.glob(os.path.join(build_lib.CSRC, "*.hip")))


@pytest.mark.parametrize("src", SOURCES, ids=[os.path.basename(s) for s in SOURCES])
def test_no_flat_memory_instructions(src, tmp_path):
    out = tmp_path / "dev.s"
    cmd = [build_lib.HIPCC, *build_lib.HIP_FLAGS, "--cuda-device-only", "-S", src, "-o", str(out)]
    subprocess.run(cmd, check=True, capture_output=True)
    kernel, bad = None, []
    for line in open(out):
        m = re.match(r"^(_Z\S+):", line)
        if m:
            kernel = m.group(1)
        if re.match(r"\s+flat_(load|store|atomic)", line):
            bad.append((kernel, line.strip()))
    assert not bad, bad[:5]
