"""CPU bounds check of the spatial-cycle tail kernel: a host build of
k_spatial_tail under AddressSanitizer and UBSan (tests/host_emu) runs every
launch shape the library can make, including the step counts nu1x = 1,
nu2x = 0 for which the library keeps the kernel switched off."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_spatial_tail_accesses_stay_in_bounds(tmp_path):
    import sys
    sys.path.insert(0, os.path.join(HERE, "host_emu"))
    import gen_tail
    gen_tail.generate(str(tmp_path))
    exe = str(tmp_path / "tail_emu")
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           "-fno-omit-frame-pointer", "-I", str(tmp_path), os.path.join(HERE, "host_emu", "tail_main.cpp"), "-o", exe]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    p = subprocess.run([exe], capture_output=True, text=True, timeout=300)
    assert p.returncode == 0, p.stderr[-4000:]
    assert "cases run: 6144" in p.stdout, p.stdout
