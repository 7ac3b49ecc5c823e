"""Host check of the symmetric split of the on-the-fly products (the index
arithmetic in csrc/sym_split.hpp, compiled here with g++): every block on or
above the diagonal in exactly one unit, the workgroup ranges contiguous and
balanced, the epilogue's slot lists, and a double-precision replay of the
kernels' accumulation (direct slot per unit, transposed slots per
workgroup and strip) that reproduces M V on a random symmetric matrix with a
ragged last block."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(os.path.dirname(HERE), "paper_2405_03474_amd", "csrc")


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_symmetric_split_partition_and_replay(tmp_path):
    exe = str(tmp_path / "sym_split_check")
    subprocess.run(["g++", "-O2", "-std=c++17", f"-I{CSRC}", "-o", exe,
                    os.path.join(HERE, "host", "sym_split_check.cpp")], check=True)
    out = subprocess.run([exe], capture_output=True, text=True, timeout=300)
    assert out.returncode == 0 and out.stdout.strip().endswith("OK"), out.stdout
