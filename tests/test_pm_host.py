"""Host check of the +/- packing index arithmetic against the dense definitions.
The element functions define every packed value; the tiled block bodies that the
pack and D-unpack kernels run are executed on the host with one thread and must
match the element functions bit for bit."""
import os
import shutil
import subprocess
import tempfile

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.mark.skipif(shutil.which("hipcc") is None and not os.path.exists("/opt/rocm/bin/hipcc"), reason="needs hipcc")
def test_pm_index_arithmetic_on_host():
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    with tempfile.TemporaryDirectory() as d:
        exe = os.path.join(d, "pm_check")
        cmd = [hipcc, "--offload-arch=gfx950", "-O1", "-g", "-fno-gpu-sanitize", "-fsanitize=address,undefined",
               "-std=c++17", "-o", exe, os.path.join(HERE, "pm_index_check.cpp"), "-x", "none"]
        res = subprocess.run(cmd, capture_output=True, text=True)
        assert res.returncode == 0, res.stderr[-3000:]
        run = subprocess.run([exe], capture_output=True, text=True, timeout=300)
        print(run.stdout)
        assert run.returncode == 0, run.stdout + run.stderr[-3000:]
        assert run.stdout.strip().endswith("OK")
