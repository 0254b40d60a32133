"""The register transforms of the spectral kernels (DCT-II, DCT-III, DCT-IV
of every power-of-two length up to 128, and the 256-band DCT-II through two
halves), compiled for the host from the kernels' own header and checked
against their cosine definitions in long double (tests/host/dct_driver.cpp).
No device is used."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

pytestmark = pytest.mark.cpu


@pytest.mark.skipif(shutil.which("hipcc") is None, reason="no hipcc")
def test_register_transforms_match_their_definitions(tmp_path):
    exe = tmp_path / "dct_driver"
    cmd = ["hipcc", "-std=c++17", "-O2", f"-I{ROOT}/include", f"-I{ROOT}/paper_1504_06847_amd/csrc",
           os.path.join(ROOT, "tests", "host", "dct_driver.cpp"), "-o", str(exe)]
    subprocess.run(cmd, check=True, capture_output=True, cwd=tmp_path)
    r = subprocess.run([str(exe)], capture_output=True, text=True)
    print(r.stdout)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "ALL OK" in r.stdout
