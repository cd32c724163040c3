"""Host check of the FP32 sincos used by the phase kernels (Cody-Waite
reduction and Taylor polynomials): compiled for the CPU with hipcc and
compared with double-precision sin/cos."""
import os
import subprocess
import tempfile

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


def test_fast_sincosf_error_bound():
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    with tempfile.TemporaryDirectory() as d:
        exe = os.path.join(d, "sincos_check")
        subprocess.check_call([hipcc, "-O2", "-x", "hip", "--offload-arch=gfx950", "-o", exe,
                               os.path.join(HERE, "host", "sincos_check.cpp")],
                              stdout=subprocess.DEVNULL, stderr=subprocess.DEVNULL)
        out = subprocess.check_output([exe], timeout=300).decode().split()
    es, ec, es_big, ec_big = (float(x) for x in out)
    # values in [-1, 1]: half an ulp of 1 is 6e-8; allow a few ulp
    assert es < 3e-7 and ec < 3e-7, (es, ec)
    assert es_big < 3e-7 and ec_big < 3e-7, (es_big, ec_big)
