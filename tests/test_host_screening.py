"""The library's reduced screening length (eq:lambert-W, Sec. II.B.2), built
for the host from the same source as the kernels, against the oracle's: W0
from its series for I_TFD at or above (7 ln 2 - 1)/2 and from log1p below,
L_R = sqrt(-(1 + W)/W) and ln L_R = (u + ln(1 + W))/2 with u = W + 1 + 2a."""
import os
import shutil
import subprocess

import numpy as np
import pytest

from oracle import oracle as O

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_reduced_length_matches_the_oracle(tmp_path):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    exe = str(tmp_path / "host_screening")
    subprocess.run([hipcc, "-O2", "-std=c++17", "-I", os.path.join(ROOT, "paper_1907_02814_amd", "csrc"),
                    "-I", os.path.join(ROOT, "include"), os.path.join(ROOT, "tests", "host_screening.cpp"),
                    "-o", exe],
                   check=True, capture_output=True)
    a_star = (7.0 * np.log(2.0) - 1.0) / 2.0          # |z| = 2^-7: where the two starts meet
    a = np.concatenate([np.geomspace(0.01, 30.0, 600), a_star * np.array([1 - 1e-9, 1.0, 1 + 1e-9])])
    out = subprocess.run([exe], input="\n".join(repr(float(x)) for x in a), capture_output=True, text=True,
                         check=True).stdout
    v = np.array([[float(t) for t in line.split()] for line in out.splitlines()])
    assert v.shape == (len(a), 3)
    Lo = np.array([O.L_reduced(x) for x in a])
    np.testing.assert_allclose(v[:, 1], Lo, rtol=1e-14, atol=0)
    np.testing.assert_allclose(v[:, 2], np.log(Lo), rtol=0, atol=1e-14)
