"""The oracle's Philox4x32-10 (Salmon et al., SC'11) bit for bit against
rocRAND's header-only engine, a third implementation of the published
generator, built here for the host: random counters and keys, and the
edge words 0 and 2^32 - 1 in every position."""
import os
import shutil
import subprocess

import numpy as np
import pytest

from oracle import oracle as O

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_philox_matches_rocrand(tmp_path):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    exe = str(tmp_path / "host_philox")
    subprocess.run([hipcc, "-O2", "-std=c++17", os.path.join(ROOT, "tests", "host_philox_rocrand.cpp"), "-o", exe],
                   check=True, capture_output=True)
    rng = np.random.default_rng(20191907)
    ins = rng.integers(0, 2 ** 32, size=(3000, 6), dtype=np.uint64)
    edge = np.array([0, 1, 2 ** 31, 2 ** 32 - 1], dtype=np.uint64)
    extra = []
    for pos in range(6):
        for v in edge:
            row = np.zeros(6, dtype=np.uint64)
            row[pos] = v
            extra.append(row)
    extra.append(np.full(6, 2 ** 32 - 1, dtype=np.uint64))
    ins = np.concatenate([ins, np.array(extra)])
    text = "\n".join(" ".join(str(int(x)) for x in row) for row in ins)
    out = subprocess.run([exe], input=text, capture_output=True, text=True, check=True).stdout.split("\n")
    ref = np.array([[int(t) for t in line.split()] for line in out if line.strip()], dtype=np.uint64)
    assert ref.shape == (len(ins), 4)
    mine = np.array([O.philox(r[:4].astype(np.uint32), r[4:].astype(np.uint32)) for r in ins], dtype=np.uint64)
    assert np.array_equal(mine, ref)
    # the outputs are not trivially the inputs
    assert not np.array_equal(mine, ins[:, :4])
