"""GPU-built tables against the oracle's, node by node."""
import numpy as np
import pytest

from oracle import oracle as O

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("Z", [29, 79])
def test_tables_match_oracle(Z):
    from gpu_parity import gpu_tables
    import paper_1907_02814_amd as cmc
    g = gpu_tables(Z)
    o = O.tables(Z)
    for name in cmc.TABLE_NAMES:
        a, b = g.export(name), o.export(name)
        assert a.shape == b.shape, name
        assert np.all(np.isfinite(a)), name
        if name.startswith("cdf"):
            err = np.abs(a - b).max()
            assert err <= 2e-14, (name, err)
        else:
            nz = b != 0
            assert np.array_equal(a == 0, b == 0), name
            rel = np.abs(a[nz] / b[nz] - 1).max()
            assert rel <= 1e-13, (name, rel)
