"""cmc_pair_cells against the oracle's pairing, bit for bit."""
import numpy as np
import pytest

from oracle import oracle as O

pytestmark = pytest.mark.gpu


def _case(na, nb, seed=0):
    rng = np.random.default_rng(seed)
    na, nb = np.asarray(na, np.int64), np.asarray(nb, np.int64)
    a_off = np.concatenate([[0], np.cumsum(na)]).astype(np.int64)
    b_off = np.concatenate([[0], np.cumsum(nb)]).astype(np.int64)
    npair = np.where((na > 0) & (nb > 0), np.maximum(na, nb), 0)
    p_off = np.concatenate([[0], np.cumsum(npair)]).astype(np.int64)
    wa = rng.lognormal(0, 1, int(a_off[-1]))
    wb = rng.lognormal(0, 1, int(b_off[-1]))
    return a_off, b_off, p_off, wa, wb


@pytest.mark.parametrize("pass_", [1, 2])
def test_pairing_bit_exact(pass_):
    import torch
    import paper_1907_02814_amd as cmc
    rng = np.random.default_rng(11)
    na = [0, 5, 1, 1, 7, 3, 4096, 8192, 1, 100, 16384, 2] + list(rng.integers(1, 3000, 40))
    nb = [5, 0, 1, 7, 1, 3, 4096, 37, 8192, 100, 16384, 2] + list(rng.integers(1, 3000, 40))
    a_off, b_off, p_off, wa, wb = _case(na, nb)
    t = lambda x: torch.from_numpy(x).cuda()
    for step in (0, 7, 2 ** 40 + 3):
        pa, pb, nab = cmc.pair_cells(t(a_off), None, t(b_off), None, t(wa), t(wb), 99, step, pass_,
                                     t(p_off))
        opa, opb, onab = O.pair_cells(a_off, None, b_off, None, wa, wb, 99, step, pass_, p_off)
        assert np.array_equal(pa.cpu().numpy(), opa)
        assert np.array_equal(pb.cpu().numpy(), opb)
        np.testing.assert_allclose(nab.cpu().numpy(), onab, rtol=1e-13, atol=0)


def test_pairing_live_counts():
    import torch
    import paper_1907_02814_amd as cmc
    na = np.array([10, 20, 30]); nb = np.array([15, 5, 30])
    a_off, b_off, _, wa, wb = _case(na, nb)
    a_cnt = np.array([4, 20, 0], np.int32); b_cnt = np.array([15, 2, 30], np.int32)
    npair = np.where((a_cnt > 0) & (b_cnt > 0), np.maximum(a_cnt, b_cnt), 0)
    p_off = np.concatenate([[0], np.cumsum(npair)]).astype(np.int64)
    t = lambda x: torch.from_numpy(x).cuda()
    pa, pb, nab = cmc.pair_cells(t(a_off), t(a_cnt), t(b_off), t(b_cnt), t(wa), t(wb), 5, 1, 1, t(p_off))
    opa, opb, onab = O.pair_cells(a_off, a_cnt, b_off, b_cnt, wa, wb, 5, 1, 1, p_off)
    assert np.array_equal(pa.cpu().numpy(), opa) and np.array_equal(pb.cpu().numpy(), opb)
