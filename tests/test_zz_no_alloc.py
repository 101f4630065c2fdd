"""cmc_collide_step_noalloc, the step for callers that cannot allocate
(its scratch is the library's static device array), against
cmc_collide_step with a caller workspace, through the C ABI: two calls in a
row, the second on a smaller workload, each compared bit for bit with the
workspace entry point on a copy of the same state (the same kernels run;
the static array keeps the first call's contents, which the second must
not see)."""
import ctypes as C

import numpy as np
import pytest

from paper_1907_02814_amd import workloads as W

pytestmark = pytest.mark.gpu


def _live(d, c):
    off = d["off"]
    n = int(d["count"][c]) if d.get("count") is not None else int(off[c + 1] - off[c])
    return [d[k][int(off[c]):int(off[c]) + n] for k in ("px", "py", "pz", "w")]


def _host(g):
    return {k: (None if v is None else v.cpu().numpy()) for k, v in g.items()}


def _same(ga, sa, gb, sb):
    assert np.array_equal(sa.ti.cpu().numpy(), sb.ti.cpu().numpy())
    assert np.array_equal(sa.td.cpu().numpy(), sb.td.cpu().numpy())
    assert int(sa.status.item()) == int(sb.status.item())
    n = sa.ti.shape[0]
    for name in ("electrons", "photons", "new_el", "new_po"):
        A, B = _host(getattr(ga, name)), _host(getattr(gb, name))
        if A.get("count") is not None:
            assert np.array_equal(A["count"], B["count"]), name
        for c in range(n):
            for x, y in zip(_live(A, c), _live(B, c)):
                assert np.array_equal(x, y), (name, c)


def test_noalloc_matches_the_workspace_entry_point():
    import torch
    import paper_1907_02814_amd as cmc
    from gpu_parity import gpu_tables
    assert cmc.get_lib().cmc_noalloc_max_cells() == 16384
    # a larger workload first, then a smaller one: uneven cells, all three
    # processes, a time step amplified so that events, sequential-step cells
    # and open pairs are many
    loads = [W.cfg3(np.random.default_rng(81), n_cells=700, dt=2e-14, lo=4, hi=3000),
             W.cfg3(np.random.default_rng(82), n_cells=90, dt=2e-14, lo=4, hi=600)]
    events = 0
    for li, wl in enumerate(loads):
        ga, gb = wl.copy().to_torch("cuda:0"), wl.copy().to_torch("cuda:0")

        def state(g, sched):
            return cmc.StepState(gpu_tables(wl.Z), g.cells, g.electrons, g.photons, g.ions, g.new_el, g.new_po,
                                 dt=wl.dt, seed=1, processes=wl.processes, precision=cmc.FP32, schedule=sched)
        sa = state(ga, cmc.SCHED_GROUP)
        sb = state(gb, cmc.SCHED_AUTO)     # untimed here: workgroup teams
        for s in range(2):
            sa.step(s)
            sb.step(s, noalloc=True)
            torch.cuda.synchronize()
            _same(ga, sa, gb, sb)
            events += int(sa.ti[:, 3:6].sum().item())
        print(f"[noalloc] workload {li}: {wl.n_cells} cells, identical to the workspace entry point")
    assert events > 1000
