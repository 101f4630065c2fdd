"""Parity at the benchmark sizes, in the launch configuration bench.py times
(automatic schedule): cfg2 in full (4096 cells x (1024 photons + 1024 Au
ions), FP32 form) against the oracle; foil-chain cells at their full size
(4096 electrons + 4096 Au ions, all processes); cfg3 in full (16384 uneven
cells, all processes) on the GPU against the oracle on a sample of its
cells (the random numbers are keyed by the global cell index); the expected
yield and its adjoint on cfg4 in full (1024 cells x 4096 electrons), both
forms, against the oracle on every cell and electron."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1907_02814_amd import workloads as W

pytestmark = pytest.mark.gpu


def test_cfg2_full_size_fp32():
    import paper_1907_02814_amd as cmc
    from gpu_parity import Parity
    wl = W.cfg2()
    P = Parity(wl, precision=cmc.FP32)
    for s in range(2):
        P.step(s)
    print(f"[parity] cfg2 full: {P.flips} flip(s); " + ", ".join(f"{k} {v:.1e}" for k, v in P.errors.items()))
    assert P.flips <= 2
    assert P.state.ti.cpu().numpy()[:, 2].sum() > 4_000_000


def test_foil_cells_full_size_fp32():
    import paper_1907_02814_amd as cmc
    from gpu_parity import Parity
    wl = W.cfg5(np.random.default_rng(1005), n_cells=192)
    P = Parity(wl, precision=cmc.FP32)
    for s in range(2):
        P.step(s)
    print(f"[parity] cfg5 cells: {P.flips} flip(s); " + ", ".join(f"{k} {v:.1e}" for k, v in P.errors.items()))
    assert P.flips <= 2
    assert P.ref.photons["count"].sum() > 0


def test_cfg3_full_sampled_cells():
    import torch
    import paper_1907_02814_amd as cmc
    from gpu_parity import compare_sampled_cells, gpu_tables
    wl = W.cfg3()
    g = wl.copy().to_torch("cuda:0")
    st = cmc.StepState(gpu_tables(wl.Z), g.cells, g.electrons, g.photons, g.ions, g.new_el, g.new_po,
                       dt=wl.dt, seed=1, processes=wl.processes, precision=cmc.FP32)
    st.step(0)
    torch.cuda.synchronize()
    sample = np.sort(np.random.default_rng(5).choice(wl.n_cells, 256, replace=False))
    # the largest cells too
    big = np.argsort(np.diff(wl.electrons["off"]) + np.diff(wl.ions["off"]))[-8:]
    sample = np.unique(np.concatenate([sample, big]))
    ref = wl.subset(sample)
    oti, otd, ost = O.collide_step(O.tables(wl.Z), ref.cells, ref.electrons, ref.photons, ref.ions,
                                   ref.new_el, ref.new_po, wl.dt, 1, 0, wl.processes)
    flips = compare_sampled_cells(g, st, ref, sample, oti, otd, 1e-5)
    print(f"[parity] cfg3 full, {len(sample)} sampled cells: {flips} with a near-threshold decision")
    assert flips <= 2
    assert oti[:, 0:3].sum() > 1e5


def _near_energy_knot(gamma, tol):
    """Electrons whose energy lies within tol node spacings of a knot of
    the Bremsstrahlung energy axes (ln(g-1) on [ln(1 keV/mc^2), 0] with 23
    nodes, ln g on [ln 2, ln 100] with 56 and on [ln 100, ln 2e4] with 75;
    the segment joins g = 2 and g = 100 are knots).  There the adjoint
    differentiates a piecewise-linear interpolant across a kink, and a
    position rounded in FP32 may take the slope of the other side."""
    mec2_ev = 510998.95
    near = np.zeros(len(gamma), bool)
    for u, u0, u1, n in ((np.log(np.maximum(gamma - 1.0, 1e-300)), np.log(1000.0 / mec2_ev), 0.0, 23),
                         (np.log(gamma), np.log(2.0), np.log(100.0), 56),
                         (np.log(gamma), np.log(100.0), np.log(2.0e4), 75)):
        pos = (u - u0) / ((u1 - u0) / (n - 1))
        near |= (pos > -1.0) & (pos < n) & (np.abs(pos - np.round(pos)) <= tol)
    return near


@pytest.mark.parametrize("precision,rtol,rtol_g", [(0, 1e-12, 1e-11), (1, 1e-5, 2e-5)])
def test_cfg4_expected_yield_full_size(precision, rtol, rtol_g):
    import torch
    import paper_1907_02814_amd as cmc
    from gpu_parity import gpu_tables
    y = W.cfg4()
    g = {k: torch.from_numpy(np.ascontiguousarray(v)).cuda() for k, v in y.items() if isinstance(v, np.ndarray)}
    args = (g["Zstar"], g["n_e"], g["T_e"], g["off"], g["px"], g["py"], g["pz"], g["w"], y["dt"])
    oargs = (y["Zstar"], y["n_e"], y["T_e"], y["off"], y["px"], y["py"], y["pz"], y["w"], y["dt"])
    Y = cmc.expected_yield(gpu_tables(29), *args, precision).cpu().numpy()
    Yo = O.expected_yield(O.tables(29), *oargs)
    print(f"[parity] cfg4 yield, precision {precision}: max rel {np.max(np.abs(Y - Yo) / np.abs(Yo)):.1e}")
    np.testing.assert_allclose(Y, Yo, rtol=rtol, atol=0)
    gY = np.linspace(0.5, 2.0, len(y["Zstar"]))
    G = cmc.expected_yield_backward(gpu_tables(29), *args, torch.from_numpy(gY).cuda(), precision)
    Go = O.expected_yield_backward(O.tables(29), *oargs, gY)
    for k in ("gZstar", "gn_e", "gT_e", "gw"):
        a, b = G[k].cpu().numpy(), Go[k]
        assert np.all(np.abs(a - b) <= rtol_g * np.abs(b) + 1e-300 + 1e-12 * rtol_g * np.abs(b).max()), k
    a = np.stack([G[k].cpu().numpy() for k in ("gpx", "gpy", "gpz")])
    b = np.stack([Go[k] for k in ("gpx", "gpy", "gpz")])
    err = np.sqrt(((a - b) ** 2).sum(0)); mag = np.sqrt((b ** 2).sum(0))
    # FP32 form: per-electron gradients within FP32 resolution of an energy
    # knot (about 1e-5 node spacings) are excluded and counted
    gamma = np.sqrt(1.0 + y["px"] ** 2 + y["py"] ** 2 + y["pz"] ** 2)
    skip = _near_energy_knot(gamma, 3e-5) if precision == cmc.FP32 else np.zeros(len(gamma), bool)
    rel = err / np.maximum(mag, 1e-300)
    print(f"[parity] cfg4 adjoint, precision {precision}: max rel momentum gradient {np.max(rel[~skip]):.1e}; "
          f"{int(skip.sum())} electron(s) near a knot excluded, {int((rel[skip] > rtol_g).sum())} of them off")
    assert skip.sum() <= 1e-3 * len(gamma)
    assert np.all(err[~skip] <= rtol_g * mag[~skip] + 1e-300)
