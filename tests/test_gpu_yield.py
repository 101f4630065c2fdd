"""Expected yield and its adjoint on the GPU against the oracle; the
autograd.Function against central finite differences."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1907_02814_amd import workloads as W

pytestmark = pytest.mark.gpu


def _dev(d):
    import torch
    return {k: torch.from_numpy(np.ascontiguousarray(v)).cuda() for k, v in d.items()
            if isinstance(v, np.ndarray)}


def _inputs(n_cells=40, per_cell=600, seed=12):
    y = W.cfg4(np.random.default_rng(seed), n_cells=n_cells, per_cell=per_cell)
    # a few non-relativistic and sub-keV electrons, and clamped / unclamped cells
    y["px"][:5] = [0.9, 0.3, 0.05, 0.01, 1e-3]
    y["py"][:5] = 0.0; y["pz"][:5] = 0.0
    return y


@pytest.mark.parametrize("precision,rtol", [(0, 1e-12), (1, 1e-5)])
def test_forward_matches_oracle(precision, rtol):
    import paper_1907_02814_amd as cmc
    from gpu_parity import gpu_tables
    y = _inputs()
    g = _dev(y)
    Y, yp = cmc.expected_yield(gpu_tables(29), g["Zstar"], g["n_e"], g["T_e"], g["off"], g["px"],
                               g["py"], g["pz"], g["w"], y["dt"], precision, per_particle=True)
    Yo, ypo = O.expected_yield(O.tables(29), y["Zstar"], y["n_e"], y["T_e"], y["off"], y["px"], y["py"],
                               y["pz"], y["w"], y["dt"], per_particle=True)
    np.testing.assert_allclose(Y.cpu().numpy(), Yo, rtol=rtol, atol=0)
    np.testing.assert_allclose(yp.cpu().numpy(), ypo, rtol=rtol, atol=1e-300)


@pytest.mark.parametrize("precision,rtol", [(0, 1e-11), (1, 2e-5)])
def test_backward_matches_oracle(precision, rtol):
    import paper_1907_02814_amd as cmc
    from gpu_parity import gpu_tables
    y = _inputs()
    g = _dev(y)
    gY = np.linspace(0.5, 2.0, len(y["Zstar"]))
    G = cmc.expected_yield_backward(gpu_tables(29), g["Zstar"], g["n_e"], g["T_e"], g["off"], g["px"],
                                    g["py"], g["pz"], g["w"], y["dt"], _dev({"a": gY})["a"], precision)
    Go = O.expected_yield_backward(O.tables(29), y["Zstar"], y["n_e"], y["T_e"], y["off"], y["px"],
                                   y["py"], y["pz"], y["w"], y["dt"], gY)
    for k in ("gZstar", "gn_e", "gT_e", "gw"):
        a, b = G[k].cpu().numpy(), Go[k]
        assert np.all(np.abs(a - b) <= rtol * np.abs(b) + 1e-300 + 1e-12 * rtol * np.abs(b).max()), k
    # momenta: per-electron vector agreement
    a = np.stack([G[k].cpu().numpy() for k in ("gpx", "gpy", "gpz")])
    b = np.stack([Go[k] for k in ("gpx", "gpy", "gpz")])
    err = np.sqrt(((a - b) ** 2).sum(0)); mag = np.sqrt((b ** 2).sum(0))
    assert np.all(err <= rtol * mag + 1e-300)


def test_autograd_function_against_finite_differences():
    import torch
    import paper_1907_02814_amd as cmc
    from gpu_parity import gpu_tables
    y = _inputs(n_cells=6, per_cell=64, seed=3)
    g = _dev(y)
    tab = gpu_tables(29)
    leaves = {k: g[k].clone().requires_grad_(True) for k in ("px", "py", "pz", "w", "Zstar", "n_e", "T_e")}
    Y = cmc.ExpectedYield.apply(leaves["px"], leaves["py"], leaves["pz"], leaves["w"], leaves["Zstar"],
                                leaves["n_e"], leaves["T_e"], g["off"], tab, y["dt"])
    wts = torch.linspace(1.0, 2.0, Y.numel(), dtype=torch.float64, device="cuda")
    (Y * wts).sum().backward()

    def f(**over):
        a = {k: over.get(k, g[k]) for k in ("px", "py", "pz", "w", "Zstar", "n_e", "T_e")}
        return cmc.expected_yield(tab, a["Zstar"], a["n_e"], a["T_e"], g["off"], a["px"], a["py"],
                                  a["pz"], a["w"], y["dt"])

    h = 1e-5
    for k in ("Zstar", "n_e", "T_e"):
        for c in range(Y.numel()):
            d = h * abs(float(g[k][c]))
            up = g[k].clone(); up[c] += d
            dn = g[k].clone(); dn[c] -= d
            fd = float(wts[c] * (f(**{k: up})[c] - f(**{k: dn})[c]) / (2 * d))
            an = float(leaves[k].grad[c])
            assert abs(fd - an) <= 2e-6 * max(abs(fd), abs(an)) + 1e-300, (k, c, fd, an)
    rng = np.random.default_rng(0)
    for _ in range(3):
        v = {k: torch.from_numpy(rng.normal(size=g["px"].numel())).cuda() for k in ("px", "py", "pz")}
        fp = (wts * f(**{k: g[k] + h * v[k] for k in v})).sum()
        fm = (wts * f(**{k: g[k] - h * v[k] for k in v})).sum()
        fd = float((fp - fm) / (2 * h))
        an = float(sum((leaves[k].grad * v[k]).sum() for k in v))
        assert abs(fd - an) <= 2e-6 * abs(an)


def _dense_inputs():
    """Cells so dense that L_D is clamped to r_i near the foot of the L axis
    (Z* close to Z = 29, n_e ~ 1e35 m^-3): I_TFD falls below 1.93, where the
    principal Lambert W branch of eq:lambert-W starts from log1p instead of
    its series about 0.  L_R = 10.5, 10.7 (inside the axis), 8.4 (below it,
    clamped) and 11.5 (I_TFD = 1.95, the series start) beside ordinary cells."""
    y = _inputs(n_cells=8, per_cell=300, seed=13)
    y["Zstar"][:4] = [29.0, 28.5, 29.0, 29.0]
    y["n_e"][:4] = [1.04e35, 1.0e35, 2.0e35, 8.0e34]
    y["T_e"][:4] = 10.0
    return y


def test_dense_cells_reach_the_general_lambert_start():
    # the premise, from the oracle: which start each dense cell takes
    y = _dense_inputs()
    a = np.array([O.screening(29, y["Zstar"][c], y["n_e"][c] / y["Zstar"][c], y["T_e"][c])["a"]
                  for c in range(4)])
    z = np.exp(-(1.0 + 2.0 * a))
    assert np.all(z[:3] > 2.0 ** -7) and z[3] <= 2.0 ** -7


@pytest.mark.parametrize("precision,rtol,rtol_g", [(0, 1e-12, 1e-11), (1, 1e-5, 2e-5)])
def test_dense_cells_against_the_oracle(precision, rtol, rtol_g):
    import paper_1907_02814_amd as cmc
    from gpu_parity import gpu_tables
    y = _dense_inputs()
    g = _dev(y)
    args = (g["Zstar"], g["n_e"], g["T_e"], g["off"], g["px"], g["py"], g["pz"], g["w"], y["dt"])
    oargs = (y["Zstar"], y["n_e"], y["T_e"], y["off"], y["px"], y["py"], y["pz"], y["w"], y["dt"])
    Y = cmc.expected_yield(gpu_tables(29), *args, precision)
    Yo = O.expected_yield(O.tables(29), *oargs)
    assert np.all(Yo[:4] > 0.0)
    np.testing.assert_allclose(Y.cpu().numpy(), Yo, rtol=rtol, atol=0)
    gY = np.linspace(0.5, 2.0, len(y["Zstar"]))
    G = cmc.expected_yield_backward(gpu_tables(29), *args, _dev({"a": gY})["a"], precision)
    Go = O.expected_yield_backward(O.tables(29), *oargs, gY)
    for k in ("gZstar", "gn_e", "gT_e", "gw"):
        a, b = G[k].cpu().numpy(), Go[k]
        assert np.all(np.abs(a - b) <= rtol_g * np.abs(b) + 1e-300 + 1e-12 * rtol_g * np.abs(b).max()), k
    a = np.stack([G[k].cpu().numpy() for k in ("gpx", "gpy", "gpz")])
    b = np.stack([Go[k] for k in ("gpx", "gpy", "gpz")])
    err = np.sqrt(((a - b) ** 2).sum(0)); mag = np.sqrt((b ** 2).sum(0))
    assert np.all(err <= rtol_g * mag + 1e-300)


def _ragged_inputs():
    """Cells of 0, 1 and team-boundary sizes (the forward runs 256 threads
    per cell, the adjoint 192), and one larger cell."""
    counts = np.array([0, 1, 63, 64, 65, 191, 192, 193, 0, 255, 256, 257, 384, 1000, 2])
    y = W.cfg4(np.random.default_rng(14), n_cells=len(counts), per_cell=int(counts.max()))
    n = int(counts.sum())
    off = np.zeros(len(counts) + 1, np.int64)
    off[1:] = np.cumsum(counts)
    for k in ("px", "py", "pz", "w"):
        y[k] = np.ascontiguousarray(y[k][:n])
    y["w"] = np.random.default_rng(15).lognormal(0.0, 0.5, n)
    y["off"] = off
    return y


@pytest.mark.parametrize("precision,rtol,rtol_g", [(0, 1e-12, 1e-11), (1, 1e-5, 2e-5)])
def test_ragged_and_empty_cells_against_the_oracle(precision, rtol, rtol_g):
    import paper_1907_02814_amd as cmc
    from gpu_parity import gpu_tables
    y = _ragged_inputs()
    g = _dev(y)
    args = (g["Zstar"], g["n_e"], g["T_e"], g["off"], g["px"], g["py"], g["pz"], g["w"], y["dt"])
    oargs = (y["Zstar"], y["n_e"], y["T_e"], y["off"], y["px"], y["py"], y["pz"], y["w"], y["dt"])
    Y, yp = cmc.expected_yield(gpu_tables(29), *args, precision, per_particle=True)
    Yo, ypo = O.expected_yield(O.tables(29), *oargs, per_particle=True)
    empty = np.diff(y["off"]) == 0
    assert np.all(Y.cpu().numpy()[empty] == 0.0)
    np.testing.assert_allclose(Y.cpu().numpy(), Yo, rtol=rtol, atol=0)
    np.testing.assert_allclose(yp.cpu().numpy(), ypo, rtol=rtol, atol=1e-300)
    gY = np.linspace(0.5, 2.0, len(y["Zstar"]))
    G = cmc.expected_yield_backward(gpu_tables(29), *args, _dev({"a": gY})["a"], precision)
    Go = O.expected_yield_backward(O.tables(29), *oargs, gY)
    for k in ("gZstar", "gn_e", "gT_e"):
        assert np.all(G[k].cpu().numpy()[empty] == 0.0), k
    for k in ("gZstar", "gn_e", "gT_e", "gw"):
        a, b = G[k].cpu().numpy(), Go[k]
        assert np.all(np.abs(a - b) <= rtol_g * np.abs(b) + 1e-300 + 1e-12 * rtol_g * np.abs(b).max()), k
    a = np.stack([G[k].cpu().numpy() for k in ("gpx", "gpy", "gpz")])
    b = np.stack([Go[k] for k in ("gpx", "gpy", "gpz")])
    err = np.sqrt(((a - b) ** 2).sum(0)); mag = np.sqrt((b ** 2).sum(0))
    assert np.all(err <= rtol_g * mag + 1e-300)


def test_zero_cells_is_a_no_op():
    import torch
    import paper_1907_02814_amd as cmc
    from gpu_parity import gpu_tables
    z = torch.zeros(0, dtype=torch.float64, device="cuda")
    off = torch.zeros(1, dtype=torch.int64, device="cuda")
    for p in (cmc.FP64, cmc.FP32):
        Y = cmc.expected_yield(gpu_tables(29), z, z, z, off, z, z, z, z, 1e-16, p)
        G = cmc.expected_yield_backward(gpu_tables(29), z, z, z, off, z, z, z, z, 1e-16, z, p)
        torch.cuda.synchronize()
        assert Y.numel() == 0 and all(v.numel() == 0 for v in G.values())
