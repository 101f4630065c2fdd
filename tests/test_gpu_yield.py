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


def check_adjoint(G, Go, rtol, label=""):
    """GPU adjoint G against the oracle's Go (computed with scale=True), to
    rtol: per electron, the momentum gradient as a vector (relative to its
    length) and dL/dw; per cell, dL/dZ*, dL/dn_e and dL/dT_e relative to
    the larger of their size and the sum of the sizes of the terms they are
    summed from (the kernel applies the cell's Jacobian once to summed
    coefficients, the oracle per electron: the two orders round apart by a
    few ulps of that sum where the terms cancel).  Returns the largest
    errors seen."""
    out = {}
    a = np.stack([G[k].cpu().numpy() for k in ("gpx", "gpy", "gpz")])
    b = np.stack([Go[k] for k in ("gpx", "gpy", "gpz")])
    err = np.sqrt(((a - b) ** 2).sum(0))
    mag = np.sqrt((b ** 2).sum(0))
    rel = np.where(err == 0, 0.0, err / np.maximum(mag, 1e-300))
    out["p"] = float(rel.max()) if rel.size else 0.0
    ga, gb = G["gw"].cpu().numpy(), Go["gw"]
    rw = np.where(ga == gb, 0.0, np.abs(ga - gb) / np.maximum(np.abs(gb), 1e-300))
    out["w"] = float(rw.max()) if rw.size else 0.0
    for q, k in enumerate(("gZstar", "gn_e", "gT_e")):
        x, y = G[k].cpu().numpy(), Go[k]
        sc = np.maximum(np.abs(y), Go["gabs"][:, q])
        r = np.where(x == y, 0.0, np.abs(x - y) / np.maximum(sc, 1e-300))
        out[k] = float(r.max()) if r.size else 0.0
    print(f"[parity] adjoint {label}: " + ", ".join(f"{k} {v:.1e}" for k, v in out.items()))
    for k, v in out.items():
        assert v <= rtol, (label, k, v, rtol)
    return out


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


@pytest.mark.parametrize("precision,rtol", [(0, 1e-12), (1, 1e-5)])
def test_backward_matches_oracle(precision, rtol):
    import paper_1907_02814_amd as cmc
    from gpu_parity import gpu_tables
    y = _inputs()
    g = _dev(y)
    gY = np.linspace(0.5, 2.0, len(y["Zstar"]))
    G = cmc.expected_yield_backward(gpu_tables(29), g["Zstar"], g["n_e"], g["T_e"], g["off"], g["px"],
                                    g["py"], g["pz"], g["w"], y["dt"], _dev({"a": gY})["a"], precision)
    Go = O.expected_yield_backward(O.tables(29), y["Zstar"], y["n_e"], y["T_e"], y["off"], y["px"],
                                   y["py"], y["pz"], y["w"], y["dt"], gY, scale=True)
    check_adjoint(G, Go, rtol, f"small, precision {precision}")


@pytest.mark.parametrize("precision", [0, 1])
def test_backward_without_the_weight_gradient(precision):
    """The adjoint asked for no gradient with respect to the weights (gw
    NULL, as timed in the benchmark) gives the other gradients bit for bit."""
    import torch
    import paper_1907_02814_amd as cmc
    from gpu_parity import gpu_tables
    y = _inputs()
    g = _dev(y)
    gY = _dev({"a": np.linspace(0.5, 2.0, len(y["Zstar"]))})["a"]
    args = (gpu_tables(29), g["Zstar"], g["n_e"], g["T_e"], g["off"], g["px"], g["py"], g["pz"], g["w"], y["dt"], gY)
    A = cmc.expected_yield_backward(*args, precision)
    B = cmc.expected_yield_backward(*args, precision, weight_grad=False)
    torch.cuda.synchronize()
    assert "gw" in A and "gw" not in B
    for k in B:
        assert torch.equal(A[k], B[k]), k


def _fd_inputs():
    """Cells of cfg4's distributions whose screening takes both Debye
    branches (L_D from the temperature, and L_D clamped to r_i), with a few
    non-relativistic electrons."""
    y = _inputs(n_cells=24, per_cell=48, seed=21)
    br = np.array([O.screening(29, y["Zstar"][c], y["n_e"][c] / y["Zstar"][c], y["T_e"][c])["branch"]
                   for c in range(24)])
    assert (br == 1).any() and (br == 2).any(), br
    return y


def test_autograd_function_against_finite_differences():
    """Central differences with h = 1e-6 relative (FP64 form): each cell
    parameter of each cell, and each momentum component of every electron
    (one batched forward per axis and sign, per-electron terms).  A point
    whose two one-sided differences disagree has a kink of the interpolant
    (a table knot, the Debye clamp, a segment join) within h: it is
    excluded and counted."""
    import torch
    import paper_1907_02814_amd as cmc
    from gpu_parity import gpu_tables
    y = _fd_inputs()
    g = _dev(y)
    tab = gpu_tables(29)
    leaves = {k: g[k].clone().requires_grad_(True) for k in ("px", "py", "pz", "w", "Zstar", "n_e", "T_e")}
    Y = cmc.ExpectedYield.apply(leaves["px"], leaves["py"], leaves["pz"], leaves["w"], leaves["Zstar"],
                                leaves["n_e"], leaves["T_e"], g["off"], tab, y["dt"])
    wts = torch.linspace(1.0, 2.0, Y.numel(), dtype=torch.float64, device="cuda")
    (Y * wts).sum().backward()

    def f(per=False, **over):
        a = {k: over.get(k, g[k]) for k in ("px", "py", "pz", "w", "Zstar", "n_e", "T_e")}
        return cmc.expected_yield(tab, a["Zstar"], a["n_e"], a["T_e"], g["off"], a["px"], a["py"],
                                  a["pz"], a["w"], y["dt"], per_particle=per)

    h = 1e-6
    tol = 1e-7
    Y0 = f()
    kinks = 0
    checked = 0
    for k in ("Zstar", "n_e", "T_e"):
        for c in range(Y.numel()):
            d = h * abs(float(g[k][c]))
            up = g[k].clone(); up[c] += d
            dn = g[k].clone(); dn[c] -= d
            yu, yd, y0 = float(f(**{k: up})[c]), float(f(**{k: dn})[c]), float(Y0[c])
            fd = float(wts[c]) * (yu - yd) / (2 * d)
            fwd, bwd = float(wts[c]) * (yu - y0) / d, float(wts[c]) * (y0 - yd) / d
            if abs(fwd - bwd) > 1e-4 * max(abs(fd), 1e-300):
                kinks += 1
                continue
            an = float(leaves[k].grad[c])
            checked += 1
            assert abs(fd - an) <= tol * max(abs(fd), abs(an)) + 1e-300, (k, c, fd, an)
    # momenta: per electron and axis, from per-electron terms
    cell = np.repeat(np.arange(Y.numel()), np.diff(y["off"]))
    wpe = wts.cpu().numpy()[cell]
    _, yp0 = f(per=True)
    yp0 = yp0.cpu().numpy()
    pmag = np.sqrt(y["px"] ** 2 + y["py"] ** 2 + y["pz"] ** 2)
    for k in ("px", "py", "pz"):
        d = h * pmag
        dt_ = torch.from_numpy(d).cuda()
        _, yu = f(per=True, **{k: g[k] + dt_})
        _, yd = f(per=True, **{k: g[k] - dt_})
        yu, yd = yu.cpu().numpy(), yd.cpu().numpy()
        fd = wpe * (yu - yd) / (2 * d)
        fwd, bwd = wpe * (yu - yp0) / d, wpe * (yp0 - yd) / d
        an = leaves[k].grad.cpu().numpy()
        # each component is judged against the length of the electron's
        # gradient (a component much smaller than that is mostly roundoff of
        # the differences)
        gnorm = np.sqrt(sum(leaves[q].grad.cpu().numpy() ** 2 for q in ("px", "py", "pz")))
        kink = np.abs(fwd - bwd) > 1e-4 * np.maximum(gnorm, 1e-300)
        sel = ~kink & (gnorm > 0)
        kinks += int((kink & (gnorm > 0)).sum())
        checked += int(sel.sum())
        err = np.abs(fd - an) / np.maximum(gnorm, 1e-300)
        assert np.all(err[sel] <= tol), (k, float(err[sel].max()))
    print(f"[parity] finite differences h=1e-6: {checked} checked, {kinks} kink(s) within h excluded")
    assert kinks <= 0.01 * checked


def test_fp32_adjoint_finite_differences_of_its_forward():
    """The FP32 form's adjoint against central differences of the FP64
    forward (h = 1e-6 relative, per electron): within the FP32 form's
    1e-5, away from kinks (excluded and counted as above)."""
    import torch
    import paper_1907_02814_amd as cmc
    from gpu_parity import gpu_tables
    y = _fd_inputs()
    g = _dev(y)
    tab = gpu_tables(29)
    ones = torch.ones(len(y["Zstar"]), dtype=torch.float64, device="cuda")
    G = cmc.expected_yield_backward(tab, g["Zstar"], g["n_e"], g["T_e"], g["off"], g["px"], g["py"], g["pz"],
                                    g["w"], y["dt"], ones, cmc.FP32)

    def f(**over):
        a = {k: over.get(k, g[k]) for k in ("px", "py", "pz")}
        return cmc.expected_yield(tab, g["Zstar"], g["n_e"], g["T_e"], g["off"], a["px"], a["py"], a["pz"],
                                  g["w"], y["dt"], per_particle=True)[1].cpu().numpy()

    h = 1e-6
    y0 = f()
    pmag = np.sqrt(y["px"] ** 2 + y["py"] ** 2 + y["pz"] ** 2)
    kinks = checked = 0
    gn = np.sqrt(sum(G["g" + q].cpu().numpy() ** 2 for q in ("px", "py", "pz")))
    for k in ("px", "py", "pz"):
        dt_ = torch.from_numpy(h * pmag).cuda()
        yu, yd = f(**{k: g[k] + dt_}), f(**{k: g[k] - dt_})
        d = h * pmag
        fd = (yu - yd) / (2 * d)
        kink = np.abs((yu - y0) / d - (y0 - yd) / d) > 1e-4 * np.maximum(gn, 1e-300)
        an = G["g" + k].cpu().numpy()
        sel = ~kink & (gn > 0)
        kinks += int(kink.sum())
        checked += int(sel.sum())
        err = np.abs(fd - an) / np.maximum(gn, 1e-300)
        assert np.all(err[sel] <= 1e-5), (k, float(err[sel].max()))
    print(f"[parity] FP32 adjoint vs finite differences: {checked} checked, {kinks} kink(s) excluded")


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


@pytest.mark.parametrize("precision,rtol", [(0, 1e-12), (1, 1e-5)])
def test_dense_cells_against_the_oracle(precision, rtol):
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
    Go = O.expected_yield_backward(O.tables(29), *oargs, gY, scale=True)
    check_adjoint(G, Go, rtol, f"dense cells, precision {precision}")


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


@pytest.mark.parametrize("precision,rtol", [(0, 1e-12), (1, 1e-5)])
def test_ragged_and_empty_cells_against_the_oracle(precision, rtol):
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
    Go = O.expected_yield_backward(O.tables(29), *oargs, gY, scale=True)
    for k in ("gZstar", "gn_e", "gT_e"):
        assert np.all(G[k].cpu().numpy()[empty] == 0.0), k
    check_adjoint(G, Go, rtol, f"ragged cells, precision {precision}")


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


def test_bad_cells_and_offsets_are_flagged_on_the_device():
    """Cells the screening model does not cover (Z* <= 0 or > Z, n_e <= 0,
    a non-finite or negative T_e) get Y = 0 and zero terms and gradients
    (CMC_ST_BAD_CELL); offsets that decrease or pass n_part skip the cell
    (CMC_ST_BAD_OFFSETS).  The C ABI is called directly, past the binding's
    own check of the offsets.  The good cells keep the oracle's values."""
    import ctypes as C
    import torch
    import paper_1907_02814_amd as cmc
    from gpu_parity import gpu_tables
    y = _inputs(n_cells=8, per_cell=64, seed=31)
    y["Zstar"][1] = 0.0
    y["Zstar"][2] = 30.0
    y["n_e"][3] = -1.0
    y["T_e"][4] = float("nan")
    g = _dev(y)
    st = torch.zeros(1, dtype=torch.int32, device="cuda")
    Y, yp = cmc.expected_yield(gpu_tables(29), g["Zstar"], g["n_e"], g["T_e"], g["off"], g["px"], g["py"],
                               g["pz"], g["w"], y["dt"], per_particle=True, status=st)
    gY = torch.ones(8, dtype=torch.float64, device="cuda")
    st2 = torch.zeros(1, dtype=torch.int32, device="cuda")
    G = cmc.expected_yield_backward(gpu_tables(29), g["Zstar"], g["n_e"], g["T_e"], g["off"], g["px"],
                                    g["py"], g["pz"], g["w"], y["dt"], gY, status=st2)
    torch.cuda.synchronize()
    assert int(st.item()) == cmc.ST_BAD_CELL and int(st2.item()) == cmc.ST_BAD_CELL
    Y, yp = Y.cpu().numpy(), yp.cpu().numpy()
    bad = [1, 2, 3, 4]
    off = y["off"]
    for c in bad:
        assert Y[c] == 0.0 and np.all(yp[off[c]:off[c + 1]] == 0.0)
        for k in ("gpx", "gpy", "gpz", "gw"):
            assert np.all(G[k].cpu().numpy()[off[c]:off[c + 1]] == 0.0)
        for k in ("gZstar", "gn_e", "gT_e"):
            assert G[k].cpu().numpy()[c] == 0.0
    good = [0, 5, 6, 7]
    Yo = O.expected_yield(O.tables(29), y["Zstar"][good], y["n_e"][good], y["T_e"][good],
                          np.concatenate([[0], np.cumsum(np.diff(off)[good])]),
                          *[np.concatenate([y[k][off[c]:off[c + 1]] for c in good]) for k in ("px", "py", "pz", "w")],
                          y["dt"])
    np.testing.assert_allclose(Y[good], Yo, rtol=1e-12, atol=0)
    # offsets: decreasing in cell 2, beyond n_part in cell 5 (raw C ABI)
    bad_off = torch.tensor([0, 64, 128, 100, 192, 256, 9999, 448, 512], dtype=torch.int64, device="cuda")
    Yb = torch.full((8,), -1.0, dtype=torch.float64, device="cuda")
    st3 = torch.zeros(1, dtype=torch.int32, device="cuda")
    L = cmc.get_lib()
    p = lambda t: C.c_void_p(t.data_ptr())
    rc = L.cmc_expected_yield(gpu_tables(29).handle, 8, p(g["Zstar"]), p(g["n_e"]), p(g["T_e"]), p(bad_off),
                              512, p(g["px"]), p(g["py"]), p(g["pz"]), p(g["w"]), y["dt"], 0, p(Yb), None,
                              p(st3), C.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert rc == 0
    torch.cuda.synchronize()
    assert int(st3.item()) & cmc.ST_BAD_OFFSETS
    Yb = Yb.cpu().numpy()
    # cell 2 (128 -> 100) and cells 5, 6 (past 512) are skipped with Y = 0
    assert Yb[2] == 0.0 and Yb[5] == 0.0 and Yb[6] == 0.0
