"""Pins of the oracle's expected-yield pass and of its analytic adjoint:
single-electron hand value from the tables, central finite differences,
and the synthetic Maxwell-Juttner generator."""
import math

import numpy as np
import pytest
from scipy import special

from oracle import oracle as O
from paper_1907_02814_amd import workloads as W

C = 299792458.0


def _one_cell(n, seed, gmin=1.5, gmax=1000.0):
    rng = np.random.default_rng(seed)
    g = np.exp(rng.uniform(math.log(gmin), math.log(gmax), n))
    px, py, pz = W.momenta_from_gamma(rng, g)
    return g, px, py, pz, rng.uniform(0.5, 2.0, n)


def test_single_electron_hand_value():
    # y = w (1 - exp(-n_i sigma_B beta c dt)) sigma_k/sigma_B, n_i = n_e/Z*
    tab = O.tables(29)
    Zs, ne, Te, dt = 7.0, 3e28, 500.0, 1e-16
    for g in (1.2, 3.0, 55.0, 900.0):
        p = math.sqrt(g * g - 1)
        sig, sk, seg, _ = tab.lookup(Zs, ne / Zs, Te, g, O.BREMS)
        y_hand = 1.7 * (-math.expm1(-(ne / Zs) * sig * (p / g) * C * dt)) * sk / sig
        Y = O.expected_yield(tab, [Zs], [ne], [Te], np.array([0, 1]), [p * 0.6], [0.0], [p * 0.8],
                             [1.7], dt)
        assert abs(Y[0] / y_hand - 1) < 1e-14


def test_below_cut_gives_zero():
    tab = O.tables(29)
    g = 1.0 + 500.0 / 510998.95    # 500 eV < 1 keV
    p = math.sqrt(g * g - 1)
    Y = O.expected_yield(tab, [5.0], [1e28], [100.0], np.array([0, 1]), [p], [0.0], [0.0], [1.0], 1e-16)
    assert Y[0] == 0.0


def _fd_check(tab, Zs, ne, Te, off, px, py, pz, w, dt, gY, h=1e-5):
    G = O.expected_yield_backward(tab, Zs, ne, Te, off, px, py, pz, w, dt, gY)
    L = lambda *a: float(np.dot(gY, O.expected_yield(tab, *a)))
    args = [np.array(Zs, float), np.array(ne, float), np.array(Te, float)]
    out = []
    for q, name in enumerate(("gZstar", "gn_e", "gT_e")):
        for c in range(len(Zs)):
            a1 = [x.copy() for x in args]; a2 = [x.copy() for x in args]
            d = h * abs(args[q][c]); a1[q][c] += d; a2[q][c] -= d
            # difference of this cell's own yield (cells are independent)
            y1 = O.expected_yield(tab, *a1, off, px, py, pz, w, dt)[c]
            y2 = O.expected_yield(tab, *a2, off, px, py, pz, w, dt)[c]
            out.append((name, c, gY[c] * (y1 - y2) / (2 * d), G[name][c]))
    # directional derivative in momentum space
    rng = np.random.default_rng(0)
    for _ in range(3):
        v = [rng.normal(size=len(px)) for _ in range(3)]
        eps = h
        fp = L(*args, off, px + eps * v[0], py + eps * v[1], pz + eps * v[2], w, dt)
        fm = L(*args, off, px - eps * v[0], py - eps * v[1], pz - eps * v[2], w, dt)
        fd = (fp - fm) / (2 * eps)
        an = sum(np.dot(G[k], vv) for k, vv in zip(("gpx", "gpy", "gpz"), v))
        out.append(("dir", -1, fd, an))
    return out


def test_gradient_matches_central_differences():
    tab = O.tables(29)
    n, m = 4, 24
    g, px, py, pz, w = _one_cell(n * m, 5, gmin=2.05, gmax=1000.0)
    off = np.arange(0, (n + 1) * m, m, dtype=np.int64)
    Zs = [3.0, 10.0, 25.0, 1.5]
    ne = [1e28, 3e29, 1e27, 8e29]
    Te = [50.0, 2000.0, 8000.0, 15.0]
    res = _fd_check(tab, Zs, ne, Te, off, px, py, pz, w, 1e-16, np.array([1.0, 2.0, 0.5, 1.3]))
    for name, c, fd, an in res:
        scale = max(abs(fd), abs(an))
        if scale == 0.0:
            continue
        assert abs(fd - an) <= 2e-6 * scale, (name, c, fd, an)


def test_gradient_nonrelativistic_electrons():
    tab = O.tables(29)
    g, px, py, pz, w = _one_cell(16, 7, gmin=1.01, gmax=1.95)
    off = np.array([0, 16], dtype=np.int64)
    res = _fd_check(tab, [6.0], [2e28], [300.0], off, px, py, pz, w, 1e-16, np.array([1.0]))
    for name, c, fd, an in res:
        scale = max(abs(fd), abs(an))
        if scale == 0.0:
            continue
        assert abs(fd - an) <= 2e-6 * scale, (name, c, fd, an)


def test_gradient_is_linear_in_upstream():
    tab = O.tables(29)
    g, px, py, pz, w = _one_cell(20, 3)
    off = np.array([0, 10, 20], dtype=np.int64)
    a = O.expected_yield_backward(tab, [4.0, 9.0], [1e28, 1e29], [40.0, 900.0], off, px, py, pz, w,
                                  1e-16, np.array([1.0, 1.0]))
    b = O.expected_yield_backward(tab, [4.0, 9.0], [1e28, 1e29], [40.0, 900.0], off, px, py, pz, w,
                                  1e-16, np.array([3.0, 0.0]))
    np.testing.assert_allclose(b["gpx"][:10], 3 * a["gpx"][:10], rtol=1e-15)
    assert np.all(b["gpx"][10:] == 0)
    Y = O.expected_yield(tab, [4.0, 9.0], [1e28, 1e29], [40.0, 900.0], off, px, py, pz, w, 1e-16)
    # Y is linear in the weights: dY/dw = y/w
    _, yp = O.expected_yield(tab, [4.0, 9.0], [1e28, 1e29], [40.0, 900.0], off, px, py, pz, w, 1e-16,
                             per_particle=True)
    np.testing.assert_allclose(a["gw"], yp / w, rtol=1e-14)
    np.testing.assert_allclose([yp[:10].sum(), yp[10:].sum()], Y, rtol=1e-14)


def test_maxwell_juttner_generator_mean():
    # <gamma> = 3 theta + K1(1/theta)/K2(1/theta) for the isotropic
    # relativistic Maxwellian of eq:mj; <T> ~ 3 theta for theta >> 1 (Sec. IV)
    rng = np.random.default_rng(1)
    for theta in (W.MJ_THETA, 0.5):
        g = W.maxwell_juttner_gamma(rng, 400000, theta)
        exact = 3 * theta + special.kv(1, 1 / theta) / special.kv(2, 1 / theta)
        assert abs(g.mean() / exact - 1) < 4e-3
    assert abs(W.MJ_THETA - 9.7848) < 1e-3
