"""Pins of the oracle's tables: node values against independent quadrature
(different integration variables, panels and rule), CDF properties, the
photon-energy cut of Sec. III.A, and inverse-CDF sampling against the
exact spectrum."""
import math

import numpy as np
import pytest

from oracle import oracle as O

Z = 29
NL = 81
LNL = (math.log(10.0), math.log(1e6))
MEC2EV = 510998.95
GX, GW = np.polynomial.legendre.leggauss(24)


def node(a, b, n, i):
    return a + i * ((b - a) / (n - 1))


def Lnode(l):
    return math.exp(node(LNL[0], LNL[1], NL, l))


def gl_panels(f, edges):
    s = 0.0
    for lo, hi in zip(edges[:-1], edges[1:]):
        t = 0.5 * (hi - lo) * GX + 0.5 * (hi + lo)
        s += 0.5 * (hi - lo) * sum(w * f(x) for w, x in zip(GW, t))
    return s


def brems_sigma_ref(g1, L, coulomb, moment=0, nr=None):
    """sigma = int dsigma/dk dk over (1e-7 (g1-1), g1-1): ln k on the lower
    half, ln g2 on the upper half (reference, independent of the table rule)."""
    T = g1 - 1.0
    klo = 1e-7 * T
    if nr is None:
        f = lambda k: O.dsdk_rel(Z, g1, k, L, coulomb) * k ** moment
    else:
        etd, Ltf, Ld = nr
        f = lambda k: O.dsdk_nr(Z, g1, k, etd, Ltf, Ld, True) * k ** moment
    lo = gl_panels(lambda v: math.exp(v) * f(math.exp(v)),
                   np.linspace(math.log(klo), math.log(0.5 * T), 121))
    if nr is None:
        hi = gl_panels(lambda v: math.exp(v) * f(g1 - math.exp(v)),
                       np.linspace(0.0, math.log(g1 - 0.5 * T), 61))
    else:
        # square-root tip of the non-relativistic spectrum: integrate in p2
        p2max = math.sqrt((g1 - 0.5 * T) ** 2 - 1.0)
        p1 = math.sqrt(T * (g1 + 1.0))

        def fp(p2):
            # eq:cs_br_nr with the Elwert factor, written in p2 so that the
            # spectrum tip keeps its digits
            g2 = math.sqrt(1.0 + p2 * p2)
            k = (p1 * p1 - p2 * p2) / (g1 + g2)
            dpp, dpm = p1 + p2, k * (g1 + g2) / (p1 + p2)

            def g(eta, LL):
                A = dpp * dpp * LL * LL + 1; B = dpm * dpm * LL * LL + 1
                return 0.5 * eta * eta * (math.log(A / B) + 1 / A - 1 / B)
            etf = 1 - etd
            br = g(etf, Ltf)
            if etd > 0:
                A2, B2 = Ltf * Ltf, Ld * Ld
                br += g(etd, Ld) + etf * etd / (B2 - A2) * (
                    A2 * math.log((dpm * dpm * B2 + 1) / (dpp * dpp * B2 + 1))
                    + B2 * math.log((dpp * dpp * A2 + 1) / (dpm * dpm * A2 + 1)))
            b1, b2, c = p1 / g1, p2 / g2, 2 * math.pi * Z / 137.035999084
            fe = b1 / b2 * (1 - math.exp(-c / b1)) / (1 - math.exp(-c / b2))
            ds = 16 * (2.8179403262e-15) ** 2 * Z * Z / 137.035999084 / (3 * k * p1 * p1) * br * fe
            return ds * k ** moment * p2 / g2
        edges = np.concatenate([[0.0], p2max * np.geomspace(1e-4, 1.0, 60)])
        hi = gl_panels(fp, edges)
    return lo + hi


@pytest.fixture(scope="module")
def tab():
    return O.tables(Z)


@pytest.mark.parametrize("i,l", [(0, 0), (10, 30), (30, 50), (55, 80), (20, 7)])
def test_brems_relativistic_nodes(tab, i, l):
    g = math.exp(node(math.log(2), math.log(100), 56, i))
    L = Lnode(l)
    s = tab.export("sigR").reshape(56, NL)[i, l]
    k = tab.export("skR").reshape(56, NL)[i, l]
    assert abs(s / brems_sigma_ref(g, L, False) - 1) < 1e-13
    assert abs(k / brems_sigma_ref(g, L, False, 1) - 1) < 1e-13


@pytest.mark.parametrize("i,l", [(0, 10), (40, 40), (74, 80)])
def test_brems_ultrarelativistic_nodes(tab, i, l):
    g = math.exp(node(math.log(100), math.log(2e4), 75, i))
    L = Lnode(l)
    s = tab.export("sigU").reshape(75, NL)[i, l]
    assert abs(s / brems_sigma_ref(g, L, True) - 1) < 1e-13


@pytest.mark.parametrize("i,e,l", [(0, 0, 0), (10, 8, 40), (22, 16, 80), (15, 3, 20)])
def test_brems_nonrelativistic_nodes(tab, i, e, l):
    g1m1 = math.exp(node(math.log(1000.0 / MEC2EV), 0.0, 23, i))
    g = 1.0 + g1m1
    etd = e / 16.0
    Ltf = 1.0 / (Z ** (1.0 / 3.0) / 137.035999084)
    Ld = Lnode(l)
    s = tab.export("sigN").reshape(23, 17, NL)[i, e, l]
    k = tab.export("skN").reshape(23, 17, NL)[i, e, l]
    ref = brems_sigma_ref(g, None, False, 0, nr=(etd, Ltf, Ld))
    refk = brems_sigma_ref(g, None, False, 1, nr=(etd, Ltf, Ld))
    assert abs(s / ref - 1) < 1e-13
    assert abs(k / refk - 1) < 1e-13


@pytest.mark.parametrize("i,l", [(0, 0), (50, 20), (120, 60), (165, 80), (90, 5)])
def test_bethe_heitler_nodes(tab, i, l):
    k = 2.0 + math.exp(node(math.log(1e-6), math.log(2e4 - 2), 166, i))
    L = Lnode(l)
    s = tab.export("sigB").reshape(166, NL)[i, l]
    # full range [1, k-1] in ln(g+ - 1 + h) panels, no symmetry used
    f = lambda gp: O.dsdgp_bh(Z, k, gp, L)
    if k - 2 < 1e-3:
        ref = gl_panels(f, np.linspace(1.0, k - 1.0, 9))
    else:
        h = 1e-3 * (k - 2)
        e = np.concatenate([1.0 + np.geomspace(h, 0.5 * (k - 2), 80) - h, [0]])[:-1]
        edges = np.concatenate([[1.0], e[1:], (k - e[::-1])[1:], [k - 1.0]])
        edges = np.unique(np.clip(edges, 1.0, k - 1.0))
        ref = gl_panels(f, edges)
    assert abs(s / ref - 1) < 1e-13


def test_cdf_rows_are_valid(tab):
    for name in ("cdfR", "cdfU", "cdfN", "cdfB", "cdfT", "cdfS"):
        c = tab.export(name).reshape(-1, 65)
        assert np.all(c[:, 0] == 0.0) and np.all(c[:, -1] == 1.0)
        assert np.all(np.diff(c, axis=1) >= 0.0), name
    for name in ("cdfB", "cdfS"):
        c = tab.export(name).reshape(-1, 65)
        assert np.all(c[:, 32] == 0.5)   # symmetric spectra (Sec. II.C)


def test_brems_cdf_interior_values(tab):
    # CDF at panel edges = partial integrals in the row abscissa
    i, l = 25, 40
    g = math.exp(node(math.log(2), math.log(100), 56, i))
    L = Lnode(l)
    row = tab.export("cdfR").reshape(56, NL, 65)[i, l]
    T = g - 1; klo = 1e-7 * T
    Y = math.log((g - klo) / 1e-7)
    tot = brems_sigma_ref(g, L, False)
    for j in (8, 32, 50):
        # t_j -> k_j: y = y_hi - (1 - t) Y, k/g2 = e^y
        ey = T * math.exp(-(1 - j / 64) * Y)
        kj = g * ey / (1 + ey)
        part = gl_panels(lambda v: math.exp(v) * O.dsdk_rel(Z, g, math.exp(v), L),
                         np.linspace(math.log(klo), math.log(kj), 121))
        assert abs(row[j] - part / tot) < 1e-12


def test_photon_energy_cut_is_negligible():
    # Sec. III.A: with n = 7 the energy radiated below k = 1e-7 (g1 - 1)
    # is a negligible fraction (epsilon ~ 1e-5) of the total
    for g1, L in ((1 + 10.0 / 0.511, 44.6), (1 + 100.0 / 0.511, 70.8), (1 + 1.0 / 0.511, 1e4)):
        T = g1 - 1
        klo = 1e-7 * T
        below = gl_panels(lambda v: math.exp(2 * v) * O.dsdk_rel(Z, g1, math.exp(v), L),
                          np.linspace(math.log(klo) - 40, math.log(klo), 81))
        total = below + brems_sigma_ref(g1, L, False, 1)
        assert below / total < 1e-5


@pytest.mark.parametrize("gamma,Zs,T", [(20.0, 10.0, 100.0), (400.0, 3.0, 1e3), (1.4, 5.0, 50.0)])
def test_brems_sampling_matches_exact_spectrum(tab, gamma, Zs, T):
    # sampled k' (inverse of the tabulated CDF) vs the exact CDF of dsigma/dk
    ni = 8.5e28
    s = O.screening(Z, Zs, ni, T)
    xi = (np.arange(2000) + 0.5) / 2000
    ks = np.array([tab.sample(Zs, ni, T, gamma, O.BREMS, x)[0] for x in xi])
    assert np.all(np.diff(ks) > 0)
    Tk = gamma - 1
    assert ks.min() >= 1e-7 * Tk * (1 - 1e-12) and ks.max() <= Tk
    # exact CDF at a few quantiles
    if gamma > 2:
        f = lambda k: O.dsdk_rel(Z, gamma, k, s["Lr"], gamma > 100)
    else:
        f = lambda k: O.dsdk_nr(Z, gamma, k, s["ed"], s["Ltf"], s["Ld"], True)
    klo = 1e-7 * Tk
    if gamma > 2:
        tot = brems_sigma_ref(gamma, s["Lr"], gamma > 100)
    else:
        tot = brems_sigma_ref(gamma, None, False, nr=(s["ed"], s["Ltf"], s["Ld"]))
    for q in (200, 1000, 1800):
        kq = ks[q]
        if kq > 0.5 * Tk:
            continue
        part = gl_panels(lambda v: math.exp(v) * f(math.exp(v)), np.linspace(math.log(klo), math.log(kq), 81))
        # interpolation in the tables (energy, screening, CDF panels)
        assert abs(part / tot - xi[q]) < 5e-3


def test_bh_sampling_range_and_symmetry(tab):
    for k in (2.0 + 1e-5, 3.0, 50.0, 1.5e4):
        xs = (np.arange(401) + 0.5) / 402
        gp = np.array([tab.sample(20.0, 5.9e28, 100.0, k, O.BH, x)[0] for x in xs])
        assert np.all(gp >= 1.0 - 1e-12) and np.all(gp <= k - 1 + 1e-9)
        assert np.all(np.diff(gp) >= 0)
        # median of a symmetric spectrum is k/2
        med = tab.sample(20.0, 5.9e28, 100.0, k, O.BH, 0.5)[0]
        assert abs(med - 0.5 * k) < 1e-9 * k


def test_trident_sampling(tab):
    for g1 in (3.5, 10.0, 300.0, 1.9e4):
        for x1 in (0.01, 0.3, 0.77, 0.999):
            gp, gm = tab.sample(0.0, 8.5e28, 1.0, g1, O.TRIDENT, x1, 0.42)
            gpair = gp + gm
            assert 2.0 - 1e-12 <= gpair <= g1 - 1 + 1e-9
            assert gp >= 1.0 - 1e-12 and gm >= 1.0 - 1e-12
            if gpair > 4.0:
                # sampled split lies where Bhabha's shape is positive
                assert (gp - 1) * (gm - 1) >= 1.0 - 1e-9
