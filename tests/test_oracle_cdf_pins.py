"""Pins of the oracle's sampling tables for pair production (Sec. II.C,
eq:dsdkbh; Sec. II.D, the Trident pair-energy interpolation and Bhabha's
positron split) and of the samplers built on them (inversion of the
cumulative distribution, Sec. III.A).

The tables store, per row, the normalised cumulative distribution at 64
panel edges of the row abscissa t, integrated panel by panel with
8-point Gauss-Legendre in a logarithmic variable (ln g_p for the pair
energy, ln(g+/g_lo) for the split, ln g+ for Bethe-Heitler, each half row
mirrored).  Here every interior value is recomputed by a different rule:
24-point Gauss-Legendre on sub-panels of the energy itself (g_p, g+), with
no mirroring, from the oracle's differential cross sections.  A wrong
Jacobian of the table variable, a wrong rewrite of the split shape's
logarithm, or a wrong mirror would fail these.  Then samples drawn through
the tables are tested against the exact distributions (Kolmogorov-Smirnov
on random draws, and the quantiles of evenly spaced draws)."""
import math

import numpy as np
import pytest
from scipy import stats

from oracle import oracle as O

Z = 79
GX, GW = np.polynomial.legendre.leggauss(24)
LNL = (math.log(10.0), math.log(1e6))


def node(a, b, n, i):
    return a + i * ((b - a) / (n - 1))


def gl(f, lo, hi, sub=3):
    """Integral of f over [lo, hi]: `sub` equal sub-panels, 24-point GL."""
    e = np.linspace(lo, hi, sub + 1)
    s = 0.0
    for a, b in zip(e[:-1], e[1:]):
        x = 0.5 * (b - a) * GX + 0.5 * (b + a)
        s += 0.5 * (b - a) * sum(w * f(t) for w, t in zip(GW, x))
    return s


def cumulative(f, edges, sub=3):
    """F at the given increasing edges (F(edges[0]) = 0), integrating f on
    each interval with `sub` sub-panels."""
    c = [0.0]
    for a, b in zip(edges[:-1], edges[1:]):
        c.append(c[-1] + gl(f, a, b, sub))
    return np.array(c)


@pytest.fixture(scope="module")
def tab():
    return O.tables(Z)


# ------------------------------------------------------------------ Trident pair energy
def trident_row_edges(g1):
    """pair energies at the panel edges of the row of g1: ln g_p = ln 2 + t V"""
    V = math.log(g1 - 1.0) - math.log(2.0)
    return np.exp(math.log(2.0) + (np.arange(65) / 64.0) * V)


@pytest.mark.parametrize("i", [1, 9, 40, 85, 123])
def test_trident_pair_energy_cdf_rows(tab, i):
    g1 = math.exp(node(math.log(3.0), math.log(2e4), 124, i))
    row = tab.export("cdfT").reshape(124, 65)[i]
    edges = trident_row_edges(g1)
    C = cumulative(lambda g: O.dsdgp_trident(Z, g1, g), edges)
    np.testing.assert_allclose(row, C / C[-1], rtol=0, atol=1e-12)


def trident_exact_cdf(g1, n=1500):
    """(g_p grid, CDF) of dsigma_T/dg_p on [2, g1 - 1] (sub-panels in g_p,
    geometric edges)."""
    edges = 2.0 + (g1 - 3.0) * (np.geomspace(1.0, 1e4, n + 1) - 1.0) / (1e4 - 1.0)
    C = cumulative(lambda g: O.dsdgp_trident(Z, g1, g), edges, sub=1)
    return edges, C / C[-1]


@pytest.mark.parametrize("g1", [
    math.exp(node(math.log(3.0), math.log(2e4), 124, 20)),        # a row of the table
    37.3, 812.0, 1.7e4])                                            # between rows
def test_trident_pair_energy_sampling(tab, g1):
    grid, F = trident_exact_cdf(g1)
    cdf = lambda x: np.interp(x, grid, F)
    # evenly spaced draws: the sampled quantiles against the exact ones
    xi = (np.arange(400) + 0.5) / 400
    gp = np.array([sum(tab.sample(0.0, 5.9e28, 1.0, g1, O.TRIDENT, x, 0.5)) for x in xi])
    assert np.all(np.diff(gp) > 0)
    assert abs(gp.min() - 2.0) < 0.1 * (g1 - 3) and gp.max() <= g1 - 1.0 + 1e-9
    assert np.max(np.abs(cdf(gp) - xi)) < 2e-3
    # random draws: Kolmogorov-Smirnov against the exact distribution
    rng = np.random.default_rng(int(g1 * 1000) % 2 ** 31)
    u = rng.random((3000, 2))
    gp = np.array([sum(tab.sample(0.0, 5.9e28, 1.0, g1, O.TRIDENT, a, b)) for a, b in u])
    assert stats.kstest(gp, cdf).pvalue > 1e-3


# ------------------------------------------------------------------ Trident positron split
def split_lower_root(gp):
    return 2.0 / (1.0 + math.sqrt(1.0 - 4.0 / gp))


@pytest.mark.parametrize("i", [1, 6, 30, 77, 119])
def test_trident_split_cdf_rows(tab, i):
    gp = math.exp(node(math.log(4.0), math.log(2e4), 120, i))
    row = tab.export("cdfS").reshape(120, 65)[i]
    glo = split_lower_root(gp)
    V = math.log(gp / (2.0 * glo))
    # panel edges of the lower half: g+ = g_lo exp(2 t V); the upper half is
    # integrated straight on, through g_p/2, not mirrored
    lower = glo * np.exp(2.0 * (np.arange(33) / 64.0) * V)
    upper = gp - lower[::-1][1:]
    edges = np.concatenate([lower, upper])
    assert abs(edges[32] - 0.5 * gp) < 1e-12 * gp and abs(edges[-1] - (gp - glo)) < 1e-12 * gp
    C = cumulative(lambda g: O.split_shape(gp, g), edges)
    np.testing.assert_allclose(row, C / C[-1], rtol=0, atol=1e-12)


def test_trident_split_sampling(tab):
    """The positron energy given the pair energy, against the exact
    conditional distribution of the split shape (probability integral
    transform of each draw, then Kolmogorov-Smirnov against U(0, 1))."""
    rng = np.random.default_rng(7)
    vals = []
    for g1 in (25.0, 600.0, 1.2e4):
        for a, b in rng.random((600, 2)):
            gplus, gminus = tab.sample(0.0, 5.9e28, 1.0, g1, O.TRIDENT, a, b)
            gp = gplus + gminus
            if gp <= 4.0:
                assert gplus == gminus       # an equal split below the shape's support
                continue
            glo = split_lower_root(gp)
            assert glo * (1 - 1e-9) <= gplus <= (gp - glo) * (1 + 1e-9)
            tot = gl(lambda g: O.split_shape(gp, g), glo, gp - glo, sub=16)
            part = gl(lambda g: O.split_shape(gp, g), glo, gplus, sub=8)
            vals.append(part / tot)
    vals = np.array(vals)
    assert len(vals) > 1000
    assert stats.kstest(vals, "uniform").pvalue > 1e-3


# ------------------------------------------------------------------ Bethe-Heitler
def bh_L(l):
    return math.exp(node(LNL[0], LNL[1], 81, l))


@pytest.mark.parametrize("i,l", [(0, 40), (30, 0), (95, 25), (140, 80), (165, 60)])
def test_bethe_heitler_cdf_rows(tab, i, l):
    k = 2.0 + math.exp(node(math.log(1e-6), math.log(2e4 - 2.0), 166, i))
    km2 = k - 2.0                 # exact: the row's k as stored
    L = bh_L(l)
    row = tab.export("cdfB").reshape(166, 81, 65)[i, l]
    V = math.log(0.5 * k)
    # in s = g+ - 1 (the row spans s in [0, k - 2], as small as 1e-6): edges
    # s = expm1(2 t V) on the lower half, k - 2 - s mirrored above
    lower = np.expm1(2.0 * (np.arange(33) / 64.0) * V)
    edges = np.concatenate([lower, km2 - lower[::-1][1:]])
    C = cumulative(lambda s: O.dsdgp_bh(Z, k, 1.0 + s, L), edges)
    # near threshold the half-row's end exp(V) and k/2 differ by the
    # rounding of k in FP64: a resolution of about ulp(k)/(k - 2) in F
    tol = 1e-12 + 4.0 * math.ulp(k) / km2
    np.testing.assert_allclose(row, C / C[-1], rtol=0, atol=tol)


@pytest.mark.parametrize("k,Zs,T", [(3.0, 20.0, 100.0), (40.0, 5.0, 1.0), (900.0, 60.0, 3e3), (1.5e4, 0.0, 1.0)])
def test_bethe_heitler_sampling(tab, k, Zs, T):
    """g+ sampled through the tables of a cell (screening length L_R of
    Sec. II.B.2, between table rows in general) against the exact
    distribution of eq:dsdkbh at that L_R."""
    ni = 5.9e28
    L = O.screening(Z, Zs, ni, T)["Lr"]
    # reference edges geometric towards both ends of [1, k - 1] (g+ - 1 =
    # expm1 of a uniform grid up to ln(k/2), mirrored), where the spectrum
    # bends; linear interpolation between 1500 of them
    half = np.expm1(np.linspace(0.0, math.log(0.5 * k), 751))
    s_edges = np.concatenate([half, (k - 2.0) - half[::-1][1:]])
    C = cumulative(lambda s: O.dsdgp_bh(Z, k, 1.0 + s, L), s_edges, sub=1)
    F = C / C[-1]
    edges = 1.0 + s_edges
    cdf = lambda x: np.interp(x, edges, F)
    xi = (np.arange(400) + 0.5) / 400
    gplus = np.array([tab.sample(Zs, ni, T, k, O.BH, x)[0] for x in xi])
    assert np.all(np.diff(gplus) >= 0)
    # the table's resolution: its rows are piecewise linear over 32 panels
    # of ln g+ per half, coarsest at g+ = k/2 where the spectrum of a photon
    # with k >> 1 is flat (at k = 1.5e4 the last panel spans 12% of it and
    # the linear inverse is off by up to 4e-3 in the cumulative)
    assert np.max(np.abs(cdf(gplus) - xi)) < 5e-3
    rng = np.random.default_rng(int(k * 10))
    gplus = np.array([tab.sample(Zs, ni, T, k, O.BH, x)[0] for x in rng.random(3000)])
    assert stats.kstest(gplus, cdf).pvalue > 1e-3
