"""Pins of the oracle's screening functions for the two-exponential
potential eq:V_TFD (Sec. II.B.2, eq:defphi1 and eq:defphi2 with the form
factor eq:defF), which the oracle computes by quadrature of the
definitions, and of the cross sections built on them (eq:csre, eq:csur,
eq:dsdkbh with these functions: the numerically computed TFD forms that
Figs. 5, 7 and 8 compare with the reduced form).

The pins are closed forms the quadrature does not use:
- one exponential (Z* = 0: q_D = 0; or only the Debye term; or equal
  lengths): the printed single-exponential forms eq:deriv_I1, eq:deriv_I2;
- the limit delta -> 0 of both functions: eq:ITFD;
- any two exponentials: the form factor squared splits into two squares
  and a cross term f_A f_B = 1 + B/(A - B) / (1 + A u^2) - A/(A - B) / (1 + B u^2)
  (A, B the squared lengths); with it both integrals are elementary but
  for one dilogarithm, written out here in mpmath at 40 digits."""
import math

import mpmath as mp
import pytest

from oracle import oracle as O



@pytest.fixture(autouse=True)
def _digits():
    """40 digits for every test here (other modules set their own)"""
    with mp.workdps(40):
        yield


def I1_single(d, L):
    """eq:deriv_I1 as printed"""
    d, L = mp.mpf(d), mp.mpf(L)
    return (L * d * (mp.atan(d * L) - mp.atan(L)) - L ** 2 / 2 * (1 - d) ** 2 / (1 + L ** 2)
            + mp.log((1 + L ** 2) / (1 + L ** 2 * d ** 2)) / 2)


def I2_single(d, L):
    """eq:deriv_I2 as printed (it gives 2 I2)"""
    d, L = mp.mpf(d), mp.mpf(L)
    two = (4 * L ** 3 * d ** 3 * (mp.atan(L * d) - mp.atan(L))
           + (1 + 3 * L ** 2 * d ** 2) * mp.log((1 + L ** 2) / (1 + L ** 2 * d ** 2))
           + 6 * L ** 4 * d ** 2 / (1 + L ** 2) * mp.log(d)
           + L ** 2 * (d - 1) * (d + 1 - 4 * L ** 2 * d ** 2) / (1 + L ** 2))
    return two / 2


def cross_terms(d, La, Lb):
    """C_k = int_d^1 kernel_k(u) f_A(u) f_B(u) du for k = 1, 2, with
    f_X = X u^2/(1 + X u^2), X = L^2 (A != B)."""
    d = mp.mpf(d)
    A, B = mp.mpf(La) ** 2, mp.mpf(Lb) ** 2
    lnd = mp.log(d)
    K1 = -lnd - mp.mpf(3) / 2 + 2 * d - d ** 2 / 2
    K2 = (-lnd - 6 * d ** 2 * (lnd / 2 - mp.mpf(1) / 4 + 1 / (4 * d ** 2))
          + 3 * d ** 2 * (1 / d ** 2 - 1) / 2 - 4 * d ** 3 * (1 / d ** 3 - 1) / 3)

    def J(X):
        sX = mp.sqrt(X)
        # antiderivatives of u^-1, u^-2, u^-3, u^-4 and ln(u/d) u^-3, each over (1 + X u^2)
        a1 = lambda u: mp.log(u) - mp.log(1 + X * u ** 2) / 2
        a2 = lambda u: -1 / u - sX * mp.atan(sX * u)
        a3 = lambda u: -1 / (2 * u ** 2) - X * mp.log(u) + X / 2 * mp.log(1 + X * u ** 2)
        a4 = lambda u: -1 / (3 * u ** 3) + X / u + X * sX * mp.atan(sX * u)
        al = lambda u: (-mp.log(u / d) / (2 * u ** 2) - 1 / (4 * u ** 2) - X * mp.log(u / d) ** 2 / 2
                        + X / 2 * (mp.log(u / d) * mp.log(1 + X * u ** 2) + mp.polylog(2, -X * u ** 2) / 2))
        D = lambda f: f(mp.mpf(1)) - f(d)
        j1 = D(a1) - 2 * d * D(a2) + d ** 2 * D(a3)
        j2 = D(a1) - 6 * d ** 2 * D(al) + 3 * d ** 2 * D(a3) - 4 * d ** 3 * D(a4)
        return j1, j2

    jA, jB = J(A), J(B)
    bA, bB = B / (A - B), -A / (A - B)
    return K1 + bA * jA[0] + bB * jB[0], K2 + bA * jA[1] + bB * jB[1]


def I12_tfd_exact(d, etf, ed, Ltf, Ld):
    c1, c2 = cross_terms(d, Ltf, Ld)
    etf, ed = mp.mpf(etf), mp.mpf(ed)
    I1 = etf ** 2 * I1_single(d, Ltf) + ed ** 2 * I1_single(d, Ld) + 2 * etf * ed * c1
    I2 = etf ** 2 * I2_single(d, Ltf) + ed ** 2 * I2_single(d, Ld) + 2 * etf * ed * c2
    return float(I1), float(I2)


def close(a, b, tol):
    assert abs(a - b) <= tol * max(1.0, abs(b)), (a, b, abs(a - b))


DELTAS = [1e-9, 3.7e-6, 2e-4, 0.013, 0.21, 0.77]


@pytest.mark.parametrize("d", DELTAS)
@pytest.mark.parametrize("L", [0.3, 44.6, 2.9e3, 8.0e5])
def test_one_exponential_is_the_printed_closed_form(d, L):
    """Z* = 0 (only the Thomas-Fermi term) and Z* = Z (only the Debye
    term) and equal lengths: eq:deriv_I1, eq:deriv_I2."""
    e1, e2 = float(I1_single(d, L)), float(I2_single(d, L))
    for args in [(1.0, 0.0, L, 1.0), (0.0, 1.0, 7.0, L), (0.4, 0.6, L, L)]:
        i1, i2 = O.I12_tfd(d, *args)
        close(i1, e1, 1e-12)
        close(i2, e2, 1e-12)


@pytest.mark.parametrize("etf,Ltf,Ld", [(0.65, 44.6, 365.4), (0.1, 44.6, 12.0), (0.9, 20.0, 9.0e5),
                                         (0.5, 3.0, 1.5e3)])
def test_delta_to_zero_is_I_tfd(etf, Ltf, Ld):
    """eq:inte: both functions tend to I_TFD (eq:ITFD) as delta -> 0;
    I2 - I_TFD is O(delta^2 L^2 ln), I1 - I_TFD is O(delta L)."""
    ed = 1.0 - etf
    a = O.I_tfd(etf, ed, Ltf, Ld)
    Lm = max(Ltf, Ld)
    d = 1e-10 / Lm
    i1, i2 = O.I12_tfd(d, etf, ed, Ltf, Ld)
    close(i2, a, 1e-12)
    assert abs(i1 - a) <= 4.0 * d * Lm + 1e-12 * a


@pytest.mark.parametrize("d", DELTAS)
@pytest.mark.parametrize("etf,Ltf,Ld", [(0.6551724137931034, 44.60347251244468, 365.36843571082875),
                                         (0.2, 44.6, 3.2e4), (0.93, 100.0, 2.5), (0.5, 1.7, 8.0e5)])
def test_two_exponentials_closed_form(d, etf, Ltf, Ld):
    """The full two-exponential functions against the partial-fraction
    closed form (dilogarithm for I2's logarithmic term)."""
    ed = 1.0 - etf
    e1, e2 = I12_tfd_exact(d, etf, ed, Ltf, Ld)
    i1, i2 = O.I12_tfd(d, etf, ed, Ltf, Ld)
    close(i1, e1, 1e-12)
    close(i2, e2, 1e-12)


def test_partial_fractions_of_the_cross_term():
    """the split of f_A f_B used by the closed form, at a few points"""
    A, B = mp.mpf(44.6) ** 2, mp.mpf(365.4) ** 2
    for u in [mp.mpf("1e-4"), mp.mpf("0.003"), mp.mpf("0.5")]:
        lhs = A * u ** 2 / (1 + A * u ** 2) * B * u ** 2 / (1 + B * u ** 2)
        rhs = 1 + B / (A - B) / (1 + A * u ** 2) - A / (A - B) / (1 + B * u ** 2)
        assert abs(lhs - rhs) < mp.mpf("1e-35")


def test_tfd_cross_sections_reduce_to_the_reduced_form_for_neutral_atoms():
    """Sec. II.B.2 and II.C.1: at Z* = 0 the reduced length is L_TF and the
    numerically computed TFD cross sections coincide with the reduced ones."""
    s = O.screening(29.0, 0.0, 8.5e28, 0.0)
    assert s["ed"] == 0.0
    for g1 in [11.0, 200.0, 2e3]:
        for x in [0.01, 0.3, 0.9]:
            k = x * (g1 - 1.0)
            for cou in (False, True):
                a = O.dsdk_rel_tfd(29.0, g1, k, s["etf"], s["ed"], s["Ltf"], s["Ld"], cou)
                b = O.dsdk_rel(29.0, g1, k, s["Lr"], cou)
                assert abs(a - b) <= 1e-12 * abs(b)
    for k in [20.0, 200.0, 2e4]:
        for x in [0.05, 0.5]:
            gp = 1.0 + x * (k - 2.0)
            a = O.dsdgp_bh_tfd(29.0, k, gp, s["etf"], s["ed"], s["Ltf"], s["Ld"])
            b = O.dsdgp_bh(29.0, k, gp, s["Lr"])
            assert abs(a - b) <= 1e-12 * abs(b)


def test_tfd_cross_sections_use_the_tfd_functions():
    """eq:csre and eq:dsdkbh written out with the pinned TFD functions"""
    Z = 29.0
    s = O.screening(Z, 10.0, 8.5e28, 1e3)
    r_e, alpha = 2.8179403262e-15, 1.0 / 137.035999084
    g1, k = 40.0, 12.0
    g2 = g1 - k
    d = k / (2 * g1 * g2)
    i1, i2 = I12_tfd_exact(d, s["etf"], s["ed"], s["Ltf"], s["Ld"])
    r = g2 / g1
    e = 4 * Z ** 2 * r_e ** 2 * alpha / k * ((1 + r * r) * (i1 + 1) - 2.0 / 3.0 * r * (i2 + 5.0 / 6.0))
    assert abs(O.dsdk_rel_tfd(Z, g1, k, s["etf"], s["ed"], s["Ltf"], s["Ld"]) - e) <= 1e-12 * e
    kk, gp = 300.0, 71.0
    gm = kk - gp
    d = kk / (2 * gp * gm)
    i1, i2 = I12_tfd_exact(d, s["etf"], s["ed"], s["Ltf"], s["Ld"])
    e = 4 * Z ** 2 * r_e ** 2 * alpha / kk ** 3 * ((gp * gp + gm * gm) * (i1 + 1) + 2.0 / 3.0 * gp * gm * (i2 + 5.0 / 6.0))
    assert abs(O.dsdgp_bh_tfd(Z, kk, gp, s["etf"], s["ed"], s["Ltf"], s["Ld"]) - e) <= 1e-12 * e
