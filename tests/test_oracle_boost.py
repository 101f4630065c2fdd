"""Pins of the oracle's frame change for moving ions (Sec. III.A): the
transform to the ion rest frame against a textbook boost written in the
rapidity form, its inverse and invariants, the ion-frame collision rate of
eq:proba2 with gamma' = gamma_e gamma_i (1 - beta_e . beta_i), and the
products of each event seen from the ion frame."""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_1907_02814_amd import workloads as W

MEC2_MEV = 0.51099895
C_LIGHT = 299792458.0


def rest_frame(u, E, p):
    """(E', p') in the frame of proper velocity u, by rapidity: the component
    along u mixes with E (cosh, sinh of the rapidity), the rest is kept."""
    u = np.asarray(u, float); p = np.asarray(p, float)
    um = math.sqrt(u @ u)
    if um == 0.0:
        return E, p.copy()
    n = u / um
    ch, sh = math.sqrt(1.0 + um * um), um
    pl = p @ n
    return ch * E - sh * pl, p + ((ch * pl - sh * E) - pl) * n


def _rand_dir(rng):
    v = rng.normal(size=3)
    return v / np.linalg.norm(v)


def test_boost_along_x_is_the_textbook_transform():
    rng = np.random.default_rng(1)
    for _ in range(50):
        eta = rng.uniform(-3, 3)
        u = np.array([math.sinh(eta), 0.0, 0.0])
        p = rng.normal(size=3) * 10
        E = math.sqrt(1 + p @ p)
        Ep, pp = O.to_ion(u, E, p)
        b, g = math.tanh(eta), math.cosh(eta)
        assert abs(Ep - g * (E - b * p[0])) <= 1e-14 * g * E
        assert abs(pp[0] - g * (p[0] - b * E)) <= 1e-14 * g * E
        assert pp[1] == p[1] and pp[2] == p[2]


def test_boost_any_direction_matches_rapidity_form_and_is_invertible():
    rng = np.random.default_rng(2)
    for _ in range(200):
        u = _rand_dir(rng) * math.exp(rng.uniform(-6, 2))
        photon = rng.random() < 0.5
        p = _rand_dir(rng) * math.exp(rng.uniform(-4, 7))
        E = math.sqrt(p @ p) if photon else math.sqrt(1 + p @ p)
        Ep, pp = O.to_ion(u, E, p)
        Er, pr = rest_frame(u, E, p)
        gi = math.sqrt(1 + u @ u)
        scale = (gi + math.sqrt(u @ u)) * E
        assert abs(Ep - Er) <= 1e-14 * scale
        assert np.all(np.abs(pp - pr) <= 1e-14 * scale)
        # invariant mass: 1 for the electron, 0 for the photon
        m2 = Ep * Ep - pp @ pp
        assert abs(m2 - (0.0 if photon else 1.0)) <= 1e-13 * scale * scale
        # and back
        q = O.from_ion(u, Ep, pp)
        assert np.all(np.abs(q - p) <= 1e-13 * scale)


def test_zero_velocity_is_the_identity_and_comoving_particle_is_at_rest():
    p = np.array([3.0, -4.0, 12.0])
    E = math.sqrt(1 + p @ p)
    Ep, pp = O.to_ion(np.zeros(3), E, p)
    assert Ep == E and np.array_equal(pp, p)
    assert np.array_equal(O.from_ion(np.zeros(3), Ep, pp), p)
    # an electron moving with the ion: proper velocity p = u
    Ep, pp = O.to_ion(p, E, p)
    assert abs(Ep - 1.0) <= 1e-13 * E and np.all(np.abs(pp) <= 1e-13 * E)


def _cells(n_cells, ne, ni, ng, e_gamma, rng, Zs=None, k=None, Z=79, gw=None):
    n_i = 5.9e28
    Wi = n_i / ni
    Zs = rng.uniform(0, Z, n_cells) if Zs is None else np.full(n_cells, Zs)
    k = np.zeros(0) if ng == 0 else k
    return W.assemble("boost", Z, 1e-16, 7, 1, Zs, np.full(n_cells, n_i),
                      np.full(n_cells, 300.0), e_gamma, np.full(n_cells * ne, Wi),
                      np.full(n_cells, ne), k, np.full(n_cells * ng, Wi) if gw is None else gw,
                      np.full(n_cells, ng), np.full(n_cells * ni, Wi), np.full(n_cells, ni), rng,
                      photon_extra=np.full(n_cells, 4 * ne), pair_cap=np.full(n_cells, 4 * (ne + ng)))


def _run(wl, tab, dt, proc, seed=1, step=0):
    return O.collide_step(tab, wl.cells, wl.electrons, wl.photons, wl.ions, wl.new_el,
                          wl.new_po, dt, seed, step, proc)


def test_ions_with_zero_velocity_behave_as_ions_at_rest():
    tab = O.tables(79)
    rng = np.random.default_rng(3)
    n_cells, ne, ng, ni = 40, 24, 24, 16
    e_g = 1 + W.log_uniform(rng, 1.0, 500.0, n_cells * ne) / MEC2_MEV
    k = (1.022 + rng.exponential(20.0, n_cells * ng)) / MEC2_MEV
    a = _cells(n_cells, ne, ni, ng, e_g, rng, k=k)
    b = a.copy()
    n = len(b.ions["w"])
    b.ions["px"], b.ions["py"], b.ions["pz"] = np.zeros(n), np.zeros(n), np.zeros(n)
    ra = _run(a, tab, 2e-12, 7, seed=4)
    rb = _run(b, tab, 2e-12, 7, seed=4)
    assert np.array_equal(ra[0], rb[0]) and ra[2] == rb[2]
    assert ra[0][:, O.I_NAMES.index("ev_br")].sum() > 50
    np.testing.assert_allclose(rb[1], ra[1], rtol=1e-14, atol=0)
    for sa, sb in ((a.electrons, b.electrons), (a.photons, b.photons), (a.new_el, b.new_el), (a.new_po, b.new_po)):
        for key in ("px", "py", "pz", "w"):
            np.testing.assert_allclose(sb[key], sa[key], rtol=1e-14, atol=0)


def test_electrons_moving_with_the_ions_do_not_radiate():
    tab = O.tables(79)
    rng = np.random.default_rng(4)
    n_cells, ne, ni = 200, 6, 6
    wl = _cells(n_cells, ne, ni, 0, np.full(n_cells * ne, 2.0), rng)
    u = np.repeat(rng.normal(size=(n_cells, 3)) * 20.0, ni, axis=0)
    rest = wl.copy()
    # electrons with the proper velocity of their cell's ions
    ue = np.repeat(u[::ni], ne, axis=0)
    for w in (wl, rest):
        w.electrons["px"], w.electrons["py"], w.electrons["pz"] = (ue[:, 0].copy(), ue[:, 1].copy(), ue[:, 2].copy())
    wl.ions["px"], wl.ions["py"], wl.ions["pz"] = u[:, 0].copy(), u[:, 1].copy(), u[:, 2].copy()
    ti, td, st = _run(wl, tab, 1e-11, O.BREMS | O.TRIDENT)
    assert ti[:, O.I_NAMES.index("ev_br")].sum() == 0 and ti[:, O.I_NAMES.index("ev_tr")].sum() == 0
    assert np.all(ti[:, O.I_NAMES.index("pairs_br")] == ne)
    ti0, _, _ = _run(rest, tab, 1e-11, O.BREMS | O.TRIDENT)
    assert ti0[:, O.I_NAMES.index("ev_br")].sum() > 100     # the same electrons radiate on ions at rest


def test_event_frequency_follows_the_ion_frame_rate():
    # eq:proba2/3 with moving ions: x = (n_e n_i / n_ei) sigma'(gamma') c |p'| dt
    # / (gamma_e gamma_i), gamma' = gamma_e gamma_i (1 - beta_e . beta_i)
    tab = O.tables(29)
    n_cells, ne, ni = 4000, 2, 2
    Zs, n_i, T = 10.0, 8.5e28, 100.0
    ge = 1 + 20.0 / MEC2_MEV
    pe = math.sqrt(ge * ge - 1)
    u = np.array([0.3, 0.0, -0.7])                  # partly head-on
    gi = math.sqrt(1 + u @ u)
    be = np.array([0.0, 0.0, pe / ge]); bi = u / gi
    gp = ge * gi * (1 - be @ bi)
    sig = tab.lookup(Zs, n_i, T, gp, O.BREMS)[0]
    Wi = n_i / ni
    rng = np.random.default_rng(5)
    wl = W.assemble("rate", 29, 1e-16, 1, 1, np.full(n_cells, Zs), np.full(n_cells, n_i),
                    np.full(n_cells, T), np.full(n_cells * ne, ge), np.full(n_cells * ne, Wi),
                    np.full(n_cells, ne), np.zeros(0), np.zeros(0), np.zeros(n_cells, np.int64),
                    np.full(n_cells * ni, Wi), np.full(n_cells, ni), rng,
                    photon_extra=np.full(n_cells, 2 * ne), pair_cap=np.full(n_cells, 4))
    m = n_cells * ne
    wl.electrons["px"], wl.electrons["py"], wl.electrons["pz"] = np.zeros(m), np.zeros(m), np.full(m, pe)
    rest = wl.copy()
    k = n_cells * ni
    wl.ions["px"], wl.ions["py"], wl.ions["pz"] = np.full(k, u[0]), np.full(k, u[1]), np.full(k, u[2])
    rate = (ne * Wi) * n_i / (2 * Wi) * sig * C_LIGHT * math.sqrt(gp * gp - 1) / (ge * gi)
    dt = 0.3 / rate
    ti, td, st = _run(wl, tab, dt, O.BREMS)
    assert st == 0
    P = -math.expm1(-rate * dt)
    n = n_cells * ne
    ev = ti[:, O.I_NAMES.index("ev_br")].sum()
    assert abs(ev - n * P) / math.sqrt(n * P * (1 - P)) < 4.5
    # the rate of the same electrons on ions at rest is far off: the test has power
    sig0 = tab.lookup(Zs, n_i, T, ge, O.BREMS)[0]
    P0 = -math.expm1(-(ne * Wi) * n_i / (2 * Wi) * sig0 * C_LIGHT * pe / ge * dt)
    assert abs(ev - n * P0) / math.sqrt(n * P0 * (1 - P0)) > 10
    ti0, _, _ = _run(rest, tab, dt, O.BREMS)
    ev0 = ti0[:, O.I_NAMES.index("ev_br")].sum()
    assert abs(ev0 - n * P0) / math.sqrt(n * P0 * (1 - P0)) < 4.5


def _cross_rel(a, b):
    return np.linalg.norm(np.cross(a, b)) / max(np.linalg.norm(a) * np.linalg.norm(b), 1e-300)


@pytest.mark.parametrize("proc,dt", [(7, 2e-12), (4, 1e-10)])
def test_products_seen_from_the_ion_frame(proc, dt):
    """One electron, one photon and one moving ion per cell.  In the ion
    frame every product travels along its parent, the electron gives up
    exactly the photon and pair energies and the photon exactly the pair
    energy; in the lab the tallies are the lab energies of the products and
    the change of the electron's Lorentz factor."""
    tab = O.tables(79)
    rng = np.random.default_rng(6)
    n_cells = 3000
    e_g = 1 + W.log_uniform(rng, 20.0, 500.0, n_cells) / MEC2_MEV
    k = (1.022 + rng.exponential(20.0, n_cells)) / MEC2_MEV
    wl = _cells(n_cells, 1, 1, 1, e_g, rng, k=k)
    W.moving_ions(wl, rng, 0.8)
    before = wl.copy()
    ti, td, st = _run(wl, tab, dt, proc, seed=8)
    assert st == 0
    I = {nm: ti[:, i] for i, nm in enumerate(O.I_NAMES)}
    D = {nm: td[:, i] for i, nm in enumerate(O.D_NAMES)}
    need = (50, 0, 50) if proc == 7 else (0, 30, 0)
    assert I["ev_br"].sum() >= need[0] and I["ev_tr"].sum() >= need[1] and I["ev_bh"].sum() >= need[2]
    E, B, Wion = wl.electrons, before.electrons, wl.ions
    ph, ne_, np_ = wl.photons, wl.new_el, wl.new_po
    checked = 0
    for c in range(n_cells):
        u = np.array([Wion["px"][c], Wion["py"][c], Wion["pz"][c]])
        p0 = np.array([B["px"][c], B["py"][c], B["pz"][c]])
        p1 = np.array([E["px"][c], E["py"][c], E["pz"][c]])
        g0, g1 = math.sqrt(1 + p0 @ p0), math.sqrt(1 + p1 @ p1)
        We = E["w"][c]
        E0, q0 = rest_frame(u, g0, p0)
        E1, q1 = rest_frame(u, g1, p1)
        lost = 0.0
        lab_br = lab_tr = lab_bh = 0.0
        gslab = ph["off"][c]
        for a in range(gslab, gslab + ph["count"][c]):
            if ph["parent"][a] != c:
                continue
            kv = np.array([ph["px"][a], ph["py"][a], ph["pz"][a]])
            kl = math.sqrt(kv @ kv)
            Ek, qk = rest_frame(u, kl, kv)
            assert _cross_rel(qk, q0) <= 1e-11
            lost += Ek
            lab_br += We * kl
        pair_e = 0.0
        for slab, sgn in ((ne_, -1), (np_, 1)):
            o = slab["off"][c]
            for a in range(o, o + slab["count"][c]):
                v = np.array([slab["px"][a], slab["py"][a], slab["pz"][a]])
                gv = math.sqrt(1 + v @ v)
                Ev, qv = rest_frame(u, gv, v)
                if a - o < I["ev_tr"][c]:          # Trident products come first (e-i pass)
                    assert slab["parent"][a] == c
                    assert _cross_rel(qv, q0) <= 1e-11
                    lost += Ev
                    lab_tr += We * gv
                else:                               # then the Bethe-Heitler products
                    kv0 = np.array([before.photons["px"][gslab], before.photons["py"][gslab],
                                    before.photons["pz"][gslab]])
                    assert slab["parent"][a] == gslab
                    k0 = math.sqrt(kv0 @ kv0)
                    Ek0, qk0 = rest_frame(u, k0, kv0)
                    assert _cross_rel(qv, qk0) <= 1e-11
                    pair_e += Ev
                    lab_bh += before.photons["w"][gslab] * gv
        if I["ev_br"][c] or I["ev_tr"][c]:
            assert _cross_rel(q1, q0) <= 1e-11
            assert abs(E0 - E1 - lost) <= 1e-12 * E0
            checked += 1
        else:
            assert np.array_equal(p0, p1)
        if I["ev_bh"][c]:
            kv0 = np.array([before.photons["px"][gslab], before.photons["py"][gslab], before.photons["pz"][gslab]])
            k0 = math.sqrt(kv0 @ kv0)
            Ek0, _ = rest_frame(u, k0, kv0)
            assert abs(Ek0 - pair_e) <= 1e-12 * Ek0
            assert abs(D["dE_ph"][c] + before.photons["w"][gslab] * k0) <= 1e-14 * Wion["w"][c] * k0 * 4
        assert abs(D["E_br"][c] - lab_br) <= 1e-14 * abs(lab_br)
        assert abs(D["E_tr"][c] - lab_tr) <= 1e-14 * abs(lab_tr)
        assert abs(D["E_bh"][c] - lab_bh) <= 1e-14 * abs(lab_bh)
        # the electron's lab energy change, from its Lorentz factors
        assert abs(D["dE_el"][c] - We * (g1 - g0)) <= 1e-14 * We * g0 * 4
    assert checked >= need[0] + need[1]
