"""Pins of the oracle's step-after operations (products joining their
populations, Sec. III.A and the chains of Sec. IV): merging a product
buffer into a population, and new slabs with headroom.  Pure data
movement: checked against hand-worked cells and against invariants on
random slabs (order kept, weights and momenta conserved but for the
dropped, counts)."""
import numpy as np

from oracle import oracle as O


def _sp(off, count, vals, parent=False):
    off = np.asarray(off, dtype=np.int64)
    m = int(off[-1])
    v = np.asarray(vals, dtype=np.float64)
    d = {"off": off, "count": None if count is None else np.asarray(count, dtype=np.int32),
         "px": v.copy(), "py": -v, "pz": 2 * v, "w": v + 0.5,
         "parent": np.arange(m, dtype=np.int64) + 1000 if parent else None}
    return d


def test_merge_hand_worked():
    # cell 0: 1 live of 3, 2 to append (fits); cell 1: full, 3 dropped;
    # cell 2: empty dst of 4, 2 to append; src slab of cell 1 holds 4 with 3 live
    dst = _sp([0, 3, 5, 9], [1, 2, 0], [0, 1, 2, 3, 4, 5, 6, 7, 8], parent=True)
    src = _sp([0, 2, 6, 8], [2, 3, 2], [10, 11, 12, 13, 14, 15, 16, 17], parent=True)
    dropped = O.merge_species(dst, src)
    assert dropped.tolist() == [0, 3, 0]
    assert dst["count"].tolist() == [3, 2, 2] and src["count"].tolist() == [0, 0, 0]
    assert dst["px"].tolist() == [0, 10, 11, 3, 4, 16, 17, 7, 8]
    assert dst["py"].tolist() == [-0.0, -10, -11, -3, -4, -16, -17, -7, -8]
    assert dst["w"].tolist() == [0.5, 10.5, 11.5, 3.5, 4.5, 16.5, 17.5, 7.5, 8.5]
    assert dst["parent"].tolist() == [1000, 1000, 1001, 1003, 1004, 1006, 1007, 1007, 1008]


def test_merge_invariants_random():
    rng = np.random.default_rng(5)
    n = 200
    cap_d = rng.integers(0, 40, n)
    cap_s = rng.integers(0, 30, n)
    cnt_d = np.minimum(rng.integers(0, 45, n), cap_d)
    cnt_s = rng.integers(0, 35, n)          # may exceed the slab: only the slab is live
    od = np.concatenate([[0], np.cumsum(cap_d)])
    os_ = np.concatenate([[0], np.cumsum(cap_s)])
    dst = _sp(od, cnt_d, rng.random(od[-1]))
    src = _sp(os_, cnt_s, rng.random(os_[-1]))
    before_d = {k: dst[k].copy() for k in ("px", "w")}
    live_s = np.minimum(cnt_s, cap_s)
    src_w = [src["w"][os_[c]:os_[c] + live_s[c]].copy() for c in range(n)]
    dropped = O.merge_species(dst, src)
    room = cap_d - cnt_d
    np.testing.assert_array_equal(dropped, np.maximum(0, live_s - room))
    np.testing.assert_array_equal(dst["count"], cnt_d + np.minimum(live_s, room))
    assert not src["count"].any()
    for c in range(n):
        a, k = od[c], int(cnt_d[c])
        nk = int(min(live_s[c], room[c]))
        # the old live particles stay, the appended ones follow in src order
        np.testing.assert_array_equal(dst["w"][a:a + k], before_d["w"][a:a + k])
        np.testing.assert_array_equal(dst["w"][a + k:a + k + nk], src_w[c][:nk])
        # slots past the new count are untouched
        np.testing.assert_array_equal(dst["px"][a + k + nk:od[c + 1]], before_d["px"][a + k + nk:od[c + 1]])
    total = sum(w.sum() for w in src_w)
    kept = sum(src_w[c][:int(min(live_s[c], room[c]))].sum() for c in range(n))
    assert abs((sum(dst["w"][od[c]:od[c] + dst["count"][c]].sum() for c in range(n))
                - sum(before_d["w"][od[c]:od[c] + cnt_d[c]].sum() for c in range(n))) - kept) < 1e-9
    assert kept <= total


def test_rebin_keeps_live_particles_and_adds_headroom():
    rng = np.random.default_rng(6)
    n = 150
    cap = rng.integers(0, 30, n)
    cnt = rng.integers(0, 35, n)
    off = np.concatenate([[0], np.cumsum(cap)])
    sp = _sp(off, cnt, rng.random(off[-1]), parent=True)
    for head in (0, 7):
        r = O.rebin(sp, head)
        live = np.minimum(cnt, cap)
        np.testing.assert_array_equal(np.diff(r["off"]), live + head)
        np.testing.assert_array_equal(r["count"], live)
        for c in range(n):
            a, b, k = off[c], r["off"][c], int(live[c])
            for key in ("px", "py", "pz", "w", "parent"):
                np.testing.assert_array_equal(r[key][b:b + k], sp[key][a:a + k])
            assert not r["w"][b + k:r["off"][c + 1]].any()
    # a population without counts (every slot live)
    full = _sp(off, None, rng.random(off[-1]))
    r = O.rebin(full, 3)
    np.testing.assert_array_equal(np.diff(r["off"]), cap + 3)
    np.testing.assert_array_equal(r["count"], cap)
