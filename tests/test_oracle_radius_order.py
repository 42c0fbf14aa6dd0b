"""Pins of the oracle's threshold-radius search by radial bins (Sec. 2.3.4)
and of the group order of the members (Sec. 2.3.5).

The threshold radius has a plain definition: with the squared distances of a
group's members to the nucleus sorted, d_0 <= d_1 <= ..., it is the innermost
d_k, k >= 1, where the enclosed density k / (K d_k^3) falls below one (in units
of Delta_L1), i.e. K^2 d_k^6 > k^2 (Sec. 2.2.2 step 1, Sec. 2.3.3), and the
group size when there is none.  It is pinned here by counting alone (the count
i has exactly i members strictly inside R^3 = i/K and no earlier crossing), and
the radial-bin search, a different route, must give the same count on every
input, including ties and values on the bin edges.
"""
from __future__ import annotations

import numpy as np
import pytest

import oracle

K2 = (4.0 * np.pi / 3.0 * 200.0) ** 2   # K = (4 pi/3) Delta_L1 nbar at Delta_L1 = 200, nbar = 1
W = 0.4 / np.sqrt(3.0)


def _t(e):
    return K2 * ((e * e) * e)


def _count_pin(e, i):
    """i is the threshold count of e, checked by counting (no sort): exactly i
    members have K^2 e^3 < i^2, and every k in [1, i) has more than k members
    with K^2 e^3 <= k^2 (the enclosed density is still at or above the
    threshold at the k-th member)."""
    m = len(e)
    T = _t(e)
    if i < m:
        assert np.count_nonzero(T < float(i) ** 2) == i
    ks = np.arange(1, min(i, m))
    if len(ks):
        c = np.count_nonzero(T[None, :] <= (ks.astype(np.float64) ** 2)[:, None], axis=1)
        assert np.all(c > ks)


def _nfw_like(rng, m, r_core, frac_bg=0.3, r_bg=4.0):
    # a cuspy cluster plus background: the crossing lies at a few core radii
    nin = int(m * (1 - frac_bg))
    r = r_core * rng.random(nin) ** 1.5
    rb = r_bg * rng.random(m - nin) ** (1 / 3)
    e = np.concatenate([[0.0], (np.concatenate([r, rb]) ** 2)[: m - 1]])
    return rng.permutation(e)


CASES = []
_rng = np.random.default_rng(20)
for _m, _rc in [(40, 0.3), (300, 0.5), (2000, 1.0), (20000, 2.0)]:
    CASES.append(("nfw", _nfw_like(_rng, _m, _rc)))
CASES.append(("uniform", np.concatenate([[0.0], (3.0 * _rng.random(999)) ** 2])))
# ties: many members at identical distances, several of them exactly on bin edges
_edges = ((np.arange(1, 9) * W) ** 2)
CASES.append(("edges", _rng.permutation(np.concatenate([[0.0], np.repeat(_edges, 7), _edges[:3] * 0.5]))))
CASES.append(("ties", _rng.permutation(np.concatenate([[0.0], np.full(50, 0.01), np.full(30, 0.2),
                                                       np.full(20, 0.9)]))))
CASES.append(("no-crossing", np.concatenate([[0.0], np.full(60, 1e-4)])))   # all deep inside: i = m
CASES.append(("crossing-at-1", np.array([0.0, 25.0, 26.0, 30.0])))        # second member already outside
CASES.append(("single", np.array([0.0])))
CASES.append(("pair", np.array([0.0, 1e-6])))


@pytest.mark.parametrize("name,e", CASES, ids=[c[0] for c in CASES])
def test_sorted_definition_pinned_by_counting(name, e):
    i, _ = oracle.radius_search(e, K2, "sort")
    assert 1 <= i <= len(e) or len(e) == 1
    _count_pin(e, i)


def test_definition_special_cases():
    assert oracle.radius_search(np.array([0.0]), K2, "sort")[0] == 1
    assert oracle.radius_search(np.concatenate([[0.0], np.full(60, 1e-4)]), K2, "sort")[0] == 61
    assert oracle.radius_search(np.array([0.0, 25.0, 26.0, 30.0]), K2, "sort")[0] == 1
    # members all at one squared distance e beyond the nucleus: the enclosed
    # density k / (K d^3) is smallest at k = 1, so the radius is there when
    # K^2 e^3 > 1 and there is no crossing (i = m) otherwise
    for e0 in (0.01, 0.0105, 0.0106, 0.1):
        e = np.concatenate([[0.0], np.full(40, e0)])
        assert oracle.radius_search(e, K2, "sort")[0] == (1 if _t(e0) > 1.0 else len(e))
    # one member per shell with K^2 e_k^3 = k^2 exactly in real numbers: the
    # crossing needs strictly more, so it comes where the shells step out further
    ks = np.arange(1, 30, dtype=np.float64)
    e = np.concatenate([[0.0], np.cbrt(ks ** 2 / K2) * 0.999, [np.cbrt(30.0 ** 2 / K2) * 1.01]])
    assert oracle.radius_search(e, K2, "sort")[0] == 30


@pytest.mark.parametrize("w", [W, W / 7.0, 3.0 * W, 100.0])
@pytest.mark.parametrize("name,e", CASES, ids=[c[0] for c in CASES])
def test_radial_bins_equal_the_definition(name, e, w):
    i_sort, _ = oracle.radius_search(e, K2, "sort")
    i_bins, searched = oracle.radius_search(e, K2, "bins", w)
    assert i_bins == i_sort
    if len(e) >= 2:
        assert searched >= 1   # the innermost occupied bin is always searched


def test_radial_bins_random_stress():
    rng = np.random.default_rng(21)
    for trial in range(300):
        m = int(rng.integers(2, 400))
        scale = float(rng.choice([0.05, 0.3, 1.0, 3.0]))
        e = (scale * rng.random(m)) ** 2
        if trial % 3 == 0:   # snap some values onto bin edges and duplicate others
            w = W
            j = rng.integers(0, 12, size=m // 4)
            e[: m // 4] = ((j + 1) * w) ** 2
            e[m // 4: m // 2] = e[0]
        else:
            w = float(rng.choice([W, W / 3.0, 2.0 * W]))
        e[rng.integers(0, m)] = 0.0
        a, _ = oracle.radius_search(e, K2, "sort")
        b, _ = oracle.radius_search(e, K2, "bins", w)
        assert a == b, (trial, m, scale, w)
        _count_pin(e, a)


def test_radial_bins_search_few_bins_on_a_cuspy_halo():
    # the point of the method: most bins are passed over by the count test
    e = _nfw_like(np.random.default_rng(22), 20000, 2.0)
    i, searched = oracle.radius_search(e, K2, "bins", W)
    nb = int(np.sqrt(e.max()) / W) + 1
    assert i == oracle.radius_search(e, K2, "sort")[0]
    assert searched <= 3 and nb > 10


@pytest.mark.parametrize("seed,n,kw", [(31, 20000, {}), (32, 12000, {"pair_frac": 0.4}),
                                       (33, 8000, {"c_roche": 1.0})])
def test_whole_pass_identical_with_radial_bins(seed, n, kw):
    from paper_2110_11408_amd import synth
    pk = {k: v for k, v in kw.items() if k in ("c_roche",)}
    sk = {k: v for k, v in kw.items() if k not in pk}
    pos, L, _ = synth.small_box(n, seed=seed, nmax=2500, **sk)
    a = oracle.find(pos, box=L, **pk)
    b = oracle.find(pos, box=L, radius="bins", **pk)
    assert a["n_halos"] > 0
    np.testing.assert_array_equal(a["halo_id"], b["halo_id"])
    np.testing.assert_array_equal(a["owner_all"], b["owner_all"])
    for k in a["table"]:
        np.testing.assert_array_equal(a["table"][k], b["table"][k])
    for k in a["found"]:
        np.testing.assert_array_equal(a["found"][k], b["found"][k])


# ------------------------------------------------------------- group order

def test_group_order_hand_case():
    halo_id = np.array([0, 5, 3, 5, 0, 3, 9, 5])
    table = np.array([3, 5, 9])
    members, start = oracle.group_order(halo_id, table)
    np.testing.assert_array_equal(members, [2, 5, 1, 3, 7, 6, 0, 4])
    np.testing.assert_array_equal(start, [0, 2, 5, 6])
    m2, s2 = oracle.group_sweep(halo_id, table, np.array([2, 3, 1]))
    np.testing.assert_array_equal(s2, start)
    for r in range(len(table) + 1):
        assert sorted(m2[s2[r]:(s2[r + 1] if r < len(table) else len(halo_id))]) == \
            sorted(members[start[r]:(start[r + 1] if r < len(table) else len(halo_id))])


def test_group_order_edge_cases():
    # no halos: everything is in the unassigned tail, in ascending order
    m, s = oracle.group_order(np.zeros(5, np.int32), np.zeros(0, np.int32))
    np.testing.assert_array_equal(m, np.arange(5))
    np.testing.assert_array_equal(s, [0])
    # every particle in one halo
    m, s = oracle.group_order(np.full(4, 2), np.array([2]))
    np.testing.assert_array_equal(m, np.arange(4))
    np.testing.assert_array_equal(s, [0, 4])
    with pytest.raises(ValueError):
        oracle.group_order(np.array([0, 7]), np.array([2]))
    with pytest.raises(ValueError):
        oracle.group_sweep(np.array([0, 7]), np.array([2]), np.array([1]))


def test_group_order_matches_the_sweep_on_a_found_box():
    from paper_2110_11408_amd import synth
    pos, L, _ = synth.small_box(20000, seed=34, nmax=2500)
    r = oracle.find(pos, box=L)
    t = r["table"]
    assert r["n_halos"] > 3
    members, start = oracle.group_order(r["halo_id"], t["id"])
    sweep, s2 = oracle.group_sweep(r["halo_id"], t["id"], t["n"])
    np.testing.assert_array_equal(start, s2)
    ends = np.append(start[1:], len(pos))
    for row in range(len(t["id"]) + 1):
        run = members[start[row]:ends[row]]
        assert np.all(np.diff(run) > 0)    # ascending original index
        np.testing.assert_array_equal(np.sort(sweep[s2[row]:ends[row]]), run)
        want = t["id"][row] if row < len(t["id"]) else 0
        assert np.all(r["halo_id"][run] == want)
        if row < len(t["id"]):
            assert len(run) == t["n"][row]
    assert np.array_equal(np.sort(members), np.arange(len(pos)))


@pytest.mark.parametrize("mode,w", [("sort", 0.0), ("bins", 0.5), ("bins", 2.5), ("bins", 100.0)])
def test_exact_tie_is_not_a_crossing(mode, w):
    # with K^2 = 1 the 8th member at e = 4 has K^2 e^3 = 64 = 8^2 exactly: the
    # enclosed density there equals the threshold, which is not "below" it, so
    # the radius is the next member's (K^2 e^3 = 91.125 > 81)
    e = np.array([0.0, 0.5, 0.6, 0.7, 0.8, 0.9, 1.0, 1.1, 4.0, 4.5, 5.0])
    assert np.all(e[1:8] ** 3 <= np.arange(1, 8) ** 2)
    assert oracle.radius_search(e, 1.0, mode, w)[0] == 9
    _count_pin_k2(e, 9, 1.0)


def _count_pin_k2(e, i, k2):
    T = k2 * ((e * e) * e)
    assert np.count_nonzero(T < float(i) ** 2) == i
