"""Pins of the oracle's redshift scaling (Sec. 2.3.1), level 2 (end of
Sec. 2.2.2) and position statistics (Table 1), against values the paper prints,
closed forms, library routines and brute force."""
from __future__ import annotations

import math

import numpy as np
import pytest
from scipy.optimize import brentq

import oracle
from paper_2110_11408_amd import synth
from tests.invariants import check_compaso


@pytest.fixture(scope="module", autouse=True)
def _built():
    oracle.build(force=False)


# ------------------------------------------------------------ redshift scaling

def test_redshift_thresholds_match_table_1():
    """Table 1: SODensityL1 258.2, SODensityL2 1033.0 at z = 0.5 with Omega_M =
    0.315, L0DensityThreshold 77.5 (scaled from 60).  The table's 0.315 is
    rounded; the printed thresholds are met to the table's last digit."""
    r = oracle.params_at_redshift(0.315, 0.5)
    assert r["delta_l1"] == pytest.approx(258.2, rel=5e-4)
    assert r["delta_l2"] == pytest.approx(1033.0, rel=5e-4)
    assert r["delta_l0_min"] == pytest.approx(77.5, rel=1e-3)
    assert r["b_kernel"] == 0.4                       # unchanged (Sec. 2.3.1)


def test_redshift_einstein_de_sitter_is_identity():
    for z in (0.0, 0.5, 3.0):
        r = oracle.params_at_redshift(1.0, z)
        assert r["delta_l1"] == 200.0 and r["delta_l2"] == 800.0 and r["delta_l0_min"] == 60.0
        assert r["l_fof"] == 0.25
    # high redshift: Omega_m(z) -> 1, the scaling tends to 1
    assert oracle.params_at_redshift(0.315, 1000.0)["delta_l1"] == pytest.approx(200.0, rel=1e-6)


def test_redshift_scaling_closed_form_and_linking_length():
    """Delta_L1(z) = 200 (18 pi^2 + 82 x - 39 x^2) / (18 pi^2 Omega_m(z)) from an
    independent evaluation of Omega_m(z) = 1 / (1 + (1/Om - 1)/(1+z)^3); the
    linking length scales as the inverse cube root of the threshold change."""
    for om, z in ((0.315, 0.0), (0.3, 1.0), (0.25, 2.5)):
        omz = 1.0 / (1.0 + (1.0 / om - 1.0) / (1.0 + z) ** 3)
        x = omz - 1.0
        expect = 200.0 * (18 * math.pi ** 2 + 82 * x - 39 * x * x) / (18 * math.pi ** 2 * omz)
        r = oracle.params_at_redshift(om, z)
        assert r["delta_l1"] == pytest.approx(expect, rel=1e-12)
        assert r["delta_l2"] == pytest.approx(4.0 * expect, rel=1e-12)
        assert r["l_fof"] * r["delta_l1"] ** (1 / 3) == pytest.approx(0.25 * 200 ** (1 / 3), rel=1e-12)


# ------------------------------------------------------------------- level 2

@pytest.fixture(scope="module")
def l2_run():
    pos, L, _ = synth.small_box(40123, seed=103, nmax=5000, pair_frac=0.2)
    res = oracle.find(pos, box=L)
    st = oracle.l2_stats(pos, res["density"], res["halo_id"], box=L)
    return pos, L, res, st


def test_l2_satisfies_the_compaso_invariants_inside_l1_haloes(l2_run):
    """Level 2 is CompaSO with Delta_L2 inside each L1 halo: every invariant of
    Sec. 2.2.2 holds with the L1 haloes as the groups."""
    pos, L, res, st = l2_run
    d2 = oracle.derive(len(pos), box=L, delta_l1=800.0)
    l2 = st["l2"]
    found = {"l0": l2[:, 0], "nucleus": l2[:, 1], "ienc": l2[:, 2], "count": l2[:, 3]}
    assert len(l2) > 10
    check_compaso(pos, L, res["density"], res["halo_id"], found, st["l2_owner"], nbar=d2["nbar"],
                  b=d2["b"], delta_l1=800.0, alpha=0.8, c_roche=2.0, floor=d2["floor"])


def test_l2_summary_fields(l2_run):
    pos, L, res, st = l2_run
    t = res["table"]
    np.testing.assert_array_equal(st["id"], t["id"])          # ascending L1 id
    np.testing.assert_array_equal(st["n"], t["n"])
    l2 = st["l2"]
    for k, hid in enumerate(st["id"]):
        mine = l2[l2[:, 0] == hid]
        assert st["n_l2"][k] == len(mine)
        if len(mine):
            assert st["l2max_nucleus"][k] == mine[0, 1] and st["l2max_n"][k] == mine[0, 3]
            top = np.sort(mine[:, 3])[::-1][:5]
            np.testing.assert_array_equal(st["l2_mass"][k][:len(top)], top.astype(float))
            assert np.all(st["l2_mass"][k][len(top):] == 0.0)
        else:
            assert st["l2max_nucleus"][k] == -1 and np.all(st["l2_mass"][k] == 0.0)
            np.testing.assert_array_equal(st["x_l2com"][k], st["x_com"][k])


def test_group_order_listing(l2_run):
    pos, L, res, st = l2_run
    g = st["gstart"]
    assert g[-1] == np.sum(res["halo_id"] > 0)
    for k, hid in enumerate(st["id"]):
        np.testing.assert_array_equal(st["members"][g[k]:g[k + 1]], np.nonzero(res["halo_id"] == hid)[0])


def _numpy_d2(pos, com, L):
    d = pos.astype(np.float64) - com
    d = np.where(d > 0.5 * L, d - L, np.where(d < -0.5 * L, d + L, d))
    return ((d[:, 0] * d[:, 0] + d[:, 1] * d[:, 1]) + d[:, 2] * d[:, 2]).astype(np.float32)


def test_r_pct_is_the_inverted_cdf_percentile(l2_run):
    """r_XX = the distance below which XX % of the members lie: numpy's
    inverted-CDF percentile of the members' distances about x_L2com."""
    pos, L, res, st = l2_run
    g = st["gstart"]
    for k in range(len(st["id"])):
        mem = st["members"][g[k]:g[k + 1]]
        d2 = _numpy_d2(pos[mem], st["x_l2com"][k], L)
        for u, xx in enumerate(oracle.PCT):
            q = np.percentile(d2, xx, method="inverted_cdf")
            assert st["r_pct"][k][u] == math.sqrt(float(q)), (k, xx)


def test_vcirc_by_brute_force_mass_counts(l2_run):
    """v_circ^2 = G M(<=r) m_p / r (G = 1) maximised over the members, with the
    enclosed count taken by counting every member at or inside each radius."""
    pos, L, res, st = l2_run
    g = st["gstart"]
    for k in range(len(st["id"])):
        mem = st["members"][g[k]:g[k + 1]]
        r = np.sqrt(_numpy_d2(pos[mem], st["x_l2com"][k], L).astype(np.float64))
        M = (r[None, :] <= r[:, None]).sum(axis=1)
        ok = r > 0
        v = np.sqrt(M[ok] / r[ok])
        assert st["vcirc_max"][k] == pytest.approx(v.max(), rel=1e-12)
        best = r[ok][v == v.max()]
        assert st["rvcirc_max"][k] in best


def test_stats_move_with_a_periodic_translation(l2_run):
    """Shifting every position by a vector (mod L) shifts both centres by it and
    leaves every other statistic unchanged (up to float32 rounding)."""
    pos, L, res, st = l2_run
    shift = np.array([L / 2, L / 3, 0.25 * L])
    pos2 = np.mod(pos.astype(np.float64) + shift, L).astype(np.float32)
    pos2[pos2 >= np.float32(L)] = 0.0
    st2 = oracle.l2_stats(pos2, res["density"], res["halo_id"], box=L)
    for key in ("x_com", "x_l2com"):
        dd = np.mod(st2[key] - st[key] - shift + L / 2, L) - L / 2
        assert np.max(np.abs(dd)) < 1e-4
    np.testing.assert_array_equal(st2["n_l2"], st["n_l2"])
    np.testing.assert_allclose(st2["r_pct"], st["r_pct"], rtol=1e-4, atol=1e-5)
    np.testing.assert_allclose(st2["vcirc_max"], st["vcirc_max"], rtol=1e-4)


def _nfw_halo(rng, n, centre, c=8.0):
    r200 = float(synth.r200(n, 1.0))
    radii = synth.nfw_radii(rng, np.array([n]), np.array([r200]))
    v = rng.standard_normal((n, 3))
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    return centre + radii[:, None] * v, r200


def test_isolated_nfw_halo_statistics():
    """One NFW halo (c = 8) in a uniform background: its first L2 nucleus is its
    L1 nucleus (the densest particle), both centres of mass lie in the core,
    r_vmax is near the NFW value 2.163 r_s and r_50 near the half-mass radius of
    the profile truncated at R200."""
    rng = np.random.default_rng(7)
    L = 30.0
    nh = 20000
    bg = (rng.random((int(L ** 3), 3)) * L)
    centre = np.array([L / 2, L / 2, L / 2])
    halo, r200 = _nfw_halo(rng, nh, centre)
    pos = np.mod(np.concatenate([bg, halo]), L).astype(np.float32)
    res = oracle.find(pos, box=L, mean_density=1.0)
    st = oracle.l2_stats(pos, res["density"], res["halo_id"], box=L, mean_density=1.0)
    k = int(np.argmax(st["n"]))
    assert st["l2max_nucleus"][k] == res["table"]["nucleus"][k]
    assert np.linalg.norm(st["x_com"][k] - centre) < 0.1 * r200
    assert np.linalg.norm(st["x_l2com"][k] - centre) < 0.05 * r200
    rs = r200 / 8.0
    assert st["rvcirc_max"][k] == pytest.approx(2.163 * rs, rel=0.25)
    mu = lambda y: math.log1p(y) - y / (1 + y)           # noqa: E731
    x50 = brentq(lambda x: mu(8 * x) / mu(8.0) - 0.5, 1e-3, 1.0)
    assert st["r_pct"][k][3] == pytest.approx(x50 * r200, rel=0.15)


def test_subhalo_inside_an_l1_halo_is_found_at_level_2():
    """A 2 000-particle halo at 0.55 R200 of a 20 000-particle one lies inside
    alpha R_L1 of the main nucleus, so L1 merges them (one L1 halo); at the
    higher L2 threshold R_L2 is smaller and the subhalo becomes an L2 halo of
    its own (the purpose of level 2, end of Sec. 2.2.2)."""
    rng = np.random.default_rng(11)
    L = 36.0
    bg = rng.random((int(L ** 3), 3)) * L
    centre = np.array([L / 2, L / 2, L / 2])
    main, r200 = _nfw_halo(rng, 20000, centre)
    sub_c = centre + np.array([0.55 * r200, 0.0, 0.0])
    sub, r200s = _nfw_halo(rng, 2000, sub_c)
    pos = np.mod(np.concatenate([bg, main, sub]), L).astype(np.float32)
    res = oracle.find(pos, box=L, mean_density=1.0)
    st = oracle.l2_stats(pos, res["density"], res["halo_id"], box=L, mean_density=1.0)
    k = int(np.argmax(st["n"]))
    near_sub = np.linalg.norm(pos[res["table"]["nucleus"]].astype(np.float64) - sub_c, axis=1) < 0.3 * r200s
    assert not np.any(near_sub), "the subhalo should not be an L1 halo of its own"
    assert st["n_l2"][k] >= 2
    l2 = st["l2"][st["l2"][:, 0] == st["id"][k]]
    d_sub = np.linalg.norm(pos[l2[:, 1]].astype(np.float64) - sub_c, axis=1)
    assert np.min(d_sub) < 0.3 * r200s
    assert st["l2_mass"][k][1] > 0 and np.all(np.diff(st["l2_mass"][k]) <= 0)


def _nfw_radii_c(rng, n, r200, c):
    """NFW radii with concentration c (inverse of the enclosed-mass fraction,
    tabulated on a fine grid), truncated at R200."""
    mu = lambda y: np.log1p(y) - y / (1 + y)            # noqa: E731
    x = np.linspace(0.0, 1.0, 200001)
    m = mu(c * x) / mu(c)
    return np.interp(rng.random(n), m, x) * r200


def test_several_l2_haloes_order_and_centres():
    """A main halo with two embedded subhaloes, the smaller one more concentrated:
    L2 creates the haloes in descending peak density (main, small, large), so
    the five largest masses must be re-ordered; the first L2 halo is the main
    one; x_L2com is the mean position of that halo's members."""
    rng = np.random.default_rng(5)
    L = 40.0
    bg = rng.random((int(L ** 3), 3)) * L
    centre = np.array([L / 2, L / 2, L / 2])
    parts, r200s = [], []
    for n, c, off in ((30000, 8.0, (0.0, 0.0, 0.0)), (4000, 3.0, (0.55, 0.0, 0.0)),
                      (1500, 30.0, (-0.5, 0.2, 0.0))):
        r200 = float(synth.r200(n, 1.0))
        if not r200s:
            r200m = r200
        cc = centre + np.array(off) * r200m
        v = rng.standard_normal((n, 3))
        v /= np.linalg.norm(v, axis=1, keepdims=True)
        parts.append(cc + _nfw_radii_c(rng, n, r200, c)[:, None] * v)
        r200s.append((cc, r200))
    pos = np.mod(np.concatenate([bg] + parts), L).astype(np.float32)
    res = oracle.find(pos, box=L, mean_density=1.0)
    st = oracle.l2_stats(pos, res["density"], res["halo_id"], box=L, mean_density=1.0)
    k = int(np.argmax(st["n"]))
    l2 = st["l2"][st["l2"][:, 0] == st["id"][k]]
    counts = l2[:, 3]
    assert len(l2) >= 3 and st["n_l2"][k] == len(l2)
    assert np.any(np.diff(counts) > 0), "creation order should not be size order here"
    np.testing.assert_array_equal(st["l2_mass"][k][:min(5, len(counts))],
                                  np.sort(counts)[::-1][:5].astype(float))
    assert st["l2max_nucleus"][k] == l2[0, 1] == res["table"]["nucleus"][k]
    # centre of mass of the first L2 halo: plain mean of minimum-image offsets
    sel = np.nonzero(st["l2_owner"] == l2[0, 1] + 1)[0]
    assert len(sel) == st["l2max_n"][k]
    ref = pos[l2[0, 1]].astype(np.float64)
    d = pos[sel].astype(np.float64) - ref
    d = d - L * np.round(d / L)
    np.testing.assert_allclose(st["x_l2com"][k], np.mod(ref + d.mean(axis=0), L), atol=1e-6)
    mem = np.nonzero(res["halo_id"] == st["id"][k])[0]
    ref1 = pos[res["table"]["nucleus"][k]].astype(np.float64)
    d1 = pos[mem].astype(np.float64) - ref1
    d1 = d1 - L * np.round(d1 / L)
    np.testing.assert_allclose(st["x_com"][k], np.mod(ref1 + d1.mean(axis=0), L), atol=1e-6)
