"""Pins of the oracle's near-threshold events (orc_events).

Labels are exact functions of the densities (every geometric predicate is the
same FP64 expression on every side), so a density field within a tolerance of
another can only change labels through the density comparisons of the method:
the L0 cut (Sec. 2.2.1), the nucleation floor, the peak test and the order of
nuclei (Sec. 2.2.2).  The events name where that can happen.  Pinned here by
  * hand-built configurations where each event is on, or just off, its bound;
  * brute force = cell list;
  * the property the events exist for: a field perturbed by at most the
    tolerance changes labels only on particles the events explain.
"""
from __future__ import annotations

import numpy as np
import pytest

import oracle
from paper_2110_11408_amd import synth
from tests.gpu_helpers import explained_mismatches, matched_agreement


@pytest.fixture(scope="module", autouse=True)
def _built():
    oracle.build(force=False)


L_BOX = 10.0
KW = dict(box=L_BOX, mean_density=1.0)   # b = 0.4, l = 0.25, floor 250.837


def _hand_case(peak_gap, order_gap, cut_gap, floor_gap):
    """Positions and densities of small clusters far apart (all offsets
    along x, spacing 0.22 < l):
      A  two members: a at 60 + cut_gap (the L0 cut), a neighbour at 100;
      E  a non-member at 60 - cut_gap next to a member at 100 (a group of its
         own that the cut particle would join);
      B  one member at floor + floor_gap and a neighbour at 100;
      C  two members 0.22 apart at 1000 and 1000 (1 + peak_gap);
      D  a chain H - J - K - I with H and I 0.66 apart, local peaks at 500 and
         500 (1 + order_gap), J and K at 100."""
    fl = oracle.derive(1000, **KW)["floor"]
    pts, dens = [], []
    def put(x, y, z, d):
        pts.append((x, y, z))
        dens.append(d)
    put(1.0, 1.0, 1.0, 60.0 + cut_gap)
    put(1.22, 1.0, 1.0, 100.0)
    put(7.0, 7.0, 7.0, fl + floor_gap)
    put(7.22, 7.0, 7.0, 100.0)
    put(3.0, 3.0, 3.0, 1000.0)
    put(3.22, 3.0, 3.0, 1000.0 * (1 + peak_gap))
    put(3.0, 7.0, 3.0, 500.0)
    put(3.22, 7.0, 3.0, 100.0)
    put(3.44, 7.0, 3.0, 100.0)
    put(3.66, 7.0, 3.0, 500.0 * (1 + order_gap))
    put(5.0, 1.0, 1.0, 60.0 - cut_gap)
    put(5.22, 1.0, 1.0, 100.0)
    return np.array(pts, np.float32), np.array(dens, np.float64)


def _events(pos, dens, tol=1e-5, mode="cells"):
    l0, _ = oracle.fof(pos, dens, **KW)
    return oracle.events(pos, dens, l0, tol=tol, mode=mode, **KW), l0


@pytest.mark.parametrize("mode", ["brute", "cells"])
def test_each_event_on_its_bound(mode):
    """Each bound of orc_events, tol = 1e-5: the L0 cut within 6e-4 of 60, the
    floor within 2.5e-3 of 250.837, a denser neighbour within b and a second
    candidate of the group within 2e-5 relative."""
    pos, dens = _hand_case(peak_gap=1.5e-5, order_gap=1.5e-5, cut_gap=5e-4, floor_gap=2e-3)
    ev, l0 = _events(pos, dens, mode=mode)
    assert ev[0] & oracle.EV_L0CUT and ev[1] & oracle.EV_GROUP
    assert ev[2] & oracle.EV_FLOOR and ev[3] & oracle.EV_GROUP
    assert ev[4] & oracle.EV_PEAK and ev[5] & oracle.EV_PEAK
    assert ev[6] & oracle.EV_ORDER and ev[9] & oracle.EV_ORDER
    assert not ev[6] & oracle.EV_PEAK                      # J (100) is far below H
    assert np.all(ev[6:10] & oracle.EV_GROUP)
    assert l0[10] == 0 and ev[10] & oracle.EV_L0CUT and ev[11] & oracle.EV_GROUP
    # the same configuration just outside every bound: no event anywhere
    pos, dens = _hand_case(peak_gap=3e-5, order_gap=3e-5, cut_gap=7e-4, floor_gap=3e-3)
    ev, _ = _events(pos, dens, mode=mode)
    assert np.all(ev == 0), ev


def test_events_follow_the_tolerance():
    """The bounds scale with tol (here 10x)."""
    pos, dens = _hand_case(peak_gap=1.5e-4, order_gap=1.5e-4, cut_gap=5e-3, floor_gap=2e-2)
    assert np.all(_events(pos, dens, tol=1e-5)[0] == 0)
    ev, _ = _events(pos, dens, tol=1e-4)
    assert ev[0] & oracle.EV_L0CUT and ev[2] & oracle.EV_FLOOR and ev[4] & oracle.EV_PEAK
    assert ev[6] & oracle.EV_ORDER


def test_brute_equals_cells():
    pos, L, _ = synth.small_box(6000, seed=31, nmax=1500, pair_frac=0.3)
    d = oracle.density(pos, box=L)
    l0, _ = oracle.fof(pos, d, box=L)
    for tol in (1e-5, 1e-3):
        a = oracle.events(pos, d, l0, tol=tol, box=L)
        b = oracle.events(pos, d, l0, tol=tol, box=L, mode="brute")
        np.testing.assert_array_equal(a, b)


@pytest.mark.parametrize("seed,tol", [(41, 2e-3), (42, 1e-3), (43, 5e-4)])
def test_perturbed_field_changes_labels_only_at_events(seed, tol):
    """A field within tol * max(Delta, 1) of the oracle's FP64 densities (random
    signs and sizes up to the bound) changes L0 and halo labels only on particles
    that the events of the unperturbed field explain, and some labels do change
    at these tolerances (so the check is not empty)."""
    pos, L, _ = synth.small_box(20000, seed=seed, nmax=3000, pair_frac=0.4)
    d = oracle.density(pos, box=L)
    ref = oracle.find(pos, box=L, density_override=d)
    ev = oracle.events(pos, d, ref["l0"], tol=tol, box=L)
    rng = np.random.default_rng(seed)
    changed = 0
    for trial in range(4):
        u = rng.uniform(-1.0, 1.0, len(d))
        if trial == 0:
            u = np.sign(u)                       # the bound itself
        dp = d + u * tol * np.maximum(np.abs(d), 1.0)
        got = oracle.find(pos, box=L, density_override=dp)
        for key in ("l0", "halo_id"):
            frac, bad = matched_agreement(got[key], ref[key])
            ok = explained_mismatches(bad, got["l0"], ref["l0"], ev)
            assert ok.all(), (key, trial, bad[~ok][:10])
            changed += len(bad)
    assert changed > 0
