"""GPU tests of the threshold-radius search by radial bins (Sec. 2.3.4;
HF_OPT_RADIUS_SEARCH = HF_RADIUS_BINS) and of the members in group order
(Sec. 2.3.5; hf_find_grouped), through the C ABI.

Bars: the radial-bin search gives the same enclosed count as the default
whole-group histogram, so every output of hf_find is identical in both modes,
and the labels are bit-exact against the oracle run with its own radial-bin
search on the GPU densities.  The group order is compared element by element
with the oracle's definition (rows in table order, ascending original index,
then the particles of no halo).  Cases: boxes of 40k (many 256-thread tiles,
ragged tails), 262k (the small benchmark box) and 3.2M particles (haloes of up
to 20000 particles: groups run by 1024-thread workgroups and searched bins
whose histograms spill to global memory), an empty input and a box without
haloes.
"""
from __future__ import annotations

import sys

import numpy as np
import pytest

import oracle
from paper_2110_11408_amd import synth
from tests.gpu_helpers import assert_same_labels

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


def _case(name):
    if name == "plain64":
        return synth.named_box("plain64")[:2]
    n, seed, nmax, pf = {"s40123": (40123, 103, 5000, 0.2), "big3m": (3200000, 206, 20000, 0.2)}[name]
    return synth.small_box(n, seed=seed, nmax=nmax, pair_frac=pf, halo_frac=0.6)[:2]


@pytest.fixture(scope="module")
def ctxs():
    oracle.build(force=False)
    from paper_2110_11408_amd.api import Context
    hist, bins = Context(0), Context(0)
    bins.set_radius_search("bins")
    assert hist.radius_search() == "histogram" and bins.radius_search() == "bins"
    return hist, bins


def _np(out):
    from paper_2110_11408_amd.api import halo_table
    return {"density": out["density"].cpu().numpy(), "l0": out["l0_id"].cpu().numpy(),
            "halo_id": out["halo_id"].cpu().numpy(), "n_halos": out["n_halos"],
            "table": halo_table(out["halos"]), "raw": out["halos"].cpu().numpy()}


@pytest.fixture(scope="module")
def runs(ctxs):
    import torch
    from paper_2110_11408_amd import _lib
    hist, bins = ctxs
    out = {}
    for name in ("s40123", "plain64", "big3m"):
        pos, L = _case(name)
        p = _lib.default_params(box=L)
        t = torch.from_numpy(np.ascontiguousarray(pos)).cuda()
        _say(f"[gpu] hf_find histogram case={name} n={len(pos)}")
        a = _np(hist.find(t, p))
        _say(f"[gpu] hf_find radial bins case={name} n={len(pos)}")
        b = bins.find(t, p)
        torch.cuda.synchronize()
        st = bins.stats()
        _say(f"[gpu] hf_find_grouped case={name} n={len(pos)}")
        gr = hist.find_grouped(t, p)
        torch.cuda.synchronize()
        out[name] = (pos, L, a, _np(b), st, {"members": gr["members"].cpu().numpy(),
                                            "halo_start": gr["halo_start"].cpu().numpy(),
                                            "halo_id": gr["halo_id"].cpu().numpy(),
                                            "n_halos": gr["n_halos"], "raw": gr["halos"].cpu().numpy()})
    return out


@pytest.mark.parametrize("name", ["s40123", "plain64", "big3m"])
def test_radial_bins_identical_to_histogram(runs, name):
    pos, L, a, b, st, _ = runs[name]
    assert a["n_halos"] > 0 and a["n_halos"] == b["n_halos"]
    for k in ("density", "l0", "halo_id", "raw"):
        np.testing.assert_array_equal(a[k], b[k], err_msg=k)
    if name == "big3m":
        # the case reaches the 1024-thread path: an L0 group above 12288 members
        assert np.bincount(a["l0"]).astype(np.int64)[1:].max() > 12288


def test_radial_bins_bit_exact_against_oracle(runs):
    pos, L, a, b, _, _ = runs["s40123"]
    ref = oracle.find(pos, box=L, density_override=b["density"].astype(np.float64), radius="bins")
    assert_same_labels(b, ref)


@pytest.mark.parametrize("name", ["s40123", "plain64", "big3m"])
def test_group_order_matches_definition(runs, name):
    pos, L, a, _, _, g = runs[name]
    # the grouped call's own labels are hf_find's
    np.testing.assert_array_equal(g["halo_id"], a["halo_id"])
    np.testing.assert_array_equal(g["raw"], a["raw"])
    members, start = oracle.group_order(g["halo_id"], a["table"]["id"])
    np.testing.assert_array_equal(g["halo_start"], start)
    np.testing.assert_array_equal(g["members"], members)
    np.testing.assert_array_equal(np.diff(start), a["table"]["n"])


def test_group_order_edge_cases(ctxs):
    import torch
    from paper_2110_11408_amd import _lib
    hist, _ = ctxs
    # a box without haloes (uniform, far below the L0 threshold): one run of
    # every particle in order
    rng = np.random.default_rng(5)
    L = 20.0
    pos = (rng.random((8000, 3)) * L).astype(np.float32)
    _say("[gpu] hf_find_grouped uniform box n=8000")
    g = hist.find_grouped(torch.from_numpy(pos).cuda(), _lib.default_params(box=L))
    torch.cuda.synchronize()
    assert g["n_halos"] == 0
    np.testing.assert_array_equal(g["halo_start"].cpu().numpy(), [0])
    np.testing.assert_array_equal(g["members"].cpu().numpy(), np.arange(8000))
    # empty input
    _say("[gpu] hf_find_grouped empty input")
    e = hist.find_grouped(torch.zeros((0, 3), dtype=torch.float32, device="cuda"),
                          _lib.default_params(box=10.0, mean_density=1.0), halos_cap=4)
    torch.cuda.synchronize()
    assert e["n_halos"] == 0
    np.testing.assert_array_equal(e["halo_start"].cpu().numpy(), [0])


def test_radial_bins_in_a_batch(ctxs):
    import torch
    from paper_2110_11408_amd import _lib
    hist, bins = ctxs
    boxes = [synth.small_box(n, seed=s, nmax=nm)[:2] for n, s, nm in
             [(20000, 301, 3000), (700, 302, 200), (45000, 303, 6000)]]
    pos = np.concatenate([b[0] for b in boxes]).astype(np.float32)
    offs = np.concatenate([[0], np.cumsum([len(b[0]) for b in boxes])])
    params = [_lib.default_params(box=L) for _, L in boxes]
    t = torch.from_numpy(pos).cuda()
    _say("[gpu] hf_find_batch histogram / radial bins, 3 boxes")
    a = hist.find_batch(t, offs, params, n_lanes=2)
    b = bins.find_batch(t, offs, params, n_lanes=2)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(a["n_halos"], b["n_halos"])
    np.testing.assert_array_equal(a["halo_id"].cpu().numpy(), b["halo_id"].cpu().numpy())
    for x, y in zip(a["halos"], b["halos"]):
        np.testing.assert_array_equal(x.cpu().numpy(), y.cpu().numpy())


def test_option_rejects_unknown_values(ctxs):
    from paper_2110_11408_amd import _lib
    from paper_2110_11408_amd._lib import HfError
    hist, _ = ctxs
    assert hist.lib.hf_set_option(hist.h, _lib.HF_OPT_RADIUS_SEARCH, 7) == _lib.HF_ERR_INVALID
    assert hist.lib.hf_set_option(hist.h, 99, 0) == _lib.HF_ERR_INVALID
    with pytest.raises(KeyError):
        hist.set_radius_search("sorted")
    assert hist.radius_search() == "histogram"
    with pytest.raises(HfError):
        hist._raise(hist.lib.hf_set_option(hist.h, 99, 0))
