"""GPU parity of hf_halo_stats (level 2 inside L1 halos and the Table 1
position statistics) against the oracle, through the C ABI.

The oracle runs on the GPU's own densities and L1 labels, so every decision
(candidates, acceptance, assignment at level 2) is taken on the same inputs:
counts, ids, the first L2 nucleus, the member lists and the centres of mass
(fixed-point sums, identical arithmetic) must agree exactly, and so must the
radii and circular velocities (float32 results of the same FP64 expressions).
"""
from __future__ import annotations

import sys

import numpy as np
import pytest

import oracle
from paper_2110_11408_amd import synth

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def ctx():
    oracle.build(force=False)
    from paper_2110_11408_amd.api import Context
    return Context(0)


def _three_halo_case():
    """A main halo with two embedded subhaloes (several L2 halos per L1 halo)."""
    rng = np.random.default_rng(5)
    L = 40.0
    bg = rng.random((int(L ** 3), 3)) * L
    centre = np.array([L / 2, L / 2, L / 2])
    mu = lambda y: np.log1p(y) - y / (1 + y)            # noqa: E731
    x = np.linspace(0.0, 1.0, 200001)
    parts = []
    r200m = float(synth.r200(30000, 1.0))
    for n, c, off in ((30000, 8.0, (0.0, 0.0, 0.0)), (4000, 3.0, (0.55, 0.0, 0.0)),
                      (1500, 30.0, (-0.5, 0.2, 0.0))):
        r200 = float(synth.r200(n, 1.0))
        radii = np.interp(rng.random(n), mu(c * x) / mu(c), x) * r200
        v = rng.standard_normal((n, 3))
        v /= np.linalg.norm(v, axis=1, keepdims=True)
        parts.append(centre + np.array(off) * r200m + radii[:, None] * v)
    pos = np.mod(np.concatenate([bg] + parts), L).astype(np.float32)
    pos[pos >= np.float32(L)] = 0.0
    return pos, L


def _case(name):
    if name == "three":
        return _three_halo_case()
    if name == "plain64":
        pos, L, _ = synth.named_box("plain64")
        return pos, L
    n, seed, nmax, pf = {"s3000": (3000, 101, 500, 0.3), "s9001": (9001, 102, 1500, 0.3),
                         "s40123": (40123, 103, 5000, 0.2)}[name]
    pos, L, _ = synth.small_box(n, seed=seed, nmax=nmax, pair_frac=pf)
    return pos, L


def _run(ctx, pos, L):
    import torch
    from paper_2110_11408_amd import _lib
    p = _lib.default_params(box=L, mean_density=1.0)
    t = torch.from_numpy(pos).cuda()
    f = ctx.find(t, p)
    st = ctx.halo_stats(t, f["density"], f["halo_id"], p, f["n_halos"])
    torch.cuda.synchronize()
    dens = f["density"].cpu().numpy().astype(np.float64)
    hid = f["halo_id"].cpu().numpy()
    ref = oracle.l2_stats(pos, dens, hid, box=L, mean_density=1.0)
    return st, ref, hid


@pytest.mark.parametrize("name", ["s3000", "s9001", "s40123", "plain64", "three"])
def test_halo_stats_match_oracle(ctx, name):
    pos, L = _case(name)
    _say(f"[gpu] hf_halo_stats case={name} n={len(pos)}")
    st, ref, hid = _run(ctx, pos, L)
    assert len(st["id"]) == len(ref["id"]) > 0
    for k in ("id", "n", "n_l2", "l2max_nucleus", "l2max_n"):
        np.testing.assert_array_equal(st[k], ref[k], err_msg=k)
    for k in ("x_com", "x_l2com", "l2_mass", "r_pct", "vcirc_max", "rvcirc_max"):
        np.testing.assert_array_equal(st[k], ref[k].astype(np.float32), err_msg=k)
    np.testing.assert_array_equal(st["group_start"].cpu().numpy(), ref["gstart"])
    np.testing.assert_array_equal(st["members"].cpu().numpy(), ref["members"])
    if name == "three":
        assert st["n_l2"].max() >= 3


def test_halo_stats_argument_errors(ctx):
    import torch
    from paper_2110_11408_amd import _lib
    from paper_2110_11408_amd._lib import HfError
    pos, L = _case("s3000")
    p = _lib.default_params(box=L, mean_density=1.0)
    t = torch.from_numpy(pos).cuda()
    f = ctx.find(t, p)
    with pytest.raises(HfError) as e:
        ctx.halo_stats(t, f["density"], f["halo_id"], p, f["n_halos"] + 1)
    assert e.value.status == _lib.HF_ERR_INVALID
    # no labelled particle: no halo, nothing to do
    zero = torch.zeros_like(f["halo_id"])
    out = ctx.halo_stats(t, f["density"], zero, p, 0)
    assert len(out["id"]) == 0


def test_halo_stats_full_size_256_sampled(ctx):
    """The 256^3 box: every halo's level 2 and statistics depend on its own
    members only, so the oracle run on a labelling restricted to 200 halos (the
    20 largest and 180 random ones) must reproduce their rows exactly."""
    import torch
    from paper_2110_11408_amd import _lib
    pos, L, _ = synth.named_box("plain256")
    _say(f"[gpu] hf_halo_stats full size n={len(pos)}")
    p = _lib.default_params(box=L)
    t = torch.from_numpy(pos).cuda()
    f = ctx.find(t, p, halos_cap=len(pos) // 64)
    st = ctx.halo_stats(t, f["density"], f["halo_id"], p, f["n_halos"], want_members=False)
    hid = f["halo_id"].cpu().numpy()
    dens = f["density"].cpu().numpy().astype(np.float64)
    del t, f
    torch.cuda.empty_cache()
    rng = np.random.default_rng(256)
    nh = len(st["id"])
    pick = np.union1d(np.argsort(-st["n"], kind="stable")[:20], rng.choice(nh, 180, replace=False))
    keep = np.isin(hid, st["id"][pick])
    ref = oracle.l2_stats(pos, dens, np.where(keep, hid, 0), box=L)
    np.testing.assert_array_equal(ref["id"], st["id"][pick])
    for k in ("n", "n_l2", "l2max_nucleus", "l2max_n"):
        np.testing.assert_array_equal(st[k][pick], ref[k], err_msg=k)
    for k in ("x_com", "x_l2com", "l2_mass", "r_pct", "vcirc_max", "rvcirc_max"):
        np.testing.assert_array_equal(st[k][pick], ref[k].astype(np.float32), err_msg=k)
