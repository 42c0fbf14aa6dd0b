"""GPU tests of the many-box call (hf_find_batch) and the request loop
(hf_server), through the C ABI.

Both run the single-box pass on several pipelines at once, so the bar is
identity: every box's density (bit for bit), L0 ids, halo ids and halo table
equal hf_find's on that box alone, whatever the lane count, the order in which
boxes run and what runs beside them.  Two boxes are also checked against the
oracle directly (labels bit-exact on the GPU densities, densities within
tolerance).
"""
from __future__ import annotations

import sys

import numpy as np
import pytest

import oracle
from paper_2110_11408_amd import synth
from tests.gpu_helpers import assert_same_labels, density_violations

pytestmark = pytest.mark.gpu

# (n, seed, nmax, halo_frac); n = 0 is an empty box of side 10.  The last box
# (3.2M particles, haloes up to 20000 particles) is of the size of the largest
# batched boxes and served requests: its largest L0 groups keep part of their
# acceptance histograms in global memory.
SPECS = [(3000, 201, 500, 0.5), (0, 0, 0, 0.0), (20000, 202, 3000, 0.6), (700, 203, 200, 0.4),
         (9001, 204, 1500, 0.5), (45000, 205, 6000, 0.3), (3200000, 206, 20000, 0.6)]
BIG = 6


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


def _boxes():
    out = []
    for n, seed, nmax, frac in SPECS:
        if n == 0:
            out.append((np.zeros((0, 3), np.float32), 10.0))
        else:
            pos, L, _ = synth.small_box(n, seed=seed, nmax=nmax, halo_frac=frac)
            out.append((pos, L))
    return out


@pytest.fixture(scope="module")
def ctx():
    oracle.build(force=False)
    from paper_2110_11408_amd.api import Context
    return Context(0)


@pytest.fixture(scope="module")
def boxes():
    return _boxes()


def _params(L, n):
    from paper_2110_11408_amd import _lib
    # an empty box has no mean density of its own
    return _lib.default_params(box=L, mean_density=0.0 if n else 1.0)


@pytest.fixture(scope="module")
def singles(ctx, boxes):
    import torch
    out = []
    for pos, L in boxes:
        if len(pos) == 0:
            out.append(None)
            continue
        _say(f"[gpu] hf_find single n={len(pos)} box={L:.3f}")
        r = ctx.find(torch.from_numpy(pos).cuda(), _params(L, len(pos)))
        out.append({k: (v.cpu().numpy() if hasattr(v, "cpu") else v) for k, v in r.items()})
    return out


def _run_batch(ctx, boxes, **kw):
    import torch
    pos = np.concatenate([b[0] for b in boxes]).astype(np.float32)
    offs = np.concatenate([[0], np.cumsum([len(b[0]) for b in boxes])])
    params = [_params(L, len(p)) for p, L in boxes]
    _say(f"[gpu] hf_find_batch boxes={len(boxes)} total={len(pos)} {kw}")
    out = ctx.find_batch(torch.from_numpy(pos).cuda(), offs, params, **kw)
    torch.cuda.synchronize()
    return offs, out


def _assert_box_equal(single, dens, l0, hid, table):
    np.testing.assert_array_equal(dens, single["density"])
    np.testing.assert_array_equal(l0, single["l0_id"])
    np.testing.assert_array_equal(hid, single["halo_id"])
    np.testing.assert_array_equal(np.asarray(table), single["halos"])


@pytest.mark.parametrize("lanes", [0, 1, 3, 16])
def test_batch_equals_single_calls(ctx, boxes, singles, lanes):
    offs, out = _run_batch(ctx, boxes, n_lanes=lanes)
    dens, l0, hid = (out[k].cpu().numpy() for k in ("density", "l0_id", "halo_id"))
    for b, single in enumerate(singles):
        a, e = offs[b], offs[b + 1]
        if single is None:
            assert e == a and out["n_halos"][b] == 0
            continue
        assert out["n_halos"][b] == single["n_halos"]
        _assert_box_equal(single, dens[a:e], l0[a:e], hid[a:e], out["halos"][b].cpu().numpy())


def test_batch_of_many_small_boxes(ctx):
    """Twenty-four boxes of 64 to 400 particles in one fused pass: wavefronts
    of the per-particle kernels span several box boundaries (the sparse-cell
    density lists such wavefronts for a kernel that reads each lane's own box
    constants).  Every box equals its single call."""
    import torch
    sizes = [150, 90, 400, 64, 200, 120, 80, 260] * 3
    small = []
    for k, n in enumerate(sizes):
        pos, L, _ = synth.small_box(n, seed=400 + k, nmax=80, halo_frac=0.5)
        small.append((pos, L))
    singles = []
    for pos, L in small:
        r = ctx.find(torch.from_numpy(pos).cuda(), _params(L, len(pos)))
        singles.append({k: (v.cpu().numpy() if hasattr(v, "cpu") else v) for k, v in r.items()})
    offs, out = _run_batch(ctx, small, n_lanes=1)
    dens, l0, hid = (out[k].cpu().numpy() for k in ("density", "l0_id", "halo_id"))
    for b, single in enumerate(singles):
        a, e = offs[b], offs[b + 1]
        assert out["n_halos"][b] == single["n_halos"]
        _assert_box_equal(single, dens[a:e], l0[a:e], hid[a:e], out["halos"][b].cpu().numpy())


def test_batch_matches_oracle(ctx, boxes):
    from paper_2110_11408_amd.api import halo_table
    offs, out = _run_batch(ctx, boxes)
    dens, l0, hid = (out[k].cpu().numpy() for k in ("density", "l0_id", "halo_id"))
    for b in (0, 4):
        pos, L = boxes[b]
        a, e = offs[b], offs[b + 1]
        ref = oracle.density(pos, box=L)
        assert len(density_violations(dens[a:e], ref)) == 0
        lab = oracle.find(pos, box=L, density_override=dens[a:e].astype(np.float64))
        g = {"l0": l0[a:e], "halo_id": hid[a:e], "n_halos": int(out["n_halos"][b]),
             "table": halo_table(out["halos"][b])}
        assert_same_labels(g, lab)


def test_batch_capacity_retry(ctx, boxes, singles):
    # every table starts with one row: the call reports the needed sizes and
    # the wrapper retries once
    offs, out = _run_batch(ctx, boxes, halos_caps=np.ones(len(boxes), np.int64))
    for b, single in enumerate(singles):
        if single is not None:
            np.testing.assert_array_equal(out["halos"][b].cpu().numpy(), single["halos"])


def test_batch_error_names_the_box(ctx, boxes):
    import torch
    from paper_2110_11408_amd import _lib
    from paper_2110_11408_amd._lib import HfError
    pos = np.concatenate([boxes[0][0], boxes[3][0]])
    offs = [0, len(boxes[0][0]), len(pos)]
    # second box: a side of 1 is less than three cells
    params = [_params(boxes[0][1], 1), _lib.default_params(box=1.0, mean_density=1.0)]
    with pytest.raises(HfError) as e:
        ctx.find_batch(torch.from_numpy(pos).cuda(), offs, params)
    assert e.value.status == _lib.HF_ERR_INVALID and "box 1" in str(e.value)


def _server_check(res, single):
    assert res["status"] == 0
    assert res["n_halos"] == single["n_halos"]
    np.testing.assert_array_equal(res["halo_id"].numpy(), single["halo_id"])
    np.testing.assert_array_equal(res["density"].numpy(), single["density"])
    np.testing.assert_array_equal(res["l0_id"].numpy(), single["l0_id"])
    np.testing.assert_array_equal(res["halos"].numpy(), single["halos"])
    assert res["t_submit"] <= res["t_start"] <= res["t_done"]


def test_server_mix_equals_single_calls(boxes, singles):
    from paper_2110_11408_amd.api import Server
    srv = Server(0, slots=3, budget_bytes=8 << 30)
    try:
        # repeats share the device with others; the 3.2M box runs beside small ones
        order = [0, 2, BIG, 3, 4, 5, 0, 5, BIG, 4, 3, 2]
        tickets = []
        for b in order:
            pos, L = boxes[b]
            _say(f"[gpu] server submit box={b} n={len(pos)}")
            tickets.append((b, srv.submit(Server.pinned_positions(pos), _params(L, len(pos)),
                                          want_density=True, want_l0=True)))
        slots = set()
        for b, t in tickets:
            res = srv.wait(t)
            _server_check(res, singles[b])
            slots.add(res["slot"])
        assert len(slots) > 1
        assert srv.held_bytes() <= 8 << 30
    finally:
        srv.close()


def test_server_budget_admission(boxes, singles):
    from paper_2110_11408_amd import _lib
    from paper_2110_11408_amd.api import Server
    from paper_2110_11408_amd._lib import HfError
    big = 5
    pos, L = boxes[big]
    one = Server(0, slots=1, budget_bytes=8 << 30)
    try:
        _server_check(one.wait(one.submit(pos, _params(L, len(pos)), want_density=True,
                                          want_l0=True)), singles[big])
        need = one.held_bytes()
    finally:
        one.close()
    # room for about one large request at a time: the others wait for memory
    budget = int(need * 1.3)
    srv = Server(0, slots=4, budget_bytes=budget)
    try:
        tickets = [(b, srv.submit(boxes[b][0], _params(boxes[b][1], len(boxes[b][0])),
                                  want_density=True, want_l0=True)) for b in (5, 2, 5, 0, 4, 5)]
        for b, t in tickets:
            _server_check(srv.wait(t), singles[b])
        assert srv.held_bytes() <= budget
        # a request larger than the whole budget is refused at submission
        huge = synth.small_box(200000, seed=9, nmax=2000)[0]
        with pytest.raises(HfError) as e:
            srv.submit(huge, _params(float(200000) ** (1 / 3), 200000))
        assert e.value.status == _lib.HF_ERR_NOMEM
    finally:
        srv.close()


def test_server_error_stays_with_its_request(boxes, singles):
    from paper_2110_11408_amd import _lib
    from paper_2110_11408_amd.api import Server
    srv = Server(0, slots=2, budget_bytes=4 << 30)
    try:
        pos, L = boxes[2]
        bad = pos.copy()
        bad[17, 1] = L * 1.5    # outside the box: rejected by the binning's range check
        t0 = srv.submit(boxes[0][0], _params(boxes[0][1], 3000), want_density=True, want_l0=True)
        t1 = srv.submit(bad, _params(L, len(pos)))
        t2 = srv.submit(pos, _params(L, len(pos)), want_density=True, want_l0=True)
        _server_check(srv.wait(t0), singles[0])
        r1 = srv.wait(t1, check=False)
        assert r1["status"] == _lib.HF_ERR_INVALID and "box" in r1["error"]
        _server_check(srv.wait(t2), singles[2])
    finally:
        srv.close()


def test_tune_batch_table_roundtrip(ctx, boxes, singles, tmp_path):
    import torch
    from paper_2110_11408_amd.api import Context
    sub = boxes[:BIG]
    pos = np.concatenate([b[0] for b in sub]).astype(np.float32)
    offs = np.concatenate([[0], np.cumsum([len(b[0]) for b in sub])])
    params = [_params(L, len(p)) for p, L in sub]
    total = int(offs[-1])
    table = tmp_path / "tune.txt"
    _say(f"[gpu] hf_tune_batch boxes={len(sub)} total={total}")
    best, ms, out = ctx.tune_batch(torch.from_numpy(pos).cuda(), offs, params, max_groups=3, reps=1,
                                   table_path=str(table))
    assert 1 <= best <= 3 and ms > 0.0
    dens, l0, hid = (out[k].cpu().numpy() for k in ("density", "l0_id", "halo_id"))
    for b, single in enumerate(singles[:BIG]):
        a, e = offs[b], offs[b + 1]
        if single is not None:
            _assert_box_equal(single, dens[a:e], l0[a:e], hid[a:e], out["halos"][b].cpu().numpy())
    lines = [ln for ln in table.read_text().splitlines() if ln.startswith("hf-tune v1 ")]
    assert len(lines) == 1
    assert f" n_boxes={len(sub)} total={total} groups={best} " in lines[0]
    # the tuned count serves batches of the same box count and a total within 25 %
    assert ctx.batch_groups(len(sub), total) == best
    assert ctx.batch_groups(len(sub), int(total * 1.2)) == best
    assert ctx.batch_groups(len(sub), total * 2) == 1
    assert ctx.batch_groups(len(sub) + 1, total) == 1
    assert ctx.batch_groups(len(sub), total, n_lanes=2) == 2
    # tuning again rewrites the shape's line instead of adding one; lines of
    # another architecture and comments are skipped on loading
    ctx.tune_batch(torch.from_numpy(pos).cuda(), offs, params, max_groups=2, reps=1, table_path=str(table))
    with open(table, "a") as f:
        f.write(f"hf-tune v1 gfx000 n_boxes={len(sub)} total={total} groups=4 ms=1.000\n# note\n")
    assert sum(ln.startswith("hf-tune v1 ") and "gfx000" not in ln
               for ln in table.read_text().splitlines()) == 1
    fresh = Context(0)
    assert fresh.batch_groups(len(sub), total) == 1
    assert fresh.load_tuning(str(table)) == 1
    tuned = ctx.batch_groups(len(sub), total)
    assert fresh.batch_groups(len(sub), total) == tuned
    offs2, out2 = _run_batch(fresh, sub)
    np.testing.assert_array_equal(out2["halo_id"].cpu().numpy(), hid)
    np.testing.assert_array_equal(out2["density"].cpu().numpy(), dens)
