"""GPU test of hf_find_noalloc through the C ABI: its outputs equal hf_find's
on the same box, bit for bit, on two calls in a row (the second on a smaller
box, so the static scratch holds the first call's contents when it starts),
and a box needing more scratch than the static array holds is refused."""
from __future__ import annotations

import sys

import numpy as np
import pytest

from paper_2110_11408_amd import synth

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


def _noalloc(ctx, pos_d, p, cap):
    import torch
    from paper_2110_11408_amd._lib import HALO_WORDS
    n = pos_d.shape[0]
    dens = torch.empty(n, dtype=torch.float32, device=pos_d.device)
    l0 = torch.empty(n, dtype=torch.int32, device=pos_d.device)
    hid = torch.empty(n, dtype=torch.int32, device=pos_d.device)
    halos = torch.empty((cap, HALO_WORDS), dtype=torch.int32, device=pos_d.device)
    nh = ctx.find_noalloc(pos_d, p, hid, halos, density=dens, l0_id=l0)
    torch.cuda.synchronize()
    return {"density": dens.cpu().numpy(), "l0_id": l0.cpu().numpy(), "halo_id": hid.cpu().numpy(),
            "n_halos": nh, "halos": halos[:nh].cpu().numpy()}


def test_noalloc_equals_find_on_two_calls():
    import torch
    from paper_2110_11408_amd import _lib
    from paper_2110_11408_amd.api import Context
    ctx = Context(0)
    for n, seed in ((262144, 61), (40123, 62)):
        pos, L, _ = synth.small_box(n, seed=seed, nmax=5000, pair_frac=0.3)
        p = _lib.default_params(box=L)
        t = torch.from_numpy(pos).cuda()
        _say(f"[gpu] hf_find_noalloc n={n}")
        got = _noalloc(ctx, t, p, cap=max(64, n // 32))
        ref = ctx.find(t, p)
        torch.cuda.synchronize()
        np.testing.assert_array_equal(got["density"], ref["density"].cpu().numpy())
        np.testing.assert_array_equal(got["l0_id"], ref["l0_id"].cpu().numpy())
        np.testing.assert_array_equal(got["halo_id"], ref["halo_id"].cpu().numpy())
        assert got["n_halos"] == ref["n_halos"] > 0
        np.testing.assert_array_equal(got["halos"], ref["halos"].cpu().numpy())
    ctx.close()


def test_noalloc_refuses_boxes_beyond_the_scratch():
    import torch
    from paper_2110_11408_amd import _lib
    from paper_2110_11408_amd._lib import HfError
    from paper_2110_11408_amd.api import Context
    ctx = Context(0)
    n = 1_500_000
    pos, L, _ = synth.small_box(n, seed=63, nmax=3000)
    t = torch.from_numpy(pos).cuda()
    _say(f"[gpu] hf_find_noalloc over the limit n={n}")
    with pytest.raises(HfError) as e:
        _noalloc(ctx, t, _lib.default_params(box=L), cap=1024)
    assert e.value.status == _lib.HF_ERR_INVALID and "static scratch" in str(e.value)
    ctx.close()
