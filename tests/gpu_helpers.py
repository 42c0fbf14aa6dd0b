"""Helpers for the GPU parity tests: run the HIP path through the C ABI and
compare it with the oracle."""
from __future__ import annotations

import numpy as np

DENS_REL = 1e-5   # |D_gpu - D_64| <= 1e-5 * max(D_64, 1)  (mean-density units)


def gpu_find(ctx, pos, **kw):
    import torch
    from paper_2110_11408_amd import _lib
    from paper_2110_11408_amd.api import halo_table
    p = _lib.default_params(**kw)
    t = torch.from_numpy(np.ascontiguousarray(pos)).cuda()
    out = ctx.find(t, p)
    torch.cuda.synchronize()
    res = {"density": out["density"].cpu().numpy(), "l0": out["l0_id"].cpu().numpy(),
           "halo_id": out["halo_id"].cpu().numpy(), "n_halos": out["n_halos"],
           "table": halo_table(out["halos"]), "stats": ctx.stats()}
    return res


def density_violations(d_gpu, d_ref):
    tol = DENS_REL * np.maximum(np.abs(d_ref), 1.0)
    return np.nonzero(np.abs(d_gpu.astype(np.float64) - d_ref) > tol)[0]


def assert_same_labels(gpu, ref):
    """Bit-exact L0 labels, halo labels and halo table."""
    np.testing.assert_array_equal(gpu["l0"], ref["l0"])
    np.testing.assert_array_equal(gpu["halo_id"], ref["halo_id"])
    assert gpu["n_halos"] == ref["n_halos"]
    t, r = gpu["table"], ref["table"]
    np.testing.assert_array_equal(t["id"], r["id"])
    np.testing.assert_array_equal(t["nucleus"], r["nucleus"])
    np.testing.assert_array_equal(t["l0_id"], r["l0"])
    np.testing.assert_array_equal(t["n"], r["n"])
    np.testing.assert_array_equal(t["n_enclosed"], r["ienc"])


def label_mapping(lab_a, lab_b):
    """Each label of a mapped to the label of b it shares most particles with
    (0 maps to 0)."""
    n = len(lab_a)
    mapping = {0: 0}
    order = np.lexsort((lab_b, lab_a))
    a_s, b_s = lab_a[order], lab_b[order]
    starts = np.flatnonzero(np.r_[True, a_s[1:] != a_s[:-1]])
    ends = np.r_[starts[1:], n]
    for s, e in zip(starts, ends):
        la = int(a_s[s])
        if la == 0:
            continue
        vals, cnt = np.unique(b_s[s:e], return_counts=True)
        mapping[la] = int(vals[np.argmax(cnt)])
    return mapping


def _apply(mapping, lab):
    keys = np.fromiter(mapping.keys(), np.int64, len(mapping))
    vals = np.fromiter(mapping.values(), np.int64, len(mapping))
    order = np.argsort(keys)
    keys, vals = keys[order], vals[order]
    idx = np.searchsorted(keys, lab)
    return vals[idx]


def matched_agreement(lab_a, lab_b):
    """Fraction of particles whose label in a maps to their label in b, where each
    label of a is mapped to the label of b it shares most particles with (0 maps
    to 0).  Returns (fraction, mismatched particle indices)."""
    n = len(lab_a)
    mapped = _apply(label_mapping(lab_a, lab_b), lab_a)
    bad = np.nonzero(mapped != lab_b)[0]
    return 1.0 - len(bad) / max(n, 1), bad


def explained_mismatches(bad, l0_other, l0_ref, ev):
    """For each mismatched particle q (indices ``bad``) whether the oracle's
    near-threshold events ``ev`` (computed on the reference field, whose L0
    labels are ``l0_ref``) explain it: q itself sits at the L0 cut, or its
    reference L0 group is touched by an event, or the other side's L0 group of
    q maps to such a group."""
    import oracle
    bad = np.asarray(bad, dtype=np.int64)
    flagged = np.unique(l0_ref[(ev & oracle.EV_GROUP) != 0])
    flagged = flagged[flagged > 0]
    mapped = _apply(label_mapping(l0_other, l0_ref), l0_other[bad])
    return (((ev[bad] & oracle.EV_L0CUT) != 0) | np.isin(l0_ref[bad], flagged) |
            np.isin(mapped, flagged))
