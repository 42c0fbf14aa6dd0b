"""Checks of a CompaSO result against properties the paper states (Sec. 2.2.2).

These are written from the statements of the method, not from the oracle's
code: they re-derive nothing by the oracle's route (no sorted-crossing search,
no cubed predicates) and use plain FP64 geometry with a small tolerance so that
only genuine violations (not last-bit rounding at exact boundaries) fail.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.spatial import cKDTree

REL = 1e-9


def min_image(d, L):
    return d - L * np.round(d / L)


def dist(pos, i, js, L):
    d = min_image(pos[js].astype(np.float64) - pos[i].astype(np.float64), L)
    return np.sqrt(np.sum(d * d, axis=1))


def denser(dens, a, b):
    return dens[a] > dens[b] or (dens[a] == dens[b] and a < b)


def check_compaso(pos, L, dens, l0, found, owner_all, *, nbar, b, delta_l1, alpha, c_roche,
                  floor, max_groups=None):
    """Assert the CompaSO invariants group by group.

    found: dict of arrays nucleus, ienc, count, l0 (creation order inside groups).
    owner_all: per particle, 1 + nucleus index of its halo (0 = none), before the cut.
    """
    K = 4.0 * math.pi / 3.0 * delta_l1 * nbar
    labels = np.unique(l0[l0 > 0])
    if max_groups is not None:
        labels = labels[:max_groups]
    tree = cKDTree(np.mod(pos.astype(np.float64), L), boxsize=L)
    fl0 = np.asarray(found["l0"])
    checked = 0
    for lab in labels:
        mem = np.nonzero(l0 == lab)[0]
        sel = np.nonzero(fl0 == lab)[0]
        nucs = np.asarray(found["nucleus"])[sel]
        ienc = np.asarray(found["ienc"])[sel]
        cnt = np.asarray(found["count"])[sel]
        m = len(mem)
        R = (ienc / K) ** (1.0 / 3.0)
        dmat = np.stack([dist(pos, int(c), mem, L) for c in nucs]) if len(nucs) else np.zeros((0, m))
        # nuclei: descending density, above the floor, local peaks within b
        for k, c in enumerate(nucs):
            assert dens[c] >= floor, (lab, c)
            if k:
                assert denser(dens, nucs[k - 1], c), ("order", lab, k)
            nb = tree.query_ball_point(pos[c].astype(np.float64) % L, b * (1 + REL))
            for j in nb:
                if j != c and l0[j] == lab and dist(pos, c, [j], L)[0] < b * (1 - REL):
                    assert not denser(dens, j, c), ("peak", lab, c, j)
            # not inside alpha R of an earlier nucleus
            for h in range(k):
                dch = dmat[h][np.searchsorted(mem, c)]
                assert dch >= alpha * R[h] * (1 - REL), ("eligibility", lab, c, nucs[h])
        # R: exactly ienc particles inside, enclosed density >= delta_l1 up to R
        for h in range(len(nucs)):
            dd = np.sort(dmat[h])
            assert np.sum(dd < R[h] * (1 - REL)) <= ienc[h] <= np.sum(dd < R[h] * (1 + REL)), \
                ("R count", lab, h)
            k = np.arange(1, min(ienc[h], m))
            assert np.all(K * dd[k] ** 3 <= k * (1 + REL)), ("innermost", lab, h)
            if ienc[h] < m:
                assert K * dd[ienc[h]] ** 3 >= ienc[h] * (1 - REL), ("crossing", lab, h)
        # completeness: every peak above the floor that is outside alpha R of all
        # denser nuclei is itself a nucleus
        cand = mem[dens[mem] >= floor]
        nucset = set(int(x) for x in nucs)
        for q in cand:
            if int(q) in nucset:
                continue
            nb = tree.query_ball_point(pos[q].astype(np.float64) % L, b * (1 + REL))
            is_peak = True
            for j in nb:
                if j != q and l0[j] == lab and dist(pos, q, [j], L)[0] < b * (1 - REL) \
                        and denser(dens, j, q):
                    is_peak = False
                    break
            if not is_peak:
                continue
            tq = np.searchsorted(mem, q)
            covered = any(denser(dens, nucs[h], q) and dmat[h][tq] < alpha * R[h] * (1 + REL)
                          for h in range(len(nucs)))
            assert covered, ("missed nucleus", lab, q)
        # assignment (step 3): fold over the spheres containing the particle in
        # creation order with the model enclosed density Delta_L1 R^2 / r^2
        # (Sec. 2.3.2): join if unassigned, move if the new value is at least
        # c_Roche times the current one.  Particles whose decision sits within
        # rounding of a boundary are skipped.
        own = owner_all[mem]
        for t in range(m):
            cur = -1
            ambiguous = False
            for h in range(len(nucs)):
                x = dmat[h][t]
                if abs(x - R[h]) <= REL * R[h]:
                    ambiguous = True
                    break
                if x >= R[h]:
                    continue
                if cur < 0:
                    cur = h
                    continue
                if x == 0.0:
                    cur = h
                    continue
                d_own = dmat[cur][t]
                ratio = (R[h] ** 2 / x ** 2) * (d_own ** 2 / R[cur] ** 2)
                if abs(ratio - c_roche) <= 1e-9 * max(c_roche, 1.0):
                    ambiguous = True
                    break
                if ratio >= c_roche:
                    cur = h
            if ambiguous:
                continue
            want = 0 if cur < 0 else int(nucs[cur]) + 1
            assert own[t] == want, ("assignment", lab, mem[t], own[t], want)
        for h, c in enumerate(nucs):
            assert cnt[h] == np.sum(own == int(c) + 1), ("count", lab, h)
        checked += 1
    return checked
