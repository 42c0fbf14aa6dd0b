"""CompaSO oracle: plain FP64 CPU reference.  TEST INFRASTRUCTURE ONLY.

Only the test suite, the package smoke check and the benchmark's CPU-baseline
leg may import this package.  The product path (the HIP library and its Python
binding) never imports it and shares no code with it.

The arithmetic lives in ``compaso_oracle.c`` (FP64, OpenMP over particles and
L0 groups, brute-force and cell-list neighbour modes); this module only marshals
arguments.  Each C function cites the passage of the paper (Hadzhiyska et al.,
CompaSO) that it follows.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "compaso_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

# Paper defaults (Table 1 and Sec. 2.2; Einstein-de Sitter thresholds 60/200).
DEFAULTS = {
    "box": 1.0,
    "mean_density": 0.0,      # <= 0: N / box^3
    "b_kernel": 0.4,          # DensityKernelRad, units of l_mean
    "l_fof": 0.25,            # FoFLinkingLength, units of l_mean
    "delta_l0_min": 60.0,     # L0DensityThreshold
    "delta_l1": 200.0,        # SODensityL1
    "alpha_elig": 0.8,        # SO_alpha_eligible
    "c_roche": 2.0,           # SO_RocheCoeff
    "n_new_min": 35.0,        # SO_NPForMinDensity
    "particle_mass": 1.0,
    "n_l1_min": 35,           # MinL1HaloNP
    "self_count": 0,          # include W(0) = 1 for the particle itself
    "delta_l2": 800.0,        # SODensityL2
}
_ORDER = ["box", "mean_density", "b_kernel", "l_fof", "delta_l0_min", "delta_l1",
          "alpha_elig", "c_roche", "n_new_min", "particle_mass", "n_l1_min", "self_count",
          "delta_l2"]
PCT = [10, 25, 33, 50, 67, 75, 90, 95, 98]   # the r_XX percentiles of l2_stats
DERIVED = ["nbar", "b", "l", "b2", "l2", "norm", "K", "K2", "floor", "A6", "C3"]


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (FP64, no contraction, OpenMP)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
                               "-std=gnu11", "-Wall", "-shared", "-fPIC", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
            build(force=True)
        lib = ctypes.CDLL(_LIB_PATH)
        P = ctypes.c_void_p
        I64 = ctypes.c_int64
        lib.orc_derive.argtypes = [P, I64, P]
        lib.orc_density.argtypes = [I64, P, P, ctypes.c_int, P]
        lib.orc_density_sample.argtypes = [I64, P, P, I64, P, P]
        lib.orc_fof.argtypes = [I64, P, P, P, ctypes.c_int, P, P]
        lib.orc_compaso.argtypes = [I64, P, P, P, P, ctypes.c_int, P, P, I64,
                                    P, P, P, P, P, P, P, I64, P, P, P, P]
        lib.orc_params_at_redshift.argtypes = [P, ctypes.c_double, ctypes.c_double, P]
        lib.orc_l2_stats.argtypes = [I64, P, P, P, P, ctypes.c_int, I64, P, P, P, I64, P, P, P, P, P]
        lib.orc_events.argtypes = [I64, P, P, P, P, ctypes.c_int, ctypes.c_double, P]
        lib.orc_radius_search.argtypes = [P, I64, ctypes.c_double, ctypes.c_int, ctypes.c_double, P]
        lib.orc_radius_search.restype = I64
        lib.orc_group_sweep.argtypes = [I64, P, I64, P, P, P, P]
        lib.orc_num_threads.restype = ctypes.c_int
        lib.orc_set_threads.argtypes = [ctypes.c_int]
        _lib = lib
    return _lib


def params_vector(**kw) -> np.ndarray:
    p = dict(DEFAULTS)
    for k, v in kw.items():
        if k not in p:
            raise KeyError(k)
        p[k] = v
    return np.array([float(p[k]) for k in _ORDER], dtype=np.float64)


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p) if a is not None else None


def _pos(pos):
    pos = np.ascontiguousarray(pos, dtype=np.float32)
    assert pos.ndim == 2 and pos.shape[1] == 3
    return pos


def derive(n: int, **kw) -> dict:
    """Derived constants (Sec. 2.2, App. B.2): see orc_derive."""
    p = params_vector(**kw)
    out = np.zeros(len(DERIVED), np.float64)
    if _load().orc_derive(_ptr(p), int(n), _ptr(out)) != 0:
        raise ValueError("invalid parameters")
    return dict(zip(DERIVED, out.tolist()))


def set_threads(k: int) -> None:
    _load().orc_set_threads(int(k))


def num_threads() -> int:
    return int(_load().orc_num_threads())


def density(pos, mode: str = "cells", **kw) -> np.ndarray:
    """Kernel density Delta (FP64) per particle (Sec. 2.2.1, App. B.2)."""
    pos = _pos(pos)
    p = params_vector(**kw)
    out = np.zeros(len(pos), np.float64)
    rc = _load().orc_density(len(pos), _ptr(pos), _ptr(p), 0 if mode == "brute" else 1, _ptr(out))
    if rc:
        raise RuntimeError(f"orc_density failed ({rc})")
    return out


def density_sample(pos, which, **kw) -> np.ndarray:
    """Kernel density of the particles listed in ``which`` only."""
    pos = _pos(pos)
    which = np.ascontiguousarray(which, dtype=np.int64)
    p = params_vector(**kw)
    out = np.zeros(len(which), np.float64)
    rc = _load().orc_density_sample(len(pos), _ptr(pos), _ptr(p), len(which), _ptr(which), _ptr(out))
    if rc:
        raise RuntimeError(f"orc_density_sample failed ({rc})")
    return out


def fof(pos, dens, mode: str = "cells", **kw):
    """L0 labels (1 + min index; 0 = not dense enough) and the group count."""
    pos = _pos(pos)
    dens = np.ascontiguousarray(dens, dtype=np.float64)
    p = params_vector(**kw)
    l0 = np.zeros(len(pos), np.int32)
    ng = np.zeros(1, np.int64)
    rc = _load().orc_fof(len(pos), _ptr(pos), _ptr(p), _ptr(dens), 0 if mode == "brute" else 1,
                         _ptr(l0), _ptr(ng))
    if rc:
        raise RuntimeError(f"orc_fof failed ({rc})")
    return l0, int(ng[0])


def compaso(pos, dens, l0, mode: str = "cells", cap: int | None = None, radius: str = "sort",
            **kw) -> dict:
    """CompaSO L1 (literal sequential loop of Sec. 2.2.2) plus the output cut.
    radius: "sort" takes R_L1 from the sorted distances, "bins" by the radial
    bins of Sec. 2.3.4 (width max(b, l)/sqrt(3)); both give the same count."""
    if radius not in ("sort", "bins"):
        raise ValueError(radius)
    pos = _pos(pos)
    n = len(pos)
    dens = np.ascontiguousarray(dens, dtype=np.float64)
    l0 = np.ascontiguousarray(l0, dtype=np.int32)
    p = params_vector(**kw)
    cap = n if cap is None else int(cap)
    halo_id = np.zeros(n, np.int32)
    owner_all = np.zeros(n, np.int32)
    t = {k: np.zeros(max(cap, 1), np.int32) for k in ("id", "nucleus", "l0", "n", "ienc")}
    f = {k: np.zeros(max(n, 1), np.int32) for k in ("nucleus", "ienc", "count", "l0")}
    nh = np.zeros(1, np.int64)
    nf = np.zeros(1, np.int64)
    rc = _load().orc_compaso(n, _ptr(pos), _ptr(p), _ptr(dens), _ptr(l0),
                             (0 if mode == "brute" else 1) | (2 if radius == "bins" else 0),
                             _ptr(halo_id), _ptr(owner_all), cap,
                             _ptr(t["id"]), _ptr(t["nucleus"]), _ptr(t["l0"]), _ptr(t["n"]),
                             _ptr(t["ienc"]), _ptr(nh), _ptr(nf), n, _ptr(f["nucleus"]),
                             _ptr(f["ienc"]), _ptr(f["count"]), _ptr(f["l0"]))
    if rc:
        raise RuntimeError(f"orc_compaso failed ({rc})")
    k = int(min(nh[0], cap))
    table = {key: v[:k].copy() for key, v in t.items()}
    found = {key: v[:int(nf[0])].copy() for key, v in f.items()}
    return {"halo_id": halo_id, "owner_all": owner_all, "table": table, "found": found,
            "n_halos": int(nh[0]), "n_found": int(nf[0])}


def find(pos, mode: str = "cells", density_override=None, radius: str = "sort", **kw) -> dict:
    """The whole pass: density (or the given field), L0 FoF, CompaSO L1, cut."""
    dens = density(pos, mode=mode, **kw) if density_override is None \
        else np.asarray(density_override, dtype=np.float64)
    l0, ng = fof(pos, dens, mode=mode, **kw)
    res = compaso(pos, dens, l0, mode=mode, radius=radius, **kw)
    res.update({"density": dens, "l0": l0, "n_groups": ng})
    return res


def radius_search(e, K2: float, mode: str = "sort", w: float = 0.0):
    """Enclosed count i of the threshold radius from the squared distances e
    of a group's members to a nucleus (the nucleus included, at 0): "sort" is
    the definition (sorted distances, first k >= 1 with K^2 d_k^6 > k^2, else
    len(e)); "bins" the radial-bin search of Sec. 2.3.4 with bin width w.
    Returns (i, number of bins searched)."""
    e = np.ascontiguousarray(e, dtype=np.float64)
    searched = np.zeros(1, np.int64)
    k = _load().orc_radius_search(_ptr(e), len(e), float(K2), 1 if mode == "bins" else 0, float(w),
                                  _ptr(searched))
    return int(k), int(searched[0])


def group_order(halo_id, table_id):
    """Members in group order, as defined: the particles of each halo of the
    table (rows in table order) in ascending original index, then the
    particles of no halo (halo_id 0) in ascending index.  Returns (members,
    start) with row r's members in members[start[r]:start[r+1]] and the
    unassigned ones from start[len(table_id)]."""
    halo_id = np.asarray(halo_id, dtype=np.int64)
    table_id = np.asarray(table_id, dtype=np.int64)
    nrows = len(table_id)
    key = _row_keys(halo_id, table_id)
    members = np.argsort(key, kind="stable").astype(np.int64)
    start = np.searchsorted(key[members], np.arange(nrows + 1), side="left").astype(np.int64)
    return members, start


def _row_keys(halo_id, table_id):
    # table row of every particle's halo, len(table_id) for halo_id 0
    nrows = len(table_id)
    if nrows == 0:
        if np.any(halo_id != 0):
            raise ValueError("a halo_id label is not in the table")
        return np.zeros(len(halo_id), np.int64)
    order = np.argsort(table_id)
    pos = np.minimum(np.searchsorted(table_id[order], halo_id), nrows - 1)
    key = np.where(halo_id == 0, nrows, order[pos]).astype(np.int64)
    bad = (halo_id != 0) & (table_id[order][pos] != halo_id)
    if bad.any():
        raise ValueError("a halo_id label is not in the table")
    return key


def group_sweep(halo_id, table_id, table_n):
    """The partition sweep of Sec. 2.3.5 (largest halo first, then the
    unassigned particles, then the other halos): (members, start) in the
    layout of group_order, with the order inside a run left by the in-place
    partitions."""
    halo_id = np.ascontiguousarray(halo_id, dtype=np.int32)
    table_id = np.ascontiguousarray(table_id, dtype=np.int32)
    table_n = np.ascontiguousarray(table_n, dtype=np.int32)
    n, nrows = len(halo_id), len(table_id)
    members = np.zeros(max(n, 1), np.int64)
    start = np.zeros(nrows + 1, np.int64)
    rc = _load().orc_group_sweep(n, _ptr(halo_id), nrows, _ptr(table_id), _ptr(table_n), _ptr(members),
                                 _ptr(start))
    if rc:
        raise ValueError("a halo_id label is not in the table")
    return members[:n], start


# bits of events(): see orc_events
EV_L0CUT, EV_FLOOR, EV_PEAK, EV_ORDER, EV_GROUP = 1, 2, 4, 8, 128


def events(pos, dens, l0, tol: float = 1e-5, mode: str = "cells", **kw) -> np.ndarray:
    """Near-threshold events per particle (uint8 bits EV_*): where a density
    field within tol * max(Delta, 1) of ``dens`` can change the labels (the L0
    cut of Sec. 2.2.1, the floor, peak test and nucleus order of Sec. 2.2.2).
    ``l0`` is the L0 labelling of ``dens``."""
    pos = _pos(pos)
    dens = np.ascontiguousarray(dens, dtype=np.float64)
    l0 = np.ascontiguousarray(l0, dtype=np.int32)
    p = params_vector(**kw)
    out = np.zeros(len(pos), np.uint8)
    rc = _load().orc_events(len(pos), _ptr(pos), _ptr(p), _ptr(dens), _ptr(l0),
                            0 if mode == "brute" else 1, float(tol), _ptr(out))
    if rc:
        raise RuntimeError(f"orc_events failed ({rc})")
    return out


def params_at_redshift(omega_m0: float, z: float, **kw) -> dict:
    """Thresholds at redshift z (Sec. 2.3.1): see orc_params_at_redshift."""
    p = params_vector(**kw)
    out = np.zeros_like(p)
    if _load().orc_params_at_redshift(_ptr(p), float(omega_m0), float(z), _ptr(out)) != 0:
        raise ValueError("invalid cosmology")
    return {k: (int(v) if k in ("n_l1_min", "self_count") else float(v)) for k, v in zip(_ORDER, out)}


def l2_stats(pos, dens, halo_id, mode: str = "cells", **kw) -> dict:
    """Level 2 inside every L1 halo and the Table 1 position statistics (end of
    Sec. 2.2.2): see orc_l2_stats.  Per-halo arrays are in ascending L1 id."""
    pos = _pos(pos)
    n = len(pos)
    dens = np.ascontiguousarray(dens, dtype=np.float64)
    halo_id = np.ascontiguousarray(halo_id, dtype=np.int32)
    p = params_vector(**kw)
    cap = int(len(np.unique(halo_id[halo_id > 0])))
    si = np.zeros((max(cap, 1), 5), np.int32)
    sf = np.zeros((max(cap, 1), 22), np.float64)
    l2 = np.zeros((max(n, 1), 4), np.int32)
    members = np.zeros(max(n, 1), np.int32)
    l2_owner = np.zeros(max(n, 1), np.int32)
    gstart = np.zeros(cap + 1, np.int64)
    nl1 = np.zeros(1, np.int64)
    nl2 = np.zeros(1, np.int64)
    rc = _load().orc_l2_stats(n, _ptr(pos), _ptr(p), _ptr(dens), _ptr(halo_id),
                              0 if mode == "brute" else 1, cap, _ptr(nl1), _ptr(si), _ptr(sf), n,
                              _ptr(l2), _ptr(nl2), _ptr(l2_owner), _ptr(members), _ptr(gstart))
    if rc:
        raise RuntimeError(f"orc_l2_stats failed ({rc})")
    k = int(nl1[0])
    si, sf = si[:k], sf[:k]
    return {"id": si[:, 0].copy(), "n": si[:, 1].copy(), "n_l2": si[:, 2].copy(),
            "l2max_nucleus": si[:, 3].copy(), "l2max_n": si[:, 4].copy(),
            "x_com": sf[:, 0:3].copy(), "x_l2com": sf[:, 3:6].copy(), "l2_mass": sf[:, 6:11].copy(),
            "r_pct": sf[:, 11:20].copy(), "vcirc_max": sf[:, 20].copy(), "rvcirc_max": sf[:, 21].copy(),
            "l2": l2[:int(nl2[0])].copy(), "l2_owner": l2_owner[:n].copy(),
            "members": members[:int(gstart[k])].copy(),
            "gstart": gstart.copy()}
