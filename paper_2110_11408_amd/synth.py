"""Seeded synthetic particle boxes for halo finding.

This module only draws inputs: uniform background particles plus NFW haloes
(concentration 8, truncated at R200m) whose particle counts follow a power law
dn/dN ~ N^-1.9.  It contains none of the group-finding arithmetic, so both the
CPU oracle and the GPU path may take their inputs from it.

All lengths are in units of the mean interparticle spacing when the box side is
N^(1/3) (mean density 1), which is the operating point of the paper's parameter
table (kernel radius 0.4, linking length 0.25, thresholds 60 and 200 times the
mean density).

Stand-in note: the paper measures AbacusSummit boxes, which are not available;
these boxes reproduce its clustering regime (a mix of unclustered background and
resolved haloes from 35 particles up) rather than its data.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

NFW_CONCENTRATION = 8.0
_OVERDENSITY = 200.0  # haloes are truncated at the radius enclosing 200x mean


@dataclasses.dataclass(frozen=True)
class BoxRecipe:
    n: int                      # total particle count
    side: float                 # periodic box side
    halo_frac: float            # fraction of particles drawn inside haloes
    nmin: int = 35              # smallest halo drawn
    nmax: int = 20000           # largest halo drawn
    slope: float = 1.9          # dn/dN ~ N^-slope
    pair_frac: float = 0.0      # fraction of haloes that sit in pairs
    triple_frac: float = 0.0    # fraction of haloes that sit in triples
    sep: tuple = (0.5, 1.5)     # companion separation in units of the primary's R200
    shuffle: bool = True        # randomise the particle order


# Named workloads (particle counts and clustering mix of the benchmark boxes).
RECIPES = {
    # 64^3 particles, half in isolated haloes of 35..20000 particles.
    "plain64": BoxRecipe(n=64 ** 3, side=64.0, halo_frac=0.5),
    # 256^3 particles, same mix, 20% of haloes in pairs at 0.5-1.5 R200.
    "plain256": BoxRecipe(n=256 ** 3, side=256.0, halo_frac=0.5, pair_frac=0.2),
    # 512^3 particles, 70% in haloes up to 200000 particles, in pairs and triples.
    "large512": BoxRecipe(n=512 ** 3, side=512.0, halo_frac=0.7, nmax=200000,
                          pair_frac=0.3, triple_frac=0.15, sep=(0.3, 1.2)),
}

RECIPE_SEED_BASE = {"plain64": 1000, "plain256": 2000, "large512": 4000}


def r200(npart, mean_density=1.0):
    """Radius enclosing 200x the mean density for a halo of npart particles."""
    return (3.0 * np.asarray(npart, dtype=np.float64)
            / (4.0 * math.pi * _OVERDENSITY * mean_density)) ** (1.0 / 3.0)


def _nfw_mass_fraction(x, c=NFW_CONCENTRATION):
    cx = c * x
    return (np.log1p(cx) - cx / (1.0 + cx)) / (math.log1p(c) - c / (1.0 + c))


_INV_TABLE = None


def _nfw_inverse_table(c=NFW_CONCENTRATION, npts=1 << 14):
    """x(m) for the truncated NFW enclosed-mass fraction, tabulated on sqrt(m).

    Each node is solved by 64 FP64 bisection steps on x in [0, 1]; between
    nodes the map is close to linear in sqrt(m) because m ~ x^2 near the centre.
    """
    global _INV_TABLE
    if _INV_TABLE is None:
        u = np.linspace(0.0, 1.0, npts)
        target = u * u
        lo = np.zeros(npts)
        hi = np.ones(npts)
        for _ in range(64):
            mid = 0.5 * (lo + hi)
            below = _nfw_mass_fraction(mid, c) < target
            lo = np.where(below, mid, lo)
            hi = np.where(below, hi, mid)
        _INV_TABLE = (u, 0.5 * (lo + hi))
    return _INV_TABLE


def nfw_radii(rng, nparticles_per_halo, r200_per_halo):
    """Radii (FP64) of NFW particles, one block per halo."""
    u_tab, x_tab = _nfw_inverse_table()
    m = rng.random(int(np.sum(nparticles_per_halo)))
    x = np.interp(np.sqrt(m), u_tab, x_tab)
    return x * np.repeat(r200_per_halo, nparticles_per_halo)


def draw_halo_sizes(rng, budget, nmin, nmax, slope):
    """Power-law halo sizes until the particle budget is used (last truncated)."""
    sizes = []
    used = 0
    a = nmin ** (1.0 - slope)
    b = nmax ** (1.0 - slope)
    while used < budget:
        chunk = rng.random(4096)
        draw = np.rint((a + chunk * (b - a)) ** (1.0 / (1.0 - slope))).astype(np.int64)
        for s in draw:
            s = int(min(s, budget - used))
            sizes.append(s)
            used += s
            if used >= budget:
                break
    return np.asarray(sizes, dtype=np.int64)


def _unit_vectors(rng, k):
    v = rng.standard_normal((k, 3))
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    return v


def _wrap_f32(pos64, side):
    """Wrap into [0, side) and cast to float32, keeping the cast inside the box."""
    p = np.mod(pos64, side)
    p32 = p.astype(np.float32)
    p32[p32 >= np.float32(side)] = np.float32(0.0)
    p32[p32 < 0] = np.float32(0.0)
    return p32


def make_box(recipe: BoxRecipe, seed: int):
    """Draw one periodic box.

    Returns (pos float32 [n, 3] C-contiguous, side, truth) where truth holds the
    planted halo centres, sizes and R200 values and, per particle, the index of
    the planted halo it was drawn in (-1 for background).
    """
    rng = np.random.default_rng(seed)
    n = int(recipe.n)
    side = float(recipe.side)
    nbar = n / side ** 3
    n_halo = int(round(recipe.halo_frac * n))
    sizes = draw_halo_sizes(rng, n_halo, recipe.nmin, recipe.nmax, recipe.slope) \
        if n_halo > 0 else np.zeros(0, np.int64)
    h = len(sizes)
    centres = rng.random((h, 3)) * side
    # Companions: consecutive haloes of a shuffled list form pairs and triples;
    # the largest of each system stays put and the others are moved next to it.
    order = rng.permutation(h)
    n_pair = int(recipe.pair_frac * h) // 2
    n_trip = int(recipe.triple_frac * h) // 3
    systems = []
    k = 0
    for _ in range(n_pair):
        systems.append(order[k:k + 2]); k += 2
    for _ in range(n_trip):
        systems.append(order[k:k + 3]); k += 3
    r200s = r200(sizes, nbar)
    for sysm in systems:
        sysm = sorted(sysm, key=lambda i: -sizes[i])
        prim = sysm[0]
        for comp in sysm[1:]:
            d = rng.uniform(recipe.sep[0], recipe.sep[1]) * r200s[prim]
            centres[comp] = centres[prim] + d * _unit_vectors(rng, 1)[0]
    n_bg = n - int(sizes.sum())
    bg = rng.random((n_bg, 3)) * side
    if h:
        radii = nfw_radii(rng, sizes, r200s)
        dirs = _unit_vectors(rng, len(radii))
        hp = np.repeat(centres, sizes, axis=0) + radii[:, None] * dirs
        pos64 = np.concatenate([bg, hp], axis=0)
        halo_of = np.concatenate([np.full(n_bg, -1, np.int64),
                                  np.repeat(np.arange(h), sizes)])
    else:
        pos64 = bg
        halo_of = np.full(n_bg, -1, np.int64)
    pos = _wrap_f32(pos64, side)
    if recipe.shuffle:
        perm = rng.permutation(n)
        pos = pos[perm]
        halo_of = halo_of[perm]
    truth = {"centres": np.mod(centres, side), "sizes": sizes, "r200": r200s,
             "halo_of": halo_of}
    return np.ascontiguousarray(pos), side, truth


def named_box(name: str, k: int = 0):
    """Box k of a named workload, seeded as base + k."""
    return make_box(RECIPES[name], RECIPE_SEED_BASE[name] + k)


def small_box(n: int, halo_frac: float = 0.5, nmax: int = 2000, seed: int = 0,
              pair_frac: float = 0.2, side: float | None = None):
    """A small box with the same generator, for parity tests."""
    side = float(n) ** (1.0 / 3.0) if side is None else float(side)
    return make_box(BoxRecipe(n=n, side=side, halo_frac=halo_frac, nmax=nmax,
                              pair_frac=pair_frac), seed)


def batch_boxes(count: int = 96, seed: int = 3000, lo: float = 24.0, hi: float = 160.0):
    """Independent periodic sub-boxes of uneven size (side log-uniform in lo..hi)."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        side = float(math.exp(rng.uniform(math.log(lo), math.log(hi))))
        n = int(round(side ** 3))
        out.append(make_box(BoxRecipe(n=n, side=side, halo_frac=0.5), seed * 1000 + i))
    return out


def request_stream(count: int, rate_hz: float, seed: int = 5000,
                   nlo: float = 1e4, nhi: float = 1e7):
    """Poisson arrivals of requests, each a seeded box with log-uniform size."""
    rng = np.random.default_rng(seed)
    t = np.cumsum(rng.exponential(1.0 / rate_hz, size=count))
    reqs = []
    for i in range(count):
        n = int(round(math.exp(rng.uniform(math.log(nlo), math.log(nhi)))))
        frac = float(rng.uniform(0.3, 0.7))
        reqs.append({"t": float(t[i]), "n": n, "side": float(n) ** (1.0 / 3.0),
                     "halo_frac": frac, "seed": seed * 1000 + i})
    return reqs
