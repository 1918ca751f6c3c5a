"""Sweeps whose returns do not sit on the lattice rays, for the binning tests.

A real sensor's returns P = {p(theta, phi, r)} (Section 2, opening paragraph)
carry their measured angles, not the nominal ring elevations and firing
azimuths.  These sweeps hold
  - one return per (ring, firing) ray with its elevation and azimuth jittered
    within the ray's own bin (so every cell of the lattice is occupied),
  - returns placed on either side of every kind of decision boundary, at
    distances spread log-uniformly from 1e-12 to 1e-3 rad: ring midpoints
    (half-way between two ring elevations) and half-firing azimuths, some of
    them moved by a few float32 ulps to the representable point nearest the
    boundary,
  - returns across the atan2 branch cut (phi = +-pi, y = +0.0 and -0.0),
  - returns above the top ring and below the bottom one, and outside the
    range window.
Coordinates are float32, as the sensor delivers them.  The margins (how far
each float32 return lies from its nearest boundary, in FP64) are measured
here so that a test can state how many returns its decisions have to get
right at each distance; returns closer than 1e-13 rad to a boundary are left
out, since two correctly rounded FP64 evaluations of atan2 may already
disagree there.
"""
from __future__ import annotations

import math

import numpy as np

MIN_MARGIN_RAD = 1e-13


def elevation_table(H, kind="uniform", seed=0, top=15.0, bottom=-25.0):
    """Descending ring elevations in radians: uniform over [bottom, top] degrees,
    or irregular (gaps drawn from 0.1 to 2 degrees, as sensors denser near the
    horizon have)."""
    if kind == "uniform":
        return np.radians(np.linspace(top, bottom, H))
    rng = np.random.Generator(np.random.PCG64(seed))
    gaps = rng.uniform(0.1, 2.0, size=H - 1)
    deg = top - np.concatenate([[0.0], np.cumsum(gaps)])
    return np.radians(deg)


def _range(el, phi, rng):
    """A smooth surface around the sensor (6-18 m) with 5 mm noise, so that the
    mesh is a plausible one."""
    return 12.0 + 4.0 * np.sin(3.0 * phi) + 2.0 * np.cos(5.0 * el) + rng.normal(0.0, 0.005, size=np.shape(el))


def _xyz(r, el, phi):
    ce = np.cos(el)
    return np.stack([r * ce * np.cos(phi), r * ce * np.sin(phi), r * np.sin(el)], axis=-1)


def _log_offsets(rng, n, lo=1e-12, hi=1e-3):
    return np.exp(rng.uniform(math.log(lo), math.log(hi), size=n)) * rng.choice([-1.0, 1.0], size=n)


def ring_margin(xyz, elev):
    """Distance in radians (FP64, from the float32 coordinates) of each return's
    elevation from the nearest ring midpoint; inf for a single ring."""
    x, y, z = (xyz[:, k].astype(np.float64) for k in range(3))
    el = np.arctan2(z, np.sqrt(x * x + y * y))
    if len(elev) < 2:
        return np.full(len(el), np.inf)
    return _nearest_gap(el, 0.5 * (elev[:-1] + elev[1:]))[0]


def _nearest_gap(v, table):
    """|v - nearest entry of `table`| and that entry, for a descending table."""
    asc = table[::-1]
    k = np.clip(np.searchsorted(asc, v), 1, len(asc) - 1) if len(asc) > 1 else np.zeros(len(v), np.int64)
    lo = asc[np.maximum(k - 1, 0)]
    hi = asc[k]
    dl, dh = np.abs(v - lo), np.abs(v - hi)
    return np.minimum(dl, dh), np.where(dl <= dh, lo, hi)


def firing_margin(xyz, W, az0):
    """Distance in radians of each return's azimuth from the nearest half-firing
    boundary az0 + (j + 1/2) 2 pi / W."""
    x, y = xyz[:, 0].astype(np.float64), xyz[:, 1].astype(np.float64)
    dphi = 2.0 * math.pi / W
    jf = (np.arctan2(y, x) - az0) / dphi
    return np.abs((jf - np.floor(jf)) - 0.5) * dphi


def in_ring_band(xyz, elev, rel=2e-6, abs_=1e-7):
    """Whether t = z / rho lies within rel * |T| + abs of a midpoint tangent T
    (rounded to float32): where the kernels leave the ring to the FP64 pass."""
    x, y, z = (xyz[:, k].astype(np.float64) for k in range(3))
    t = z / np.sqrt(x * x + y * y)
    if len(elev) < 2:
        return np.zeros(len(t), bool)
    T = np.tan(0.5 * (elev[:-1] + elev[1:])).astype(np.float32).astype(np.float64)
    d, Tn = _nearest_gap(t, T)
    return d <= rel * np.abs(Tn) + abs_


def in_firing_band(xyz, W, az0, band=0.02):
    """Whether the firing estimate lies within `band` firings of a half-firing
    boundary: where the kernels leave the firing to the FP64 pass."""
    return firing_margin(xyz, W, az0) <= band * 2.0 * math.pi / W


def _nudge(xyz32, margin_fn, rng, cols, steps=4):
    """Move each return by up to `steps` float32 ulps in the coordinates `cols`
    to the representable point with the smallest margin not below MIN_MARGIN_RAD."""
    best = xyz32.copy()
    best_m = margin_fn(best)
    best_m = np.where(best_m >= MIN_MARGIN_RAD, best_m, np.inf)
    grid = np.array(np.meshgrid(*[np.arange(-steps, steps + 1)] * len(cols), indexing="ij")).reshape(len(cols), -1).T
    for off in grid:
        cand = xyz32.copy()
        for c, k in zip(cols, off):
            v = cand[:, c]
            ok = np.abs(v) > 1e-30     # stepping the bits of a normal float never crosses zero
            bits = v.view(np.int32).astype(np.int64) + int(k)
            moved = bits.astype(np.int32).view(np.float32)
            cand[:, c] = np.where(ok, moved, v)
        m = margin_fn(cand)
        take = (m >= MIN_MARGIN_RAD) & (m < best_m)
        best[take] = cand[take]
        best_m = np.where(take, m, best_m)
    return best


def off_lattice_sweep(H, W, az0, elev, seed, n_boundary=20000, dense=True):
    """One sweep of float32 returns (see the module docstring) and a dict of
    per-return tags: 'ring_b' / 'firing_b' mark the returns placed at a ring
    midpoint / half-firing boundary."""
    rng = np.random.Generator(np.random.PCG64(seed))
    elev = np.asarray(elev, np.float64)
    dphi = 2.0 * math.pi / W
    gap_up = np.empty(H)
    gap_dn = np.empty(H)
    if H > 1:
        d = elev[:-1] - elev[1:]
        gap_up[1:] = d / 2
        gap_dn[:-1] = d / 2
        gap_up[0] = gap_dn[0]
        gap_dn[-1] = gap_up[-1]
    else:
        gap_up[:] = gap_dn[:] = 0.01
    parts, tags = [], []

    def add(pts, tag):
        parts.append(pts.astype(np.float32))
        tags.append(np.full(len(pts), tag, np.int8))

    if dense:
        jj, ii = np.meshgrid(np.arange(W), np.arange(H), indexing="ij")   # firing order
        ii, jj = ii.reshape(-1), jj.reshape(-1)
        u = rng.uniform(-0.45, 0.45, size=ii.size)
        el = elev[ii] + np.where(u > 0, u * gap_up[ii], u * gap_dn[ii])
        phi = az0 + (jj + rng.uniform(-0.45, 0.45, size=ii.size)) * dphi
        add(_xyz(_range(el, phi, rng), el, phi), 0)

    nb = n_boundary
    if H > 1:
        # ring midpoints, azimuth anywhere
        i = rng.integers(0, H - 1, size=nb)
        el = 0.5 * (elev[i] + elev[i + 1]) + _log_offsets(rng, nb)
        phi = rng.uniform(-math.pi, math.pi, size=nb)
        pts = _xyz(_range(el, phi, rng), el, phi).astype(np.float32)
        half = nb // 2
        pts[:half] = _nudge(pts[:half], lambda p: ring_margin(p, elev), rng, cols=(2,), steps=6)
        add(pts, 1)
    # half-firing boundaries, elevation anywhere in the table
    j = rng.integers(0, W, size=nb)
    phi = az0 + (j + 0.5) * dphi + np.clip(_log_offsets(rng, nb), -0.45 * dphi, 0.45 * dphi)
    el = rng.uniform(elev[-1], elev[0], size=nb) if H > 1 else np.full(nb, elev[0])
    pts = _xyz(_range(el, phi, rng), el, phi).astype(np.float32)
    half = nb // 2
    pts[:half] = _nudge(pts[:half], lambda p: firing_margin(p, W, az0), rng, cols=(0, 1), steps=4)
    add(pts, 2)
    # both boundaries at once
    if H > 1:
        m = nb // 4
        i = rng.integers(0, H - 1, size=m)
        el = 0.5 * (elev[i] + elev[i + 1]) + _log_offsets(rng, m)
        jb = rng.integers(0, W, size=m)
        phi = az0 + (jb + 0.5) * dphi + np.clip(_log_offsets(rng, m), -0.45 * dphi, 0.45 * dphi)
        add(_xyz(_range(el, phi, rng), el, phi), 3)
    # across the atan2 branch cut: phi = pi - d and -pi + d, and y = +0.0 / -0.0 exactly
    m = 2000
    d = np.abs(_log_offsets(rng, m, 1e-12, 1e-2))
    el = rng.uniform(elev[-1], elev[0], size=m) if H > 1 else np.full(m, elev[0])
    phi = np.where(rng.random(m) < 0.5, math.pi - d, -math.pi + d)
    pts = _xyz(_range(el, phi, rng), el, phi).astype(np.float32)
    pts[:100, 1] = 0.0
    pts[100:200, 1] = -0.0
    pts[:200, 0] = -np.abs(pts[:200, 0]) - 1.0
    add(pts, 4)
    # beyond the table's elevations (nearest ring: the top or the bottom one),
    # and outside the range window
    m = 500
    el = np.concatenate([elev[0] + rng.uniform(0.01, 0.4, m), elev[-1] - rng.uniform(0.01, 0.4, m)])
    phi = rng.uniform(-math.pi, math.pi, size=2 * m)
    add(_xyz(_range(el, phi, rng), el, phi), 5)
    r = np.concatenate([rng.uniform(0.2, 0.99, m), rng.uniform(60.5, 100.0, m)])
    el = rng.uniform(elev[-1], elev[0], size=2 * m) if H > 1 else np.full(2 * m, elev[0])
    phi = rng.uniform(-math.pi, math.pi, size=2 * m)
    add(_xyz(r, el, phi), 6)

    xyz = np.concatenate(parts)
    tag = np.concatenate(tags)
    # returns within MIN_MARGIN_RAD of a boundary are left out
    keep = (ring_margin(xyz, elev) >= MIN_MARGIN_RAD) & (firing_margin(xyz, W, az0) >= MIN_MARGIN_RAD)
    xyz, tag = xyz[keep], tag[keep]
    perm = rng.permutation(len(xyz))
    return np.ascontiguousarray(xyz[perm]), tag[perm]
