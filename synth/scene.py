"""Seeded synthetic spinning-Lidar sweeps.

This module is input generation only: a sensor model (rings at fixed elevations,
uniform azimuth firings), a float64 ray caster against simple primitives, range
noise along the ray and random dropouts. It contains none of the segmentation
method's arithmetic (no binning, meshing, normals or labelling); both the GPU
path's tests and the oracle's tests draw their inputs from here.

Sensor convention (the paper's spherical form p(theta, phi, r), Section 2):
ring 0 is the topmost laser and rings count downwards; azimuth phi is measured
counter-clockwise about +z from +x, and firing j has phi_j = az0 + j * 2*pi / W.
Points are emitted in firing order: shot j outer, ring i inner.

Random numbers come from numpy's PCG64 with the seed given; a frame of a batch
uses seed ``base * 1_000_003 + frame_index``.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

# Elevation span (top, bottom) in degrees per ring count.  16/64/128 rings take
# the spans the workloads name; 32 rings use an HDL-32E-like span (an external
# assumption: the paper names the sensor but not its field of view).
ELEV_SPANS_DEG = {
    16: (15.0, -15.0),
    32: (10.67, -30.67),
    64: (3.0, -25.0),
    128: (15.0, -25.0),
}

GROUND_Z = -1.7
WALL_HEIGHT = 12.0
MAX_EMIT_RANGE = 120.0

# primitive ids: 0 ground, 1 wall +y, 2 wall -y, then per object
PRIM_GROUND = 0
PRIM_WALL_POS = 1
PRIM_WALL_NEG = 2
PRIM_OBJ_BASE = 16


@dataclass(frozen=True)
class Sensor:
    n_rings: int
    n_azimuth: int
    elev_top_deg: float
    elev_bottom_deg: float
    az0: float = 0.0

    @staticmethod
    def standard(n_rings: int, n_azimuth: int) -> "Sensor":
        top, bot = ELEV_SPANS_DEG[n_rings]
        return Sensor(n_rings, n_azimuth, top, bot)

    def elevations(self) -> np.ndarray:
        """Ring elevations in radians, float64, strictly descending (ring 0 = top)."""
        if self.n_rings == 1:
            return np.array([math.radians(self.elev_top_deg)], dtype=np.float64)
        deg = np.linspace(self.elev_top_deg, self.elev_bottom_deg, self.n_rings, dtype=np.float64)
        return np.radians(deg)

    def azimuths(self) -> np.ndarray:
        return self.az0 + np.arange(self.n_azimuth, dtype=np.float64) * (2.0 * math.pi / self.n_azimuth)

    def rays(self) -> np.ndarray:
        """Unit ray directions, float64 [H, W, 3]."""
        e = self.elevations()[:, None]
        a = self.azimuths()[None, :]
        ce = np.cos(e)
        return np.stack([ce * np.cos(a), ce * np.sin(a), np.sin(e) * np.ones_like(a)], axis=-1)


@dataclass
class Scene:
    ground_normal: np.ndarray = field(default_factory=lambda: np.array([0.0, 0.0, 1.0]))
    ground_point: np.ndarray = field(default_factory=lambda: np.array([0.0, 0.0, GROUND_Z]))
    walls: tuple = ()                        # (d_pos, d_neg) or ()
    boxes: list = field(default_factory=list)      # (xmin, ymin, zmin, xmax, ymax, zmax)
    cylinders: list = field(default_factory=list)  # (cx, cy, r, z0, z1)
    spheres: list = field(default_factory=list)    # (cx, cy, cz, r)

    @property
    def flat_ground(self) -> bool:
        return bool(self.ground_normal[0] == 0.0 and self.ground_normal[1] == 0.0)

    def ground_z_at(self, x: float, y: float) -> float:
        n = self.ground_normal
        p0 = self.ground_point
        return float(p0[2] - (n[0] * (x - p0[0]) + n[1] * (y - p0[1])) / n[2])


# ----------------------------------------------------------------------------
# scene construction


def _place(rng, n, radius_fn, scene, placed, street, dmin=3.0, dmax=60.0, tries=200):
    """Draw n object footprints (cx, cy, R) without overlap; returns list of (cx, cy, R, extra)."""
    out = []
    for _ in range(n):
        for _t in range(tries):
            R, extra = radius_fn()
            if street:
                dpos, dneg = scene.walls
                cx = rng.uniform(-dmax, dmax)
                lo, hi = -dneg + R + 0.2, dpos - R - 0.2
                if hi <= lo:
                    continue
                cy = rng.uniform(lo, hi)
            else:
                d = rng.uniform(dmin, dmax)
                a = rng.uniform(0.0, 2.0 * math.pi)
                cx, cy = d * math.cos(a), d * math.sin(a)
            dist = math.hypot(cx, cy)
            if dist - R < max(1.0, dmin - R) or dist < dmin:
                continue
            if any(math.hypot(cx - px, cy - py) < R + pr + 0.1 for px, py, pr in placed):
                continue
            placed.append((cx, cy, R))
            out.append((cx, cy, R, extra))
            break
    return out


def make_scene(kind: str, rng: np.random.Generator, *, n_boxes=0, n_cyl=0, n_sph=0,
               sloped=False, walls=False, dmax=60.0) -> Scene:
    """kind is a label only; the counts and flags decide the content."""
    sc = Scene()
    if sloped:
        alpha = math.radians(rng.uniform(0.0, 8.0))
        beta = rng.uniform(0.0, 2.0 * math.pi)
        axis = np.array([math.cos(beta), math.sin(beta), 0.0])
        # rotate +z about the horizontal axis by alpha (Rodrigues)
        z = np.array([0.0, 0.0, 1.0])
        n = z * math.cos(alpha) + np.cross(axis, z) * math.sin(alpha)
        sc.ground_normal = n / np.linalg.norm(n)
    if walls:
        sc.walls = (rng.uniform(8.0, 15.0), rng.uniform(8.0, 15.0))
    street = bool(walls)
    placed: list = []

    def box_r():
        s = rng.uniform(1.0, 4.0, size=3)
        return 0.5 * math.hypot(s[0], s[1]), s

    for cx, cy, _R, s in _place(rng, n_boxes, box_r, sc, placed, street, dmax=dmax):
        zb = sc.ground_z_at(cx, cy) if not sc.flat_ground else GROUND_Z
        sc.boxes.append((cx - s[0] / 2, cy - s[1] / 2, zb, cx + s[0] / 2, cy + s[1] / 2, zb + s[2]))

    def cyl_r():
        return 0.3, rng.uniform(1.0, 3.0)

    for cx, cy, R, h in _place(rng, n_cyl, cyl_r, sc, placed, street, dmax=dmax):
        zb = sc.ground_z_at(cx, cy)
        sc.cylinders.append((cx, cy, R, zb - 0.5, zb + h))

    def sph_r():
        r = rng.uniform(0.5, 2.0)
        return r, r

    for cx, cy, R, r in _place(rng, n_sph, sph_r, sc, placed, street, dmax=dmax):
        sc.spheres.append((cx, cy, sc.ground_z_at(cx, cy) + r, r))
    return sc


# ----------------------------------------------------------------------------
# ray casting (float64)


def _az_window(sensor: Sensor, cx: float, cy: float, R: float) -> np.ndarray:
    """Azimuth columns whose rays can meet a footprint of radius R at (cx, cy)."""
    W = sensor.n_azimuth
    d = math.hypot(cx, cy)
    half = math.asin(min(1.0, R / d)) if d > R else math.pi
    half += 2.0 * (2.0 * math.pi / W)
    if half >= math.pi:
        return np.arange(W)
    phi = math.atan2(cy, cx)
    step = 2.0 * math.pi / W
    j0 = math.floor((phi - half - sensor.az0) / step)
    j1 = math.ceil((phi + half - sensor.az0) / step)
    if j1 - j0 + 1 >= W:
        return np.arange(W)
    return np.arange(j0, j1 + 1) % W


def cast(sensor: Sensor, scene: Scene):
    """Nearest hit per ray.

    Returns (t [H,W] float64, inf = miss; prim [H,W] int32, -1 = miss;
    snap_axis [H,W] int8, -1 = not an axis-aligned face; snap_val [H,W] float64).
    """
    U = sensor.rays()
    H, W = sensor.n_rings, sensor.n_azimuth
    t = np.full((H, W), np.inf)
    prim = np.full((H, W), -1, dtype=np.int32)
    sax = np.full((H, W), -1, dtype=np.int8)
    sval = np.zeros((H, W))
    ux, uy, uz = U[..., 0], U[..., 1], U[..., 2]

    def update(cols, tc, pid, ax, val):
        """tc: [H, len(cols)] candidate t (inf = no hit); pid/ax/val scalars or arrays."""
        sub_t = t[:, cols]
        better = tc < sub_t
        if not better.any():
            return
        sub_t = np.where(better, tc, sub_t)
        t[:, cols] = sub_t
        p = prim[:, cols]
        prim[:, cols] = np.where(better, pid, p)
        a = sax[:, cols]
        sax[:, cols] = np.where(better, ax, a)
        v = sval[:, cols]
        sval[:, cols] = np.where(better, val, v)

    allc = np.arange(W)
    # ground plane n.(x - p0) = 0
    n = scene.ground_normal
    p0 = scene.ground_point
    den = n[0] * ux + n[1] * uy + n[2] * uz
    with np.errstate(divide="ignore", invalid="ignore"):
        tg = np.where(den < -1e-12, float(n @ p0) / den, np.inf)
    tg = np.where(tg > 0, tg, np.inf)
    update(allc, tg, PRIM_GROUND, 2 if scene.flat_ground else -1, GROUND_Z)

    if scene.walls:
        dpos, dneg = scene.walls
        top = GROUND_Z + WALL_HEIGHT
        with np.errstate(divide="ignore", invalid="ignore"):
            tw = np.where(uy > 1e-12, dpos / uy, np.inf)
            tw = np.where((tw > 0) & (tw * uz <= top), tw, np.inf)
            update(allc, tw, PRIM_WALL_POS, 1, dpos)
            tw = np.where(uy < -1e-12, -dneg / uy, np.inf)
            tw = np.where((tw > 0) & (tw * uz <= top), tw, np.inf)
            update(allc, tw, PRIM_WALL_NEG, 1, -dneg)

    pid = PRIM_OBJ_BASE
    for (x0, y0, z0, x1, y1, z1) in scene.boxes:
        cx, cy = 0.5 * (x0 + x1), 0.5 * (y0 + y1)
        R = 0.5 * math.hypot(x1 - x0, y1 - y0)
        cols = _az_window(sensor, cx, cy, R)
        vx, vy, vz = ux[:, cols], uy[:, cols], uz[:, cols]
        lo = np.array([x0, y0, z0])
        hi = np.array([x1, y1, z1])
        with np.errstate(divide="ignore", invalid="ignore"):
            tn = np.full(vx.shape, -np.inf)
            tf = np.full(vx.shape, np.inf)
            axn = np.full(vx.shape, -1, dtype=np.int8)
            valn = np.zeros(vx.shape)
            for a, v in enumerate((vx, vy, vz)):
                t1 = lo[a] / v
                t2 = hi[a] / v
                near = np.minimum(t1, t2)
                far = np.maximum(t1, t2)
                # rays parallel to the slab: inside iff 0 in [lo, hi]
                par = np.abs(v) < 1e-15
                inside = (lo[a] <= 0.0) & (0.0 <= hi[a])
                near = np.where(par, np.where(inside, -np.inf, np.inf), near)
                far = np.where(par, np.where(inside, np.inf, -np.inf), far)
                sel = near > tn
                tn = np.where(sel, near, tn)
                axn = np.where(sel, np.int8(a), axn)
                valn = np.where(sel, np.where(v > 0, lo[a], hi[a]), valn)
                tf = np.minimum(tf, far)
        hit = (tn <= tf) & (tn > 0)
        tc = np.where(hit, tn, np.inf)
        # face id: 6 per box, axis*2 + side
        side = np.where(valn == np.take(hi, np.maximum(axn, 0)), 1, 0)
        fid = pid + 2 * np.maximum(axn, 0).astype(np.int32) + side
        update(cols, tc, fid, axn, valn)
        pid += 6

    for (cx, cy, r, z0, z1) in scene.cylinders:
        cols = _az_window(sensor, cx, cy, r)
        vx, vy, vz = ux[:, cols], uy[:, cols], uz[:, cols]
        a = vx * vx + vy * vy
        b = -2.0 * (vx * cx + vy * cy)
        c = cx * cx + cy * cy - r * r
        with np.errstate(divide="ignore", invalid="ignore"):
            disc = b * b - 4 * a * c
            ts = (-b - np.sqrt(np.where(disc >= 0, disc, np.nan))) / (2 * a)
            zs = ts * vz
            side_ok = (disc >= 0) & (ts > 0) & (zs >= z0) & (zs <= z1)
            tside = np.where(side_ok, ts, np.inf)
            tcap = np.where(np.abs(vz) > 1e-12, z1 / vz, np.inf)
            px = tcap * vx - cx
            py = tcap * vy - cy
            cap_ok = (tcap > 0) & (px * px + py * py <= r * r)
            tcap = np.where(cap_ok, tcap, np.inf)
        use_cap = tcap < tside
        tc = np.minimum(tside, tcap)
        update(cols, tc, np.where(use_cap, pid + 1, pid), np.where(use_cap, np.int8(2), np.int8(-1)),
               np.where(use_cap, z1, 0.0))
        pid += 2

    for (cx, cy, cz, r) in scene.spheres:
        cols = _az_window(sensor, cx, cy, r)
        vx, vy, vz = ux[:, cols], uy[:, cols], uz[:, cols]
        b = vx * cx + vy * cy + vz * cz
        c = cx * cx + cy * cy + cz * cz - r * r
        disc = b * b - c
        with np.errstate(invalid="ignore"):
            ts = b - np.sqrt(np.where(disc >= 0, disc, np.nan))
        tc = np.where((disc >= 0) & (ts > 0), ts, np.inf)
        update(cols, tc, pid, -1, 0.0)
        pid += 1
    return t, prim, sax, sval


# ----------------------------------------------------------------------------
# frames


@dataclass
class Frame:
    sensor: Sensor
    xyz: np.ndarray        # float32 [N, 3], firing order
    ring: np.ndarray       # int32 [N], generating ray's ring
    col: np.ndarray        # int32 [N], generating ray's azimuth column
    prim: np.ndarray       # int32 [N], primitive (face) id of the hit
    seed: int = 0
    scene: Scene | None = None

    @property
    def n_points(self) -> int:
        return int(self.xyz.shape[0])


def sample_frame(sensor: Sensor, scene: Scene, cast_result, *, sigma: float, dropout: float,
                 rng: np.random.Generator, max_range: float = MAX_EMIT_RANGE, seed: int = 0) -> Frame:
    """Turn a cast into one sweep: range noise along the ray, dropouts, firing order."""
    t, prim, sax, sval = cast_result
    H, W = sensor.n_rings, sensor.n_azimuth
    U = sensor.rays()
    noise = rng.standard_normal((H, W)) * sigma if sigma > 0 else np.zeros((H, W))
    keep = rng.random((H, W)) >= dropout
    r = t + noise
    emit = np.isfinite(t) & (t <= max_range) & keep & (r > 0)
    with np.errstate(invalid="ignore"):
        pts = np.where(emit[..., None], r[..., None] * U, 0.0)
    xyz = pts.astype(np.float32)
    if sigma == 0:
        # noise-free axis-aligned faces: every hit shares the face's float32 constant
        for ax in range(3):
            m = sax == ax
            xyz[..., ax] = np.where(m, sval.astype(np.float32), xyz[..., ax])
    ii, jj = np.meshgrid(np.arange(H, dtype=np.int32), np.arange(W, dtype=np.int32), indexing="ij")
    # firing order: shot (column) outer, ring inner
    emitT = emit.T.reshape(-1)
    return Frame(
        sensor=sensor,
        xyz=np.ascontiguousarray(xyz.transpose(1, 0, 2).reshape(-1, 3)[emitT]),
        ring=ii.T.reshape(-1)[emitT].copy(),
        col=jj.T.reshape(-1)[emitT].copy(),
        prim=prim.T.reshape(-1)[emitT].copy(),
        seed=seed,
        scene=scene,
    )


SCENE_KINDS = {
    # ground + 3 boxes + 2 cylinders, objects 3-40 m around the sensor
    "simple": dict(n_boxes=3, n_cyl=2, n_sph=0, sloped=False, walls=False),
    # street: ground, two walls, 20 boxes, 10 cylinders, 5 spheres
    "street": dict(n_boxes=20, n_cyl=10, n_sph=5, sloped=False, walls=True),
    # dense urban: 40 boxes, 20 cylinders, 10 spheres, ground sloped 0-8 degrees
    "urban": dict(n_boxes=40, n_cyl=20, n_sph=10, sloped=True, walls=False),
    # noise-free geometry checks
    "ground": dict(n_boxes=0, n_cyl=0, n_sph=0, sloped=False, walls=False),
    # ground alone, tilted 0-8 degrees: the far rings meet it at grazing angles
    "sloped_ground": dict(n_boxes=0, n_cyl=0, n_sph=0, sloped=True, walls=False),
    "boxes": dict(n_boxes=6, n_cyl=0, n_sph=0, sloped=False, walls=False),
    "spheres": dict(n_boxes=0, n_cyl=0, n_sph=6, sloped=False, walls=False),
    "walls": dict(n_boxes=0, n_cyl=0, n_sph=0, sloped=False, walls=True),
}


def make_frame(sensor: Sensor, kind: str, seed: int, *, sigma: float, dropout: float,
               max_range: float = MAX_EMIT_RANGE) -> Frame:
    rng = np.random.Generator(np.random.PCG64(seed))
    spec = dict(SCENE_KINDS[kind])
    dmax = 40.0 if kind in ("simple", "boxes", "spheres") else 60.0
    sc = make_scene(kind, rng, dmax=dmax, **spec)
    cr = cast(sensor, sc)
    return sample_frame(sensor, sc, cr, sigma=sigma, dropout=dropout, rng=rng, max_range=max_range,
                        seed=seed)


def frame_seed(base: int, index: int) -> int:
    return base * 1_000_003 + index
