"""Helpers for the GPU parity tests: run the HIP path, compare with the oracle."""
from __future__ import annotations

import numpy as np

import oracle

THR = (0.2, 0.2, 0.2)
NORMAL_TOL_RAD = 1e-5
MARGIN = 1e-4


def geometry(sensor, s=1, wrap=1):
    import paper_2005_02704_amd as lp
    return lp.SensorGeometry(sensor.elevations(), sensor.n_azimuth, s, wrap, sensor.az0)


def pad_normals(normals, sensor, s=1):
    """Caller-given normals (one row per vertex) padded with zero rows to the
    sensor's vertex capacity H * W / s, the size the binding asks for."""
    n = np.ascontiguousarray(normals, np.float32).reshape(-1, 3)
    rows = sensor.n_rings * (sensor.n_azimuth // s)
    out = np.zeros((max(rows, n.shape[0]), 3), np.float32)
    out[:n.shape[0]] = n
    return out


def run_gpu(ctx, items, launch="plain", r_min=1.0, r_max=60.0, thr=THR, predicate=0, cos_min=0.0, min_segment=0,
            point_labels=False, score_radius=None):
    """items: list of (xyz float32 [N,3] numpy, synth.Sensor, s, wrap, normals_in or None
    [, truth ids int32 [N] or None [, reported rings uint8 [N]]]); score_radius (with
    truth ids) asks for the edge counts."""
    import torch
    import paper_2005_02704_amd as lp
    inputs = []
    for it in items:
        xyz, sen, s, wrap, nin = it[:5]
        x = torch.from_numpy(np.ascontiguousarray(xyz, np.float32)).cuda()
        n = torch.from_numpy(pad_normals(nin, sen, s)).cuda() if nin is not None else None
        tr = torch.from_numpy(np.ascontiguousarray(it[5], np.int32)).cuda() if len(it) > 5 and it[5] is not None \
            else None
        rg = torch.from_numpy(np.ascontiguousarray(it[6], np.uint8)).cuda() if len(it) > 6 else None
        inputs.append((x, geometry(sen, s, wrap), n, tr, rg))
    params = lp.make_params(r_min, r_max, thr, predicate, cos_min, min_segment,
                            score_radius if score_radius is not None else 1)
    outs = lp.lidar_mesh_segment(ctx, inputs, params, launch=launch, point_labels=point_labels,
                                 scores=score_radius is not None)
    torch.cuda.synchronize()
    res = []
    for o in outs:
        t = o.trimmed()
        res.append(dict(vertices=t["vertices"].cpu().numpy(), normals=t["normals"].cpu().numpy(),
                        labels=t["labels"].cpu().numpy(), triangles=t["triangles"].cpu().numpy(),
                        vertex_point=t["vertex_point"].cpu().numpy(), counts=t["counts"],
                        point_labels=t["point_labels"].cpu().numpy() if t["point_labels"] is not None else None,
                        edge_counts=t["edge_counts"]))
    return res


def run_oracle(xyz, sen, s=1, wrap=1, r_min=1.0, r_max=60.0, thr=THR, **kw):
    return oracle.mesh_segment(xyz, sen.n_rings, sen.n_azimuth, s, sen.elevations(), az0=sen.az0,
                               r_min=r_min, r_max=r_max, thr=thr, wrap=wrap, **kw)


def normal_angles(a, b):
    a = a.astype(np.float64)
    b = b.astype(np.float64)
    return np.arctan2(np.linalg.norm(np.cross(a, b), axis=1), np.einsum("ij,ij->i", a, b))


def check_geometry(g, r, tol=NORMAL_TOL_RAD):
    """Vertices, vertex_point, triangles bit-exact; normals within tol; same has-normal set."""
    assert g["counts"][0] == r.vertices.shape[0], (g["counts"], r.counts)
    assert g["counts"][1] == r.triangles.shape[0], (g["counts"], r.counts)
    assert np.array_equal(g["vertices"], r.vertices)
    assert np.array_equal(g["vertex_point"], r.vertex_point)
    assert np.array_equal(g["triangles"], r.triangles)
    hg = np.any(g["normals"] != 0, axis=1)
    hr = np.any(r.normals64 != 0, axis=1)
    assert np.array_equal(hg, hr)
    if hr.any():
        ang = normal_angles(g["normals"][hr], r.normals64[hr])
        assert ang.max() <= tol, f"max normal angle {ang.max():.3e} rad"
        return float(ang.max())
    return 0.0


def partition_refines(fine, coarse):
    """Every class of `fine` lies inside one class of `coarse`."""
    m = {}
    for a, b in zip(fine.tolist(), coarse.tolist()):
        if m.setdefault(a, b) != b:
            return False
    return True


def sandwich(g_labels, xyz, sen, s=1, wrap=1, r_min=1.0, r_max=60.0, thr=THR, margin=MARGIN):
    """Partition bounds from the oracle at thresholds thr -/+ margin on its own normals."""
    lo = run_oracle(xyz, sen, s, wrap, r_min, r_max, tuple(t - margin for t in thr))
    hi = run_oracle(xyz, sen, s, wrap, r_min, r_max, tuple(t + margin for t in thr))
    return partition_refines(lo.labels, g_labels) and partition_refines(g_labels, hi.labels)


def margin_clear(xyz, sen, s=1, wrap=1, r_min=1.0, r_max=60.0, thr=THR, margin=MARGIN, rounds=12):
    """Drop points until no mesh join of the oracle's mesh has a normal-component
    difference within `margin` of its threshold (between two vertices with normals).

    Decisions there could go either way under FP32 rounding of the normals; a
    dropped point is just another dropout.  Returns the reduced float32 points."""
    xyz = np.ascontiguousarray(xyz, np.float32)
    H = sen.n_rings
    Wp = sen.n_azimuth // s
    for _ in range(rounds):
        cp = oracle.bin_points(xyz, H, sen.n_azimuth, s, sen.elevations(), sen.az0, r_min, r_max)
        valid = (cp >= 0).astype(np.uint8)
        cell_xyz = np.zeros((H * Wp, 3), np.float32)
        cell_xyz[valid == 1] = xyz[cp[valid == 1]]
        n64, hasn = oracle.normals(H, Wp, wrap, cell_xyz, valid)
        n32 = n64.astype(np.float32).astype(np.float64)
        bad = np.zeros(H * Wp, bool)
        ii = np.tile(np.arange(H), Wp)
        kk = np.repeat(np.arange(Wp), H)
        c = np.arange(H * Wp)
        for di, dk in ((1, 0), (1, 1), (0, 1)):
            i2 = ii + di
            k2 = kk + dk
            ok = i2 < H
            if wrap:
                k2 = k2 % Wp
            else:
                ok &= k2 < Wp
            q = np.where(ok, k2 * H + np.minimum(i2, H - 1), 0)
            both = ok & (hasn[c] == 1) & (hasn[q] == 1)
            d = np.abs(n32[c] - n32[q])
            near = np.any(np.abs(d - np.asarray(thr)) < margin, axis=1)
            hit = both & near
            bad[c[hit]] = True
        if not bad.any():
            return xyz
        drop = cp[bad]
        keep = np.ones(xyz.shape[0], bool)
        keep[drop] = False
        xyz = xyz[keep]
    raise RuntimeError("margin clearing did not converge")


def margin_clear_cos(xyz, sen, cos_min, s=1, wrap=1, r_min=1.0, r_max=60.0, margin=MARGIN, rounds=12):
    """As margin_clear, for the cosine test: drop points until no mesh join between
    two vertices with normals has a dot product within `margin` of cos_min."""
    xyz = np.ascontiguousarray(xyz, np.float32)
    H = sen.n_rings
    Wp = sen.n_azimuth // s
    for _ in range(rounds):
        cp = oracle.bin_points(xyz, H, sen.n_azimuth, s, sen.elevations(), sen.az0, r_min, r_max)
        valid = (cp >= 0).astype(np.uint8)
        cell_xyz = np.zeros((H * Wp, 3), np.float32)
        cell_xyz[valid == 1] = xyz[cp[valid == 1]]
        n64, hasn = oracle.normals(H, Wp, wrap, cell_xyz, valid)
        n32 = n64.astype(np.float32).astype(np.float64)
        bad = np.zeros(H * Wp, bool)
        ii = np.tile(np.arange(H), Wp)
        kk = np.repeat(np.arange(Wp), H)
        c = np.arange(H * Wp)
        for di, dk in ((1, 0), (1, 1), (0, 1)):
            i2 = ii + di
            k2 = kk + dk
            ok = i2 < H
            if wrap:
                k2 = k2 % Wp
            else:
                ok &= k2 < Wp
            q = np.where(ok, k2 * H + np.minimum(i2, H - 1), 0)
            both = ok & (hasn[c] == 1) & (hasn[q] == 1)
            dot = np.einsum("ij,ij->i", n32[c], n32[q])
            hit = both & (np.abs(dot - cos_min) < margin)
            bad[c[hit]] = True
        if not bad.any():
            return xyz
        keep = np.ones(xyz.shape[0], bool)
        keep[cp[bad]] = False
        xyz = xyz[keep]
    raise RuntimeError("margin clearing did not converge")
