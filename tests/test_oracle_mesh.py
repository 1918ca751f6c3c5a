"""Pins for the oracle's mesh M and triangles (Section 2, Mesh Construction)."""
import numpy as np
import pytest

import oracle
import synth
from oracle_helpers import cliques3, joins


def _edges_from_mask(mask):
    return int(sum(bin(int(m)).count("1") for m in mask)) // 2


@pytest.mark.parametrize("H,Wp", [(1, 3), (2, 3), (4, 5), (16, 64), (7, 33)])
def test_closed_cylinder_closed_forms(H, Wp):
    # Fully occupied closed lattice: V = H W', E = (3H - 2) W', T = 2 (H - 1) W',
    # Euler characteristic of a cylinder V - E + T = 0.
    valid = np.ones(H * Wp, np.uint8)
    mask = oracle.mesh_mask(H, Wp, 1, valid)
    E = _edges_from_mask(mask)
    T = oracle.triangles(H, Wp, 1, valid).shape[0]
    V = H * Wp
    assert E == (3 * H - 2) * Wp
    assert T == 2 * (H - 1) * Wp
    assert V - E + T == 0


@pytest.mark.parametrize("H,Wp", [(1, 4), (2, 3), (5, 6), (16, 40)])
def test_open_sheet_closed_forms(H, Wp):
    # Without the seam the lattice is a disc: V - E + T = 1.
    valid = np.ones(H * Wp, np.uint8)
    E = _edges_from_mask(oracle.mesh_mask(H, Wp, 0, valid))
    T = oracle.triangles(H, Wp, 0, valid).shape[0]
    assert E == H * (Wp - 1) + (H - 1) * Wp + (H - 1) * (Wp - 1)
    assert T == 2 * (H - 1) * (Wp - 1)
    assert H * Wp - E + T == 1


def test_single_ring_has_no_triangles():
    valid = np.ones(1 * 50, np.uint8)
    assert oracle.triangles(1, 50, 1, valid).shape[0] == 0


@pytest.mark.parametrize("H,Wp,wrap", [(3, 4, 1), (4, 5, 0), (3, 6, 1), (5, 7, 1), (2, 9, 0)])
def test_random_masks_match_the_forward_join_rule(H, Wp, wrap):
    rng = np.random.Generator(np.random.PCG64(H * 100 + Wp))
    for _ in range(200):
        valid = (rng.random(H * Wp) < 0.7).astype(np.uint8)
        J = joins(H, Wp, wrap, valid)
        mask = oracle.mesh_mask(H, Wp, wrap, valid)
        assert _edges_from_mask(mask) == len(J)
        # the 6-slot mask is symmetric: each join seen from both ends
        deg = np.zeros(H * Wp, int)
        for e in J:
            for v in e:
                deg[v] += 1
        assert np.array_equal(deg, [bin(int(m)).count("1") for m in mask])
        # surface triangles are exactly the 3-cliques of the join graph (W' >= 4)
        tri = oracle.triangles(H, Wp, wrap, valid)
        vidx = np.cumsum(valid) - 1
        cells = np.nonzero(valid)[0]
        got = {frozenset(cells[list(t)]) for t in tri}
        assert len(got) == tri.shape[0]
        if Wp >= 4:
            assert got == cliques3(J)


@pytest.mark.parametrize("name", ["c1_16x1800", "c2_64x2048"])
def test_triangle_orientation_faces_away_from_sensor(name):
    # For triangle (p0,p1,p2), ((p1-p0) x (p2-p0)) . p0 = det(p0,p1,p2), whose sign is
    # fixed by the lattice (rings downward, azimuth anticlockwise): positive.
    f = synth.workload_frames(name)[0]
    r = oracle.mesh_segment_frame(f)
    v = r.vertices.astype(np.float64)
    t = r.triangles
    p0, p1, p2 = v[t[:, 0]], v[t[:, 1]], v[t[:, 2]]
    d = np.einsum("ij,ij->i", np.cross(p1 - p0, p2 - p0), p0)
    assert t.shape[0] > 1000
    assert np.all(d > 0)


def test_vertices_are_the_kept_points_in_firing_order():
    f = synth.workload_frames("c2_64x2048")[0]
    r = oracle.mesh_segment_frame(f, s=2)
    assert np.array_equal(r.vertices, f.xyz[r.vertex_point])
    key = f.col[r.vertex_point].astype(np.int64) * f.sensor.n_rings + f.ring[r.vertex_point]
    assert np.all(np.diff(key) > 0)
