"""Pins for the oracle's steps after Algorithm 1 (Section 2, Segmentation by
Surface Homogeneity, last paragraph) and for its cosine similarity test.

  * back-fill: "Due to sub-sampling, all points in P will not get a label" --
    they take the label of the nearest labelled point along the horizontal
    sweep; checked against a brute force over every (point, vertex) pair on
    tiny lattices, the tie rule, the seam, and the kept points themselves;
  * removal of segments with too few points: the surviving labels are exactly
    those carried by at least min_size vertices;
  * cosine test: Algorithm 1 with n_p . n_q > cos_min equals the connected
    components of the cosine-similar joins, and a closed form on a strip.
"""
import itertools

import numpy as np
import pytest

import oracle
import synth
from oracle_helpers import closure_components, joins, union_find_labels


# ---------------------------------------------------------------- back-fill

def _brute_backfill(ring, firing, H, W, s, wrap, cell_label):
    """Every (point, vertex) pair: the nearest vertex of the point's ring by firing
    distance (the shorter way round on a closed sweep), the earlier one on a tie."""
    Wp = W // s
    out = np.zeros(len(ring), np.int32)
    for p, (i, j) in enumerate(zip(ring, firing)):
        if i < 0:
            continue
        cands = []
        for k in range(Wp):
            lab = cell_label[k * H + i]
            if lab < 0:
                continue
            jk = k * s
            if wrap:
                back, fwd = (j - jk) % W, (jk - j) % W
            else:
                back = j - jk if jk <= j else None
                fwd = jk - j if jk >= j else None
            # (distance, 0 = reached going back along the sweep, 1 = going forward)
            options = [(d, side) for d, side in ((back, 0), (fwd, 1)) if d is not None]
            cands.append((min(options), lab))
        if cands:
            out[p] = min(cands)[1]
    return out


@pytest.mark.parametrize("H,W,s,wrap", [(2, 12, 3, 1), (3, 10, 2, 0), (1, 15, 5, 1), (2, 8, 1, 1), (3, 9, 3, 0)])
def test_backfill_equals_brute_force(H, W, s, wrap):
    rng = np.random.Generator(np.random.PCG64(H * 100 + W * 10 + s + wrap))
    Wp = W // s
    for trial in range(40):
        cell_label = np.where(rng.random(H * Wp) < 0.5, rng.integers(0, 5, H * Wp), -1).astype(np.int32)
        n = 30
        ring = rng.integers(-1, H, n).astype(np.int32)
        firing = np.where(ring >= 0, rng.integers(0, W, n), -1).astype(np.int32)
        got = oracle.backfill(ring, firing, H, W, s, wrap, cell_label)
        want = _brute_backfill(ring, firing, H, W, s, wrap, cell_label)
        assert np.array_equal(got, want), (trial, got, want)


def test_backfill_tie_takes_the_earlier_firing():
    # ring 0 of W=12, s=4: vertices at firings 0 (label 7) and 4 (label 9); the
    # point at firing 2 is equidistant and takes the earlier one, firing 3 the later
    H, W, s = 1, 12, 4
    cell_label = np.array([7, 9, -1], np.int32)
    lab = oracle.backfill(np.zeros(3, np.int32), np.array([2, 3, 1], np.int32), H, W, s, 0, cell_label)
    assert lab.tolist() == [7, 9, 7]


def test_backfill_across_the_seam_and_empty_rings():
    H, W, s = 2, 12, 3
    # ring 0: only the vertex at firing 0; ring 1: no vertex at all
    cell_label = np.array([5, -1, -1, -1, -1, -1, -1, -1], np.int32)
    ring = np.array([0, 0, 1, -1], np.int32)
    firing = np.array([11, 7, 4, -1], np.int32)
    closed = oracle.backfill(ring, firing, H, W, s, 1, cell_label)
    assert closed.tolist() == [5, 5, 0, 0]
    # on an open sweep firing 11 is still nearest to firing 0 (the only vertex)
    opened = oracle.backfill(ring, firing, H, W, s, 0, cell_label)
    assert opened.tolist() == [5, 5, 0, 0]


def test_point_cells_are_the_generating_rays():
    """Rays are fired at bin centres, so every used point's (ring, firing) is the
    generator's own (ring, column)."""
    f = synth.workload_frames("c1_16x1800")[0]
    sen = f.sensor
    ring, firing = oracle.point_cells(f.xyz, sen.n_rings, sen.n_azimuth, sen.elevations(), sen.az0)
    used = ring >= 0
    assert used.mean() > 0.5
    assert np.array_equal(ring[used], f.ring[used])
    assert np.array_equal(firing[used], f.col[used])


@pytest.mark.parametrize("s", [1, 5])
def test_point_labels_of_kept_points_and_sampled_columns(s):
    f = synth.workload_frames("paper_32x1800")[0]
    sen = f.sensor
    r = oracle.mesh_segment_frame(f, s=s, point_labels=True)
    # a kept point carries its vertex's label
    assert np.array_equal(r.point_labels[r.vertex_point], r.labels)
    # points in a sampled column that hold a vertex take that vertex's label
    ring, firing = oracle.point_cells(f.xyz, sen.n_rings, sen.n_azimuth, sen.elevations(), sen.az0)
    cell_label = np.full(sen.n_rings * (sen.n_azimuth // s), -1, np.int64)
    cp = oracle.bin_points(f.xyz, sen.n_rings, sen.n_azimuth, s, sen.elevations(), sen.az0)
    cell_label[cp >= 0] = r.labels
    sampled = (ring >= 0) & (firing % s == 0)
    c = (firing[sampled] // s) * sen.n_rings + ring[sampled]
    has = cell_label[c] >= 0
    assert np.array_equal(r.point_labels[sampled][has], cell_label[c][has])
    # unused points have label 0; with s = 1 every used point lies in a vertex's cell
    assert np.all(r.point_labels[ring < 0] == 0)
    if s == 1:
        assert np.all(r.point_labels[ring >= 0] > 0)


# ---------------------------------------------------------------- segment removal

@pytest.mark.parametrize("m", [0, 1, 2, 5, 40])
def test_prune_keeps_exactly_the_large_segments(m):
    f = synth.workload_frames("c1_16x1800")[0]
    full = oracle.mesh_segment_frame(f)
    pruned = oracle.mesh_segment_frame(f, min_segment=m)
    K = full.counts[2]
    size = np.bincount(full.labels, minlength=K + 1)
    keep = size[full.labels] >= max(m, 1)
    assert np.array_equal(pruned.labels[keep], full.labels[keep])
    assert np.all(pruned.labels[~keep] == 0)
    assert pruned.counts[2] == K
    if m <= 1:
        assert np.array_equal(pruned.labels, full.labels)


# ---------------------------------------------------------------- cosine test

@pytest.mark.parametrize("H,Wp,wrap", [(2, 3, 1), (3, 3, 1), (2, 4, 0), (3, 4, 0)])
def test_cosine_algorithm1_equals_connected_components(H, Wp, wrap):
    n = H * Wp
    rng = np.random.Generator(np.random.PCG64(n * 13 + wrap))
    cos_min = 0.9
    for bits in itertools.product([0, 1], repeat=n):
        valid = np.array(bits, np.uint8)
        # normals at multiples of 15 degrees in the x-y plane: dots are cos(15 m deg),
        # never near 0.9 (cos 15 = 0.966, cos 30 = 0.866)
        ang = rng.integers(0, 24, size=n) * (np.pi / 12)
        normals = np.stack([np.cos(ang), np.sin(ang), np.zeros(n)], axis=1).astype(np.float32)
        hasn = (rng.random(n) < 0.85).astype(np.uint8) & valid
        lab, K = oracle.labels(H, Wp, wrap, valid, hasn, normals, predicate=1, cos_min=cos_min)
        nodes = [c for c in range(n) if valid[c]]
        sim = []
        for e in joins(H, Wp, wrap, valid):
            a, b = tuple(e)
            if hasn[a] and hasn[b] and float(np.dot(normals[a].astype(np.float64), normals[b])) > cos_min:
                sim.append((a, b))
        uf, Kuf = union_find_labels(n, nodes, sim)
        assert K == Kuf and np.array_equal(lab, uf)
        R = closure_components(n, sim)
        for a in nodes:
            for b in nodes:
                assert (lab[a] == lab[b]) == bool(R[a, b])


@pytest.mark.parametrize("deg,joined", [(5.0, True), (9.9, True), (10.1, False), (30.0, False)])
def test_cosine_threshold_closed_form(deg, joined):
    """Two vertices on a strip with normals deg degrees apart, cos_min = cos 10 deg."""
    a = np.radians(deg)
    normals = np.float32([[0, 0, 1], [np.sin(a), 0, np.cos(a)]])
    valid = np.ones(2, np.uint8)
    lab, K = oracle.labels(1, 2, 0, valid, valid, normals, predicate=1, cos_min=np.cos(np.radians(10.0)))
    assert (K == 1) == joined


def test_cosine_separates_noise_free_faces():
    """Noise-free boxes on the ground: vertices with exact axis normals of different
    orientations (90 degrees apart) never share a segment at cos_min = cos 5 deg,
    and the interior of the ground plane is one segment."""
    sen = synth.Sensor.standard(32, 1024)
    f = synth.make_frame(sen, "boxes", 3, sigma=0.0, dropout=0.0)
    r = oracle.mesh_segment_frame(f, predicate=1, cos_min=float(np.cos(np.radians(5.0))))
    n = r.normals
    groups = {}
    for axis in range(3):
        for sign in (-1.0, 1.0):
            exact = (n[:, axis] == sign) & np.all(np.delete(n, axis, axis=1) == 0, axis=1)
            if exact.any():
                groups[(axis, sign)] = set(np.unique(r.labels[exact]).tolist())
    keys = list(groups)
    for a in range(len(keys)):
        for b in range(a + 1, len(keys)):
            assert not (groups[keys[a]] & groups[keys[b]]), (keys[a], keys[b])
    # ground (z = -1.7, normal -z) within 8 m: one segment
    v = r.vertices
    ground = (v[:, 2] == np.float32(-1.7)) & (np.hypot(v[:, 0], v[:, 1]) < 8.0) & (n[:, 2] == -1.0)
    assert len(np.unique(r.labels[ground])) == 1
