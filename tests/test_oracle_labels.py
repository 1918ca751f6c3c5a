"""Pins for the oracle's Algorithm 1 (Section 2, Segmentation by Surface Homogeneity).

Algorithm 1 floods from each unlabelled seed through neighbours whose normal
components all differ by less than the thresholds.  The test is symmetric, so
its label classes are the connected components of the graph (vertices, similar
joins); checked here against union-find and a transitive-closure brute force on
every validity mask of tiny lattices.
"""
import itertools

import numpy as np
import pytest

import oracle
import synth
from oracle_helpers import closure_components, joins, union_find_labels

THR = (0.2, 0.2, 0.2)


def _similar(a, b, na, nb, hasn):
    if not (hasn[a] and hasn[b]):
        return False
    return all(abs(float(na[c]) - float(nb[c])) < THR[c] for c in range(3))


@pytest.mark.parametrize("H,Wp,wrap", [(2, 3, 1), (3, 3, 1), (2, 4, 0), (3, 4, 1), (3, 4, 0), (2, 5, 1)])
def test_algorithm1_equals_connected_components_exhaustive(H, Wp, wrap):
    n = H * Wp
    rng = np.random.Generator(np.random.PCG64(n * 7 + wrap))
    masks = list(itertools.product([0, 1], repeat=n))
    for bits in masks:
        valid = np.array(bits, np.uint8)
        # normals on a 1/8 lattice: differences are multiples of 1/8, never near 0.2
        normals = (rng.integers(-8, 9, size=(n, 3)) / 8.0).astype(np.float32)
        hasn = (rng.random(n) < 0.85).astype(np.uint8) & valid
        lab, K = oracle.labels(H, Wp, wrap, valid, hasn, normals, THR)
        nodes = [c for c in range(n) if valid[c]]
        sim = [tuple(e) for e in joins(H, Wp, wrap, valid)
               if _similar(*tuple(e), normals[tuple(e)[0]], normals[tuple(e)[1]], hasn)]
        uf, Kuf = union_find_labels(n, nodes, sim)
        assert K == Kuf
        assert np.array_equal(lab, uf), (bits, lab, uf)
        R = closure_components(n, sim)
        for a in nodes:
            for b in nodes:
                assert (lab[a] == lab[b]) == bool(R[a, b])
        assert np.all(lab[valid == 0] == 0)


def test_labels_numbered_by_first_vertex_in_firing_order():
    H, Wp = 4, 6
    valid = np.ones(H * Wp, np.uint8)
    rng = np.random.Generator(np.random.PCG64(1))
    normals = (rng.integers(-2, 3, size=(H * Wp, 3)) / 2.0).astype(np.float32)
    lab, K = oracle.labels(H, Wp, 1, valid, valid, normals, THR)
    first = {}
    for c, l in enumerate(lab):
        first.setdefault(l, c)
    assert [l for l, _ in sorted(first.items(), key=lambda kv: kv[1])] == list(range(1, K + 1))


def test_vertex_without_normal_is_a_singleton():
    H, Wp = 3, 5
    valid = np.ones(H * Wp, np.uint8)
    normals = np.tile(np.float32([0, 0, -1]), (H * Wp, 1))
    hasn = valid.copy()
    hasn[7] = 0
    lab, K = oracle.labels(H, Wp, 1, valid, hasn, normals, THR)
    assert K == 2 and np.sum(lab == lab[7]) == 1


def test_threshold_is_strict():
    H, Wp = 1, 3
    valid = np.ones(3, np.uint8)
    normals = np.float32([[0, 0, 1], [0.25, 0, 1], [0.5, 0, 1]])
    # differences of exactly 0.25 (exact in binary): thr 0.25 is not enough, 0.2500001 is
    lab, K = oracle.labels(H, Wp, 0, valid, valid, normals, (0.25, 0.25, 0.25))
    assert K == 3
    lab, K = oracle.labels(H, Wp, 0, valid, valid, normals, (0.2500001, 0.2500001, 0.2500001))
    assert K == 1


def _interior(f, r, H, Wp):
    """Vertices whose incident triangles all lie on their own primitive."""
    prim = f.prim[r.vertex_point]
    inc = [[] for _ in range(r.vertices.shape[0])]
    for n, t in enumerate(r.triangles):
        for v in t:
            inc[v].append(n)
    out = []
    for v in range(r.vertices.shape[0]):
        if len(inc[v]) < 6:
            continue
        corners = {int(x) for t in inc[v] for x in r.triangles[t]}
        if all(prim[q] == prim[v] for q in corners):
            out.append(v)
    return np.array(out), prim


def _floating_boxes_frame():
    from synth.scene import Scene, cast, sample_frame
    sen = synth.Sensor.standard(64, 2048)
    sc = Scene()
    sc.ground_point = np.array([0.0, 0.0, -1000.0])   # no ground within range
    sc.boxes = [(6.0, 3.0, -1.0, 9.0, 6.5, 1.5), (-8.0, -9.0, -0.5, -5.0, -4.0, 2.0),
                (10.0, -3.0, -2.0, 12.0, -1.0, 0.5)]
    f = sample_frame(sen, sc, cast(sen, sc), sigma=0.0, dropout=0.0,
                     rng=np.random.Generator(np.random.PCG64(0)))
    return sen, f


def test_noise_free_floating_box_faces_are_distinct_segments():
    # Each visible face of a floating box is a plane with an exact constant normal;
    # adjacent faces differ by 1.0 in two components, so their interiors never merge.
    sen, f = _floating_boxes_frame()
    r = oracle.mesh_segment_frame(f)
    inner, prim = _interior(f, r, sen.n_rings, sen.n_azimuth)
    by_prim = {}
    for v in inner:
        by_prim.setdefault(int(prim[v]), set()).add(int(r.labels[v]))
    assert len(by_prim) == 6
    for p, labs in by_prim.items():
        assert len(labs) == 1, (p, labs)
    flat = [next(iter(l)) for l in by_prim.values()]
    assert len(set(flat)) == len(flat)


@pytest.mark.parametrize("kind,seed", [("walls", 5), ("ground", 1)])
def test_noise_free_planar_faces_interior_is_one_segment(kind, seed):
    # ground and walls: each plane's interior vertices share one label (creases may
    # chain ground and wall through blended vertices, so distinctness is not asserted)
    sen = synth.Sensor.standard(64, 2048)
    f = synth.make_frame(sen, kind, seed, sigma=0.0, dropout=0.0)
    r = oracle.mesh_segment_frame(f)
    inner, prim = _interior(f, r, sen.n_rings, sen.n_azimuth)
    by_prim = {}
    for v in inner:
        by_prim.setdefault(int(prim[v]), set()).add(int(r.labels[v]))
    assert len(by_prim) >= 1
    for p, labs in by_prim.items():
        assert len(labs) == 1, (p, labs)
