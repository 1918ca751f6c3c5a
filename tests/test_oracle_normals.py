"""Pins for the oracle's normals (Section 2, Normal Estimation).

What geometry fixes:
  * noise-free axis-aligned planes: the normal is exactly +-axis (each edge has an
    exactly-zero component there, so every cross product has two exact zeros);
  * spheres: each incident triangle's normal lies at asin(R_circ / rho) from the
    radial line, and a positively weighted sum stays inside that cone;
  * every triangle normal satisfies N . p > 0 (lattice orientation), so every
    vertex normal does too;
  * a closed form for mutually orthogonal edge vectors pins the pairing and the
    1/(|V_t| + |V_t+1|) weighting (tests/golden/normal_weighting.json);
  * a closed form for a full six-neighbour star with axis-aligned edges of
    distinct lengths (also rotated exactly) pins all six pairs, their cyclic
    order, the closing pair F x A and the weight of each.
"""
import json
import math
import os

import numpy as np
import pytest

import oracle
import synth
from synth.scene import PRIM_OBJ_BASE

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _run(f, s=1, **kw):
    return oracle.mesh_segment_frame(f, s=s, **kw)


def _incident(tri, V):
    inc = [[] for _ in range(V)]
    for n, t in enumerate(tri):
        for v in t:
            inc[v].append(n)
    return inc


def test_weighting_closed_form():
    # Anchor p at ring 0, column 1 of a 2 x 4 open lattice; only A=(1,1), B=(1,2),
    # C=(0,2) present, so the incident pairs are (A,B) and (B,C).  With
    # V_A = a e1, V_B = b e2, V_C = c e3:  A x B / (a+b) + B x C / (b+c)
    #   = (bc/(b+c), 0, ab/(a+b)).
    g = json.load(open(os.path.join(GOLDEN, "normal_weighting.json")))
    for case in g["cases"]:
        a, b, c = case["a"], case["b"], case["c"]
        p = np.array(case["p"], np.float64)
        H, Wp = 2, 4
        cell = lambda i, k: k * H + i  # noqa: E731
        xyz = np.zeros((H * Wp, 3), np.float32)
        valid = np.zeros(H * Wp, np.uint8)
        for (i, k), q in [((0, 1), p), ((1, 1), p + [a, 0, 0]), ((1, 2), p + [0, b, 0]),
                          ((0, 2), p + [0, 0, c])]:
            xyz[cell(i, k)] = q
            valid[cell(i, k)] = 1
        n, h = oracle.normals(H, Wp, 0, xyz, valid)
        assert h[cell(0, 1)] == 1
        np.testing.assert_allclose(n[cell(0, 1)], case["expected_normal"], rtol=0, atol=1e-15)


SIX_LENGTHS = [(1, 2, 3, 4, 5, 6), (6, 1, 5, 2, 4, 3), (1, 1, 1, 1, 1, 1), (2, 7, 1, 8, 2, 8)]
# Rotations with rational entries (3-4-5 about z, 5-12-13 about x), so that
# lattice coordinates that are multiples of 65 stay integers after rotation.
ROT_Z = np.array([[3, -4, 0], [4, 3, 0], [0, 0, 5]], np.float64) / 5.0
ROT_X = np.array([[13, 0, 0], [0, 5, -12], [0, 12, 5]], np.float64) / 13.0


@pytest.mark.parametrize("lengths", SIX_LENGTHS)
@pytest.mark.parametrize("rot", ["none", "z", "xz"])
def test_weighting_closed_form_all_six_pairs(lengths, rot):
    # Anchor p at ring 1, column 1 of a 3 x 3 open lattice with all six
    # neighbours, named in the anticlockwise order of Section 2: A = (2,1),
    # B = (2,2), C = (1,2), D = (0,1), E = (0,0), F = (1,0) (ring, column).
    # With V_A = a e1, V_B = b e2, V_C = c e3, V_D = -d e1, V_E = -e e2,
    # V_F = -f e3 the six consecutive products are
    #   A x B = ab e3, B x C = bc e1, C x D = -cd e2,
    #   D x E = de e3, E x F = ef e1, F x A = -fa e2,
    # so the weighted sum is
    #   (bc/(b+c) + ef/(e+f), -(cd/(c+d) + fa/(f+a)), ab/(a+b) + de/(d+e)).
    # A proper rotation R of every edge rotates each product and keeps every
    # length, so the normal of the rotated star is R n.  Every pair, its order,
    # its sign and its weight enter one component; dropping the closing pair
    # F x A, permuting the neighbours or changing the weight moves the result
    # far beyond the tolerance.
    a, b, c, d, e, f = (65.0 * x for x in lengths)
    s = np.array([b * c / (b + c) + e * f / (e + f),
                  -(c * d / (c + d) + f * a / (f + a)),
                  a * b / (a + b) + d * e / (d + e)])
    R = {"none": np.eye(3), "z": ROT_Z, "xz": ROT_X @ ROT_Z}[rot]
    expected = R @ (s / np.linalg.norm(s))
    p = np.array([1300.0, -650.0, 390.0])
    H, Wp = 3, 3
    cell = lambda i, k: k * H + i  # noqa: E731
    xyz = np.zeros((H * Wp, 3), np.float32)
    valid = np.zeros(H * Wp, np.uint8)
    star = [((1, 1), [0, 0, 0]), ((2, 1), [a, 0, 0]), ((2, 2), [0, b, 0]), ((1, 2), [0, 0, c]),
            ((0, 1), [-d, 0, 0]), ((0, 0), [0, -e, 0]), ((1, 0), [0, 0, -f])]
    for (i, k), v in star:
        q = p + R @ np.array(v, np.float64)
        assert np.all(q == np.round(q)) and np.all(np.abs(q) < 2 ** 24)  # exact in FP32
        xyz[cell(i, k)] = q
        valid[cell(i, k)] = 1
    n, h = oracle.normals(H, Wp, 0, xyz, valid)
    assert h[cell(1, 1)] == 1
    np.testing.assert_allclose(n[cell(1, 1)], expected, rtol=0, atol=1e-14)


def test_noise_free_ground_normals_are_exact():
    sen = synth.Sensor.standard(32, 1024)
    f = synth.make_frame(sen, "ground", 2, sigma=0.0, dropout=0.0)
    r = _run(f)
    has = np.any(r.normals64 != 0, axis=1)
    assert has.sum() > 0.9 * r.vertices.shape[0]
    assert np.all(r.normals64[has] == [0.0, 0.0, -1.0])
    assert np.all(r.normals[has] == np.float32([0.0, 0.0, -1.0]))


@pytest.mark.parametrize("kind,seed", [("boxes", 3), ("walls", 4), ("boxes", 8)])
def test_noise_free_axis_faces_are_exact(kind, seed):
    sen = synth.Sensor.standard(64, 2048)
    f = synth.make_frame(sen, kind, seed, sigma=0.0, dropout=0.0)
    r = _run(f)
    prim = f.prim[r.vertex_point]
    inc = _incident(r.triangles, r.vertices.shape[0])
    cr = synth.cast(sen, f.scene)
    # axis of each primitive from the caster (-1 when not an axis-aligned plane)
    sax = cr[2][f.ring[r.vertex_point], f.col[r.vertex_point]]
    checked = 0
    for v in range(r.vertices.shape[0]):
        if not inc[v] or sax[v] < 0:
            continue
        corners = {int(x) for t in inc[v] for x in r.triangles[t]}
        if any(prim[q] != prim[v] for q in corners):
            continue
        ax = int(sax[v])
        exp = np.zeros(3)
        exp[ax] = math.copysign(1.0, r.vertices[v, ax])
        assert np.array_equal(r.normals64[v], exp), (v, r.normals64[v], exp)
        checked += 1
    assert checked > 1000


def test_sphere_normals_lie_in_the_circumcentre_cone():
    sen = synth.Sensor.standard(128, 4096)
    f = synth.make_frame(sen, "spheres", 5, sigma=0.0, dropout=0.0)
    r = _run(f)
    prim = f.prim[r.vertex_point]
    inc = _incident(r.triangles, r.vertices.shape[0])
    V = r.vertices.astype(np.float64)
    checked = 0
    for v in range(V.shape[0]):
        sid = prim[v] - PRIM_OBJ_BASE
        if sid < 0 or not inc[v]:
            continue
        corners = {int(x) for t in inc[v] for x in r.triangles[t]}
        if any(prim[q] != prim[v] for q in corners):
            continue
        cx, cy, cz, rho = f.scene.spheres[sid]
        O = np.array([cx, cy, cz])
        bound = 0.0
        for t in inc[v]:
            a, b, c = V[r.triangles[t]]
            la, lb, lc = np.linalg.norm(b - c), np.linalg.norm(a - c), np.linalg.norm(a - b)
            area = 0.5 * np.linalg.norm(np.cross(b - a, c - a))
            Rc = la * lb * lc / (4 * area)
            # the points sit on the sphere only to float32 rounding: use the vertex's radius
            bound = max(bound, math.asin(min(1.0, Rc / np.linalg.norm(V[v] - O))))
        u = O - V[v]
        n = r.normals64[v]
        ang = math.atan2(np.linalg.norm(np.cross(n, u)), float(n @ u))
        # float32 coordinates (~1e-6 m rounding at these ranges) over 5-20 cm edges
        # tilt each triangle's plane by up to ~2e-5 rad relative to the true sphere
        assert ang <= bound + 5e-5, (v, ang, bound)
        checked += 1
    assert checked > 500


@pytest.mark.parametrize("name,s", [("c1_16x1800", 1), ("c2_64x2048", 2), ("c4_128x4096", 2)])
def test_normal_invariants_on_noisy_frames(name, s):
    f = synth.workload_frames(name)[0]
    r = _run(f, s=s)
    inc = _incident(r.triangles, r.vertices.shape[0])
    has = np.any(r.normals64 != 0, axis=1)
    has_tri = np.array([len(x) > 0 for x in inc])
    assert np.array_equal(has, has_tri)
    n = r.normals64[has]
    np.testing.assert_allclose(np.linalg.norm(n, axis=1), 1.0, atol=1e-12)
    assert np.all(np.einsum("ij,ij->i", n, r.vertices[has].astype(np.float64)) > 0)
    # float32 output is the FP64 normal rounded once
    assert np.array_equal(r.normals, r.normals64.astype(np.float32))
