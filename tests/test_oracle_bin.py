"""Pins for the oracle's binning and sub-sampling (Section 2, opening paragraph;
Mesh Construction's 'within range of the Lidar')."""
import math

import numpy as np
import pytest

import oracle
import synth


def _expected_cells(f, s):
    H = f.sensor.n_rings
    Wp = f.sensor.n_azimuth // s
    exp = np.full(H * Wp, -1, dtype=np.int64)
    keep = f.col % s == 0
    idx = np.nonzero(keep)[0]
    exp[(f.col[keep] // s) * H + f.ring[keep]] = idx
    return exp


@pytest.mark.parametrize("name", ["c1_16x1800", "c2_64x2048"])
def test_generated_points_land_in_their_lattice_cells(name):
    # The generator knows which (ring, firing) produced each point: binning must
    # recover it exactly (rays sit at lattice centres, half a bin from any boundary).
    f = synth.workload_frames(name)[0]
    sen = f.sensor
    cp = oracle.bin_points(f.xyz, sen.n_rings, sen.n_azimuth, 1, sen.elevations(),
                           r_min=0.5, r_max=500.0)
    assert np.array_equal(cp, _expected_cells(f, 1))


@pytest.mark.parametrize("s", [2, 4, 5])
def test_subsampling_keeps_every_sth_firing(s):
    sen = synth.Sensor.standard(32, 1800 if s == 5 else 2048)
    f = synth.make_frame(sen, "street", 11, sigma=0.01, dropout=0.1)
    cp = oracle.bin_points(f.xyz, sen.n_rings, sen.n_azimuth, s, sen.elevations(),
                           r_min=0.5, r_max=500.0)
    assert np.array_equal(cp, _expected_cells(f, s))


def test_range_window_is_inclusive():
    xyz = np.array([[3, 4, 0], [0, 6, 8.0]], dtype=np.float32)  # r = 5 exactly at 0 deg; r = 10 at 90 deg
    W = 360
    cp = oracle.bin_points(xyz, 1, W, 1, [0.0], r_min=5.0, r_max=10.0)
    assert sorted(cp[cp >= 0].tolist()) == [0, 1]
    cp = oracle.bin_points(xyz, 1, W, 1, [0.0], r_min=np.nextafter(5.0, 6.0), r_max=10.0)
    assert sorted(cp[cp >= 0].tolist()) == [1]
    cp = oracle.bin_points(xyz, 1, W, 1, [0.0], r_min=5.0, r_max=np.nextafter(10.0, 0.0))
    assert sorted(cp[cp >= 0].tolist()) == [0]


def test_collision_nearest_return_then_lower_index():
    d = np.array([1.0, 0.0, 0.0])
    xyz = np.array([10 * d, 7 * d, 7 * d, 8 * d], dtype=np.float32)
    cp = oracle.bin_points(xyz, 1, 8, 1, [0.0], r_min=1.0, r_max=60.0)
    assert cp[0] == 1 and np.all(cp[1:] == -1)


def test_non_finite_points_are_skipped():
    f = synth.workload_frames("c1_16x1800")[0]
    sen = f.sensor
    xyz = f.xyz.copy()
    bad = [5, 77, 1000]
    xyz[5, 0] = np.nan
    xyz[77, 2] = np.inf
    xyz[1000, 1] = -np.inf
    cp = oracle.bin_points(xyz, sen.n_rings, sen.n_azimuth, 1, sen.elevations(), r_min=0.5, r_max=500)
    exp = _expected_cells(f, 1)
    for b in bad:
        exp[exp == b] = -1
    assert np.array_equal(cp, exp)


def test_permutation_invariance():
    f = synth.workload_frames("c1_16x1800")[0]
    sen = f.sensor
    rng = np.random.Generator(np.random.PCG64(5))
    perm = rng.permutation(f.n_points)
    cp = oracle.bin_points(f.xyz, sen.n_rings, sen.n_azimuth, 1, sen.elevations())
    cq = oracle.bin_points(f.xyz[perm], sen.n_rings, sen.n_azimuth, 1, sen.elevations())
    mapped = np.where(cq >= 0, perm[np.maximum(cq, 0)], -1)
    assert np.array_equal(mapped, cp)


def test_azimuth_seam_and_rounding():
    W = 360
    step = 2 * math.pi / W

    def pt(phi):
        return [20 * math.cos(phi), 20 * math.sin(phi), 0.0]

    cases = {-0.3 * step: 0, 2 * math.pi - 0.4 * step: 0, 0.6 * step: 1, 359.4 * step: 359,
             180.45 * step: 180, 180.55 * step: 181}
    xyz = np.array([pt(p) for p in cases], dtype=np.float32)
    for n, (phi, col) in enumerate(cases.items()):
        cp = oracle.bin_points(xyz[n:n + 1], 1, W, 1, [0.0])
        assert np.nonzero(cp >= 0)[0].tolist() == [col], (phi, col)


def test_ring_is_nearest_elevation():
    elev = np.radians([10.0, 0.0, -10.0])
    W = 4
    # elevations 6 deg -> ring 0, 4 deg -> ring 1, -4.9 -> ring 1, -5.1 -> ring 2, 40 -> ring 0
    for deg, ring in [(6.0, 0), (4.0, 1), (-4.9, 1), (-5.1, 2), (40.0, 0), (-60.0, 2)]:
        e = math.radians(deg)
        xyz = np.array([[10 * math.cos(e), 0.0, 10 * math.sin(e)]], dtype=np.float32)
        cp = oracle.bin_points(xyz, 3, W, 1, elev)
        assert np.nonzero(cp >= 0)[0].tolist() == [ring], deg


def test_ring_tie_goes_to_the_upper_ring():
    # elevations +a and -a: a point at elevation exactly 0 is equidistant (exactly)
    a = math.radians(1.0)
    xyz = np.array([[10.0, 0.0, 0.0]], dtype=np.float32)
    cp = oracle.bin_points(xyz, 2, 8, 1, np.array([a, -a]))
    assert np.nonzero(cp >= 0)[0].tolist() == [0]


# ---------------------------------------------------------------- reported rings

def test_reported_rings_equal_to_the_generating_ones_change_nothing():
    f = synth.workload_frames("c2_64x2048")[0]
    sen = f.sensor
    by_elev = oracle.bin_points(f.xyz, sen.n_rings, sen.n_azimuth, 2, sen.elevations(), r_min=0.5, r_max=500.0)
    given = oracle.bin_points(f.xyz, sen.n_rings, sen.n_azimuth, 2, sen.elevations(), r_min=0.5, r_max=500.0,
                              ring_ids=f.ring.astype(np.uint8))
    assert np.array_equal(given, by_elev)


def test_reported_rings_decide_the_ring_alone():
    """A relabelled ring map moves every point to its reported ring (in its own
    firing), whatever the elevation table says; a ring beyond the lattice drops
    the point."""
    f = synth.workload_frames("c1_16x1800")[0]
    sen = f.sensor
    H, W = sen.n_rings, sen.n_azimuth
    rng = np.random.Generator(np.random.PCG64(5))
    perm = rng.permutation(H)
    reported = perm[f.ring].astype(np.uint8)
    out_of_range = rng.random(f.n_points) < 0.05
    reported[out_of_range] = H + 3
    # a different (still descending) elevation table must not matter
    fake_elev = np.linspace(0.5, -0.5, H)
    cp = oracle.bin_points(f.xyz, H, W, 1, fake_elev, r_min=0.5, r_max=500.0, ring_ids=reported)
    exp = np.full(H * W, -1, dtype=np.int64)
    keep = ~out_of_range
    exp[f.col[keep] * H + reported[keep]] = np.nonzero(keep)[0]
    assert np.array_equal(cp, exp)
    ring, firing = oracle.point_cells(f.xyz, H, W, fake_elev, r_min=0.5, r_max=500.0, ring_ids=reported)
    assert np.array_equal(ring[keep], reported[keep].astype(np.int32))
    assert np.array_equal(firing[keep], f.col[keep])
    assert np.all(ring[out_of_range] == -1)


def test_reported_rings_through_the_whole_path():
    f = synth.workload_frames("paper_32x1800")[0]
    sen = f.sensor
    a = oracle.mesh_segment_frame(f, s=5)
    b = oracle.mesh_segment_frame(f, s=5, ring_ids=f.ring.astype(np.uint8))
    assert np.array_equal(a.vertices, b.vertices) and np.array_equal(a.labels, b.labels)
    assert np.array_equal(a.triangles, b.triangles)
