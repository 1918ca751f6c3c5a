"""Input generator: determinism, firing order, rays at lattice centres."""
import numpy as np

import synth


def test_same_seed_same_bytes():
    a = synth.workload_frames("c1_16x1800")[0]
    b = synth.workload_frames("c1_16x1800")[0]
    assert a.xyz.tobytes() == b.xyz.tobytes()
    assert np.array_equal(a.prim, b.prim)
    c = synth.workload_frames("c1_16x1800", base_seed=99)[0]
    assert c.xyz.shape != a.xyz.shape or c.xyz.tobytes() != a.xyz.tobytes()


def test_firing_order():
    f = synth.workload_frames("c1_16x1800")[0]
    key = f.col.astype(np.int64) * f.sensor.n_rings + f.ring
    assert np.all(np.diff(key) > 0)


def test_points_lie_on_their_rays():
    f = synth.workload_frames("c2_64x2048")[0]
    U = f.sensor.rays()[f.ring, f.col]
    p = f.xyz.astype(np.float64)
    r = np.linalg.norm(p, axis=1)
    cosang = np.einsum("ij,ij->i", p, U) / r
    assert np.all(cosang > 1 - 1e-12)


def test_noise_free_axis_faces_snap():
    sen = synth.Sensor.standard(16, 512)
    f = synth.make_frame(sen, "ground", 3, sigma=0.0, dropout=0.0)
    assert np.all(f.xyz[:, 2] == np.float32(-1.7))


def test_batch_shapes_are_uneven():
    sens = synth.batch_sensors(64, 5)
    assert {s.n_rings for s in sens} == {16, 32, 64, 128}
    assert {s.n_azimuth for s in sens} == {1024, 2048, 4096}
