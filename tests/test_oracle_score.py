"""Pins for the oracle's edge scores, the accuracy measure of the evaluation
(Section 3: segment edge points and ground-truth edge points, each dilated,
compared by precision, recall and F1).

  * brute force on tiny lattices: edges from the forward-join rule alone and
    the dilation as an explicit set of lattice cells within R steps;
  * closed forms: a straight boundary between two column blocks, moved by d
    columns, is found exactly when d - 1 <= R (inner column) and d <= R (outer);
  * a closed sweep cut into two halves has two boundaries;
  * identical partitions (under any renaming of the ids) score 1, a single
    segment finds no edge at all.
"""
import numpy as np
import pytest

import oracle
import synth
from oracle_helpers import joins


def _brute(H, Wp, wrap, label, truth, R):
    valid = label >= 0
    seg, tru = set(), set()
    for e in joins(H, Wp, wrap, valid):
        a, b = tuple(e)
        if label[a] != label[b]:
            seg |= {a, b}
        if truth[a] != truth[b]:
            tru |= {a, b}

    def dilate(S):
        out = set()
        for c in S:
            k, i = divmod(c, H)
            for dk in range(-R, R + 1):
                kk = k + dk
                if wrap:
                    kk %= Wp
                elif not 0 <= kk < Wp:
                    continue
                for di in range(-R, R + 1):
                    if 0 <= i + di < H:
                        out.add(kk * H + i + di)
        return out

    return len(seg), len(tru), len(seg & dilate(tru)), len(tru & dilate(seg))


@pytest.mark.parametrize("H,Wp,wrap", [(3, 4, 0), (3, 5, 1), (1, 6, 1), (4, 3, 1), (5, 7, 0), (2, 9, 1)])
def test_edge_scores_equal_brute_force(H, Wp, wrap):
    rng = np.random.Generator(np.random.PCG64(H * 31 + Wp * 7 + wrap))
    for trial in range(60):
        n = H * Wp
        occ = rng.random(n) < 0.8
        label = np.where(occ, rng.integers(1, 4, n), -1).astype(np.int32)
        truth = rng.integers(0, 3, n).astype(np.int32)
        R = int(rng.integers(0, 4))
        got = oracle.edge_scores(H, Wp, wrap, label, truth, R)
        assert got == _brute(H, Wp, wrap, label, truth, R), (trial, R)


@pytest.mark.parametrize("d", [1, 2, 3])
@pytest.mark.parametrize("R", [0, 1, 2, 3])
def test_shifted_boundary_closed_form(d, R):
    H, Wp, m = 5, 12, 4
    col = np.repeat(np.arange(Wp), H)
    truth = (col >= m).astype(np.int32) + 7
    label = (col >= m + d).astype(np.int32) + 1
    n_seg, n_tru, found, recalled = oracle.edge_scores(H, Wp, 0, label, truth, R)
    assert n_seg == n_tru == 2 * H
    want = H * int(d - 1 <= R) + H * int(d <= R)
    assert found == recalled == want


def test_closed_sweep_has_two_boundaries():
    H, Wp = 3, 10
    col = np.repeat(np.arange(Wp), H)
    label = (col >= Wp // 2).astype(np.int32)
    closed = oracle.edge_scores(H, Wp, 1, label, label, 0)
    opened = oracle.edge_scores(H, Wp, 0, label, label, 0)
    assert closed == (4 * H,) * 4
    assert opened == (2 * H,) * 4


def test_identical_partitions_and_single_segment():
    f = synth.workload_frames("c1_16x1800")[0]
    sen = f.sensor
    r = oracle.mesh_segment_frame(f)
    cp = oracle.bin_points(f.xyz, sen.n_rings, sen.n_azimuth, 1, sen.elevations(), sen.az0)
    truth = f.prim[cp[cp >= 0]]
    # the truth, renamed, as the segmentation: every edge found and recalled at R = 0
    renamed = (truth * 7 + 3).astype(np.int32)
    c = oracle.frame_edge_scores(f.xyz, f.prim, sen.n_rings, sen.n_azimuth, 1, sen.elevations(), renamed,
                                 az0=sen.az0, radius=0)
    assert c[0] == c[1] == c[2] == c[3] > 0
    assert oracle.precision_recall_f1(c) == (1.0, 1.0, 1.0)
    # one segment: no segment edge, nothing recalled
    one = np.ones_like(r.labels)
    c1 = oracle.frame_edge_scores(f.xyz, f.prim, sen.n_rings, sen.n_azimuth, 1, sen.elevations(), one,
                                  az0=sen.az0, radius=2)
    assert c1[0] == 0 and c1[2] == 0 and c1[3] == 0 and c1[1] == c[1]
    assert oracle.precision_recall_f1(c1) == (0.0, 0.0, 0.0)
    # a larger radius never scores fewer hits
    prev = None
    for R in range(4):
        cr = oracle.frame_edge_scores(f.xyz, f.prim, sen.n_rings, sen.n_azimuth, 1, sen.elevations(), r.labels,
                                      az0=sen.az0, radius=R)
        if prev is not None:
            assert cr[:2] == prev[:2] and cr[2] >= prev[2] and cr[3] >= prev[3]
        prev = cr


def test_precision_recall_f1_closed_form():
    assert oracle.precision_recall_f1((10, 20, 5, 10)) == (0.5, 0.5, 0.5)
    p, r, f = oracle.precision_recall_f1((4, 8, 3, 2))
    assert (p, r) == (0.75, 0.25) and abs(f - 2 * 0.75 * 0.25 / 1.0) < 1e-15
    assert oracle.precision_recall_f1((0, 0, 0, 0)) == (1.0, 1.0, 1.0)
