"""Pin: the oracle's ring and firing decisions for returns placed within
1e-13 .. 1e-3 rad of the decision boundaries (ring midpoints, half-firing
azimuths, the atan2 branch cut, az0 anywhere in [-2 pi, 2 pi]) equal the
decisions taken independently in x87 extended precision (64-bit significand,
long double atan2 and sqrt of the exact float32 coordinates, exact pi).

The binning reading is: the ring of nearest elevation (tie: lower index) and
the firing round((phi - az0) / (2 pi / W)) mod W, round half away from zero
(Section 2, opening paragraph, P = {p(theta, phi, r)} on the sensor's lattice).
At these distances from a boundary FP64 and extended precision agree, so any
slip in the oracle's definition (a sign, an offset of half a firing, a wrong
tie side, az0 applied the wrong way) fails here."""
import math

import numpy as np
import pytest

import oracle
from binning_inputs import elevation_table, off_lattice_sweep

LD = np.longdouble
CASES = [(16, 1800, 0.0, "uniform"), (32, 1800, 2 * math.pi - 1e-3, "irregular"),
         (64, 16385, -2 * math.pi + 1e-3, "uniform"), (128, 4096, 0.37, "irregular")]


def _extended_decisions(xyz, H, W, elev, az0, r_min=1.0, r_max=60.0):
    if np.finfo(LD).nmant < 63:
        pytest.skip("long double is not the x87 extended format here")
    x, y, z = (xyz[:, k].astype(LD) for k in range(3))
    r2 = x * x + y * y + z * z
    used = np.isfinite(r2) & (r2 >= LD(r_min) ** 2) & (r2 <= LD(r_max) ** 2)
    el = np.arctan2(z, np.sqrt(x * x + y * y))
    d = np.abs(el[:, None] - elev.astype(LD)[None, :])
    ring = np.argmin(d, axis=1).astype(np.int32)              # first (upper) ring on a tie
    pi = np.arctan2(LD(0), LD(-1))
    jf = (np.arctan2(y, x) - LD(az0)) / (2 * pi / W)
    j = np.floor(np.abs(jf) + LD(0.5)) * np.sign(jf)          # round half away from zero
    firing = (j.astype(np.int64) % W).astype(np.int32)
    return np.where(used, ring, -1), np.where(used, firing, -1)


@pytest.mark.parametrize("H,W,az0,kind", CASES)
def test_oracle_bins_boundary_returns_as_extended_precision(H, W, az0, kind):
    el = elevation_table(H, kind, seed=H)
    xyz, tag = off_lattice_sweep(H, W, az0, el, seed=W + H, n_boundary=6000, dense=False)
    ring, firing = oracle.point_cells(xyz, H, W, el, az0, 1.0, 60.0)
    want_r, want_f = _extended_decisions(xyz, H, W, el, az0)
    assert np.array_equal(ring < 0, want_r < 0)
    bad = np.flatnonzero((ring != want_r) | (firing != want_f))
    assert bad.size == 0, (bad[:5], ring[bad[:5]], want_r[bad[:5]], firing[bad[:5]], want_f[bad[:5]], tag[bad[:5]])
    # the boundary returns are there: both sides of ring midpoints and of half firings
    assert (tag == 1).sum() > 5000 and (tag == 2).sum() > 5000
