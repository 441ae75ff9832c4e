"""Host pieces of the rigid-against-elastic wall shear stress comparison:
the wall-site selection against a brute-force scan, and the pointwise
statistics on known inputs.  No GPU."""
import numpy as np

from paper_2108_08783_amd import inputs, wall_shear


def test_wall_sites_match_a_brute_force_scan():
    rng = np.random.default_rng(5)
    g = inputs.random_labels((9, 10, 11), rng)
    lab = g.labels
    nz, ny, nx = lab.shape
    want = []
    k = 0
    for z in range(nz):
        for y in range(ny):
            for x in range(nx):
                if lab[z, y, x] != inputs.FLUID:
                    continue
                if any(lab[z - dz, y - dy, x - dx] == inputs.WALL
                       for dx, dy, dz in inputs._OFFS18):
                    want.append(k)
                k += 1
    assert np.array_equal(wall_shear.wall_sites(g), np.array(want))


def test_compare_statistics():
    b = np.array([1.0, 2.0, 4.0, 0.0])
    a = np.array([0.5, 2.5, 2.0, 9.0])
    s = wall_shear.compare(a, b, floor=0.1)
    assert s["sites"] == 3
    assert s["frac_lower"] == 2 / 3
    assert s["median_ratio"] == 0.5
    assert abs(s["slope"] - (0.5 + 5 + 8) / 21) < 1e-15
