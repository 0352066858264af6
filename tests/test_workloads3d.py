"""Host-side checks of the three-dimensional input generators: the round
nozzle's bore, wall classes and open-row validity, and the sphere distance."""
import math

import numpy as np

import workloads as W


def test_round_nozzle_geometry():
    nx, ny, nz, r, L = 64, 40, 48, 10.0, 16
    w = W.round_nozzle_wall3d(nx, ny, nz, r, L)
    assert w.shape == (ny, nz, nx)
    sec = w[0]
    bore = sec == W.FLUID
    # the bore is the disc of radius r about the section centre
    assert abs(bore.sum() - math.pi * r * r) < 2 * math.pi * r
    zc, xc = (nz - 1) / 2, (nx - 1) / 2
    zz, xx = np.nonzero(bore)
    assert np.all((xx - xc) ** 2 + (zz - zc) ** 2 < r * r)
    # mirror symmetric about the centre in x and in z
    assert np.array_equal(sec, sec[::-1, :]) and np.array_equal(sec, sec[:, ::-1])
    # inner wall: exactly the solid nodes with a bore node among their 8 section neighbours
    near = np.zeros_like(bore)
    for dz in (-1, 0, 1):
        for dx in (-1, 0, 1):
            near |= np.roll(np.roll(bore, dz, 0), dx, 1)
    assert np.array_equal(sec == W.WALL_INNER, near & ~bore)
    assert np.all(w[:L] == sec[None]) and np.all(w[L:] == W.FLUID)


def test_round_nozzle_presets_respect_the_open_row_rule():
    for c in (W.config_round_nozzle_small(), W.config_round_nozzle_eject()):
        w, p = c["wall"], c["params"]
        assert p["bc_y"] == W.BC_OPEN
        # a fluid node of row 0 (ny-1) has fluid directly above (below) it
        assert not np.any((w[0] == W.FLUID) & (w[1] != W.FLUID))
        assert not np.any((w[-1] == W.FLUID) & (w[-2] != W.FLUID))
        assert p["gamma"] * p["sigma"] <= 0.005 + 1e-12   # the 3-D stability reading


def test_spheres_distance_periodic_and_not():
    n = 20
    d = W.spheres_distance3d(n, n, n, [(1.0, 1.0, 1.0, 4.0)])
    # nearest image: the node at (n-1, n-1, n-1) is sqrt(12) from the centre
    assert abs(d[n - 1, n - 1, n - 1] - (4.0 - math.sqrt(12.0))) < 1e-12
    d2 = W.spheres_distance3d(n, n, n, [(1.0, 1.0, 1.0, 4.0)], periodic_y=False)
    # without the y image the same node is (2, 18, 2) away in (x, y, z)
    assert abs(d2[n - 1, n - 1, n - 1] - (4.0 - math.sqrt(2 * 2 + 18 * 18 + 2 * 2))) < 1e-12
