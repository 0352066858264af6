"""Pins of the three-dimensional FP64 oracle (D3Q19 f, D3Q7 g).

The strongest pin is the reduction to two dimensions: summed along one axis,
D3Q19 has the D2Q9 weights and D3Q7 the D2Q5 ones, so a state and geometry
that do not vary along z (or along x) must evolve exactly, up to rounding, as
the already pinned two-dimensional oracle, walls, wetting ghosts, open rows,
per-phase relaxation and the force pulse included.  The other pins fix what
the projection cannot see: the lattice moments, the exchange of x and z
(rotation symmetry), exact conservation and the force impulse in full 3-D, and
the three-dimensional Laplace law."""
import numpy as np
import pytest

import workloads as W

# D2Q9 of the two-dimensional oracle: c_0..c_8
EX2 = np.array([0, 1, 0, -1, 0, 1, -1, -1, 1])
EY2 = np.array([0, 0, 1, 0, -1, 1, 1, -1, -1])


def test_velocity_set_moments(oracle3d_mod):
    """Isotropy of D3Q19 up to fourth order, opposites, and D3Q7 = rest + axes."""
    c, w, opp = oracle3d_mod.velocity_set()
    assert len({tuple(v) for v in c}) == 19 and np.all(np.abs(c).sum(1) <= 2)
    assert w.sum() == pytest.approx(1.0, abs=1e-15)
    d = np.eye(3)
    assert np.allclose(np.einsum("i,ia->a", w, c), 0, atol=1e-15)
    assert np.allclose(np.einsum("i,ia,ib->ab", w, c, c), d / 3, atol=1e-15)
    assert np.allclose(np.einsum("i,ia,ib,ic->abc", w, c, c, c), 0, atol=1e-15)
    t4 = (np.einsum("ab,cd->abcd", d, d) + np.einsum("ac,bd->abcd", d, d) + np.einsum("ad,bc->abcd", d, d)) / 9
    assert np.allclose(np.einsum("i,ia,ib,ic,id->abcd", w, c, c, c, c), t4, atol=1e-15)
    assert np.all(c[opp] == -c)
    assert np.all(c[0] == 0) and sorted(map(tuple, c[1:7])) == sorted(map(tuple, np.vstack([d, -d]).astype(int)))


def _project(a3, c3, axis_keep, e2x, e2y):
    """Sum 3-D populations over the velocities whose in-plane components are
    (e2x[j], e2y[j]); axis_keep names the 3-D axis (0 = x, 2 = z) that plays
    the two-dimensional x."""
    out = []
    for j in range(len(e2x)):
        sel = [i for i in range(len(a3)) if c3[i, axis_keep] == e2x[j] and c3[i, 1] == e2y[j]]
        out.append(sum(a3[i] for i in sel))
    return np.array(out)


def _nozzle2d(nx, ny):
    x0, w, L = nx // 4, nx // 2, ny // 3
    p = W.base_params(nx, ny, force_rows=L, t_pos=60, t_neg=30, t_idle=1000, f_pos=1e-3, f_neg=5e-4,
                      tau_ink=0.8, theta_inner=60.0, theta_outer=120.0)
    return p, W.nozzle_wall(nx, ny, x0, w, L), W.meniscus_distance(nx, ny, L) + \
        0.3 * np.sin(2 * np.pi * np.arange(nx) / nx)[None, :]


@pytest.mark.parametrize("axis", ["z", "x"])
def test_invariant_state_reduces_to_the_2d_oracle(oracle_mod, oracle3d_mod, axis):
    """A nozzle with walls of two contact angles, open rows, per-phase tau and
    the +/- pulse, extruded along z (or x): the projected 3-D populations
    equal the 2-D oracle's after 150 steps, in every slice."""
    n2, ny, depth = 24, 72, 3
    p2, wall2, d2 = _nozzle2d(n2, ny)
    s2 = oracle_mod.OracleSim(p2, wall2)
    s2.init_distance(d2)
    s2.step(150)
    f2, g2 = s2.get_state()
    if axis == "z":      # 2-D x is 3-D x; the state repeats along z
        p3 = dict(p2, nz=depth)
        wall3 = np.repeat(wall2[:, None, :], depth, axis=1)
        d3 = np.repeat(d2[:, None, :], depth, axis=1)
        keep = 0
    else:                # 2-D x is 3-D z; the state repeats along x
        p3 = dict(p2, nx=depth, nz=n2)
        wall3 = np.repeat(wall2[:, :, None], depth, axis=2)
        d3 = np.repeat(d2[:, :, None], depth, axis=2)
        keep = 2
    s3 = oracle3d_mod.Oracle3D(p3, wall3)
    s3.init_distance(d3)
    s3.step(150)
    f3, g3 = s3.get_state()
    c3, _, _ = oracle3d_mod.velocity_set()
    pf = _project(f3, c3, keep, EX2, EY2)
    pg = _project(g3, c3[:7], keep, EX2[:5], EY2[:5])
    for k in range(depth):
        sl = (slice(None), slice(None), k, slice(None)) if axis == "z" else (slice(None), slice(None), slice(None), k)
        ef = np.max(np.abs(pf[sl] - f2)) / np.max(np.abs(f2))
        eg = np.max(np.abs(pg[sl] - g2)) / np.max(np.abs(g2))
        assert ef < 1e-12 and eg < 1e-12, (axis, k, ef, eg)
    # the flow is not trivial: the pulse moved the ink
    assert np.max(np.abs(s2.moments()["uy"])) > 1e-3


def test_equilibrium_moments(oracle3d_mod):
    """A uniform-phi state with a set velocity: sum f = n, sum c f = n u,
    sum c c f = p I + n u u with p = n/3 + phi mu (mu = 0 at phi = phi*);
    sum g = phi, sum c g = phi u / q."""
    O3 = oracle3d_mod
    p = W.base_params3d(4, 4, 4, bc_y=0)
    wall = np.zeros((4, 4, 4), np.uint8)
    s = O3.Oracle3D(p, wall)
    d = s.derived()
    u = np.array([0.03, -0.05, 0.02])
    s.init_phi(np.full((4, 4, 4), 0.7 * d["phi_star"]), *(np.full((4, 4, 4), v) for v in u))
    f, g = s.get_state()
    fl = s.fields()
    c, _, _ = O3.velocity_set()
    fk, gk = f[:, 1, 2, 3], g[:, 1, 2, 3]
    n0, ph, mu = d["n0"], 0.7 * d["phi_star"], fl["mu"][1, 2, 3]
    assert fk.sum() == pytest.approx(n0, abs=1e-15)
    assert np.allclose(c.T @ fk, n0 * u, atol=1e-15)
    assert np.allclose(np.einsum("i,ia,ib->ab", fk, c, c), (n0 / 3 + ph * mu) * np.eye(3) + n0 * np.outer(u, u),
                       atol=1e-15)
    assert gk.sum() == pytest.approx(ph, abs=1e-15)
    assert np.allclose(c[:7].T @ gk, ph * u / d["q"], atol=1e-15)
    assert np.allclose(np.einsum("i,ia,ib->ab", gk, c[:7], c[:7]), p["gamma"] * mu * np.eye(3), atol=1e-15)
    assert abs(mu) > 1e-4   # phi = 0.7 phi* is off the minimum: the mu terms are tested


@pytest.mark.parametrize("phase", [1.0, -1.0])
def test_uniform_state_is_a_fixed_point(oracle3d_mod, phase):
    O3 = oracle3d_mod
    p = W.base_params3d(6, 6, 6, bc_y=0, tau_ink=0.7)
    s = O3.Oracle3D(p, np.zeros((6, 6, 6), np.uint8))
    s.init_phi(np.full((6, 6, 6), phase * s.derived()["phi_star"]))
    f0, g0 = s.get_state()
    s.step(25)
    f1, g1 = s.get_state()
    assert np.max(np.abs(f1 - f0)) < 1e-15 and np.max(np.abs(g1 - g0)) < 1e-15


def _blob_case(O3, n=16, ny=20, seed=3, walls=True, **kw):
    rng = W.SplitMix64(seed)
    sph = [(rng.uniform(0, n), rng.uniform(4, ny - 4), rng.uniform(0, n), rng.uniform(3, 5)) for _ in range(3)]
    p = W.base_params3d(n, ny, n, bc_y=0, tau_ink=0.8, theta_inner=50.0, theta_outer=130.0, **kw)
    wall = np.zeros((ny, n, n), np.uint8)
    if walls:
        wall[0:2] = W.WALL_OUTER
        wall[2:ny // 2, 3:6, 4:9] = W.WALL_INNER
    d = W.spheres_distance3d(n, ny, n, sph)
    return p, wall, d


def test_mass_of_both_components_conserved(oracle3d_mod):
    """Closed box (periodic, a floor and a solid block with wetting walls):
    sum n and sum phi stay fixed to round-off."""
    O3 = oracle3d_mod
    p, wall, d = _blob_case(O3)
    s = O3.Oracle3D(p, wall)
    s.init_distance(d)
    a = s.diag()
    s.step(200)
    b = s.diag()
    assert abs(b["mass_n"] - a["mass_n"]) < 1e-12 * a["mass_n"]
    assert abs(b["mass_phi"] - a["mass_phi"]) < 1e-12 * abs(a["mass_n"])
    assert b["max_u"] > 1e-4   # the blobs move (curvature and wetting drive them)


def test_momentum_change_equals_force_impulse(oracle3d_mod):
    """phi = phi* everywhere, a uniform body force on every node: the total
    momentum sum_x sum_i c_i f_i grows by N F per step exactly."""
    O3 = oracle3d_mod
    n = 6
    F = 3e-5
    p = W.base_params3d(n, n, n, bc_y=0, force_rows=n, t_pos=10 ** 6, f_pos=F, tau_ink=0.9, tau_amb=0.9)
    s = O3.Oracle3D(p, np.zeros((n, n, n), np.uint8))
    s.init_phi(np.full((n, n, n), s.derived()["phi_star"]))
    s.step(40)
    m = s.diag()["mom"]
    assert m[1] == pytest.approx(40 * n ** 3 * F, rel=1e-11)
    assert abs(m[0]) < 1e-12 and abs(m[2]) < 1e-12   # round-off of 216-node sums


def test_rotation_about_the_jet_axis(oracle3d_mod):
    """A quarter turn about y maps (x, z) to (z, -x): evolving the turned
    state gives the turned result (tests the x-z coupling that the two
    projections do not see)."""
    O3 = oracle3d_mod
    p, wall, d = _blob_case(O3, n=14, ny=16, seed=9)
    rot = lambda a: np.ascontiguousarray(np.rot90(a, k=1, axes=(1, 2)))   # [y, z, x] -> quarter turn in z-x
    s1 = O3.Oracle3D(p, wall)
    s1.init_distance(d)
    s1.step(60)
    s2 = O3.Oracle3D(p, rot(wall))
    s2.init_distance(rot(d))
    s2.step(60)
    a, b = s1.fields(), s2.fields()
    for k in ("n", "phi", "uy"):
        assert np.max(np.abs(rot(a[k]) - b[k])) < 1e-12 * max(1.0, np.max(np.abs(a[k]))), k
    # np.rot90 on axes (z, x) takes (z, x) -> (x', -z'): velocities turn with it
    uxr, uzr = rot(a["ux"]), rot(a["uz"])
    ok1 = np.max(np.abs(b["uz"] - uxr)) < 1e-12 and np.max(np.abs(b["ux"] + uzr)) < 1e-12
    ok2 = np.max(np.abs(b["uz"] + uxr)) < 1e-12 and np.max(np.abs(b["ux"] - uzr)) < 1e-12
    assert ok1 or ok2
    assert np.max(np.abs(a["ux"])) > 1e-5


@pytest.mark.slow
def test_laplace_law_3d(oracle3d_mod):
    """Static spherical drops: the thermodynamic pressure
    p0 = n/3 + phi mu - psi jumps by 2 sigma / R (three-dimensional Laplace
    law; the two-dimensional law is sigma / R)."""
    O3 = oracle3d_mod
    sigma = 0.01
    for R0 in (8.0, 11.0):
        L = int(2 * R0 + 18)
        p = W.base_params3d(L, L, L, bc_y=0, sigma=sigma)
        s = O3.Oracle3D(p, np.zeros((L, L, L), np.uint8))
        c = L / 2
        s.init_distance(W.spheres_distance3d(L, L, L, [(c, c, c, R0)]))
        s.step(1500)
        fl = s.fields()
        dd = s.derived()
        p0 = fl["n"] / 3 + fl["phi"] * fl["mu"] - dd["beta"] * (fl["phi"] ** 2 - dd["phi_star"] ** 2) ** 2
        m = L // 2
        dp = p0[m - 1:m + 2, m - 1:m + 2, m - 1:m + 2].mean() - p0[:2, :2, :2].mean()
        # a small drop in a finite box slowly dissolves: R is the radius of
        # the sphere with the drop's present ink volume
        R = (3 * (fl["phi"] > 0).sum() / (4 * np.pi)) ** (1 / 3)
        assert R == pytest.approx(R0, rel=0.06)
        assert dp * R / (2 * sigma) == pytest.approx(1.0, rel=0.05), (R0, R, dp)
