"""Parity of the three-dimensional HIP path (ij3_* through the C ABI) with the
FP64 three-dimensional oracle, on the same seeded inputs.

Tolerances, FP32 against FP64 (as for the two-dimensional path): after one
step every distribution within 2e-6 of the oracle (values are O(0.5) and a
node's update is a few dozen FP32 operations at ~6e-8 relative each); over
many steps relative L2 <= 1e-5 on n, phi, n + phi and the velocity vector
field.  Diagnostics: sums within their FP32 inputs' rounding; ink counts
differ only where |phi| is at rounding level."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


def rel_l2(a, b):
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


def _np(t):
    return t.detach().cpu().numpy().astype(np.float64)


def _case(name):
    """Small lattices that span several workgroups and ragged tails in x and z."""
    if name == "round_nozzle":
        c = W.config_round_nozzle_small()
        return c["params"], c["wall"], c["distance"]
    if name == "blobs_walls_ragged":
        nx, ny, nz = 70, 24, 7
        p = W.base_params3d(nx, ny, nz, bc_y=W.BC_PERIODIC, tau_ink=0.7, tau_amb=1.1, tau_phi=0.9, gamma=0.8,
                            theta_inner=40.0, theta_outer=135.0, force_rows=ny, f_pos=2e-5, t_pos=10 ** 6)
        wall = np.zeros((ny, nz, nx), np.uint8)
        wall[0:2] = W.WALL_OUTER
        wall[8:12, 2:5, 30:41] = W.WALL_INNER
        d = W.spheres_distance3d(nx, ny, nz, [(20.3, 12.1, 3.0, 6.5), (55.0, 16.0, 4.5, 4.0)])
        return p, wall, d
    if name == "narrow_open":
        nx, ny, nz = 3, 30, 3
        p = W.base_params3d(nx, ny, nz, bc_y=W.BC_OPEN, force_rows=12, f_pos=1e-4, t_pos=10 ** 6)
        y = np.arange(ny)[:, None, None].astype(float)
        return p, np.zeros((ny, nz, nx), np.uint8), np.broadcast_to(12.5 - y, (ny, nz, nx)).copy()
    raise KeyError(name)


CASES = ["round_nozzle", "blobs_walls_ragged", "narrow_open"]


def _pair(O3, p, wall, d):
    from paper_1702_04487_amd import lbm3d
    o = O3.Oracle3D(p, wall)
    o.init_distance(d)
    g = lbm3d.Sim3D(p, wall)
    g.init_distance(d)
    return o, g


def _compare_state(o, g, tol):
    fo, go = o.get_state()
    fg, gg = g.state()
    fl = (o.wall == 0)[None]
    df = np.abs(np.where(fl, _np(fg) - fo, 0.0)).max()
    dg = np.abs(np.where(fl, _np(gg) - go, 0.0)).max()
    assert df < tol and dg < tol, (df, dg)


def _compare_fields(o, g, tol):
    mo = o.fields()
    mg = {k: _np(v) for k, v in g.moments().items()}
    fl = o.wall == 0
    errs = {k: rel_l2(mg[k][fl], mo[k][fl]) for k in ("n", "phi")}
    errs["rho"] = rel_l2((mg["n"] + mg["phi"])[fl], (mo["n"] + mo["phi"])[fl])
    errs["u"] = rel_l2(np.stack([mg[k][fl] for k in ("ux", "uy", "uz")]),
                       np.stack([mo[k][fl] for k in ("ux", "uy", "uz")]))
    bad = {k: v for k, v in errs.items() if not v <= tol}
    assert not bad, errs
    return errs


@pytest.mark.parametrize("name", CASES)
def test_initial_state_matches_oracle(oracle3d_mod, gpu_lib, name):
    print("3-D initial state", name, flush=True)
    o, g = _pair(oracle3d_mod, *_case(name))
    _compare_state(o, g, 2e-6)


@pytest.mark.parametrize("name", CASES)
def test_one_step_and_twenty_steps(oracle3d_mod, gpu_lib, name):
    print("3-D 1 + 19 steps", name, flush=True)
    o, g = _pair(oracle3d_mod, *_case(name))
    o.step(1)
    g.step(1)
    _compare_state(o, g, 2e-6)
    o.step(19)
    g.step(19)
    assert g.t == o.t == 20
    _compare_fields(o, g, 1e-5)


def test_round_nozzle_pulse(oracle3d_mod, gpu_lib):
    """The 32 x 96 x 32 round nozzle through its +/- pulse (60 + 30 steps)
    and after: fields within 1e-5 relative L2 at every checkpoint to step
    300 and at step 1000, when the velocity has decayed tenfold to the
    spurious currents at the rim (max |u| ~ 1e-3).  That late velocity is
    the most sensitive quantity: it is held by the double-precision update
    of g_0 and its stored remainder (with g_0 rounded to float every step
    the relative error reached 7e-5)."""
    print("3-D round nozzle 1000 steps", flush=True)
    c = W.config_round_nozzle_small()
    o, g = _pair(oracle3d_mod, c["params"], c["wall"], c["distance"])
    worst = {}
    for t in (60, 90, 200, 300):
        o.step(t - o.t)
        g.step(t - g.t)
        for k, v in _compare_fields(o, g, 1e-5).items():
            worst[k] = max(worst.get(k, 0.0), v)
        if t == 90:
            assert np.max(np.abs(o.fields()["uy"])) > 1e-3   # the pulse moved the ink
    print("worst relative L2 to step 300:", worst)
    o.step(1000 - o.t)
    g.step(1000 - g.t)
    mo = o.fields()
    mg = {k: _np(v) for k, v in g.moments().items()}
    fl = o.wall == 0
    e = {k: rel_l2(mg[k][fl], mo[k][fl]) for k in ("n", "phi")}
    e["u"] = rel_l2(np.stack([mg[k][fl] for k in ("ux", "uy", "uz")]), np.stack([mo[k][fl] for k in ("ux", "uy", "uz")]))
    print("relative L2 at step 1000:", e)
    assert e["n"] <= 1e-5 and e["phi"] <= 1e-5 and e["u"] <= 1e-5, e


def test_diagnostics_match_oracle(oracle3d_mod, gpu_lib):
    print("3-D diagnostics", flush=True)
    c = W.config_round_nozzle_small()
    o, g = _pair(oracle3d_mod, c["params"], c["wall"], c["distance"])
    row0 = c["row0"]
    for t in (0, 70, 150):
        o.step(t - o.t)
        g.step(t - g.t)
        s = g.sample(row0)
        od = o.diag(row0)
        assert s["mass_n"] == pytest.approx(od["mass_n"], rel=1e-6)
        assert s["mass_phi"] == pytest.approx(od["mass_phi"], rel=1e-5, abs=1e-6 * od["mass_n"])
        scale = np.abs(od["mom"]).sum()
        assert np.all(np.abs(s["mom"] - od["mom"]) <= 1e-5 * scale + 1e-9), (s["mom"], od["mom"])
        assert s["max_u"] == pytest.approx(od["max_u"], rel=1e-4, abs=1e-7)
        assert s["nan_count"] == 0
        phi = o.fields()["phi"]
        amb = ((np.abs(phi) < 1e-5) & (c["wall"] == 0)).sum(axis=(1, 2))
        assert np.all(np.abs(s["row_count"] - od["row_count"]) <= amb)
        assert np.all(s["row_count"][:row0] == 0)
        scale_u = np.abs(od["row_uy"]).max() + 1e-12
        assert np.all(np.abs(s["row_uy"] - od["row_uy"]) <= 1e-4 * scale_u + 1e-7 * od["row_count"])
        # the device's droplet segments are the oracle's segments of the same rows
        from oracle.oracle import segments
        a_min = int(round(4 * c["params"]["width"] ** 3))
        want = segments(s["row_count"], s["row_uy"], row0, a_min, band=4)
        got = s["drops"]
        for k in ("n_detached", "largest_count", "largest_top", "largest_bottom"):
            assert got[k] == want[k], (k, got, want)
        for k in ("largest_uy", "head_uy", "tail_uy"):
            assert got[k] == pytest.approx(want[k], rel=1e-12, abs=1e-15), (k, got, want)


def test_closed_box_conserves_mass(gpu_lib):
    """Periodic box with a floor and a block: sum n and sum phi stay fixed to
    float rounding over 400 steps."""
    print("3-D closed box 400 steps", flush=True)
    from paper_1702_04487_amd import lbm3d
    p, wall, d = _case("blobs_walls_ragged")
    g = lbm3d.Sim3D(p, wall)
    g.init_distance(d)
    a = g.sample()
    g.step(400)
    b = g.sample()
    assert abs(b["mass_n"] - a["mass_n"]) < 2e-6 * a["mass_n"]
    assert abs(b["mass_phi"] - a["mass_phi"]) < 2e-6 * a["mass_n"]
    assert b["max_u"] > 1e-4 and b["nan_count"] == 0


def test_state_round_trip_and_restart(oracle3d_mod, gpu_lib):
    """A state written through ij3_set_state reads back, and stepping it
    matches the oracle stepped from the same state."""
    print("3-D set_state / restart", flush=True)
    from paper_1702_04487_amd import lbm3d
    p, wall, d = _case("round_nozzle")
    o = oracle3d_mod.Oracle3D(p, wall)
    o.init_distance(d)
    o.step(30)
    fo, go = o.get_state()
    g = lbm3d.Sim3D(p, wall)
    g.set_state(fo, go, t=30)
    fg, gg = g.state()
    fl = (wall == 0)[None]
    assert np.abs(np.where(fl, _np(fg) - fo, 0)).max() < 1e-7
    assert np.abs(np.where(fl, _np(gg) - go, 0)).max() < 1e-7
    o.step(5)
    g.step(5)
    assert g.t == 35
    _compare_state(o, g, 2e-6)


def test_errors(gpu_lib):
    from paper_1702_04487_amd import lbm, lbm3d
    p, wall, d = _case("narrow_open")
    g = lbm3d.Sim3D(p, wall)
    with pytest.raises(lbm.LBMError) as e:
        g.step(1)
    assert e.value.code == lbm.IJ_ERR_STATE
    bad = wall.copy()
    bad[1] = W.WALL_OUTER        # an open row's fluid node with a wall inside it
    with pytest.raises(lbm.LBMError) as e:
        lbm3d.Sim3D(p, bad)
    assert e.value.code == lbm.IJ_ERR_INVALID_ARG
    g.init_distance(d)
    for kw in (dict(a_min=0), dict(band=0)):
        with pytest.raises(lbm.LBMError) as e:
            g.sample(0, **kw)
        assert e.value.code == lbm.IJ_ERR_INVALID_ARG


def _window_compare(O3, p_full, wall, d, g_mom, y0, z0, x0, h, dz, dx, k, bc_y):
    """The oracle on a window of the full lattice: after k steps every node
    farther than 2k + 2 from a window edge that is not a true boundary
    depends only on initial data inside the window (the stencil plus
    streaming reach is two nodes per step), so there it equals the full run."""
    ny, nz, nx = wall.shape
    ys, zs, xs = np.arange(y0, y0 + h) % ny, np.arange(z0, z0 + dz) % nz, np.arange(x0, x0 + dx) % nx
    pw = dict(p_full, nx=dx, ny=h, nz=dz, bc_y=bc_y)
    pw["force_rows"] = int(np.clip(p_full["force_rows"] - y0, 0, h))
    ow = O3.Oracle3D(pw, wall[np.ix_(ys, zs, xs)])
    ow.init_distance(d[np.ix_(ys, zs, xs)])
    ow.step(k)
    mo = ow.fields()
    m = 2 * k + 2
    open_y = bc_y == W.BC_OPEN
    r0 = 0 if (open_y and y0 == 0) else m
    r1 = h if (open_y and y0 + h == ny) else h - m
    inner = (slice(r0, r1), slice(m, dz - m), slice(m, dx - m))
    fl = wall[np.ix_(ys, zs, xs)][inner] == 0
    out = {}
    for key in ("n", "phi", "ux", "uy", "uz"):
        out[key] = np.abs(g_mom[key][np.ix_(ys, zs, xs)][inner][fl] - mo[key][inner][fl]).max()
    return out


def test_full_size_round_nozzle_sampled(oracle3d_mod, gpu_lib):
    """256 x 512 x 256 round nozzle at full size (the benchmarked launch):
    windows computed by the oracle (the bore's open bottom, the bore wall,
    the nozzle exit with the meniscus, the chamber and the open top) agree
    with the GPU run."""
    print("3-D full size 256x512x256", flush=True)
    from paper_1702_04487_amd import lbm3d
    c = W.config_round_nozzle()
    p, wall, d = c["params"], c["wall"], c["distance"]
    g = lbm3d.Sim3D(p, wall)
    g.init_distance(d)
    k = 5
    g.step(k)
    gm = {key: _np(v) for key, v in g.moments().items()}
    del g
    ny, nz, nx = wall.shape
    r, L = c["nozzle"]
    cx = (nx - 1) / 2
    spots = [(0, int(cx), int(cx - r), W.BC_OPEN),                  # open bottom row, bore wall
             (L - 18, int(cx + 10), int(cx + r - 4), W.BC_PERIODIC),  # nozzle exit, meniscus on the rim
             (300, 40, 200, W.BC_PERIODIC),                          # chamber
             (ny - 36, 100, 7, W.BC_OPEN)]                           # open top row
    for (yc, zc, xc, bc) in spots:
        y0 = 0 if bc == W.BC_OPEN and yc == 0 else yc
        errs = _window_compare(oracle3d_mod, p, wall, d, gm, y0, zc - 18, xc - 18, 36, 36, 36, k, bc)
        print("window", (yc, zc, xc), errs, flush=True)
        assert errs["n"] < 2e-6 and errs["phi"] < 2e-6, errs
        assert max(errs["ux"], errs["uy"], errs["uz"]) < 1e-7, errs


def _cap_angle(phi_slice, xc):
    """Contact angle through the ink of a cap on the wall surface y = 1.5 in
    one x-y slice through its axis: 2 atan(2h / b), b the base width
    extrapolated to the wall from the first two fluid rows, h the height."""
    def cross(a, idx):
        for i0, i1 in zip(idx[:-1], idx[1:]):
            if a[i0] > 0 >= a[i1]:
                return i0 + a[i0] / (a[i0] - a[i1]) * (i1 - i0)
        raise AssertionError("no interface crossing")
    nyv, nxv = phi_slice.shape
    base = lambda row: cross(phi_slice[row], list(range(xc, nxv))) - cross(phi_slice[row], list(range(xc, -1, -1)))
    b2, b3 = base(2), base(3)
    b = b2 + 0.5 * (b2 - b3)
    h = cross(phi_slice[:, xc], list(range(2, nyv))) - 1.5
    return np.degrees(2 * np.arctan(2 * h / b))


@pytest.mark.parametrize("theta", [60.0, 90.0, 120.0])
def test_sessile_drop_contact_angle_3d(gpu_lib, theta):
    """A hemisphere of radius 18 on a flat wetting wall (72 x 38 x 72,
    12000 steps, beyond what the oracle runs in a test) relaxes to a
    spherical cap whose contact angle equals the set angle within 3 degrees
    (Young's law with the Cahn wall of the wetting ghost)."""
    print("3-D sessile drop", theta, flush=True)
    from paper_1702_04487_amd import lbm3d
    R = 18
    nx = nz = 4 * R
    ny = int(1.6 * R) + 10
    p = W.base_params3d(nx, ny, nz, bc_y=W.BC_PERIODIC, theta_inner=theta, theta_outer=theta)
    wall = np.zeros((ny, nz, nx), np.uint8)
    wall[0:2] = W.WALL_INNER
    d = W.spheres_distance3d(nx, ny, nz, [(nx / 2, 1.5, nz / 2, R)], periodic_y=False)
    g = lbm3d.Sim3D(p, wall)
    g.init_distance(d)
    g.step(12000)
    phi = _np(g.moments()["phi"])
    s = g.sample()
    assert s["nan_count"] == 0
    ang_x = _cap_angle(phi[:, nz // 2, :], nx // 2)
    ang_z = _cap_angle(phi[:, :, nx // 2], nz // 2)
    print("angles", ang_x, ang_z)
    assert ang_x == pytest.approx(theta, abs=3.0) and ang_z == pytest.approx(theta, abs=3.0)


def test_round_nozzle_ejects_ink(gpu_lib):
    """A push and a pull through the 16-radius round bore: the column of ink
    above the exit pinches off from the bore (a detached run of ink rows
    above the exit, from the per-slice ink counts of ij3_sample) between
    steps 12 000 and 18 000, with no non-finite node and speeds below 0.2."""
    print("3-D ejection 128x512x128", flush=True)
    from oracle.oracle import segments
    from paper_1702_04487_amd import lbm3d
    c = W.config_round_nozzle_eject()
    g = lbm3d.Sim3D(c["params"], c["wall"])
    g.init_distance(c["distance"])
    first = None
    while g.t < c["steps"]:
        g.step(500)
        s = g.sample(c["row0"])
        assert s["nan_count"] == 0 and s["max_u"] < 0.2, (g.t, s["max_u"])
        seg = segments(s["row_count"], s["row_uy"], c["row0"], int(round(4 * c["params"]["width"] ** 3)), band=4)
        d = s["drops"]
        assert d["n_detached"] == seg["n_detached"] and d["largest_count"] == seg["largest_count"], (d, seg)
        assert d["largest_top"] == seg["largest_top"] and d["largest_bottom"] == seg["largest_bottom"]
        if d["n_detached"] and first is None:
            first = g.t
            print("detached at", first, "drop", d, flush=True)
    assert first is not None and 12000 <= first <= 18000, first


def test_degenerate_lattices(oracle3d_mod, gpu_lib):
    """Edge cases: a lattice with no fluid node steps and samples to zeros;
    the smallest open lattice (3 x 3 x 3, one interior row) and a lattice
    with no solid node (an empty ghost list) match the oracle."""
    print("3-D degenerate lattices", flush=True)
    from paper_1702_04487_amd import lbm3d
    p = W.base_params3d(5, 4, 3, bc_y=W.BC_PERIODIC)
    solid = np.full((4, 3, 5), W.WALL_OUTER, np.uint8)
    g = lbm3d.Sim3D(p, solid)
    g.init_distance(np.zeros((4, 3, 5)))
    g.step(3)
    s = g.sample()
    assert s["mass_n"] == 0.0 and s["mass_phi"] == 0.0 and s["nan_count"] == 0 and g.t == 3
    f, gg = g.state()
    assert float(f.abs().max()) == 0.0 and float(gg.abs().max()) == 0.0
    for p, d in [(W.base_params3d(3, 3, 3, bc_y=W.BC_OPEN, force_rows=3, f_pos=1e-4, t_pos=10 ** 6),
                  np.broadcast_to(1.2 - np.arange(3.0)[:, None, None], (3, 3, 3)).copy()),
                 (W.base_params3d(9, 7, 5, bc_y=W.BC_PERIODIC, gamma=0.5),
                  W.spheres_distance3d(9, 7, 5, [(4.0, 3.0, 2.0, 2.5)]))]:
        wall = np.zeros((p["ny"], p["nz"], p["nx"]), np.uint8)
        o, g = _pair(oracle3d_mod, p, wall, d)
        o.step(10)
        g.step(10)
        _compare_state(o, g, 2e-6)


def test_checkpoint_resume(gpu_lib):
    """A run stopped at step 40, read out through ij3_get_state and resumed in
    a new handle through ij3_set_state, ends where the uninterrupted run
    ends (to the float rounding of removing and restoring the stored shift
    of f)."""
    print("3-D checkpoint / resume", flush=True)
    from paper_1702_04487_amd import lbm3d
    c = W.config_round_nozzle_small()
    a = lbm3d.Sim3D(c["params"], c["wall"])
    a.init_distance(c["distance"])
    a.step(80)
    fa, ga = a.state()
    b = lbm3d.Sim3D(c["params"], c["wall"])
    b.init_distance(c["distance"])
    b.step(40)
    f40, g40 = b.state()
    r = lbm3d.Sim3D(c["params"], c["wall"])
    r.set_state(f40, g40, t=40)
    r.step(40)
    assert r.t == 80
    fr, gr = r.state()
    fl = (c["wall"] == 0)[None]
    assert np.abs(np.where(fl, _np(fr) - _np(fa), 0)).max() < 1e-6
    assert np.abs(np.where(fl, _np(gr) - _np(ga), 0)).max() < 1e-6


def test_checkpoint_resume_is_bitwise(gpu_lib):
    """ij3_save_state at step 40 and ij3_load_state in a new handle: 41 more
    steps end bit for bit where the uninterrupted run ends; a blob does not
    load into a lattice with other walls."""
    print("3-D checkpoint blob", flush=True)
    import torch
    from paper_1702_04487_amd import lbm3d
    c = W.config_round_nozzle_small()
    a = lbm3d.Sim3D(c["params"], c["wall"])
    a.init_distance(c["distance"])
    a.step(40)
    blob = a.save_state()
    b = lbm3d.Sim3D(c["params"], c["wall"])
    b.load_state(blob)
    assert b.t == 40
    a.step(41)
    b.step(41)
    for x, y in zip(a.state(), b.state()):
        assert bool((x.contiguous().view(torch.int32) == y.contiguous().view(torch.int32)).all())
    other = c["wall"].copy()
    other[0, 0, 0] = 2 if other[0, 0, 0] != 2 else 1
    with pytest.raises(gpu_lib.LBMError):
        lbm3d.Sim3D(c["params"], other).load_state(blob)


def paper_fluid_nozzle3d():
    """A 40 x 72 x 40 round nozzle (bore radius 10, plate y < 24) with the
    paper preset's fluid: densities 1000 / 1 (phi* = 499.5), W 3, sigma 1.08,
    tau 0.85 / 0.8 and its mobility and pulse amplitudes (in steps)."""
    pp = W.config_paper()["params"]
    nx = nz = 40
    ny, r, L = 72, 10.0, 24
    p = W.base_params3d(nx, ny, nz, **{k: pp[k] for k in ("rho_ink", "rho_amb", "sigma", "width", "gamma",
                                                          "tau_ink", "tau_amb", "tau_phi", "f_pos", "f_neg")})
    p.update(force_rows=L, t_pos=200, t_neg=100, t_idle=10 ** 6, theta_inner=60.0, theta_outer=120.0)
    return p, W.round_nozzle_wall3d(nx, ny, nz, r, L), W.meniscus_distance3d(nx, ny, nz, L)


def test_paper_fluid_matches_oracle(oracle3d_mod, gpu_lib):
    """At the paper's density ratio (phi* = 499.5) the rest population g_0 is
    about phi; its float remainder keeps the 3-D path within 1e-5 relative L2
    of the oracle through the pulse."""
    print("3-D paper fluid", flush=True)
    o, g = _pair(oracle3d_mod, *paper_fluid_nozzle3d())
    worst = {}
    for t in (100, 300):
        o.step(t - o.t)
        g.step(t - g.t)
        for k, v in _compare_fields(o, g, 1e-5).items():
            worst[k] = max(worst.get(k, 0.0), v)
    print("worst relative L2:", worst)
