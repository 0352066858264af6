"""Parity of the HIP library (through its C ABI) with the FP64 oracle, on the
same seeded inputs.

Tolerances: FP32 against FP64.  One step: every distribution within 2e-6 of
the oracle (values are O(0.5); FP32 rounding of a handful of operations is
~1e-7).  Fields over many steps: relative L2 <= 1e-5 on n, phi, rho = n + phi
and on the velocity vector field u = (ux, uy), checked at pre-breakup
checkpoints.  The
fused kernel against the unfused reference kernels of the same library:
bitwise equal (same arithmetic, same rounding)."""
import math

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


def rel_l2(a, b):
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


def _np(t):
    return t.detach().cpu().numpy().astype(np.float64)


# ------------------------------------------------------------ test cases
def _case(name):
    """Small lattices that span several tiles and a ragged tail."""
    if name == "periodic_drops":
        nx, ny = 40, 36
        p = W.base_params(nx, ny, bc_y=W.BC_PERIODIC, tau_ink=0.7, tau_amb=1.1, tau_phi=0.9,
                          force_rows=ny, f_pos=3e-5, t_pos=10 ** 6, gamma=0.8)
        wall = np.zeros((ny, nx), np.uint8)
        d = W.discs_distance(nx, ny, [(15.3, 17.1, 7.5), (32.0, 6.0, 4.0)])
        return p, wall, d
    if name == "nozzle_ragged":
        nx, ny, x0, w, L = 100, 72, 41, 18, 20
        p = W.base_params(nx, ny, force_rows=L, t_pos=5, t_neg=4, t_idle=3, periodic_pulse=1,
                          f_pos=2e-4, f_neg=1e-4, tau_ink=0.8, theta_inner=60.0, theta_outer=120.0)
        return p, W.nozzle_wall(nx, ny, x0, w, L), W.meniscus_distance(nx, ny, L) + 2.0
    if name == "walls_block":
        nx, ny = 70, 45
        p = W.base_params(nx, ny, bc_y=W.BC_PERIODIC, theta_inner=40.0, theta_outer=135.0,
                          tau_ink=0.75, force_rows=ny, f_pos=1e-5, t_pos=10 ** 6)
        wall = W.flat_wall(nx, ny, (0, 1))
        wall[20:26, 30:41] = W.WALL_OUTER
        wall[30:33, 5:7] = W.WALL_INNER
        d = W.discs_distance(nx, ny, [(35.0, 12.0, 9.0), (10.0, 36.0, 6.0)])
        return p, wall, d
    if name == "narrow_open":
        nx, ny = 3, 50
        p = W.base_params(nx, ny, bc_y=W.BC_OPEN, force_rows=20, f_pos=1e-4, t_pos=10 ** 6)
        y = np.arange(ny)[:, None].astype(float)
        return p, np.zeros((ny, nx), np.uint8), np.broadcast_to(20.5 - y, (ny, nx)).copy()
    raise KeyError(name)


CASES = ["periodic_drops", "nozzle_ragged", "walls_block", "narrow_open"]


def _pair(O, gpu, p, wall, d):
    o = O.OracleSim(p, wall)
    o.init_distance(d)
    g = gpu.Sim(p, wall)
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
    mo = o.moments()
    mg = {k: _np(v) for k, v in g.moments().items()}
    fl = o.wall == 0
    errs = {}
    for k in ("n", "phi"):
        errs[k] = rel_l2(mg[k][fl], mo[k][fl])
    errs["rho"] = rel_l2((mg["n"] + mg["phi"])[fl], (mo["n"] + mo["phi"])[fl])
    # velocity as a vector field: relative L2 of (ux, uy) together (a
    # component that is nearly zero by symmetry has no meaningful relative error)
    errs["u"] = rel_l2(np.stack([mg["ux"][fl], mg["uy"][fl]]), np.stack([mo["ux"][fl], mo["uy"][fl]]))
    bad = {k: v for k, v in errs.items() if not v <= tol}
    assert not bad, errs
    return errs


# ------------------------------------------------------------------ tests
@pytest.mark.parametrize("name", CASES)
def test_initial_state_matches_oracle(oracle_mod, gpu_lib, name):
    p, wall, d = _case(name)
    o, g = _pair(oracle_mod, gpu_lib, p, wall, d)
    _compare_state(o, g, 2e-6)


@pytest.mark.parametrize("name", CASES)
def test_one_step_and_twenty_steps(oracle_mod, gpu_lib, name):
    p, wall, d = _case(name)
    o, g = _pair(oracle_mod, gpu_lib, p, wall, d)
    o.step(1)
    g.step(1)
    _compare_state(o, g, 2e-6)
    o.step(19)
    g.step(19)
    assert g.t == o.t == 20
    _compare_fields(o, g, 1e-5)


@pytest.mark.parametrize("name", CASES + ["nozzle_small"])
def test_fused_kernel_equals_reference_kernels_bitwise(gpu_lib, name):
    if name == "nozzle_small":
        c = W.config_nozzle_small()
        p, wall, d = c["params"], c["wall"], c["distance"]
    else:
        p, wall, d = _case(name)
    ref = gpu_lib.Sim(p, wall)
    ref.init_distance(d)
    ref.step_reference(40)
    fr, gr = ref.state()
    for waves, rows in [(1, 1), (1, 7), (2, 16), (4, 64), (4, 5), (1, 1000)]:
        s = gpu_lib.Sim(p, wall)
        s.set_tiling(waves, rows)
        s.init_distance(d)
        s.step(40)
        f, g = s.state()
        fl = (wall == 0)[None]
        assert np.array_equal(np.where(fl, _np(f), 0), np.where(fl, _np(fr), 0)), (waves, rows)
        assert np.array_equal(np.where(fl, _np(g), 0), np.where(fl, _np(gr), 0)), (waves, rows)


def test_autotune_restores_state(gpu_lib):
    """The autotuner's trial steps leave no trace: the distributions and the
    step counter are as before, and later steps equal those of an untuned
    run bit for bit (every tile shape computes the same bits)."""
    p, wall, d = _case("nozzle_ragged")
    a, b = gpu_lib.Sim(p, wall), gpu_lib.Sim(p, wall)
    for s in (a, b):
        s.init_distance(d)
        s.step(7)
    f0, g0 = a.state()
    w, r, ms = a.autotune(4)
    assert (w, r) in [(x, y) for x in (1, 2, 4) for y in (8, 16, 32, 64)] and ms > 0
    f1, g1 = a.state()
    assert a.t == 7
    assert np.array_equal(_np(f0), _np(f1)) and np.array_equal(_np(g0), _np(g1))
    a.step(21)
    b.step(21)
    fl = (wall == 0)[None]
    for x, y in zip(a.state(), b.state()):
        assert np.array_equal(np.where(fl, _np(x), 0), np.where(fl, _np(y), 0))
    with pytest.raises(gpu_lib.LBMError):
        a.autotune(1)


@pytest.mark.parametrize("name,tiling", [("nozzle_small", (4, 32)), ("nozzle_ragged", (1, 7)),
                                         ("walls_block", (2, 16)), ("narrow_open", (4, 64)),
                                         ("periodic_drops", (4, 5))])
def test_fused_sample_equals_separate_pass(gpu_lib, name, tiling):
    """A step at a sampling time takes the sample inside the collide kernels
    (per-piece row partials); the record equals that of the separate
    diagnostics pass on the same state bit for bit (both reduce the same
    per-node terms in the same order), and the sampling steps leave the
    update bit for bit unchanged."""
    if name == "nozzle_small":
        c = W.config_nozzle_small()
        p, wall, d = dict(c["params"], diag_row0=c["row0"]), c["wall"], c["distance"]
    else:
        p, wall, d = _case(name)
        p = dict(p, diag_row0=p["ny"] // 4)
    K = 25
    a = gpu_lib.Sim(dict(p, diag_every=K), wall)
    b = gpu_lib.Sim(dict(p, diag_every=0), wall)
    for s in (a, b):
        s.set_tiling(*tiling)
        s.init_distance(d)
    for _ in range(8):
        b.diag_sample()
        b.step(K)
        a.step(K)
    sa, sb = a.samples(), b.samples()
    assert len(sa) == len(sb) == 8
    for x, y in zip(sa, sb):
        assert repr(x) == repr(y), (x, y)
    fl = (wall == 0)[None]
    for u, v in zip(a.state(), b.state()):
        assert np.array_equal(np.where(fl, _np(u), 0), np.where(fl, _np(v), 0))


def test_nozzle_64x256_1000_steps(oracle_mod, gpu_lib):
    """The 64 x 256 nozzle workload, pulse +1e-4 x 200, -5e-5 x 100, idle:
    fields within 1e-5 relative L2 of the FP64 oracle at every checkpoint."""
    c = W.config_nozzle_small()
    o, g = _pair(oracle_mod, gpu_lib, c["params"], c["wall"], c["distance"])
    worst = {}
    for t in (100, 250, 500, 750, 1000):
        o.step(t - o.t)
        g.step(t - g.t)
        errs = _compare_fields(o, g, 1e-5)
        for k, v in errs.items():
            worst[k] = max(worst.get(k, 0.0), v)
    print("worst relative L2:", worst)


def test_diagnostics_match_oracle(oracle_mod, gpu_lib):
    c = W.config_nozzle_small()
    o, g = _pair(oracle_mod, gpu_lib, dict(c["params"], diag_row0=c["row0"]), c["wall"], c["distance"])
    for t in (0, 150, 400):
        o.step(t - o.t)
        g.step(t - g.t)
        g.diag_sample()
        od = o.diag(c["row0"])
        cnt, uy = g.row_profile()
        s = g.samples()[-1]
        assert s["step"] == t
        assert s["mass_n"] == pytest.approx(od["mass_n"], rel=1e-6)
        assert s["mass_phi"] == pytest.approx(od["mass_phi"], rel=1e-5)
        assert s["mom_y"] == pytest.approx(od["mom_y"], rel=1e-5, abs=1e-8)
        assert abs(s["mom_x"] - od["mom_x"]) <= 1e-5 * (abs(od["mom_x"]) + abs(od["mom_y"])) + 1e-9
        assert s["max_u"] == pytest.approx(od["max_u"], rel=1e-4, abs=1e-7)
        assert s["nan_count"] == 0
        # ink counts: a mismatch is allowed only where |phi| is at rounding level
        phi = o.moments()["phi"]
        amb = ((np.abs(phi) < 1e-5) & (c["wall"] == 0)).sum(axis=1)
        assert np.all(np.abs(cnt - od["row_count"]) <= amb)
        from oracle.oracle import segments
        seg = segments(od["row_count"], od["row_uy"], c["row0"], 4 * c["params"]["width"] ** 2)
        assert s["n_detached"] == seg["n_detached"]


def test_checkpoint_resume_is_bitwise(gpu_lib):
    c = W.config_nozzle_small()
    a = gpu_lib.Sim(c["params"], c["wall"])
    a.init_distance(c["distance"])
    a.step(120)
    f, g = a.state()
    b = gpu_lib.Sim(c["params"], c["wall"])
    b.init_distance(c["distance"])
    b.set_state(f, g, a.t)
    a.step(80)
    b.step(80)
    fa, ga = a.state()
    fb, gb = b.state()
    fl = (c["wall"] == 0)[None]
    # the state round trip adds and removes w_i n0 in float; after that the
    # two runs perform identical arithmetic
    assert np.abs(np.where(fl, _np(fa) - _np(fb), 0)).max() < 1e-6
    assert np.array_equal(np.where(fl, _np(ga), 0), np.where(fl, _np(gb), 0)) or \
        np.abs(np.where(fl, _np(ga) - _np(gb), 0)).max() < 1e-6


def test_stability_guard_and_errors(gpu_lib):
    c = W.config_nozzle_small()
    p = dict(c["params"], f_pos=5e-2, t_pos=10 ** 6, diag_every=10, u_limit=0.3)
    s = gpu_lib.Sim(p, c["wall"])
    s.init_distance(c["distance"])
    s.step(300)
    assert s.check() == gpu_lib.IJ_ERR_UNSTABLE
    with pytest.raises(gpu_lib.LBMError) as e:
        s.step(1)
    assert e.value.code == gpu_lib.IJ_ERR_UNSTABLE
    d = s.diagnostics()
    assert d["unstable_step"] >= 0
    # step before init
    s2 = gpu_lib.Sim(c["params"], c["wall"])
    with pytest.raises(gpu_lib.LBMError) as e:
        s2.step(1)
    assert e.value.code == gpu_lib.IJ_ERR_STATE


def test_attached_caller_buffers(gpu_lib):
    import torch
    c = W.config_nozzle_small()
    a = gpu_lib.Sim(c["params"], c["wall"])
    n = a.required_bytes()
    ta = torch.empty(n, dtype=torch.uint8, device="cuda")
    tb = torch.empty(n, dtype=torch.uint8, device="cuda")
    a.attach(ta, tb)
    a.init_distance(c["distance"])
    a.step(50)
    b = gpu_lib.Sim(c["params"], c["wall"])
    b.init_distance(c["distance"])
    b.step(50)
    assert np.array_equal(_np(a.state()[0]), _np(b.state()[0]))


# --------------------------------------------------- full-size sampling
def _window_compare(O, p_full, wall, d, g_mom, y0, x0, hw, ww, k, bc_y):
    """Run the oracle on a window of the full lattice.  After k steps every
    node farther than 2k from the window edge depends only on initial data
    inside the window (the stencil plus streaming reach is two nodes per
    step), so there the window run equals the full run."""
    ny, nx = wall.shape
    ys = (np.arange(y0, y0 + hw)) % ny
    xs = (np.arange(x0, x0 + ww)) % nx
    pw = dict(p_full, nx=ww, ny=hw, bc_y=bc_y)
    pw["force_rows"] = int(np.clip(p_full["force_rows"] - y0, 0, hw))
    ow = O.OracleSim(pw, wall[np.ix_(ys, xs)])
    ow.init_distance(d[np.ix_(ys, xs)])
    ow.step(k)
    mo = ow.moments()
    m = 2 * k + 2
    open_y = bc_y == W.BC_OPEN
    r0 = 0 if (open_y and y0 == 0) else m
    r1 = hw if (open_y and y0 + hw == ny) else hw - m
    c0, c1 = (0, ww) if ww == nx else (m, ww - m)
    inner = (slice(r0, r1), slice(c0, c1))
    fl = wall[np.ix_(ys, xs)][inner] == 0
    out = {}
    for key in ("n", "phi", "ux", "uy"):
        gv = g_mom[key][np.ix_(ys, xs)][inner][fl]
        ov = mo[key][inner][fl]
        out[key] = np.abs(gv - ov).max()
    return out


def test_full_size_droplet_field_sampled(oracle_mod, gpu_lib):
    """2048 x 16384 disc field at full size with the default tiling: windows
    of the lattice computed by the oracle agree with the GPU run."""
    c = W.config_droplet_field()
    p, wall, d = c["params"], c["wall"], c["distance"]
    g = gpu_lib.Sim(p, wall)
    g.init_distance(d)
    k = 6
    g.step(k)
    gm = {key: _np(v) for key, v in g.moments().items()}
    rng = np.random.default_rng(3)
    spots = [(0, 100), (16380 - 40, 2000)] + [(int(rng.integers(0, 16384)), int(rng.integers(0, 2048)))
                                            for _ in range(6)]
    for (y0, x0) in spots:
        errs = _window_compare(oracle_mod, p, wall, d, gm, y0 - 24, x0 - 24, 72, 72, k, W.BC_PERIODIC)
        assert errs["n"] < 2e-6 and errs["phi"] < 2e-6, errs
        assert errs["ux"] < 1e-7 and errs["uy"] < 1e-7, errs


def test_full_size_droplet_field_conserves_mass(gpu_lib):
    c = W.config_droplet_field()
    p, wall, d = c["params"], c["wall"], c["distance"]
    g = gpu_lib.Sim(p, wall)
    g.init_distance(d)
    g.diag_sample()
    g.step(200)
    g.diag_sample()
    s0, s1 = g.samples()[-2:]
    assert s1["nan_count"] == 0
    assert abs(s1["mass_n"] - s0["mass_n"]) < 2e-6 * abs(s0["mass_n"])
    assert abs(s1["mass_phi"] - s0["mass_phi"]) < 2e-5 * abs(s0["mass_phi"])


def test_full_size_single_nozzle_sampled(oracle_mod, gpu_lib):
    """256 x 2048 nozzle at full size: full-width windows (nozzle inlet, exit
    and chamber) computed by the oracle agree with the GPU run."""
    c = W.config_nozzle_single()
    p, wall = c["params"], c["wall"]
    d = W.meniscus_distance(p["nx"], p["ny"], c["nozzle"][2])
    g = gpu_lib.Sim(p, wall)
    g.init_distance(d)
    k = 8
    g.step(k)
    gm = {key: _np(v) for key, v in g.moments().items()}
    for y0 in (0, 224, 1000, 2048 - 64):
        errs = _window_compare(oracle_mod, p, wall, d, gm, y0, 0, 64, p["nx"], k, W.BC_OPEN)
        assert errs["n"] < 2e-6 and errs["phi"] < 2e-6, (y0, errs)
        assert errs["ux"] < 1e-7 and errs["uy"] < 1e-7, (y0, errs)


def test_largest_accepted_lattice_sampled(oracle_mod, gpu_lib):
    """The largest lattice the library accepts (ny = 65535, 15 * ny * pitch
    just under 2^31 with nx = 2048): 32-bit row offsets at their limit.
    Windows at the first and last rows agree with the oracle after k steps;
    zero steps is a no-op."""
    nx, ny = 2048, 65535
    p = W.base_params(nx, ny, bc_y=W.BC_PERIODIC, force_rows=ny, tau_ink=0.8, theta_inner=120.0,
                      theta_outer=120.0)
    wall = W.flat_wall(nx, ny, (0, 1))
    # a periodic lattice of discs (radius 40 every 128 nodes, shifted per row of discs)
    y = np.arange(ny, dtype=np.float64)[:, None]
    x = np.arange(nx, dtype=np.float64)[None, :]
    cy = np.floor(y / 128.0) * 128.0 + 64.0
    cx = np.floor((x + 37.0 * np.floor(y / 128.0)) / 128.0) * 128.0 + 64.0 - 37.0 * np.floor(y / 128.0)
    d = 40.0 - np.sqrt((x - cx) ** 2 + (y - cy) ** 2)
    d[:4] = -50.0
    g = gpu_lib.Sim(p, wall)
    g.init_distance(d)
    g.step(0)
    assert g.t == 0
    k = 4
    g.step(k)
    gm = {key: _np(v) for key, v in g.moments().items()}
    for (y0, x0) in [(0, 200), (ny - 72, 1800), (ny - 40, 1000), (32768, 64)]:
        errs = _window_compare(oracle_mod, p, wall, d, gm, y0 - 16, x0 - 16, 72, 72, k, W.BC_PERIODIC)
        assert errs["n"] < 2e-6 and errs["phi"] < 2e-6, (y0, errs)
        assert errs["ux"] < 1e-7 and errs["uy"] < 1e-7, (y0, errs)
