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


from parity_util import compare_fields as _compare_fields
from parity_util import compare_state as _compare_state
from parity_util import np64 as _np
from parity_util import rel_l2  # noqa: F401
from parity_util import window_compare as _window_compare


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
    if name == "box_corners":
        # a closed box (inner wall class) with an L-shaped obstacle (outer
        # class): solid nodes whose only fluid neighbour is diagonal take the
        # corner rule of the wetting ghost
        n = 40
        p = W.base_params(n, n, bc_y=W.BC_PERIODIC, theta_inner=60.0, theta_outer=120.0, tau_ink=0.7,
                          tau_amb=1.1, tau_phi=0.9, force_rows=n, f_pos=2e-5, t_pos=10 ** 6)
        wall = np.zeros((n, n), np.uint8)
        wall[4:6, 4:36] = wall[34:36, 4:36] = W.WALL_INNER
        wall[4:36, 4:6] = wall[4:36, 34:36] = W.WALL_INNER
        wall[12:16, 12:26] = W.WALL_OUTER
        wall[12:28, 12:16] = W.WALL_OUTER
        d = W.discs_distance(n, n, [(9.5, 9.0, 5.0), (29.0, 28.5, 6.0), (20.0, 19.0, 3.5)])
        return p, wall, d
    if name == "narrow_open":
        nx, ny = 3, 50
        p = W.base_params(nx, ny, bc_y=W.BC_OPEN, force_rows=20, f_pos=1e-4, t_pos=10 ** 6)
        y = np.arange(ny)[:, None].astype(float)
        return p, np.zeros((ny, nx), np.uint8), np.broadcast_to(20.5 - y, (ny, nx)).copy()
    raise KeyError(name)


CASES = ["periodic_drops", "nozzle_ragged", "walls_block", "box_corners", "narrow_open"]


def _pair(O, gpu, p, wall, d):
    o = O.OracleSim(p, wall)
    o.init_distance(d)
    g = gpu.Sim(p, wall)
    g.init_distance(d)
    return o, g


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
    _compare_fields(o, g, 1e-5, elementwise=True)


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
    assert (w, r) in [(x, y) for x in (1, 2, 4) for y in (1, 8, 16, 32, 64)] and ms > 0
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
    fields within 1e-5 relative L2 of the FP64 oracle at every checkpoint,
    and every node's n and phi within 1e-5 of n0 and phi*."""
    c = W.config_nozzle_small()
    o, g = _pair(oracle_mod, gpu_lib, c["params"], c["wall"], c["distance"])
    worst = {}
    for t in (100, 250, 500, 750, 1000):
        o.step(t - o.t)
        g.step(t - g.t)
        errs = _compare_fields(o, g, 1e-5, elementwise=True)
        for k, v in errs.items():
            worst[k] = max(worst.get(k, 0.0), v)
    print("worst relative L2:", worst)


def test_box_corners_300_steps(oracle_mod, gpu_lib):
    """The closed box with an L-shaped obstacle (corner ghosts of both wall
    classes) while the drops wet the walls and the body force stirs the box:
    fields within 1e-5 relative L2 of the FP64 oracle, and every node's n and
    phi within 1e-5 of n0 and phi*, at steps 100 and 300."""
    p, wall, d = _case("box_corners")
    o, g = _pair(oracle_mod, gpu_lib, p, wall, d)
    for t in (100, 300):
        o.step(t - o.t)
        g.step(t - g.t)
        print(t, _compare_fields(o, g, 1e-5, elementwise=True))


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


def _bits(t):
    import torch
    return t.contiguous().view(torch.int32).cpu().numpy()


def test_checkpoint_resume_is_bitwise(gpu_lib):
    """A run saved at step 120 (ij_save_state) and resumed in a new handle
    (ij_load_state) is bit for bit the uninterrupted run 80 steps later, and
    the pulse phase follows the restored step counter."""
    c = W.config_nozzle_small()
    p = dict(c["params"], periodic_pulse=1, t_pos=70, t_neg=40, t_idle=30)
    a = gpu_lib.Sim(p, c["wall"])
    a.init_distance(c["distance"])
    a.step(120)
    blob = a.save_state()
    b = gpu_lib.Sim(p, c["wall"])
    b.load_state(blob)
    assert b.t == 120
    a.step(81)
    b.step(81)
    for x, y in zip(a.state(), b.state()):
        assert np.array_equal(_bits(x), _bits(y))
    # a blob fits only a handle with the same lattice and walls
    other = c["wall"].copy()
    other[0, 0] = 2 if other[0, 0] != 2 else 1
    with pytest.raises(gpu_lib.LBMError) as e:
        gpu_lib.Sim(p, other).load_state(blob)
    assert e.value.code == gpu_lib.IJ_ERR_INVALID_ARG
    with pytest.raises(gpu_lib.LBMError):
        gpu_lib.Sim(dict(p, nx=65), np.zeros((p["ny"], 65), np.uint8)).load_state(blob)
    with pytest.raises(gpu_lib.LBMError):
        b.load_state(blob[:-1])


def test_state_round_trip_resume(gpu_lib):
    """ij_get_state / ij_set_state exchange unshifted float distributions:
    the round trip adds and removes w_i n0 in float and drops the g_0
    remainder, so a resumed run is close to (not bit for bit) the original."""
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
    assert np.abs(np.where(fl, _np(fa) - _np(fb), 0)).max() < 1e-6
    assert np.abs(np.where(fl, _np(ga) - _np(gb), 0)).max() < 1e-6


@pytest.mark.parametrize("kind", ["nan", "negative_density"])
def test_guard_flags_injected_fault(gpu_lib, kind):
    """A non-finite population, or a node whose density n = sum f is not
    positive, written through ij_set_state is caught by the stability guard
    at the next sample: ij_check and ij_step report IJ_ERR_UNSTABLE at that
    step."""
    c = W.config_nozzle_small()
    p = dict(c["params"], diag_every=5)
    s = gpu_lib.Sim(p, c["wall"])
    s.init_distance(c["distance"])
    s.step(10)
    assert s.check() == gpu_lib.IJ_OK
    f, g = s.state()
    f = f.clone()
    y, x = 150, 30   # a fluid node of the chamber
    assert c["wall"][y, x] == 0
    if kind == "nan":
        f[3, y, x] = float("nan")
    else:
        w = [4 / 9] + [1 / 9] * 4 + [1 / 36] * 4
        for i in range(9):
            f[i, y, x] = -0.05 * w[i]   # n = -0.05 at rest
    s.set_state(f, g, 10)
    s.step(1)
    assert s.check() == gpu_lib.IJ_ERR_UNSTABLE
    assert s.diagnostics()["unstable_step"] == 10
    assert s.samples()[-1]["nan_count"] >= 1
    with pytest.raises(gpu_lib.LBMError) as e:
        s.step(1)
    assert e.value.code == gpu_lib.IJ_ERR_UNSTABLE


@pytest.mark.parametrize("name", ["nozzle_small", "nozzle_ragged", "narrow_open", "walls_block"])
def test_every_fluid_slot_is_written(gpu_lib, name):
    """The destination buffer is filled with NaN bit patterns (floats and the
    16-bit remainder plane) before a step: afterwards every population of
    every fluid node is finite and equal, bit for bit, to a run on a clean
    buffer, so the step writes every fluid slot it owns."""
    import torch
    if name == "nozzle_small":
        c = W.config_nozzle_small()
        p, wall, d = c["params"], c["wall"], c["distance"]
    else:
        p, wall, d = _case(name)
    ref = gpu_lib.Sim(p, wall)
    ref.init_distance(d)
    ref.step(3)
    s = gpu_lib.Sim(p, wall)
    n = s.required_bytes()
    ta = torch.zeros(n, dtype=torch.uint8, device="cuda")
    tb = torch.zeros(n, dtype=torch.uint8, device="cuda")
    s.attach(ta, tb)
    s.init_distance(d)
    for _ in range(3):
        # the buffer the next step writes (buffers alternate: A at even steps)
        (tb if s.t % 2 == 0 else ta).fill_(0xFF)
        s.step(1)
    fl = (wall == 0)[None]
    for x, y in zip(s.state(), ref.state()):
        xv = _np(x)
        assert np.isfinite(np.where(fl, xv, 0.0)).all()
        assert np.array_equal(np.where(fl, _bits(x), 0), np.where(fl, _bits(y), 0))


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


def test_solid_mask_from_the_device(gpu_lib):
    """ij_set_solid_mask with a device mask sets the same walls as
    ij_set_wall with the host copy: the two runs are bit for bit equal, and
    a mask with a bad wall class is refused from either side."""
    import torch
    c = _case("walls_block")
    p, wall, d = c
    a = gpu_lib.Sim(p, np.zeros_like(wall))
    a.set_wall(torch.from_numpy(np.ascontiguousarray(wall)).cuda())
    a.init_distance(d)
    a.step(40)
    b = gpu_lib.Sim(p, np.zeros_like(wall))
    b.set_wall(wall)
    b.init_distance(d)
    b.step(40)
    for x, y in zip(a.state(), b.state()):
        assert np.array_equal(_bits(x), _bits(y))
    bad = wall.copy()
    bad[3, 3] = 7
    with pytest.raises(gpu_lib.LBMError) as e:
        a.set_wall(torch.from_numpy(bad).cuda())
    assert e.value.code == gpu_lib.IJ_ERR_INVALID_ARG


# --------------------------------------------------- full-size sampling
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
