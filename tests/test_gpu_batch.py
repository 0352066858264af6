"""Batches of independent lattices (parameter sweeps) through the C ABI:
every case of a batch evolves bit for bit as when it is stepped alone,
with or without captured graphs, at any tile shape; a case that fails the
stability guard is frozen and flagged without touching the others; the
autotuner leaves the state unchanged."""
import numpy as np
import pytest

import workloads as W
from parity_util import compare_fields, compare_state, np64, window_compare

pytestmark = pytest.mark.gpu

K = 10   # diagnostics interval of these tests


def _cases():
    """Four uneven cases: nozzles of different sizes, angles, tensions and
    pulses, and a periodic box with drops and interior walls."""
    out = []
    for (nx, ny, x0, w, L, theta, sigma, gamma, fp, tp, fn, tn, ti, per) in [
            (100, 72, 41, 18, 20, 60.0, 0.01, 1.0, 2e-4, 5, 1e-4, 4, 3, 1),
            (64, 130, 24, 16, 40, 120.0, 0.005, 1.0, 1e-4, 30, 5e-5, 20, 40, 0),
            (150, 64, 60, 24, 16, 35.0, 0.015, 0.5, 5e-5, 12, 5e-5, 12, 12, 1)]:
        p = W.base_params(nx, ny, force_rows=L, t_pos=tp, t_neg=tn, t_idle=ti, periodic_pulse=per, f_pos=fp,
                          f_neg=fn, tau_ink=0.8, theta_inner=theta, theta_outer=100.0, sigma=sigma, gamma=gamma,
                          diag_every=K, diag_row0=L)
        out.append((p, W.nozzle_wall(nx, ny, x0, w, L), W.meniscus_distance(nx, ny, L) + 2.0))
    nx, ny = 70, 45
    p = W.base_params(nx, ny, bc_y=W.BC_PERIODIC, theta_inner=40.0, theta_outer=135.0, tau_ink=0.75,
                      force_rows=ny, f_pos=1e-5, t_pos=10 ** 6, diag_every=K, diag_row0=2)
    wall = W.flat_wall(nx, ny, (0, 1))
    wall[20:26, 30:41] = W.WALL_OUTER
    out.append((p, wall, W.discs_distance(nx, ny, [(35.0, 12.0, 9.0), (10.0, 36.0, 6.0)])))
    # wider than one 256-column strip: full strips plus a tail of 44 columns
    nx, ny = 300, 40
    p = W.base_params(nx, ny, bc_y=W.BC_PERIODIC, tau_ink=0.85, force_rows=ny, f_pos=2e-5, t_pos=10 ** 6,
                      diag_every=K, diag_row0=2)
    wall = W.flat_wall(nx, ny, (0, 1))
    out.append((p, wall, W.discs_distance(nx, ny, [(60.0, 20.0, 10.0), (250.0, 18.0, 12.0), (290.0, 30.0, 6.0)])))
    return out


def _batch(L, cases):
    b = L.Batch([c[0] for c in cases], [c[1] for c in cases])
    for sim, (_, _, d) in zip(b.cases, cases):
        sim.init_distance(d)
    return b


def _singles(L, cases, steps):
    out = []
    for p, wall, d in cases:
        s = L.Sim(p, wall)
        s.init_distance(d)
        s.step(steps)
        out.append(s)
    return out


def _bits(t):
    import torch
    return t.contiguous().view(torch.int32)


def _same(a, b):
    """Bit patterns of both states are equal (solid nodes read as 0)."""
    fa, ga = a.state()
    fb, gb = b.state()
    return bool((_bits(fa) == _bits(fb)).all() and (_bits(ga) == _bits(gb)).all())


def _same_samples(a, b):
    sa, sb = a.samples(), b.samples()
    return len(sa) == len(sb) and all(repr(x) == repr(y) for x, y in zip(sa, sb))


def test_batch_matches_single_runs_bitwise(gpu_lib):
    L = gpu_lib
    cases = _cases()
    b = _batch(L, cases)
    b.step(57)
    b.step(73)
    assert b.t == 130
    singles = _singles(L, cases, 130)
    for i, (bc, sc) in enumerate(zip(b.cases, singles)):
        assert bc.check() == L.IJ_OK and sc.check() == L.IJ_OK, i
        assert bc.t == 130 and _same(bc, sc), i
        assert _same_samples(bc, sc), i
    with pytest.raises(L.LBMError):
        b.cases[0].step(1)   # a member is stepped by its batch only
    b.close()


def test_batch_graph_replay_equals_launches(gpu_lib):
    L = gpu_lib
    cases = _cases()
    ref = _batch(L, cases)
    ref.step(3)
    ref.step(97)
    ref.step(45)
    g = _batch(L, cases)
    g.set_graph(20)
    g.step(3)       # unaligned start, then replays of 20-step graphs and a tail
    g.step(97)
    g.step(45)
    for i, (a, c) in enumerate(zip(ref.cases, g.cases)):
        assert a.check() == L.IJ_OK, i
        assert _same(a, c), i
        assert _same_samples(a, c), i
    ref.close()
    g.close()


def test_batch_members_match_oracle(oracle_mod, gpu_lib):
    """Each of the five uneven members of a batch against the FP64 oracle
    run on its own: every distribution within 2e-6 after one step, and the
    fields within 1e-5 relative L2 (n and phi also node by node against n0
    and phi*) after 200 steps of their pulses."""
    L, O = gpu_lib, oracle_mod
    cases = _cases()
    b = _batch(L, cases)
    b.set_graph(20)
    oracles = []
    for p, wall, d in cases:
        o = O.OracleSim(p, wall)
        o.init_distance(d)
        oracles.append(o)
    b.step(1)
    for i, (o, g) in enumerate(zip(oracles, b.cases)):
        o.step(1)
        print("batch member", i, "one step", compare_state(o, g, 2e-6), flush=True)
    b.step(199)
    for i, (o, g) in enumerate(zip(oracles, b.cases)):
        o.step(199)
        assert g.t == o.t == 200
        print("batch member", i, "200 steps", compare_fields(o, g, 1e-5, elementwise=True), flush=True)
    b.close()


def test_sweep_table_cases_full_size_windows(oracle_mod, gpu_lib):
    """Four cases of the 256-case sweep table (scaled variant, full lattice
    sizes up to 384 x 3072) stepped as one batch: full-width windows of the
    nozzle inlet, exit, chamber and top computed by the oracle agree with
    the batch (distributions' moments within 2e-6, velocities within 1e-7)."""
    L, O = gpu_lib, oracle_mod
    table = W.sweep_cases(256, 1234, stable=True)[:4]
    b = L.Batch([c["params"] for c in table], [W.case_wall(c) for c in table])
    for sim, c in zip(b.cases, table):
        sim.init_distance(W.case_distance(c))
    k = 6
    b.step(k)
    for sim, c in zip(b.cases, table):
        p = c["params"]
        wall, d = W.case_wall(c), W.case_distance(c)
        gm = {key: np64(v) for key, v in sim.moments().items()}
        L_ = c["nozzle"][2]
        for y0 in (0, L_ - 32, p["ny"] // 2, p["ny"] - 64):
            errs = window_compare(O, p, wall, d, gm, y0, 0, 64, p["nx"], k, W.BC_OPEN)
            assert errs["n"] < 2e-6 and errs["phi"] < 2e-6, (c["name"], y0, errs)
            assert errs["ux"] < 1e-7 and errs["uy"] < 1e-7, (c["name"], y0, errs)
    b.close()


def test_batch_unstable_case_is_frozen_and_flagged(gpu_lib):
    """A case driven far beyond the speed bound trips the guard: it is frozen
    at the failing sample (its state stays that of the sample's step, read
    back correctly after an odd number of further steps, and its later
    samples all see that state) while the other cases go on bit for bit."""
    L = gpu_lib
    cases = _cases()
    p, wall, d = cases[1]
    cases[1] = (dict(p, f_pos=0.05, t_pos=10 ** 6, t_neg=0, t_idle=0, periodic_pulse=0), wall, d)
    b = _batch(L, cases)
    b.set_graph(20)
    b.step(200)
    diag = b.cases[1].diagnostics()
    tf = diag["unstable_step"]
    assert tf >= 0 and b.cases[1].check() == L.IJ_ERR_UNSTABLE
    singles = _singles(L, [c for i, c in enumerate(cases) if i != 1], 200)
    for bc, sc in zip([c for i, c in enumerate(b.cases) if i != 1], singles):
        assert _same(bc, sc) and _same_samples(bc, sc)
        assert bc.check() == L.IJ_OK
    # the frozen state: that of the case stepped alone to the failing sample
    ref = _singles(L, [cases[1]], tf)[0]
    for extra in (0, 7, 4):
        b.step(extra)
        assert _same(b.cases[1], ref), extra
    smp = [x for x in b.cases[1].samples() if x["step"] >= tf]
    assert len(smp) > 3 and all(x["mass_n"] == smp[0]["mass_n"] for x in smp)
    # every later record repeats the failing sample (the state has not moved), field by field
    same = lambda u, v: u == v or (u != u and v != v)   # noqa: E731  (NaN equals NaN here)
    for x in smp[1:]:
        assert all(same(x[k], smp[0][k]) for k in smp[0] if k != "step"), (x, smp[0])
    b.close()


def test_batch_autotune_keeps_state_and_caches(gpu_lib):
    L = gpu_lib
    cases = _cases()
    b = _batch(L, cases)
    b.step(20)
    before = [c.state() for c in b.cases]
    w, r, m, per, ms = b.autotune(6)
    assert (w, r, m, per) == b.tiling() and w in (1, 2, 4) and r in (1, 16, 32, 64) and ms > 0
    for c, (f0, g0) in zip(b.cases, before):
        f1, g1 = c.state()
        assert bool((f0 == f1).all() and (g0 == g1).all())
    assert b.t == 20
    b.step(40)
    singles = _singles(L, cases, 60)
    for bc, sc in zip(b.cases, singles):
        assert _same(bc, sc) and _same_samples(bc, sc)
    b2 = _batch(L, cases)
    w2, r2, m2, p2, ms2 = b2.autotune(6)
    assert (w2, r2, m2, p2) == (w, r, m, per) and ms2 == -1.0   # same shapes: from the cache
    b.close()
    b2.close()


def test_batch_tile_shapes_are_bitwise_equal(gpu_lib):
    L = gpu_lib
    cases = _cases()
    runs = []
    for shape in [(1, 16, False, True), (2, 7, True, False), (4, 64, False, False), (4, 32, True, True),
                  (4, 1, False, False), (2, 1, False, True), (1, 1, False, False), (1, 1, True, True)]:
        b = _batch(L, cases)
        b.set_tiling(*shape)
        b.set_graph(10)
        b.step(50)
        runs.append(b)
    for i in range(len(cases)):
        for other in runs[1:]:
            assert _same(runs[0].cases[i], other.cases[i]), i
    for b in runs:
        b.close()


def test_batch_member_over_4gib_steps_as_alone(gpu_lib):
    """A member whose buffer takes more than 4 GiB (2048 x 37000 nodes, 4.4 GB
    per buffer: row bases past 32-bit byte offsets) evolves bit for bit as when
    stepped alone, beside a small member, with one and two waves per row
    workgroup."""
    import torch
    L = gpu_lib
    big_nx, big_ny = 2048, 37000
    pb = W.base_params(big_nx, big_ny, bc_y=W.BC_PERIODIC, tau_ink=0.8, force_rows=big_ny, f_pos=1e-5,
                       t_pos=10 ** 6, diag_every=K, diag_row0=2)
    cases = [(pb, W.flat_wall(big_nx, big_ny, (0, 1)),
              W.discs_distance(big_nx, big_ny, [(300.0, 60.0, 40.0), (1500.0, 36900.0, 50.0), (2040.0, 18000.0, 30.0)])),
             _cases()[0]]
    print("member bytes per buffer:", big_ny * (14 * 2048 + 1024) * 4, flush=True)
    b = _batch(L, cases)
    b.set_tiling(1, 1, False, False)
    b.step(3)
    b.set_tiling(2, 1, False, True)
    b.step(2)
    singles = _singles(L, cases, 5)
    for i, (bc, sc) in enumerate(zip(b.cases, singles)):
        assert bc.check() == L.IJ_OK and sc.check() == L.IJ_OK, i
        assert _same(bc, sc), i
    b.close()
    del b, singles
    torch.cuda.empty_cache()
