"""Breakup step, drop velocity, drop volume and the satellite flag of the
GPU library against the FP64 oracle (task tolerance: 1 % on breakup time and
drop velocity), on a drop that pinches off from an ink layer.  Both sides
start from the same float32 phi and velocity fields; the oracle's series of
row segments is reduced by the oracle's own breakup summary, the library's
by its own (ij_get_diagnostics)."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


def _inputs(cfg):
    p = cfg["params"]
    phi_star = 0.5 * (p["rho_ink"] - p["rho_amb"])
    phi = phi_star * np.tanh(2.0 * cfg["distance"] / p["width"])
    phi = np.where(cfg["wall"] != 0, 0.0, phi).astype(np.float32)
    return phi, cfg["uy"].astype(np.float32)


def test_breakup_time_and_drop_velocity_match_oracle(oracle_mod, gpu_lib):
    O, L = oracle_mod, gpu_lib
    cfg = W.config_pinch_off()
    p, wall, row0, K, steps = cfg["params"], cfg["wall"], cfg["row0"], cfg["diag_every"], cfg["steps"]
    ny = p["ny"]
    phi, uy = _inputs(cfg)

    o = O.OracleSim(p, wall)
    o.init_phi(phi.astype(np.float64), None, uy.astype(np.float64))
    series = []
    for k in range(0, steps + 1, K):
        if o.t < k:
            o.step(k - o.t)
        d = o.diag(row0)
        seg = O.segments(d["row_count"], d["row_uy"], row0, 4 * p["width"] ** 2, O.band_rows(p["width"]))
        seg["step"] = k
        series.append(seg)
    ref = O.breakup_summary(series, ny, p["width"])
    o.close()
    assert ref["breakup_step"] > 0 and np.isfinite(ref["v_drop"]), ref

    g = L.Sim(dict(p, diag_row0=row0, diag_every=K), wall)
    g.init_phi(phi, None, uy)
    g.step(steps)
    g.diag_sample()
    gd = g.diagnostics()
    print("oracle", ref, "gpu", {k: gd[k] for k in ("breakup_step", "v_drop", "vol_drop", "satellite")})
    assert g.check() == L.IJ_OK
    tb = ref["breakup_step"]
    assert abs(gd["breakup_step"] - tb) <= 0.01 * tb
    assert abs(gd["v_drop"] - ref["v_drop"]) <= 0.01 * abs(ref["v_drop"])
    assert abs(gd["vol_drop"] - ref["vol_drop"]) <= 0.01 * ref["vol_drop"]
    assert gd["satellite"] == ref["satellite"]
    assert gd["drop_len"] == ref["drop_len"] > 0

    # Fig. 3 / Fig. 4 quantities, sample by sample: the drop's extent exactly
    # and the head and tail velocities within 1e-4 relative plus 1e-5 of the
    # sample's largest speed (the field tolerance: FP32 velocities carry an
    # error that scales with the flow, not with the slow drop tip)
    gs = {s["step"]: s for s in g.samples()}
    n_cmp = 0
    for r in series:
        s = gs[r["step"]]
        assert (s["n_detached"], s["largest_top"], s["largest_bottom"]) == \
            (r["n_detached"], r["largest_top"], r["largest_bottom"]), r["step"]
        if r["n_detached"]:
            tol = 1e-4 * max(abs(r["head_uy"]), abs(r["tail_uy"])) + 1e-5 * s["max_u"]
            assert abs(s["head_uy"] - r["head_uy"]) <= tol, (r["step"], s["head_uy"], r["head_uy"])
            assert abs(s["tail_uy"] - r["tail_uy"]) <= tol, (r["step"], s["tail_uy"], r["tail_uy"])
            n_cmp += 1
    assert n_cmp >= 10


def _compare_summary(gd, ref, what):
    """Breakup step within 1 % (the task tolerance; with samples every 50
    steps that is the same sample or its neighbour), drop velocity and
    volume within 1 %, the satellite flag and the filament length at breakup
    equal."""
    tb = ref["breakup_step"]
    assert tb > 0 and np.isfinite(ref["v_drop"]), (what, ref)
    assert abs(gd["breakup_step"] - tb) <= 0.01 * tb, (what, gd["breakup_step"], tb)
    assert abs(gd["v_drop"] - ref["v_drop"]) <= 0.01 * abs(ref["v_drop"]), (what, gd["v_drop"], ref["v_drop"])
    assert abs(gd["vol_drop"] - ref["vol_drop"]) <= 0.01 * ref["vol_drop"], (what, gd["vol_drop"], ref["vol_drop"])
    assert gd["satellite"] == ref["satellite"], what
    assert gd["drop_len"] == ref["drop_len"], (what, gd["drop_len"], ref["drop_len"])


def test_print_event_and_pulse_train_match_oracle(oracle_mod, gpu_lib):
    """A print event of the paper's validation set-up (Results, "Reproducing
    the experiment"; Fig. 4 at 90 degrees) and the start of a pulse train
    ("Actuation modeling": a full period, the idle time as a control): the
    800 x 200 nozzle lattice at density ratio 1000; the +5 us push and -3 us
    pull pinch the filament off, the drop flies, and after 40 us of idle the
    next push drives a new jet into the drop, which reconnects it.  The
    library and the FP64 oracle, sampled every 50 steps, give the same
    breakup time, drop velocity, drop volume, satellite flag and filament
    length (within 1 %), and the same sequence of detachment and
    reconnection (each step within 1 %)."""
    from parity_util import oracle_series
    O, L = oracle_mod, gpu_lib
    c = W.config_paper(theta=90.0, periodic_pulse=True, pulse_us=(5.0, 3.0, 40.0))
    K = 50
    p = dict(c["params"], diag_row0=c["row0"], diag_every=K)
    u = c["units"]
    n_steps = u.steps(56.0)
    print("paper preset 90 deg, pulse train: FP64 oracle to", n_steps, flush=True)
    series = oracle_series(O, p, c["wall"], c["row0"], K, n_steps)
    ref = O.breakup_summary(series, p["ny"], p["width"])
    g = L.Sim(p, c["wall"])
    g.init_distance(c["distance"])
    g.step(n_steps + 1)   # the step at t samples its input state: up to the oracle's last sample
    gd = g.diagnostics()
    print("oracle", ref, f"({u.microseconds(ref['breakup_step']):.2f} us, {u.velocity_ms(ref['v_drop']):+.4f} m/s)",
          "gpu", {k: gd[k] for k in ("breakup_step", "v_drop", "vol_drop", "satellite", "drop_len")}, flush=True)
    assert g.check() == L.IJ_OK
    _compare_summary(gd, ref, "paper preset 90 deg")
    assert ref["breakup_step"] < p["t_pos"] + p["t_neg"] + p["t_idle"]   # the first drop, before the next push

    def events(ss):
        """steps at which the number of detached drops changes from 0 to
        more (detach) or back to 0 (reconnect)"""
        out, prev = [], 0
        for s in ss:
            now = s["n_detached"] > 0
            if now != (prev > 0):
                out.append(("detach" if now else "reconnect", s["step"]))
            prev = s["n_detached"]
        return out

    ev_o = events(series)
    ev_g = events([s for s in g.samples() if s["step"] <= n_steps])
    print("events: oracle", ev_o, "gpu", ev_g, flush=True)
    assert [e[0] for e in ev_o][:2] == ["detach", "reconnect"], ev_o
    assert [e[0] for e in ev_g] == [e[0] for e in ev_o]
    for (_, a), (_, b) in zip(ev_g, ev_o):
        assert abs(a - b) <= 0.01 * b, (ev_g, ev_o)
    # the second push starts before the reconnection
    assert ev_o[1][1] > p["t_pos"] + p["t_neg"] + p["t_idle"]


# Two cases of the stored surrogate data (contact angles 32 and 145 degrees), each a print event of the 256 x 2048 nozzle with a periodic
# pulse; their targets were written by the batched solver.
STORED = [("sweep_seed9_768.npz", 264), ("sweep_seed8_768.npz", 516)]


def test_stored_sweep_cases_match_oracle(oracle_mod, gpu_lib):
    """The FP64 oracle reruns two cases of the stored training data at
    their parameters (init, pulse and diagnostics as the batched solver that
    wrote them): the stored breakup step, drop velocity and volume agree
    within 1 %, and so does the library stepping them now as a batch."""
    import os
    from paper_1702_04487_amd import surrogate as S
    from parity_util import oracle_series
    O, L = oracle_mod, gpu_lib
    rows = []
    for fn, i in STORED:
        d = np.load(os.path.join(S.DATA_DIR, fn))
        rows.append((d["x"][i], d["y"][i]))
    params = [S.case_params(x) for x, _ in rows]
    b = L.Batch(params)
    for sim in b.cases:
        sim.init_default()
    refs = []
    for (x, y), p in zip(rows, params):
        g = S.GEOMETRY
        wall = W.nozzle_wall(p["nx"], p["ny"], p["nozzle_x0"], p["nozzle_w"], p["nozzle_len"])
        print(f"stored case theta {x[0]:.1f}: FP64 oracle", flush=True)
        # to 3050 steps past the first detached drop: the drop-velocity window
        series = oracle_series(O, p, wall, g["L"], S.DIAG_EVERY, S.HORIZON,
                               stop=lambda ss: any(s["n_detached"] for s in ss) and
                               ss[-1]["step"] >= next(s["step"] for s in ss if s["n_detached"]) + 3050)
        ref = O.breakup_summary(series, p["ny"], p["width"])
        refs.append((ref, series[-1]["step"]))
    b.set_graph(S.DIAG_EVERY)
    b.step(max(r[1] for r in refs) + 1)
    for (x, y), (ref, _), sim in zip(rows, refs, b.cases):
        gd = sim.diagnostics()
        print(f"theta {x[0]:.1f}: stored {y[:3]}, oracle {ref}, library now",
              {k: gd[k] for k in ("breakup_step", "v_drop", "vol_drop")}, flush=True)
        stored = dict(breakup_step=int(y[0]), v_drop=float(y[1]), vol_drop=int(y[2]), satellite=int(y[3]),
                      drop_len=ref["drop_len"])
        _compare_summary(stored, ref, ("stored", x[0]))
        _compare_summary(gd, ref, ("library", x[0]))
    b.close()
