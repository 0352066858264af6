"""The paper's validation lattice (Results, "Reproducing the experiment"):
800 x 200, nozzle 120 high with radius 40, densities 1000/1 (phi* = 499.5),
W = 3, tau_n = 0.85, tau_phi = 0.8, sigma = 1.08.  The GPU library against the
FP64 oracle on the full lattice while the positive pulse drives the ink: at
this density ratio the populations are O(100) and the order parameter O(500),
so this is the case that exercises the precision design (shifted f, the
double-precision phi path and the g_0 remainder plane)."""
import numpy as np
import pytest

import workloads as W
from test_gpu_parity import _compare_fields, _pair

pytestmark = pytest.mark.gpu


def test_paper_preset_matches_oracle(oracle_mod, gpu_lib):
    c = W.config_paper()
    o, g = _pair(oracle_mod, gpu_lib, c["params"], c["wall"], c["distance"])
    worst = {}
    for t in (100, 300, 600):
        o.step(t - o.t)
        g.step(t - g.t)
        for k, v in _compare_fields(o, g, 1e-5).items():
            worst[k] = max(worst.get(k, 0.0), v)
    print("worst relative L2:", worst)


THETAS = (30.0, 60.0, 90.0, 120.0, 150.0)
SIGMAS = (20.0, 40.0, 60.0, 85.0)   # mN/m
# A weaker push and pull (found by a scan of the unprinted amplitudes) that
# puts the 90-degree breakup inside the paper's 50-60 us window
WINDOW_PULSE = dict(f_pos=0.04, f_neg=0.0464)


def test_paper_trends(gpu_lib):
    """Discussion, Figs. 5 and 7: with the paper preset (pulse of this
    preset, see config_paper), the filament breaks up later on a more
    hydrophobic nozzle wall and sooner with a higher surface tension.  The
    force amplitudes are not printed, so the absolute times are pinned at
    one point only: with the weaker WINDOW_PULSE the 90-degree filament
    breaks up between 50 and 60 us, as in the paper's validation run
    (Results, "Reproducing the experiment"; Fig. 4(c): 51.89 us), and the
    contact-angle trend holds there too.  (That pulse is too weak to pinch
    the filament off above 30 mN/m, so the surface-tension sweep keeps the
    preset's pulse.)  Also the recoil of the tail after the pinch-off
    (Fig. 3)."""
    specs = [dict(theta=t) for t in THETAS] + [dict(sigma_mn_per_m=s) for s in SIGMAS] + \
        [dict(theta=t, **WINDOW_PULSE) for t in THETAS]
    cfgs = [W.config_paper(**sp) for sp in specs]
    b = gpu_lib.Batch([dict(c["params"], diag_row0=c["row0"], diag_every=50) for c in cfgs],
                      [c["wall"] for c in cfgs])
    for sim, c in zip(b.cases, cfgs):
        sim.init_distance(c["distance"])
    b.set_graph(50)
    b.step(40000)
    u = cfgs[0]["units"]
    res = []
    for sp, sim in zip(specs, b.cases):
        d = sim.diagnostics()
        assert d["unstable_step"] < 0, sp
        assert d["breakup_step"] > 0, sp
        res.append((u.microseconds(d["breakup_step"]), u.velocity_ms(d["v_drop"])))
        print(sp, f"breakup {res[-1][0]:.1f} us, drop velocity {res[-1][1]:+.3f} m/s")
    # Fig. 3 at 90 degrees: after the pinch-off the tail recoils towards the
    # head (tail faster than head over the first 3 us) and the drop contracts
    k90 = THETAS.index(90.0)
    sim = b.cases[k90]
    tb = sim.diagnostics()["breakup_step"]
    after = [x for x in sim.samples() if x["step"] >= tb and x["largest_count"] > 0]
    early = [x for x in after if x["step"] <= tb + u.steps(3.0)]
    recoil = np.mean([x["tail_uy"] - x["head_uy"] for x in early])
    length = [x["largest_top"] - x["largest_bottom"] + 1 for x in after]
    print(f"90 deg: tail - head over the first 3 us {u.velocity_ms(recoil):+.3f} m/s; "
          f"drop length {length[0]} -> {length[-1]} rows over {u.microseconds(after[-1]['step'] - tb):.1f} us")
    assert recoil > 0 and length[-1] < length[0] - 5
    tb_theta = [r[0] for r in res[:len(THETAS)]]
    tb_sigma = [r[0] for r in res[len(THETAS):len(THETAS) + len(SIGMAS)]]
    tb_window = [r[0] for r in res[len(THETAS) + len(SIGMAS):]]
    # the paper's validation window at 90 degrees, and the contact-angle trend at that pulse
    assert 50.0 <= tb_window[THETAS.index(90.0)] <= 60.0, tb_window
    assert all(a <= b for a, b in zip(tb_window, tb_window[1:])) and tb_window[-1] > tb_window[0] + 2.0
    # breakup later with the contact angle (paper: 37 -> 62 us from 30 to 150 deg)
    assert all(a <= b for a, b in zip(tb_theta, tb_theta[1:])) and tb_theta[-1] > tb_theta[0] + 2.0
    # breakup sooner with the surface tension (paper: 18 us sooner from 20 to 85 mN/m)
    assert all(a >= b for a, b in zip(tb_sigma, tb_sigma[1:])) and tb_sigma[-1] < tb_sigma[0] - 2.0
