"""Unit conversion of the paper preset (Results, "Reproducing the
experiment"): the radius fixes the length unit, the lattice viscosity
(tau_n - 1/2) / 3 the time unit, the liquid density the mass unit."""
import math

import workloads as W


def test_units_of_the_validation_run():
    u = W.PaperUnits()
    assert math.isclose(u.dx, 0.375e-6, rel_tol=1e-12)                 # 15 um over 40 nodes
    nu_lu = (0.85 - 0.5) / 3.0
    assert math.isclose(u.dt, nu_lu * u.dx ** 2 / (9.3e-3 / 930.0), rel_tol=1e-12)
    assert math.isclose(u.dt, 1.640625e-9, rel_tol=1e-9)
    # sigma = 1.08 in lattice units is the oil's 20.2 mN/m within 3 %
    assert abs(u.sigma_mn_per_m(1.08) - 20.2) / 20.2 < 0.03
    assert math.isclose(u.sigma_lu(u.sigma_mn_per_m(1.08)), 1.08, rel_tol=1e-12)
    # the breakup window of Fig. 2 (50-60 us) and the 1.5 m/s drop in lattice units
    assert (u.steps(50.0), u.steps(60.0)) == (30476, 36571)
    assert math.isclose(u.velocity_ms(1.5 * u.dt / u.dx), 1.5, rel_tol=1e-12)


def test_paper_preset_geometry_and_pulse():
    c = W.config_paper(theta=120.0, sigma_mn_per_m=50.0)
    p, wall = c["params"], c["wall"]
    assert (p["nx"], p["ny"]) == (200, 800) and wall.shape == (800, 200)
    # 80-wide channel (radius 40) through a 120-row plate, centred
    assert (wall[:120, 60:140] == W.FLUID).all() and (wall[:120, 59] == W.WALL_INNER).all()
    assert (wall[:120, 140] == W.WALL_INNER).all() and (wall[120:] == W.FLUID).all()
    assert math.isclose(p["rho_ink"] - p["rho_amb"], 2 * 499.5)
    u = c["units"]
    assert (p["t_pos"], p["t_neg"], p["t_idle"]) == (u.steps(5.0), u.steps(3.0), u.steps(8.0))
    assert math.isclose(u.sigma_mn_per_m(p["sigma"]), 50.0, rel_tol=1e-12)
    assert p["theta_inner"] == 120.0
