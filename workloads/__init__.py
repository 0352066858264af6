"""Seeded synthetic workloads: lattice geometry, initial signed-distance
fields, parameter presets and sweep case tables.

Both the FP64 oracle and the GPU library take their inputs from here.  The
module holds no arithmetic of the lattice Boltzmann method itself: it builds
wall masks, signed distances to the ink region and parameter tables, and each
side turns them into distributions on its own.

Geometry follows the paper's simulation set-up (Results, "Reproducing the
experiment"): periodic left/right, a nozzle channel at the bottom opening into
an ambient chamber, open ("fully developed") bottom and top rows, wetting
walls.  The validation lattice of the paper (800 x 200, nozzle 120 high, radius
40) is replaced by the synthetic configurations below, which keep its
structure.
"""
from __future__ import annotations

import math
from typing import Iterable, List, Sequence, Tuple

import numpy as np

FLUID, WALL_INNER, WALL_OUTER = 0, 1, 2
BC_PERIODIC, BC_OPEN = 0, 1

MASK64 = (1 << 64) - 1


# ------------------------------------------------------------------ RNG
class SplitMix64:
    """SplitMix64 (Steele, Lea & Flood, OOPSLA 2014): counter-based 64-bit
    generator, used for every seeded draw so that the sequence is fixed by
    its published definition rather than by a library version."""

    def __init__(self, seed: int):
        self.state = seed & MASK64

    def next_u64(self) -> int:
        self.state = (self.state + 0x9E3779B97F4A7C15) & MASK64
        z = self.state
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK64
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK64
        return z ^ (z >> 31)

    def uniform(self, lo: float = 0.0, hi: float = 1.0) -> float:
        return lo + (hi - lo) * ((self.next_u64() >> 11) * (1.0 / (1 << 53)))

    def randint(self, lo: int, hi: int) -> int:
        """Uniform integer in [lo, hi] (inclusive)."""
        return lo + int(self.uniform() * (hi - lo + 1)) if hi > lo else lo


# ------------------------------------------------------------- geometry
def nozzle_wall(nx: int, ny: int, x0: int, w: int, length: int) -> np.ndarray:
    """Solid band y < length except the channel x0 <= x < x0 + w.  The two
    columns that line the channel are the inner wall (class 1, the nozzle
    inner wall whose contact angle the paper varies); the rest of the band,
    including its top face, is the outer plate (class 2)."""
    wall = np.zeros((ny, nx), dtype=np.uint8)
    if w <= 0 or length <= 0:
        return wall
    wall[:length, :] = WALL_OUTER
    wall[:length, x0:x0 + w] = FLUID
    wall[:length, (x0 - 1) % nx] = WALL_INNER
    wall[:length, (x0 + w) % nx] = WALL_INNER
    return wall


def channel_wall(nx: int, ny: int, x0: int, w: int) -> np.ndarray:
    """Full-height vertical channel x0 <= x < x0 + w between inner walls."""
    wall = np.full((ny, nx), WALL_INNER, dtype=np.uint8)
    wall[:, x0:x0 + w] = FLUID
    return wall


def flat_wall(nx: int, ny: int, rows: Iterable[int] = (0,), cls: int = WALL_INNER) -> np.ndarray:
    wall = np.zeros((ny, nx), dtype=np.uint8)
    for r in rows:
        wall[r, :] = cls
    return wall


# ------------------------------------------------------ signed distances
def meniscus_distance(nx: int, ny: int, length: int) -> np.ndarray:
    """Ink fills the rows below the nozzle exit: flat meniscus half a node
    above the last nozzle row.  Positive inside the ink."""
    y = np.arange(ny, dtype=np.float64)[:, None]
    return np.broadcast_to(length - 0.5 - y, (ny, nx)).copy()


def discs_distance(nx: int, ny: int, discs: Sequence[Tuple[float, float, float]],
                   periodic: bool = True, far: float = -1.0e3) -> np.ndarray:
    """Signed distance to a union of discs (max over discs of R - |x - c|),
    evaluated within a margin of each disc; `far` elsewhere."""
    d = np.full((ny, nx), far, dtype=np.float64)
    margin = 24.0
    for (cx, cy, r) in discs:
        ext = int(math.ceil(r + margin))
        xs = np.arange(int(math.floor(cx)) - ext, int(math.floor(cx)) + ext + 2)
        ys = np.arange(int(math.floor(cy)) - ext, int(math.floor(cy)) + ext + 2)
        if periodic:
            xi, yi = xs % nx, ys % ny
        else:
            kx = (xs >= 0) & (xs < nx)
            ky = (ys >= 0) & (ys < ny)
            xs, ys = xs[kx], ys[ky]
            xi, yi = xs, ys
        dist = np.sqrt((xs[None, :] - cx) ** 2 + (ys[:, None] - cy) ** 2)
        sub = d[np.ix_(yi, xi)]
        d[np.ix_(yi, xi)] = np.maximum(sub, r - dist)
    return d


def sample_discs(nx: int, ny: int, seed: int = 0, rmin: float = 8.0, rmax: float = 64.0,
                 gap: float = 4.0, area_frac: float = 0.25, y_lo: float = 1.0,
                 max_tries: int = 2_000_000) -> List[Tuple[float, float, float]]:
    """Non-overlapping discs (clearance >= gap, periodic in x and y) with radii
    uniform in [rmin, rmax] and uniform centres, drawn by rejection until the
    ink area fraction reaches area_frac.  Discs stay at least `gap` away from
    the rows y < y_lo (a flat wall there and its periodic image)."""
    rng = SplitMix64(seed)
    cx = np.zeros(0)
    cy = np.zeros(0)
    rr = np.zeros(0)
    area = 0.0
    target = area_frac * nx * ny
    tries = 0
    while area < target and tries < max_tries:
        tries += 1
        r = rng.uniform(rmin, rmax)
        x = rng.uniform(0.0, nx)
        y = rng.uniform(y_lo + gap + r, ny - gap - r)
        if y_lo + gap + r >= ny - gap - r:
            continue
        if len(rr):
            dx = np.abs(cx - x)
            dx = np.minimum(dx, nx - dx)
            dy = np.abs(cy - y)
            dy = np.minimum(dy, ny - dy)
            if np.any(np.sqrt(dx * dx + dy * dy) < rr + r + gap):
                continue
        cx = np.append(cx, x)
        cy = np.append(cy, y)
        rr = np.append(rr, r)
        area += math.pi * r * r
    return list(zip(cx.tolist(), cy.tolist(), rr.tolist()))


# -------------------------------------------------------------- presets
def base_params(nx: int, ny: int, **kw) -> dict:
    p = dict(nx=nx, ny=ny, bc_y=BC_OPEN, force_rows=0, t_pos=0, t_neg=0, t_idle=0,
             periodic_pulse=0, rho_ink=1.0, rho_amb=0.1, sigma=0.01, width=4.0, gamma=1.0,
             tau_ink=1.0, tau_amb=1.0, tau_phi=1.0, theta_inner=90.0, theta_outer=90.0,
             f_pos=0.0, f_neg=0.0)
    p.update(kw)
    return p


def config_nozzle_small() -> dict:
    """64 x 256 nozzle case (FP64 parity workload): channel 16 wide and 64
    long, density 1.0/0.1, tau 1, contact angle 90 deg, pulse +1e-4 for 200
    steps, -5e-5 for 100, then idle; 1000 steps."""
    nx, ny, x0, w, L = 64, 256, 24, 16, 64
    p = base_params(nx, ny, force_rows=L, t_pos=200, t_neg=100, t_idle=700,
                    f_pos=1e-4, f_neg=5e-5)
    return dict(name="nozzle_64x256", params=p, wall=nozzle_wall(nx, ny, x0, w, L),
                distance=meniscus_distance(nx, ny, L), row0=L, steps=1000,
                nozzle=(x0, w, L))


def config_nozzle_single() -> dict:
    """256 x 2048 single nozzle case: channel 32 wide and 256 long, contact
    angle 60 deg, tau 0.8 ink / 1.0 ambient, pulse +2e-4 for 2000 steps,
    -1e-4 for 1000, idle to 60000 steps."""
    nx, ny, w, L = 256, 2048, 32, 256
    x0 = (nx - w) // 2
    p = base_params(nx, ny, force_rows=L, t_pos=2000, t_neg=1000, t_idle=57000,
                    f_pos=2e-4, f_neg=1e-4, tau_ink=0.8, theta_inner=60.0)
    return dict(name="nozzle_256x2048", params=p, wall=nozzle_wall(nx, ny, x0, w, L),
                distance=None, row0=L, steps=60000, nozzle=(x0, w, L))


class PaperUnits:
    """Lattice <-> physical units of the paper's validation run (Results,
    "Reproducing the experiment"): silicone oil of density 930 kg/m^3,
    viscosity 9.3 mPa s, nozzle radius 15 um = 40 nodes.  The length unit
    follows from the radius, the time unit from the kinematic viscosity
    nu = (tau_n - 1/2) / 3 of the lattice (tau_n = 0.85, so nu = 0.1167; the
    0.17 printed beside it would put sigma = 1.08 at 9.3 mN/m instead of the
    oil's 20.2), the mass unit from the liquid density (1000 in the
    lattice)."""

    def __init__(self, radius_um: float = 15.0, radius_lu: float = 40.0, tau_n: float = 0.85,
                 rho_phys: float = 930.0, mu_phys: float = 9.3e-3, rho_lu: float = 1000.0):
        self.dx = radius_um * 1e-6 / radius_lu                       # m per node
        self.nu_lu = (tau_n - 0.5) / 3.0
        self.dt = self.nu_lu * self.dx ** 2 / (mu_phys / rho_phys)     # s per step
        self.dm = rho_phys / rho_lu * self.dx ** 3                     # kg per lattice mass unit

    def steps(self, microseconds: float) -> int:
        return int(round(microseconds * 1e-6 / self.dt))

    def microseconds(self, steps: float) -> float:
        return steps * self.dt * 1e6

    def velocity_ms(self, u_lu: float) -> float:
        return u_lu * self.dx / self.dt

    def sigma_lu(self, sigma_mn_per_m: float) -> float:
        # N/m = kg / s^2
        return sigma_mn_per_m * 1e-3 * self.dt ** 2 / self.dm

    def sigma_mn_per_m(self, sigma_lu: float) -> float:
        return sigma_lu * self.dm / self.dt ** 2 * 1e3


# Mobility of the paper preset (the paper does not print it).  The
# Cahn-Hilliard diffusivity of a bulk phase is theta_M * d(mu)/d(phi) =
# theta_M * 8 beta phi*^2 = theta_M * 6 sigma / (W phi*^2); at phi* = 499.5 a
# mobility of order one leaves the interface practically frozen (four orders
# below the presets above).  GAMMA_PAPER gives the diffusivity of the presets
# above (sigma 0.01, W 4, phi* 0.45, Gamma 1, tau_phi 1: 8.2e-3) at sigma
# 1.08, W 3, tau_phi 0.8.  For other sigma the mobility scales as 1.08 /
# sigma, which keeps that diffusivity and theta_M * kappa (the explicit
# scheme's fourth-order term) fixed: at a fixed Gamma, theta_M kappa pi^4
# grows from 0.45 at sigma 1.08 to 1.95 at 85 mN/m, and the runs above
# 30 mN/m went unstable within 300 steps.
GAMMA_PAPER = 1.07e4

# Pulse amplitudes of the paper preset (not printed in the paper): a push and
# a 16 % stronger pull that pinch the ejected filament off at about 42 us at
# 90 degrees, and stay within the speed guard over the whole 20-85 mN/m range
# (a 0.07 / 0.08 pulse breaks at 45 us but trips the guard from 50 mN/m up).
F_POS_PAPER, F_NEG_PAPER = 5.0e-2, 5.8e-2


def config_paper(theta: float = 90.0, sigma_mn_per_m: float = None, f_pos: float = F_POS_PAPER,
                 f_neg: float = F_NEG_PAPER, gamma: float = None, pulse_us=(5.0, 3.0, 8.0),
                 periodic_pulse: bool = False, steps_us: float = 130.0, theta_outer: float = 90.0) -> dict:
    """The paper's validation lattice: 200 wide and 800 long (jet along y),
    nozzle 120 high with radius 40 (an 80-wide channel), densities 1000/1
    (phi* = 499.5), W = 3, tau_n = 0.85, tau_phi = 0.8, sigma = 1.08 (or the
    value of sigma_mn_per_m in physical units), periodic sides, open top and
    bottom rows, contact angle theta on the nozzle inner wall.  Pulse: +5 us,
    -3 us, 8 us idle (Fig. 1), converted with PaperUnits.  The force
    amplitudes and the mobility are not printed in the paper: f_pos, f_neg
    and gamma (default GAMMA_PAPER * 1.08 / sigma) are this preset's
    choice."""
    u = PaperUnits()
    nx, ny, L, w = 200, 800, 120, 80
    x0 = (nx - w) // 2
    sigma = 1.08 if sigma_mn_per_m is None else u.sigma_lu(sigma_mn_per_m)
    if gamma is None:
        gamma = GAMMA_PAPER * 1.08 / sigma
    tp, tn, ti = (u.steps(t) for t in pulse_us)
    p = base_params(nx, ny, force_rows=L, t_pos=tp, t_neg=tn, t_idle=ti, periodic_pulse=int(periodic_pulse),
                    rho_ink=1000.0, rho_amb=1.0, sigma=sigma, width=3.0, gamma=gamma, tau_ink=0.85,
                    tau_amb=0.85, tau_phi=0.8, theta_inner=theta, theta_outer=theta_outer, f_pos=f_pos,
                    f_neg=f_neg)
    return dict(name=f"paper_{nx}x{ny}", params=p, wall=nozzle_wall(nx, ny, x0, w, L),
                distance=meniscus_distance(nx, ny, L), row0=L, steps=u.steps(steps_us), nozzle=(x0, w, L),
                units=u)


def config_droplet_field(nx: int = 2048, ny: int = 16384, seed: int = 0,
                         with_distance: bool = True) -> dict:
    """Roofline stress: seeded disc field (radii 8-64, ink area >= 25 %),
    periodic in x and y, a flat wetting wall at 120 deg in rows y = 0, 1 (two
    rows, so that each face of the wall sees only its own side), no driving
    force, tau 0.8 ink / 1.0 ambient, 5000 steps."""
    p = base_params(nx, ny, bc_y=BC_PERIODIC, force_rows=ny, tau_ink=0.8,
                    theta_inner=120.0, theta_outer=120.0)
    cfg = dict(name=f"droplets_{nx}x{ny}", params=p, wall=flat_wall(nx, ny, (0, 1)), row0=2,
               steps=5000, nozzle=None)
    if with_distance:
        discs = sample_discs(nx, ny, seed=seed, rmin=8.0, rmax=min(64.0, ny / 8, nx / 8),
                             gap=p["width"], area_frac=0.25, y_lo=2.0)
        cfg["discs"] = discs
        cfg["distance"] = discs_distance(nx, ny, discs, periodic=True)
    return cfg


def config_pinch_off(nx: int = 96, ny: int = 320, u_blob: float = 0.05) -> dict:
    """A drop that detaches: an ink layer on a two-row flat wall (rows 0, 1,
    90 deg), a neck one interface width wide rising from it, and a disc of
    radius 22 on top of the neck given an upward velocity u_blob (smoothly
    cut off 2 nodes outside the disc).  The neck is thinner than the
    interface profile, so it pinches and the disc detaches (breakup near
    step 900).  Periodic in x and y; no driving force; diagnostics every 10
    steps from row 2.  Returns the signed distance to the ink region and the
    initial u_y."""
    p = base_params(nx, ny, bc_y=BC_PERIODIC, force_rows=0, tau_ink=0.8)
    wall = flat_wall(nx, ny, (0, 1))
    cx, cy, r, neck = nx / 2.0, 120.0, 22.0, 4.0
    y = np.arange(ny, dtype=np.float64)[:, None]
    x = np.arange(nx, dtype=np.float64)[None, :] + 0.5
    d_layer = np.broadcast_to(24.0 - y, (ny, nx))
    d_neck = np.minimum(np.minimum(neck / 2 - np.abs(x - cx), 100.0 - y), y - 10.0)
    rb = np.sqrt((x - cx) ** 2 + (y - cy) ** 2)
    d = np.maximum(np.maximum(d_layer, d_neck), r - rb)
    uy = u_blob * 0.5 * (1.0 - np.tanh((rb - r - 2.0) / 3.0))
    uy = np.where(wall != 0, 0.0, uy)
    return dict(name=f"pinch_off_{nx}x{ny}", params=p, wall=wall, distance=np.ascontiguousarray(d),
                uy=np.ascontiguousarray(uy), row0=2, diag_every=10, steps=4000, nozzle=None)


def sweep_cases(n: int = 256, seed: int = 1234, steps: int = 40000,
                nx_range=(128, 384), ny_range=(1024, 3072), w_range=(12, 40),
                theta_range=(30.0, 150.0), sigma_range=(0.005, 0.02),
                f_range=(5e-5, 3e-4), t_range=(500, 3000), periodic_pulse=0,
                stable: bool = False, u_cap: float = 0.2, gamma_sigma_max: float = 0.01,
                diag_every: int = 50) -> List[dict]:
    """Seeded table of independent nozzle cases for a parameter sweep
    (contact angle x surface tension x pulse, uneven lattice sizes).

    With ``stable`` the table is the scaled variant used for measurement and
    training data: the mobility Gamma is lowered so that Gamma * sigma <=
    gamma_sigma_max (larger products are numerically unstable at W = 4), and
    both pulse amplitudes are scaled by one factor so that the viscous
    centreline speed of the nozzle channel, F w^2 / (8 n0 nu_ink), stays at or
    below u_cap.  The draws (and so every other parameter) are the same."""
    rng = SplitMix64(seed)
    out = []
    for k in range(n):
        nx = rng.randint(*nx_range)
        ny = rng.randint(*ny_range)
        w = rng.randint(*w_range)
        theta = rng.uniform(*theta_range)
        sigma = math.exp(rng.uniform(math.log(sigma_range[0]), math.log(sigma_range[1])))
        fp = rng.uniform(*f_range)
        fn = rng.uniform(*f_range)
        tp = rng.randint(*t_range)
        tn = rng.randint(*t_range)
        ti = rng.randint(*t_range)
        L = ny // 8
        x0 = (nx - w) // 2
        gamma = 1.0
        if stable:
            gamma = min(1.0, gamma_sigma_max / sigma)
            n0 = 0.5 * (1.0 + 0.1)
            nu_ink = (0.8 - 0.5) / 3.0
            bound = max(fp, fn) * w * w / (8.0 * n0 * nu_ink)
            scale = min(1.0, u_cap / bound)
            fp, fn = fp * scale, fn * scale
        p = base_params(nx, ny, force_rows=L, t_pos=tp, t_neg=tn, t_idle=ti,
                        periodic_pulse=periodic_pulse, f_pos=fp, f_neg=fn, tau_ink=0.8,
                        theta_inner=theta, sigma=sigma, gamma=gamma, nozzle_x0=x0, nozzle_w=w,
                        nozzle_len=L, diag_row0=L, diag_every=diag_every)
        out.append(dict(name=f"case{k}", params=p, nozzle=(x0, w, L), row0=L, steps=steps))
    return out


def case_wall(case: dict) -> np.ndarray:
    p = case["params"]
    x0, w, L = case["nozzle"]
    return nozzle_wall(p["nx"], p["ny"], x0, w, L)


def case_distance(case: dict) -> np.ndarray:
    p = case["params"]
    return meniscus_distance(p["nx"], p["ny"], case["nozzle"][2])


# ------------------------------------------------------------ surrogate
def splitmix64_array(seed: int, n: int, offset: int = 0) -> np.ndarray:
    """Outputs offset .. offset+n-1 of SplitMix64 started at `seed`
    (vectorised; the same sequence as SplitMix64(seed).next_u64())."""
    with np.errstate(over="ignore"):
        k = np.arange(offset + 1, offset + n + 1, dtype=np.uint64)
        z = np.uint64(seed & MASK64) + k * np.uint64(0x9E3779B97F4A7C15)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        return z ^ (z >> np.uint64(31))


def uniform_array(seed: int, n: int, lo: float = 0.0, hi: float = 1.0, offset: int = 0) -> np.ndarray:
    u = (splitmix64_array(seed, n, offset) >> np.uint64(11)).astype(np.float64) * (1.0 / (1 << 53))
    return lo + (hi - lo) * u


MLP_SIZES = (7, 128, 128, 4)


def mlp_init(seed: int) -> dict:
    """Initial weights of one ensemble member: W and b uniform in
    +/- 1/sqrt(fan_in) (float64; W1 [128, 7], W2 [128, 128], W3 [4, 128]).
    Random biases make the members differ in where their units switch on,
    which the ensemble spread needs: with zero biases the trust region
    answered 57 % of the held-out cases instead of 65 %."""
    out, off = {}, 0
    for l, (fi, fo) in enumerate(zip(MLP_SIZES[:-1], MLP_SIZES[1:]), start=1):
        a = 1.0 / math.sqrt(fi)
        out[f"W{l}"] = uniform_array(seed, fo * fi, -a, a, off).reshape(fo, fi)
        off += fo * fi
        out[f"b{l}"] = uniform_array(seed, fo, -a, a, off)
        off += fo
    return out


def minibatch_order(seed: int, n: int, steps: int, batch: int) -> np.ndarray:
    """[steps, batch] sample indices drawn uniformly from [0, n) (int32)."""
    u = uniform_array(seed, steps * batch)
    return np.minimum((u * n).astype(np.int64), n - 1).astype(np.int32).reshape(steps, batch)


# ------------------------------------------------- three-dimensional inputs
# Arrays are indexed [y, z, x]: x periodic (width), y the jet direction,
# z periodic (depth).
def round_nozzle_wall3d(nx: int, ny: int, nz: int, radius: float, length: int,
                        xc: float = None, zc: float = None) -> np.ndarray:
    """Solid plate y < length with a round bore of the given radius about
    (xc, zc) (default: the centre of the x-z section).  Solid nodes next to the
    bore in the x-z plane (8 neighbours) are the inner wall (class 1); the rest
    of the plate, including its top face, is the outer plate (class 2)."""
    xc = (nx - 1) / 2.0 if xc is None else xc
    zc = (nz - 1) / 2.0 if zc is None else zc
    z, x = np.meshgrid(np.arange(nz, dtype=np.float64), np.arange(nx, dtype=np.float64), indexing="ij")
    bore = (x - xc) ** 2 + (z - zc) ** 2 < radius * radius
    near = np.zeros_like(bore)
    for dz in (-1, 0, 1):
        for dx in (-1, 0, 1):
            near |= np.roll(np.roll(bore, dz, axis=0), dx, axis=1)
    sec = np.where(bore, FLUID, np.where(near, WALL_INNER, WALL_OUTER)).astype(np.uint8)
    wall = np.zeros((ny, nz, nx), dtype=np.uint8)
    if length > 0:
        wall[:length] = sec[None]
    return wall


def meniscus_distance3d(nx: int, ny: int, nz: int, length: int) -> np.ndarray:
    """Ink below the nozzle exit, flat meniscus half a node above the last
    nozzle row; positive inside the ink."""
    y = np.arange(ny, dtype=np.float64)[:, None, None]
    return np.broadcast_to(length - 0.5 - y, (ny, nz, nx)).copy()


def spheres_distance3d(nx: int, ny: int, nz: int, spheres: Sequence[Tuple[float, float, float, float]],
                       far: float = -1.0e3, periodic_y: bool = True) -> np.ndarray:
    """Signed distance to a union of spheres (cx, cy, cz, r) in a box periodic
    in x and z, and in y unless periodic_y is False (max over spheres of
    r - |x - c|, nearest image)."""
    y, z, x = np.meshgrid(np.arange(ny, dtype=np.float64), np.arange(nz, dtype=np.float64),
                          np.arange(nx, dtype=np.float64), indexing="ij")
    d = np.full((ny, nz, nx), far, dtype=np.float64)
    for (cx, cy, cz, r) in spheres:
        dx = np.abs(x - cx)
        dx = np.minimum(dx, nx - dx)
        dy = np.abs(y - cy)
        if periodic_y:
            dy = np.minimum(dy, ny - dy)
        dz = np.abs(z - cz)
        dz = np.minimum(dz, nz - dz)
        d = np.maximum(d, r - np.sqrt(dx * dx + dy * dy + dz * dz))
    return d


def base_params3d(nx: int, ny: int, nz: int, **kw) -> dict:
    p = base_params(nx, ny, **kw)
    p["nz"] = nz
    return p


def config_round_nozzle_small() -> dict:
    """32 x 96 x 32 round nozzle (FP64 parity workload): bore radius 8 and
    length 32, density 1.0/0.1, tau 0.8 ink / 1.0 ambient, Gamma 0.5, contact
    angles 60 (bore) and 120 (plate), pulse +1e-3 for 60 steps, -5e-4 for 30,
    idle."""
    nx, ny, nz, r, L = 32, 96, 32, 8.0, 32
    p = base_params3d(nx, ny, nz, force_rows=L, t_pos=60, t_neg=30, t_idle=1000, f_pos=1e-3, f_neg=5e-4,
                      tau_ink=0.8, theta_inner=60.0, theta_outer=120.0, gamma=0.5)
    return dict(name="round_nozzle_32x96x32", params=p, wall=round_nozzle_wall3d(nx, ny, nz, r, L),
                distance=meniscus_distance3d(nx, ny, nz, L), row0=L, steps=200, nozzle=(r, L))


def config_round_nozzle(nx: int = 256, ny: int = 512, nz: int = 256) -> dict:
    """256 x 512 x 256 round nozzle (33.6 M nodes, the node count of the
    2048 x 16384 droplet field): bore radius 32 and length 128, the ejecting
    case's fluid (Gamma 0.5), its pulse scaled by (16/32)^2 to the same
    viscous speed bound in the wider bore, durations by 2^2."""
    r, L = 32.0, 128
    p = base_params3d(nx, ny, nz, force_rows=L, t_pos=32000, t_neg=12000, t_idle=10 ** 6, f_pos=3e-5,
                      f_neg=3e-5, tau_ink=0.8, theta_inner=60.0, theta_outer=120.0, gamma=0.5)
    return dict(name=f"round_nozzle_{nx}x{ny}x{nz}", params=p, wall=round_nozzle_wall3d(nx, ny, nz, r, L),
                distance=meniscus_distance3d(nx, ny, nz, L), row0=L, steps=60000, nozzle=(r, L))


def config_round_nozzle_eject() -> dict:
    """128 x 512 x 128 round nozzle that ejects ink: bore radius 16 and
    length 96, density 1.0/0.1, tau 0.8 ink / 1.0 ambient, sigma 0.01,
    Gamma 0.5 (at Gamma 1 the three-dimensional update blows up at the
    interface), contact angles 60 (bore) and 120 (plate); push +1.2e-4 for
    8000 steps (speed about 0.14, near the viscous bound of the bore), pull
    -1.2e-4 for 3000, idle; the neck pinches off near step 15 500."""
    nx = nz = 128
    ny, r, L = 512, 16.0, 96
    p = base_params3d(nx, ny, nz, force_rows=L, t_pos=8000, t_neg=3000, t_idle=10 ** 6, f_pos=1.2e-4,
                      f_neg=1.2e-4, tau_ink=0.8, theta_inner=60.0, theta_outer=120.0, gamma=0.5)
    return dict(name="round_nozzle_eject_128x512x128", params=p, wall=round_nozzle_wall3d(nx, ny, nz, r, L),
                distance=meniscus_distance3d(nx, ny, nz, L), row0=L, steps=18000, nozzle=(r, L))
