"""Comparison helpers shared by the GPU parity tests (not a test module).

Tolerances are the parity bar of FP32 against the FP64 oracle: relative L2
over fluid nodes of n, phi, rho = n + phi and the velocity vector field
(one bound for all), and, where asked, an element-wise bound on n and phi
relative to their natural scales n0 and phi* (so that an error concentrated
at a few interface nodes cannot hide in a global norm)."""
import numpy as np


def rel_l2(a, b):
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


def np64(t):
    return t.detach().cpu().numpy().astype(np.float64)


def compare_state(o, g, tol):
    """Every distribution of every fluid node within tol (absolute)."""
    fo, go = o.get_state()
    fg, gg = g.state()
    fl = (o.wall == 0)[None]
    df = np.abs(np.where(fl, np64(fg) - fo, 0.0)).max()
    dg = np.abs(np.where(fl, np64(gg) - go, 0.0)).max()
    assert df < tol and dg < tol, (df, dg)
    return df, dg


def field_errors(o, g):
    mo = o.moments()
    mg = {k: np64(v) for k, v in g.moments().items()}
    fl = o.wall == 0
    errs = {}
    for k in ("n", "phi"):
        errs[k] = rel_l2(mg[k][fl], mo[k][fl])
    errs["rho"] = rel_l2((mg["n"] + mg["phi"])[fl], (mo["n"] + mo["phi"])[fl])
    # velocity as a vector field: relative L2 of (ux, uy) together (a
    # component that is nearly zero by symmetry has no meaningful relative error)
    errs["u"] = rel_l2(np.stack([mg["ux"][fl], mg["uy"][fl]]), np.stack([mo["ux"][fl], mo["uy"][fl]]))
    d = o.derived()
    errs["n_max"] = np.abs(mg["n"] - mo["n"])[fl].max() / d["n0"]
    errs["phi_max"] = np.abs(mg["phi"] - mo["phi"])[fl].max() / d["phi_star"]
    return errs


def compare_fields(o, g, tol, elementwise=False):
    """Relative L2 <= tol on n, phi, rho and u; with elementwise, also
    max |dn| <= tol n0 and max |dphi| <= tol phi* over every fluid node."""
    errs = field_errors(o, g)
    keys = ["n", "phi", "rho", "u"] + (["n_max", "phi_max"] if elementwise else [])
    bad = {k: errs[k] for k in keys if not errs[k] <= tol}
    assert not bad, errs
    return errs


def window_compare(O, p_full, wall, d, g_mom, y0, x0, hw, ww, k, bc_y):
    """Run the oracle on a window of the full lattice.  After k steps every
    node farther than 2k from the window edge depends only on initial data
    inside the window (the stencil plus streaming reach is two nodes per
    step), so there the window run equals the full run.  Returns the largest
    absolute difference of n, phi, ux, uy over those nodes."""
    import workloads as W
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


def oracle_series(O, p, wall, row0, K, n_steps, init=None, stop=None):
    """Diagnostics samples of the FP64 oracle every K steps from step 0 to
    n_steps (or until stop(series) is true): the per-sample segment records
    of the rows y >= row0.  init(o) sets the initial state (default: ink in
    the rows below row0 with a flat meniscus)."""
    o = O.OracleSim(p, wall)
    if init is None:
        import workloads as W
        o.init_distance(W.meniscus_distance(p["nx"], p["ny"], row0))
    else:
        init(o)
    series = []
    for k in range(0, n_steps + 1, K):
        if o.t < k:
            o.step(k - o.t)
        d = o.diag(row0)
        seg = O.segments(d["row_count"], d["row_uy"], row0, 4 * p["width"] ** 2, O.band_rows(p["width"]))
        seg["step"] = k
        seg["nan_count"] = d["nan_count"]
        series.append(seg)
        if stop is not None and stop(series):
            break
    o.close()
    return series

