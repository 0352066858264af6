"""Pins of the oracle's droplet diagnostics: the row-segment reading of
breakup against 8-connected component labelling on synthetic ink fields, the
C reduction against a direct count, and the breakup summary on a hand-made
sample series."""
import numpy as np
import pytest
from scipy import ndimage

import workloads as W


def _ink_field(ny, nx, row0, blobs, column_top):
    """phi > 0 inside the listed discs and in an ink column from row0 up to
    column_top (exclusive) around the axis."""
    y, x = np.mgrid[0:ny, 0:nx].astype(float)
    phi = -np.ones((ny, nx))
    xc = nx / 2
    if column_top > row0:
        phi[(y >= row0) & (y < column_top) & (np.abs(x - xc) < 5)] = 1.0
    for (cy, r) in blobs:
        phi[(x - xc) ** 2 + (y - cy) ** 2 < r * r] = 1.0
    return phi


@pytest.mark.parametrize("seed", range(12))
def test_row_segments_match_component_labelling(seed):
    from oracle.oracle import segments
    rng = np.random.default_rng(seed)
    ny, nx, row0 = 200, 48, 20
    column_top = int(rng.integers(row0, row0 + 40))
    blobs = []
    y = column_top + rng.integers(2, 10)
    while True:
        r = float(rng.uniform(1.5, 9.0))
        cy = y + r
        if cy + r >= ny - 1:
            break
        blobs.append((cy, r))
        y = int(cy + r + rng.integers(2, 12))
    phi = _ink_field(ny, nx, row0, blobs, column_top)
    ink = phi > 0
    ink[:row0] = False
    a_min = 20
    lab, nlab = ndimage.label(ink, structure=np.ones((3, 3)))
    detached = 0
    sizes = []
    for k in range(1, nlab + 1):
        ys = np.where((lab == k).any(axis=1))[0]
        area = int((lab == k).sum())
        if ys.min() > row0 and area >= a_min:
            detached += 1
            sizes.append(area)
    row_count = ink.sum(axis=1)
    row_uy = row_count * 0.01
    seg = segments(row_count, row_uy, row0, a_min)
    assert seg["n_detached"] == detached
    if detached:
        assert seg["largest_count"] == max(sizes)
        assert seg["largest_uy"] == pytest.approx(0.01 * max(sizes))


def test_segment_head_tail_and_length():
    """A detached drop of constant width 12 over rows 40..69 whose ink moves
    at u_y = 0.001 y: the head (top 3 rows) and tail (bottom 3 rows) mean
    velocities are 0.001 times the mean row of those bands, 0.068 and 0.041."""
    from oracle.oracle import segments, band_rows
    row_count = np.zeros(100, dtype=np.int64)
    row_count[:10] = 5                       # attached: the run that holds row0 = 0
    row_count[40:70] = 12
    row_uy = row_count * 0.001 * np.arange(100)
    band = band_rows(3.0)
    seg = segments(row_count, row_uy, 0, 20, band)
    assert band == 3 and seg["n_detached"] == 1
    assert (seg["largest_bottom"], seg["largest_top"]) == (40, 69)
    assert seg["head_uy"] == pytest.approx(0.068, rel=1e-12)
    assert seg["tail_uy"] == pytest.approx(0.041, rel=1e-12)
    assert band_rows(4.0) == 4 and band_rows(2.5) == 3 and band_rows(0.5) == 1


def test_diag_reduction_matches_direct_count(oracle_mod):
    cfg = W.config_nozzle_small()
    s = oracle_mod.OracleSim(cfg["params"], cfg["wall"])
    s.init_distance(cfg["distance"])
    s.step(150)
    fl = s.fields()
    dg = s.diag(cfg["row0"])
    fluid = cfg["wall"] == 0
    ink = (fl["phi"] > 0) & fluid
    exp = ink.sum(axis=1)
    exp[: cfg["row0"]] = 0
    assert np.array_equal(dg["row_count"], exp)
    expu = np.where(ink, fl["uy"], 0.0).sum(axis=1)
    expu[: cfg["row0"]] = 0
    assert np.allclose(dg["row_uy"], expu, rtol=1e-12, atol=1e-18)
    assert dg["mass_n"] == pytest.approx(fl["n"][fluid].sum(), rel=1e-12)
    assert dg["mass_phi"] == pytest.approx(fl["phi"][fluid].sum(), rel=1e-12)
    assert dg["max_u"] == pytest.approx(np.hypot(fl["ux"], fl["uy"])[fluid].max(), rel=1e-14)
    assert dg["nan_count"] == 0


def test_breakup_summary_on_synthetic_series():
    from oracle.oracle import breakup_summary
    samples = []
    for step in range(0, 9000, 50):
        if step < 3000:
            rec = dict(step=step, n_detached=0, largest_count=0, largest_uy=0.0, largest_top=-1)
        else:
            n_det = 2 if step >= 5000 else 1
            rec = dict(step=step, n_detached=n_det, largest_count=400,
                       largest_uy=400 * (0.01 + 1e-6 * step), largest_top=100, largest_bottom=60)
        samples.append(rec)
    out = breakup_summary(samples, ny=1000, width=4.0)
    assert out["breakup_step"] == 3000
    vs = [0.01 + 1e-6 * s for s in range(4000, 6001, 50)]
    assert out["v_drop"] == pytest.approx(np.mean(vs), rel=1e-12)
    assert out["vol_drop"] == 400 and out["satellite"] == 1 and out["drop_len"] == 41
    none = breakup_summary(samples[:10], ny=1000, width=4.0)
    assert none["breakup_step"] == -1 and np.isnan(none["v_drop"])
