"""Comparison helpers shared by the GPU parity tests (no method arithmetic).

Metrics (stated once, used everywhere):
  particles  position error |dx| / dx in cell units per axis, momentum error
             |du| / max(|u|, 1e-6); matched by id
  fields     relative L2 per component, ||a - b|| / ||b|| (components whose
             reference norm is below 1e-30 compare by max-abs instead)
  per cell   |a - b| / (|b| + 1e-6 max|b|) per cell and component; a cell
             whose value cancels to a small fraction of the component's
             scale carries the rounding of that scale, so the bar holds for
             99.9% of the cells and every cell's error stays within the bar
             times the component's scale (|a - b| <= bar max|b|)
"""
import numpy as np


def match_particles(a: dict, b: dict):
    ia = np.argsort(a["id"], kind="stable"); ib = np.argsort(b["id"], kind="stable")
    assert len(ia) == len(ib), "particle counts differ: %d vs %d" % (len(ia), len(ib))
    assert np.array_equal(a["id"][ia], b["id"][ib]), "particle ids differ"
    return ia, ib


def particle_errors(gpu: dict, ora: dict, dx, box):
    ig, io = match_particles(gpu, ora)
    xg, xo = gpu["x"][ig], ora["x"][io]
    d = np.abs(xg - xo)
    box = np.asarray(box, float)
    d = np.minimum(d, box - d)           # periodic wrap
    pos = (d / np.asarray(dx, float)).max() if len(d) else 0.0
    ug, uo = gpu["u"][ig], ora["u"][io]
    mom = (np.linalg.norm(ug - uo, axis=1) / np.maximum(np.linalg.norm(uo, axis=1), 1e-6)).max() if len(ug) else 0.0
    w = (np.abs(gpu["w"][ig] - ora["w"][io]) / np.abs(ora["w"][io])).max() if len(ug) else 0.0
    return pos, mom, w


def rel_l2(a, b):
    a = np.asarray(a, float); b = np.asarray(b, float)
    nb = np.linalg.norm(b)
    if nb < 1e-30:
        return float(np.abs(a - b).max())
    return float(np.linalg.norm(a - b) / nb)


FIELDS = ["ex", "ey", "ez", "bx", "by", "bz", "jx", "jy", "jz"]


def field_errors(gpu, ora, comps=FIELDS):
    return {c: rel_l2(gpu.get_field(c), ora.get_field(c)) for c in comps}



def cell_errors(gpu, ora, comps=FIELDS):
    """Per component: (max per-cell error, its 99.9th percentile, max |a - b| /
    max|b|) with the per-cell metric above."""
    out = {}
    for c in comps:
        a = np.asarray(gpu.get_field(c), float); b = np.asarray(ora.get_field(c), float)
        scale = np.abs(b).max()
        if scale == 0.0:
            out[c] = (float(np.abs(a).max()), float(np.abs(a).max()), float(np.abs(a).max()))
            continue
        e = np.abs(a - b) / (np.abs(b) + 1e-6 * scale)
        out[c] = (float(e.max()), float(np.percentile(e, 99.9)), float(np.abs(a - b).max() / scale))
    return out


def assert_cells(errs, bar):
    """99.9% of the cells within `bar`, every cell's error within `bar` of
    the component's scale (see the metric's note)."""
    for c, (mx, p999, absr) in errs.items():
        assert p999 <= bar, (c, "99.9th percentile", p999, bar)
        assert absr <= bar, (c, "max |a - b| / max|b|", absr, bar)
