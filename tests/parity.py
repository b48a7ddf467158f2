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
  diagnostics every hk_diag field: step exactly; time, and kinetic and
             fallback fractions, absolutely; energies (fields, particles,
             fluids, ledgers) on the scale of the total energy; particle
             counts exactly (FP32 Monte Carlo flips aside, counted by the
             event tests); fluid mass and total charge relatively; the Gauss
             residuals relatively, plus a stated round-off floor
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



def cell_errors(gpu, ora, comps=FIELDS, bar=1e-5):
    """Per component: (max per-cell error, its 99.9th percentile, max |a - b| /
    max|b|, fraction of cells within `bar`) with the per-cell metric above."""
    out = {}
    for c in comps:
        a = np.asarray(gpu.get_field(c), float); b = np.asarray(ora.get_field(c), float)
        scale = np.abs(b).max()
        if scale == 0.0:
            m = float(np.abs(a).max())
            out[c] = (m, m, m, float((np.abs(a) <= bar).mean()))
            continue
        e = np.abs(a - b) / (np.abs(b) + 1e-6 * scale)
        out[c] = (float(e.max()), float(np.percentile(e, 99.9)), float(np.abs(a - b).max() / scale),
                  float((e <= bar).mean()))
    return out


def assert_cells(errs, bar, p999_bar=None):
    """Every cell's error within `bar` of the component's scale, and 99.9% of
    the cells within p999_bar (default `bar`) in the per-cell metric.  In
    FP32 a cell whose value cancels to a small part of the component's scale
    carries a few units of rounding of that scale: its relative error can
    exceed the bar while |a - b| stays near 1e-7 max|b|."""
    p999_bar = bar if p999_bar is None else p999_bar
    for c, (mx, p999, absr, frac) in errs.items():
        assert absr <= bar, (c, "max |a - b| / max|b|", absr, bar)
        assert p999 <= p999_bar, (c, "99.9th percentile", p999, p999_bar)

ENERGY_KEYS = ("kin", "fluid_kin", "fluid_th")
LEDGER_KEYS = ("u_e", "u_b", "conv_loss", "ion_energy", "photon_energy")


def diag_errors(dg: dict, do: dict, nsp: int):
    """Per hk_diag field, the error in the metric above (counts: absolute
    difference; the rest: relative to their scale)."""
    etot = sum(abs(do[k]) for k in LEDGER_KEYS) + sum(abs(v) for k in ENERGY_KEYS for v in do[k][:nsp])
    etot = max(etot, 1e-300)
    out = {"step": abs(dg["step"] - do["step"]), "t": abs(dg["t"] - do["t"]) / max(abs(do["t"]), 1.0)}
    for k in LEDGER_KEYS:
        out[k] = abs(dg[k] - do[k]) / etot
    for k in ENERGY_KEYS:
        out[k] = max(abs(a - b) for a, b in zip(dg[k][:nsp], do[k][:nsp])) / etot
    out["count"] = max(abs(a - b) for a, b in zip(dg["count"][:nsp], do["count"][:nsp]))
    fm = max(sum(abs(v) for v in do["fluid_mass"][:nsp]), 1e-300)
    out["fluid_mass"] = max(abs(a - b) for a, b in zip(dg["fluid_mass"][:nsp], do["fluid_mass"][:nsp])) / fm
    out["charge_total"] = abs(dg["charge_total"] - do["charge_total"]) / max(abs(do["charge_total"]), 1e-300)
    for k in ("kinetic_fraction", "fallback_fraction"):
        out[k] = abs(dg[k] - do[k])
    return out


def assert_diag(dg: dict, do: dict, nsp: int, tol: float, gauss_bound: float, frac_tol: float = 0.0,
                count_tol: float = 0.0):
    e = diag_errors(dg, do, nsp)
    print("diagnostics errors:", {k: "%.1e" % v for k, v in e.items()})
    assert e["step"] == 0 and e["t"] <= 1e-12
    for k in LEDGER_KEYS + ENERGY_KEYS + ("fluid_mass", "charge_total"):
        assert e[k] <= tol, (k, e[k], tol)
    assert e["count"] <= count_tol, ("count", e["count"])
    for k in ("kinetic_fraction", "fallback_fraction"):
        assert e[k] <= frac_tol, (k, e[k])
    for k in ("gauss_max", "gauss_l2"):
        assert abs(dg[k] - do[k]) <= tol * abs(do[k]) + gauss_bound, (k, dg[k], do[k], gauss_bound)
