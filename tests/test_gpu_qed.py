"""GPU parity of the QED Monte Carlo (photon emission, pair creation, photon
transport) against the FP64 oracle, event by event through the shared Philox
counters and child ids."""
import math

import numpy as np
import pytest

from paper_2510_11174_amd import configs
from tests.parity import field_errors, rel_l2

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def hk():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2510_11174_amd import hk as hkmod
    return hkmod


def _box(photons_convert):
    """Periodic 4^3 box (dx 0.2), laser off; species electron, positron, photon."""
    cfg = configs.qed_hybrid(4, 4, 4, mode="all_pic", dx=0.2, ppc=1)
    cfg["grid"]["bc_x"] = "periodic"
    cfg["laser"]["enabled"] = False
    sp = cfg["species"]
    cfg["species"] = [dict(sp[0], profile="none", fluid=False, qed=not photons_convert),
                      dict(sp[2], profile="none", qed=not photons_convert),
                      dict(sp[3])]
    return cfg


def _uniform_b(sim, B0):
    for c in ("ex", "ey", "ez", "by", "bz"):
        sim.set_field(c, np.zeros(sim.shape))
    sim.set_field("bx", np.full(sim.shape, B0))


def _by_id(p):
    o = np.argsort(p["id"], kind="stable")
    return {k: v[o] for k, v in p.items()}


def _compare_sets(pg, po, what):
    """Common ids, and the ids found on one side only."""
    ig = set(pg["id"].tolist()); io = set(po["id"].tolist())
    only = len(ig ^ io)
    common = np.array(sorted(ig & io), dtype=np.uint64)
    a = _by_id(pg); b = _by_id(po)
    sa = np.isin(a["id"], common); sb = np.isin(b["id"], common)
    print("%s: gpu %d oracle %d common %d one-sided %d" % (what, len(ig), len(io), len(common), only))
    return {k: v[sa] for k, v in a.items()}, {k: v[sb] for k, v in b.items()}, only


def _setup(hk, oracle_mod, prec, photons_convert, B0, n, u_mag, seed):
    cfg = _box(photons_convert)
    print("case: qed box", "pairs" if photons_convert else "emission", prec, flush=True)
    g = hk.Sim(cfg, precision=prec); o = oracle_mod.Oracle(cfg)
    for s in (g, o):
        _uniform_b(s, B0)
    rng = np.random.default_rng(seed)
    x = rng.uniform(0, 0.8, (n, 3))
    u = np.zeros((n, 3)); u[:, 2] = u_mag
    w = np.full(n, 1e-9)
    ids = np.arange(n, dtype=np.uint64) * 7919 + 11
    sp = 2 if photons_convert else 0
    g.set_particles(sp, x, u, w, ids=ids)
    o.set_particles(sp, x, u, w, ids=ids)
    return cfg, g, o


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_emission_events(hk, oracle_mod, prec):
    # gamma = 1000 electrons across a uniform B (chi = 1): which electrons emit,
    # when, and which photons they make, compared id by id over 4 steps
    a_s = oracle_mod.schwinger_field(0.8)
    gamma0 = 1000.0
    B0 = 1.0 * a_s / math.sqrt(gamma0 ** 2 - 1)
    n = 1500
    cfg, g, o = _setup(hk, oracle_mod, prec, False, B0, n, math.sqrt(gamma0 ** 2 - 1), 5)
    # the optical depths both sides drew for the set particles
    tg, to = _by_id(g.get_particles(0))["tau"], _by_id(o.get_particles(0))["tau"]
    np.testing.assert_allclose(tg, to, rtol=1e-15, atol=0)
    # step by step: an electron whose momentum departs from the oracle's in a
    # step emitted on one side only, which FP32 may do only when its optical
    # depth and that step's decrement W dt agree to rounding (|tau - W dt| <=
    # 1e-5 W dt, from the oracle's view of the step); it is then left out
    tol = 1e-5 if prec == "f32" else 1e-12
    flipped, near = set(), []
    for step in range(4):
        probe = o.qed_probe(0)
        g.step(1); o.step(1)
        eg, eo, e_only = _compare_sets(g.get_particles(0), o.get_particles(0), "electrons")
        assert e_only == 0
        ue = np.linalg.norm(eg["u"] - eo["u"], axis=1) / np.linalg.norm(eo["u"], axis=1)
        for q in np.nonzero(ue > 1e-3)[0]:
            pid = int(eg["id"][q])
            if pid in flipped:
                continue
            flipped.add(pid)
            assert prec == "f32", ("FP64 emission differs", step, pid)
            tau, dtau = probe[pid]
            assert abs(tau - dtau) <= 1e-5 * dtau, ("emission decided differently far from its threshold",
                                                    step, pid, tau, dtau)
            near.append(abs(tau - dtau) / dtau)
    eg, eo, e_only = _compare_sets(g.get_particles(0), o.get_particles(0), "electrons")
    pg, po, p_only = _compare_sets(g.get_particles(2), o.get_particles(2), "photons")
    assert len(po["id"]) > 0.3 * n
    keep = ~np.isin(eg["id"], np.array(sorted(flipped), dtype=np.uint64))
    ue = np.linalg.norm(eg["u"] - eo["u"], axis=1) / np.linalg.norm(eo["u"], axis=1)
    print("electron momentum rel err (no flip) %.2e; flips %d (max |tau - W dt| / W dt %.1e); photons "
          "one-sided %d" % (ue[keep].max(), len(flipped), max(near) if near else 0.0, p_only))
    assert ue[keep].max() <= 10 * tol
    assert p_only <= len(flipped)
    du = np.linalg.norm(pg["u"] - po["u"], axis=1) / np.linalg.norm(po["u"], axis=1)
    assert du.max() <= 10 * tol
    # photon optical depths fall with chi from FP32 fields after birth
    np.testing.assert_allclose(pg["tau"], po["tau"], rtol=1e-6 if prec == "f32" else 1e-12)
    dg, do = g.diagnostics(), o.diagnostics()
    assert dg["photon_energy"] == pytest.approx(do["photon_energy"], rel=1e-2 if prec == "f32" else 1e-10)


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_pair_events(hk, oracle_mod, prec):
    # eps = 5000 photons across a uniform B (chi = 20): conversions id by id,
    # pair momenta, and the energy books of both sides
    a_s = oracle_mod.schwinger_field(0.8)
    eps, chi0 = 5000.0, 20.0
    B0 = chi0 * a_s / eps
    n = 1500
    cfg, g, o = _setup(hk, oracle_mod, prec, True, B0, n, eps, 6)
    # step by step: a photon present on one side only after a step converted
    # on the other, which FP32 may do only when its optical depth and the
    # step's decrement agree to rounding (|tau - W dt| <= 1e-5 W dt)
    tol = 1e-5 if prec == "f32" else 1e-12
    flips, near = 0, []
    for step in range(4):
        probe = o.qed_probe(2)
        gone_before = set(probe) - set(g.get_particles(2)["id"].tolist())
        g.step(1); o.step(1)
        ig = set(g.get_particles(2)["id"].tolist()); io = set(o.get_particles(2)["id"].tolist())
        for pid in sorted((ig ^ io) & set(probe)):
            if pid in gone_before:
                continue
            flips += 1
            assert prec == "f32", ("FP64 pair creation differs", step, pid)
            tau, dtau = probe[pid]
            assert abs(tau - dtau) <= 1e-5 * dtau, ("pair creation decided differently far from its threshold",
                                                    step, pid, tau, dtau)
            near.append(abs(tau - dtau) / dtau)
    _, _, ph_only = _compare_sets(g.get_particles(2), o.get_particles(2), "photons")
    eg, eo, e_only = _compare_sets(g.get_particles(0), o.get_particles(0), "electrons")
    qg, qo, q_only = _compare_sets(g.get_particles(1), o.get_particles(1), "positrons")
    print("pair flips %d (max |tau - W dt| / W dt %.1e)" % (flips, max(near) if near else 0.0))
    assert len(eo["id"]) > 0.2 * n
    assert ph_only == flips and e_only == ph_only and q_only == ph_only
    # slow pair members gyrate by up to ~100 rad per step in this field, which
    # amplifies the rounding of the rotation: 1e-10 in FP64
    for a, b in ((eg, eo), (qg, qo)):
        du = np.linalg.norm(a["u"] - b["u"], axis=1) / np.linalg.norm(b["u"], axis=1)
        assert du.max() <= (1e-4 if prec == "f32" else 1e-10)
    dg, do = g.diagnostics(), o.diagnostics()
    eg_tot = sum(dg["kin"]) + dg["photon_energy"]
    eo_tot = sum(do["kin"]) + do["photon_energy"]
    assert eg_tot == pytest.approx(eo_tot, rel=1e-5 if prec == "f32" else 1e-11)
    assert dg["gauss_max"] < (1e-5 if prec == "f32" else 1e-12)


def _foil(mode, nx=32):
    # a thin dense foil under a circularly polarized a0 = 200 pulse, short
    # enough that QED sets in within the test's steps
    cfg = configs.qed_hybrid(nx, 8, 8, mode=mode, ppc=2)
    for sp in cfg["species"]:
        if sp.get("profile") == "foil":
            sp["x0"] = 0.6
            sp["length"] = 0.4
    cfg["laser"]["duration"] = 2.0
    cfg["laser"]["t_center"] = 3.0
    return cfg


@pytest.mark.parametrize("prec", ["f32", "f64"])
@pytest.mark.parametrize("mode", ["all_pic", "threshold"])
def test_qed_foil(hk, oracle_mod, prec, mode):
    cfg = _foil(mode)
    print("case:", cfg["name"], mode, prec, flush=True)
    g = hk.Sim(cfg, precision=prec); o = oracle_mod.Oracle(cfg)
    steps = 160
    g.step(steps); o.step(steps)
    counts = [(g.count(s), o.count(s)) for s in range(4)]
    dg, do = g.diagnostics(), o.diagnostics()
    errs = field_errors(g, o, ["ex", "ey", "ez", "bx", "by", "bz"])
    print("counts", counts, "photon ledger %.3e / %.3e" % (dg["photon_energy"], do["photon_energy"]),
          {k: "%.1e" % v for k, v in errs.items()})
    assert counts[3][1] > 0 or do["photon_energy"] > 0, "no QED activity in the oracle"
    if prec == "f64":
        assert all(a == b for a, b in counts)
        assert max(errs.values()) <= 1e-9
        assert dg["photon_energy"] == pytest.approx(do["photon_energy"], rel=1e-9)
    else:
        for a, b in counts[2:]:
            assert abs(a - b) <= max(3, 0.05 * b)
        vec = {f: rel_l2(np.stack([g.get_field(f + c) for c in "xyz"]),
                         np.stack([o.get_field(f + c) for c in "xyz"])) for f in "eb"}
        assert max(vec.values()) <= 1e-3
