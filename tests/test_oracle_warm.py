"""Pins of the oracle's warm (adiabatic) fluid, CPU only: the Bohm-Gross
dispersion of electron plasma waves, energy conservation with the thermal
energy counted, and the energy bookkeeping of both conversions."""
import math

import numpy as np
import pytest

from paper_2510_11174_amd import configs

GA = 5.0 / 3.0


def _warm_cfg(nx, mode, u_th=0.0):
    cfg = configs.plain_hybrid(nx, 2, 2, mode=mode)
    cfg["grid"]["bc_x"] = "periodic"
    cfg["laser"]["enabled"] = False
    cfg["species"][0]["u_th"] = u_th
    cfg["species"][0]["gamma_ad"] = GA
    return cfg


def _wave(oracle_mod, T, steps=2000, amp=1e-4):
    """Standing electron plasma wave u_x = amp sin(k x) on a uniform warm
    fluid of temperature T; returns (dt, k dx, E_x time series at the node of
    largest field, energies (first, last))."""
    nx = 32
    cfg = _warm_cfg(nx, "all_fluid")
    o = oracle_mod.Oracle(cfg)
    o.step(1)   # absorbs the initial particles into the node fluid
    n, u = o.get_fluid(0)
    n0 = 0.01
    n[..., :nx] = n0
    d = cfg["grid"]["dx"]
    k = 2 * math.pi / (nx * d)
    x = np.arange(nx + 1) * d
    u[...] = 0
    u[..., :nx, 0] = amp * np.sin(k * x[:nx])
    o.set_fluid(0, n, u)
    o.set_pressure(0, np.where(n > 0, n0 * T, 0.0))
    for c in ("ex", "ey", "ez", "bx", "by", "bz", "jx", "jy", "jz"):
        o.set_field(c, np.zeros(o.shape))

    def energy():
        dg = o.diagnostics()
        return dg["u_e"] + dg["u_b"] + sum(dg["fluid_kin"]) + sum(dg["fluid_th"]) + dg["conv_loss"]

    e0 = energy()
    ex = []
    for _ in range(steps):
        o.step(1)
        ex.append(o.get_field("ex")[0, 0, nx // 4])
    return cfg["grid"]["dt"], k * d, np.array(ex), (e0, energy())


def _frequency(dt, ex, w0):
    """Frequency of a single sinusoid by least squares around w0."""
    t = dt * np.arange(1, len(ex) + 1)
    best = None
    for w in np.linspace(0.9 * w0, 1.1 * w0, 2001):
        A = np.stack([np.sin(w * t), np.cos(w * t)], 1)
        coef, *_ = np.linalg.lstsq(A, ex, rcond=None)
        r = np.linalg.norm(A @ coef - ex)
        if best is None or r < best[0]:
            best = (r, w)
    return best[1]


@pytest.mark.parametrize("T", [0.0, 0.006])
def test_bohm_gross_dispersion(oracle_mod, T):
    # the scheme's Bohm-Gross relation: w^2 = w_p^2 cos^2(k dx / 2) + gamma T
    # k_eff^2 / m, k_eff = sin(k dx) / dx.  The field reaches the node as the
    # mean of its two faces and the current is the face mean of the node
    # velocities (a factor cos(k dx / 2) each); the pressure gradient and the
    # flux divergence are both central over two cells (k_eff)
    dt, kdx, ex, _ = _wave(oracle_mod, T)
    d = 0.2
    wp2 = 0.01
    keff = math.sin(kdx) / d
    w_th = math.sqrt(wp2 * math.cos(kdx / 2) ** 2 + GA * T * keff ** 2)
    w_num = 2 / dt * math.asin(w_th * dt / 2)
    w = _frequency(dt, ex, w_num)
    print("T %.3g: w %.6f predicted %.6f (w_p %.4f)" % (T, w, w_num, math.sqrt(wp2)))
    assert abs(w - w_num) < 2e-4 * w_num
    if T > 0:
        assert w > 1.3 * math.sqrt(wp2)


def test_energy_with_heat_conserved(oracle_mod):
    _, _, ex, (e0, e1) = _wave(oracle_mod, 0.006, steps=400, amp=1e-3)
    print("energy %.10e -> %.10e" % (e0, e1))
    assert abs(e1 - e0) < 2e-4 * e0


def test_absorption_turns_spread_into_heat(oracle_mod):
    # every node fluid from the start: the first step absorbs particles with a
    # thermal spread (pushed through zero fields first); their kinetic energy
    # equals the fluid's kinetic plus thermal energy, nothing goes to the
    # ledger (the fields gain the energy of the virtual moves' current, as in
    # the cold model)
    cfg = _warm_cfg(8, "all_fluid", u_th=0.05)
    o = oracle_mod.Oracle(cfg)
    d0 = o.diagnostics()
    ke0 = sum(d0["kin"])
    o.set_field("ex", np.zeros(o.shape))
    o.step(1)
    d1 = o.diagnostics()
    print("particle KE %.12e; fluid kin %.3e, heat %.12e, fields %.3e, ledger %.3e" % (
        ke0, sum(d1["fluid_kin"]), sum(d1["fluid_th"]), d1["u_e"] + d1["u_b"], d1["conv_loss"]))
    assert d1["conv_loss"] == 0.0
    assert abs(sum(d1["fluid_kin"]) + sum(d1["fluid_th"]) - ke0) < 1e-12 * ke0
    # temperature: p / n close to m u_th^2 (4 particles per cell, so sampled)
    n, _ = o.get_fluid(0)
    p = o.get_pressure(0)
    T = p[n > 0].sum() / n[n > 0].sum()
    assert 0.6 * 0.05 ** 2 < T < 1.4 * 0.05 ** 2


def test_spawn_samples_the_temperature(oracle_mod):
    # a warm fluid node switched to kinetic becomes particles with the thermal
    # spread; fluid kinetic plus thermal energy = particle energy + ledger
    cfg = _warm_cfg(8, "all_fluid", u_th=0.0)
    cfg["species"][0]["ppc"] = 64
    o = oracle_mod.Oracle(cfg)
    o.step(1)
    n, u = o.get_fluid(0)
    u[...] = 0; u[..., 0] = np.where(n > 0, 0.02, 0.0)
    o.set_fluid(0, n, u)
    T = 0.004
    o.set_pressure(0, np.where(n > 0, n * T, 0.0))
    for c in ("ex", "ey", "ez", "bx", "by", "bz", "jx", "jy", "jz"):
        o.set_field(c, np.zeros(o.shape))
    d0 = o.diagnostics()
    e_fluid = sum(d0["fluid_kin"]) + sum(d0["fluid_th"])
    o.set_switch_mode("all_pic")
    o.set_switch(np.ones(o.shape, np.uint8))
    o.step(1)
    d1 = o.diagnostics()
    pr = o.get_particles(0)
    ue = pr["u"]
    print("fluid energy %.8e; particles %.8e + ledger %.3e; spread %.4f (sqrt T %.4f)" % (
        e_fluid, sum(d1["kin"]), d1["conv_loss"], ue[:, 1].std(), math.sqrt(T)))
    assert sum(d1["fluid_mass"]) == 0.0
    assert abs(ue[:, 1].std() - math.sqrt(T)) < 0.05 * math.sqrt(T)
    assert abs(ue[:, 0].mean() - 0.02) < 0.05 * math.sqrt(T)
    assert abs(sum(d1["kin"]) + d1["conv_loss"] + d1["u_e"] + d1["u_b"] - e_fluid) < 1e-3 * e_fluid


def test_absorption_into_negative_density(oracle_mod):
    # a node whose fluid density went negative (a donor-cell step can drain
    # more than a node holds) absorbs particles: where the merged mass stays
    # negative the node keeps no entropy and the heat goes to the ledger, so
    # particle kinetic energy = fluid kinetic + thermal energy + ledger still
    cfg = _warm_cfg(8, "all_fluid", u_th=0.05)
    o = oracle_mod.Oracle(cfg)
    n, u = o.get_fluid(0)
    n[:] = 0.0
    n[0, 0, 2] = -1.0          # far below what its particles bring (0.01)
    n[1, 1, 5] = -0.0005       # a small deficit: merged mass and pressure stay positive
    n[0, 1, 6] = -0.004        # merged mass positive; the negative mass amplifies the merged
                               # flow, whose energy may or may not exceed what the particles bring
    u[:] = 0.0
    o.set_fluid(0, n, u)
    o.set_pressure(0, np.zeros_like(n))
    o.set_field("ex", np.zeros(o.shape))
    ke0 = sum(o.diagnostics()["kin"])
    o.step(1)
    d = o.diagnostics()
    n1, u1 = o.get_fluid(0)
    p1 = o.get_pressure(0)
    print("n at the drained nodes %.4f %.4f %.4f; p %.3e %.3e %.3e; ledger %.6e" % (
        n1[0, 0, 2], n1[1, 1, 5], n1[0, 1, 6], p1[0, 0, 2], p1[1, 1, 5], p1[0, 1, 6], d["conv_loss"]))
    assert np.isfinite(p1).all() and np.isfinite(u1).all()
    assert n1[0, 0, 2] < 0 and p1[0, 0, 2] == 0.0
    assert n1[1, 1, 5] > 0 and p1[1, 1, 5] > 0
    assert n1[0, 1, 6] > 0 and p1[0, 1, 6] >= 0.0
    assert d["conv_loss"] > 0
    total = sum(d["fluid_kin"]) + sum(d["fluid_th"]) + d["conv_loss"]
    assert abs(total - ke0) < 1e-12 * ke0
