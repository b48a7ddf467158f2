"""Workload presets: plain parameter dictionaries, no arithmetic of the method.

Units are normalized laser units (c = omega0 = m_e = e = 1; lambda = 2 pi).
The same dictionary drives the HIP library and the test oracle.  The time step
is the Courant number times the 3D vacuum limit of the Yee scheme.

The paper runs a 16^3 grid in SI units (Methodology, grid and time-step
paragraphs); the workloads below are the synthetic stand-ins with the shapes
of the method's use cases: an underdense plasma driven by a moderate laser,
an ionizing gas jet, and a relativistic foil with QED.
"""
from __future__ import annotations

import copy
import math

TWO_PI = 2.0 * math.pi
HE_IP_EV = [24.587387936, 54.4177650]     # He I, He II ionization potentials (NIST ASD)
SEED_BASE = 0x2510111740


def courant_dt(dx, dy, dz, cfl):
    return cfl / math.sqrt(1.0 / dx ** 2 + 1.0 / dy ** 2 + 1.0 / dz ** 2)


def _grid(nx, ny, nz, d, cfl=0.95, bc_x="open"):
    return {"nx": nx, "ny": ny, "nz": nz, "dx": d, "dy": d, "dz": d, "cfl": cfl,
            "dt": courant_dt(d, d, d, cfl), "bc_x": bc_x}


def _run(seed, mode="threshold", **kw):
    # thr_sigma_u = 0.02: at 0.05 the ionizing-helium run converts warm electrons
    # (spread 0.02-0.05) to cold fluid and its fields drift far from all-PIC
    r = {"seed": seed, "switch_mode": mode, "switch_every": 1, "dilation": 1, "hysteresis": 2,
         "enable_ionization": False, "enable_qed": False, "thr_a": 0.5, "thr_grad": 0.2,
         "thr_sigma_u": 0.02, "thr_ion": 1e-6, "thr_chi": 1e-3, "n_floor": 1e-10,
         "spawn_frac": 0.5}
    r.update(kw)
    return r


def plain_hybrid(nx=32, ny=16, nz=16, mode="threshold", seed=None):
    """Underdense plasma, 0.01 n_c electrons (4 ppc, u_th 1e-3) on an immobile
    ion background, linear Gaussian pulse a0 = 1, waist 4 lambda, duration 10,
    entering at x = 0; dx = 0.2, CFL 0.95, periodic y/z, open x."""
    return {
        "name": "plain_hybrid_%dx%dx%d" % (nx, ny, nz),
        "grid": _grid(nx, ny, nz, 0.2),
        "species": [{"kind": "electron", "charge": -1.0, "mass": 1.0, "ppc": 4,
                     "profile": "uniform", "n0": 0.01, "u_th": 1e-3, "mobile": True,
                     "fluid": True}],
        "laser": {"enabled": True, "polarization": "linear", "a0": 1.0, "waist": 4 * TWO_PI,
                  "duration": 10.0, "t_center": 20.0, "i_antenna": 2, "lambda_um": 0.8},
        "run": _run(SEED_BASE + 1 if seed is None else seed, mode),
        "steps": 200,
    }


def ionization_hybrid(nx=128, ny=64, nz=64, mode="threshold", seed=None, dx=0.1, ppc=8):
    """Neutral helium, 0.1 n_c atoms with a linear up-ramp over 10 lambda from
    x = 0, 8 particles per cell, immobile atoms; a0 = 10 linear pulse, waist
    6 lambda, duration 15; ADK/multiphoton ionization through He II."""
    return {
        "name": "ionization_hybrid_%dx%dx%d" % (nx, ny, nz),
        "grid": _grid(nx, ny, nz, dx),
        "species": [
            {"kind": "electron", "charge": -1.0, "mass": 1.0, "ppc": ppc, "profile": "none",
             "n0": 0.2, "u_th": 0.0, "mobile": True, "fluid": True},
            {"kind": "ion", "charge": 0.0, "mass": 4.0 * 1836.15267343, "ppc": ppc,
             "profile": "ramp", "n0": 0.1, "x0": 0.0, "length": 10 * TWO_PI, "u_th": 0.0,
             "mobile": False, "fluid": False, "ionizable": True, "z_max": 2, "target": 0,
             "ip_ev": HE_IP_EV},
        ],
        "laser": {"enabled": True, "polarization": "linear", "a0": 10.0, "waist": 6 * TWO_PI,
                  "duration": 15.0, "t_center": 30.0, "i_antenna": 2, "lambda_um": 0.8},
        "run": _run(SEED_BASE + 2 if seed is None else seed, mode, enable_ionization=True),
        "steps": 2000,
    }


def qed_hybrid(nx=256, ny=128, nz=128, mode="threshold", seed=None, dx=0.05, ppc=16):
    """Pre-ionized hydrogen foil, 10 n_c, 1 lambda thick from x = 3.2, 16
    particles per cell per species, mobile protons (mass 1836); circular pulse
    a0 = 200, waist 3 lambda, duration 20; photon emission and pair creation."""
    foil = {"profile": "foil", "n0": 10.0, "x0": 3.2, "length": TWO_PI, "u_th": 1e-3}
    return {
        "name": "qed_hybrid_%dx%dx%d" % (nx, ny, nz),
        "grid": _grid(nx, ny, nz, dx),
        "species": [
            dict(kind="electron", charge=-1.0, mass=1.0, ppc=ppc, mobile=True, fluid=True,
                 qed=True, **foil),
            dict(kind="ion", charge=1.0, mass=1836.15267343, ppc=ppc, mobile=True, fluid=True,
                 **foil),
            dict(kind="positron", charge=1.0, mass=1.0, ppc=ppc, profile="none", n0=10.0,
                 mobile=True, fluid=False, qed=True),
            dict(kind="photon", charge=0.0, mass=0.0, ppc=0, profile="none", mobile=True,
                 fluid=False, qed=True),
        ],
        "laser": {"enabled": True, "polarization": "circular", "a0": 200.0,
                  "waist": 3 * TWO_PI, "duration": 20.0, "t_center": 40.0, "i_antenna": 2,
                  "lambda_um": 0.8},
        "run": _run(SEED_BASE + 3 if seed is None else seed, mode, enable_qed=True),
        "steps": 1000,
    }


def full_foil(a0=50.0, nx=512, ny=256, nz=256, mode="threshold", seed=None, dx=0.05, ppc=16,
              duration=10.0):
    """Full-size learned-hybrid workload, foil target: 512 x 256 x 256 cells
    (33.5 M), dx = 0.05, a pre-ionized hydrogen foil at 10 n_c, 1 lambda thick
    from x = 3.2, 16 particles per cell per species, mobile protons; circular
    pulse of amplitude a0 (5, 50 or 200 in the sweep), waist 3 lambda, field
    half-width `duration` = 10 centred at t = 2 duration, so its front reaches
    the foil near step 300 and its peak near step 850; photon emission and
    pair creation on; the switch is re-evaluated every 10 steps."""
    foil = {"profile": "foil", "n0": 10.0, "x0": 3.2, "length": TWO_PI, "u_th": 1e-3}
    return {
        "name": "full_foil_a%g_%dx%dx%d" % (a0, nx, ny, nz),
        "grid": _grid(nx, ny, nz, dx),
        "species": [
            dict(kind="electron", charge=-1.0, mass=1.0, ppc=ppc, mobile=True, fluid=True,
                 qed=True, **foil),
            dict(kind="ion", charge=1.0, mass=1836.15267343, ppc=ppc, mobile=True, fluid=True,
                 **foil),
            dict(kind="positron", charge=1.0, mass=1.0, ppc=ppc, profile="none", n0=10.0,
                 mobile=True, fluid=False, qed=True),
            dict(kind="photon", charge=0.0, mass=0.0, ppc=0, profile="none", mobile=True,
                 fluid=False, qed=True),
        ],
        "laser": {"enabled": True, "polarization": "circular", "a0": float(a0),
                  "waist": 3 * TWO_PI, "duration": duration, "t_center": 2 * duration,
                  "i_antenna": 2, "lambda_um": 0.8},
        "run": _run(SEED_BASE + 5 if seed is None else seed, mode, enable_qed=True,
                    enable_ionization=True, switch_every=10),
        "steps": 500,
    }


def full_gas(a0=50.0, nx=512, ny=256, nz=256, mode="threshold", seed=None, dx=0.05, ppc=16,
             duration=10.0):
    """Full-size learned-hybrid workload, gas target: 512 x 256 x 256 cells,
    dx = 0.05, neutral helium at 0.5 n_c filling the box from x = 3.2, 16
    particles per cell, immobile atoms ionized through He II (ADK/multiphoton);
    circular pulse as for the foil; photon emission on for the freed
    electrons; switch every 10 steps."""
    return {
        "name": "full_gas_a%g_%dx%dx%d" % (a0, nx, ny, nz),
        "grid": _grid(nx, ny, nz, dx),
        "species": [
            {"kind": "electron", "charge": -1.0, "mass": 1.0, "ppc": ppc, "profile": "none",
             "n0": 1.0, "u_th": 0.0, "mobile": True, "fluid": True, "qed": True},
            {"kind": "ion", "charge": 0.0, "mass": 4.0 * 1836.15267343, "ppc": ppc,
             "profile": "foil", "n0": 0.5, "x0": 3.2, "length": nx * dx, "u_th": 0.0,
             "mobile": False, "fluid": False, "ionizable": True, "z_max": 2, "target": 0,
             "ip_ev": HE_IP_EV},
            dict(kind="positron", charge=1.0, mass=1.0, ppc=ppc, profile="none", n0=1.0,
                 mobile=True, fluid=False, qed=True),
            dict(kind="photon", charge=0.0, mass=0.0, ppc=0, profile="none", mobile=True,
                 fluid=False, qed=True),
        ],
        "laser": {"enabled": True, "polarization": "circular", "a0": float(a0),
                  "waist": 3 * TWO_PI, "duration": duration, "t_center": 2 * duration,
                  "i_antenna": 2, "lambda_um": 0.8},
        "run": _run(SEED_BASE + 5 if seed is None else seed, mode, enable_qed=True,
                    enable_ionization=True, switch_every=10),
        "steps": 500,
    }


PRESETS = {"plain_hybrid": plain_hybrid, "ionization_hybrid": ionization_hybrid,
           "qed_hybrid": qed_hybrid, "full_foil": full_foil, "full_gas": full_gas}


def with_mode(cfg, mode):
    c = copy.deepcopy(cfg)
    c["run"]["switch_mode"] = mode
    return c
