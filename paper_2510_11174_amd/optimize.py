"""Laser-parameter optimization by differential evolution over hybrid runs.

Paper: Introduction, contributions paragraph (laser intensity, duration and
spot size are tuned by differential evolution to reach a plasma-energy
target) and the Methodology's closing stage (final parameter optimization).
The search is the classic DE/rand/1/bin of Storn and Price (1997): for each
member x_i a mutant v = x_r1 + F (x_r2 - x_r3) from three other members,
crossed over parameter by parameter with probability CR (one parameter, jrand,
always from v), clipped to the bounds, and kept if it scores no worse.  Every
score is a full run of the library's hybrid step; the random draws come from
`draws.de_draws`.

Parameters: a0 (intensity), duration (1/omega0) and waist (c/omega0) of the
laser; the score is |U_plasma - target| / target, U_plasma the particle plus
fluid kinetic energy after `steps` steps (library diagnostics, FP64 sums).
"""
from __future__ import annotations

import copy
import math
import time

import numpy as np

from . import draws

PARAMS = ("a0", "duration", "waist")


def plasma_energy(diag: dict) -> float:
    return float(sum(diag["kin"]) + sum(diag["fluid_kin"]))


def with_laser(cfg: dict, x) -> dict:
    c = copy.deepcopy(cfg)
    for k, v in zip(PARAMS, x):
        c["laser"][k] = float(v)
    c["laser"]["t_center"] = 2.0 * float(x[1])
    return c


def run_energy(hk, cfg: dict, x, steps: int, precision: str = "f32") -> float:
    """Plasma energy after `steps` steps of the hybrid with laser parameters x."""
    sim = hk.Sim(with_laser(cfg, x), precision=precision)
    sim.step(steps)
    e = plasma_energy(sim.diagnostics())
    sim.close()
    return e


def differential_evolution(score, lo, hi, pop=8, gens=10, F=0.7, CR=0.9, seed=0, log=None):
    """DE/rand/1/bin.  score(x) -> float (lower is better); lo, hi bounds.
    Returns (best x, best score, history of the best score per generation,
    number of evaluations)."""
    lo = np.asarray(lo, float); hi = np.asarray(hi, float)
    dim = lo.size
    d = draws.de_draws(seed, pop, dim, gens)
    X = lo + d["init"] * (hi - lo)
    S = np.array([score(x) for x in X])
    nev = pop
    hist = [float(S.min())]
    for g in range(gens):
        for i in range(pop):
            r1, r2, r3 = d["pick"][g, i]
            v = np.clip(X[r1] + F * (X[r2] - X[r3]), lo, hi)
            take = d["u"][g, i] < CR
            take[d["jrand"][g, i]] = True
            t = np.where(take, v, X[i])
            st = score(t)
            nev += 1
            if st <= S[i]:
                X[i], S[i] = t, st
        hist.append(float(S.min()))
        if log:
            log("generation %d best %.4e" % (g + 1, hist[-1]))
    b = int(np.argmin(S))
    return X[b], float(S[b]), hist, nev


def optimize_laser(hk, cfg: dict, target: float, lo, hi, steps: int, pop=8, gens=6, seed=0,
                   precision: str = "f32", log=None) -> dict:
    """Search a0, duration and waist so that the plasma energy after `steps`
    steps reaches `target`.  Returns the best parameters, their energy and the
    search's timing."""
    t0 = time.perf_counter()

    def score(x):
        return abs(run_energy(hk, cfg, x, steps, precision) - target) / target

    x, s, hist, nev = differential_evolution(score, lo, hi, pop, gens, seed=seed, log=log)
    dt = time.perf_counter() - t0
    return {"x": dict(zip(PARAMS, map(float, x))), "rel_error": s, "history": hist, "evaluations": nev,
            "seconds": dt, "runs_per_s": nev / dt, "steps_per_s": nev * steps / dt}
