"""Oracle of the laser-parameter search (test infrastructure only: the tests,
the smoke check and the bench's CPU leg use it).

Differential evolution, DE/rand/1/bin (Storn and Price, 1997), written as
plain loops: for each member i, mutant component k = x[r1][k] + F (x[r2][k] -
x[r3][k]) clipped to the bounds, taken when the uniform for k is below CR or
k is jrand, else the member's own value; the trial replaces the member when
its score is not worse.  The draws (donors, jrand, uniforms, first
population) are the seeded inputs both sides read; the score of a candidate
is the oracle simulation's plasma energy after a number of steps.

Paper: Introduction, contributions paragraph (intensity, duration and spot
size tuned by differential evolution to a plasma-energy target).
"""
from __future__ import annotations

import copy


def de(score, lo, hi, draws, F=0.7, CR=0.9):
    pop, dim = len(draws["init"]), len(lo)
    X = [[lo[k] + draws["init"][i][k] * (hi[k] - lo[k]) for k in range(dim)] for i in range(pop)]
    S = [score(x) for x in X]
    best = [min(S)]
    for g in range(len(draws["pick"])):
        for i in range(pop):
            r1, r2, r3 = (int(j) for j in draws["pick"][g][i])
            t = []
            for k in range(dim):
                v = X[r1][k] + F * (X[r2][k] - X[r3][k])
                v = min(max(v, lo[k]), hi[k])
                t.append(v if (draws["u"][g][i][k] < CR or k == int(draws["jrand"][g][i])) else X[i][k])
            st = score(t)
            if st <= S[i]:
                X[i], S[i] = t, st
        best.append(min(S))
    b = min(range(pop), key=lambda i: S[i])
    return X[b], S[b], best


def plasma_energy_after(oracle_mod, cfg, x, steps):
    """Plasma (particle + fluid) kinetic energy of the oracle run with laser
    a0, duration, waist = x (pulse centre at twice the duration)."""
    c = copy.deepcopy(cfg)
    c["laser"]["a0"], c["laser"]["duration"], c["laser"]["waist"] = (float(v) for v in x)
    c["laser"]["t_center"] = 2.0 * float(x[1])
    o = oracle_mod.Oracle(c)
    o.step(steps)
    d = o.diagnostics()
    o.close()
    return float(sum(d["kin"]) + sum(d["fluid_kin"]))
