"""Seeded random draws of the laser-parameter search (inputs only, no
arithmetic of the method): the search and its test oracle both read them, so
the two explore the same candidates.

For generation g and member i of a population of P over D parameters:
  pick[g, i]  three distinct members, none equal to i (the donor indices);
  jrand[g, i] one parameter that always takes the mutant's value;
  u[g, i, :]  uniforms in [0, 1) for the crossover test;
  init[i, :]  uniforms in [0, 1) placing the first population in the bounds.
"""
from __future__ import annotations

import numpy as np


def de_draws(seed: int, pop: int, dim: int, gens: int) -> dict:
    if pop < 4:
        raise ValueError("the search needs at least 4 members")
    rng = np.random.default_rng(seed)
    init = rng.random((pop, dim))
    pick = np.empty((gens, pop, 3), np.int64)
    for g in range(gens):
        for i in range(pop):
            others = [j for j in range(pop) if j != i]
            pick[g, i] = rng.choice(others, 3, replace=False)
    jrand = rng.integers(0, dim, (gens, pop))
    u = rng.random((gens, pop, dim))
    return {"init": init, "pick": pick, "jrand": jrand, "u": u}
