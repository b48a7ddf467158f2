"""The laser-parameter search on the CPU: differential evolution reaches the
minimum of analytic scores, and the library's search and the oracle's
independent loops take identical steps from the same draws."""
import math

import numpy as np

from oracle import de as ode
from paper_2510_11174_amd import draws, optimize


def test_draws_are_valid():
    d = draws.de_draws(3, 6, 3, 4)
    for g in range(4):
        for i in range(6):
            p = list(d["pick"][g, i])
            assert len(set(p)) == 3 and i not in p and all(0 <= j < 6 for j in p)
    assert d["jrand"].min() >= 0 and d["jrand"].max() < 3
    assert d["u"].min() >= 0 and d["u"].max() < 1


def test_sphere_minimum():
    lo, hi = [-5.0] * 3, [5.0] * 3
    x, s, hist, nev = optimize.differential_evolution(lambda x: float(np.sum((np.asarray(x) - 1.5) ** 2)), lo, hi,
                                                       pop=12, gens=80, seed=1)
    assert s < 1e-6 and np.allclose(x, 1.5, atol=1e-3)
    assert all(b <= a for a, b in zip(hist, hist[1:]))      # elitist: never worse
    assert nev == 12 * 81


def test_rosenbrock_valley():
    f = lambda x: (1 - x[0]) ** 2 + 100 * (x[1] - x[0] ** 2) ** 2
    x, s, _, _ = optimize.differential_evolution(f, [-2, -1], [2, 3], pop=20, gens=200, seed=2)
    assert s < 1e-6 and abs(x[0] - 1) < 1e-2 and abs(x[1] - 1) < 2e-2


def test_library_and_oracle_searches_agree():
    f = lambda x: math.sin(3 * x[0]) + (x[1] - 0.3) ** 2 + 0.1 * x[2] ** 2
    lo, hi = [-1.0, -1.0, -2.0], [1.0, 1.0, 2.0]
    x, s, hist, _ = optimize.differential_evolution(f, lo, hi, pop=7, gens=12, seed=4)
    xo, so, histo = ode.de(f, lo, hi, draws.de_draws(4, 7, 3, 12))
    assert list(x) == list(xo) and s == so and hist == histo
