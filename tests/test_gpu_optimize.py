"""The laser-parameter search on the GPU: with FP64 runs of the library's
hybrid step as the score it takes the same path as the oracle's search over
oracle runs (same draws, scores equal to FP64 rounding), and on the FP32
library it reaches a plasma-energy target set by a known laser."""
import numpy as np
import pytest

from oracle import de as ode
from paper_2510_11174_amd import configs, draws, optimize

pytestmark = pytest.mark.gpu

LO, HI = [0.5, 2.0, 2.0], [2.0, 5.0, 10.0]   # a0, duration, waist


@pytest.fixture(scope="module")
def hk():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2510_11174_amd import hk as hkmod
    return hkmod


def test_search_matches_oracle(hk, oracle_mod):
    cfg = configs.plain_hybrid(16, 8, 8)
    steps, target = 60, 0.04
    print("case: DE on", cfg["name"], "FP64 against the oracle", flush=True)
    seen = []

    def gpu_score(x):
        e = optimize.run_energy(hk, cfg, x, steps, precision="f64")
        seen.append(e)
        return abs(e - target) / target

    def oracle_score(x):
        return abs(ode.plasma_energy_after(oracle_mod, cfg, x, steps) - target) / target

    x, s, hist, nev = optimize.differential_evolution(gpu_score, LO, HI, pop=5, gens=3, seed=7)
    xo, so, histo = ode.de(oracle_score, LO, HI, draws.de_draws(7, 5, 3, 3))
    print("best GPU %s %.6e, oracle %s %.6e; energies %.4f..%.4f" % (x, s, xo, so, min(seen), max(seen)))
    assert list(x) == list(xo)
    assert s == pytest.approx(so, rel=1e-8, abs=1e-12)
    np.testing.assert_allclose(hist, histo, rtol=1e-8, atol=1e-12)


def test_search_reaches_energy_target(hk):
    cfg = configs.plain_hybrid(32, 16, 16)
    steps = 120
    ref = [1.2, 3.5, 6.0]
    target = optimize.run_energy(hk, cfg, ref, steps)
    print("case: DE on", cfg["name"], "target %.5f (laser %s)" % (target, ref), flush=True)
    r = optimize.optimize_laser(hk, cfg, target, LO, HI, steps, pop=8, gens=6, seed=3)
    print("best %s rel error %.3e; %d runs, %.1f runs/s, %.0f steps/s" % (
        r["x"], r["rel_error"], r["evaluations"], r["runs_per_s"], r["steps_per_s"]))
    assert r["rel_error"] < 0.05
    assert all(b <= a for a, b in zip(r["history"], r["history"][1:]))
