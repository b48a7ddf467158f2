"""Pins of the oracle's training labels for the learned switch.

The label of a node (the reading stated with hk_dump_training: the paper
trains its switch on data the simulation makes but does not print the label)
fires on (a) a conversion energy e = (1/2)(sum w |u|^2 - |sum w u|^2 / sum w)
above 1e-3 of the node's kinetic energy (1/2) sum w |u|^2 with a momentum
spread sqrt(2 e / sum w) at or above thr_sigma_u, (b) a possible ionization,
(c) a possible QED emission.  Each case below is a hand-built state whose
moments are worked out by hand: two macro-particles on one node, a uniform
field, a particle of known momentum.
"""
import numpy as np
import pytest

import oracle
from paper_2510_11174_amd import configs

pytestmark = pytest.mark.filterwarnings("ignore")


def _plain(**run):
    cfg = configs.plain_hybrid(16, 16, 16, mode="all_pic")
    cfg["laser"]["enabled"] = False
    cfg["species"][0]["profile"] = "none"
    cfg["run"].update(run)
    return cfg


def _pair(o, v, d, w=0.25, node=(5, 6, 7)):
    """Two particles of weight w on one node, u_x = v + d and v - d."""
    dx = o.cfg["grid"]["dx"]
    x = np.array([[node[0] * dx, node[1] * dx, node[2] * dx]] * 2) + 1e-3 * dx
    u = np.array([[v + d, 0.0, 0.0], [v - d, 0.0, 0.0]])
    o.set_particles(0, x, u, np.array([w, w]))
    return node


@pytest.mark.parametrize("d,expect", [(0.05, 1), (0.019, 0)])
def test_spread_at_rest(d, expect):
    # at rest the whole kinetic energy is thermal (ratio 1): the label follows
    # the spread d against thr_sigma_u = 0.02; e = w d^2 exactly
    o = oracle.Oracle(_plain())
    i, j, k = _pair(o, 0.0, d)
    raw, cond = o.training_node()
    assert cond[k, j, i] & 1 == expect
    assert raw[k, j, i, 8] == pytest.approx(0.25 * d * d, rel=1e-12)
    assert int((cond & 1).sum()) == expect
    o.close()


@pytest.mark.parametrize("v,expect", [(1.0, 1), (2.0, 0)])
def test_coherent_drift_is_fluid(v, expect):
    # spread d = 0.05 on a drift v: e / KE = d^2 / (v^2 + d^2); 2.5e-3 / 1.0025
    # is above 1e-3, 2.5e-3 / 4.0025 below
    o = oracle.Oracle(_plain())
    i, j, k = _pair(o, v, 0.05)
    raw, cond = o.training_node()
    assert cond[k, j, i] & 1 == expect
    # KE = (1/2) w ((v + d)^2 + (v - d)^2) = w (v^2 + d^2), e = w d^2
    ke = 0.25 * (v * v + 0.05 ** 2)
    assert raw[k, j, i, 8] / ke == pytest.approx(0.05 ** 2 / (v * v + 0.05 ** 2), rel=1e-9)
    o.close()


def test_node_inputs_channels():
    # the density and rms-momentum channels of the pair: n = 2 w / dV,
    # |p|_rms = sqrt(v^2 + d^2)
    o = oracle.Oracle(_plain())
    i, j, k = _pair(o, 0.3, 0.04)
    raw, _ = o.training_node()
    dv = o.cfg["grid"]["dx"] ** 3
    assert raw[k, j, i, 6] == pytest.approx(0.5 / dv, rel=1e-12)
    assert raw[k, j, i, 7] == pytest.approx(np.hypot(0.3, 0.04), rel=1e-12)
    assert raw[..., 6].sum() == pytest.approx(0.5 / dv, rel=1e-12)
    o.close()


def _helium(field):
    cfg = configs.ionization_hybrid(16, 16, 16, mode="all_pic")
    cfg["laser"]["enabled"] = False
    for sp in cfg["species"]:
        sp["profile"] = "none"
    o = oracle.Oracle(cfg)
    dx = cfg["grid"]["dx"]
    o.set_particles(1, np.array([[4 * dx, 4 * dx, 4 * dx]]) + 1e-3 * dx, np.zeros((1, 3)), np.array([0.1]),
                    z=np.array([0]))
    if field:
        o.set_field("ey", np.full(o.shape, field))
    return o


def test_ionization_possible():
    # neutral helium under a field of 1 (4.0e12 V/m, 7.8 atomic units, far
    # above the barrier-suppression field of He I) ionizes within a step;
    # without field, or away from the atom, nothing is possible
    for field, expect in ((1.0, 2), (0.0, 0)):
        o = _helium(field)
        _, cond = o.training_node()
        assert cond[4, 4, 4] & 2 == expect
        assert int(((cond & 2) > 0).sum()) == (1 if expect else 0)
        o.close()


def test_qed_possible():
    # chi = gamma |E| / a_s with a_s = m c^2 / (hbar omega0): 510998.95 eV over
    # 1239.84198 eV nm / 800 nm = 329718.8 at 0.8 um; u = 100 under E = 10
    # gives chi = 3.0e-3 >= 1e-3, u = 1 gives 4.3e-5
    a_s = oracle.schwinger_field(0.8)
    assert a_s == pytest.approx(510998.95 / (1239.84198 / 800.0), rel=1e-6)
    for u0, expect in ((100.0, 4), (1.0, 0)):
        cfg = _plain(enable_qed=True)
        cfg["species"][0]["qed"] = True
        o = oracle.Oracle(cfg)
        dx = cfg["grid"]["dx"]
        o.set_particles(0, np.array([[3 * dx, 3 * dx, 3 * dx]]) + 1e-3 * dx, np.array([[0.0, 0.0, u0]]),
                        np.array([0.1]))
        o.set_field("ex", np.full(o.shape, 10.0))
        _, cond = o.training_node()
        chi = np.sqrt(1 + u0 * u0) * 10.0 / a_s
        assert (chi >= 1e-3) == bool(expect)
        assert cond[3, 3, 3] & 4 == expect
        o.close()
