"""Pins of the oracle's QED module (CPU only): Airy functions against
scipy.special.airy, the rate asymptotes of the emission and pair spectra, the
tables against an independent scipy quadrature, and Monte Carlo statistics
and conservation laws in constant fields."""
import math

import numpy as np
import pytest
from scipy import integrate, special

from paper_2510_11174_amd import configs

ALPHA = 7.2973525693e-3


def test_airy_matches_scipy(oracle_mod):
    for z in [1e-8, 1e-3, 0.1, 0.7, 1.0, 2.5, 6.0, 15.0, 40.0]:
        ai, aip, iai = oracle_mod.airy(z)
        ref_ai, ref_aip, _, _ = special.airy(z)
        ref_i = integrate.quad(lambda x: special.airy(x)[0], z, np.inf, epsabs=0, epsrel=1e-13,
                               limit=200)[0]
        assert ai == pytest.approx(ref_ai, rel=1e-12)
        assert aip == pytest.approx(ref_aip, rel=1e-12)
        assert iai == pytest.approx(ref_i, rel=1e-11)


def _scipy_emission(chi, delta):
    z = (delta / (chi * (1 - delta))) ** (2 / 3)
    ai, aip, _, _ = special.airy(z)
    iai = integrate.quad(lambda x: special.airy(x)[0], z, np.inf, epsabs=0, epsrel=1e-13, limit=200)[0]
    return -iai - (2 / z + chi * delta * math.sqrt(z)) * aip


def test_spectra_match_scipy_airy(oracle_mod):
    # the spectra written out with an independent Airy evaluation
    for chi, d in [(0.01, 0.003), (1.0, 0.2), (1.0, 0.9), (50.0, 0.99)]:
        assert oracle_mod.emission_spectrum(chi, d) == pytest.approx(_scipy_emission(chi, d), rel=1e-10)
        z = (1 / (chi * d * (1 - d))) ** (2 / 3)
        ai, aip, _, _ = special.airy(z)
        iai = integrate.quad(lambda x: special.airy(x)[0], z, np.inf, epsabs=0, epsrel=1e-13, limit=200)[0]
        assert oracle_mod.pair_spectrum(chi, d) == pytest.approx(iai + (2 / z - chi * math.sqrt(z)) * aip,
                                                                 rel=1e-9)


def test_emission_rate_asymptotes(oracle_mod):
    # chi << 1: photon number rate -> 5 / (2 sqrt 3) chi (classical synchrotron)
    lim = 5 / (2 * math.sqrt(3))
    r5 = oracle_mod.qed_total("emission", 1e-5) / 1e-5
    r4 = oracle_mod.qed_total("emission", 1e-4) / 1e-4
    assert abs(r5 - lim) < abs(r4 - lim) < 2e-4
    assert r5 == pytest.approx(lim, rel=2e-5)
    # chi >> 1: -> 14 Gamma(2/3) / (9 3^(1/3)) chi^(2/3)
    big = 14 * special.gamma(2 / 3) / (9 * 3 ** (1 / 3))
    assert oracle_mod.qed_total("emission", 1e8) / 1e8 ** (2 / 3) == pytest.approx(big, rel=2e-4)
    # emitted power: (2/3) chi^2 times the Gaunt factor 1 - (55 sqrt 3 / 16) chi + 48 chi^2
    chi = 1e-3
    gaunt = oracle_mod.qed_total("power", chi) / (2 / 3 * chi ** 2)
    assert gaunt == pytest.approx(1 - 55 * math.sqrt(3) / 16 * chi + 48 * chi ** 2, abs=3e-6)


def test_pair_rate_asymptotes(oracle_mod):
    # chi << 1: -> 3 sqrt 3 / (16 sqrt 2) chi exp(-8 / (3 chi)); the ratio climbs to it
    lim = 3 * math.sqrt(3) / (16 * math.sqrt(2))
    ratios = [oracle_mod.qed_total("pair", c) / (c * math.exp(-8 / (3 * c))) for c in (0.05, 0.02, 0.005)]
    assert ratios[0] < ratios[1] < ratios[2] < lim
    assert ratios[2] == pytest.approx(lim, rel=2e-3)
    # chi >> 1: -> 0.3796 chi^(2/3)
    assert oracle_mod.qed_total("pair", 1e12) / 1e12 ** (2 / 3) == pytest.approx(0.379612, rel=1e-5)


@pytest.fixture(scope="module")
def tables(oracle_mod):
    return oracle_mod.qed_tables()


def _delta(x):
    return x ** 3 / (x ** 3 + (1 - x) ** 3)


def test_tables_against_scipy_quadrature(oracle_mod, tables):
    We, Wb, Xe, Xb = tables
    chis = 10 ** (-3 + 6 * np.arange(256) / 255)
    assert np.all(np.diff(We) > 0) and np.all(np.diff(Wb) >= 0)
    assert np.all(np.diff(Xe, axis=1) > 0) and np.all(np.diff(Xb, axis=1) > 0)
    for i in (0, 128, 255):
        chi = chis[i]
        f = lambda d: _scipy_emission(chi, d)
        pts = [chi * 0.1, chi, min(0.5, 10 * chi)]
        tot = integrate.quad(f, 0, 1, points=pts, epsabs=0, epsrel=1e-11, limit=400)[0]
        assert We[i] == pytest.approx(tot, rel=1e-8)
        for j in (5, 64, 120):
            d = _delta(Xe[i, j])
            part = integrate.quad(f, 0, d, points=[p for p in pts if p < d], epsabs=0, epsrel=1e-11,
                                  limit=400)[0]
            assert part / tot == pytest.approx((j + 0.5) / 128, abs=1e-7)
    # pair table at chi = 10 (row where chi_i is nearest) against scipy
    i = int(round((1 + 3) * 255 / 6))
    chi = chis[i]
    tot = integrate.quad(lambda d: oracle_mod.pair_spectrum(chi, d), 0, 1, epsabs=0, epsrel=1e-11,
                         limit=400)[0]
    assert Wb[i] == pytest.approx(tot, rel=1e-8)
    # symmetric spectrum: the median split is 1/2 and the table is antisymmetric about it
    np.testing.assert_allclose(_delta(Xb[i, ::-1]), 1 - _delta(Xb[i]), atol=1e-8)


def _qed_box(photons_convert=False):
    """Periodic 4^3 box, laser off, uniform B along x; particles are placed by
    the test.  Species: electron (qed), positron, photon."""
    cfg = configs.qed_hybrid(4, 4, 4, mode="all_pic", dx=0.2, ppc=1)
    cfg["grid"]["bc_x"] = "periodic"
    cfg["laser"]["enabled"] = False
    sp = cfg["species"]
    cfg["species"] = [dict(sp[0], profile="none", fluid=False, qed=not photons_convert),
                      dict(sp[2], profile="none", qed=not photons_convert),
                      dict(sp[3])]
    return cfg


def _set_uniform_b(o, B0):
    for c in ("ex", "ey", "ez", "by", "bz"):
        o.set_field(c, np.zeros(o.shape))
    o.set_field("bx", np.full(o.shape, B0))


def _uniform_points(n, box, seed):
    rng = np.random.default_rng(seed)
    return rng.uniform(0, 1, (n, 3)) * np.asarray(box)


def test_emission_first_event_statistics(oracle_mod):
    # u perpendicular to a uniform B: gamma and chi stay constant until the first
    # emission, so the fraction that has emitted after N steps is 1 - exp(-W N dt)
    a_s = oracle_mod.schwinger_field(0.8)
    gamma0, chi0 = 1000.0, 1.0
    B0 = chi0 * a_s / math.sqrt(gamma0 ** 2 - 1)
    cfg = _qed_box()
    o = oracle_mod.Oracle(cfg)
    _set_uniform_b(o, B0)
    n = 2000
    box = [4 * 0.2] * 3
    x = _uniform_points(n, box, 1)
    u = np.zeros((n, 3)); u[:, 2] = math.sqrt(gamma0 ** 2 - 1)
    w = np.full(n, 1e-12)
    o.set_particles(0, x, u, w, ids=np.arange(n, dtype=np.uint64) + 1000)
    # the optical depths of set particles: draw them as new particles would
    dt = cfg["grid"]["dt"]
    N = 3
    p0 = o.get_particles(0)
    o.step(N)
    p1 = o.get_particles(0)
    order = np.argsort(p1["id"]); p1 = {k: v[order] for k, v in p1.items()}
    order = np.argsort(p0["id"]); p0 = {k: v[order] for k, v in p0.items()}
    g1 = np.sqrt(1 + (p1["u"] ** 2).sum(1))
    emitted = g1 < gamma0 * (1 - 1e-9)
    W = ALPHA * a_s / gamma0 * oracle_mod.qed_total("emission", chi0)
    # the first emission happens when the running integral W t exceeds the initial tau
    expect = (p0["tau"] <= W * dt * N).mean()
    assert abs(emitted.mean() - expect) <= 2.0 / n    # the table W differs from the exact one
    # and the initial optical depths are exponential: compare with 1 - exp(-W N dt)
    pexp = 1 - math.exp(-W * dt * N)
    sigma = math.sqrt(pexp * (1 - pexp) / n)
    assert abs(emitted.mean() - pexp) < 4 * sigma


def _splitmix64(x):
    m = (1 << 64) - 1
    z = (x + 0x9E3779B97F4A7C15) & m
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & m
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & m
    return z ^ (z >> 31)


def _child(parent, step, k):
    return _splitmix64(int(parent) ^ _splitmix64((step << 8) | k))


def test_emission_conserves_momentum(oracle_mod):
    # one step: the photon takes k = delta u before the push; a uniform B keeps
    # |u| in the push, so |u_after| + |k| = |u_before| for each emitter
    a_s = oracle_mod.schwinger_field(0.8)
    gamma0 = 2000.0
    B0 = 2.0 * a_s / math.sqrt(gamma0 ** 2 - 1)
    cfg = _qed_box()
    o = oracle_mod.Oracle(cfg)
    _set_uniform_b(o, B0)
    n = 400
    x = _uniform_points(n, [0.8] * 3, 2)
    u0 = math.sqrt(gamma0 ** 2 - 1)
    u = np.zeros((n, 3)); u[:, 2] = u0
    ids = np.arange(n, dtype=np.uint64) + 7
    o.set_particles(0, x, u, np.full(n, 1e-12), ids=ids, tau=np.full(n, 1e-9))
    o.step(1)
    pe = o.get_particles(0)
    ph = o.get_particles(2)
    assert len(ph["id"]) > 0.5 * n        # every electron had tau ~ 0: most photons are hard
    by_id = {int(i): k for k, i in enumerate(pe["id"])}
    for k, pid in enumerate(ph["id"]):
        parent = [i for i in ids if _child(i, 0, 1) == int(pid)]
        assert len(parent) == 1
        e = by_id[int(parent[0])]
        ue = np.linalg.norm(pe["u"][e]); kk = np.linalg.norm(ph["u"][k])
        assert ue + kk == pytest.approx(u0, rel=1e-13)


def test_pair_creation_conserves_energy_and_charge(oracle_mod):
    # photons in a uniform B (leptons without emission): photon + lepton energy
    # plus the ledger is constant, div E - rho stays at its initial value, and
    # the converted fraction follows 1 - exp(-W N dt) (chi fixed by k and B)
    a_s = oracle_mod.schwinger_field(0.8)
    eps, chi0 = 5000.0, 2.0
    B0 = chi0 * a_s / eps
    cfg = _qed_box(photons_convert=True)
    o = oracle_mod.Oracle(cfg)
    _set_uniform_b(o, B0)
    n = 2000
    x = _uniform_points(n, [0.8] * 3, 3)
    k = np.zeros((n, 3)); k[:, 2] = eps
    ids = np.arange(n, dtype=np.uint64) + 99
    o.set_particles(2, x, k, np.full(n, 1e-9), ids=ids)
    # optical depths of new photons: -ln(1 - r), r from Philox (id, 2^32 - 1, tag 17)
    key = [cfg["run"]["seed"] & 0xFFFFFFFF, cfg["run"]["seed"] >> 32]
    taus = [-math.log(1 - oracle_mod.uniform(int(oracle_mod.philox(
        [int(i) & 0xFFFFFFFF, int(i) >> 32, 0xFFFFFFFF, 17 << 8], key)[0]))) for i in ids]
    np.testing.assert_array_equal(o.get_particles(2)["tau"], taus)
    d0 = o.diagnostics()
    e0 = sum(d0["kin"]) + d0["photon_energy"]
    dt = cfg["grid"]["dt"]
    N = 4
    o.step(N)
    d1 = o.diagnostics()
    e1 = sum(d1["kin"]) + d1["photon_energy"]
    assert e1 == pytest.approx(e0, rel=1e-10)
    assert d1["gauss_max"] < 1e-9
    conv = 1 - o.count(2) / n
    assert o.count(0) == o.count(1) == n - o.count(2)
    W = ALPHA * a_s / eps * oracle_mod.qed_total("pair", chi0)
    pexp = 1 - math.exp(-W * dt * N)
    sigma = math.sqrt(pexp * (1 - pexp) / n)
    assert abs(conv - pexp) < 4 * sigma
