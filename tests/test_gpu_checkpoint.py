"""Checkpoint and resume through the C ABI (hk_save / hk_load): a run saved at
step n and resumed in a fresh context matches the uninterrupted run, with the
same switch maps, ionization events and particle ids."""
import numpy as np
import pytest

from paper_2510_11174_amd import configs
from tests.parity import match_particles, rel_l2

pytestmark = pytest.mark.gpu

FIELDS = ["ex", "ey", "ez", "bx", "by", "bz", "jx", "jy", "jz"]


@pytest.fixture(scope="module")
def hk():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2510_11174_amd import hk as hkmod
    return hkmod


def _state(s, nsp):
    f = {c: s.get_field(c).astype(np.float64) for c in FIELDS}
    p = [s.get_particles(k) for k in range(nsp)]
    return f, p, s.get_switch().copy(), s.diagnostics()


def _compare(a, b, tol):
    fa, pa, sa, da = a
    fb, pb, sb, db = b
    assert (sa == sb).all()
    for c in FIELDS:
        assert rel_l2(fa[c], fb[c]) <= tol, c
    for x, y in zip(pa, pb):
        assert len(x["id"]) == len(y["id"])
        assert (np.sort(x["id"]) == np.sort(y["id"])).all()
        i, j = match_particles(x, y)
        assert (x["z"][i] == y["z"][j]).all()
        for k in ("x", "u", "w"):
            d = np.abs(x[k][i] - y[k][j]).max() if len(i) else 0.0
            assert d <= tol * max(1.0, np.abs(y[k][j]).max() if len(j) else 1.0), k
    assert da["step"] == db["step"] and abs(da["t"] - db["t"]) <= 1e-12


@pytest.mark.parametrize("prec", ["f32", "f64"])
@pytest.mark.parametrize("case", ["plain_threshold", "ionization"])
def test_resume_matches_uninterrupted(hk, tmp_path, prec, case):
    if case == "plain_threshold":
        cfg = configs.plain_hybrid(32, 16, 16, mode="threshold")
        cfg["species"][0]["u_th"] = 0.05      # a mixed map: conversions both ways
        n1, n2, nsp = 20, 20, 1
    else:
        cfg = configs.ionization_hybrid(32, 16, 16, mode="threshold", ppc=4)
        n1, n2, nsp = 40, 20, 2
    print("case:", case, prec, flush=True)
    path = str(tmp_path / "ck.bin")
    a = hk.Sim(cfg, precision=prec)
    a.step(n1)
    a.save(path)
    # the restored state is the saved one, bit for bit
    b = hk.Sim(cfg, precision=prec)
    b.load(path)
    _compare(_state(a, nsp), _state(b, nsp), 0.0)
    a.step(n2); b.step(n2)
    # then both runs go on alike.  Float atomics add in any order, and the
    # restored particles are re-binned, so FP64 LDS sums take another order:
    # rounding noise that the a0 = 10 ionizing pulse amplifies to ~1e-11 in 20
    # steps.  In FP32 that noise can flip an ionization draw next to its
    # threshold, so the ionizing case continues in FP64 only.
    if not (case == "ionization" and prec == "f32"):
        tol = 1e-4 if prec == "f32" else (1e-9 if case == "ionization" else 1e-11)
        _compare(_state(a, nsp), _state(b, nsp), tol)
    a.close(); b.close()


def test_load_rejects_other_grid(hk, tmp_path):
    path = str(tmp_path / "ck.bin")
    a = hk.Sim(configs.plain_hybrid(16, 8, 8), precision="f32")
    a.step(2)
    a.save(path)
    b = hk.Sim(configs.plain_hybrid(16, 8, 16), precision="f32")
    with pytest.raises(RuntimeError):
        b.load(path)
    c = hk.Sim(configs.plain_hybrid(16, 8, 8), precision="f64")
    with pytest.raises(RuntimeError):
        c.load(path)
    with pytest.raises(RuntimeError):
        c.load(str(tmp_path / "missing.bin"))
    a.close(); b.close(); c.close()


def test_load_failures_leave_or_poison(hk, tmp_path):
    # a header that does not match changes nothing: the context steps on as
    # if the call had not happened; a body cut short poisons the context
    print("case: checkpoint header mismatch and truncated body", flush=True)
    path = str(tmp_path / "ck.bin")
    cfg = configs.plain_hybrid(16, 8, 8)
    a = hk.Sim(cfg, precision="f32")
    a.step(3)
    a.save(path)
    other = hk.Sim(configs.plain_hybrid(16, 8, 16), precision="f32")
    other.step(1)
    before = other.get_field("ey").copy()
    with pytest.raises(RuntimeError):
        other.load(path)
    assert np.array_equal(other.get_field("ey"), before)
    other.step(1)                      # still usable
    with open(path, "rb") as fh:
        blob = fh.read()
    cut = str(tmp_path / "cut.bin")
    with open(cut, "wb") as fh:
        fh.write(blob[: len(blob) // 2])
    b = hk.Sim(cfg, precision="f32")
    with pytest.raises(RuntimeError):
        b.load(cut)
    with pytest.raises(RuntimeError) as e:
        b.step(1)
    assert "poisoned" in str(e.value) or "HK_ESTATE" in str(e.value)
    a.close(); other.close(); b.close()
