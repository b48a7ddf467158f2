"""The allocation-free switch-network forward (hk_cnn_forward_noalloc) against
hk_cnn_forward: the same kernels on the library's static scratch array, so
the logits must be identical, on two calls in a row (the second smaller, so it
runs over what the first left in the array), plus the size limit."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def hk():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2510_11174_amd import hk as hkmod
    return hkmod


def _net(hk):
    from paper_2510_11174_amd import train as T
    c = hk.CNN(seed=5)
    c.set_params(T.init_params(7))
    return c


def test_noalloc_matches_forward(hk):
    import torch
    c = _net(hk)
    rng = np.random.default_rng(41)
    # second call smaller than the first: the scratch array still holds the
    # first call's activations where the second does not write
    for shape in [(4, 24, 40, 33), (1, 11, 13, 19)]:
        print("case: cnn forward_noalloc", shape, flush=True)
        x = torch.tensor(rng.normal(0, 1, shape + (8,)).astype(np.float32), device="cuda")
        ref = c.forward(x)
        got = c.forward_noalloc(x)
        torch.cuda.synchronize()
        assert got.shape == ref.shape
        assert torch.equal(got, ref), float((got - ref).abs().max())
    c.close()


def test_noalloc_limit(hk):
    import torch
    c = _net(hk)
    # exactly at the limit: 2^18 voxels
    x = torch.zeros((1, 64, 64, 64, 8), device="cuda")
    out = c.forward_noalloc(x)
    torch.cuda.synchronize()
    assert torch.equal(out, c.forward(x))
    # beyond it: a clear error, nothing launched
    x = torch.zeros((1, 65, 64, 64, 8), device="cuda")
    with pytest.raises(hk.HKError) as ei:
        c.forward_noalloc(x)
    assert ei.value.code == -1 and "exceed" in str(ei.value)
    c.close()
