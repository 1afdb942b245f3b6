"""The no-workspace variant of closure_moments against closure_moments.

closure_moments_noalloc keeps its partial sums in a static device array
instead of a caller workspace; the kernels are the same, so the results
must be identical bit for bit. Two calls in a row, the second with fewer
channels and points, check that the array's leftovers from the first call
do not leak into the second.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def E():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1902_02508_amd import eles
    return eles


def _data(shape, seed):
    import torch
    rng = np.random.default_rng(seed)
    scale = np.arange(1, shape[1] + 1, dtype=np.float64)[None, :, None] * 0.7
    a = rng.standard_normal((shape[0], shape[1], int(np.prod(shape[2:])))) * scale + 2.5
    return torch.from_numpy(a.reshape(shape).astype(np.float32)).cuda()


def test_noalloc_moments_equal_workspace_moments(E):
    import torch
    big = _data((3, 10, 33, 17, 40), 1)
    small = _data((2, 6, 5, 9, 7), 2)
    for data in (big, small):
        ref = E.moments(data)
        got = E.moments_noalloc(data)
        torch.cuda.synchronize()
        print("noalloc moments", tuple(data.shape), "max |diff|",
              float((got - ref).abs().max()), flush=True)
        assert torch.equal(got, ref)
    # the largest channel count the static array takes, then one past it
    wide = _data((1, E.MOMENTS_NOALLOC_MAX_CHAN, 3, 4, 5), 3)
    assert torch.equal(E.moments_noalloc(wide), E.moments(wide))
    over = _data((1, E.MOMENTS_NOALLOC_MAX_CHAN + 1, 2, 2, 2), 4)
    out = torch.empty((2, E.MOMENTS_NOALLOC_MAX_CHAN + 1), dtype=torch.float64, device=over.device)
    st = E.lib.closure_moments_noalloc(E._ptr(over), E.MOMENTS_NOALLOC_MAX_CHAN + 1, 1, 8, E._ptr(out), None)
    assert st == E.ELES_ENOSPACE
    assert E.lib.closure_moments_noalloc(None, 3, 1, 8, E._ptr(out), None) == E.ELES_EINVAL
