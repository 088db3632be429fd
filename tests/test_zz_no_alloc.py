"""wamct_idiv_noalloc (the context-free I-divergence that allocates nothing: its partial sums
live in a static per-device buffer) against wamct_idiv of a context on the same q: equal bit
for bit, on two calls in a row (the second with a smaller input, which reuses the buffer the
first filled) in FP32 and FP64, for one scan and a stack. Size limits are rejected on the host."""
import numpy as np
import pytest
import torch

from paper_1508_04458_amd import synth

pytestmark = pytest.mark.gpu


def _case(name, dtype, scans, seed):
    from paper_1508_04458_amd import api
    P = synth.make_problem(name)
    tdt = torch.float32 if dtype == "f32" else torch.float64
    rng = np.random.default_rng(seed)
    d = np.stack([P.d] * scans) if scans > 1 else P.d
    d = d + rng.integers(0, 3, size=d.shape) * (d > 0)      # distinct scans, zero counts kept
    q = np.maximum(d, 1.0) * rng.uniform(0.5, 1.5, size=d.shape)
    c = api.Context(P.geom, P.levels, dtype, batch=scans)
    dd = torch.as_tensor(d.reshape(scans, -1), dtype=tdt, device="cuda").contiguous()
    qq = torch.as_tensor(q.reshape(scans, -1), dtype=tdt, device="cuda").contiguous()
    c.set_data(dd if scans > 1 else dd[0], [P.i0] * scans if scans > 1 else P.i0)
    want = c.idiv(qq if scans > 1 else qq[0]).reshape(-1)
    return dd, qq, want


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_idiv_noalloc_equals_idiv_twice_in_a_row(dtype):
    from paper_1508_04458_amd import api
    big = _case("fan128", dtype, 3, 1)        # 3 scans x 46,080 rays
    small = _case("parallel64", dtype, 1, 2)  # 1 scan x 8,640 rays: the buffer holds the first call's sums
    for dd, qq, want in (big, small):
        out = torch.full((dd.shape[0],), float("nan"), dtype=torch.float64, device="cuda")
        api.idiv_noalloc(dd if dd.shape[0] > 1 else dd[0], qq if qq.shape[0] > 1 else qq[0], out)
        torch.cuda.synchronize()
        np.testing.assert_array_equal(out.cpu().numpy(), want.cpu().numpy())
        assert np.all(np.isfinite(out.cpu().numpy()))


def test_idiv_noalloc_limits():
    from paper_1508_04458_amd import api, _lib
    x = torch.ones(8, dtype=torch.float32, device="cuda")
    out = torch.zeros(1, dtype=torch.float64, device="cuda")
    # too many partial sums for the static buffer: rejected before any launch
    n = api.NOALLOC_MAX_PARTIALS * api.NOALLOC_RAYS_PER_PARTIAL + 1
    st = _lib.lib.wamct_idiv_noalloc(_lib.F32, n, 1, api._ptr(x), api._ptr(x), api._ptr(out), None)
    assert st == _lib.E_INVALID
    assert b"static buffer" in _lib.lib.wamct_last_error(None)
    st = _lib.lib.wamct_idiv_noalloc(_lib.F32, 4, 70000, api._ptr(x), api._ptr(x), api._ptr(out), None)
    assert st == _lib.E_INVALID
    st = _lib.lib.wamct_idiv_noalloc(7, 4, 1, api._ptr(x), api._ptr(x), api._ptr(out), None)
    assert st == _lib.E_INVALID
    st = _lib.lib.wamct_idiv_noalloc(_lib.F32, 4, 1, None, api._ptr(x), api._ptr(out), None)
    assert st == _lib.E_INVALID
    # the largest accepted size: exactly the buffer
    m = api.NOALLOC_RAYS_PER_PARTIAL * 4096
    d = torch.full((256, m), 2.0, dtype=torch.float32, device="cuda")
    q = torch.full((256, m), 1.0, dtype=torch.float32, device="cuda")
    out = torch.zeros(256, dtype=torch.float64, device="cuda")
    api.idiv_noalloc(d, q, out)
    torch.cuda.synchronize()
    want = m * (1.0 - 2.0 + 2.0 * np.log(2.0))
    np.testing.assert_allclose(out.cpu().numpy(), want, rtol=1e-12)
