"""The allocation-free weight gradient (mpm_nn_wgrad_noalloc, for callers
that cannot allocate device memory) against the entry point it mirrors
(mpm_nn_wgrad with a caller-allocated workspace): the same kernels in the
same order, so the results must agree bit for bit.  Two calls in a row,
the second on a smaller input (the library's scratch keeps the first
call's partial sums), for a 3^3 layer and a stride-2 layer; a request whose
partial sums do not fit the scratch is refused (-3) before any launch."""
import ctypes as ct

import numpy as np
import pytest

from gpu_util import announce

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    assert torch.cuda.is_available(), "GPU tests need the MI355X"
    from paper_2302_04659_amd import unet
    L = unet.nn_lib()
    vp, i, ll = ct.c_void_p, ct.c_int, ct.c_longlong
    L.mpm_nn_wgrad_noalloc.argtypes = [i, vp, i, i, i, i, i, i, i, vp, i, i, i, ll, vp, i, vp]
    return torch, L


def _bf16(torch, shape, seed):
    g = torch.Generator(device="cpu").manual_seed(seed)
    return torch.randn(shape, generator=g).to(torch.bfloat16).view(torch.int16).cuda()


@pytest.mark.parametrize("kind,taps", [(0, 27), (2, 8)])
def test_noalloc_wgrad_matches_workspace_entry_point(env, kind, taps):
    torch, L = env
    cin, cout, chunk = 64, 32, 256
    stream = torch.cuda.current_stream().cuda_stream
    for call, (n, d) in enumerate([(2, 16), (1, 8)]):        # the second call is smaller
        announce("no-alloc wgrad kind", kind, "call", call, "n", n, "d", d)
        od = d // 2 if kind == 2 else d
        x = _bf16(torch, (n, d, d, d, cin), 10 * call + kind)
        g = _bf16(torch, (n, od, od, od, cout), 10 * call + kind + 1)
        nvox = n * od ** 3
        nchunk = (nvox + chunk - 1) // chunk
        partial = torch.zeros(nchunk * taps * cin * cout, dtype=torch.float32, device="cuda")
        gw_ref = torch.zeros((taps, cin, cout), dtype=torch.float32, device="cuda")
        gw = torch.full((taps, cin, cout), float("nan"), dtype=torch.float32, device="cuda")
        r1 = L.mpm_nn_wgrad(kind, x.data_ptr(), n, d, d, d, cin, 0, cin, g.data_ptr(), cout, 0, cout, chunk,
                            partial.data_ptr(), gw_ref.data_ptr(), 0, stream)
        r2 = L.mpm_nn_wgrad_noalloc(kind, x.data_ptr(), n, d, d, d, cin, 0, cin, g.data_ptr(), cout, 0, cout, chunk,
                                    gw.data_ptr(), 0, stream)
        torch.cuda.synchronize()
        assert r1 == 0 and r2 == 0
        assert torch.isfinite(gw_ref).all()
        assert torch.equal(gw, gw_ref), float((gw - gw_ref).abs().max())
    # partial sums beyond the scratch: refused, nothing launched
    big = L.mpm_nn_wgrad_noalloc(kind, x.data_ptr(), 64, 64, 64, 64, cin, 0, cin, g.data_ptr(), cout, 0, cout, 16,
                                 gw.data_ptr(), 0, stream)
    assert big == -3
