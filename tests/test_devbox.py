"""The device black box used for the large synthetic workloads must give the
same values as the host black box (both are input generators; neither is part
of the reconstruction)."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("k,ni,nj,i_first", [(2, 100, 7, 1), (3, 1000, 31, 1), (4, 3000, 31, 1), (4, 257, 64, 1000)])
def test_device_eval_matches_host(k, ni, nj, i_first):
    import torch
    p = synth.make_prime()
    poly = synth.random_poly(p, 5, 12, 6000, seed=77)
    box = synth.DeviceBlackBox(poly, nthreads=16)
    g = synth.SplitMix64(1234 + k)
    y = g.uniform_block(2, p - 1, 5)
    anchor = g.uniform_block(1, p, 5)
    xk = g.uniform_block(1, p, nj)
    want = box.host.eval(k, i_first, ni, y, anchor, xk)
    out = torch.zeros(ni * nj, dtype=torch.int64, device="cuda")
    torch.cuda.synchronize()
    box.device_eval(k, i_first, ni, y, anchor, xk, out.data_ptr(), 0)
    got = out.cpu().numpy().view(np.uint64)
    assert np.array_equal(got, want)
