"""The device black box used for the large synthetic workloads must give the
same values as the host black box (both are input generators; neither is part
of the reconstruction)."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("nvars,nterms,k,ni,nj,i_first", [
    (5, 6000, 2, 100, 7, 1), (5, 6000, 3, 1000, 31, 1), (5, 6000, 4, 3000, 31, 1), (5, 6000, 4, 257, 40, 1000),
    (5, 6000, 5, 100, 31, 1),            # many groups, few powers: groups split across workgroups
    (6, 20000, 6, 3000, 40, 77),         # more than 512 groups per workgroup: column normalisation
    (3, 500, 1, 50, 3, 1)])
def test_device_eval_matches_host(nvars, nterms, k, ni, nj, i_first):
    import torch
    p = synth.make_prime()
    poly = synth.random_poly(p, nvars, 12, nterms, seed=77)
    box = synth.DeviceBlackBox(poly, nthreads=16)
    g = synth.SplitMix64(1234 + k)
    y = g.uniform_block(2, p - 1, nvars)
    anchor = g.uniform_block(1, p, nvars)
    xk = g.uniform_block(1, p, nj)
    want = box.host.eval(k, i_first, ni, y, anchor, xk)
    out = torch.zeros(ni * nj, dtype=torch.int64, device="cuda")
    torch.cuda.synchronize()
    box.device_eval(k, i_first, ni, y, anchor, xk, out.data_ptr(), 0)
    got = out.cpu().numpy().view(np.uint64)
    assert np.array_equal(got, want)


def test_device_eval_rational_matches_host():
    import torch
    rw = synth.rational_workload(5, 12, 800, 600, 31)
    box = synth.DeviceBlackBox(rw.num, rw.den, nthreads=16)
    g = synth.SplitMix64(99)
    for k, ni, nj in ((3, 500, 42), (5, 700, 42)):
        y = g.uniform_block(2, rw.p - 1, 5)
        anchor = g.uniform_block(1, rw.p, 5)
        xk = g.uniform_block(1, rw.p, nj)
        want = box.host.eval(k, 1, ni, y, anchor, xk)
        out = torch.zeros(ni * nj, dtype=torch.int64, device="cuda")
        torch.cuda.synchronize()
        box.device_eval(k, 1, ni, y, anchor, xk, out.data_ptr(), 0)
        assert np.array_equal(out.cpu().numpy().view(np.uint64), want)
