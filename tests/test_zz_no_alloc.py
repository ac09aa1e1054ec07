"""The no-allocation solve (zr_vandermonde_solve_noalloc) against the
allocating one (zr_vandermonde_solve) through the C ABI: bit-identical
solutions and statuses on two calls in a row, the second with a smaller
system, so that the second call reads a workspace the first one left filled;
and a system too large for the fixed workspace is refused before any device
work."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.uint64).view(np.int64)).cuda()


def _system(p, t, R, seed):
    g = synth.SplitMix64(seed)
    m = g.uniform_block(1, p, t)
    assert len(set(int(x) for x in m)) == t
    rhs = g.uniform_block(0, p, t * R).reshape(R, t)
    return m, rhs


def _both(zr, p, m, rhs):
    import torch
    t, R = len(m), rhs.shape[0]
    d_m, d_r = _dev(m), _dev(rhs.reshape(-1))
    ref_out = torch.full_like(d_r, -1)
    got_out = torch.full_like(d_r, -1)
    ref_st = torch.full((1,), 99, dtype=torch.int32, device="cuda")
    got_st = torch.full((1,), 99, dtype=torch.int32, device="cuda")
    L = zr.lib()
    s = zr._stream(None)
    assert L.zr_vandermonde_solve(p, t, R, d_m.data_ptr(), d_r.data_ptr(), ref_out.data_ptr(), ref_st.data_ptr(),
                                  s) == 0
    assert zr.vandermonde_solve_noalloc(p, d_m, d_r, got_out, got_st, t, R) == 0
    torch.cuda.synchronize()
    ref = ref_out.cpu().numpy().view(np.uint64).reshape(R, t)
    got = got_out.cpu().numpy().view(np.uint64).reshape(R, t)
    return ref, got, int(ref_st.item()), int(got_st.item())


def test_noalloc_equals_allocating_solve_twice():
    import paper_2505_24256_amd as zr
    p = synth.make_prime()
    # first: 40 right-hand sides, more chunks than the fixed workspace holds
    # partial-sum slots for (the chunks take the slots in turn over several
    # launches); second: fewer chunks, all with a slot of their own; third:
    # smaller and with fewer right-hand sides (one wave per tile)
    for t, R, seed in ((20000, 40, 70), (6000, 40, 71), (700, 7, 72)):
        m, rhs = _system(p, t, R, seed)
        print(f"[no-alloc] t={t} R={R} seed={seed}", flush=True)
        ref, got, st_ref, st_got = _both(zr, p, m, rhs)
        assert st_ref == 0 and st_got == 0
        assert np.array_equal(got, ref)
        # the solution reproduces the right-hand sides: sum_l a_l m_l^i = v_i
        i = np.array([1, t // 2, t], dtype=np.uint64)
        for j in (0, R - 1):
            for ii in i:
                acc = 0
                for l in range(t):
                    acc = (acc + int(got[j, l]) * pow(int(m[l]), int(ii), p)) % p
                assert acc == int(rhs[j, int(ii) - 1])


def test_noalloc_singular_and_empty():
    import torch
    import paper_2505_24256_amd as zr
    p = synth.make_prime()
    m, rhs = _system(p, 300, 12, 73)
    m[17] = m[200]
    ref, got, st_ref, st_got = _both(zr, p, m, rhs)
    assert st_ref == -3 and st_got == -3
    d = torch.zeros(1, dtype=torch.int64, device="cuda")
    st = torch.full((1,), 99, dtype=torch.int32, device="cuda")
    assert zr.vandermonde_solve_noalloc(p, d, d, d, st, 0, 5) == 0
    torch.cuda.synchronize()
    assert int(st.item()) == 0


def test_noalloc_refuses_systems_beyond_its_workspace():
    import torch
    import paper_2505_24256_amd as zr
    p = synth.make_prime()
    t, R = 200_000, 40
    d = torch.zeros(1, dtype=torch.int64, device="cuda")
    st = torch.full((1,), 99, dtype=torch.int32, device="cuda")
    # refused on the host before any device work: the one-word buffers are never touched
    assert zr.vandermonde_solve_noalloc(p, d, d, d, st, t, R) == -1
    assert b"workspace" in zr.lib().zr_last_error()
    torch.cuda.synchronize()
    assert int(st.item()) == 99
