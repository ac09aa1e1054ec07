"""GPU parity of the per-slice Thiele step (eq. 2) through zr_thiele_slices.

Each slice of a launch is compared with the oracle's Thiele on the same nodes
and samples, bit for bit: the status, and for a confirmed slice the degrees
and every coefficient of A and B (zero above the degree).  Launches mix slices
that confirm, that meet a vanishing inverse difference (ZR_EDEGEN) and that run
out of samples (ZR_EPROBE), at node counts on both sides of every register
group boundary of the wavefront form (nk + 1 = 64, 128, 256, 512) and beyond
it (the one-lane-per-slice form), with ragged slice counts."""
import random
import sys

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

ZR_EDEGEN, ZR_EPROBE = -4, -5


def _note(msg):
    print(f"[gpu-test] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def zr():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2505_24256_amd as m
    m.lib()
    return m


def _poly_at(c, x, p):
    v = 0
    for a in reversed(c):
        v = (v * x + a) % p
    return v


def _slice(rng, p, X, kind):
    """Samples of one slice at the nodes X."""
    if kind == "rational":
        a, b = rng.randint(0, 12), rng.randint(0, 12)
        num = [rng.randrange(p) for _ in range(a + 1)]
        den = [rng.randrange(1, p) for _ in range(b + 1)]
        out = []
        for x in X:
            d = _poly_at(den, x, p)
            out.append(_poly_at(num, x, p) * pow(d, p - 2, p) % p if d else 0)
        return out
    if kind == "poly":
        c = [rng.randrange(p) for _ in range(rng.randint(0, len(X)))]
        return [_poly_at(c, x, p) for x in X]
    if kind == "random":
        return [rng.randrange(p) for _ in X]
    if kind == "zero":
        return [0] * len(X)
    if kind == "const":
        v = rng.randrange(1, p)
        return [v] * len(X)
    if kind == "repeat":  # few distinct values: vanishing inverse differences
        vals = [rng.randrange(p) for _ in range(2)]
        return [rng.choice(vals) for _ in X]
    raise ValueError(kind)


KINDS = ["rational", "rational", "poly", "random", "zero", "const", "repeat"]


def _run(zr, p, nk, T, seed, kinds=KINDS):
    rng = random.Random(f"thiele/{p}/{nk}/{T}/{seed}")
    X = rng.sample(range(p), nk) if p < 1 << 20 else [rng.randrange(p) for _ in range(nk)]
    assert len(set(X)) == nk
    cols = [_slice(rng, p, X, kinds[i % len(kinds)]) for i in range(T)]
    F = np.array(cols, dtype=np.uint64).T.reshape(nk, T) if T else np.zeros((nk, 0), np.uint64)
    _note(f"thiele p={p} nk={nk} T={T}")
    A, B, da, db, st = zr.thiele_slices(p, X, F)
    seen = set()
    for i in range(T):
        try:
            oa, ob = oracle.thiele(p, X, F[:, i])
            want = 0
        except oracle.OracleError as e:
            want = e.code
        assert st[i] == want, (i, kinds[i % len(kinds)], st[i], want)
        seen.add(want)
        if want:
            assert da[i] == -1 and db[i] == -1
            continue
        assert da[i] == len(oa) - 1 and db[i] == len(ob) - 1, i
        assert np.array_equal(A[:len(oa), i], oa) and np.array_equal(B[:len(ob), i], ob), i
        assert not A[len(oa):, i].any() and not B[len(ob):, i].any(), i
    return seen


@pytest.mark.parametrize("nk,T", [(2, 7), (3, 1), (12, 65), (42, 200), (63, 9), (64, 9), (65, 5), (127, 6),
                                  (128, 5), (200, 4), (255, 3), (256, 3), (511, 2)])
def test_thiele_slices_match_oracle(zr, nk, T):
    _run(zr, synth.make_prime(), nk, T, seed=1)


def test_thiele_slices_statuses_all_occur(zr):
    seen = _run(zr, synth.make_prime(), 20, 70, seed=2)
    assert seen == {0, ZR_EDEGEN, ZR_EPROBE}


@pytest.mark.parametrize("p", [3, 13, 257, 65537])
def test_thiele_slices_small_primes(zr, p):
    """Small fields make zero inverse differences and zero tails frequent."""
    nk = min(p, 12)
    _run(zr, p, nk, 300, seed=3)


def test_thiele_slices_one_lane_form(zr):
    """nk > 511 takes the one-lane-per-slice kernel."""
    _run(zr, synth.make_prime(), 520, 3, seed=4, kinds=["rational", "poly", "zero"])


def test_thiele_slices_empty_and_errors(zr):
    p = synth.make_prime()
    A, B, da, db, st = zr.thiele_slices(p, [1, 2, 3], np.zeros((3, 0), np.uint64))
    assert A.shape == (4, 0) and st.shape == (0,)
    A, B, da, db, st = zr.thiele_slices(p, [5], np.array([[7, 8]], dtype=np.uint64))
    assert list(st) == [ZR_EPROBE, ZR_EPROBE]
    with pytest.raises(zr.ZippelError) as ei:
        zr.thiele_slices(p + 2 if not synth.is_prime(p + 2) else p + 4, [1, 2], np.ones((2, 1), np.uint64))
    assert ei.value.code == zr.ZR_ENOTPRIME
