"""GPU parity of the one-system transposed Vandermonde solve (§1, §2.2) for
both forms of its dot-product pass on the integer vector ALU: one wave per
right-hand-side tile, and the producer/consumer form.  Each solve goes
through zr_vandermonde_solve and is compared with the oracle's solve bit for
bit; sizes straddle the row blocks (64), the chunks and the right-hand-side
tiles (1, 2, 15, 16, 17, 30, 33, 40), the uneven tile splits (31 to 50) and the
right-hand-side groups (64, 70, 100, 127), and the values include the edges of
the field and small primes."""
import random
import sys

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

VARIANTS = ["waves", "producer_consumer"]


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
    yield m
    m.solve_variant()


def _system(p, t, R, seed):
    rng = random.Random(f"vs/{p}/{t}/{R}/{seed}")
    m = set()
    while len(m) < t:
        m.add(rng.randrange(1, p))
    m = np.array(sorted(m, key=lambda _: rng.random()), dtype=np.uint64)
    rhs = np.array([[rng.randrange(p) for _ in range(t)] for _ in range(R)], dtype=np.uint64).reshape(R, t)
    return m, rhs


@pytest.mark.parametrize("variant", VARIANTS)
@pytest.mark.parametrize("t,R", [(1, 1), (2, 3), (15, 1), (16, 2), (17, 5), (63, 10), (64, 16), (65, 17),
                                 (200, 30), (1000, 33), (777, 40), (1100, 15), (2500, 30), (300, 64),
                                 (640, 70), (1000, 100), (129, 127), (100, 33), (250, 40), (900, 36),
                                 (700, 41), (600, 45), (500, 50)])
def test_solve_matches_oracle(zr, variant, t, R):
    p = synth.make_prime()
    m, rhs = _system(p, t, R, 1)
    zr.solve_variant(variant)
    _note(f"solve {variant} t={t} R={R}")
    got, st = zr.vandermonde_solve(p, m, rhs)
    assert st == 0
    assert np.array_equal(got, oracle.vandermonde_solve(p, m, rhs))


@pytest.mark.parametrize("variant", VARIANTS)
def test_solve_field_edges(zr, variant):
    """Largest prime below 2^63, values at 0, 1, p-1, p/2 +- 1."""
    p = (1 << 63) - 25
    h = p // 2
    m = np.array([1, 2, p - 1, p - 2, 1 << 62, 3, h, h + 1, h + 2, h - 1] + list(range(5, 75)), dtype=np.uint64)
    t = len(m)
    vals = [p - 1, 0, 1, h, h + 1, h - 1]
    rhs = np.array([[vals[(i * 7 + j) % len(vals)] for i in range(t)] for j in range(18)], dtype=np.uint64)
    zr.solve_variant(variant)
    got, st = zr.vandermonde_solve(p, m, rhs)
    assert st == 0
    assert np.array_equal(got, oracle.vandermonde_solve(p, m, rhs))


@pytest.mark.parametrize("variant", VARIANTS)
@pytest.mark.parametrize("p", [65537, (1 << 40) + 15, 2305843009213693951])
def test_solve_other_primes(zr, variant, p):
    assert synth.is_prime(p)
    m, rhs = _system(p, 300, 9, 2)
    zr.solve_variant(variant)
    got, st = zr.vandermonde_solve(p, m, rhs)
    assert st == 0
    assert np.array_equal(got, oracle.vandermonde_solve(p, m, rhs))


@pytest.mark.parametrize("variant", VARIANTS)
def test_solve_singular_and_empty(zr, variant):
    p = synth.make_prime()
    zr.solve_variant(variant)
    _, st = zr.vandermonde_solve(p, np.array([5, 9, 5], dtype=np.uint64), np.array([[1, 2, 3]], dtype=np.uint64))
    assert st == zr.ZR_ESINGULAR
    _, st = zr.vandermonde_solve(p, np.array([4, 0], dtype=np.uint64), np.array([[1, 2]], dtype=np.uint64))
    assert st == zr.ZR_ESINGULAR
    got, st = zr.vandermonde_solve(p, np.zeros(0, dtype=np.uint64), np.zeros((2, 0), dtype=np.uint64))
    assert st == 0 and got.size == 0


@pytest.mark.parametrize("variant", VARIANTS)
@pytest.mark.parametrize("t,R", [(10_000, 30), (20_000, 40)])
def test_solve_large_sampled_rows(zr, variant, t, R):
    """Full-size systems (the n = 6 stage size and a larger one) with both
    passes: rows sampled and solved one by one by the oracle."""
    p = synth.make_prime()
    g = synth.SplitMix64(t + R)
    m = g.uniform_block(1, p, t)
    assert len(set(int(x) for x in m)) == t
    rhs = g.uniform_block(0, p, t * R).reshape(R, t)
    zr.solve_variant(variant)
    _note(f"solve {variant} t={t} R={R}")
    got, st = zr.vandermonde_solve(p, m, rhs)
    assert st == 0
    rng = random.Random(t)
    rows = sorted(rng.sample(range(t), 40) + [0, 1, 15, 16, t - 1])
    want = oracle.vandermonde_solve_rows(p, m, rhs, rows)
    assert np.array_equal(got[:, rows], want)


def test_unknown_variant_rejected(zr):
    """Only the two integer vector ALU passes exist; any other value is an
    argument error that leaves the selection unchanged."""
    zr.solve_variant("waves")
    assert zr.lib().zr_solve_variant(2) == zr.ZR_EINVAL
    assert zr.lib().zr_solve_variant(-1) == zr.ZR_EINVAL
    p = synth.make_prime()
    m, rhs = _system(p, 40, 3, 4)
    got, st = zr.vandermonde_solve(p, m, rhs)
    assert st == 0 and np.array_equal(got, oracle.vandermonde_solve(p, m, rhs))
    zr.solve_variant()


def test_timing_dots_only(zr):
    """zr_timing_enable(2) brackets only the solve's dot-product launches;
    zr_timing_enable(1) every named launch."""
    p = synth.make_prime()
    m, rhs = _system(p, 700, 12, 3)
    zr.solve_variant()
    try:
        zr.timing(True, dots_only=True)
        zr.timing_reset()
        got, st = zr.vandermonde_solve(p, m, rhs)
        n_dots, ms_dots = zr.timing_get("vs_dots")
        n_pack, _ = zr.timing_get("vs_pack")
        assert st == 0 and n_dots == 1 and ms_dots > 0 and n_pack == 0
        zr.timing(True)
        zr.timing_reset()
        zr.vandermonde_solve(p, m, rhs)
        assert zr.timing_get("vs_dots")[0] == 1 and zr.timing_get("vs_pack")[0] == 1
    finally:
        zr.timing(False)
    assert np.array_equal(got, oracle.vandermonde_solve(p, m, rhs))
