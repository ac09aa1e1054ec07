"""GPU parity: the HIP path through the C ABI against the CPU oracle, bit for bit.

Every comparison is exact (integers mod p).  Inputs come from the seeded input
module; expected values come from the oracle or from the hidden polynomial the
inputs were generated from."""
import os
import random
import sys

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu


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


def _box(zr, hidden, den=None):
    b = synth.BlackBox(hidden, den)
    return zr.HostBlackBox(b.eval, hidden.nvars)


def _rand_distinct(rng, p, t):
    s = set()
    while len(s) < t:
        s.add(rng.randrange(1, p))
    return list(s)


# ---------------------------------------------------------------- Vandermonde solve

@pytest.mark.parametrize("case", [
    [(1, 1), (2, 3), (7, 2)],
    [(63, 10), (64, 10), (65, 11), (130, 30)],
    [(300, 30), (1000, 33), (777, 40)],
    [(2500, 30)],
    [(40, 1), (97, 2), (5, 48), (129, 64)],
    # producer/consumer queue: one class (10 right-hand sides per consumer
    # wave) holding systems of 2, 3 and 6 tiles, beside a one-wave system
    # (R = 10) and a class of narrower tiles (R = 11)
    [(200, 19), (150, 30), (90, 10), (70, 11), (300, 60), (64, 20)],
])
def test_vandermonde_batch_matches_oracle(zr, case):
    p = synth.make_prime()
    rng = random.Random(str(case))
    systems = []
    for t, R in case:
        m = _rand_distinct(rng, p, t)
        rhs = np.array([[rng.randrange(p) for _ in range(t)] for _ in range(R)], dtype=np.uint64)
        systems.append((np.array(m, dtype=np.uint64), rhs))
    _note(f"vandermonde batch {case}")
    got, status = zr.vandermonde_solve_batch(p, systems)
    assert list(status) == [0] * len(case)
    for (m, rhs), a in zip(systems, got):
        want = oracle.vandermonde_solve(p, m, rhs)
        assert np.array_equal(a, want)


def test_vandermonde_batch_edge_values(zr):
    """Monomial values and right-hand sides at the edges of the field."""
    p = (1 << 63) - 25
    m = np.array([1, 2, p - 1, p - 2, (1 << 62), 3], dtype=np.uint64)
    rhs = np.array([[p - 1] * 6, [0] * 6, [1, 0, p - 1, 0, 1, 0]], dtype=np.uint64)
    got, status = zr.vandermonde_solve_batch(p, [(m, rhs)])
    assert status[0] == 0
    assert np.array_equal(got[0], oracle.vandermonde_solve(p, m, rhs))


def test_vandermonde_batch_singular_and_empty(zr):
    p = synth.make_prime()
    good = (np.array([5, 7, 11], dtype=np.uint64), np.array([[1, 2, 3]], dtype=np.uint64))
    dup = (np.array([5, 9, 5], dtype=np.uint64), np.array([[1, 2, 3]], dtype=np.uint64))
    zero = (np.array([4, 0], dtype=np.uint64), np.array([[1, 2]], dtype=np.uint64))
    empty = (np.zeros(0, dtype=np.uint64), np.zeros((2, 0), dtype=np.uint64))
    got, status = zr.vandermonde_solve_batch(p, [good, dup, empty, zero])
    assert list(status) == [0, zr.ZR_ESINGULAR, 0, zr.ZR_ESINGULAR]
    assert np.array_equal(got[0], oracle.vandermonde_solve(p, *good))


def test_vandermonde_large_sampled_rows(zr):
    """t = 10^4 with 30 right-hand sides (the config-2 stage size): rows sampled."""
    p = synth.make_prime()
    rng = random.Random(77)
    t, R = 10_000, 30
    g = synth.SplitMix64(5)
    m = g.uniform_block(1, p, t)
    assert len(set(int(x) for x in m)) == t
    rhs = g.uniform_block(0, p, t * R).reshape(R, t)
    _note("vandermonde t=10^4 R=30")
    got, status = zr.vandermonde_solve_batch(p, [(m, rhs)])
    assert status[0] == 0
    rows = sorted(rng.sample(range(t), 48) + [0, t - 1])
    want = oracle.vandermonde_solve_rows(p, m, rhs, rows)
    assert np.array_equal(got[0][:, rows], want)


# ---------------------------------------------------------------- polynomial Zippel

def test_zippel_config1_every_stage(zr):
    w = synth.config_workload(1)
    box = _box(zr, w.hidden)
    obox = synth.BlackBox(w.hidden)
    for L in range(1, 4):
        _note(f"config1 stage {L}")
        e, c = zr.reconstruct(w.p, w.deg, box, sched=w.schedule, last_stage=L)
        oe, oc = oracle.zippel(w.p, w.deg, w.schedule, obox, last_stage=L)
        assert np.array_equal(e, oe) and np.array_equal(c, oc)
    assert np.array_equal(e, w.hidden.exps) and np.array_equal(c, w.hidden.coefs)


@pytest.mark.parametrize("nvars,deg,nterms,seed", [(1, 12, 5, 1), (2, 6, 49, 2), (2, 9, 20, 3), (4, 8, 300, 4),
                                                   (5, 3, 1, 5), (3, 0, 1, 6), (4, 12, 2000, 21),
                                                   (3, 40, 700, 9), (6, 2, 729, 10)])
def test_zippel_matches_oracle(zr, nvars, deg, nterms, seed):
    w = synth.poly_workload("t", nvars, deg, nterms, seed, 1000 + seed, nprobes=2)
    _note(f"zippel n={nvars} d={deg} t={nterms}")
    e, c = zr.reconstruct(w.p, w.deg, _box(zr, w.hidden), sched=w.schedule)
    oe, oc = oracle.zippel(w.p, w.deg, w.schedule, synth.BlackBox(w.hidden))
    assert np.array_equal(e, oe) and np.array_equal(c, oc)
    assert np.array_equal(e, w.hidden.exps) and np.array_equal(c, w.hidden.coefs)


def test_zippel_seed_schedule_equals_explicit(zr):
    w = synth.config_workload(1)
    e1, c1 = zr.reconstruct(w.p, w.deg, _box(zr, w.hidden), sched=w.schedule)
    e2, c2 = zr.reconstruct(w.p, w.deg, _box(zr, w.hidden), seed=1001, nprobes=2)
    assert np.array_equal(e1, e2) and np.array_equal(c1, c2)


def test_zippel_small_prime(zr):
    p = 1000003
    hidden = synth.random_poly(p, 3, [3, 2, 4], 40, 77)
    sched = synth.make_schedule(p, 3, [3, 2, 4], 5, 2)
    e, c = zr.reconstruct(p, [3, 2, 4], _box(zr, hidden), sched=sched)
    oe, oc = oracle.zippel(p, [3, 2, 4], sched, synth.BlackBox(hidden))
    assert np.array_equal(e, oe) and np.array_equal(c, oc)


def test_zippel_config2_full(zr):
    """Full config 2 (n=6, D=30, t=10^4): exact recovery, equal to the oracle."""
    w = synth.config_workload(2)
    _note("config2 gpu")
    e, c = zr.reconstruct(w.p, w.deg, _box(zr, w.hidden), sched=w.schedule)
    assert np.array_equal(e, w.hidden.exps) and np.array_equal(c, w.hidden.coefs)
    _note("config2 oracle")
    oe, oc = oracle.zippel(w.p, w.deg, w.schedule, synth.BlackBox(w.hidden), nthreads=16)
    assert np.array_equal(e, oe) and np.array_equal(c, oc)


def test_zippel_deterministic_repeat(zr):
    w = synth.poly_workload("r", 5, 10, 3000, 31, 1031)
    box = _box(zr, w.hidden)
    r1 = zr.reconstruct(w.p, w.deg, box, sched=w.schedule)
    r2 = zr.reconstruct(w.p, w.deg, box, sched=w.schedule)
    assert np.array_equal(r1[0], r2[0]) and np.array_equal(r1[1], r2[1])


# ---------------------------------------------------------------- failures

def test_zippel_failure_statuses(zr):
    p = synth.make_prime()
    exps = np.array([[1, 0, 0], [0, 1, 0], [1, 1, 1]], dtype=np.uint16)
    hidden = synth.SparsePoly(p, 3, exps, np.array([3, 5, 7], dtype=np.uint64)).sorted()
    sched = synth.make_schedule(p, 3, [2, 2, 2], 1, 0)
    sched.y[1] = sched.y[0]
    with pytest.raises(zr.ZippelError) as ei:
        zr.reconstruct(p, [2, 2, 2], _box(zr, hidden), sched=sched)
    assert ei.value.code == zr.ZR_ESINGULAR

    w = synth.poly_workload("lo", 3, 6, 30, 8, 1008, nprobes=3)
    with pytest.raises(zr.ZippelError) as ei:
        zr.reconstruct(w.p, [6, 6, 3], _box(zr, w.hidden), sched=synth.make_schedule(w.p, 3, [6, 6, 3], 1008, 3))
    assert ei.value.code == zr.ZR_EPROBE

    def broken(*a):
        raise RuntimeError("down")

    with pytest.raises(zr.ZippelError) as ei:
        zr.reconstruct(w.p, w.deg, zr.HostBlackBox(broken, 3), sched=w.schedule)
    assert ei.value.code == zr.ZR_EBLACKBOX
    composite = w.p + 2 if not synth.is_prime(w.p + 2) else w.p + 4
    with pytest.raises(zr.ZippelError) as ei:
        zr.reconstruct(composite, w.deg, _box(zr, w.hidden), sched=w.schedule)
    assert ei.value.code == zr.ZR_ENOTPRIME


# ---------------------------------------------------------------- balanced Zippel

@pytest.mark.parametrize("nvars,total,tn,td,seed", [(2, 5, 6, 4, 1), (3, 6, 12, 9, 7), (4, 8, 40, 25, 3),
                                                   (3, 4, 1, 1, 5), (5, 20, 60, 30, 11), (5, 20, 400, 300, 12)])
def test_balanced_matches_oracle(zr, nvars, total, tn, td, seed):
    rw = synth.rational_workload(nvars, total, tn, td, seed)
    _note(f"balanced n={nvars} tn={tn} td={td}")
    (en, cn), (ed, cd) = zr.balanced_reconstruct(rw.p, rw.deg_num, rw.deg_den, _box(zr, rw.num, rw.den),
                                                 sched=rw.schedule)
    (on, ocn), (od, ocd) = oracle.balanced_zippel(rw.p, rw.deg_num, rw.deg_den, rw.schedule,
                                                 synth.BlackBox(rw.num, rw.den))
    assert np.array_equal(en, on) and np.array_equal(cn, ocn)
    assert np.array_equal(ed, od) and np.array_equal(cd, ocd)
    assert np.array_equal(en, rw.num.exps) and np.array_equal(cn, rw.num.coefs)
    assert np.array_equal(ed, rw.den.exps) and np.array_equal(cd, rw.den.coefs)


def test_balanced_intermediate_stages(zr):
    rw = synth.rational_workload(4, 8, 30, 20, 13)
    for L in (1, 2, 3):
        (en, cn), (ed, cd) = zr.balanced_reconstruct(rw.p, rw.deg_num, rw.deg_den, _box(zr, rw.num, rw.den),
                                                     sched=rw.schedule, last_stage=L)
        (on, ocn), (od, ocd) = oracle.balanced_zippel(rw.p, rw.deg_num, rw.deg_den, rw.schedule,
                                                     synth.BlackBox(rw.num, rw.den), last_stage=L)
        assert np.array_equal(en, on) and np.array_equal(cn, ocn)
        assert np.array_equal(ed, od) and np.array_equal(cd, ocd)


def test_balanced_enorm(zr):
    p = synth.make_prime()
    num = synth.SparsePoly(p, 2, np.array([[0, 0], [1, 1]], dtype=np.uint16), np.array([4, 9], dtype=np.uint64))
    den = synth.SparsePoly(p, 2, np.array([[1, 0], [0, 2]], dtype=np.uint16), np.array([1, 3], dtype=np.uint64))
    dn, dd = [2, 2], [2, 2]
    J = [synth.thiele_nodes_needed(a, b) for a, b in zip(dn, dd)]
    sched = synth.make_schedule(p, 2, J, 4, 1)
    with pytest.raises(zr.ZippelError) as ei:
        zr.balanced_reconstruct(p, dn, dd, _box(zr, num.sorted(), den.sorted()), sched=sched)
    assert ei.value.code == zr.ZR_ENORM


def test_zippel_one_wave_pass(zr):
    """The one-wave-per-tile dot-product pass gives the same result as the
    default (producer/consumer) one (systems with 12 and 30 right-hand sides)."""
    for nvars, deg, nterms, seed in ((4, 12, 2000, 21), (3, 30, 3000, 33)):
        w = synth.poly_workload("pc", nvars, deg, nterms, seed, 1000 + seed, nprobes=2)
        base = zr.reconstruct(w.p, w.deg, _box(zr, w.hidden), sched=w.schedule)
        try:
            zr.solve_variant("waves")
            pc = zr.reconstruct(w.p, w.deg, _box(zr, w.hidden), sched=w.schedule)
        finally:
            zr.solve_variant()
        assert np.array_equal(base[0], pc[0]) and np.array_equal(base[1], pc[1])
        assert np.array_equal(pc[0], w.hidden.exps) and np.array_equal(pc[1], w.hidden.coefs)


# ---------------------------------------------------------------- resumption from a stage's result

@pytest.mark.parametrize("nvars,deg,nterms,seed,k", [(3, 10, 50, 1, 2), (3, 10, 50, 1, 3), (4, 12, 900, 23, 3),
                                                     (5, 8, 2000, 31, 5)])
def test_resume_from_oracle_stage(zr, nvars, deg, nterms, seed, k):
    """Stages k..n run from the oracle's stage-(k-1) result equal the
    oracle's whole reconstruction (and the hidden polynomial)."""
    w = synth.poly_workload("resume", nvars, deg, nterms, seed, 1000 + seed, nprobes=2)
    box = synth.BlackBox(w.hidden)
    start = oracle.zippel(w.p, w.deg, w.schedule, box, last_stage=k - 1)
    _note(f"resume at stage {k}: n={nvars} t={nterms}, start of {len(start[1])} terms")
    e, c = zr.reconstruct(w.p, w.deg, _box(zr, w.hidden), sched=w.schedule, first_stage=k, start=start)
    oe, oc = oracle.zippel(w.p, w.deg, w.schedule, box)
    assert np.array_equal(e, oe) and np.array_equal(c, oc)
    assert np.array_equal(e, w.hidden.exps) and np.array_equal(c, w.hidden.coefs)
    # stopping early after resuming: stage L's result
    if k < nvars:
        e, c = zr.reconstruct(w.p, w.deg, _box(zr, w.hidden), sched=w.schedule, first_stage=k, start=start,
                              last_stage=k)
        oe, oc = oracle.zippel(w.p, w.deg, w.schedule, box, last_stage=k)
        assert np.array_equal(e, oe) and np.array_equal(c, oc)


def test_resume_rejects_bad_start(zr):
    w = synth.config_workload(1)
    box = _box(zr, w.hidden)
    e, c = oracle.zippel(w.p, w.deg, w.schedule, synth.BlackBox(w.hidden), last_stage=1)
    bad = []
    e2 = e.copy()
    e2[0, 1] = 1  # an exponent of a variable not reached yet
    bad.append((2, (e2, c)))
    bad.append((2, (e[::-1].copy(), c[::-1].copy())))  # not ascending
    c2 = c.copy()
    c2[0] = w.p  # coefficient out of range
    bad.append((2, (e, c2)))
    e3 = e.copy()
    e3[-1, 0] = w.deg[0] + 1  # beyond the degree bound
    bad.append((2, (e3, c)))
    bad.append((5, (e, c)))  # beyond the last stage
    for k, st in bad:
        with pytest.raises(zr.ZippelError) as ei:
            zr.reconstruct(w.p, w.deg, box, sched=w.schedule, first_stage=k, start=st)
        assert ei.value.code == zr.ZR_EINVAL
    # an empty start skeleton is a valid (zero) polynomial at stage 1
    z = (np.zeros((0, 3), np.uint16), np.zeros(0, np.uint64))
    e, c = zr.reconstruct(w.p, w.deg, box, sched=w.schedule, first_stage=2, start=z, nprobes=0)
    assert len(c) == 0
