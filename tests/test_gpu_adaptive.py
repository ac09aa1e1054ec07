"""Reconstruction without degree bounds (zippel_reconstruct_adaptive) on the
GPU against the oracle's early-terminating reconstruction on the same
schedule: the same polynomial (the hidden one), the same degree found for
every variable (its true degree), caps far above the degrees, one or two
confirming orders, and a cap below a degree failing with EPROBE."""
import sys

import numpy as np
import pytest

import synth
from oracle import adaptive as oad

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


@pytest.mark.parametrize("nvars,deg,t,cap,confirm", [(3, [5, 8, 3], 60, 12, 1), (3, [5, 8, 3], 60, 12, 2),
                                                     (4, 7, 500, 30, 1), (5, [12, 3, 9, 1, 12], 3000, 40, 2)])
def test_adaptive_matches_oracle(zr, nvars, deg, t, cap, confirm):
    p = synth.make_prime()
    h = synth.random_poly(p, nvars, deg, t, 500 + t + confirm)
    true = [int(h.exps[:, v].max()) for v in range(nvars)]
    caps = [cap] * nvars
    sched = synth.make_schedule(p, nvars, [c + confirm for c in caps], 1500 + t, 2)
    _note(f"adaptive n={nvars} t={t} cap={cap} confirm={confirm}")
    e, c, found = zr.reconstruct_adaptive(p, caps, zr.HostBlackBox(synth.BlackBox(h).eval, nvars), sched=sched,
                                          confirm=confirm)
    assert np.array_equal(e, h.exps) and np.array_equal(c, h.coefs)
    assert found == true
    if t <= 500:
        oe, oc, ofound = oad.adaptive_zippel(p, caps, sched, synth.BlackBox(h), confirm=confirm)
        assert np.array_equal(e, oe) and np.array_equal(c, oc) and found == ofound


def test_adaptive_cap_below_degree(zr):
    p = synth.make_prime()
    h = synth.random_poly(p, 2, [6, 4], 20, 45)
    caps = [int(h.exps[:, 0].max()) - 1, 10]
    sched = synth.make_schedule(p, 2, [c + 1 for c in caps], 1045, 0)
    with pytest.raises(zr.ZippelError) as ei:
        zr.reconstruct_adaptive(p, caps, zr.HostBlackBox(synth.BlackBox(h).eval, 2), sched=sched, confirm=1)
    assert ei.value.code == zr.ZR_EPROBE


def test_adaptive_seeded_schedule_equals_fixed_bounds(zr):
    """With the true degrees found, the result equals the fixed-bound path on
    a schedule whose node lists start with the same nodes."""
    p = synth.make_prime()
    h = synth.random_poly(p, 4, 9, 800, 46)
    sched = synth.make_schedule(p, 4, [21] * 4, 1046, 2)
    e, c, found = zr.reconstruct_adaptive(p, [20] * 4, zr.HostBlackBox(synth.BlackBox(h).eval, 4), sched=sched)
    fe, fc = zr.reconstruct(p, found, zr.HostBlackBox(synth.BlackBox(h).eval, 4), sched=sched)
    assert np.array_equal(e, fe) and np.array_equal(c, fc)
