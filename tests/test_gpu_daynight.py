"""The day / night energy cycle on the GPU (Experiment: energy is added to and
removed from the substrate in a day / night cycle): single steps at every
phase against the oracle, the exact energy ledger over many steps (checked
on the device by the step itself and here on the host), every physics
tiling, and batched worlds with different cycles."""
import sys

import numpy as np
import pytest

import oracle
from tests import gpu_helpers as gh

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

PERIOD, NOON, NIGHT = 8, 3_000_017, 40_000


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def stream():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch.cuda.Stream()


@pytest.mark.parametrize("W,H,layers,hidden", [(130, 70, 2, 32), (64, 64, 3, 64)])
def test_day_night_steps_match_oracle(stream, W, H, layers, hidden):
    init = gh.heterogeneous_world(W, H, n_genomes=6, layers=layers, hidden=hidden, seed=W + 7 * H)
    w = gh.make_world(init, stream)
    w.set_daylight(PERIOD, NOON, NIGHT)
    d = gh.oracle_desc(init.spec)
    d.day_period, d.day_inject, d.night_num = PERIOD, NOON, NIGHT
    nets = oracle.nets_for(d, init.params)
    prev_mass = None
    for k in range(PERIOD + 1):   # noon through the night to the next noon
        st_in = w.get_state()
        st = w.step(1, stats=True)
        led = w.energy_ledger()
        out = w.get_state()
        d.cycle_step = k
        ref, info = oracle.step(d, gh.oracle_state_from(st_in), nets, want_margins=True)
        rep = gh.compare_step(out, ref, info["margins"], max_band_frac=1e-2)
        assert st["error_word"] == 0
        assert led["injected_last"] == info["injected"]          # independent of E1: exact
        assert abs(led["removed_last"] - info["removed"]) <= 1e-5 * max(1, info["removed"]) + 16
        m_in = int(st_in["E"].sum() + st_in["I"].sum())
        assert st["mass_quanta"] == m_in + led["injected_last"] - led["removed_last"]
        assert st["mass_quanta"] == int(out["E"].sum() + out["I"].sum())
        if prev_mass is not None:
            assert m_in == prev_mass
        prev_mass = st["mass_quanta"]
        say("  phase", k, "injected", led["injected_last"], "removed", led["removed_last"], rep)
    w.close()


@pytest.mark.parametrize("prec", [0, 1])
def test_day_night_ledger_over_many_steps(stream, prec):
    """30 steps over three periods of 10: each step's total mass equals the
    previous plus the injected minus the removed quanta (the device checks it
    too: no error bit), the running totals add up, energy stays non-negative,
    and every physics tiling steps to identical states."""
    init = gh.heterogeneous_world(96, 80, n_genomes=5, layers=2, hidden=32, seed=9, precision=prec)
    outs = []
    for tile in (0, 1, 2, 3):
        w = gh.make_world(init, stream)
        w.set_tuning(2, 0, tile)
        w.set_daylight(10, 1_500_000, 65_536)
        m = int(init.E.sum() + init.I.sum())
        inj = rem = 0
        for _ in range(30):
            st = w.step(1, stats=True)
            led = w.energy_ledger()
            assert st["error_word"] == 0
            assert st["mass_quanta"] == m + led["injected_last"] - led["removed_last"]
            assert st["mass_fp64"] == float(st["mass_quanta"])
            m = st["mass_quanta"]
            inj += led["injected_last"]
            rem += led["removed_last"]
        assert (led["injected_total"], led["removed_total"]) == (inj, rem)
        assert inj > 0 and rem > 0
        out = w.get_state()
        assert (out["E"] >= 0).all() and int(out["E"].sum() + out["I"].sum()) == m
        outs.append(out)
        w.close()
    for o in outs[1:]:
        for ch in ("E", "I", "C", "G", "R"):
            np.testing.assert_array_equal(o[ch], outs[0][ch])


def test_day_night_batched_worlds_equal_alone(stream):
    from paper_2406_09654_amd.world import Batch
    cycles = [(0, 0, 0), (6, 2_000_000, 30_000), (11, 500_000, 65_536)]
    inits = [gh.heterogeneous_world(s, s + 9, n_genomes=4, seed=50 + k) for k, s in enumerate([40, 77, 64])]
    alone = []
    for init, cyc in zip(inits, cycles):
        w = gh.make_world(init, stream)
        w.set_daylight(*cyc)
        w.step(7)
        alone.append((w.get_state(), w.energy_ledger()))
        w.close()
    worlds = [gh.make_world(init, stream) for init in inits]
    for w, cyc in zip(worlds, cycles):
        w.set_daylight(*cyc)
    b = Batch(4, stream)
    b.set_worlds(worlds)
    b.step(7)
    b.sync()
    for k, w in enumerate(worlds):
        out = w.get_state()
        for ch in ("E", "I", "C", "G", "R"):
            np.testing.assert_array_equal(out[ch], alone[k][0][ch])
        assert w.energy_ledger() == alone[k][1]
        assert w.stats()["error_word"] == 0
    b.close()
    for w in worlds:
        w.close()


def test_day_night_rejects_bad_arguments(stream):
    from paper_2406_09654_amd.binding import CoralaiError
    init = gh.heterogeneous_world(8, 8, n_genomes=2, seed=1)
    w = gh.make_world(init, stream)
    for args in [(1, 10, 10), (-3, 10, 10), (8, -1, 10), (8, 1 << 40, 10), (8, 10, 65537)]:
        with pytest.raises(CoralaiError):
            w.set_daylight(*args)
    w.close()
