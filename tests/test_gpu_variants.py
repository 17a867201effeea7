"""Physics variants on the GPU: hard-max exploration (the whole exploration
budget to the maximal explore actuator) and energy transport along the flow
directions, alone and together, with and without the day / night cycle,
against the oracle, over every physics tiling, and in a batch."""
import sys

import numpy as np
import pytest

import oracle
from tests import gpu_helpers as gh

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def stream():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch.cuda.Stream()


VARIANTS = [(1, 0.0), (0, 0.3), (1, 0.25)]


def make(init, stream, hard, kappa_e, precision=None):
    from paper_2406_09654_amd.binding import WORLD_ENERGY_FLOWS
    from paper_2406_09654_amd.world import World
    w = World.from_init(init, stream=stream, precision=precision, flags=WORLD_ENERGY_FLOWS)
    w.set_physics_variant(hard, kappa_e)
    return w


@pytest.mark.parametrize("hard,kappa_e", VARIANTS)
@pytest.mark.parametrize("W,H,layers,hidden", [(37, 23, 2, 32), (130, 70, 2, 32), (64, 64, 3, 64)])
def test_variant_steps_match_oracle(stream, hard, kappa_e, W, H, layers, hidden):
    init = gh.heterogeneous_world(W, H, n_genomes=6, layers=layers, hidden=hidden, seed=3 * W + H)
    d = gh.oracle_desc(init.spec)
    d.explore_mode, d.kappa_energy = hard, float(np.float32(kappa_e))
    nets = oracle.nets_for(d, init.params)
    w = make(init, stream, hard, kappa_e)
    m0 = int(init.E.sum() + init.I.sum())
    for k in range(3):
        st_in = w.get_state()
        st = w.step(1, stats=True)
        out = w.get_state()
        ref, info = oracle.step(d, gh.oracle_state_from(st_in), nets, want_margins=True)
        rep = gh.compare_step(out, ref, info["margins"], max_band_frac=1e-2,
                              ledger_outside_band=bool(hard))
        assert st["error_word"] == 0 and st["mass_quanta"] == m0
        assert int(out["E"].sum() + out["I"].sum()) == m0
        say("  step", k, "hard", hard, "kappa_e", kappa_e, rep)
    if kappa_e > 0:
        assert not np.array_equal(w.get_state()["E"], init.E)
    w.close()


@pytest.mark.parametrize("prec", [0, 1])
def test_variants_identical_over_tilings_with_cycle(stream, prec):
    """Hard max with energy transport and the day / night cycle: the four
    physics tilings and the graph / direct paths give identical states, and
    the mass ledger is exact."""
    init = gh.heterogeneous_world(96, 52, n_genomes=5, seed=8, precision=prec)
    outs = []
    for tile, strm in [(0, stream), (1, None), (2, stream), (3, stream), (3, None)]:
        w = make(init, strm, 1, 0.2)
        w.set_tuning(2, 0, tile)
        w.set_daylight(6, 700_000, 30_000)
        m = int(init.E.sum() + init.I.sum())
        for _ in range(8):
            st = w.step(1, stats=True)
            led = w.energy_ledger()
            assert st["error_word"] == 0
            assert st["mass_quanta"] == m + led["injected_last"] - led["removed_last"]
            m = st["mass_quanta"]
        outs.append(w.get_state())
        w.close()
    for o in outs[1:]:
        for ch in ("E", "I", "C", "G", "R"):
            np.testing.assert_array_equal(o[ch], outs[0][ch])


def test_variant_batch_equals_alone(stream):
    from paper_2406_09654_amd.world import Batch
    inits = [gh.heterogeneous_world(s, s + 5, n_genomes=4, seed=90 + k) for k, s in enumerate([48, 70, 33])]
    alone = []
    for init, (hard, ke) in zip(inits, VARIANTS):
        w = make(init, stream, hard, ke)
        w.step(5)
        alone.append(w.get_state())
        w.close()
    worlds = [make(init, stream, hard, ke) for init, (hard, ke) in zip(inits, VARIANTS)]
    b = Batch(4, stream)
    b.set_worlds(worlds)
    b.step(5)
    b.sync()
    for k, w in enumerate(worlds):
        out = w.get_state()
        for ch in ("E", "I", "C", "G", "R"):
            np.testing.assert_array_equal(out[ch], alone[k][ch])
    b.close()
    for w in worlds:
        w.close()


def test_variant_argument_checks(stream):
    from paper_2406_09654_amd.binding import CoralaiError
    init = gh.heterogeneous_world(8, 8, n_genomes=2, seed=1)
    w = gh.make_world(init, stream)                 # no energy flow records
    with pytest.raises(CoralaiError):
        w.set_physics_variant(0, 0.5)
    w.set_physics_variant(1, 0.0)                   # hard max needs nothing extra
    for args in [(2, 0.0), (-1, 0.0)]:
        with pytest.raises(CoralaiError):
            w.set_physics_variant(*args)
    w.close()
    w = make(init, stream, 0, 0.5)
    with pytest.raises(CoralaiError):               # debug_physics is infrastructure-only
        w.debug_physics(np.zeros(64, np.int64), np.zeros((64, 8), np.uint32), np.zeros(64, np.uint8))
    for bad in (-0.1, 1.5):
        with pytest.raises(CoralaiError):
            w.set_physics_variant(0, bad)
    w.close()
