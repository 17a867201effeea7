"""Merging on the GPU (Abstract: survival, merging and mutation; System
Design: NEAT's crossover operator applied through the physics): the merges'
cells, parents, slots and the children's parameters bit for bit against the
oracle, the regenerated networks, the births and lineage, capacity
exhaustion, the degenerate rates, and steps after merging against the
oracle step."""
import numpy as np
import pytest

import oracle
from tests import gpu_helpers as gh

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def stream():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch.cuda.Stream()


def say(msg):
    print(f"[merge] {msg}", flush=True)


def _oracle_merge(w, init, cap, rate, step_index):
    st = w.get_state()
    live = np.unique(st["G"])
    P = np.zeros((cap, 56))
    P[live] = w.get_genomes(live).astype(np.float64)
    d = gh.oracle_desc(init.spec)
    return st, P, oracle.merge(d, st["G"], st["R"], cap, P, init.spec.seed, step_index, rate)


@pytest.mark.parametrize("layers,hidden,prec", [(2, 32, 0), (3, 64, 0), (3, 64, 1)])
def test_merge_matches_oracle(stream, layers, hidden, prec):
    say(f"merge {layers} {hidden} prec {prec}")
    ng, cap = 40, 2048
    init = gh.heterogeneous_world(300, 200, n_genomes=ng, capacity=cap, layers=layers,
                                  hidden=hidden, precision=prec, seed=31)
    w = gh.make_world(init, stream)
    d = gh.oracle_desc(init.spec)
    rate = 3e-3
    for s in range(1, 4):
        w.step(1)
        before, P, (G2, P2, (hc, hs, ha, hb), dropped) = _oracle_merge(w, init, cap, rate, s)
        st = w.merge(rate, s)
        out = w.get_state()
        np.testing.assert_array_equal(out["G"], G2)             # merge set and slots: exact
        for ch in ("E", "I", "C", "R"):
            np.testing.assert_array_equal(out[ch], before[ch])   # only the genome map changes
        assert st["hits"] == len(hc) > 50 and st["dropped_hits"] == dropped == 0
        new = hs[hs >= 0]
        np.testing.assert_array_equal(w.get_genomes(new).astype(np.float64), P2[new])  # copies: exact
        cells, a, b, slots = w.births()
        np.testing.assert_array_equal(cells, hc)
        np.testing.assert_array_equal(a, ha)
        np.testing.assert_array_equal(b, hb)
        np.testing.assert_array_equal(slots, hs)
        lp, lp2, lb = w.lineage(new)
        np.testing.assert_array_equal(lp, ha)
        np.testing.assert_array_equal(lp2, hb)
        assert (lb == s).all()
        tol = 1e-5 if prec == 0 else 4e-3
        for sl in new[:6]:
            ref = oracle.cppn_to_net(d, P2[sl])
            assert gh.normwise(w.debug_get_weights(int(sl), ref.size), ref) <= tol
    w.close()


def test_step_after_merging_matches_oracle(stream):
    """The children's networks drive the next step: the step after a merge
    matches the oracle's step of the merged state (FP32, near-tie band)."""
    say("step after merge")
    ng, cap = 24, 512
    init = gh.heterogeneous_world(160, 120, n_genomes=ng, capacity=cap, seed=8)
    w = gh.make_world(init, stream)
    w.step(2)
    before, P, (G2, P2, (hc, hs, ha, hb), dropped) = _oracle_merge(w, init, cap, 0.01, 2)
    w.merge(0.01, 2)
    assert len(hs) > 100 and dropped == 0
    merged = w.get_state()
    np.testing.assert_array_equal(merged["G"], G2)
    d = gh.oracle_desc(init.spec)
    slots = np.unique(G2).astype(np.int32)
    st = gh.oracle_state_from(merged)
    ref, info = gh.oracle_step_slots(d, st, slots, P2[slots], want_margins=True)
    w.step(1)
    gh.compare_step(w.get_state(), ref, info["margins"], max_band_frac=1e-2)
    w.close()


def test_merge_capacity_exhaustion_and_degenerate_rates(stream):
    say("merge capacity")
    W, H, cap = 120, 100, 16
    init = gh.heterogeneous_world(W, H, n_genomes=10, capacity=cap, seed=5)
    w = gh.make_world(init, stream)
    st0 = w.merge(0.0, 1)                                   # rate 0: nothing happens
    assert st0["hits"] == 0
    np.testing.assert_array_equal(w.get_state()["G"], init.G)
    assert len(w.births()[0]) == 0
    before, P, (G2, P2, (hc, hs, ha, hb), dropped) = _oracle_merge(w, init, cap, 0.02, 3)
    st = w.merge(0.02, 3)
    np.testing.assert_array_equal(w.get_state()["G"], G2)
    assert st["dropped_hits"] == dropped > 0 and st["hits"] == len(hc)
    new = hs[hs >= 0]
    assert len(new) == cap - 10
    np.testing.assert_array_equal(w.get_genomes(new).astype(np.float64), P2[new])
    w.close()
    # a world of one genome never merges, at any rate
    init1 = gh.heterogeneous_world(64, 48, n_genomes=1, capacity=8, seed=6)
    w1 = gh.make_world(init1, stream)
    st1 = w1.merge(1.0, 5)
    assert st1["hits"] == 0
    np.testing.assert_array_equal(w1.get_state()["G"], init1.G)
    w1.close()


def test_merge_rate_one_and_set_genomes_clears_births(stream):
    """Rate 1: every cell facing another genome merges (free slots permitting);
    coralai_set_genomes leaves no births to report."""
    say("merge rate 1")
    W, H, ng = 50, 40, 6
    cap = W * H + ng
    init = gh.heterogeneous_world(W, H, n_genomes=ng, capacity=cap, seed=12)
    w = gh.make_world(init, stream)
    before, P, (G2, P2, (hc, hs, ha, hb), dropped) = _oracle_merge(w, init, cap, 1.0, 0)
    st = w.merge(1.0, 0)
    np.testing.assert_array_equal(w.get_state()["G"], G2)
    assert st["hits"] == len(hc) > 1000 and dropped == 0
    assert len(w.births()[0]) == len(hc)
    w.set_genomes(np.array([0], np.int32), init.params[:1])
    assert len(w.births()[0]) == 0
    w.close()
