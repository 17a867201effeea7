"""Phylogeny and genetic similarity on the GPU (Discussion: NEAT's measure of
genetic similarity; phylogeny tracking): every radiation call's births and
every slot's lineage against the oracle's radiation over several steps, and
the NEAT compatibility distance matrix against the oracle."""
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


def test_births_and_lineage_match_oracle_radiation(stream):
    ng, cap = 40, 2048
    init = gh.heterogeneous_world(300, 200, n_genomes=ng, capacity=cap, seed=19)
    w = gh.make_world(init, stream)
    parents, parents2, births = w.lineage(np.arange(ng))
    assert (parents == -1).all() and (parents2 == -1).all() and (births == 0).all()
    rate, sigma = 2e-3, 0.1
    edges = {}
    for s in range(1, 6):
        w.step(1)
        before = w.get_state()["G"]
        P = np.zeros((cap, 56))
        live = np.unique(before)
        P[live] = w.get_genomes(live).astype(np.float64)
        st = w.radiate(rate, sigma, s)
        G2, P2, hits, dropped = oracle.radiate(before, cap, P, init.spec.seed, s, rate, sigma)
        cells, par, slots = oracle.births(before, hits)
        gc, gp, gp2, gs = w.births()
        np.testing.assert_array_equal(gc, cells)
        np.testing.assert_array_equal(gp, par)
        np.testing.assert_array_equal(gs, slots)
        assert (gp2 == -1).all()                    # a mutation has one parent
        assert st["hits"] - st["dropped_hits"] == len(cells) > 50
        lp, lp2, lb = w.lineage(gs)
        np.testing.assert_array_equal(lp, par)
        assert (lp2 == -1).all()
        assert (lb == s).all()
        for c, p, sl in zip(gc, gp, gs):
            edges[int(sl)] = (int(p), s)
    # slots freed by takeovers are reused: the lineage holds their latest genome
    lp, _, lb = w.lineage(np.array(sorted(edges), np.int32))
    assert [(int(p), int(b)) for p, b in zip(lp, lb)] == [edges[k] for k in sorted(edges)]
    w.close()


@pytest.mark.parametrize("c3", [1.0, 0.4])
def test_genetic_distance_matrix_matches_oracle(stream, c3):
    ng = 70
    init = gh.heterogeneous_world(32, 32, n_genomes=ng, capacity=128, seed=4)
    w = gh.make_world(init, stream)
    w.radiate(0.05, 0.1, 1)                      # children at distance ~0.08 from their parents
    slots = np.unique(w.get_state()["G"]).astype(np.int32)
    a, b = slots[: len(slots) // 2], slots
    got = w.genetic_distance(a, b, c3)
    pa = w.get_genomes(a).astype(np.float64)
    pb = w.get_genomes(b).astype(np.float64)
    ref = np.array([[oracle.genetic_distance(x, y, c3) for y in pb] for x in pa])
    np.testing.assert_allclose(got, ref, rtol=2e-6, atol=1e-7)
    sq = w.genetic_distance(slots, slots, c3)
    np.testing.assert_array_equal(sq, sq.T)       # |a - b| = |b - a| summed in one order
    assert (np.diag(sq) == 0).all()
    w.close()
