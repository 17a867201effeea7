"""NEAT's structural genes on the GPU (System Design: NEAT's mutation and
crossover operators, over the bounded superset of the CPPN): networks of
genomes with direct connections and added nodes against the oracle,
structural mutation in radiation and crossover in merging bit-exact in
their integer decisions, the compatibility distance with excess and
disjoint genes, and a step of such genomes against the oracle step."""
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
    print(f"[structure] {msg}", flush=True)


def rand_ext32(rng, n, p_on=0.5):
    from paper_2406_09654_amd.binding import GENOME_EXT_DTYPE
    e = np.zeros(n, GENOME_EXT_DTYPE)
    for k in range(n):
        e[k]["conn_mask"] = sum(1 << c for c in range(10) if rng.random() < p_on)
        e[k]["node_mask"] = sum(1 << q for q in range(16) if rng.random() < p_on)
        e[k]["node_act"] = int(rng.integers(0, 1 << 32, dtype=np.uint64))
        e[k]["conn_w"] = rng.standard_normal(10)
        e[k]["node_in"] = rng.standard_normal(16)
        e[k]["node_out"] = rng.standard_normal(16)
    return e


def to_oracle(e32):
    """float32 records -> the oracle's FP64 records (exact widening)."""
    x = oracle.empty_ext(len(e32))
    for f in ("conn_mask", "node_mask", "node_act", "conn_w", "node_in", "node_out"):
        x[f] = e32[f]
    return x


def live_ext(w, cap):
    """Every slot's structural genes, as oracle records."""
    return to_oracle(w.genome_ext(np.arange(cap, dtype=np.int32)))


@pytest.mark.parametrize("layers,hidden,prec", [(2, 32, 0), (3, 64, 0), (3, 64, 1)])
def test_structural_networks_match_oracle(stream, layers, hidden, prec):
    say(f"networks {layers} {hidden} prec {prec}")
    rng = np.random.default_rng(61)
    ng = 8
    init = gh.heterogeneous_world(16, 16, n_genomes=ng, layers=layers, hidden=hidden, precision=prec, seed=5)
    w = gh.make_world(init, stream)
    ext = rand_ext32(rng, ng)
    ext[0]["conn_mask"] = ext[0]["node_mask"] = 0   # slot 0 stays the base CPPN
    slots = np.arange(ng, dtype=np.int32)
    w.set_genome_ext(slots, ext)
    back = w.genome_ext(slots)
    assert back.tobytes() == ext.tobytes()           # round trip, bit for bit
    d = gh.oracle_desc(init.spec)
    X = to_oracle(ext)
    tol = 1e-5 if prec == 0 else 4e-3
    for s in range(ng):
        ref = oracle.cppn_to_net_x(d, init.params[s].astype(np.float64), X[s])
        got = w.debug_get_weights(int(s), ref.size)
        assert gh.normwise(got, ref) <= tol, (s, gh.normwise(got, ref))
    # set_genomes clears the structure
    w.set_genomes(slots[:2], init.params[:2])
    assert (w.genome_ext(slots[:2])["node_mask"] == 0).all() and (w.genome_ext(slots[:2])["conn_mask"] == 0).all()
    w.close()


def test_structural_radiation_matches_oracle(stream):
    say("radiation")
    rng = np.random.default_rng(62)
    ng, cap = 30, 1024
    init = gh.heterogeneous_world(200, 150, n_genomes=ng, capacity=cap, seed=23)
    w = gh.make_world(init, stream)
    w.set_genome_ext(np.arange(ng, dtype=np.int32), rand_ext32(rng, ng, 0.3))
    w.set_structural_mutation(0.5, 0.5)
    d = gh.oracle_desc(init.spec)
    for s in (1, 2):
        w.step(1)
        before = w.get_state()["G"]
        P = np.zeros((cap, 56))
        live = np.unique(before)
        P[live] = w.get_genomes(live).astype(np.float64)
        X = live_ext(w, cap)
        st = w.radiate(2e-3, 0.1, s)
        G2, P2, X2, (hc, hs), dropped = oracle.radiate_x(before, cap, P, X, init.spec.seed, s, 2e-3, 0.1, 0.5, 0.5)
        np.testing.assert_array_equal(w.get_state()["G"], G2)
        new = hs[hs >= 0]
        assert st["hits"] == len(hc) and len(new) > 30 and dropped == 0
        np.testing.assert_allclose(w.get_genomes(new), P2[new], rtol=0, atol=2e-6)
        got = live_ext(w, cap)[new]
        for f in ("conn_mask", "node_mask", "node_act"):
            np.testing.assert_array_equal(got[f], X2[new][f])
        for f in ("conn_w", "node_in", "node_out"):
            np.testing.assert_allclose(got[f], X2[new][f], rtol=0, atol=2e-6)
        parents = before.ravel()[hc[hs >= 0]]
        grown = (got["conn_mask"] != X[parents]["conn_mask"]) | (got["node_mask"] != X[parents]["node_mask"])
        assert grown.sum() > 5                                     # structural mutations happened
        for sl in new[:6]:
            ref = oracle.cppn_to_net_x(d, P2[sl], X2[sl])
            assert gh.normwise(w.debug_get_weights(int(sl), ref.size), ref) <= 1e-5
    w.close()


def test_structural_merge_and_step_match_oracle(stream):
    say("merge + step")
    rng = np.random.default_rng(63)
    ng, cap = 24, 512
    init = gh.heterogeneous_world(160, 120, n_genomes=ng, capacity=cap, seed=29)
    w = gh.make_world(init, stream)
    w.set_genome_ext(np.arange(ng, dtype=np.int32), rand_ext32(rng, ng, 0.5))
    w.step(1)
    st0 = w.get_state()
    live = np.unique(st0["G"])
    P = np.zeros((cap, 56))
    P[live] = w.get_genomes(live).astype(np.float64)
    X = live_ext(w, cap)
    d = gh.oracle_desc(init.spec)
    G2, P2, X2, (hc, hs, ha, hb), dropped = oracle.merge_x(d, st0["G"], st0["R"], cap, P, X, init.spec.seed, 1, 0.01)
    w.merge(0.01, 1)
    merged = w.get_state()
    np.testing.assert_array_equal(merged["G"], G2)
    new = hs[hs >= 0]
    assert len(new) > 50
    got = live_ext(w, cap)[new]
    for f in ("conn_mask", "node_mask", "node_act", "conn_w", "node_in", "node_out"):
        np.testing.assert_array_equal(got[f], X2[new][f])          # copies: exact
    # the step of the merged state against the oracle's, with every genome's structure
    slots = np.unique(G2).astype(np.int32)
    lut = np.full(cap, -1, np.int64)
    lut[slots] = np.arange(slots.size)
    nets = oracle.nets_for_x(d, P2[slots], X2[slots])
    s2 = oracle.State(merged["E"], merged["I"], merged["C"], lut[merged["G"]].astype(np.int32), merged["R"])
    ref, info = oracle.step(d, s2, nets, want_margins=True)
    ref.G = slots[ref.G].astype(np.int32)
    w.step(1)
    gh.compare_step(w.get_state(), ref, info["margins"], max_band_frac=1e-2)
    w.close()


def test_structural_genetic_distance_matches_oracle(stream):
    say("distance")
    rng = np.random.default_rng(64)
    ng = 40
    init = gh.heterogeneous_world(32, 32, n_genomes=ng, capacity=64, seed=4)
    w = gh.make_world(init, stream)
    ext = rand_ext32(rng, ng, 0.4)
    ext[:5]["conn_mask"] = 0
    ext[:5]["node_mask"] = 0
    slots = np.arange(ng, dtype=np.int32)
    w.set_genome_ext(slots, ext)
    X = to_oracle(ext)
    P = init.params.astype(np.float64)
    for c1, c2, c3 in [(1.0, 1.0, 0.4), (2.0, 0.5, 1.0)]:
        got = w.genetic_distance(slots, slots, c3, c1, c2)
        ref = np.array([[oracle.genetic_distance_x(P[a], X[a], P[b], X[b], c1, c2, c3) for b in range(ng)]
                        for a in range(ng)])
        np.testing.assert_allclose(got, ref, rtol=2e-6, atol=1e-6)
    w.close()
