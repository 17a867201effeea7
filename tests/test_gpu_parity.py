"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle on
the same seeded inputs.  Sizes span several tiles and ragged tails; the
full-size workloads are checked on row bands the oracle computes exactly."""
import sys

import numpy as np
import pytest

import oracle
import workloads as wl
from tests import gpu_helpers as gh

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def stream():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2406_09654_amd as P
    P.lib()
    return torch.cuda.Stream()


# ------------------------------------------------------------------ pieces

@pytest.mark.parametrize("layers,hidden,prec", [(2, 32, 0), (3, 64, 0), (2, 64, 1), (3, 32, 1)])
def test_cppn_weights_match_oracle(stream, layers, hidden, prec):
    say("cppn", layers, hidden, prec)
    init = gh.heterogeneous_world(8, 8, n_genomes=5, layers=layers, hidden=hidden, precision=prec,
                                  seed=3, scale=1.0)
    w = gh.make_world(init, stream)
    d = gh.oracle_desc(init.spec)
    size = oracle.net_size(d)
    for s in range(5):
        got = w.debug_get_weights(s, size)
        ref = oracle.cppn_to_net(d, init.params[s].astype(np.float64))
        tol = 1e-6 if prec == 0 else 4e-3   # fp32: FP64 CPPN rounded once; bf16: 2^-9 relative
        assert gh.normwise(got, ref) <= tol, (s, gh.normwise(got, ref))
    w.close()


@pytest.mark.parametrize("layers,scale", [(2, 1.0), (3, 1.0), (3, 4.0)])
def test_fp32_cppn_weights_within_two_roundings(stream, layers, scale):
    """FP32 networks: each weight is the FP64 CPPN value rounded to FP32 when
    stored and again when the debug hook divides out the stored scale factor
    (not a power of 2 for most rows), so each element is within two FP32
    roundings of the oracle's FP64 value.  A parameter scale of 4 takes the
    sin arguments over many quadrants, the gaussians to underflow and the
    tanh nodes into saturation."""
    say("cppn fp32 elementwise", layers, scale)
    init = gh.heterogeneous_world(8, 8, n_genomes=6, layers=layers, hidden=64, precision=0, seed=11,
                                  scale=scale)
    w = gh.make_world(init, stream)
    d = gh.oracle_desc(init.spec)
    size = oracle.net_size(d)
    for s in range(6):
        got = w.debug_get_weights(s, size).astype(np.float64)
        ref = oracle.cppn_to_net(d, init.params[s].astype(np.float64))
        bound = 2.0 ** -22 * np.abs(ref) + 1e-12 * np.abs(ref).max()
        bad = np.flatnonzero(np.abs(got - ref) > bound)
        assert bad.size == 0, (s, bad[:5], got[bad[:5]], ref[bad[:5]])
    w.close()


def _tanh_part_max(params, layers):
    """Largest |column part| or |row part| of the tanh nodes (k = 2, 6) over
    the layers: a_k x1 + b_k y_l + d_k y_l+1 + e_k and c_k x2, |x| <= 1."""
    p = params.astype(np.float64).reshape(len(params), 56)
    m = 0.0
    for k in (2, 6):
        a, b, c, d, e = (p[:, 5 * k + j] for j in range(5))
        for l in range(layers):
            y0, y1 = -1 + 2 * l / layers, -1 + 2 * (l + 1) / layers
            m = max(m, float(np.max(np.abs(a) + np.abs(b * y0 + d * y1 + e))), float(np.max(np.abs(c))))
    return m


@pytest.mark.parametrize("prec,scale,limit", [(1, 16.0, 40.0), (0, 160.0, 300.0)])
def test_cppn_weights_large_parameters(stream, prec, scale, limit):
    """Parameters large enough that some tanh node's column or row part
    leaves the range of the tabulated exponentials (40 in FP32, 300 in FP64):
    those genomes evaluate tanh of the sum directly, and still match the
    oracle (BF16 normwise, FP32 within two roundings per element)."""
    say("cppn large parameters", prec, scale)
    init = gh.heterogeneous_world(8, 8, n_genomes=6, layers=3, hidden=64, precision=prec, seed=23, scale=scale)
    assert _tanh_part_max(init.params, 3) > limit
    w = gh.make_world(init, stream)
    d = gh.oracle_desc(init.spec)
    size = oracle.net_size(d)
    for s in range(6):
        got = w.debug_get_weights(s, size).astype(np.float64)
        ref = oracle.cppn_to_net(d, init.params[s].astype(np.float64))
        if prec == 1:
            assert gh.normwise(got, ref) <= 4e-3, (s, gh.normwise(got, ref))
        else:
            bound = 2.0 ** -22 * np.abs(ref) + 1e-12 * np.abs(ref).max()
            bad = np.flatnonzero(np.abs(got - ref) > bound)
            assert bad.size == 0, (s, bad[:5], got[bad[:5]], ref[bad[:5]])
    w.close()


@pytest.mark.parametrize("prec", [0, 1])
def test_debug_weights_roundtrip(stream, prec):
    """Flat weights in, flat weights out: exact up to the one rounding of the
    stored value (hidden layers are stored times 2 log2 e)."""
    init = gh.heterogeneous_world(4, 4, n_genomes=2, layers=3, hidden=64, seed=1, precision=prec)
    w = gh.make_world(init, stream)
    d = gh.oracle_desc(init.spec)
    flat = np.random.default_rng(0).standard_normal(oracle.net_size(d)).astype(np.float32)
    w.debug_set_weights(1, flat)
    got = w.debug_get_weights(1, flat.size)
    rtol = 2.5e-7 if prec == 0 else 2 ** -8
    np.testing.assert_allclose(got, flat, rtol=rtol, atol=0)
    w.close()


@pytest.mark.parametrize("W,H,ng,cap", [(1, 1, 1, 1), (37, 23, 5, 9), (64, 64, 16, 16),
                                        (300, 200, 70, 128),
                                        # ~1 750 genomes per 64 x 64 tile: the scatter's
                                        # table fills and most runs take the cursor path
                                        (256, 130, 2000, 2048),
                                        # more than 1024 slot blocks of 512: the scan's
                                        # three-pass form
                                        (64, 64, 16, 600_000)])
def test_buckets_match_numpy(stream, W, H, ng, cap):
    say("buckets", W, H)
    init = gh.heterogeneous_world(W, H, n_genomes=ng, capacity=cap, seed=W)
    w = gh.make_world(init, stream)
    counts, offsets, perm = w.debug_buckets()
    G = init.G.ravel()
    ref_c = np.bincount(G, minlength=cap)
    np.testing.assert_array_equal(counts, ref_c)
    np.testing.assert_array_equal(offsets, np.concatenate([[0], np.cumsum(ref_c)]))
    # perm: each genome's segment holds exactly its cells (order inside unspecified)
    assert np.array_equal(np.sort(perm), np.arange(W * H))
    np.testing.assert_array_equal(G[perm], np.repeat(np.arange(cap), ref_c))
    w.close()


@pytest.mark.parametrize("W,H,layers,hidden,act_cells", [(37, 23, 2, 32, 1), (64, 64, 2, 32, 2),
                                                         (65, 3, 3, 64, 4), (130, 70, 3, 64, 2),
                                                         (5, 7, 2, 64, 4)])
def test_actuators_match_oracle_fp32(stream, W, H, layers, hidden, act_cells):
    say("act", W, H, layers, hidden, act_cells)
    init = gh.heterogeneous_world(W, H, n_genomes=7, layers=layers, hidden=hidden, seed=W + H)
    w = gh.make_world(init, stream)
    w.set_tuning(act_cells, 0, 0)
    act = w.debug_actuators()
    d = gh.oracle_desc(init.spec)
    s = oracle.State.from_init(init)
    _, info = oracle.step(d, s, oracle.nets_for(d, init.params), want_act=True)
    err = gh.normwise(act, info["act"])
    assert err <= gh.TOL, err
    w.close()


def test_physics_from_oracle_records_is_bit_exact(stream):
    say("physics from records")
    for (W, H, tile) in [(37, 23, 0), (64, 64, 1), (70, 33, 2), (1, 1, 0), (2, 2, 1), (3, 5, 2),
                         (37, 23, 3), (1, 1, 3), (2, 3, 3), (130, 67, 3),
                         # widths divisible by 4 take four cells per thread (row wrap at both ends)
                         (4, 1, 3), (4, 4, 3), (8, 3, 3), (64, 64, 3), (128, 33, 3)]:
        init = gh.heterogeneous_world(W, H, n_genomes=4, seed=W * 7 + H)
        d = gh.oracle_desc(init.spec)
        s = oracle.State.from_init(init)
        _, info = oracle.step(d, s, oracle.nets_for(d, init.params), want_records=True)
        rec = info["records"].ravel()
        I2, G2, R2, tk = oracle.physics_from_records(d, rec["i1"], rec["flow"], rec["explore_dir"],
                                                     init.G, init.R)
        w = gh.make_world(init, stream)
        w.set_tuning(2, 0, tile)
        w.debug_physics(rec["i1"], rec["flow"].astype(np.uint32), rec["explore_dir"].astype(np.uint8))
        out = w.get_state()
        np.testing.assert_array_equal(out["I"], I2)
        np.testing.assert_array_equal(out["G"], G2)
        np.testing.assert_array_equal(out["R"], R2)
        np.testing.assert_array_equal(out["E"], init.E)
        w.close()


# ------------------------------------------------------------------ whole step

STEP_CASES = [(1, 1, 2, 32), (2, 2, 2, 32), (3, 5, 3, 64), (37, 23, 2, 32), (64, 64, 3, 64),
              (130, 70, 2, 32), (257, 65, 3, 64)]


@pytest.mark.parametrize("W,H,layers,hidden", STEP_CASES)
def test_single_step_matches_oracle_fp32(stream, W, H, layers, hidden):
    say("step", W, H, layers, hidden)
    init = gh.heterogeneous_world(W, H, n_genomes=6, layers=layers, hidden=hidden, seed=W * 3 + H)
    w = gh.make_world(init, stream)
    st = w.step(1, stats=True)
    out = w.get_state()
    d = gh.oracle_desc(init.spec)
    ref, info = oracle.step(d, oracle.State.from_init(init), oracle.nets_for(d, init.params),
                            want_margins=True)
    rep = gh.compare_step(out, ref, info["margins"], max_band_frac=1e-2)
    m0 = int(init.E.sum() + init.I.sum())
    assert int(out["E"].sum() + out["I"].sum()) == m0
    assert st["mass_quanta"] == m0 and st["mass_fp64"] == float(m0)
    assert st["error_word"] == 0
    say("  report", rep, "takeovers gpu", st["takeovers"], "oracle", info["takeovers"])
    w.close()


def test_small_genomes_step_matches_oracle_every_tuning(stream):
    """400 genomes drawn per cell on 48x40 (about 5 cells each, some empty),
    as radiation leaves them: nearly every unit starts a run of a new genome
    (prefetched cell indices across runs, weights loaded behind the gather)
    and holds at most 16 cells (one network pass; the other column groups
    are skipped).  Each tuning matches the oracle, and all give identical
    results."""
    say("small genomes")
    init = gh.heterogeneous_world(48, 40, n_genomes=400, capacity=512, layers=3, hidden=64, seed=17)
    d = gh.oracle_desc(init.spec)
    ref, info = oracle.step(d, oracle.State.from_init(init), oracle.nets_for(d, init.params),
                            want_margins=True)
    counts = np.bincount(init.G.ravel(), minlength=512)
    assert counts.max() <= 16 and (counts[:400] == 0).any()
    first = None
    for tuning in [(1, 0, 2), (2, 0, 0), (4, 0, 1), (1, 1, 3), (4, 1, 2)]:
        say("  tuning", tuning)
        w = gh.make_world(init, stream)
        w.set_tuning(*tuning)
        st = w.step(1, stats=True)
        out = w.get_state()
        gh.compare_step(out, ref, info["margins"], max_band_frac=1e-2)
        assert st["error_word"] == 0
        assert int(out["E"].sum() + out["I"].sum()) == int(init.E.sum() + init.I.sum())
        if first is None:
            first = out
        else:
            for k in ("E", "I", "C", "G", "R"):
                np.testing.assert_array_equal(out[k], first[k])
        w.close()


def test_plain_64_trajectory_snapshots(stream):
    """The 64x64 plain-method workload: single steps from GPU states taken
    along a 100-step GPU trajectory (steps 0, 10, 50, 99)."""
    init = wl.config_plain_64()
    w = gh.make_world(init, stream)
    d = gh.oracle_desc(init.spec)
    nets = oracle.nets_for(d, init.params)
    m0 = int(init.E.sum() + init.I.sum())
    done = 0
    for snap in [0, 10, 50, 99]:
        if snap > done:
            w.step(snap - done)
            done = snap
        st_in = w.get_state()
        stats = w.step(1, stats=True)
        done += 1
        out = w.get_state()
        ref, info = oracle.step(d, gh.oracle_state_from(st_in), nets, want_margins=True)
        rep = gh.compare_step(out, ref, info["margins"])
        assert stats["mass_quanta"] == m0
        say("  snapshot", snap, rep)
    w.close()


def test_blobs_1024_step_fp32_and_bf16_error(stream):
    """1024x1024, 256 genomes: FP32 within tolerance; BF16 error reported."""
    init = wl.config_blobs_1024(precision=0)
    d = gh.oracle_desc(init.spec)
    nets = oracle.nets_for(d, init.params)
    ref, info = oracle.step(d, oracle.State.from_init(init), nets, want_margins=True)
    w = gh.make_world(init, stream)
    w.step(1)
    rep = gh.compare_step(w.get_state(), ref, info["margins"])
    say("  fp32 1024:", rep)
    w.close()
    wb = gh.make_world(init, stream, precision=1)
    wb.step(1)
    out = wb.get_state()
    err = {ch: gh.normwise(out[ch], getattr(ref, ch)) for ch in ("E", "I")}
    err["C"] = max(gh.normwise(out["C"][c], ref.C[c]) for c in range(4))
    err["G_mismatch_rate"] = float((out["G"] != ref.G).mean())
    say("  bf16 1024 error vs FP64 oracle:", err)
    assert err["E"] < 1e-2 and err["I"] < 1e-2 and err["C"] < 5e-2
    assert int(out["E"].sum() + out["I"].sum()) == int(init.E.sum() + init.I.sum())
    wb.close()


@pytest.mark.parametrize("prec", [1, 0])
def test_zipf_4096_row_bands(stream, prec):
    """The 4096x4096 workload (4096 Zipf genomes, 54-64-64-14) at full size,
    in the launch configuration the bench times: rows the oracle computes
    exactly (top, middle, the wrap rows) compared with the GPU step."""
    say("zipf 4096 prec", prec)
    init = wl.config_zipf_4096(precision=prec)
    w = gh.make_world(init, stream)
    w.step(1)
    out = w.get_state()
    d = gh.oracle_desc(init.spec)
    used = np.unique(np.concatenate([init.G[:9].ravel(), init.G[2040:2057].ravel(),
                                     init.G[-9:].ravel()]))
    nets = gh.oracle_nets(d, init.params[used], slots=used, cap=init.params.shape[0])
    s = oracle.State.from_init(init)
    for rows in [(0, 8), (2044, 2052), (4088, 4096)]:
        ref, info = oracle.step(d, s, nets, rows=rows, want_margins=True)
        if prec == 0:
            rep = gh.compare_step(out, ref, info["margins"], rows=rows)
        else:
            sl = slice(*rows)
            rep = {ch: gh.normwise(out[ch][sl], getattr(ref, ch)[sl]) for ch in ("E", "I")}
            rep["G_mismatch_rate"] = float((out["G"][sl] != ref.G[sl]).mean())
            assert rep["E"] < 1e-2 and rep["I"] < 1e-2
        say("  rows", rows, rep)
    assert int(out["E"].sum() + out["I"].sum()) == int(init.E.sum() + init.I.sum())
    w.close()


# ------------------------------------------------------------------ invariants on the GPU

def test_translation_invariance_bit_identical(stream):
    init = gh.heterogeneous_world(96, 64, n_genomes=5, seed=11)
    w = gh.make_world(init, stream)
    w.step(1)
    base = w.get_state()
    w.close()
    for dx, dy in [(1, 0), (17, 5), (95, 63)]:
        roll = lambda a: np.roll(a, (dy, dx), axis=(-2, -1))
        ri = wl.WorldInit(init.spec, roll(init.E), roll(init.I), roll(init.C), roll(init.G),
                          roll(init.R), init.slots, init.params)
        w = gh.make_world(ri, stream)
        w.step(1)
        out = w.get_state()
        for ch in ("E", "I", "C", "G", "R"):
            np.testing.assert_array_equal(out[ch], roll(base[ch]))
        w.close()


@pytest.mark.parametrize("W", [150, 152])
def test_tuning_choices_and_graph_give_identical_results(stream, W):
    init = gh.heterogeneous_world(W, 90, n_genomes=9, layers=3, hidden=64, seed=5)
    outs = []
    for act, waves, tile, strm in [(1, 0, 0, stream), (2, 1, 1, stream), (4, 0, 2, None),
                                   (2, 0, 0, None), (2, 1, 3, stream), (1, 1, 3, None),
                                   (4, 1, 3, stream)]:
        w = gh.make_world(init, strm)
        w.set_tuning(act, waves, tile)
        w.step(3)
        outs.append(w.get_state())
        w.close()
    for o in outs[1:]:
        for ch in ("E", "I", "C", "G", "R"):
            np.testing.assert_array_equal(o[ch], outs[0][ch])


@pytest.mark.parametrize("layers,hidden", [(3, 64), (2, 32)])
def test_bf16_tuning_choices_are_identical(stream, layers, hidden):
    """BF16 worlds: both network forms (register budgets) at every column-group
    width and every physics tiling step to the same state."""
    say("bf16 tunings", layers, hidden)
    init = gh.heterogeneous_world(150, 90, n_genomes=9, layers=layers, hidden=hidden, seed=5, precision=1)
    outs = []
    for act, waves, tile in [(1, 0, 0), (1, 1, 0), (2, 1, 3), (4, 0, 1), (4, 1, 3), (2, 0, 2)]:
        w = gh.make_world(init, stream)
        w.set_tuning(act, waves, tile)
        w.step(3)
        outs.append(w.get_state())
        w.close()
    for o in outs[1:]:
        for ch in ("E", "I", "C", "G", "R"):
            np.testing.assert_array_equal(o[ch], outs[0][ch])


def test_mass_conserved_many_steps(stream):
    init = gh.heterogeneous_world(128, 96, n_genomes=8, seed=21)
    w = gh.make_world(init, stream)
    m0 = int(init.E.sum() + init.I.sum())
    for _ in range(5):
        st = w.step(10, stats=True)
        assert st["mass_quanta"] == m0 and st["mass_fp64"] == float(m0)
    out = w.get_state()
    assert int(out["E"].sum() + out["I"].sum()) == m0
    assert (out["E"] >= 0).all() and (out["I"] >= 0).all()
    w.close()


def test_autotune_keeps_state(stream):
    init = gh.heterogeneous_world(200, 120, n_genomes=6, seed=2)
    w = gh.make_world(init, stream)
    before = w.get_state()
    act, waves, tile = w.autotune()
    assert act in (1, 2, 4) and waves in (0, 1) and tile in (0, 1, 2, 3)
    after = w.get_state()
    for ch in before:
        np.testing.assert_array_equal(before[ch], after[ch])
    w.close()


# ------------------------------------------------------------------ radiation

def test_radiate_matches_oracle(stream):
    say("radiate")
    W, H, cap = 300, 200, 400
    init = gh.heterogeneous_world(W, H, n_genomes=40, capacity=cap, layers=3, hidden=64, seed=9,
                                  scale=1.0)
    w = gh.make_world(init, stream)
    step_index, rate, sigma = 7, 2e-3, 0.1
    st = w.radiate(rate, sigma, step_index)
    out = w.get_state()
    P = np.zeros((cap, 56))
    P[:40] = init.params.astype(np.float64)
    G2, P2, (hc, hs), dropped = oracle.radiate(init.G, cap, P, init.spec.seed, step_index, rate,
                                               sigma)
    np.testing.assert_array_equal(out["G"], G2)                  # hit set and slots: exact
    assert st["hits"] == len(hc) and st["dropped_hits"] == dropped
    new = hs[hs >= 0]
    assert len(new) > 100
    got = w.get_genomes(new)
    np.testing.assert_allclose(got, P2[new], rtol=0, atol=2e-6)
    d = gh.oracle_desc(init.spec)
    for s in new[:10]:
        ref = oracle.cppn_to_net(d, P2[s])
        assert gh.normwise(w.debug_get_weights(int(s), ref.size), ref) <= 1e-5
    w.close()


def test_radiate_after_steps_uses_the_counts_the_steps_kept(stream):
    """Right after a step, radiation takes its free slots from the genome
    counts that physics kept up to date through the takeovers (genomes that
    lost their last cell become free); the result equals radiating the same
    state from a new histogram, and the oracle's."""
    from paper_2406_09654_amd.world import World
    ng, cap = 1000, 1008      # ~2 cells per genome: takeovers empty whole genomes
    init = gh.heterogeneous_world(48, 40, n_genomes=ng, capacity=cap, seed=21)
    w = gh.make_world(init, stream)
    tk = sum(w.step(1, stats=True)["takeovers"] for _ in range(3))
    mid = w.get_state()
    c0 = np.bincount(init.G.ravel(), minlength=cap)
    c1 = np.bincount(mid["G"].ravel(), minlength=cap)
    assert tk > 100 and int(((c0 > 0) & (c1 == 0)).sum()) > 20
    rate, sigma, step_index = 0.1, 0.1, 4
    st = w.radiate(rate, sigma, step_index)
    assert st["hits"] > int((c0 == 0).sum())   # the freed slots are needed
    out = w.get_state()
    ref_w = World.from_init(init, stream=stream)
    ref_w.set_state(mid["E"], mid["I"], mid["C"], mid["G"], mid["R"])
    st2 = ref_w.radiate(rate, sigma, step_index)
    ref = ref_w.get_state()
    np.testing.assert_array_equal(out["G"], ref["G"])
    assert (st["hits"], st["dropped_hits"]) == (st2["hits"], st2["dropped_hits"])
    P = np.zeros((cap, 56))
    P[:ng] = init.params.astype(np.float64)
    G2, P2, (hc, hs), dropped = oracle.radiate(mid["G"], cap, P, init.spec.seed, step_index, rate, sigma)
    np.testing.assert_array_equal(out["G"], G2)
    assert st["hits"] == len(hc) and st["dropped_hits"] == dropped
    new = hs[hs >= 0]
    np.testing.assert_array_equal(w.get_genomes(new), ref_w.get_genomes(new))
    w.close()
    ref_w.close()


def test_radiate_capacity_exhaustion_drops_deterministically(stream):
    W, H, cap = 120, 100, 12
    init = gh.heterogeneous_world(W, H, n_genomes=10, capacity=cap, seed=4)
    w = gh.make_world(init, stream)
    st = w.radiate(0.01, 0.1, 3)
    G2, _, (hc, hs), dropped = oracle.radiate(init.G, cap, np.pad(init.params.astype(np.float64),
                                                                  ((0, cap - 10), (0, 0))),
                                              init.spec.seed, 3, 0.01, 0.1)
    np.testing.assert_array_equal(w.get_state()["G"], G2)
    assert st["dropped_hits"] == dropped > 0 and st["hits"] == len(hc)
    w.close()


# ------------------------------------------------------------------ batched form

def test_batch_equals_each_world_alone(stream):
    from paper_2406_09654_amd.world import Batch
    inits = [gh.heterogeneous_world(s, s + 7 * k, n_genomes=3 + k, seed=100 + k, precision=1)
             for k, s in enumerate([64, 96, 33, 130, 1, 200])]
    alone = []
    for init in inits:
        w = gh.make_world(init, stream)
        w.step(3)
        alone.append(w.get_state())
        w.close()
    worlds = [gh.make_world(init, stream) for init in inits]
    b = Batch(8, stream)
    b.set_worlds(worlds)
    b.step(3)
    b.sync()
    for k, w in enumerate(worlds):
        out = w.get_state()
        for ch in ("E", "I", "C", "G", "R"):
            np.testing.assert_array_equal(out[ch], alone[k][ch])
    # change the set without a new graph: drop two, step again
    b.set_worlds(worlds[2:])
    b.step(1)
    b.sync()
    for k, w in enumerate(worlds[2:], start=2):
        w2 = gh.make_world(inits[k], stream)
        w2.step(4)
        ref = w2.get_state()
        out = w.get_state()
        for ch in ("E", "I", "C", "G", "R"):
            np.testing.assert_array_equal(out[ch], ref[ch])
        w2.close()
    b.close()
    for w in worlds:
        w.close()


def test_batch_fp32_single_step_matches_oracle(stream):
    """FP32 worlds of different sizes (one of 1x1) stepped once together by the
    batched graph: each world's step matches the oracle."""
    from paper_2406_09654_amd.world import Batch
    inits = [gh.heterogeneous_world(s, s + 5 * k, n_genomes=3 + k, seed=300 + k, precision=0)
             for k, s in enumerate([64, 96, 33, 130, 1, 200, 17])]
    worlds = [gh.make_world(init, stream) for init in inits]
    b = Batch(8, stream)
    b.set_worlds(worlds)
    b.step(1)
    b.sync()
    for init, w in zip(inits, worlds):
        d = gh.oracle_desc(init.spec)
        ref, info = oracle.step(d, oracle.State.from_init(init), oracle.nets_for(d, init.params),
                                want_margins=True)
        rep = gh.compare_step(w.get_state(), ref, info["margins"], max_band_frac=1e-2)
        say("  batched world", init.spec.width, init.spec.height, rep)
    b.close()
    for w in worlds:
        w.close()


def test_batched_512_world_set_fp32_sample_matches_oracle(stream):
    """The 512-world batched workload (sides 64..512, 8..128 genomes), run
    with FP32 networks in one autotuned batched step; 16 sampled worlds
    match the oracle."""
    from paper_2406_09654_amd.world import Batch
    specs = wl.batched_world_specs(512)
    inits = [wl.batched_world(side, ng, seed, precision=0) for side, ng, seed in specs]
    worlds = [gh.make_world(init, stream) for init in inits]
    b = Batch(512, stream)
    b.set_worlds(worlds)
    tuning = b.autotune()
    b.step(1)
    b.sync()
    pick = np.random.default_rng(5).choice(512, 16, replace=False)
    for k in pick:
        init = inits[k]
        d = gh.oracle_desc(init.spec)
        ref, info = oracle.step(d, oracle.State.from_init(init), oracle.nets_for(d, init.params),
                                want_margins=True)
        rep = gh.compare_step(worlds[k].get_state(), ref, info["margins"], max_band_frac=1e-2)
        say("  world", int(k), init.spec.width, "tuning", tuning, rep)
    b.close()
    for w in worlds:
        w.close()


# ------------------------------------------------------------------ error paths

def test_bad_genome_is_reported(stream):
    from paper_2406_09654_amd.binding import CoralaiError, CORALAI_E_GENOME
    init = gh.heterogeneous_world(16, 16, n_genomes=3, capacity=4, seed=1)
    init.G[3, 3] = 3          # slot 3 exists but has no parameters
    w = gh.make_world(init, stream)
    with pytest.raises(CoralaiError) as e:
        w.step(1, stats=True)
    assert e.value.code == CORALAI_E_GENOME
    st = w.stats()            # reported once, then cleared
    assert st["error_word"] == 0
    w.close()


def test_nonfinite_cppn_parameters_are_reported(stream):
    """A genome whose CPPN parameters are not finite: set_genomes reports a
    numeric error once and stores zero weights, never NaN."""
    from paper_2406_09654_amd.binding import CoralaiError, CORALAI_E_NUMERIC
    init = gh.heterogeneous_world(16, 16, n_genomes=3, capacity=4, seed=2)
    w = gh.make_world(init, stream)
    bad = init.params[:1].copy()
    bad[0, :] = np.nan
    with pytest.raises(CoralaiError) as e:
        w.set_genomes(np.array([3], np.int32), bad)
    assert e.value.code == CORALAI_E_NUMERIC
    assert w.stats()["error_word"] == 0           # reported once, then cleared
    d = gh.oracle_desc(init.spec)
    wt = w.debug_get_weights(3, oracle.net_size(d))
    assert np.isfinite(wt).all() and (wt == 0).all()
    w.close()


def test_ledger_overflow_is_reported_and_mass_still_conserved(stream):
    """A flow budget of 2^31 quanta or more (I1 above 512 mass units at kappa
    1/4) sets the ledger error bit rather than wrapping; the clamped plan
    still conserves mass exactly."""
    from paper_2406_09654_amd.binding import CoralaiError, CORALAI_E_NUMERIC, ERR_LEDGER
    init = gh.heterogeneous_world(24, 20, n_genomes=3, seed=3)
    init.I[5, 7] = 600 << 24
    w = gh.make_world(init, stream)
    m0 = int(init.E.sum() + init.I.sum())
    w.step(1)
    with pytest.raises(CoralaiError) as e:
        w.sync()
    assert e.value.code == CORALAI_E_NUMERIC and "0x%x" % ERR_LEDGER in str(e.value)
    out = w.get_state()
    assert int(out["E"].sum() + out["I"].sum()) == m0
    w.close()


def test_resume_from_checkpoint_is_bit_identical(stream):
    """Checkpoint (state, live genomes, step count) and resume in a new world:
    steps, radiation and merging continue bit for bit, with the day / night
    cycle in phase."""
    ng, cap = 30, 1024
    init = gh.heterogeneous_world(96, 80, n_genomes=ng, capacity=cap, seed=17)
    cycle = (10, 1 << 18, 2048)
    a = gh.make_world(init, stream)
    a.set_daylight(*cycle)
    for s in range(1, 8):
        a.step(1)
        a.radiate(2e-3, 0.1, s)
    ck = a.get_state()
    slots = np.unique(ck["G"]).astype(np.int32)
    params = a.get_genomes(slots)
    steps = a.stats()["steps"]
    assert steps == 7
    b = gh.make_world(init, stream)
    b.set_daylight(*cycle)
    b.set_genomes(slots, params)
    b.set_state(ck["E"], ck["I"], ck["C"], ck["G"], ck["R"])
    b.set_step_count(steps)
    for s in range(8, 14):
        for w in (a, b):
            w.step(1)
            w.radiate(2e-3, 0.1, s)
            w.merge(2e-3, s)
    oa, ob = a.get_state(), b.get_state()
    for ch in ("E", "I", "C", "G", "R"):
        np.testing.assert_array_equal(oa[ch], ob[ch], err_msg=ch)
    assert a.stats()["steps"] == b.stats()["steps"] == 13
    la, lb = a.energy_ledger(), b.energy_ledger()
    assert (la["injected_last"], la["removed_last"]) == (lb["injected_last"], lb["removed_last"])
    a.close()
    b.close()
