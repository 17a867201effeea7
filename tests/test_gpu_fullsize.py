"""GPU parity at full size and on the states the bench times.

The 4096x4096 workload (4096 Zipf genomes over 65536 Voronoi patches,
54-64-64-14 networks, radiation 1e-4 per cell per step with sigma 0.1) is
compared with the FP64 oracle on every row, from the initial state and from
the state the bench reaches (five steps each followed by radiation, the
autotuner, then 22 more steps with radiation), where tens of thousands of
one-cell genomes from radiation share a 2^17-slot table.  Radiation itself is
compared with the oracle on that state.  BF16 networks: every segmentation of
the unit list gives bit-identical results, and the error against the oracle
is reported."""
import json
import sys

import numpy as np
import pytest

import oracle
import workloads as wl
from tests import gpu_helpers as gh

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

RATE, SIGMA = wl.RADIATION_RATE, wl.RADIATION_SIGMA
WARMUP, AFTER_TUNE, TIMED = 5, 2, 20     # the bench's trajectory


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def stream():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2406_09654_amd as P
    P.lib()
    return torch.cuda.Stream()


def bench_trajectory(w):
    """Advance as the bench does (each step followed by radiation; the
    autotuner after the warmup steps).  Returns (steps done, tuning)."""
    k = 0

    def adv(n):
        nonlocal k
        for _ in range(n):
            w.step(1)
            k += 1
            w.radiate(RATE, SIGMA, k, stats=False)

    adv(WARMUP)
    tuning = w.autotune()
    adv(AFTER_TUNE + TIMED)
    st = w.stats()
    assert st["error_word"] == 0
    return k, tuning


def record_bf16_error(key: str, err: dict) -> None:
    """With CORALAI_BF16_ERROR_OUT set, merge the statement into that JSON
    file (with the hash of the network and weight kernel sources it holds
    for), from which the committed summary is written."""
    import hashlib
    import os
    path = os.environ.get("CORALAI_BF16_ERROR_OUT")
    if not path:
        return
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    h = hashlib.sha256()
    for rel in ("paper_2406_09654_amd/csrc/kernels_act.hip", "paper_2406_09654_amd/csrc/coralai_internal.h",
                "paper_2406_09654_amd/csrc/kernels_genome.hip"):
        with open(os.path.join(root, rel), "rb") as f:
            h.update(f.read())
    rec = {}
    if os.path.exists(path):
        with open(path) as f:
            rec = json.load(f)
    rec["source_sha256"] = h.hexdigest()
    rec[key] = err
    with open(path, "w") as f:
        json.dump(rec, f)


def bf16_error(out: dict, ref) -> dict:
    err = {ch: gh.normwise(out[ch], getattr(ref, ch)) for ch in ("E", "I")}
    err["C"] = max(gh.normwise(out["C"][c], ref.C[c]) for c in range(4))
    err["G_mismatch_rate"] = float((out["G"] != ref.G).mean())
    err["R_mismatch_rate"] = float((out["R"] != ref.R).mean())
    return err


def test_zipf_4096_initial_step_every_row_fp32(stream):
    say("4096 initial fp32")
    init = wl.config_zipf_4096(precision=0)
    w = gh.make_world(init, stream)
    w.set_tuning(1, 1, 2)
    act = w.debug_actuators()
    st = w.step(1, stats=True)
    out = w.get_state()
    w.close()
    d = gh.oracle_desc(init.spec)
    ref, info = oracle.step(d, oracle.State.from_init(init), oracle.nets_for(d, init.params),
                            want_margins=True, want_act=True)
    act_err = gh.normwise(act, info["act"])
    assert act_err <= gh.TOL, act_err
    rep = gh.compare_step(out, ref, info["margins"], act_ref=info["act"])
    rep["actuators"] = act_err
    assert st["mass_quanta"] == int(init.E.sum() + init.I.sum())
    assert st["takeovers"] == info["takeovers"] or rep["G_mismatch_total"] > 0
    say("  report", rep)


@pytest.mark.parametrize("prec", [0, 1])
def test_zipf_4096_bench_state_step_and_radiation(stream, prec):
    """From the state the bench times: one step on every row against the
    oracle (FP32: parity; BF16: error reported, segmentations identical),
    then radiation after it against the oracle's radiation, and merging
    after that against the oracle's merging."""
    say("4096 bench state prec", prec)
    init = wl.config_zipf_4096(precision=prec)
    cap = init.spec.genome_capacity
    w = gh.make_world(init, stream)
    k, tuning = bench_trajectory(w)
    st0 = w.get_state()
    live0 = np.unique(st0["G"])
    say("  after", k, "steps: tuning", tuning, "live genomes", live0.size,
        "one-cell genomes", int((np.bincount(st0["G"].ravel(), minlength=cap) == 1).sum()))
    assert live0.size > 20000
    slots, params = gh.live_genomes(w, st0["G"])
    d = gh.oracle_desc(init.spec)
    ref, info = gh.oracle_step_slots(d, gh.oracle_state_from(st0), slots, params,
                                     want_margins=True, want_act=True)
    act = w.debug_actuators()
    act_err = gh.normwise(act, info["act"])
    st = w.step(1, stats=True)
    out = w.get_state()
    m0 = int(init.E.sum() + init.I.sum())
    assert st["mass_quanta"] == m0 and st["mass_fp64"] == float(m0)
    if prec == 0:
        assert act_err <= gh.TOL, act_err
        rep = gh.compare_step(out, ref, info["margins"], act_ref=info["act"])
        rep["actuators"] = act_err
        say("  fp32 report", rep)
    else:
        # the BF16 form is reported, not graded: bounds here only catch a
        # broken kernel (its error comes from bf16 inputs in first layers
        # that cancel to a small fraction of their terms)
        err = bf16_error(out, ref)
        err["actuators"] = act_err
        err["actuator_abs_p50_p999_max"] = [float(v) for v in np.quantile(
            np.abs(act.reshape(-1, 14) - info["act"].reshape(-1, 14)).max(axis=1), [0.5, 0.999, 1.0])]
        say("BF16_ERROR_4096_BENCH_STATE " + json.dumps(err))
        record_bf16_error("zipf_4096_after_%d_steps" % k, err)
        assert err["E"] < 0.1 and err["I"] < 0.1 and act_err < 0.2
        # the four-segment deal of the unit list against one and two segments
        for nseg in (1, 2):
            w2 = gh.make_world(init, stream)
            w2.set_genomes(slots, params.astype(np.float32))
            w2.set_state(st0["E"], st0["I"], st0["C"], st0["G"], st0["R"])
            w2.set_tuning(*tuning)
            w2.debug_set_act_segments(nseg)
            w2.step(1)
            o2 = w2.get_state()
            w2.close()
            for ch in ("E", "I", "C", "G", "R"):
                np.testing.assert_array_equal(o2[ch], out[ch], err_msg="segments %d %s" % (nseg, ch))
    # radiation after step k + 1, from the counts the steps kept
    rst = w.radiate(RATE, SIGMA, k + 1)
    after = w.get_state()
    P = np.zeros((cap, 56))
    live1 = np.unique(out["G"])
    P[live1] = w.get_genomes(live1).astype(np.float64)
    G2, P2, (hc, hs), dropped = oracle.radiate(out["G"], cap, P, init.spec.seed, k + 1, RATE, SIGMA)
    np.testing.assert_array_equal(after["G"], G2)
    assert rst["hits"] == len(hc) and rst["dropped_hits"] == dropped
    new = hs[hs >= 0]
    assert len(new) > 1000
    np.testing.assert_allclose(w.get_genomes(new), P2[new], rtol=0, atol=2e-6)
    for s in new[:: max(1, len(new) // 5)][:5]:
        refw = oracle.cppn_to_net(d, P2[s])
        tol = 1e-5 if prec == 0 else 4e-3
        assert gh.normwise(w.debug_get_weights(int(s), refw.size), refw) <= tol
    say("  radiation: hits", rst["hits"], "dropped", rst["dropped_hits"])
    # merging after the radiation, at the full size: merge set, slots and the
    # children's parameters exact
    live2 = np.unique(after["G"])
    P = np.zeros((cap, 56))
    P[live2] = w.get_genomes(live2).astype(np.float64)
    mst = w.merge(RATE, k + 1)
    G3, P3, (mc, ms, ma, mb), mdropped = oracle.merge(d, after["G"], after["R"], cap, P, init.spec.seed,
                                                      k + 1, RATE)
    np.testing.assert_array_equal(w.get_state()["G"], G3)
    assert mst["hits"] == len(mc) > 100 and mst["dropped_hits"] == mdropped
    new = ms[ms >= 0]
    np.testing.assert_array_equal(w.get_genomes(new).astype(np.float64), P3[new])
    say("  merging: merges", mst["hits"], "dropped", mst["dropped_hits"])
    w.close()


def test_blobs_1024_bf16_error_statement(stream):
    """The 1024x1024 blob workload: the BF16 form's per-step error against the
    FP64 oracle, per channel, with the G/R mismatch rate, from the initial
    state and after ten steps."""
    init = wl.config_blobs_1024(precision=1)
    d = gh.oracle_desc(init.spec)
    nets = oracle.nets_for(d, init.params)
    w = gh.make_world(init, stream)
    errs = {}
    for snap in (0, 10):
        if snap:
            w.step(snap)
        st_in = w.get_state()
        w.step(1)
        out = w.get_state()
        ref, _ = oracle.step(d, gh.oracle_state_from(st_in), nets)
        errs["step_%d" % snap] = bf16_error(out, ref)
        assert errs["step_%d" % snap]["E"] < 0.1 and errs["step_%d" % snap]["I"] < 0.1
    say("BF16_ERROR_1024 " + json.dumps(errs))
    record_bf16_error("blobs_1024", errs)
    w.close()


def test_fp32_cppn_scale_2_steps(stream):
    """FP32 single steps with CPPN parameters N(0, 4): larger weights and
    actuators than the configs' N(0, 1), as radiation's mutations produce
    over a long run."""
    for (W, H, layers, hidden) in [(64, 64, 3, 64), (130, 70, 2, 32), (257, 65, 3, 64)]:
        init = gh.heterogeneous_world(W, H, n_genomes=6, layers=layers, hidden=hidden,
                                      seed=W * 5 + H, scale=2.0)
        w = gh.make_world(init, stream)
        act = w.debug_actuators()
        w.step(1)
        out = w.get_state()
        w.close()
        d = gh.oracle_desc(init.spec)
        ref, info = oracle.step(d, oracle.State.from_init(init), oracle.nets_for(d, init.params),
                                want_margins=True, want_act=True)
        act_err = gh.normwise(act, info["act"])
        assert act_err <= gh.TOL, act_err
        rep = gh.compare_step(out, ref, info["margins"], max_band_frac=1e-2)
        say("  scale 2", W, H, "actuators", act_err, rep)
