#!/usr/bin/env python3
"""Throughput of the per-step ecosystem update on one MI355X.

Workload: the 4096x4096 periodic world with 4096 Zipf(s=1.1) genomes over
65536 Voronoi patches, 54-64-64-14 networks, radiation 1e-4 per cell per
step with sigma 0.1.  One step = one whole pass of the hot path: genome
bucketing, sense + network (grouped GEMM on MFMA) + actuator epilogue,
exploration/takeover physics with the FP64 + int64 mass reduction, then
radiation (Philox hits, slot assignment, CPPN weight regeneration).  Inputs
are resident in HBM before timing starts.

value = cell-updates/s with BF16 networks (FP32 accumulation); the FP32
network form is measured on the same input and reported beside it.
Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "cell-updates/sec at 4096² (FP32 vs BF16); p50/p99 step latency under serving load"
PEAK_HBM = 8.0e12            # bytes/s
PEAK_BF16 = 2.5e15           # dense MFMA FLOP/s
PEAK_FP32 = 157.3e12         # FLOP/s
# transcendental ops/s: the FP32 vector peak of 157.3 TFLOP/s is 256 CUs x
# 128 FMA lanes/clock x 2 FLOP x 2.4 GHz; exp2 / rcp / log issue at a quarter
# of that lane rate, 32 lanes per CU per clock: 256 x 32 x 2.4 GHz
PEAK_TRANS = 256 * 32 * 2.4e9
ACT_BYTES_PER_CELL = 100   # reads ledger pair, comm, perm entry (36 B); writes comm, ledger pair, flows (64 B)
PHYS_BYTES_PER_CELL = 74   # reads flow record, ledger pair, genome, rotation (53 B); writes 21 B
RATE, SIGMA = 1e-4, 0.1
BYTES_PER_CELL_STEP = 190  # two-pass design: act (100 B) + physics (74 B) + bucketing (~12 B) + finalize
# Serving request rate: 0.8 x the 512-world batched capacity measured when
# the rate was frozen (1.55e10 cell-updates/s) divided by the mean request
# work, E[side^2] E[steps] for log-uniform side 128..2048 and steps 10..1000:
# (2048^2 - 128^2) / (2 ln 16) x (1000 - 10) / ln 100 = 7.53e5 x 215 = 1.62e8
SERVING_RATE = 77.0


def flops_per_cell(hidden: int, layers: int) -> int:
    widths = [54] + [hidden] * (layers - 1) + [14]
    return 2 * sum(widths[k] * widths[k + 1] for k in range(layers))


def trans_per_cell(hidden: int, layers: int) -> int:
    # tanh = exp + reciprocal per hidden unit; 6 sigmoids (exp + reciprocal);
    # 8 softmax exponentials and one reciprocal of their sum
    return 2 * hidden * (layers - 1) + 2 * 6 + 8 + 1


def weight_bytes_per_genome(hidden: int, layers: int) -> int:
    """Bytes of one genome's BF16 network as the network kernel reads it:
    fragments of 1 KiB (16-row tiles x 32-wide K-steps; the 54 inputs take
    2 K-steps) and the FP32 biases."""
    mt, ks0, ksh = hidden // 16, 2, hidden // 32
    frags = mt * ks0 + (mt * ksh if layers == 3 else 0) + ksh
    return 1024 * frags + 4 * (hidden * (layers - 1) + 16)


ACT_SOURCES = ["paper_2406_09654_amd/csrc/kernels_act.hip", "paper_2406_09654_amd/csrc/coralai_internal.h"]
NET_SOURCES = ACT_SOURCES + ["paper_2406_09654_amd/csrc/kernels_genome.hip"]
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_act_bf16_4096_hbm_traffic.md")
BF16_ERROR_FILE = os.path.join(ROOT, "profiles", "bf16_error_vs_oracle.md")


def sources_sha256(paths) -> str:
    import hashlib
    h = hashlib.sha256()
    for rel in paths:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def act_sources_sha256() -> str:
    return sources_sha256(ACT_SOURCES)


def bf16_error_statement():
    """The BF16 form's error against the FP64 oracle, as the GPU parity tests
    measured it (committed summary); None when the network or weight kernels
    changed since."""
    if not os.path.exists(BF16_ERROR_FILE):
        return None
    with open(BF16_ERROR_FILE) as f:
        for line in f:
            if line.startswith("bf16_error_json: "):
                rec = json.loads(line[len("bf16_error_json: "):])
                if rec.get("source_sha256") != sources_sha256(NET_SOURCES):
                    return {"stale": "network or weight kernels changed since the measurement"}
                rec["source"] = os.path.relpath(BF16_ERROR_FILE, ROOT)
                return rec
    return None


def act_traffic(tuning):
    """HBM bytes per launch of the BF16 network kernel from the committed
    rocprofv3 counter summary (FETCH_SIZE and WRITE_SIZE, scaled by the copy
    calibration), for the launch configuration the bench ran.  None when the
    summary is missing, has no line for that configuration, or the kernel's
    sources changed since the counters were taken."""
    if not os.path.exists(TRAFFIC_FILE):
        return None, "no counter summary"
    # the network kernel's traffic depends on (act_cells, act_waves), not on the physics tiling
    want = ",".join(str(v) for v in tuning[:2]) if tuning is not None else None
    stale = False
    with open(TRAFFIC_FILE) as f:
        for line in f:
            if not line.startswith("traffic:"):
                continue
            fields = dict(kv.partition("=")[::2] for kv in line.split()[1:])
            if fields.get("tuning") != want:
                continue
            if fields.get("source_sha256") != act_sources_sha256():
                stale = True
                continue
            return int(fields["bytes_per_launch"]), "FETCH_SIZE x %s + WRITE_SIZE x %s per launch, %s" % (
                fields.get("fetch_factor"), fields.get("write_factor"), os.path.relpath(TRAFFIC_FILE, ROOT))
    return None, ("kernel changed since the counters were taken" if stale
                  else "no counters for tuning %s" % want)


def run_form(init, precision: int, steps: int, warmup: int, stream, autotune: bool, tuning=None):
    """One form on the 4096^2 trajectory: warmup steps, the autotuner, two
    more steps, then `steps` steps on the production path (each step one
    captured graph replay, radiation after it; no profiling); then the same
    steps of the same trajectory with live phase timing (direct launches
    with HIP events between the phases on the world's stream), whose
    network-kernel time gives the roofline."""
    import torch

    from paper_2406_09654_amd.world import World

    w = World.from_init(init, stream=stream, precision=precision)
    if tuning is not None:
        w.set_tuning(*tuning)
    step_index = 0

    def advance(n):
        nonlocal step_index
        for _ in range(n):
            w.step(1)
            step_index += 1
            w.radiate(RATE, SIGMA, step_index, stats=False)

    advance(warmup)
    if tuning is None and autotune:
        # tuned on a state past the first steps (which take over a large share
        # of the random initial grid), then two more untimed steps
        tuning = w.autotune()
        advance(2)
    w.sync()
    torch.cuda.synchronize()
    first = step_index + 1
    t0 = time.perf_counter()
    advance(steps)
    w.sync()
    torch.cuda.synchronize()
    t_graph = time.perf_counter() - t0
    w.close()
    # the same steps again on a second world with the same tuning (the
    # trajectory does not depend on the launch configuration), now with the
    # phases timed
    w = World.from_init(init, stream=stream, precision=precision)
    w.set_tuning(*tuning)
    step_index = 0
    advance(first - 1)
    w.sync()
    live_start = w.stats()["live_genomes"]
    w.set_profiling(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    advance(steps)
    w.sync()
    torch.cuda.synchronize()
    t_phase = time.perf_counter() - t0
    prof = w.profile()
    st = w.stats()
    w.set_profiling(False)
    w.close()
    del w
    torch.cuda.empty_cache()
    N = init.spec.width * init.spec.height
    return {
        "value": N * steps / t_graph,
        "ms_per_step": 1e3 * t_graph / steps,
        "timed_steps": [first, first + steps - 1],
        "phase_timed": {"value": N * steps / t_phase, "ms_per_step": 1e3 * t_phase / steps,
                        "timed_steps": [first, first + steps - 1]},
        "phase_ms": {k: (v[0] / v[1] if v[1] else None) for k, v in prof.items()},
        "stats": st,
        "live_genomes_window": [live_start, st["live_genomes"]],
        "tuning": tuning,
    }


VARIANTS = [
    ("day_night", "day/night cycle, period 100 steps, 2^-6 mass units per cell at noon, 1/64 of a cell's energy per step at midnight",
     dict(daylight=(100, 1 << 18, 1024))),
    ("hard_max", "hard-max exploration (the whole budget to the maximal explore actuator)", dict(variant=(1, 0.0))),
    ("energy_transport", "energy transport: 1/4 of a cell's energy along the flow directions", dict(variant=(0, 0.25))),
    ("merging", "merging (NEAT crossover with the faced neighbour's genome) at 1e-4 per cell per step, after radiation",
     dict(merge=RATE)),
    ("structural_mutation", "radiation with NEAT's add-connection and add-node, each with probability 0.5 per hit",
     dict(structural=(0.5, 0.5))),
]


def run_variants(init, precision: int, steps: int, warmup: int, tuning, stream):
    """The 4096^2 step with each physics option on, on the production path
    (graph replay + radiation), same tuning as the plain form; merging adds a
    merging call after each radiation call."""
    import torch

    from paper_2406_09654_amd.binding import WORLD_ENERGY_FLOWS
    from paper_2406_09654_amd.world import World

    out = {}
    N = init.spec.width * init.spec.height
    for name, what, opts in VARIANTS:
        flags = WORLD_ENERGY_FLOWS if "variant" in opts and opts["variant"][1] > 0 else 0
        w = World.from_init(init, stream=stream, precision=precision, flags=flags)
        w.set_tuning(*tuning)
        if "daylight" in opts:
            w.set_daylight(*opts["daylight"])
        if "variant" in opts:
            w.set_physics_variant(*opts["variant"])
        if "structural" in opts:
            w.set_structural_mutation(*opts["structural"])
        k = 0
        for _ in range(warmup):
            w.step(1)
            k += 1
            w.radiate(RATE, SIGMA, k, stats=False)
            if "merge" in opts:
                w.merge(opts["merge"], k, stats=False)
        w.sync()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            w.step(1)
            k += 1
            w.radiate(RATE, SIGMA, k, stats=False)
            if "merge" in opts:
                w.merge(opts["merge"], k, stats=False)
        w.sync()
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        st = w.stats()
        assert st["error_word"] == 0
        out[name] = {"what": what, "value": N * steps / dt, "ms_per_step": 1e3 * dt / steps,
                     "timed_steps": [warmup + 1, warmup + steps]}
        w.close()
        del w
        torch.cuda.empty_cache()
    return out


def run_long(init, precision: int, n_steps: int, tuning, stream, block: int = 100):
    """The 4096^2 workload run as configured: n_steps steps, each followed by
    radiation at 1e-4, in blocks of `block` steps (queued without waiting;
    the block's end waits and reads the statistics of its last step and
    radiation call)."""
    import torch

    from paper_2406_09654_amd.world import World

    w = World.from_init(init, stream=stream, precision=precision)
    w.set_tuning(*tuning)
    N = init.spec.width * init.spec.height
    blocks = []
    k = 0
    torch.cuda.synchronize()
    t_all = time.perf_counter()
    while k < n_steps:
        n = min(block, n_steps - k)
        t0 = time.perf_counter()
        for _ in range(n - 1):
            w.step(1)
            k += 1
            w.radiate(RATE, SIGMA, k, stats=False)
        st_step = w.step(1, stats=True)
        k += 1
        st = w.radiate(RATE, SIGMA, k, stats=True)
        dt = time.perf_counter() - t0
        blocks.append({"steps": [k - n + 1, k], "ms_per_step": 1e3 * dt / n,
                       "live_genomes": st_step["live_genomes"], "takeovers_last_step": st_step["takeovers"],
                       "hits_last_call": st["hits"], "dropped_hits_last_call": st["dropped_hits"]})
        assert st["error_word"] == 0 and st_step["mass_quanta"] == int(init.E.sum() + init.I.sum())
    total = time.perf_counter() - t_all
    w.close()
    del w
    torch.cuda.empty_cache()
    last = [b for b in blocks if b["steps"][0] > n_steps - block]
    return {"steps": n_steps, "value": N * n_steps / total, "ms_per_step_mean": 1e3 * total / n_steps,
            "ms_per_step_last_block": last[-1]["ms_per_step"] if last else None,
            "live_genomes_end": blocks[-1]["live_genomes"], "genome_capacity": init.spec.genome_capacity,
            "dropped_hits_last_call": blocks[-1]["dropped_hits_last_call"],
            "hits_last_call": blocks[-1]["hits_last_call"], "blocks": blocks, "tuning": tuning}


def run_batched(n_worlds: int, steps: int, warmup: int, alone_steps: int):
    """512 uneven worlds (side U{64..512}, 8..128 genomes, 54-32-14 BF16 nets)
    advanced by one captured batched step, against the same worlds stepped one
    by one on the same stream."""
    import torch

    import workloads as wl
    from paper_2406_09654_amd.world import Batch, World

    specs = wl.batched_world_specs(n_worlds)
    print("[bench] batched: generating %d worlds" % n_worlds, file=sys.stderr, flush=True)
    inits = [wl.batched_world(side, ng, seed, precision=1) for side, ng, seed in specs]
    stream = torch.cuda.Stream()
    worlds = [World.from_init(i, stream=stream, precision=1) for i in inits]
    cells = sum(w.N for w in worlds)
    b = Batch(n_worlds, stream)
    b.set_worlds(worlds)
    tuning = b.autotune()
    b.step(warmup)
    b.sync()
    t0 = time.perf_counter()
    b.step(steps)
    b.sync()
    t_b = time.perf_counter() - t0
    b.set_worlds([])
    for w in worlds:
        w.step(1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(alone_steps):
        for w in worlds:
            w.step(1)
    torch.cuda.synchronize()
    t_a = time.perf_counter() - t0
    b.close()
    for w in worlds:
        w.close()
    del worlds
    torch.cuda.empty_cache()
    return {"worlds": n_worlds, "cells_per_step": cells, "steps": steps, "tuning": tuning,
            "value": cells * steps / t_b, "ms_per_step": 1e3 * t_b / steps,
            "one_by_one_value": cells * alone_steps / t_a,
            "one_by_one_ms_per_step": 1e3 * t_a / alone_steps,
            "speedup_vs_one_by_one": (cells * steps / t_b) / (cells * alone_steps / t_a),
            "unit": "cell-updates/s", "dtype": "bf16"}


def run_serving(n_requests: int, rate: float):
    """Poisson request stream (side log-uniform 128..2048, 16..1024 genomes,
    10..1000 steps, blob states), served by continuous batching in FP32 and
    in BF16."""
    import torch

    import workloads as wl
    from paper_2406_09654_amd.serving import Server

    reqs = wl.poisson_requests(n_requests, rate)
    print("[bench] serving: generating %d requests" % n_requests, file=sys.stderr, flush=True)
    inits = {r.rid: wl.request_world(r) for r in reqs}
    out = {"requests": n_requests, "rate_per_s": rate,
           "cell_updates": int(sum(r.side * r.side * r.n_steps for r in reqs))}
    for prec, name in [(0, "fp32"), (1, "bf16")]:
        srv = Server(precision=prec, max_worlds=64)
        # warm the graph and the kernels on a tiny request set
        srv.run(reqs[:2], inits, arrivals="step")
        rep = srv.run(reqs, inits)
        srv.close()
        torch.cuda.empty_cache()
        out[name] = {k: rep[k] for k in ("step_latency_ms_p50", "step_latency_ms_p99",
                                         "time_to_completion_s_p50", "time_to_completion_s_p99",
                                         "cell_updates_per_s", "cell_updates_per_gpu_busy_s",
                                         "wall_s", "batched_steps", "mean_resident")}
        print("[bench] serving %s: %s" % (name, out[name]), file=sys.stderr, flush=True)
    return out


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _omp_threads(n: int) -> None:
    """Set the OpenMP thread count of the runtime the oracle is linked with."""
    import ctypes
    ctypes.CDLL("libgomp.so.1").omp_set_num_threads(int(n))


def cpu_baseline(init, target_s: float = 12.0, one_thread_s: float = 5.0):
    """The FP64 oracle (as it stands, OpenMP over cells) on a band of rows of
    the same state, widened to the whole grid and then repeated until about
    target_s seconds of CPU work have been timed; then on one thread."""
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    out = _cpu_baseline(init, target_s, threads)
    _omp_threads(1)
    try:
        one = _cpu_baseline(init, one_thread_s, 1)
    finally:
        _omp_threads(threads)
    out["one_thread"] = {"value": one["value"], "cores": 1, "sample": one["sample"]}
    out["cpu_model"] = cpu_model()
    return out


def _cpu_baseline(init, target_s: float, threads: int):
    import numpy as np

    import oracle

    d = oracle.Desc.from_spec(init.spec)
    s = oracle.State.from_init(init)
    H = init.spec.height
    nets = np.zeros((init.params.shape[0], oracle.net_size(d)))
    have = set()

    def need_nets(y0, y1):
        for g in np.unique(init.G[max(0, y0 - 1): y1 + 1]):
            if int(g) not in have:
                nets[g] = oracle.cppn_to_net(d, init.params[g].astype(np.float64))
                have.add(int(g))

    rows = 16
    while True:
        y0 = H // 2 - rows // 2
        need_nets(y0, y0 + rows)
        t0 = time.perf_counter()
        oracle.step(d, s, nets, rows=(y0, y0 + rows))
        dt = time.perf_counter() - t0
        if dt >= target_s or rows >= H:
            break
        rows = min(H, max(rows * 2, int(rows * target_s / max(dt, 1e-3) * 1.1)))
    cells, total, reps = rows * init.spec.width, dt, 1
    while total < target_s and rows >= H:
        t0 = time.perf_counter()
        oracle.step(d, s, nets)
        total += time.perf_counter() - t0
        reps += 1
    return {"value": cells * reps / total, "unit": "cell-updates/s", "cores": threads,
            "kind": "oracle",
            "sample": "FP64 oracle step (sense, network, actuation, physics) on %d full rows "
                      "(%d cells) of the same %dx%d state, %d time(s), %.1f s on %d OpenMP "
                      "threads; radiation not included"
                      % (rows, cells, init.spec.width, H, reps, total, threads)}


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--size", type=int, default=4096, help="grid side (4096 = the named workload)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--bf16-only", action="store_true")
    ap.add_argument("--tuning-bf16", default=None,
                    help="act_cells,act_waves,phys_tile for the BF16 form instead of autotuning")
    ap.add_argument("--tuning-fp32", default=None,
                    help="act_cells,act_waves,phys_tile for the FP32 form instead of autotuning")
    ap.add_argument("--no-batched", action="store_true", help="skip the 512-world batched form")
    ap.add_argument("--no-serving", action="store_true", help="skip the serving form")
    ap.add_argument("--serving-requests", type=int, default=256)
    ap.add_argument("--serving-rate", type=float, default=SERVING_RATE,
                    help="Poisson arrivals per second (default: 0.8 x the batched capacity / mean request work)")
    ap.add_argument("--long-steps", type=int, default=1000,
                    help="steps of the as-configured 4096^2 run per form (0 skips it)")
    ap.add_argument("--no-variants", action="store_true",
                    help="skip the 4096^2 step with the day/night cycle, hard max and energy transport")
    ap.add_argument("--batched-only", action="store_true",
                    help="profiling aid: run only the 512-world batched form and print its block")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="first run one plain device copy of 512 MiB (scales the HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        return 2

    import torch

    import workloads as wl

    assert torch.cuda.is_available(), "bench.py needs the GPU"
    torch.cuda.set_device(0)
    if args.copy_calibration:
        src = torch.ones(1 << 27, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    if args.batched_only:
        b = run_batched(512, args.steps, 3, 3)
        print(json.dumps({"metric": "batched cell-updates/s (512 worlds, profiling run)", "value": b["value"],
                          "unit": "cell-updates/s", "n_gpus": 1, "steps": args.steps, "batched": b}), flush=True)
        return 0
    side = args.size
    patches = max(1, 65536 * side * side // (4096 * 4096))
    print("[bench] generating %dx%d workload" % (side, side), file=sys.stderr, flush=True)
    init = wl.config_zipf_4096(precision=1, width=side, height=side, n_patches=patches)
    stream = torch.cuda.Stream()
    N = side * side
    hidden, layers = init.spec.hidden, init.spec.n_weight_layers

    forms = {}
    fixed = {"bf16": args.tuning_bf16, "fp32": args.tuning_fp32}
    for prec, name in ([(1, "bf16")] if args.bf16_only else [(1, "bf16"), (0, "fp32")]):
        print("[bench] %s: warmup %d, timed %d steps" % (name, args.warmup, args.steps),
              file=sys.stderr, flush=True)
        tun = tuple(int(v) for v in fixed[name].split(",")) if fixed[name] else None
        forms[name] = run_form(init, prec, args.steps, args.warmup, stream,
                               not args.no_autotune, tun)
        print("[bench] %s: %.3e cell-updates/s, %.3f ms/step, phases %s" % (
            name, forms[name]["value"], forms[name]["ms_per_step"], forms[name]["phase_ms"]),
            file=sys.stderr, flush=True)

    variants = None
    if not args.no_variants:
        print("[bench] bf16 physics options", file=sys.stderr, flush=True)
        variants = run_variants(init, 1, args.steps, args.warmup + 2, forms["bf16"]["tuning"], stream)
        print("[bench] options: %s" % {k: round(v["ms_per_step"], 3) for k, v in variants.items()},
              file=sys.stderr, flush=True)

    long_runs = {}
    if args.long_steps > 0 and side == 4096:
        for prec, name in ([(1, "bf16")] if args.bf16_only else [(1, "bf16"), (0, "fp32")]):
            print("[bench] %s: %d steps as configured" % (name, args.long_steps), file=sys.stderr, flush=True)
            long_runs[name] = run_long(init, prec, args.long_steps, forms[name]["tuning"], stream)
            print("[bench] %s long run: %.3f ms/step mean, %.3f last block, live genomes %d, dropped %d"
                  % (name, long_runs[name]["ms_per_step_mean"], long_runs[name]["ms_per_step_last_block"],
                     long_runs[name]["live_genomes_end"], long_runs[name]["dropped_hits_last_call"]),
                  file=sys.stderr, flush=True)

    bf = forms["bf16"]
    act_ms = bf["phase_ms"]["act"]
    trans = trans_per_cell(hidden, layers) * N
    traffic, traffic_note = act_traffic(bf["tuning"])
    # the kernel is bound by the vector-memory pipeline (the counter summary
    # and the design notes give the evidence), so its roofline is memory:
    # the cells' algorithmic bytes plus each live genome's weights once
    live = 0.5 * sum(bf["live_genomes_window"])
    wbytes = weight_bytes_per_genome(hidden, layers)
    act_bytes = ACT_BYTES_PER_CELL * N + live * wbytes
    roof = {"kernel": "k_act (sense + grouped MLP + epilogue)", "bound": "hbm",
            "achieved": act_bytes / (act_ms * 1e-3) / 1e9, "peak": PEAK_HBM / 1e9,
            "unit": "GB/s", "frac": act_bytes / (act_ms * 1e-3) / PEAK_HBM,
            "traffic": traffic, "traffic_note": traffic_note,
            "per_unit": "%d B per cell x %d cells, plus %d B of BF16 weights and biases per live genome "
                        "x %.0f live genomes (mean over the timed steps), per launch"
                        % (ACT_BYTES_PER_CELL, N, wbytes, live),
            "limiter": "vector-memory pipeline (texture data path busy most of the launch, requests "
                       "waiting on L2); profiles/k_act_4096_memory_pipeline.md",
            "transcendental": {"achieved": trans / (act_ms * 1e-3), "peak": PEAK_TRANS,
                               "unit": "op/s", "frac": trans / (act_ms * 1e-3) / PEAK_TRANS,
                               "per_unit": "%d per cell" % trans_per_cell(hidden, layers)},
            "mfma_frac_bf16": flops_per_cell(hidden, layers) * N / (act_ms * 1e-3) / PEAK_BF16}
    out = {
        "metric": METRIC,
        "value": bf["value"],
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": bf["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "bf16",
        "data": "synthetic",
        "config": {"workload": "%dx%d periodic world, 4096 Zipf(1.1) genomes over %d Voronoi "
                               "patches, 54-64-64-14 networks (BF16 MFMA, FP32 accumulate), "
                               "int64 ledger physics, radiation 1e-4/cell/step sigma 0.1"
                               % (side, side, patches),
                   "cells": N, "genomes": 4096, "network": "54-64-64-14"},
        "roofline": roof,
        "timed_steps": bf["timed_steps"],
        "path": "captured step graph per step, radiation after each step, no profiling",
        "phase_timed": bf["phase_timed"],
        "phase_ms_per_step": bf["phase_ms"],
        "tuning": bf["tuning"],
        "bf16_error": bf16_error_statement(),
    }
    if "fp32" in forms:
        f = forms["fp32"]
        fa = f["phase_ms"]["act"]
        fl = flops_per_cell(hidden, layers) * N
        out["fp32"] = {"value": f["value"], "ms_per_step": f["ms_per_step"],
                       "timed_steps": f["timed_steps"], "phase_timed": f["phase_timed"],
                       "phase_ms_per_step": f["phase_ms"], "tuning": f["tuning"],
                       "roofline": {"kernel": "k_act", "bound": "mfma", "achieved": fl / (fa * 1e-3) / 1e12,
                                    "peak": PEAK_FP32 / 1e12, "unit": "TFLOP/s",
                                    "frac": fl / (fa * 1e-3) / PEAK_FP32, "traffic": None}}
        out["bf16_over_fp32"] = bf["value"] / f["value"]
    phys_ms = bf["phase_ms"]["physics"]
    out["physics_roofline"] = {"bound": "hbm", "achieved": PHYS_BYTES_PER_CELL * N / (phys_ms * 1e-3) / 1e9,
                               "peak": PEAK_HBM / 1e9, "unit": "GB/s",
                               "frac": PHYS_BYTES_PER_CELL * N / (phys_ms * 1e-3) / PEAK_HBM,
                               "per_unit": "%d B per cell (reads the 32-byte flow record, boundary ledger pair, "
                                           "genome, rotation; writes ledger pair, genome, rotation)"
                                           % PHYS_BYTES_PER_CELL}
    if variants:
        out["physics_options_bf16"] = variants
    if long_runs:
        out["long_run"] = long_runs
    if not args.no_batched:
        out["batched"] = run_batched(512, 20, 3, 3)
        b = out["batched"]
        b["roofline"] = {"bound": "hbm", "unit": "GB/s", "peak": PEAK_HBM / 1e9,
                         "achieved": b["value"] * BYTES_PER_CELL_STEP / 1e9,
                         "frac": b["value"] * BYTES_PER_CELL_STEP / PEAK_HBM,
                         "per_unit": "%d B per cell-update (the two-pass design's act, physics and "
                                     "bucketing bytes), whole batched step" % BYTES_PER_CELL_STEP}
        print("[bench] batched: %s" % out["batched"], file=sys.stderr, flush=True)
    if not args.no_serving:
        out["serving"] = run_serving(args.serving_requests, args.serving_rate)
    if not args.no_cpu_baseline:
        print("[bench] oracle CPU baseline", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(init)
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
