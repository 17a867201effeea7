"""Serving form on the GPU: continuous batching gives every request the same
result as stepping its world alone, whatever else shares its steps."""
import numpy as np
import pytest
import torch

import oracle
import workloads as wl
from tests import gpu_helpers as gh

pytestmark = pytest.mark.gpu


def _requests():
    # arrivals by batched-step index: later requests join while earlier ones run,
    # some retire while others continue
    spec = [(0, 48, 6, 5), (0, 80, 11, 3), (2, 33, 4, 7), (3, 129, 9, 4), (5, 64, 16, 2),
            (5, 17, 3, 6), (9, 100, 20, 3)]
    reqs = [wl.Request(k, float(a), side, ng, steps, 7000 + k)
            for k, (a, side, ng, steps) in enumerate(spec)]
    return reqs, {r.rid: wl.request_world(r) for r in reqs}


@pytest.mark.parametrize("prec", [0, 1])
def test_served_results_equal_each_world_alone(prec):
    from paper_2406_09654_amd.serving import Server
    from paper_2406_09654_amd.world import World
    reqs, inits = _requests()
    srv = Server(precision=prec, max_worlds=4, max_chunk=2)
    rep = srv.run(reqs, inits, arrivals="step", keep_states=True)
    srv.close()
    assert rep["n_requests"] == len(reqs)
    assert rep["mean_resident"] > 1.0           # requests really shared steps
    s = torch.cuda.Stream()
    for r in reqs:
        res = rep["results"][r.rid]
        assert len(res.step_ids) == r.n_steps
        w = World.from_init(inits[r.rid], stream=s, precision=prec)
        w.step(r.n_steps)
        ref = w.get_state()
        w.close()
        for ch in ("E", "I", "C", "G", "R"):
            np.testing.assert_array_equal(res.state[ch].cpu().numpy(), ref[ch], err_msg="%d %s" % (r.rid, ch))


def test_admission_by_bytes_limits_residency():
    from paper_2406_09654_amd.serving import Server
    reqs, inits = _requests()
    srv = Server(precision=1, max_worlds=8)
    biggest = max(srv.footprint(inits[r.rid]) for r in reqs)
    srv.close()
    srv = Server(precision=1, max_worlds=8, hbm_budget=biggest + 1)
    rep = srv.run(reqs, inits, arrivals="step")
    srv.close()
    # one world at a time fits when the largest one is resident
    assert rep["n_requests"] == len(reqs)
    assert all(len(rep["results"][r.rid].step_ids) == r.n_steps for r in reqs)
    assert rep["step_latency_ms_p99"] >= rep["step_latency_ms_p50"] > 0


def test_served_one_step_requests_match_oracle():
    """FP32 serving: requests of one step arrive while longer ones run, so
    each is stepped in a batch with others; each result matches the
    oracle's single step from the request's seeded state."""
    from paper_2406_09654_amd.serving import Server
    spec = [(0, 96, 12, 6), (0, 40, 5, 1), (1, 70, 9, 1), (1, 128, 30, 4), (2, 33, 4, 1),
            (3, 150, 20, 1), (3, 64, 16, 1), (5, 100, 8, 1)]
    reqs = [wl.Request(k, float(a), side, ng, steps, 8100 + k)
            for k, (a, side, ng, steps) in enumerate(spec)]
    inits = {r.rid: wl.request_world(r) for r in reqs}
    srv = Server(precision=0, max_worlds=4, max_chunk=1)
    rep = srv.run(reqs, inits, arrivals="step", keep_states=True)
    srv.close()
    assert rep["mean_resident"] > 1.0
    for r in reqs:
        if r.n_steps != 1:
            continue
        init = inits[r.rid]
        d = gh.oracle_desc(init.spec)
        ref, info = oracle.step(d, oracle.State.from_init(init), oracle.nets_for(d, init.params),
                                want_margins=True)
        st = {k: v.cpu().numpy() for k, v in rep["results"][r.rid].state.items()}
        gh.compare_step(st, ref, info["margins"], max_band_frac=1e-2)
