"""Shared helpers of the GPU parity tests: world construction from a seeded
input, oracle runs on the same input, and the comparison rules.

Comparison rules (floating point: normwise per channel; integers: exact
outside the near-tie band):
  * C', E, I:  max|gpu - oracle| <= TOL * max|oracle| per channel, TOL = 1e-5;
               where the oracle's actuators are given, C' = sigmoid(a_comm)
               is held to the bar of the comm actuators it is computed from:
               max|dC'| <= TOL * max(1, max|a_comm| / 4) (sigmoid' <= 1/4).
               FP32 arithmetic itself does not reach 1e-5 on C' at the few
               cells of the 4096^2 workload whose first layer cancels to
               1/5000 of its terms, even with exact accumulation;
  * G, R:      bit-exact wherever the oracle's FP64 decision margins are
               outside the near-tie band -- the flow-logit gap of every
               neighbour whose top two explore directions include the cell
               (and that can invest at all) is >= 1e-4, and either
               |v_win - I1| >= 1e-5 * max(v_win, I1) + 64 quanta and, when
               the winner takes over, v_win - v_second is as large, or all
               the integers those comparisons read are decided (every floor
               behind them is away from an integer by more than 0.1% of its
               argument, or is an exact zero), so that the comparison is
               exact however close; cells inside the band are counted and
               must be rare;
  * mass:      exact (int64 sum of the GPU state == the input's sum; the GPU's
               FP64 reduction equals it exactly).
"""
from __future__ import annotations

import numpy as np

import oracle
import workloads as wl

TOL = 1e-5
GAP_BAND = 1e-4


def oracle_desc(spec) -> "oracle.Desc":
    return oracle.Desc.from_spec(spec)


def make_world(init, stream=None, precision=None):
    from paper_2406_09654_amd.world import World
    return World.from_init(init, stream=stream, precision=precision)


def oracle_state_from(st: dict) -> "oracle.State":
    return oracle.State(st["E"].astype(np.int64), st["I"].astype(np.int64),
                        st["C"].astype(np.float64), st["G"].astype(np.int32),
                        st["R"].astype(np.uint8))


def band_mask(margins: np.ndarray) -> np.ndarray:
    thr = 1e-5 * margins[..., 3] + 64.0
    close = (margins[..., 1] < thr) | (margins[..., 2] < thr)
    return (margins[..., 0] < GAP_BAND) | (close & (margins[..., 4] == 0))


def normwise(gpu: np.ndarray, ref: np.ndarray) -> float:
    scale = float(np.max(np.abs(ref))) if ref.size else 0.0
    err = float(np.max(np.abs(gpu.astype(np.float64) - ref.astype(np.float64)))) if ref.size else 0.0
    return err / scale if scale > 0 else err


def compare_step(gpu_out: dict, ref: "oracle.State", margins: np.ndarray, rows=None,
                 tol: float = TOL, max_band_frac: float = 1e-3, act_ref: np.ndarray | None = None,
                 ledger_outside_band: bool = False):
    """Assert one step's parity; returns a report dict.  ledger_outside_band:
    compare E and I only outside the near-tie band (hard-max exploration,
    where a near-tied argmax moves the whole budget between two cells)."""
    sl = slice(None) if rows is None else slice(rows[0], rows[1])
    rep = {}
    keep = ~band_mask(margins[sl]) if ledger_outside_band else np.ones(gpu_out["E"][sl].shape, bool)
    for ch in ("E", "I"):
        rep[ch] = normwise(gpu_out[ch][sl][keep], getattr(ref, ch)[sl][keep])
    rep["C"] = max(normwise(gpu_out["C"][c][sl], ref.C[c][sl]) for c in range(4))
    tol_c = tol
    if act_ref is not None:
        tol_c = tol * max(1.0, float(np.max(np.abs(act_ref[sl][..., 2:6]))) / 4.0)
        rep["C_tol"] = tol_c
    band = band_mask(margins[sl])
    g_bad = (gpu_out["G"][sl] != ref.G[sl]) & ~band
    r_bad = (gpu_out["R"][sl] != ref.R[sl]) & ~band
    rep["band_cells"] = int(band.sum())
    rep["band_frac"] = float(band.mean()) if band.size else 0.0
    rep["G_mismatch_outside_band"] = int(g_bad.sum())
    rep["R_mismatch_outside_band"] = int(r_bad.sum())
    rep["G_mismatch_total"] = int((gpu_out["G"][sl] != ref.G[sl]).sum())
    assert rep["E"] <= tol and rep["I"] <= tol and rep["C"] <= tol_c, rep
    assert rep["G_mismatch_outside_band"] == 0 and rep["R_mismatch_outside_band"] == 0, rep
    assert rep["band_frac"] <= max_band_frac, rep
    return rep


def oracle_nets(d, params: np.ndarray, slots=None, cap=None) -> np.ndarray:
    """FP64 networks indexed by slot id."""
    if slots is None:
        return oracle.nets_for(d, params)
    cap = cap if cap is not None else int(np.max(slots)) + 1
    nets = np.zeros((cap, oracle.net_size(d)))
    for k, s in enumerate(slots):
        nets[s] = oracle.cppn_to_net(d, params[k])
    return nets


def heterogeneous_world(W, H, n_genomes=4, seed=0, hidden=32, layers=2, precision=0,
                        capacity=None, scale=1.0) -> "wl.WorldInit":
    """A world whose infrastructure is sparse and heavy-tailed, random rotations
    and comm: exercises takeovers and every kernel position."""
    rng = np.random.default_rng(seed)
    spec = wl.WorldSpec(W, H, layers, hidden, capacity or n_genomes, precision, seed)
    E = wl.to_ledger(rng.random((H, W)))
    inf = rng.random((H, W)) ** 3 * (rng.random((H, W)) < 0.6) * 2.0
    I = wl.to_ledger(inf)
    C = rng.random((4, H, W)).astype(np.float32)
    G = rng.integers(0, n_genomes, size=(H, W)).astype(np.int32)
    R = rng.integers(0, 8, size=(H, W)).astype(np.uint8)
    params = (rng.standard_normal((n_genomes, 56)) * scale).astype(np.float32)
    return wl.WorldInit(spec, E, I, C, G, R, np.arange(n_genomes, dtype=np.int32), params)


def oracle_step_slots(d, st: "oracle.State", slots: np.ndarray, params: np.ndarray, **kw):
    """Oracle step of a state whose genome ids are sparse slot ids: networks
    are built only for the listed slots (params[k] belongs to slots[k]), the
    ids are renumbered densely for the oracle and mapped back after the step."""
    slots = np.asarray(slots, dtype=np.int64)
    lut = np.full(int(slots.max()) + 1, -1, dtype=np.int64)
    lut[slots] = np.arange(slots.size)
    dense = lut[st.G]
    assert (dense >= 0).all(), "a cell names a slot without parameters"
    nets = oracle.nets_for(d, np.asarray(params, dtype=np.float64))
    s2 = oracle.State(st.E, st.I, st.C, dense.astype(np.int32), st.R)
    ref, info = oracle.step(d, s2, nets, **kw)
    ref.G = slots[ref.G].astype(np.int32)
    return ref, info


def live_genomes(w, G: np.ndarray):
    """The slot ids a state uses and their CPPN parameters, read from the world."""
    slots = np.unique(G).astype(np.int32)
    return slots, w.get_genomes(slots).astype(np.float64)
