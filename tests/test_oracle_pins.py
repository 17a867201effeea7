"""Pins of the FP64 oracle against things other than itself (CPU only).

Each test fixes the oracle to brute force, a closed form, an invariant or a
library routine, so that a dropped term, a wrong sign or index, or a
transposed operand anywhere in it fails at least one of them.
"""
import math

import numpy as np
import pytest

import workloads as wl
from tests import brute_force as bf


def tiny_world(oracle, W, H, n_genomes=3, hidden=8, layers=2, seed=1, scale=1.0,
               sparse_infra=True):
    rng = np.random.default_rng(seed)
    E = wl.to_ledger(rng.random((H, W)))
    inf = rng.random((H, W)) ** 3
    if sparse_infra:
        inf *= rng.random((H, W)) < 0.6
    I = wl.to_ledger(inf * 2.0)
    C = rng.random((4, H, W))
    G = rng.integers(0, n_genomes, size=(H, W)).astype(np.int32)
    R = rng.integers(0, 8, size=(H, W)).astype(np.uint8)
    params = rng.standard_normal((n_genomes, 56)) * scale
    d = oracle.Desc(W, H, layers, hidden)
    return d, oracle.State(E, I, C, G, R), params


def bf_world(d, s, params, oracle):
    widths = d.widths()
    nets = [bf.build_net(list(map(float, p)), widths) for p in params]
    cycle = (d.day_period, d.day_inject, d.night_num, d.cycle_step) if d.day_period else None
    return bf.World(d.width, d.height, [int(v) for v in s.E.ravel()], [int(v) for v in s.I.ravel()],
                    [list(map(float, s.C[k].ravel())) for k in range(4)],
                    [int(v) for v in s.G.ravel()], [int(v) for v in s.R.ravel()], nets,
                    d.rho_invest, d.rho_liquidate, d.kappa_flow, cycle,
                    hard_max=d.explore_mode == 1, kappa_energy=d.kappa_energy)


# ---------------------------------------------------------------- geometry

def test_direction_and_kernel_order_tables(oracle_lib):
    """The oracle's kernel order equals sorting directions by angular distance."""
    for r in range(8):
        order = bf.kernel_order(r)
        assert [oracle_lib.kernel_dir(r, p) for p in range(1, 9)] == order
        assert order[0] == r and order[-1] == (r + 4) % 8
    assert [bf.direction_vector(d) for d in range(8)] == [
        (1, 0), (1, -1), (0, -1), (-1, -1), (-1, 0), (-1, 1), (0, 1), (1, 1)]


def test_sense_vector_by_hand(oracle_lib):
    """u[p*6+ch] enumerated by hand for one cell of a 5x4 grid."""
    d, s, _ = tiny_world(oracle_lib, 5, 4, seed=3)
    i = 0                      # corner cell: every neighbour wraps
    s.R[0, 0] = 3
    u = oracle_lib.sense(d, s, i)
    order = [3, 4, 2, 5, 1, 6, 0, 7]      # r, r+1, r-1, r+2, r-2, r+3, r-3, r+4
    vec = {0: (1, 0), 1: (1, -1), 2: (0, -1), 3: (-1, -1), 4: (-1, 0), 5: (-1, 1), 6: (0, 1),
           7: (1, 1)}
    cells = [(0, 0)] + [((vec[k][0]) % 5, (vec[k][1]) % 4) for k in order]
    for p, (x, y) in enumerate(cells):
        assert u[p * 6 + 0] == s.E[y, x] * 2.0 ** -24
        assert u[p * 6 + 1] == s.I[y, x] * 2.0 ** -24
        for c in range(4):
            assert u[p * 6 + 2 + c] == s.C[c, y, x]


# ---------------------------------------------------------------- CPPN

def test_cppn_identity_node_gives_coordinate_weights(oracle_lib):
    """Only the identity node (k=3) passes x_in: W_l[o, j] = x_{l,j} / sqrt(L_l), b = 0."""
    d = oracle_lib.Desc(4, 4, 3, 16)
    p = np.zeros(56)
    p[3 * 5 + 0] = 1.0          # h_3 = x1
    p[40 + 3] = 1.0             # weight output = h_3
    net = oracle_lib.cppn_to_net(d, p)
    for l, (w, b) in enumerate(oracle_lib.unflatten(d, net)):
        lin = d.widths()[l]
        x = -1.0 + 2.0 * np.arange(lin) / (lin - 1)
        np.testing.assert_allclose(w, np.broadcast_to(x / math.sqrt(lin), w.shape),
                                   rtol=4e-16, atol=0)
        np.testing.assert_array_equal(b, 0.0)


@pytest.mark.parametrize("node,fn", [(0, np.sin), (1, lambda s: np.exp(-s * s)), (2, np.tanh),
                                     (4, np.sin), (6, np.tanh), (7, lambda s: s)])
def test_cppn_single_node_against_numpy(oracle_lib, node, fn):
    """One hidden node wired from y_out and x_out; bias output from the same node."""
    d = oracle_lib.Desc(4, 4, 2, 32)
    p = np.zeros(56)
    p[node * 5 + 2] = 0.7       # x2 (x_out)
    p[node * 5 + 3] = -1.3      # y2 (y_out)
    p[node * 5 + 4] = 0.25      # constant input
    p[40 + node] = 2.0
    p[48 + node] = -0.5
    (w0, b0), (w1, b1) = oracle_lib.unflatten(d, oracle_lib.cppn_to_net(d, p))
    for l, (w, b) in enumerate([(w0, b0), (w1, b1)]):
        lin, lout = d.widths()[l], d.widths()[l + 1]
        yo = -1.0 + 2.0 * (l + 1) / 2
        xo = -1.0 + 2.0 * np.arange(lout) / (lout - 1)
        s = 0.7 * xo - 1.3 * yo + 0.25
        np.testing.assert_allclose(w, np.repeat((2.0 * fn(s) / math.sqrt(lin))[:, None], lin, 1),
                                   rtol=1e-15, atol=1e-15)
        np.testing.assert_allclose(b, -0.5 * fn(s), rtol=1e-15, atol=1e-15)


def test_cppn_matches_bruteforce_random(oracle_lib):
    rng = np.random.default_rng(5)
    d = oracle_lib.Desc(4, 4, 3, 16)
    p = rng.standard_normal(56)
    net = oracle_lib.cppn_to_net(d, p)
    layers = bf.build_net(list(p), d.widths())
    flat = []
    for W, b in layers:
        flat += [v for row in W for v in row] + b
    np.testing.assert_array_equal(net, np.array(flat))


# ---------------------------------------------------------------- network

@pytest.mark.parametrize("layers,hidden", [(2, 32), (3, 64)])
def test_forward_against_numpy_mlp(oracle_lib, layers, hidden):
    rng = np.random.default_rng(11)
    d = oracle_lib.Desc(4, 4, layers, hidden)
    net = oracle_lib.cppn_to_net(d, rng.standard_normal(56))
    u = rng.random(54)
    x = u
    lays = oracle_lib.unflatten(d, net)
    for k, (w, b) in enumerate(lays):
        x = w @ x + b
        if k < len(lays) - 1:
            x = np.tanh(x)
    np.testing.assert_allclose(oracle_lib.forward(d, net, u), x, rtol=1e-12, atol=1e-13)


# ---------------------------------------------------------------- whole step vs brute force

@pytest.mark.parametrize("W,H,layers,hidden", [(1, 1, 2, 8), (2, 2, 2, 8), (1, 5, 2, 8),
                                               (3, 3, 3, 8), (5, 7, 2, 8), (8, 8, 2, 16),
                                               (6, 4, 3, 8)])
def test_step_matches_bruteforce(oracle_lib, W, H, layers, hidden):
    for seed in range(3):
        d, s, params = tiny_world(oracle_lib, W, H, hidden=hidden, layers=layers, seed=seed,
                                  scale=2.0)
        nets = oracle_lib.nets_for(d, params)
        s2, info = oracle_lib.step(d, s, nets, want_act=True)
        bw = bf_world(d, s, params, oracle_lib)
        E2, I2, C2, G2, R2, tk, plans = bw.step()
        assert s2.E.ravel().tolist() == E2
        assert s2.I.ravel().tolist() == I2
        assert s2.G.ravel().tolist() == G2
        assert s2.R.ravel().tolist() == R2
        assert info["takeovers"] == tk
        np.testing.assert_allclose(s2.C.reshape(4, -1), np.array(C2), rtol=0, atol=1e-14)
        act = np.array([p["act"] for p in plans])
        np.testing.assert_allclose(info["act"].reshape(-1, 14), act, rtol=0, atol=1e-13)


@pytest.mark.parametrize("W,H,layers,hidden", [(5, 7, 2, 8), (8, 8, 2, 16), (6, 4, 3, 8),
                                               (1, 5, 2, 8), (2, 2, 2, 8)])
def test_near_tie_margins_match_bruteforce(oracle_lib, W, H, layers, hidden):
    """The oracle's near-tie report (the margins that decide which cells the
    GPU parity tests excuse from the exact G/R comparison) equals the same
    five numbers recomputed target by target from the brute-force plans:
    the neighbours' logit gaps toward the target, |v_win - I1|, the ranking
    margin, the magnitude and the decided flag.  A third of the cells carry
    no mass, so exact-zero budgets, idle neighbours and decided ties occur."""
    seen = np.zeros(5, bool)
    for seed in range(4):
        d, s, params = tiny_world(oracle_lib, W, H, hidden=hidden, layers=layers, seed=seed,
                                  scale=2.0)
        empty = np.random.default_rng(100 + seed).random((H, W)) < 0.35
        s.E[empty] = 0
        s.I[empty] = 0
        _, info = oracle_lib.step(d, s, oracle_lib.nets_for(d, params), want_margins=True)
        bw = bf_world(d, s, params, oracle_lib)
        plans = [bw.plan(i) for i in range(W * H)]
        ref = np.array([bw.margins(plans, t) for t in range(W * H)])
        got = info["margins"].reshape(-1, 5)
        np.testing.assert_array_equal(got, ref)
        seen |= [np.isfinite(ref[:, 0]).any(), np.isfinite(ref[:, 1]).any(),
                 np.isfinite(ref[:, 2]).any(), (ref[:, 4] == 1).any(), (ref[:, 4] == 0).any()]
    if W * H >= 20:
        assert seen.all(), seen


def test_bruteforce_exercises_takeovers(oracle_lib):
    """The brute-force cases above include takeovers (else they would not pin the rule)."""
    total = 0
    for seed in range(3):
        d, s, params = tiny_world(oracle_lib, 8, 8, hidden=16, seed=seed, scale=2.0)
        _, info = oracle_lib.step(d, s, oracle_lib.nets_for(d, params))
        total += info["takeovers"]
    assert total > 0


def test_step_rows_equal_full_step(oracle_lib):
    d, s, params = tiny_world(oracle_lib, 9, 11, hidden=8, seed=4, scale=2.0)
    nets = oracle_lib.nets_for(d, params)
    full, _ = oracle_lib.step(d, s, nets)
    for y0, y1 in [(0, 3), (3, 4), (8, 11), (10, 11), (0, 11)]:
        part, _ = oracle_lib.step(d, s, nets, rows=(y0, y1))
        for a, b in [(part.E, full.E), (part.I, full.I), (part.G, full.G), (part.R, full.R)]:
            np.testing.assert_array_equal(a[y0:y1], b[y0:y1])
        np.testing.assert_array_equal(part.C[:, y0:y1], full.C[:, y0:y1])


# ---------------------------------------------------------------- invariants

def test_mass_conserved_exactly_over_many_steps(oracle_lib):
    init = wl.config_plain_64()
    d = oracle_lib.Desc.from_spec(init.spec)
    nets = oracle_lib.nets_for(d, init.params)
    s = oracle_lib.State.from_init(init)
    m0 = oracle_lib.mass(s.E, s.I)
    assert m0 == int(s.E.sum() + s.I.sum())
    for _ in range(25):
        s, _ = oracle_lib.step(d, s, nets)
        assert oracle_lib.mass(s.E, s.I) == m0
        assert (s.E >= 0).all() and (s.I >= 0).all()


def test_translation_invariance(oracle_lib):
    d, s, params = tiny_world(oracle_lib, 12, 10, hidden=8, seed=7, scale=2.0)
    nets = oracle_lib.nets_for(d, params)
    out, _ = oracle_lib.step(d, s, nets)
    for dx, dy in [(1, 0), (0, 1), (5, 3), (11, 9)]:
        roll = lambda a: np.roll(a, (dy, dx), axis=(-2, -1))
        rs = oracle_lib.State(roll(s.E), roll(s.I), roll(s.C), roll(s.G), roll(s.R))
        ro, _ = oracle_lib.step(d, rs, nets)
        for a, b in [(ro.E, out.E), (ro.I, out.I), (ro.C, out.C), (ro.G, out.G), (ro.R, out.R)]:
            np.testing.assert_array_equal(a, roll(b))


def test_rotation_covariance(oracle_lib):
    """Rotating the grid 90 degrees counter-clockwise and every rotation by +2
    commutes with the step (explorer ties aside; random states have none)."""
    d, s, params = tiny_world(oracle_lib, 9, 7, hidden=8, seed=9, scale=2.0)
    nets = oracle_lib.nets_for(d, params)
    out, info = oracle_lib.step(d, s, nets, want_margins=True)
    # exact explorer ties only matter where they decide a takeover
    tied = (info["margins"][..., 2] == 0) & (out.G != s.G)
    assert not tied.any() and info["takeovers"] > 0
    rot = lambda a: np.rot90(a, 1, axes=(-2, -1)).copy()
    rs = oracle_lib.State(rot(s.E), rot(s.I), rot(s.C), rot(s.G), ((rot(s.R) + 2) % 8).astype(np.uint8))
    dr = oracle_lib.Desc(d.height, d.width, d.n_weight_layers, d.hidden)
    ro, _ = oracle_lib.step(dr, rs, nets)
    np.testing.assert_array_equal(ro.E, rot(out.E))
    np.testing.assert_array_equal(ro.I, rot(out.I))
    np.testing.assert_array_equal(ro.G, rot(out.G))
    np.testing.assert_array_equal(ro.R, (rot(out.R) + 2) % 8)
    np.testing.assert_array_equal(ro.C, rot(out.C))


# ---------------------------------------------------------------- closed forms

def test_uniform_logit_genome_closed_form(oracle_lib):
    """B = 0 makes every weight and bias 0, so a = 0: sigma = 1/2, softmax = 1/8,
    explore = position 1 = the cell's own rotation.  The step is then an
    8-neighbour diffusion of floor(F/8) written with np.roll."""
    rng = np.random.default_rng(2)
    W, H = 10, 8
    E = wl.to_ledger(rng.random((H, W)))
    I = wl.to_ledger(rng.random((H, W)) ** 4 * (rng.random((H, W)) < 0.5) * 3)
    R = rng.integers(0, 8, (H, W)).astype(np.uint8)
    G = rng.integers(0, 2, (H, W)).astype(np.int32)
    s = oracle_lib.State(E, I, rng.random((4, H, W)), G, R)
    d = oracle_lib.Desc(W, H, 2, 32)
    params = rng.standard_normal((2, 56))
    params[:, 40:] = 0.0
    out, _ = oracle_lib.step(d, s, oracle_lib.nets_for(d, params))

    rho = d.rho_invest
    x_inv = np.floor(rho * 0.5 * E.astype(np.float64)).astype(np.int64)
    x_liq = np.floor(rho * 0.5 * I.astype(np.float64)).astype(np.int64)
    E1, I1 = E - x_inv + x_liq, I + x_inv - x_liq
    F = np.floor(0.25 * I1.astype(np.float64)).astype(np.int64)
    f = F // 8
    vec = [(1, 0), (1, -1), (0, -1), (-1, -1), (-1, 0), (-1, 1), (0, 1), (1, 1)]
    # neighbour at direction d of cell (y, x) seen from the target: roll by -vec
    nb = lambda a, dd: np.roll(a, (-vec[dd][1], -vec[dd][0]), axis=(0, 1))
    I2 = I1 - 8 * f + sum(nb(f, dd) for dd in range(8))
    best = np.full((H, W), -1, np.int64)
    bestg, bestr = G.copy(), R.copy()
    for dd in range(8):
        cand = (nb(R.astype(np.int64), dd) == (dd + 4) % 8)
        v = np.where(cand, nb(f, dd), -1)
        upd = v > best
        best = np.where(upd, v, best)
        bestg = np.where(upd, nb(G, dd), bestg)
        bestr = np.where(upd, (dd + 4) % 8, bestr)
    take = (best >= 0) & (best > I1)
    G2 = np.where(take, bestg, G)
    R2 = np.where(take, bestr, R)
    np.testing.assert_array_equal(out.E, E1)
    np.testing.assert_array_equal(out.I, I2)
    np.testing.assert_array_equal(out.G, G2)
    np.testing.assert_array_equal(out.R, R2)
    np.testing.assert_array_equal(out.C, 0.5)
    assert take.sum() > 0


def test_one_by_one_world(oracle_lib):
    """Every direction aliases to the cell itself: all flow returns, no takeover."""
    for seed in range(5):
        d, s, params = tiny_world(oracle_lib, 1, 1, seed=seed, scale=3.0)
        out, info = oracle_lib.step(d, s, oracle_lib.nets_for(d, params), want_records=True)
        rec = info["records"][0, 0]
        assert out.I[0, 0] == rec["i1"] and out.E[0, 0] == rec["e1"]
        assert out.E[0, 0] + out.I[0, 0] == s.E[0, 0] + s.I[0, 0]
        assert out.G[0, 0] == s.G[0, 0] and out.R[0, 0] == s.R[0, 0]
        assert info["takeovers"] == 0


def test_zero_mass_world(oracle_lib):
    d, s, params = tiny_world(oracle_lib, 6, 5, seed=2)
    s.E[:] = 0
    s.I[:] = 0
    nets = oracle_lib.nets_for(d, params)
    out, info = oracle_lib.step(d, s, nets, want_act=True)
    assert (out.E == 0).all() and (out.I == 0).all()
    np.testing.assert_array_equal(out.G, s.G)
    np.testing.assert_array_equal(out.R, s.R)
    a = info["act"]
    np.testing.assert_allclose(np.moveaxis(out.C, 0, -1), 1 / (1 + np.exp(-a[..., 2:6])),
                               rtol=1e-15)


def test_actuation_by_hand(oracle_lib):
    """Records for a 1x1 world with hand-set weights: only biases, so a = b."""
    d = oracle_lib.Desc(1, 1, 2, 8)
    net = np.zeros(oracle_lib.net_size(d))
    bias = np.array([0.0, 2.0, -1.0, 0.0, 1.0, 3.0, 0.5, 2.5, 2.5, -1.0, 0.0, 1.0, 0.0, 0.0])
    net[-14:] = bias
    E = 1_000_003
    I = 2_000_005
    s = oracle_lib.State(np.array([[E]], np.int64), np.array([[I]], np.int64),
                         np.zeros((4, 1, 1)), np.zeros((1, 1), np.int32),
                         np.array([[5]], np.uint8))
    out, info = oracle_lib.step(d, s, net[None], want_records=True)
    rec = info["records"][0, 0]
    sg = lambda x: 1 / (1 + math.exp(-x))
    x_inv = math.floor(d.rho_invest * sg(0.0) * E)
    x_liq = math.floor(d.rho_liquidate * sg(2.0) * I)
    assert rec["e1"] == E - x_inv + x_liq and rec["i1"] == I + x_inv - x_liq
    F = math.floor(0.25 * rec["i1"])
    lg = bias[6:]
    w = np.exp(lg - lg.max())
    w /= w.sum()
    used, flows = 0, []
    for p in range(8):
        f = min(math.floor(w[p] * F), F - used)
        used += f
        flows.append(f)
    order = bf.kernel_order(5)
    for p in range(8):
        assert rec["flow"][order[p]] == flows[p]
    assert rec["explore_pos"] == 2            # logits 2.5 at p=2 and p=3: lowest wins
    assert rec["explore_dir"] == order[1]
    np.testing.assert_allclose(out.C.ravel(), [sg(-1.0), sg(0.0), sg(1.0), sg(3.0)], rtol=1e-15)


# ---------------------------------------------------------------- physics from records

def test_physics_from_records_matches_step(oracle_lib):
    d, s, params = tiny_world(oracle_lib, 7, 6, seed=8, scale=2.0)
    nets = oracle_lib.nets_for(d, params)
    out, info = oracle_lib.step(d, s, nets, want_records=True)
    rec = info["records"].ravel()
    I2, G2, R2, tk = oracle_lib.physics_from_records(d, rec["i1"], rec["flow"],
                                                     rec["explore_dir"], s.G, s.R)
    np.testing.assert_array_equal(I2, out.I)
    np.testing.assert_array_equal(G2, out.G)
    np.testing.assert_array_equal(R2, out.R)
    assert tk == info["takeovers"]


def test_physics_push_view_conserves(oracle_lib):
    """Random records: the pull-form physics equals a push-form scatter."""
    rng = np.random.default_rng(4)
    W, H = 9, 5
    d = oracle_lib.Desc(W, H)
    N = W * H
    i1 = rng.integers(0, 1 << 30, N)
    flow = rng.integers(0, 1 << 26, (N, 8))
    ed = rng.integers(0, 8, N)
    G = rng.integers(0, 5, (H, W)).astype(np.int32)
    R = rng.integers(0, 8, (H, W)).astype(np.uint8)
    I2, G2, R2, _ = oracle_lib.physics_from_records(d, i1, flow, ed, G, R)
    push = i1 - flow.sum(1)
    vec = [(1, 0), (1, -1), (0, -1), (-1, -1), (-1, 0), (-1, 1), (0, 1), (1, 1)]
    for i in range(N):
        x, y = i % W, i // W
        for k in range(8):
            j = ((y + vec[k][1]) % H) * W + (x + vec[k][0]) % W
            push[j] += flow[i, k]
    np.testing.assert_array_equal(I2.ravel(), push)
    assert I2.sum() == i1.sum()


# ---------------------------------------------------------------- buckets

@pytest.mark.parametrize("n,cap", [(0, 4), (1, 1), (1000, 7), (4096, 300)])
def test_buckets_against_numpy(oracle_lib, n, cap):
    rng = np.random.default_rng(n)
    G = rng.integers(0, cap, n).astype(np.int32)
    counts, offsets, perm = oracle_lib.buckets(G, cap)
    np.testing.assert_array_equal(counts, np.bincount(G, minlength=cap))
    np.testing.assert_array_equal(offsets, np.concatenate([[0], np.cumsum(counts)]))
    np.testing.assert_array_equal(perm, np.argsort(G, kind="stable"))


# ---------------------------------------------------------------- Philox / radiation draws

def _numpy_block(counter, key):
    """numpy's Philox4x64-10 increments its 256-bit counter before drawing."""
    v = sum(int(x) << (64 * k) for k, x in enumerate(counter))
    v = (v - 1) % (1 << 256)
    c = [(v >> (64 * k)) & ((1 << 64) - 1) for k in range(4)]
    g = np.random.Philox(key=np.array(key, np.uint64), counter=np.array(c, np.uint64))
    return g.random_raw(4)


def test_philox_against_numpy(oracle_lib):
    rng = np.random.default_rng(0)
    cases = [((0, 0, 0, 0), (0, 0)), ((1, 0, 0, 0), (0, 0)), ((0, 1, 0, 0), (7, 0)),
             ((12345, 99, 3, 0), (2 ** 64 - 1, 0))]
    for _ in range(20):
        cases.append((tuple(int(v) for v in rng.integers(0, 2 ** 63, 4, dtype=np.int64)),
                      (int(rng.integers(0, 2 ** 63)), 0)))
    for ctr, key in cases:
        np.testing.assert_array_equal(oracle_lib.philox(ctr, key), _numpy_block(ctr, key))


def test_uniforms_exact_and_open_interval(oracle_lib):
    for o in [0, 1, (1 << 41) - 1, 1 << 41, (1 << 64) - 1, 0x123456789ABCDEF0]:
        u = oracle_lib.uniform(o)
        assert 0.0 < u < 1.0
        assert float(np.float32(u)) == u                  # exact in FP32
        assert u == (2 * (o >> 41) + 1) / 2.0 ** 24


def test_mutation_normals_are_box_muller_of_the_blocks(oracle_lib):
    seed, i, s = 77, 1234, 9
    z = oracle_lib.mutation_normals(seed, i, s)
    for b in range(14):
        o = _numpy_block((i, s, 1 + b, 0), (seed, 0))
        u = [(2 * (int(v) >> 41) + 1) / 2.0 ** 24 for v in o]
        for h in range(2):
            r = math.sqrt(-2 * math.log(u[2 * h]))
            assert z[4 * b + 2 * h] == pytest.approx(r * math.cos(2 * math.pi * u[2 * h + 1]), abs=1e-15)
            assert z[4 * b + 2 * h + 1] == pytest.approx(r * math.sin(2 * math.pi * u[2 * h + 1]), abs=1e-15)


def test_mutation_normals_distribution(oracle_lib):
    from scipy import stats
    z = np.concatenate([oracle_lib.mutation_normals(3, i, 1) for i in range(4000)])
    assert stats.kstest(z, "norm").pvalue > 1e-3
    assert abs(z.mean()) < 0.02 and abs(z.std() - 1) < 0.02


def test_hit_threshold(oracle_lib):
    assert oracle_lib.hit_threshold(0.0) == 0
    assert oracle_lib.hit_threshold(1e-4) == math.floor(1e-4 * 2.0 ** 64)
    assert oracle_lib.hit_threshold(0.5) == 1 << 63
    assert oracle_lib.hit_threshold(1.0) == 2 ** 64 - 1


def test_radiate_against_bruteforce(oracle_lib):
    """Hit set from numpy Philox; slot assignment and parameters re-derived."""
    rng = np.random.default_rng(6)
    W, H, cap = 40, 30, 20
    G = rng.integers(0, 8, (H, W)).astype(np.int32)
    G[G == 5] = 4                       # leave a hole below the highest id
    params = np.zeros((cap, 56))
    params[:8] = rng.standard_normal((8, 56))
    seed, s, rate, sigma = 42, 17, 0.02, 0.1
    G2, P2, (hc, hs), dropped = oracle_lib.radiate(G, cap, params, seed, s, rate, sigma)
    T = math.floor(rate * 2.0 ** 64)
    # cells 4k..4k+3 take the four words of the block at counter (k, s, 0, 0)
    hits = [i for i in range(W * H) if int(_numpy_block((i // 4, s, 0, 0), (seed, 0))[i % 4]) < T]
    free = [g for g in range(cap) if g not in set(G.ravel().tolist())]
    assert hc.tolist() == hits
    assert len(hits) > len(free)        # capacity exhaustion exercised
    assert dropped == len(hits) - len(free)
    Gf = G.ravel().copy()
    for k, i in enumerate(hits):
        if k < len(free):
            assert hs[k] == free[k]
            z = oracle_lib.mutation_normals(seed, i, s)
            np.testing.assert_allclose(P2[free[k]], params[Gf[i]] + sigma * z, rtol=0, atol=1e-15)
            Gf[i] = free[k]
        else:
            assert hs[k] == -1
    np.testing.assert_array_equal(G2.ravel(), Gf)


def test_hit_counts_binomial(oracle_lib):
    """Hits per call follow Binomial(N, rate): one draw per cell."""
    W = H = 200
    G = np.zeros((H, W), np.int32)
    counts = []
    for s in range(1, 9):
        _, _, (hc, _), _ = oracle_lib.radiate(G, 2, np.zeros((2, 56)), 5, s, 0.01, 0.1)
        counts.append(len(hc))
    n, p = W * H, 0.01
    mean = np.mean(counts)
    assert abs(mean - n * p) < 4 * math.sqrt(n * p * (1 - p) / len(counts))


# ---------------------------------------------------------------- day / night cycle

@pytest.mark.parametrize("period,q", [(8, 0), (8, 1), (8, 3), (8, 4), (8, 6), (10, 5), (7, 3)])
def test_day_night_step_matches_bruteforce(oracle_lib, period, q):
    """With the cycle on, every phase (noon, morning, dusk, midnight, and odd
    periods whose midnight falls between steps) matches the brute force."""
    for seed in range(2):
        d, s, params = tiny_world(oracle_lib, 6, 5, hidden=8, seed=seed, scale=2.0)
        d.day_period, d.day_inject, d.night_num, d.cycle_step = period, 3_000_017, 40_000, 3 * period + q
        s2, info = oracle_lib.step(d, s, oracle_lib.nets_for(d, params))
        E2, I2, C2, G2, R2, tk, _ = bf_world(d, s, params, oracle_lib).step()
        assert s2.E.ravel().tolist() == E2
        assert s2.I.ravel().tolist() == I2
        assert s2.G.ravel().tolist() == G2 and s2.R.ravel().tolist() == R2


def test_day_night_uniform_world_closed_form(oracle_lib):
    """A uniform world under a genome whose CPPN output layer is zero (a = 0:
    sigmoid 1/2, softmax 1/8): every cell's E1 = E - floor(E/20) + floor(I/20)
    and the cycle adds floor(A L / P) by day or removes
    floor(floor(E1 num / 65536) (-L) / P) by night, with L = P at noon, P/2 an
    eighth of a period later, 0 at a quarter, -P at midnight."""
    W = H = 6
    e, i = 5_000_000, 3_000_000
    E = np.full((H, W), e, np.int64)
    I = np.full((H, W), i, np.int64)
    C = np.zeros((4, H, W))
    G = np.zeros((H, W), np.int32)
    R = np.zeros((H, W), np.uint8)
    p = np.random.default_rng(1).standard_normal(56)
    p[40:] = 0.0
    e1 = e - e // 20 + i // 20
    A, num, P = 1_000_003, 30_000, 16
    for q, L in [(0, 16), (2, 8), (4, 0), (6, -8), (8, -16), (12, 0), (14, 8)]:
        d = oracle_lib.Desc(W, H, 2, 8, day_period=P, day_inject=A, night_num=num, cycle_step=5 * P + q)
        s2, info = oracle_lib.step(d, oracle_lib.State(E, I, C, G, R), oracle_lib.nets_for(d, p[None]))
        gain = A * L // P if L > 0 else 0
        loss = (e1 * num // 65536) * (-L) // P if L < 0 else 0
        assert (s2.E == e1 + gain - loss).all(), (q, int(s2.E[0, 0]), e1, gain, loss)
        assert info["injected"] == gain * W * H and info["removed"] == loss * W * H
    # midnight with the whole fraction removes all the energy
    d = oracle_lib.Desc(W, H, 2, 8, day_period=P, day_inject=A, night_num=65536, cycle_step=P // 2)
    s2, _ = oracle_lib.step(d, oracle_lib.State(E, I, C, G, R), oracle_lib.nets_for(d, p[None]))
    assert (s2.E == 0).all()


def test_day_night_ledger_balance_over_cycles(oracle_lib):
    """Over two periods of the 64x64 workload the total mass moves by exactly
    the injected minus the removed quanta at every step, and a full period's
    injection with P = 4 is one noon's worth (A per cell)."""
    init = wl.config_plain_64()
    d = oracle_lib.Desc.from_spec(init.spec)
    nets = oracle_lib.nets_for(d, init.params)
    s = oracle_lib.State.from_init(init)
    d.day_period, d.day_inject, d.night_num = 4, 2_000_000, 20_000
    m = oracle_lib.mass(s.E, s.I)
    inj_total = 0
    for k in range(8):
        d.cycle_step = k
        s, info = oracle_lib.step(d, s, nets)
        m2 = oracle_lib.mass(s.E, s.I)
        assert m2 == m + info["injected"] - info["removed"]
        assert (info["removed"] > 0) == (k % 4 == 2)
        m = m2
        inj_total += info["injected"]
    assert inj_total == 2 * 2_000_000 * 64 * 64


def test_day_night_off_is_the_plain_step(oracle_lib):
    d, s, params = tiny_world(oracle_lib, 9, 7, hidden=8, seed=3)
    nets = oracle_lib.nets_for(d, params)
    a, ia = oracle_lib.step(d, s, nets, want_records=True)
    d.day_inject, d.night_num, d.cycle_step = 123456, 4000, 17   # period 0: no cycle
    b, ib = oracle_lib.step(d, s, nets)
    for x, y in [(a.E, b.E), (a.I, b.I), (a.G, b.G), (a.R, b.R)]:
        np.testing.assert_array_equal(x, y)
    np.testing.assert_array_equal(a.E, ia["records"]["e1"])
    assert ib["injected"] == 0 and ib["removed"] == 0


# ---------------------------------------------------------------- physics variants

@pytest.mark.parametrize("hard,kappa_e,cycle", [(True, 0.0, False), (False, 0.3, False), (True, 0.25, False),
                                                 (True, 0.2, True)])
def test_physics_variants_match_bruteforce(oracle_lib, hard, kappa_e, cycle):
    """Hard-max exploration (the whole budget to the maximal explore
    actuator) and energy transport along the flow directions, alone, together
    and with the day / night cycle, against the brute force on tiny grids
    (including 1x1 and 2x2, where directions alias)."""
    for (W, H) in [(1, 1), (2, 2), (5, 7), (6, 4)]:
        for seed in range(2):
            d, s, params = tiny_world(oracle_lib, W, H, hidden=8, seed=seed, scale=2.0)
            d.explore_mode, d.kappa_energy = (1 if hard else 0), kappa_e
            if cycle:
                d.day_period, d.day_inject, d.night_num, d.cycle_step = 6, 1_000_003, 50_000, 4
            s2, info = oracle_lib.step(d, s, oracle_lib.nets_for(d, params))
            E2, I2, C2, G2, R2, tk, _ = bf_world(d, s, params, oracle_lib).step()
            assert s2.E.ravel().tolist() == E2, (W, H, seed)
            assert s2.I.ravel().tolist() == I2
            assert s2.G.ravel().tolist() == G2 and s2.R.ravel().tolist() == R2
            assert info["takeovers"] == tk


def test_physics_variants_conserve_mass(oracle_lib):
    init = wl.config_plain_64()
    d = oracle_lib.Desc.from_spec(init.spec)
    d.explore_mode, d.kappa_energy = 1, 0.25
    nets = oracle_lib.nets_for(d, init.params)
    s = oracle_lib.State.from_init(init)
    m0 = oracle_lib.mass(s.E, s.I)
    e0 = int(s.E.sum())
    moved = 0
    for _ in range(10):
        s2, _ = oracle_lib.step(d, s, nets)
        assert oracle_lib.mass(s2.E, s2.I) == m0
        assert (s2.E >= 0).all() and (s2.I >= 0).all()
        moved += int(np.abs(s2.E - s.E).sum())
        s = s2
    assert moved > 0


def test_hard_max_uniform_logit_closed_form(oracle_lib):
    """Zero output layer (a = 0): the maximal explore actuator is position 1,
    the cell's own rotation, so under hard max every cell sends its whole
    budget F = floor(I1 / 4) to the neighbour its rotation points at, and its
    energy budget floor(kappa_E E1) the same way: two np.roll sums."""
    rng = np.random.default_rng(4)
    W, H = 7, 5
    E = wl.to_ledger(rng.random((H, W)))
    I = wl.to_ledger(rng.random((H, W)))
    C = rng.random((4, H, W))
    G = np.zeros((H, W), np.int32)
    R = rng.integers(0, 8, (H, W)).astype(np.uint8)
    p = rng.standard_normal(56)
    p[40:] = 0.0
    d = oracle_lib.Desc(W, H, 2, 8, explore_mode=1, kappa_energy=0.5)
    s2, _ = oracle_lib.step(d, oracle_lib.State(E, I, C, G, R), oracle_lib.nets_for(d, p[None]))
    e1 = E - E // 20 + I // 20
    i1 = I + E // 20 - I // 20
    F = i1 // 4
    FE = np.floor(0.5 * e1.astype(np.float64)).astype(np.int64)
    i2 = i1 - F
    e2 = e1 - FE
    dirs = [(1, 0), (1, -1), (0, -1), (-1, -1), (-1, 0), (-1, 1), (0, 1), (1, 1)]
    for r, (dx, dy) in enumerate(dirs):
        on = R == r
        i2 = i2 + np.roll(np.where(on, F, 0), (dy, dx), axis=(0, 1))
        e2 = e2 + np.roll(np.where(on, FE, 0), (dy, dx), axis=(0, 1))
    np.testing.assert_array_equal(s2.I, i2)
    np.testing.assert_array_equal(s2.E, e2)


# ---------------------------------------------------------------- genetic distance, phylogeny

def test_genetic_distance_properties(oracle_lib):
    """NEAT compatibility distance with all genes matching: zero for a genome
    and itself, c3 |t| for a uniform shift by t, symmetric, the triangle
    inequality, and numpy's mean absolute difference."""
    rng = np.random.default_rng(12)
    P = rng.standard_normal((6, 56))
    assert oracle_lib.genetic_distance(P[0], P[0], 0.4) == 0.0
    assert abs(oracle_lib.genetic_distance(P[1], P[1] + 0.375, 2.0) - 0.75) < 1e-15
    for i in range(6):
        for j in range(6):
            dij = oracle_lib.genetic_distance(P[i], P[j], 1.5)
            assert dij == oracle_lib.genetic_distance(P[j], P[i], 1.5)
            assert abs(dij - 1.5 * np.mean(np.abs(P[i] - P[j]))) < 1e-14
            for k in range(6):
                assert dij <= oracle_lib.genetic_distance(P[i], P[k], 1.5) + \
                    oracle_lib.genetic_distance(P[k], P[j], 1.5) + 1e-14


def test_births_follow_the_radiated_cells(oracle_lib):
    """A radiation call's births: the parent of each new slot is the genome its
    cell held before the call, and the new slot is the one the cell holds
    after it."""
    rng = np.random.default_rng(3)
    G = rng.integers(0, 5, (30, 40)).astype(np.int32)
    cap = 64
    P = np.zeros((cap, 56))
    P[:5] = rng.standard_normal((5, 56))
    G2, P2, hits, dropped = oracle_lib.radiate(G, cap, P, 7, 3, 0.02, 0.1)
    cells, parents, slots = oracle_lib.births(G, hits)
    assert len(cells) > 10 and dropped == 0
    np.testing.assert_array_equal(G.ravel()[cells], parents)
    np.testing.assert_array_equal(G2.ravel()[cells], slots)
    assert np.all(np.diff(cells) > 0) and len(np.unique(slots)) == len(slots)
    # each child is its parent plus the mutation: genetic distance sigma E|z| on average
    d = np.array([oracle_lib.genetic_distance(P2[s], P[p]) for s, p in zip(slots, parents)])
    assert 0.05 < d.mean() < 0.11


# ---------------------------------------------------------------- merging (NEAT crossover)

def _facing(i, r, W, H):
    """The neighbour cell i faces: direction r points 45 r degrees
    counter-clockwise from +x with y pointing down, so its unit step is
    (round(cos), -round(sin)) of that angle."""
    ang = math.radians(45 * int(r))
    dx, dy = int(round(math.cos(ang))), -int(round(math.sin(ang)))
    x, y = i % W, i // W
    return ((y + dy) % H) * W + (x + dx) % W


def _merge_world(seed, W=40, H=30, n_genomes=6, cap=24):
    rng = np.random.default_rng(seed)
    G = rng.integers(0, n_genomes, (H, W)).astype(np.int32)
    G[G == 3] = 2                        # leave a hole below the highest id
    R = rng.integers(0, 8, (H, W)).astype(np.uint8)
    P = np.zeros((cap, 56))
    P[:n_genomes] = rng.standard_normal((n_genomes, 56))
    return G, R, P


def test_merge_against_bruteforce(oracle_lib):
    """Candidates from numpy Philox, partner from the trigonometric direction,
    the snapshot rule (a partner's genome as it was before the call), slot
    assignment in cell order, capacity exhaustion and the gene-wise crossover
    re-derived from the mask block."""
    W, H, cap = 40, 30, 150
    G, R, P = _merge_world(5, W, H, cap=cap)
    seed, s, rate = 99, 12, 0.2
    d = oracle_lib.Desc(W, H)
    G2, P2, (hc, hs, ha, hb), dropped = oracle_lib.merge(d, G, R, cap, P, seed, s, rate)
    T = math.floor(rate * 2.0 ** 64)
    Gf = G.ravel()
    cand = [i for i in range(W * H) if int(_numpy_block((i // 4, s, 0, 1), (seed, 0))[i % 4]) < T]
    merges = [i for i in cand if Gf[_facing(i, R.ravel()[i], W, H)] != Gf[i]]
    assert len(cand) > len(merges) > 0  # same-genome partners are skipped
    free = [g for g in range(cap) if g not in set(Gf.tolist())]
    assert len(merges) > len(free)      # capacity exhaustion exercised
    assert hc.tolist() == merges and dropped == len(merges) - len(free)
    # some partner is itself an earlier merge: the snapshot rule matters
    assert set(_facing(i, R.ravel()[i], W, H) for i in merges[:len(free)]) & set(merges[:len(free)])
    Gexp = Gf.copy()
    for k, i in enumerate(merges):
        a, b = Gf[i], Gf[_facing(i, R.ravel()[i], W, H)]
        assert (ha[k], hb[k]) == (a, b)
        if k >= len(free):
            assert hs[k] == -1
            continue
        assert hs[k] == free[k]
        mask = int(_numpy_block((i, s, 0, 2), (seed, 0))[0])
        child = np.array([P[b, m] if (mask >> m) & 1 else P[a, m] for m in range(56)])
        np.testing.assert_array_equal(P2[free[k]], child)
        Gexp[i] = free[k]
    np.testing.assert_array_equal(G2.ravel(), Gexp)
    # the parents' parameters are untouched
    used = np.unique(Gf)
    np.testing.assert_array_equal(P2[used], P[used])


def test_merge_degenerate_cases(oracle_lib):
    """Rate 0 merges nothing; a world of one genome never merges at any rate;
    rate 1 makes every cell with a foreign partner a candidate."""
    W, H, cap = 16, 12, 400
    G, R, P = _merge_world(8, W, H, cap=cap)
    d = oracle_lib.Desc(W, H)
    G2, P2, hits, dropped = oracle_lib.merge(d, G, R, cap, P, 1, 2, 0.0)
    assert len(hits[0]) == 0 and dropped == 0
    np.testing.assert_array_equal(G2, G)
    np.testing.assert_array_equal(P2, P)
    Gu = np.full_like(G, 4)
    G2, _, hits, _ = oracle_lib.merge(d, Gu, R, cap, P, 1, 2, 1.0)
    assert len(hits[0]) == 0
    np.testing.assert_array_equal(G2, Gu)
    G2, P2, (hc, hs, ha, hb), dropped = oracle_lib.merge(d, G, R, cap, P, 1, 2, 1.0)
    Gf = G.ravel()
    expect = [i for i in range(W * H) if Gf[_facing(i, R.ravel()[i], W, H)] != Gf[i]]
    assert hc.tolist() == expect and dropped == 0
    free = [g for g in range(cap) if g not in set(Gf.tolist())]
    np.testing.assert_array_equal(G2.ravel()[expect], free[:len(expect)])


def test_merge_crossover_is_gene_wise_and_fair(oracle_lib):
    """Every child gene equals one parent's gene at that position, and over
    many merges each parent supplies half of the genes (binomial bound)."""
    W, H, cap = 64, 64, 4096
    G, R, P = _merge_world(21, W, H, n_genomes=6, cap=cap)
    d = oracle_lib.Desc(W, H)
    G2, P2, (hc, hs, ha, hb), dropped = oracle_lib.merge(d, G, R, cap, P, 4, 40, 0.2)
    took = hs >= 0
    assert took.sum() > 300 and dropped == 0
    child, A, B = P2[hs[took]], P[ha[took]], P[hb[took]]
    from_a, from_b = child == A, child == B
    assert np.all(from_a | from_b)
    n = from_b.size
    k = from_b.sum()
    assert abs(k - n / 2) < 5 * math.sqrt(n / 4)


def test_merge_births_record_both_parents(oracle_lib):
    """The merges' new slots are distinct, listed in cell order, and each new
    genome sits at distance at most that of its parents from either parent
    (a crossover never leaves the box the parents span)."""
    W, H, cap = 40, 30, 128
    G, R, P = _merge_world(30, W, H, cap=cap)
    d = oracle_lib.Desc(W, H)
    G2, P2, (hc, hs, ha, hb), dropped = oracle_lib.merge(d, G, R, cap, P, 3, 9, 0.05)
    assert dropped == 0 and len(hc) > 10
    assert np.all(np.diff(hc) > 0) and len(np.unique(hs)) == len(hs)
    np.testing.assert_array_equal(G2.ravel()[hc], hs)
    for s_, a, b in zip(hs, ha, hb):
        dab = oracle_lib.genetic_distance(P[a], P[b])
        assert oracle_lib.genetic_distance(P2[s_], P[a]) + oracle_lib.genetic_distance(P2[s_], P[b]) \
            == pytest.approx(dab, rel=1e-12)


# ---------------------------------------------------------------- structural genes (NEAT)

def _rand_ext(rng, n, p_on=0.5):
    e = oracle_lib_ext_empty(n)
    for k in range(n):
        e[k]["conn_mask"] = int(sum(1 << c for c in range(10) if rng.random() < p_on))
        e[k]["node_mask"] = int(sum(1 << q for q in range(16) if rng.random() < p_on))
        e[k]["node_act"] = int(rng.integers(0, 1 << 32, dtype=np.uint64))
        e[k]["conn_w"] = rng.standard_normal(10)
        e[k]["node_in"] = rng.standard_normal(16)
        e[k]["node_out"] = rng.standard_normal(16)
    return e


def oracle_lib_ext_empty(n):
    import oracle
    return oracle.empty_ext(n)


def _bf_cppn_x(p, e, z):
    """The structural CPPN from its definition, scalar Python."""
    fns = [math.sin, lambda s: math.exp(-s * s), math.tanh, lambda s: s]
    h = [fns[k % 4](sum(p[5 * k + m] * z[m] for m in range(5))) for k in range(8)]
    out = []
    for o in range(2):
        acc = 0.0
        for j in range(8):
            k = 2 * j + o
            if (int(e["node_mask"]) >> k) & 1:
                act = (int(e["node_act"]) >> (2 * k)) & 3
                acc += e["node_out"][k] * fns[act](e["node_in"][k] * h[j])
            else:
                acc += p[40 + 8 * o + j] * h[j]
        for m in range(5):
            if (int(e["conn_mask"]) >> (5 * o + m)) & 1:
                acc += e["conn_w"][5 * o + m] * z[m]
        out.append(acc)
    return out


def test_structural_cppn_against_bruteforce(oracle_lib):
    """Networks of genomes with random structural genes (direct connections,
    added nodes with every activation) against a scalar evaluation of the
    definition at every substrate query; empty structure is the base CPPN."""
    rng = np.random.default_rng(41)
    d = oracle_lib.Desc(6, 6, 2, 32)
    for trial in range(4):
        p = rng.standard_normal(56)
        e = _rand_ext(rng, 1)[0]
        net = oracle_lib.cppn_to_net_x(d, p, e)
        widths = [54, 32, 14]
        off = 0
        for l in range(2):
            Li, Lo = widths[l], widths[l + 1]
            yi, yo = -1 + 2 * l / 2, -1 + 2 * (l + 1) / 2
            for o in range(0, Lo, 5):
                for j in range(0, Li, 7):
                    z = [-1 + 2 * j / (Li - 1), yi, -1 + 2 * o / (Lo - 1), yo, 1.0]
                    ref = _bf_cppn_x(p, e, z)[0] / math.sqrt(Li)
                    assert abs(net[off + o * Li + j] - ref) <= 1e-12 * max(1.0, abs(ref))
            off += Lo * Li
            for o in range(Lo):
                z = [0.0, yi, -1 + 2 * o / (Lo - 1), yo, 1.0]
                ref = _bf_cppn_x(p, e, z)[1]
                assert abs(net[off + o] - ref) <= 1e-12 * max(1.0, abs(ref))
            off += Lo
        np.testing.assert_array_equal(oracle_lib.cppn_to_net_x(d, p, oracle_lib.empty_ext(1)[0]),
                                      oracle_lib.cppn_to_net(d, p))


def test_structural_radiation_against_bruteforce(oracle_lib):
    """Radiation with structural mutation: base genes as plain radiation,
    the enabled structural genes' weights perturbed by Box-Muller normals of
    the blocks (i, s, 16 + b, 0) (disabled ones kept), and the
    add-connection / add-node decisions, positions, new weights and
    activations from the block (i, s, 15, 0) (numpy Philox)."""
    rng = np.random.default_rng(44)
    W, H, cap = 40, 30, 160
    G = rng.integers(0, 6, (H, W)).astype(np.int32)
    P = np.zeros((cap, 56))
    P[:6] = rng.standard_normal((6, 56))
    X = oracle_lib.empty_ext(cap)
    X[:6] = _rand_ext(rng, 6, 0.3)
    seed, s, rate, sigma, pc, pn = 5, 11, 0.05, 0.1, 0.5, 0.5
    G2, P2, X2, (hc, hs), dropped = oracle_lib.radiate_x(G, cap, P, X, seed, s, rate, sigma, pc, pn)
    Gb, Pb, (hcb, hsb), db = oracle_lib.radiate(G, cap, P, seed, s, rate, sigma)
    np.testing.assert_array_equal(G2, Gb)
    np.testing.assert_array_equal(P2, Pb)
    assert hc.tolist() == hcb.tolist() and dropped == db == 0 and len(hc) > 40
    Tc, Tn = math.floor(pc * 2.0 ** 64), math.floor(pn * 2.0 ** 64)
    n_conn = n_node = 0
    for i, slot in zip(hc, hs):
        par = G.ravel()[i]
        z = []
        for b in range(11):
            o = _numpy_block((int(i), s, 16 + b, 0), (seed, 0))
            for h in range(2):
                u1 = (2 * (int(o[2 * h]) >> 41) + 1) * 2.0 ** -24
                u2 = (2 * (int(o[2 * h + 1]) >> 41) + 1) * 2.0 ** -24
                rr = math.sqrt(-2 * math.log(u1))
                z += [rr * math.cos(2 * math.pi * u2), rr * math.sin(2 * math.pi * u2)]
        w_par = np.concatenate([X[par]["conn_w"], X[par]["node_in"], X[par]["node_out"]])
        cm, nm, na = int(X[par]["conn_mask"]), int(X[par]["node_mask"]), int(X[par]["node_act"])
        on = np.array([(cm >> m) & 1 for m in range(10)] + [(nm >> q) & 1 for q in range(16)] * 2, bool)
        w_exp = np.where(on, w_par + sigma * np.array(z[:42]), w_par)
        o = [int(v) for v in _numpy_block((int(i), s, 15, 0), (seed, 0))]
        if o[0] < Tc:
            cc = (o[2] & 0xffff) % 10
            if not (cm >> cc) & 1:
                cm |= 1 << cc
                w_exp[cc] = sigma * z[cc]
                n_conn += 1
        if o[1] < Tn:
            k = ((o[2] >> 16) & 0xffff) % 16
            if not (nm >> k) & 1:
                nm |= 1 << k
                na = (na & ~(3 << (2 * k))) | ((o[3] & 3) << (2 * k))
                w_exp[10 + k] = 1.0
                w_exp[26 + k] = P2[slot, 40 + 8 * (k & 1) + (k >> 1)]
                n_node += 1
        c = X2[slot]
        assert (int(c["conn_mask"]), int(c["node_mask"]), int(c["node_act"])) == (cm, nm, na)
        got = np.concatenate([c["conn_w"], c["node_in"], c["node_out"]])
        np.testing.assert_allclose(got, w_exp, rtol=0, atol=1e-14)
    assert n_conn > 10 and n_node > 10


def test_add_node_with_identity_keeps_the_network(oracle_lib):
    """NEAT's add-node: the split connection's weight moves to the new node's
    out-connection and its in-weight is 1, so with the identity activation
    the network is unchanged (sigma 0, every hit adds a node)."""
    rng = np.random.default_rng(45)
    W, H, cap = 24, 20, 600
    G = rng.integers(0, 3, (H, W)).astype(np.int32)
    P = np.zeros((cap, 56))
    P[:3] = rng.standard_normal((3, 56))
    X = oracle_lib.empty_ext(cap)
    d = oracle_lib.Desc(6, 6, 2, 32)
    G2, P2, X2, (hc, hs), dropped = oracle_lib.radiate_x(G, cap, P, X, 3, 4, 0.5, 0.0, 0.0, 1.0)
    n_id = 0
    for i, slot in zip(hc, hs):
        e = X2[slot]
        assert bin(int(e["node_mask"])).count("1") == 1 and int(e["conn_mask"]) == 0
        k = int(e["node_mask"]).bit_length() - 1
        if (int(e["node_act"]) >> (2 * k)) & 3 == 3:
            np.testing.assert_allclose(oracle_lib.cppn_to_net_x(d, P2[slot], e),
                                       oracle_lib.cppn_to_net(d, P[G.ravel()[i]]), rtol=0, atol=1e-14)
            n_id += 1
    assert n_id > 10


def test_structural_merge_against_bruteforce(oracle_lib):
    """Merging with structural genes: base genes as plain merging; each
    direct-connection and added-node position whole from b where bit c of
    word 1 (bit k of word 2) of the block (i, s, 0, 2) is set, else from a."""
    W, H, cap = 40, 30, 300
    G, R, P = _merge_world(7, W, H, cap=cap)
    rng = np.random.default_rng(46)
    X = oracle_lib.empty_ext(cap)
    X[:6] = _rand_ext(rng, 6, 0.5)
    d = oracle_lib.Desc(W, H)
    seed, s = 9, 3
    G2, P2, X2, (hc, hs, ha, hb), dropped = oracle_lib.merge_x(d, G, R, cap, P, X, seed, s, 0.1)
    Gm, Pm, (hcm, hsm, ham, hbm), dm = oracle_lib.merge(d, G, R, cap, P, seed, s, 0.1)
    np.testing.assert_array_equal(G2, Gm)
    np.testing.assert_array_equal(P2, Pm)
    assert len(hc) > 50 and dropped == dm
    for i, slot, a, b in zip(hc, hs, ha, hb):
        if slot < 0:
            continue
        o = [int(v) for v in _numpy_block((int(i), s, 0, 2), (seed, 0))]
        c = X2[slot]
        for q in range(10):
            src = X[b] if (o[1] >> q) & 1 else X[a]
            assert ((int(c["conn_mask"]) >> q) & 1) == ((int(src["conn_mask"]) >> q) & 1)
            assert c["conn_w"][q] == src["conn_w"][q]
        for q in range(16):
            src = X[b] if (o[2] >> q) & 1 else X[a]
            assert ((int(c["node_mask"]) >> q) & 1) == ((int(src["node_mask"]) >> q) & 1)
            assert ((int(c["node_act"]) >> (2 * q)) & 3) == ((int(src["node_act"]) >> (2 * q)) & 3)
            assert (c["node_in"][q], c["node_out"][q]) == (src["node_in"][q], src["node_out"][q])


def _bf_distance(pa, ea, pb, eb, c1, c2, c3):
    """NEAT compatibility distance from its definition over innovation-numbered genes."""
    def genes(p, e):
        g = {m: p[m] for m in range(56)}
        for c in range(10):
            if (int(e["conn_mask"]) >> c) & 1:
                g[56 + c] = e["conn_w"][c]
        for q in range(16):
            if (int(e["node_mask"]) >> q) & 1:
                g[66 + 2 * q] = e["node_in"][q]
                g[67 + 2 * q] = e["node_out"][q]
        return g
    A, B = genes(pa, ea), genes(pb, eb)
    cut = min(max(A), max(B))
    match = [k for k in A if k in B]
    other = [k for k in set(A) ^ set(B)]
    E = sum(1 for k in other if k > cut)
    D = len(other) - E
    N = max(len(A), len(B))
    Wbar = sum(abs(A[k] - B[k]) for k in match) / len(match)
    return c1 * E / N + c2 * D / N + c3 * Wbar


def test_structural_genetic_distance_against_definition(oracle_lib):
    rng = np.random.default_rng(47)
    for _ in range(40):
        pa, pb = rng.standard_normal(56), rng.standard_normal(56)
        ea, eb = _rand_ext(rng, 2, rng.random())
        for c1, c2, c3 in [(1.0, 1.0, 0.4), (2.0, 0.5, 1.0)]:
            got = oracle_lib.genetic_distance_x(pa, ea, pb, eb, c1, c2, c3)
            assert abs(got - _bf_distance(pa, ea, pb, eb, c1, c2, c3)) < 1e-12
            assert got == oracle_lib.genetic_distance_x(pb, eb, pa, ea, c1, c2, c3)
        assert oracle_lib.genetic_distance_x(pa, ea, pa, ea) == 0.0
    e0 = oracle_lib.empty_ext(1)[0]
    assert abs(oracle_lib.genetic_distance_x(pa, e0, pb, e0, 1, 1, 0.7)
               - oracle_lib.genetic_distance(pa, pb, 0.7)) < 1e-15
