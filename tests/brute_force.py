"""Pure-Python brute force of one update step, written pull-from-definition.

A test pin for the C oracle on tiny grids.  It shares nothing with the
oracle: the direction vectors come from the 45-degree angles, the kernel order
from sorting directions by angular distance to the cell's rotation, and each
target cell recomputes the actions of every neighbour it pulls from.  Every
number is a Python float (IEEE double) or int.
"""
from __future__ import annotations

import math

Q = 2.0 ** -24


def direction_vector(d: int) -> tuple[int, int]:
    """Direction d points 45*d degrees counter-clockwise from +x on a screen
    whose y axis points down."""
    th = math.radians(45.0 * d)
    c, s = math.cos(th), math.sin(th)
    dx = 0 if abs(c) < 1e-9 else (1 if c > 0 else -1)
    dy = 0 if abs(s) < 1e-9 else (-1 if s > 0 else 1)
    return dx, dy


def kernel_order(r: int) -> list[int]:
    """The 8 neighbour directions by increasing angular distance to rotation r;
    within an equal-distance pair the counter-clockwise one comes first."""
    def key(d):
        ccw = (d - r) % 8
        dist = min(ccw, 8 - ccw)
        return (dist, 0 if ccw == dist else 1)
    return sorted(range(8), key=key)


def cppn_eval(p, z):
    zz = list(z) + [1.0]
    acts = [math.sin, lambda s: math.exp(-s * s), math.tanh, lambda s: s]
    h = []
    for k in range(8):
        s = 0.0
        for m in range(5):
            s += p[k * 5 + m] * zz[m]
        h.append(acts[k % 4](s))
    out = []
    for o in range(2):
        s = 0.0
        for k in range(8):
            s += p[40 + o * 8 + k] * h[k]
        out.append(s)
    return out


def build_net(p, widths):
    """HyperNEAT: layer l neurons at x = -1 + 2j/(L-1), y = -1 + 2l/n."""
    n = len(widths) - 1
    layers = []
    for l in range(n):
        lin, lout = widths[l], widths[l + 1]
        yi, yo = -1.0 + 2.0 * l / n, -1.0 + 2.0 * (l + 1) / n
        W = [[cppn_eval(p, (-1.0 + 2.0 * j / (lin - 1), yi, -1.0 + 2.0 * o / (lout - 1), yo))[0]
              * (1.0 / math.sqrt(lin)) for j in range(lin)] for o in range(lout)]
        b = [cppn_eval(p, (0.0, yi, -1.0 + 2.0 * o / (lout - 1), yo))[1] for o in range(lout)]
        layers.append((W, b))
    return layers


def run_net(layers, u):
    x = list(u)
    for li, (W, b) in enumerate(layers):
        y = []
        for o in range(len(W)):
            s = 0.0
            for j in range(len(x)):
                s += W[o][j] * x[j]
            s += b[o]
            y.append(s if li == len(layers) - 1 else math.tanh(s))
        x = y
    return x


def sig(x):
    return 1.0 / (1.0 + math.exp(-x))


# Relative perturbation of a floored argument within which an FP32 evaluation
# of the same step may move it (the near-tie report of the parity tests).
FLOOR_REL = 1e-3


def floor_decided(x):
    """Every value within FLOOR_REL * x of x has the same floor, or x is an
    exact zero."""
    return x == 0.0 or math.floor(x * (1.0 - FLOOR_REL)) == math.floor(x * (1.0 + FLOOR_REL))


def daylight(step, period):
    """Daylight of a step in a cycle of `period` steps, as an integer in
    [-period, period]: period at noon (step 0 of the cycle), falling linearly
    to 0 a quarter cycle later and to -period at midnight, then back."""
    hours_since_noon = step % period
    hours_to_noon = min(hours_since_noon, period - hours_since_noon)
    return period - 4 * hours_to_noon


class World:
    def __init__(self, W, H, E, I, C, G, R, nets, rho_i, rho_l, kappa, cycle=None,
                 hard_max=False, kappa_energy=0.0):
        self.W, self.H = W, H
        self.E, self.I, self.C, self.G, self.R = E, I, C, G, R   # flat lists; C = 4 lists
        self.nets = nets
        self.rho_i, self.rho_l, self.kappa = rho_i, rho_l, kappa
        # day / night cycle: (period, quanta per cell at noon, removal over 65536, step)
        self.cycle = cycle
        # physics variants: the whole exploration budget to the maximal
        # explore actuator; energy moving along the same directions
        self.hard_max = hard_max
        self.kappa_energy = kappa_energy

    def at(self, x, y):
        return (y % self.H) * self.W + (x % self.W)

    def neighbour(self, i, d):
        dx, dy = direction_vector(d)
        return self.at(i % self.W + dx, i // self.W + dy)

    def plan(self, i):
        """Everything cell i decides this step, from the pre-step state."""
        order = kernel_order(self.R[i] % 8)
        cells = [i] + [self.neighbour(i, d) for d in order]
        u = []
        for c in cells:
            u += [self.E[c] * Q, self.I[c] * Q] + [self.C[k][c] for k in range(4)]
        a = run_net(self.nets[self.G[i]], u)
        e, inf = self.E[i], self.I[i]
        args = [self.rho_i * sig(a[0]) * e, self.rho_l * sig(a[1]) * inf]
        x_inv = min(e, math.floor(args[0]))
        x_liq = min(inf, math.floor(args[1]))
        e1, i1 = e - x_inv + x_liq, inf + x_inv - x_liq
        comm = [sig(a[2 + k]) for k in range(4)]
        logits = a[6:14]
        m = max(logits)
        ex = [math.exp(v - m) for v in logits]
        tot = 0.0
        for v in ex:
            tot += v
        args.append(self.kappa * i1)
        F = math.floor(args[-1])
        best = logits.index(m)

        def split(budget, record):
            out, used = {}, 0
            for p in range(8):
                if self.hard_max:
                    amount = budget if p == best else 0
                else:
                    share = (ex[p] / tot) * budget
                    if record:
                        args.append(share)
                    amount = min(math.floor(share), budget - used)
                used += amount
                out[order[p]] = amount
            return out

        flows = split(F, True)
        eflows = {d: 0 for d in range(8)}
        if self.kappa_energy > 0:
            eflows = split(math.floor(self.kappa_energy * e1), False)
        return dict(e1=e1, i1=i1, comm=comm, flows=flows, eflows=eflows, explore=order[best], act=a,
                    order=order, logits=logits, exact=all(floor_decided(x) for x in args))

    def margins(self, plans, t):
        """The near-tie report of target t, from the plans of its neighbours:
        (smallest top-1 minus top-2 flow-logit gap of a neighbour whose two
        leading explore directions include t and whose flows are not all
        decided zeros; |v_win - I1(t)|; v_win - v_second on a takeover;
        max(v_win, I1(t)); 1.0 when I1(t) and every explorer's flows are
        decided integers)."""
        pt = plans[t]
        gap = math.inf
        cands = []
        for d in range(8):
            n = self.neighbour(t, d)
            pn = plans[n]
            back = (d + 4) % 8
            lg = pn["logits"]
            top1 = max(range(8), key=lambda k: (lg[k], -k))
            top2 = max((k for k in range(8) if k != top1), key=lambda k: (lg[k], -k))
            idle = pn["exact"] and all(v == 0 for v in pn["flows"].values())
            if back in (pn["order"][top1], pn["order"][top2]) and not idle:
                gap = min(gap, lg[top1] - lg[top2])
            if pn["explore"] == back:
                cands.append((pn["flows"][back], d, pn["exact"]))
        if not cands:
            return [gap, math.inf, math.inf, 0.0, 1.0 if pt["exact"] else 0.0]
        win = cands[0]
        for c in cands[1:]:
            if c[0] > win[0]:
                win = c
        take = float(abs(win[0] - pt["i1"]))
        mag = float(max(win[0], pt["i1"]))
        rank = math.inf
        others = [c[0] for c in cands if c is not win]
        if win[0] > pt["i1"] and others:
            rank = float(win[0] - max(others))
        decided = pt["exact"] and all(c[2] for c in cands)
        return [gap, take, rank, mag, 1.0 if decided else 0.0]

    def step(self):
        N = self.W * self.H
        plans = [self.plan(i) for i in range(N)]
        E2, I2, G2, R2 = [0] * N, [0] * N, [0] * N, [0] * N
        C2 = [[0.0] * N for _ in range(4)]
        takeovers = 0
        for t in range(N):
            pt = plans[t]
            inflow = 0
            best = None
            for d in range(8):
                n = self.neighbour(t, d)
                back = (d + 4) % 8
                amount = plans[n]["flows"][back]
                inflow += amount
                if plans[n]["explore"] == back and (best is None or amount > best[0]):
                    best = (amount, d, n)
            I2[t] = pt["i1"] - sum(pt["flows"].values()) + inflow
            energy = pt["e1"] - sum(pt["eflows"].values())
            for d in range(8):
                energy += plans[self.neighbour(t, d)]["eflows"][(d + 4) % 8]
            E2[t] = energy
            if self.cycle is not None:
                period, noon_quanta, removal, step = self.cycle
                light = daylight(step, period)
                if light > 0:
                    E2[t] += noon_quanta * light // period
                elif light < 0:
                    E2[t] -= (energy * removal // 65536) * (-light) // period
            for k in range(4):
                C2[k][t] = pt["comm"][k]
            G2[t], R2[t] = self.G[t], self.R[t]
            if best is not None and best[0] > pt["i1"]:
                G2[t], R2[t] = self.G[best[2]], (best[1] + 4) % 8
                takeovers += 1
        return E2, I2, C2, G2, R2, takeovers, plans
